"""MI355X-native w-stacking imager (HIP kernels behind a C ABI, include/wsg.h).

Submodules:
  wsg    ctypes binding of libwsg.so (argument marshalling only)
  synth  seeded synthetic interferometer inputs
  build  hipcc build of libwsg.so for gfx950
  serve  continuous-batching imaging server
Nothing is loaded at import time.
"""
