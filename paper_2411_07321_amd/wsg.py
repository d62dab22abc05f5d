"""ctypes binding of libwsg (include/wsg.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts
numpy arrays / torch tensors into pointers, sizes and memory spaces, and
turns status codes into exceptions.  There is no fallback: if libwsg.so is
missing or no device is present, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwsg.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUSY, EUNSUPPORTED, ECANCELED = 0, -1, -2, -3, -4, -5, -6
PREC = {"f64": 0, "f32_phase64": 1, "f32_phase32": 2}
MEM_HOST, MEM_DEVICE = 0, 1
GRID_CORRECT, NORMALIZE, PER_CHANNEL, NAIVE_NM1, W_FOLD = 1, 2, 4, 8, 16

# symbols declared in include/wsg.h
SYMBOLS = ("wsg_create", "wsg_destroy", "wsg_strerror", "wsg_last_error", "wsg_set_budget",
           "wsg_set_timing", "wsg_check", "wsg_footprint", "wsg_n_images", "wsg_image",
           "wsg_image_noalloc",
           "wsg_stage_grid", "wsg_stage_fft", "wsg_stage_wcorrect", "wsg_autotune",
           "wsg_server_create", "wsg_server_destroy", "wsg_server_submit", "wsg_server_poll",
           "wsg_server_wait", "wsg_server_memory", "wsg_trim", "wsg_context_stream",
           "wsg_accum_begin", "wsg_accum_footprint", "wsg_accum_add", "wsg_accum_finish",
           "wsg_accum_destroy", "wsg_submit", "wsg_poll", "wsg_wait", "wsg_cancel",
           "wsg_server_cancel", "wsg_probe_rates", "wsg_probe_lds")


class WsgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"wsg status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("grid_n", ctypes.c_int32), ("n_wplanes", ctypes.c_int32),
                ("support", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cell_rad", ctypes.c_double), ("kernel_sigma", ctypes.c_double),
                ("w_min", ctypes.c_double), ("w_max", ctypes.c_double),
                ("plane_lo", ctypes.c_int32), ("plane_hi", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tile", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("kernel_beta", ctypes.c_double),
                ("w_support", ctypes.c_int32), ("planes_per_pass", ctypes.c_int32)]


class Vis(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_chan", ctypes.c_int32), ("mem", ctypes.c_int32),
                ("row_period", ctypes.c_int64), ("uvw", ctypes.c_void_p), ("freq_hz", ctypes.c_void_p), ("vis", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_used", ctypes.c_int64), ("n_flagged", ctypes.c_int64),
                ("n_dropped", ctypes.c_int64), ("n_records", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_tile_rows", ctypes.c_int64),
                ("sum_w", ctypes.c_double),
                ("w_min", ctypes.c_double), ("w_max", ctypes.c_double),
                ("ms_prep", ctypes.c_float), ("ms_count", ctypes.c_float),
                ("ms_scatter", ctypes.c_float), ("ms_zero", ctypes.c_float),
                ("ms_grid", ctypes.c_float), ("ms_occupancy", ctypes.c_float),
                ("ms_fft1", ctypes.c_float), ("ms_fft2_wcorr", ctypes.c_float),
                ("ms_total", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class JobInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double),
                ("footprint", ctypes.c_uint64), ("stats", Stats)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "stats"}
        d["stats"] = self.stats.as_dict()
        return d


_lib = None


def load() -> ctypes.CDLL:
    """Load libwsg.so (built in-tree by paper_2411_07321_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        # torch brings its own HIP runtime; loading it first makes the library bind
        # to that same runtime (one per process).  Loaded the other way round, a
        # second runtime initialises the device first and torch then finds none.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        P, S = ctypes.c_void_p, ctypes.c_int32
        lib.wsg_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
        lib.wsg_destroy.argtypes = [P]
        lib.wsg_destroy.restype = None
        lib.wsg_strerror.argtypes = [S]
        lib.wsg_strerror.restype = ctypes.c_char_p
        lib.wsg_last_error.argtypes = [P]
        lib.wsg_last_error.restype = ctypes.c_char_p
        lib.wsg_set_budget.argtypes = [P, ctypes.c_uint64]
        lib.wsg_set_timing.argtypes = [P, S]
        lib.wsg_check.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Vis)]
        lib.wsg_footprint.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Vis),
                                      ctypes.POINTER(ctypes.c_uint64)]
        lib.wsg_n_images.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Vis)]
        lib.wsg_image.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(Vis), P, S, P,
                                  ctypes.POINTER(Stats)]
        lib.wsg_image_noalloc.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(Vis), P, P,
                                          ctypes.POINTER(Stats)]
        lib.wsg_submit.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(Vis), P, S,
                                   ctypes.POINTER(ctypes.c_uint64)]
        lib.wsg_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(S), ctypes.POINTER(Stats)]
        lib.wsg_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Stats)]
        lib.wsg_cancel.argtypes = [P, ctypes.c_uint64]
        lib.wsg_probe_rates.argtypes = [ctypes.c_int, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        lib.wsg_probe_lds.argtypes = [ctypes.c_int, S, ctypes.POINTER(ctypes.c_double)]
        lib.wsg_server_cancel.argtypes = [P, ctypes.c_uint64]
        lib.wsg_stage_grid.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(Vis), P, S, P,
                                       ctypes.POINTER(Stats)]
        lib.wsg_stage_fft.argtypes = [P, ctypes.POINTER(Params), P, ctypes.c_int64, S, P]
        lib.wsg_stage_wcorrect.argtypes = [P, ctypes.POINTER(Params), P, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           P, S, P]
        lib.wsg_autotune.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(Vis),
                                     ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
        lib.wsg_server_create.argtypes = [ctypes.c_int, S, ctypes.c_uint64, ctypes.POINTER(P)]
        lib.wsg_server_destroy.argtypes = [P]
        lib.wsg_server_destroy.restype = None
        lib.wsg_server_submit.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(Vis), P, S,
                                          ctypes.POINTER(ctypes.c_uint64)]
        lib.wsg_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(S),
                                        ctypes.POINTER(JobInfo)]
        lib.wsg_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(JobInfo)]
        lib.wsg_server_memory.argtypes = [P, ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.POINTER(ctypes.c_uint64)]
        lib.wsg_trim.argtypes = [P]
        lib.wsg_context_stream.argtypes = [P]
        lib.wsg_context_stream.restype = P
        lib.wsg_accum_begin.argtypes = [P, ctypes.POINTER(Params), S, P, ctypes.POINTER(P)]
        lib.wsg_accum_footprint.argtypes = [ctypes.POINTER(Params), S,
                                            ctypes.POINTER(ctypes.c_uint64)]
        lib.wsg_accum_add.argtypes = [P, ctypes.POINTER(Vis), P]
        lib.wsg_accum_finish.argtypes = [P, P, S, P, ctypes.POINTER(Stats)]
        lib.wsg_accum_destroy.argtypes = [P]
        lib.wsg_accum_destroy.restype = None
        for name in ("wsg_create", "wsg_set_budget", "wsg_set_timing", "wsg_check",
                     "wsg_footprint", "wsg_image", "wsg_image_noalloc", "wsg_stage_grid", "wsg_stage_fft",
                     "wsg_stage_wcorrect", "wsg_autotune", "wsg_server_create",
                     "wsg_server_submit", "wsg_server_poll", "wsg_server_wait",
                     "wsg_server_memory", "wsg_trim", "wsg_accum_begin", "wsg_accum_footprint",
                     "wsg_accum_add", "wsg_accum_finish", "wsg_submit", "wsg_poll", "wsg_wait",
                     "wsg_cancel", "wsg_server_cancel", "wsg_probe_rates", "wsg_probe_lds"):
            getattr(lib, name).restype = S
        lib.wsg_n_images.restype = S
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load().wsg_strerror(status).decode()


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr_mem(x):
    """(pointer, memory space) of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None, None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr(), (MEM_DEVICE if x.is_cuda else MEM_HOST)
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return x.ctypes.data, MEM_HOST
    raise TypeError(f"unsupported buffer type {type(x)}")


def _numel(x) -> int:
    return int(x.numel()) if _is_torch(x) else int(x.size)


def _kind(x) -> tuple[str, int]:
    """('c' complex | 'f' float | 'u' unsigned | 'b' bool | 'i' int, bytes per element)."""
    if _is_torch(x):
        dt = x.dtype
        size = x.element_size()
        if dt.is_complex:
            return "c", size
        if dt.is_floating_point:
            return "f", size
        return ("b" if str(dt) == "torch.bool" else ("u" if str(dt) == "torch.uint8" else "i")), size
    return x.dtype.kind, x.dtype.itemsize


def _check_inputs(params: Params, vb: "VisBuffers"):
    """The library reads vis, weights and flags with the element types of the precision
    and assumes [n_rows][n_chan] extents (the C ABI carries no sizes): check them here."""
    uvw, vis, wts, flags = vb.keep[:4]
    rows, nch = vb.desc.n_rows, vb.desc.n_chan
    f64 = params.precision == PREC["f64"]
    if _kind(uvw) != ("f", 8) or _numel(uvw) != 3 * rows:
        raise ValueError("uvw must be float64 [n_rows, 3]")
    if _kind(vis) != ("c", 16 if f64 else 8) or _numel(vis) != rows * nch:
        raise ValueError(f"vis must be {'complex128' if f64 else 'complex64'} [n_rows, n_chan] "
                         "for this precision")
    if wts is not None and (_kind(wts) != ("f", 8 if f64 else 4) or _numel(wts) != rows * nch):
        raise ValueError(f"weights must be {'float64' if f64 else 'float32'} [n_rows, n_chan] "
                         "for this precision")
    if flags is not None and (_kind(flags)[1] != 1 or _numel(flags) != rows * nch):
        raise ValueError("flags must be one byte per element, [n_rows, n_chan]")


def _check_out(out, n_elems: int, kind: tuple, what: str):
    if _kind(out) != kind or _numel(out) < n_elems:
        raise ValueError(f"{what} must hold at least {n_elems} elements of "
                         f"{ {('f', 8): 'float64', ('c', 16): 'complex128', ('c', 8): 'complex64'}[kind] }")


KERNEL = {"gauss": 0, "kb": 1}


def make_params(grid_n, n_wplanes, support, cell_rad, precision="f32_phase64", kernel_sigma=0.9,
                w_min=None, w_max=None, plane_lo=0, plane_hi=0, grid_correct=True,
                normalize=True, per_channel=False, naive_nm1=False, tile=0, kernel="gauss",
                kernel_beta=0.0, w_fold=False, w_support=1, planes_per_pass=0) -> Params:
    """kernel: "gauss" (width kernel_sigma) or "kb" (Kaiser-Bessel, shape kernel_beta;
    0 = the library's default for the support).  w_fold: grid rows with w < 0 at their
    Hermitian mirror.  w_support: planes a visibility spreads over (1: its own).
    planes_per_pass: planes of each image in the w-stack at a time (0: all)."""
    flags = (GRID_CORRECT if grid_correct else 0) | (NORMALIZE if normalize else 0) | \
        (PER_CHANNEL if per_channel else 0) | (NAIVE_NM1 if naive_nm1 else 0) | \
        (W_FOLD if w_fold else 0)
    return Params(int(grid_n), int(n_wplanes), int(support), PREC[precision], float(cell_rad),
                  float(kernel_sigma), math.nan if w_min is None else float(w_min),
                  math.nan if w_max is None else float(w_max), int(plane_lo), int(plane_hi),
                  flags, int(tile), KERNEL[kernel], float(kernel_beta), int(w_support),
                  int(planes_per_pass))


@dataclass
class VisBuffers:
    """Keeps the arrays behind a Vis descriptor alive for the duration of a call."""
    desc: Vis
    keep: tuple


def make_vis(uvw, vis, weights=None, flags=None, freq_hz=None, row_period=0) -> VisBuffers:
    """Describe measurements: uvw [rows,3] f64, vis [rows,n_chan] complex, weights and flags
    [rows,n_chan] or None, freq_hz (host) or None.  All buffers in one memory space.
    row_period: baselines per time slice of time-major data (a performance hint)."""
    pu, mu = _ptr_mem(uvw)
    pv, mv = _ptr_mem(vis)
    pw, mw = _ptr_mem(weights)
    pf, mf = _ptr_mem(flags)
    spaces = {m for m in (mu, mv, mw, mf) if m is not None}
    if len(spaces) > 1:
        raise ValueError("uvw, vis, weights and flags must live in one memory space")
    n_rows = uvw.shape[0]
    n_chan = vis.shape[1] if vis.ndim == 2 else 1
    fq = None
    if freq_hz is not None:
        fq = np.ascontiguousarray(freq_hz, dtype=np.float64)
    d = Vis(int(n_rows), int(n_chan), spaces.pop() if spaces else MEM_HOST, int(row_period), pu,
            None if fq is None else fq.ctypes.data, pv, pw, pf)
    return VisBuffers(d, (uvw, vis, weights, flags, fq))


def _mesh_kind(params: Params) -> tuple:
    return ("c", 16) if params.precision == PREC["f64"] else ("c", 8)


def _stream_of(x, stream):
    if stream is not None:
        return stream
    if _is_torch(x) and x.is_cuda:
        import torch
        return torch.cuda.current_stream(x.device).cuda_stream
    return None


class Context:
    """One library context on one HIP device (owns workspace and its own stream).

    Calls run on the stream given, else on torch's current stream of the output
    tensor, else (host outputs) on HIP's null stream; `ctx.stream` is the
    context's own stream."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        st = lib.wsg_create(int(device), ctypes.byref(h))
        if st != OK:
            raise WsgError(st, f"wsg_create(device={device}) failed: {strerror(st)}")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().wsg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st: int, what: str):
        if st != OK:
            detail = load().wsg_last_error(self._h).decode()
            raise WsgError(st, f"{what}: {strerror(st)} ({detail})")

    @property
    def stream(self) -> int:
        """The context's own hipStream_t, as an integer handle."""
        return load().wsg_context_stream(self._h)

    def set_budget(self, nbytes: int):
        self._check(load().wsg_set_budget(self._h, int(nbytes)), "wsg_set_budget")

    def set_timing(self, on: bool):
        self._check(load().wsg_set_timing(self._h, 1 if on else 0), "wsg_set_timing")

    def image(self, params: Params, vb: VisBuffers, out, stream=None, stats: bool = True):
        """Run the method; `out` is [n_images,N,N] (or [N,N]) float64 host array or device
        tensor.  Returns per-image stats (list of dicts) when stats is True."""
        po, mo = _ptr_mem(out)
        n_img = load().wsg_n_images(ctypes.byref(params), ctypes.byref(vb.desc))
        _check_inputs(params, vb)
        _check_out(out, max(1, n_img) * params.grid_n ** 2, ("f", 8), "the image")
        st_arr = (Stats * max(1, n_img))() if stats else None
        s = _stream_of(out, stream)
        rc = load().wsg_image(self._h, ctypes.byref(params), ctypes.byref(vb.desc), po, mo,
                              s, st_arr)
        self._check(rc, "wsg_image")
        return [x.as_dict() for x in st_arr] if stats else None

    def image_noalloc(self, params: Params, vb: VisBuffers, out, stream=None, stats: bool = True):
        """wsg_image_noalloc: the method with no allocation, on the library's static
        workspace (device inputs and image only; small jobs)."""
        po, mo = _ptr_mem(out)
        if mo != MEM_DEVICE or vb.desc.mem != MEM_DEVICE:
            raise ValueError("image_noalloc takes device inputs and a device image")
        n_img = load().wsg_n_images(ctypes.byref(params), ctypes.byref(vb.desc))
        _check_inputs(params, vb)
        _check_out(out, max(1, n_img) * params.grid_n ** 2, ("f", 8), "the image")
        st_arr = (Stats * max(1, n_img))() if stats else None
        s = _stream_of(out, stream)
        rc = load().wsg_image_noalloc(self._h, ctypes.byref(params), ctypes.byref(vb.desc), po, s,
                                      st_arr)
        self._check(rc, "wsg_image_noalloc")
        return [x.as_dict() for x in st_arr] if stats else None

    def submit(self, params: Params, vb: VisBuffers, out) -> int:
        """wsg_submit: queue a job on this context; `vb` and `out` are kept alive here
        until the job is reported by poll / wait."""
        po, mo = _ptr_mem(out)
        _check_inputs(params, vb)
        _check_out(out, max(1, n_images(params, vb)) * params.grid_n ** 2, ("f", 8), "the image")
        t = ctypes.c_uint64(0)
        self._check(load().wsg_submit(self._h, ctypes.byref(params), ctypes.byref(vb.desc), po, mo,
                                      ctypes.byref(t)), "wsg_submit")
        if not hasattr(self, "_jobs"):
            self._jobs = {}
        self._jobs[t.value] = (params, vb, out, max(1, n_images(params, vb)))
        return int(t.value)

    def _report(self, ticket, rc, st_arr):
        self._jobs.pop(ticket, None)
        return rc, ([x.as_dict() for x in st_arr] if rc == OK else None)

    def poll(self, ticket: int):
        """wsg_poll: (False, None, None) while the job runs, else (True, status, stats)."""
        n_img = self._jobs[ticket][3]
        done = ctypes.c_int32(0)
        st_arr = (Stats * n_img)()
        rc = load().wsg_poll(self._h, int(ticket), ctypes.byref(done), st_arr)
        if not done.value:
            self._check(rc, "wsg_poll")
            return False, None, None
        return (True,) + self._report(ticket, rc, st_arr)

    def wait(self, ticket: int):
        """wsg_wait: (status, stats) of the job."""
        n_img = self._jobs[ticket][3]
        st_arr = (Stats * n_img)()
        rc = load().wsg_wait(self._h, int(ticket), st_arr)
        return self._report(ticket, rc, st_arr)

    def cancel(self, ticket: int) -> int:
        """wsg_cancel: OK, or EBUSY once the job is on the device."""
        return load().wsg_cancel(self._h, int(ticket))

    def stage_grid(self, params: Params, vb: VisBuffers, out, stream=None):
        po, mo = _ptr_mem(out)
        n_img = load().wsg_n_images(ctypes.byref(params), ctypes.byref(vb.desc))
        _check_inputs(params, vb)
        n_pl = (params.plane_hi - params.plane_lo) if params.plane_hi > params.plane_lo \
            else params.n_wplanes
        _check_out(out, max(1, n_img) * n_pl * params.grid_n ** 2, _mesh_kind(params), "the grid")
        st_arr = (Stats * max(1, n_img))()
        rc = load().wsg_stage_grid(self._h, ctypes.byref(params), ctypes.byref(vb.desc), po, mo,
                                   _stream_of(out, stream), st_arr)
        self._check(rc, "wsg_stage_grid")
        return [x.as_dict() for x in st_arr]

    def stage_fft(self, params: Params, planes, stream=None):
        po, mo = _ptr_mem(planes)
        n = planes.shape[0] if planes.ndim == 3 else 1
        _check_out(planes, n * params.grid_n ** 2, _mesh_kind(params), "the planes")
        rc = load().wsg_stage_fft(self._h, ctypes.byref(params), po, int(n), mo,
                                  _stream_of(planes, stream))
        self._check(rc, "wsg_stage_fft")

    def stage_wcorrect(self, params: Params, planes, w_min, w_max, sum_w, out, stream=None):
        pp, mp = _ptr_mem(planes)
        po, mo = _ptr_mem(out)
        if mp != mo:
            raise ValueError("planes and image must live in one memory space")
        n = planes.shape[0] if planes.ndim == 3 else 1
        _check_out(planes, n * params.grid_n ** 2, _mesh_kind(params), "the planes")
        _check_out(out, params.grid_n ** 2, ("f", 8), "the image")
        rc = load().wsg_stage_wcorrect(self._h, ctypes.byref(params), pp, int(n), float(w_min),
                                       float(w_max), float(sum_w), po, mo,
                                       _stream_of(out, stream))
        self._check(rc, "wsg_stage_wcorrect")

    def autotune(self, params: Params, vb: VisBuffers, cache_path: str | None = None):
        """wsg_autotune: (tile, planes_per_pass) chosen for this job shape (0 = all planes)."""
        best, ppp = ctypes.c_int32(0), ctypes.c_int32(0)
        rc = load().wsg_autotune(self._h, ctypes.byref(params), ctypes.byref(vb.desc),
                                 None if cache_path is None else cache_path.encode(),
                                 ctypes.byref(best), ctypes.byref(ppp))
        self._check(rc, "wsg_autotune")
        return int(best.value), int(ppp.value)


class Accum:
    """A chunked imaging job on a context: begin (allocates and clears the w-stack),
    add chunks of visibilities (time or frequency slices), finish into the image.
    Needs a given w range.  Use as a context manager or call close()."""

    def __init__(self, ctx: Context, params: Params, n_chan: int, stream=None):
        h = ctypes.c_void_p()
        self._ctx = ctx
        self._params = params
        self._n_img = n_chan if (params.flags & PER_CHANNEL) else 1
        rc = load().wsg_accum_begin(ctx._h, ctypes.byref(params), int(n_chan), stream,
                                    ctypes.byref(h))
        ctx._check(rc, "wsg_accum_begin")
        self._h = h

    def add(self, vb: VisBuffers, stream=None):
        """Bin and grid one chunk; device chunks run on torch's current stream unless a
        stream is given, host chunks on HIP's null stream."""
        keep = vb.keep
        s = _stream_of(next((x for x in keep if x is not None and _is_torch(x)), None), stream)
        _check_inputs(self._params, vb)
        self._ctx._check(load().wsg_accum_add(self._h, ctypes.byref(vb.desc), s), "wsg_accum_add")

    def finish(self, out, stream=None):
        """Transform, w-correct and sum into `out` ([n_images,N,N] float64, host array or
        device tensor); returns per-image stats of all chunks."""
        po, mo = _ptr_mem(out)
        _check_out(out, self._n_img * self._params.grid_n ** 2, ("f", 8), "the image")
        st_arr = (Stats * self._n_img)()
        rc = load().wsg_accum_finish(self._h, po, mo, _stream_of(out, stream), st_arr)
        self._ctx._check(rc, "wsg_accum_finish")
        return [x.as_dict() for x in st_arr]

    def close(self):
        if getattr(self, "_h", None):
            load().wsg_accum_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def accum_footprint(params: Params, n_chan: int) -> int:
    out = ctypes.c_uint64(0)
    st = load().wsg_accum_footprint(ctypes.byref(params), int(n_chan), ctypes.byref(out))
    if st != OK:
        raise WsgError(st, f"wsg_accum_footprint: {strerror(st)}")
    return int(out.value)


class Server:
    """Continuous-batching imaging server (n_slots concurrent jobs, device-memory budget)."""

    def __init__(self, device: int = 0, n_slots: int = 4, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        st = load().wsg_server_create(int(device), int(n_slots), int(hbm_budget), ctypes.byref(h))
        if st != OK:
            raise WsgError(st, f"wsg_server_create: {strerror(st)}")
        self._h = h
        self._keep = {}

    def submit(self, params: Params, vb: VisBuffers, out) -> int:
        """Queue a job; `out` must stay valid until the job is reported done."""
        po, mo = _ptr_mem(out)
        _check_inputs(params, vb)
        _check_out(out, max(1, n_images(params, vb)) * params.grid_n ** 2, ("f", 8), "the image")
        t = ctypes.c_uint64(0)
        st = load().wsg_server_submit(self._h, ctypes.byref(params), ctypes.byref(vb.desc), po,
                                      mo, ctypes.byref(t))
        if st != OK:
            raise WsgError(st, f"wsg_server_submit: {strerror(st)}")
        self._keep[t.value] = (params, vb, out)
        return int(t.value)

    def poll(self, ticket: int):
        done = ctypes.c_int32(0)
        info = JobInfo()
        st = load().wsg_server_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(info))
        if st != OK:
            raise WsgError(st, "wsg_server_poll: unknown ticket")
        if done.value:
            self._keep.pop(ticket, None)
            return True, info.as_dict()
        return False, None

    def wait(self, ticket: int) -> dict:
        info = JobInfo()
        st = load().wsg_server_wait(self._h, int(ticket), ctypes.byref(info))
        if st != OK:
            raise WsgError(st, "wsg_server_wait: unknown ticket")
        self._keep.pop(ticket, None)
        return info.as_dict()

    def cancel(self, ticket: int) -> int:
        """wsg_server_cancel: OK (a queued job dropped, reported ECANCELED) or EBUSY."""
        return load().wsg_server_cancel(self._h, int(ticket))

    def memory(self):
        held, peak = ctypes.c_uint64(0), ctypes.c_uint64(0)
        load().wsg_server_memory(self._h, ctypes.byref(held), ctypes.byref(peak))
        return int(held.value), int(peak.value)

    def close(self):
        if getattr(self, "_h", None):
            load().wsg_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def check(params: Params, vb: VisBuffers | None = None) -> int:
    return load().wsg_check(ctypes.byref(params), None if vb is None else ctypes.byref(vb.desc))


def footprint(params: Params, vb: VisBuffers) -> int:
    out = ctypes.c_uint64(0)
    st = load().wsg_footprint(ctypes.byref(params), ctypes.byref(vb.desc), ctypes.byref(out))
    if st != OK:
        raise WsgError(st, f"wsg_footprint: {strerror(st)}")
    return int(out.value)


def n_images(params: Params, vb: VisBuffers) -> int:
    return int(load().wsg_n_images(ctypes.byref(params), ctypes.byref(vb.desc)))


def params_for(ds, **over) -> Params:
    """Parameters of a synthetic Dataset (paper_2411_07321_amd.synth), with overrides."""
    kw = dict(grid_n=ds.grid_n, n_wplanes=ds.n_wplanes, support=ds.support, cell_rad=ds.cell_rad,
              precision=ds.precision, kernel_sigma=ds.kernel_sigma, per_channel=ds.per_channel)
    kw.update(over)
    return make_params(**kw)


def probe_rates(device: int = 0, copy_bytes: int = 1 << 31) -> dict:
    """wsg_probe_rates: measured FP64 LDS atomic-add rate and device copy bandwidth."""
    lds, cp = ctypes.c_double(0.0), ctypes.c_double(0.0)
    st = load().wsg_probe_rates(int(device), int(copy_bytes), ctypes.byref(lds), ctypes.byref(cp))
    if st != OK:
        raise WsgError(st, f"wsg_probe_rates: {strerror(st)}")
    return {"lds_f64_adds_per_s": lds.value, "copy_bytes_per_s": cp.value}


# kinds of wsg_probe_lds
LDS_PROBES = {"f64": 0, "f32": 1, "f64_2way": 2, "f64_16way": 3}


def probe_lds(device: int = 0) -> dict:
    """wsg_probe_lds for every kind: LDS atomic adds per second (FP64 and FP32 with
    every lane on its own bank, FP64 with 2 and 16 lanes per bank pair)."""
    out = {}
    for name, kind in LDS_PROBES.items():
        r = ctypes.c_double(0.0)
        st = load().wsg_probe_lds(int(device), int(kind), ctypes.byref(r))
        if st != OK:
            raise WsgError(st, f"wsg_probe_lds: {strerror(st)}")
        out[name] = r.value
    return out
