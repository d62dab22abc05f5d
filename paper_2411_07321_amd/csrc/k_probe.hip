// Device probes for the roofline: rates that the vendor does not publish, measured
// with the same compiler and flags as the imaging kernels.
//
//   k_probe_lds_add  FP64 atomic adds into LDS without a returned value, the operation
//                    the gridder's tile flushes are made of (ds_add_f64): every lane of
//                    a wave adds to its own double, consecutive lanes on consecutive
//                    doubles, so no two lanes of an instruction share a bank pair and
//                    the rate is the LDS atomic issue limit.
//   k_probe_copy     16-byte loads and stores over a large buffer: the device-memory
//                    bandwidth a streaming kernel can reach.
#include "wsg_internal.h"

#include <algorithm>

namespace wsg {

namespace {

constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void k_probe_lds_add(int iters, double *__restrict__ out) {
    __shared__ double buf[kProbeThreads * 4];
    for (int i = threadIdx.x; i < kProbeThreads * 4; i += blockDim.x) buf[i] = 0.0;
    __syncthreads();
    // four independent slots per lane keep several atomics in flight
    double *a = buf + threadIdx.x;
    const double d = 1.0 + threadIdx.x * 1e-3;
    for (int it = 0; it < iters; ++it) {
        atomicAdd(a, d);
        atomicAdd(a + kProbeThreads, d);
        atomicAdd(a + 2 * kProbeThreads, d);
        atomicAdd(a + 3 * kProbeThreads, d);
    }
    __syncthreads();
    double s = buf[threadIdx.x] + buf[threadIdx.x + kProbeThreads] + buf[threadIdx.x + 2 * kProbeThreads] +
               buf[threadIdx.x + 3 * kProbeThreads];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const float4 *__restrict__ in,
                                                             float4 *__restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

}  // namespace

void launch_probe_lds_add(int blocks, int iters, double *out, hipStream_t s) {
    k_probe_lds_add<<<blocks, kProbeThreads, 0, s>>>(iters, out);
}

int probe_lds_add_threads() { return kProbeThreads; }

void launch_probe_copy(const void *in, void *out, size_t bytes, int n_cu, hipStream_t s) {
    const size_t n = bytes / sizeof(float4);
    const unsigned blocks = (unsigned)std::min<size_t>((n + kProbeThreads - 1) / kProbeThreads,
                                                       (size_t)std::max(n_cu, 1) * 16);
    k_probe_copy<<<blocks, kProbeThreads, 0, s>>>((const float4 *)in, (float4 *)out, n);
}

}  // namespace wsg
