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
//   k_probe_lds_kind LDS atomic adds of either width with lanes STRIDE words apart
//                    (wsg_probe_lds): what the FP64 rate loses to bank conflicts, and
//                    the FP32 rate an FP32 tile would see.
#include "wsg_internal.h"
#include "wsg.h"

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

// Lane i adds to element i * STRIDE of four slots: STRIDE 1 puts no two lanes of an
// instruction on one bank (FP32) or bank pair (FP64); larger strides fold lanes onto
// the same banks.  Every index stays below 4 * kProbeThreads * STRIDE.
template <typename T, int STRIDE>
__global__ __launch_bounds__(kProbeThreads) void k_probe_lds_kind(int iters, T *__restrict__ out) {
    __shared__ T buf[kProbeThreads * 4 * STRIDE];
    for (int i = threadIdx.x; i < kProbeThreads * 4 * STRIDE; i += blockDim.x) buf[i] = T(0);
    __syncthreads();
    T *a = buf + threadIdx.x * STRIDE;
    const T d = (T)(1.0 + threadIdx.x * 1e-3);
    for (int it = 0; it < iters; ++it) {
        atomicAdd(a, d);
        atomicAdd(a + kProbeThreads * STRIDE, d);
        atomicAdd(a + 2 * kProbeThreads * STRIDE, d);
        atomicAdd(a + 3 * kProbeThreads * STRIDE, d);
    }
    __syncthreads();
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = buf[threadIdx.x * STRIDE];
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

extern "C" {

wsg_status wsg_probe_lds(int device, int32_t kind, double *adds_per_s) {
    using namespace wsg;
    if (!adds_per_s) return WSG_EINVAL;
    *adds_per_s = 0.0;
    if (kind < 0 || kind > 3) return WSG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return WSG_EDEVICE;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n_cu <= 0)
        return WSG_EDEVICE;
    const int blocks = n_cu * 8, iters = kind == 1 ? 256 : 2048;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *out = nullptr;
    wsg_status rc = WSG_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = WSG_EDEVICE;
    } else if (hipMalloc(&out, (size_t)blocks * kProbeThreads * sizeof(double)) != hipSuccess) {
        rc = WSG_ENOMEM;
    } else {
        float best = 1e30f;
        for (int rep = 0; rep < 4 && rc == WSG_OK; ++rep) {
            (void)hipEventRecord(e0, s);
            switch (kind) {
            case 0: k_probe_lds_kind<double, 1><<<blocks, kProbeThreads, 0, s>>>(iters, (double *)out); break;
            case 1: k_probe_lds_kind<float, 1><<<blocks, kProbeThreads, 0, s>>>(iters, (float *)out); break;
            case 2: k_probe_lds_kind<double, 2><<<blocks, kProbeThreads, 0, s>>>(iters, (double *)out); break;
            default: k_probe_lds_kind<double, 16><<<blocks, kProbeThreads, 0, s>>>(iters, (double *)out); break;
            }
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
                rc = WSG_EDEVICE;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0 && ms < best) best = ms;   // the first launch warms up
        }
        if (rc == WSG_OK) *adds_per_s = (double)blocks * kProbeThreads * 4.0 * iters / (best * 1e-3);
    }
    if (s) (void)hipStreamSynchronize(s);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    return rc;
}

}  // extern "C"
