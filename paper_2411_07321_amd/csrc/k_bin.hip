// Binning of visibilities by (image, w-plane, uv tile): a counting sort.
//
// Sec. 2 of the paper buckets the visibilities of each mesh slab before the
// convolution ("an array is created for each slab").  Here the buckets are
// square uv tiles of every w-plane, so that the gridding kernel can keep one
// tile in LDS.  A visibility whose footprint crosses a tile edge is recorded
// in every tile it touches (at most four); each tile then owns its cells and
// writes them once, without global atomics.
//
// Pass structure:
//   k_prep     validity of every element, per-image w range and counts (one
//              thread per (row, channel) element, grid-stride loops whose
//              stride is a multiple of n_chan so a thread stays on one channel)
//   k_finalize plane geometry per image (given range or the data's)
//   k_count    per-bin counts, n_used and sum of weights
//   scan       bin offsets
//   k_scatter  compact records into their bins
//
// k_count and k_scatter follow tracks: rows are viewed as [time][P] with P
// the row period (baselines per time slice), and a thread walks one
// (baseline, channel) through L consecutive time slices.  A track moves
// slowly across the mesh, so consecutive elements of a thread mostly fall in
// the same bins: a "run" is a maximal stretch of consecutive elements whose
// footprints all touch one bin, and each run costs one global atomic instead
// of one per element (the scatter first sizes the runs of a block of time
// slices, then reserves their slots).  This matters because the uv coverage is extremely
// uneven: the short baselines of a dense core all land in the few central
// tiles, and per-element atomics there serialise.  Records of one run stay
// contiguous inside their bin.
#include "wsg_internal.h"

#include <algorithm>

namespace wsg {

namespace {

constexpr int kThreads = 256;
constexpr int kBatch = 4;          // elements of a track whose loads are issued together

__device__ __forceinline__ unsigned long long order_key(double d) {
    unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// x = u * scale + half with two roundings (no contraction), as the method states.
__device__ __forceinline__ double mesh_coord(double u, double scale, double half) {
#pragma clang fp contract(off)
    double t = u * scale;
    return t + half;
}

__device__ __forceinline__ bool footprint_fits(double x, int N, int h, int &i0) {
    double f = floor(x + 0.5);
    if (!(f >= (double)h && f <= (double)(N - 1 - h))) return false;
    i0 = (int)f;
    return true;
}

template <typename VT, typename WT>
struct ElemIO;

template <>
struct ElemIO<double, double> {
    static __device__ __forceinline__ void load(const void *vis, const void *wts, int64_t e,
                                                double &vr, double &vi, double &w) {
        const double *v = (const double *)vis;
        vr = v[2 * e];
        vi = v[2 * e + 1];
        w = wts ? ((const double *)wts)[e] : 1.0;
    }
};
template <>
struct ElemIO<float, float> {
    static __device__ __forceinline__ void load(const void *vis, const void *wts, int64_t e,
                                                double &vr, double &vi, double &w) {
        const float2 v = ((const float2 *)vis)[e];
        vr = (double)v.x;
        vi = (double)v.y;
        w = wts ? (double)((const float *)wts)[e] : 1.0;
    }
};

__device__ __forceinline__ bool is_finite(double a) { return isfinite(a); }

// Every test except the w range (O2 of the method's reading).
template <typename VT>
__device__ __forceinline__ bool valid0(const JobGeom &g, const double *uvw, const void *vis,
                                       const void *wts, const uint8_t *flags, int64_t e,
                                       int64_t r, int c, bool &flagged, double &w_out) {
    flagged = flags && flags[e];
    if (flagged) return false;
    double vr, vi, wt;
    ElemIO<VT, VT>::load(vis, wts, e, vr, vi, wt);
    if (!(wt > 0.0) || !is_finite(wt)) return false;
    double sc = g.chan_scale[c];
    double u = uvw[3 * r] * sc, v = uvw[3 * r + 1] * sc, w = uvw[3 * r + 2] * sc;
    if (!is_finite(u) || !is_finite(v) || !is_finite(w)) return false;
    if (!is_finite(vr) || !is_finite(vi)) return false;
    int i0, j0;
    if (!footprint_fits(mesh_coord(u, g.scale, g.half), g.N, g.h, i0)) return false;
    if (!footprint_fits(mesh_coord(v, g.scale, g.half), g.N, g.h, j0)) return false;
    w_out = w;
    return true;
}

// grid-stride geometry: stride a multiple of n_chan
__host__ int blocks_for(int64_t n_elem, int n_chan) {
    int64_t want = (n_elem + kThreads - 1) / kThreads;
    int64_t cap = 4096;
    int64_t b = std::min<int64_t>(std::max<int64_t>(want, 1), cap);
    // make b * kThreads a multiple of n_chan
    int64_t g = n_chan;
    int64_t t = kThreads;
    while (t % 2 == 0 && g % 2 == 0) { t /= 2; g /= 2; }
    // after removing common factors of two, b must be a multiple of the odd part
    // of n_chan not shared with kThreads (kThreads is a power of two)
    int64_t need = g;
    b = ((b + need - 1) / need) * need;
    return (int)b;
}

template <typename VT>
__global__ __launch_bounds__(kThreads) void k_prep(JobGeom g, const double *__restrict__ uvw,
                                                   const void *__restrict__ vis,
                                                   const void *__restrict__ wts,
                                                   const uint8_t *__restrict__ flags,
                                                   uint8_t *__restrict__ mask, ImgState *st) {
    __shared__ unsigned long long s_min[256], s_max[256], s_flag[256], s_valid[256];
    const int n_img = g.n_img;
    for (int i = threadIdx.x; i < n_img; i += blockDim.x) {
        s_min[i] = ~0ull;
        s_max[i] = 0ull;
        s_flag[i] = 0;
        s_valid[i] = 0;
    }
    __syncthreads();
    const int64_t n_elem = g.n_rows * (int64_t)g.n_chan;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long kmin = ~0ull, kmax = 0ull, nf = 0, nv = 0;
    const int c = (int)(e0 % g.n_chan);
    for (int64_t e = e0; e < n_elem; e += stride) {
        int64_t r = e / g.n_chan;
        bool fl;
        double w;
        bool ok = valid0<VT>(g, uvw, vis, wts, flags, e, r, c, fl, w);
        mask[e] = ok ? 1 : 0;
        nf += fl ? 1 : 0;
        if (ok) {
            ++nv;
            unsigned long long k = order_key(w);
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
        }
    }
    const int img = (n_img > 1) ? c : 0;
    if (n_img == 1) {
        // wave reduction, then one LDS atomic per wave
        for (int off = 32; off > 0; off >>= 1) {
            unsigned long long a = __shfl_xor(kmin, off);
            unsigned long long b = __shfl_xor(kmax, off);
            kmin = a < kmin ? a : kmin;
            kmax = b > kmax ? b : kmax;
            nf += __shfl_xor(nf, off);
            nv += __shfl_xor(nv, off);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin(&s_min[0], kmin);
            atomicMax(&s_max[0], kmax);
            atomicAdd(&s_flag[0], nf);
            atomicAdd(&s_valid[0], nv);
        }
    } else {
        atomicMin(&s_min[img], kmin);
        atomicMax(&s_max[img], kmax);
        atomicAdd(&s_flag[img], nf);
        atomicAdd(&s_valid[img], nv);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_img; i += blockDim.x) {
        if (s_valid[i]) {
            atomicMin(&st[i].wmin_key, s_min[i]);
            atomicMax(&st[i].wmax_key, s_max[i]);
            atomicAdd(&st[i].n_valid0, s_valid[i]);
        }
        if (s_flag[i]) atomicAdd(&st[i].n_flagged, s_flag[i]);
    }
}

__global__ void k_finalize(JobGeom g, ImgState *st) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n_img) return;
    ImgState &s = st[i];
    double lo, hi;
    if (g.range_given) {
        lo = g.w_min_given;
        hi = g.w_max_given;
    } else if (s.n_valid0 > 0) {
        lo = key_value(s.wmin_key);
        hi = key_value(s.wmax_key);
    } else {
        lo = 0.0;
        hi = 0.0;
    }
    s.w_min = lo;
    s.w_max = hi;
    s.dw = (hi - lo) / (double)g.n_w;
    s.inv_dw = s.dw > 0.0 ? 1.0 / s.dw : 0.0;
}

// Nearest plane: k = min(n_w - 1, floor((w - w_min) / dw)) with the IEEE quotient.
// The quotient is first formed with the reciprocal; the two can floor differently
// only when it lies within a few ulps (< 1e-9 here, as it is below 65536) of an
// integer, and only then is the division done.
__device__ __forceinline__ int plane_of(double w, double w_min, double dw, double inv_dw, int n_w) {
    if (dw == 0.0) return 0;
    const double d = w - w_min;
    double q = d * inv_dw;
    double f = q - floor(q);
    if (f < 1e-9 || f > 1.0 - 1e-9) q = d / dw;
    int k = (int)floor(q);
    return k > n_w - 1 ? n_w - 1 : k;
}

struct Placed {
    int k;
    int i0, j0;
    double x, y;
};

// A valid element inside the w range: its plane, nearest cell and position, from
// the row's (u, v, w) as stored and the channel's scale.
__device__ __forceinline__ bool place_vals(const JobGeom &g, const ImgState &s, double um,
                                           double vm, double wm, double sc, Placed &pl) {
    double w = wm * sc;
    if (!(w >= s.w_min && w <= s.w_max)) return false;
    double u = um * sc, v = vm * sc;
    pl.x = mesh_coord(u, g.scale, g.half);
    pl.y = mesh_coord(v, g.scale, g.half);
    pl.i0 = (int)floor(pl.x + 0.5);
    pl.j0 = (int)floor(pl.y + 0.5);
    pl.k = plane_of(w, s.w_min, s.dw, s.inv_dw, g.n_w);
    return true;
}

__device__ __forceinline__ bool place(const JobGeom &g, const ImgState &s, const double *uvw,
                                      int64_t r, int c, Placed &pl) {
    return place_vals(g, s, uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], g.chan_scale[c], pl);
}

__device__ __forceinline__ int64_t bin_base(const JobGeom &g, int img, int kl) {
    return ((int64_t)img * g.n_pl + kl) << (2 * g.logNT);
}

// Bins touched by one element's footprint (0, 1, 2 or 4), in a fixed order.
struct Keys {
    int n;
    uint32_t k[4];
};

__device__ __forceinline__ bool has_key(const Keys &ks, uint32_t key) {
    bool f = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) f |= (i < ks.n) && ks.k[i] == key;
    return f;
}

// (channel, baseline, time block) of a track thread
struct Track {
    int c;
    int64_t b, t0, t1;
    bool ok;
};

__device__ __forceinline__ Track track_of(const JobGeom &g, int64_t idx) {
    Track tr;
    tr.c = (int)(idx % g.n_chan);
    int64_t rest = idx / g.n_chan;
    tr.b = rest % g.P;
    int64_t tb = rest / g.P;
    tr.t0 = tb * g.L;
    tr.t1 = min(g.n_t, tr.t0 + g.L);
    tr.ok = tb < g.n_tb;
    return tr;
}

template <bool F64W>
__global__ __launch_bounds__(kThreads) void k_count(JobGeom g, const double *__restrict__ uvw,
                                                    const void *__restrict__ wts,
                                                    const uint8_t *__restrict__ mask,
                                                    ImgState *st, uint32_t *__restrict__ counts) {
    __shared__ unsigned long long s_used[256];
    __shared__ double s_sumw[256];
    const int n_img = g.n_img;
    for (int i = threadIdx.x; i < n_img; i += blockDim.x) {
        s_used[i] = 0;
        s_sumw[i] = 0.0;
    }
    __syncthreads();
    const Track tr = track_of(g, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    const int img = (n_img > 1) ? tr.c : 0;
    unsigned long long nu = 0;
    double sw = 0.0;
    if (tr.ok) {
        const ImgState s = st[img];
        uint32_t okey[4] = {0, 0, 0, 0};
        uint32_t ocnt[4] = {0, 0, 0, 0};
        const double sc = g.chan_scale[tr.c];
        int64_t t_end = tr.t1;
        if (t_end > tr.t0 && (t_end - 1) * g.P + tr.b >= g.n_rows) t_end = (g.n_rows - 1 - tr.b) / g.P + 1;
        for (int64_t t0b = tr.t0; t0b < t_end; t0b += kBatch) {
        // the loads of kBatch elements are issued together
        uint8_t mb[kBatch];
        double ub[kBatch], vb[kBatch], wb[kBatch], wtb[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int64_t t = min(t0b + j, t_end - 1);
            const int64_t r = t * g.P + tr.b;
            const int64_t e = r * g.n_chan + tr.c;
            mb[j] = (t0b + j < t_end) ? mask[e] : 0;
            ub[j] = uvw[3 * r];
            vb[j] = uvw[3 * r + 1];
            wb[j] = uvw[3 * r + 2];
            wtb[j] = wts ? (F64W ? ((const double *)wts)[e] : (double)((const float *)wts)[e]) : 1.0;
        }
        for (int j = 0; j < kBatch && t0b + j < t_end; ++j) {
            Placed pl;
            Keys ks;
            ks.n = 0;
            const bool in_range = place_vals(g, s, ub[j], vb[j], wb[j], sc, pl);
            if (mb[j] && in_range) {
                ++nu;
                sw += wtb[j];
                int kl = pl.k - g.plane_lo;
                if (kl >= 0 && kl < g.n_pl) {
                    int64_t base = bin_base(g, img, kl);
                    int tx0 = (pl.i0 - g.h) >> g.logT, tx1 = (pl.i0 + g.h) >> g.logT;
                    int ty0 = (pl.j0 - g.h) >> g.logT, ty1 = (pl.j0 + g.h) >> g.logT;
                    for (int ty = ty0; ty <= ty1; ++ty)
                        for (int tx = tx0; tx <= tx1; ++tx)
                            ks.k[ks.n++] = (uint32_t)(base + (int64_t)ty * g.NT + tx);
                }
            }
            // close runs whose bin this element does not touch
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (ocnt[q] && !has_key(ks, okey[q])) {
                    atomicAdd(&counts[okey[q]], ocnt[q]);
                    ocnt[q] = 0;
                }
            // extend or open runs
            for (int i = 0; i < ks.n; ++i) {
                bool done = false;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (!done && ocnt[q] && okey[q] == ks.k[i]) {
                        ++ocnt[q];
                        done = true;
                    }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (!done && ocnt[q] == 0) {
                        okey[q] = ks.k[i];
                        ocnt[q] = 1;
                        done = true;
                    }
            }
        }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (ocnt[j]) atomicAdd(&counts[okey[j]], ocnt[j]);
    }
    if (n_img == 1) {
        for (int off = 32; off > 0; off >>= 1) {
            nu += __shfl_xor(nu, off);
            sw += __shfl_xor(sw, off);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&s_used[0], nu);
            atomicAdd(&s_sumw[0], sw);
        }
    } else if (tr.ok) {
        atomicAdd(&s_used[img], nu);
        atomicAdd(&s_sumw[img], sw);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_img; i += blockDim.x) {
        if (s_used[i]) {
            atomicAdd(&st[i].n_used, s_used[i]);
            atomicAdd(&st[i].sum_w, s_sumw[i]);
        }
    }
}

template <typename VT>
__device__ __forceinline__ void write_record(void *records, uint32_t slot, const JobGeom &g,
                                             const Placed &pl, uint32_t key, double vr, double vi,
                                             double wt) {
    uint32_t t = key & ((1u << (2 * g.logNT)) - 1u);
    int ty = (int)(t >> g.logNT), tx = (int)(t & (uint32_t)(g.NT - 1));
    double fx = pl.x - (double)pl.i0;
    double fy = pl.y - (double)pl.j0;
    if constexpr (sizeof(VT) == 8) {
        RecF64 rec;
        rec.fx = fx;
        rec.fy = fy;
        rec.re = wt * vr;
        rec.im = wt * vi;
        rec.li = pl.i0 - (tx << g.logT);
        rec.lj = pl.j0 - (ty << g.logT);
        ((RecF64 *)records)[slot] = rec;
    } else {
        uint32_t qx = (uint32_t)fmin((fx + 0.5) * 16777216.0 + 0.5, 16777215.0);
        uint32_t qy = (uint32_t)fmin((fy + 0.5) * 16777216.0 + 0.5, 16777215.0);
        RecF32 rec;
        rec.px = ((uint32_t)(pl.i0 - (tx << g.logT) + g.h) << kFracBits) | qx;
        rec.py = ((uint32_t)(pl.j0 - (ty << g.logT) + g.h) << kFracBits) | qy;
        rec.re = (float)wt * (float)vr;
        rec.im = (float)wt * (float)vi;
        ((RecF32 *)records)[slot] = rec;
    }
}

// The scatter walks the same tracks in blocks of kScatL time slices, in three
// phases with the same trip count on every lane (so no lane waits on another's
// inner loop):
//   1. the bins of each element, packed into one word, into LDS;
//   2. backwards through the block, the length of the run that starts at each
//      (element, bin);
//   3. forwards, one slot reservation per run (an atomic on the bin's cursor),
//      then the records.
constexpr int kScatThreads = 128;
constexpr int kScatL = 64;
constexpr uint32_t kNoKey = 0xffffffffu;

// base bin (lowest tile) in bits 0..26, bit 27: also the tile to the right, bit 28:
// also the tile above
__device__ __forceinline__ uint32_t pack_placed(const JobGeom &g, int img, const Placed &pl) {
    int kl = pl.k - g.plane_lo;
    if (kl < 0 || kl >= g.n_pl) return kNoKey;
    int tx0 = (pl.i0 - g.h) >> g.logT, tx1 = (pl.i0 + g.h) >> g.logT;
    int ty0 = (pl.j0 - g.h) >> g.logT, ty1 = (pl.j0 + g.h) >> g.logT;
    uint32_t base = (uint32_t)(bin_base(g, img, kl) + ((int64_t)ty0 << g.logNT) + tx0);
    return base | ((uint32_t)(tx1 > tx0) << 27) | ((uint32_t)(ty1 > ty0) << 28);
}

__device__ __forceinline__ void unpack_keys(uint32_t pk, int NT, Keys &ks) {
    ks.n = 0;
    if (pk == kNoKey) return;
    uint32_t b = pk & 0x7ffffffu;
    bool cx = (pk >> 27) & 1u, cy = (pk >> 28) & 1u;
    ks.k[ks.n++] = b;
    if (cx) ks.k[ks.n++] = b + 1;
    if (cy) ks.k[ks.n++] = b + (uint32_t)NT;
    if (cx && cy) ks.k[ks.n++] = b + (uint32_t)NT + 1;
}

template <typename VT>
__global__ __launch_bounds__(kScatThreads) void k_scatter(JobGeom g, const double *__restrict__ uvw,
                                                          const void *__restrict__ vis,
                                                          const void *__restrict__ wts,
                                                          const uint8_t *__restrict__ mask,
                                                          const ImgState *st, uint32_t *cursor,
                                                          void *__restrict__ records, uint32_t capacity,
                                                          uint32_t *overflow) {
    // one word per element: the packed bins (phase 1), then, in place, the 4 x
    // 8-bit run lengths (phase 2); phase 3 recomputes the bins
    __shared__ uint32_t s_key[kScatL][kScatThreads];
    const int lane = threadIdx.x;
    // track of this thread: blocks of kScatL time slices
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + lane;
    const int c = (int)(idx % g.n_chan);
    const int64_t rest = idx / g.n_chan;
    const int64_t b = rest % g.P;
    const int64_t tb = rest / g.P;
    const int64_t t0 = tb * kScatL;
    const bool ok = t0 < g.n_t;
    const int img = (g.n_img > 1) ? c : 0;
    const ImgState s = st[ok ? img : 0];
    int nt = 0;
    if (ok) {
        int64_t t1 = min(g.n_t, t0 + kScatL);
        for (int64_t t = t0; t < t1; ++t) {
            if (t * g.P + b >= g.n_rows) break;
            ++nt;
        }
    }
    const double sc = g.chan_scale[c];
    // phase 1: packed bins (the loads of kBatch elements are issued together)
    for (int k0 = 0; k0 < kScatL; k0 += kBatch) {
        uint8_t m[kBatch];
        double u[kBatch], v[kBatch], w[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int k = k0 + j;
            const bool in = k < nt;
            // clamped to a real row so that no load can leave the buffers
            const int64_t r = min((t0 + min(k, max(nt - 1, 0))) * g.P + b, g.n_rows - 1);
            m[j] = in ? mask[r * g.n_chan + c] : 0;
            u[j] = in ? uvw[3 * r] : 0.0;
            v[j] = in ? uvw[3 * r + 1] : 0.0;
            w[j] = in ? uvw[3 * r + 2] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            Placed pl;
            uint32_t pk = kNoKey;
            if (m[j] && place_vals(g, s, u[j], v[j], w[j], sc, pl)) pk = pack_placed(g, img, pl);
            s_key[k0 + j][lane] = pk;
        }
    }
    // phase 2: run lengths, backwards; `open` holds the bins of element k+1 with the
    // length of their run from k+1 on
    {
        uint32_t okey[4] = {kNoKey, kNoKey, kNoKey, kNoKey};
        uint32_t olen[4] = {0, 0, 0, 0};
        for (int k = kScatL - 1; k >= 0; --k) {
            Keys ks;
            unpack_keys(s_key[k][lane], g.NT, ks);
            uint32_t nkey[4] = {kNoKey, kNoKey, kNoKey, kNoKey};
            uint32_t nlen[4] = {0, 0, 0, 0};
            uint32_t packed = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= ks.n) continue;
                uint32_t len = 1;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (okey[j] == ks.k[i]) len = olen[j] + 1;
                nkey[i] = ks.k[i];
                nlen[i] = len;
                packed |= min(len, 255u) << (8 * i);
            }
            s_key[k][lane] = packed;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                okey[i] = nkey[i];
                olen[i] = nlen[i];
            }
        }
    }
    // phase 3: forwards, one reservation per run
    uint32_t okey[4] = {kNoKey, kNoKey, kNoKey, kNoKey};
    uint32_t onext[4] = {0, 0, 0, 0};
    uint32_t orem[4] = {0, 0, 0, 0};
    for (int k0 = 0; k0 < nt; k0 += kBatch) {
        uint8_t m[kBatch];
        double u[kBatch], v[kBatch], w[kBatch], vr[kBatch], vi[kBatch], wt[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int k = min(k0 + j, nt - 1);
            const int64_t r = (t0 + k) * g.P + b;
            const int64_t e = r * g.n_chan + c;
            m[j] = (k0 + j < nt) ? mask[e] : 0;
            u[j] = uvw[3 * r];
            v[j] = uvw[3 * r + 1];
            w[j] = uvw[3 * r + 2];
            ElemIO<VT, VT>::load(vis, wts, e, vr[j], vi[j], wt[j]);
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
        Placed pl;
        if (!m[j] || !place_vals(g, s, u[j], v[j], w[j], sc, pl)) continue;
        const uint32_t pk = pack_placed(g, img, pl);
        if (pk == kNoKey) continue;
        Keys ks;
        unpack_keys(pk, g.NT, ks);
        const uint32_t lens = s_key[k0 + j][lane];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i >= ks.n) continue;
            const uint32_t key = ks.k[i];
            uint32_t slot = 0;
            bool have = false;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (!have && orem[j] && okey[j] == key) {
                    slot = onext[j]++;
                    --orem[j];
                    have = true;
                }
            if (!have) {
                const uint32_t len = (lens >> (8 * i)) & 0xffu;
                const uint32_t base = atomicAdd(&cursor[key], len);
                slot = base;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (!have && orem[j] == 0) {
                        okey[j] = key;
                        onext[j] = base + 1;
                        orem[j] = len - 1;
                        have = true;
                    }
            }
            // the counting pass sized the buffer; a slot beyond it would mean the two
            // passes disagree: never write there, report it instead
            if (slot < capacity)
                write_record<VT>(records, slot, g, pl, key, vr[j], vi[j], wt[j]);
            else
                atomicAdd(overflow, 1u);
        }
        }
    }
}

// ---------------------------------------------------------------- scan
constexpr int kScanBlock = 1024;   // elements per block (256 threads x 4)

__global__ __launch_bounds__(256) void k_scan_block(const uint32_t *in, uint32_t *out, size_t n,
                                                    uint32_t *block_sums) {
    __shared__ uint32_t s[256];
    size_t base = (size_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t v[4];
    uint32_t sum = 0;
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        sum += v[i];
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - sum;   // exclusive prefix of this thread
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 255 && block_sums) block_sums[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t *out, size_t n, const uint32_t *block_off) {
    size_t base = (size_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t add = block_off[blockIdx.x];
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] += add;
}

__global__ void k_chunks(const uint32_t *counts, uint32_t *nchunk, size_t n, uint32_t chunk) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c = counts[i];
    // an empty bin has no work item: its tile is cleared by the zero pass
    nchunk[i] = (c + chunk - 1) / chunk;
}

__global__ void k_item_map(const uint32_t *nchunk, const uint32_t *item_off, uint32_t *item_bin,
                           size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t o = item_off[i];
    for (uint32_t c = 0; c < nchunk[i]; ++c) item_bin[o + c] = (uint32_t)i;
}

__global__ void k_post_norm(int n_img, ImgState *st, int normalize) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_img) return;
    double sw = st[i].sum_w;
    st[i].inv_norm = normalize ? (sw > 0.0 ? 1.0 / sw : 0.0) : 1.0;
}

}  // namespace

void launch_prep(const JobGeom &g, bool f64, const double *uvw, const void *vis, const void *wts,
                 const uint8_t *flags, uint8_t *mask, ImgState *st, hipStream_t s) {
    int64_t n_elem = g.n_rows * (int64_t)g.n_chan;
    if (n_elem == 0) return;
    int blocks = blocks_for(n_elem, g.n_chan);
    if (f64)
        k_prep<double><<<blocks, kThreads, 0, s>>>(g, uvw, vis, wts, flags, mask, st);
    else
        k_prep<float><<<blocks, kThreads, 0, s>>>(g, uvw, vis, wts, flags, mask, st);
}

void launch_finalize_range(const JobGeom &g, ImgState *st, hipStream_t s) {
    k_finalize<<<(g.n_img + 63) / 64, 64, 0, s>>>(g, st);
}

int64_t track_threads(const JobGeom &g) { return (int64_t)g.n_chan * g.P * g.n_tb; }

void launch_count(const JobGeom &g, const double *uvw, const void *wts, bool f64,
                  const uint8_t *mask, ImgState *st, uint32_t *counts, hipStream_t s) {
    int64_t n_elem = g.n_rows * (int64_t)g.n_chan;
    if (n_elem == 0) return;
    unsigned blocks = (unsigned)((track_threads(g) + kThreads - 1) / kThreads);
    if (f64)
        k_count<true><<<blocks, kThreads, 0, s>>>(g, uvw, wts, mask, st, counts);
    else
        k_count<false><<<blocks, kThreads, 0, s>>>(g, uvw, wts, mask, st, counts);
}

void launch_scatter(const JobGeom &g, const double *uvw, const void *vis, const void *wts,
                    bool f64, const uint8_t *mask, const ImgState *st, uint32_t *cursor,
                    void *records, uint32_t capacity, uint32_t *overflow, hipStream_t s) {
    int64_t n_elem = g.n_rows * (int64_t)g.n_chan;
    if (n_elem == 0) return;
    int64_t threads = (int64_t)g.n_chan * g.P * ((g.n_t + kScatL - 1) / kScatL);
    unsigned blocks = (unsigned)((threads + kScatThreads - 1) / kScatThreads);
    if (f64)
        k_scatter<double><<<blocks, kScatThreads, 0, s>>>(g, uvw, vis, wts, mask, st, cursor,
                                                          records, capacity, overflow);
    else
        k_scatter<float><<<blocks, kScatThreads, 0, s>>>(g, uvw, vis, wts, mask, st, cursor,
                                                         records, capacity, overflow);
}

size_t scan_tmp_elems(size_t n) {
    size_t total = 0;
    while (n > (size_t)kScanBlock) {
        size_t nb = (n + kScanBlock - 1) / kScanBlock;
        total += 2 * nb;   // block sums and their scan
        n = nb;
    }
    return total + 1;
}

void launch_scan(const uint32_t *in, uint32_t *out, size_t n, uint32_t *tmp, hipStream_t s) {
    if (n == 0) return;
    size_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb == 1) {
        k_scan_block<<<1, 256, 0, s>>>(in, out, n, nullptr);
        return;
    }
    uint32_t *sums = tmp;
    uint32_t *sums_scan = tmp + nb;
    k_scan_block<<<(unsigned)nb, 256, 0, s>>>(in, out, n, sums);
    launch_scan(sums, sums_scan, nb, tmp + 2 * nb, s);
    k_scan_add<<<(unsigned)nb, 256, 0, s>>>(out, n, sums_scan);
}

void launch_chunks(const uint32_t *counts, uint32_t *nchunk, size_t n_bins, uint32_t chunk,
                   hipStream_t s) {
    k_chunks<<<(unsigned)((n_bins + 255) / 256), 256, 0, s>>>(counts, nchunk, n_bins, chunk);
}

void launch_item_map(const uint32_t *nchunk, const uint32_t *item_off, uint32_t *item_bin,
                     size_t n_bins, hipStream_t s) {
    k_item_map<<<(unsigned)((n_bins + 255) / 256), 256, 0, s>>>(nchunk, item_off, item_bin, n_bins);
}

void launch_post_norm(int n_img, ImgState *st, bool normalize, hipStream_t s) {
    k_post_norm<<<(n_img + 63) / 64, 64, 0, s>>>(n_img, st, normalize ? 1 : 0);
}

}  // namespace wsg
