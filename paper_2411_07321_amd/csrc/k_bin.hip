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
#pragma clang fp contract(off)
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
    // every product and difference rounded on its own (no contraction), so that both
    // binning passes, and the oracle, take the same decisions
#pragma clang fp contract(off)
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

// One binning thread: kStretch consecutive time slices of the track of baseline
// b (rows t*P + b) in channel c.  Consecutive threads take consecutive channels,
// then baselines, so that the loads of a wave fall on neighbouring rows.
struct Stretch {
    int c;
    int64_t b, t0, t_end;   // time slices [t0, t_end)
    bool ok;
};

__device__ __forceinline__ Stretch stretch_of(const JobGeom &g, int64_t idx) {
    Stretch sr;
    sr.c = (int)(idx % g.n_chan);
    const int64_t rest = idx / g.n_chan;
    sr.b = rest % g.P;
    const int64_t tb = rest / g.P;
    sr.ok = tb < g.n_tb;
    sr.t0 = tb * kStretch;
    int64_t t1 = min(g.n_t, sr.t0 + kStretch);
    // the last time slice may be short of P rows
    if (sr.ok && t1 > sr.t0 && (t1 - 1) * g.P + sr.b >= g.n_rows) t1 = (g.n_rows - 1 - sr.b) / g.P + 1;
    sr.t_end = sr.ok ? max(t1, sr.t0) : sr.t0;
    return sr;
}

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

// the 1, 2 or 4 bins in a fixed order: base, then right or above, then above,
// then above-right (positions are static, so the keys stay in registers)
__device__ __forceinline__ void unpack_keys(uint32_t pk, int NT, Keys &ks) {
    const uint32_t b = pk & 0x7ffffffu;
    const bool cx = (pk >> 27) & 1u, cy = (pk >> 28) & 1u;
    ks.k[0] = b;
    ks.k[1] = cx ? b + 1u : b + (uint32_t)NT;
    ks.k[2] = b + (uint32_t)NT;
    ks.k[3] = b + (uint32_t)NT + 1u;
    ks.n = pk == kNoKey ? 0 : (cx && cy) ? 4 : (cx || cy) ? 2 : 1;
}

constexpr int kBinThreads = 256;

// Counting pass.  Along its stretch a thread tracks runs of elements with the
// same packed bins (a track moves slowly, so runs are long) and adds each run to
// its private table of (bin, records) in LDS; a table that would exceed kTab
// bins sends the rest of the stretch's runs straight to the global counts.  At
// the end the table goes to `counts` (one atomic per entry) and, for the
// scatter, to tab / tab_n.
template <bool F64W>
__global__ __launch_bounds__(kBinThreads) void k_count(JobGeom g, const double *__restrict__ uvw,
                                                       const void *__restrict__ wts,
                                                       const uint8_t *__restrict__ mask,
                                                       ImgState *st, uint32_t *__restrict__ cls_counts,
                                                       int n_cls, TabEntry *__restrict__ tab,
                                                       uint32_t *__restrict__ tab_n) {
    __shared__ uint32_t s_tb[kTab][kBinThreads];
    __shared__ uint32_t s_tc[kTab][kBinThreads];
    __shared__ unsigned long long s_used[256];
    __shared__ double s_sumw[256];
    const int n_img = g.n_img;
    const int lane = threadIdx.x;
    for (int i = lane; i < n_img; i += blockDim.x) {
        s_used[i] = 0;
        s_sumw[i] = 0.0;
    }
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + lane;
    const Stretch sr = stretch_of(g, idx);
    const int img = (n_img > 1) ? sr.c : 0;
    const size_t n_bins = (size_t)g.n_img * g.n_pl << (2 * g.logNT);
    uint32_t *counts = cls_counts + (size_t)(blockIdx.x % (unsigned)n_cls) * n_bins;
    unsigned long long nu = 0;
    double sw = 0.0;
    if (sr.ok) {
        const ImgState s = st[img];
        const double sc = g.chan_scale[sr.c];
        int n_ent = 0;
        bool ovf = false;
        uint32_t cur = kNoKey, run = 0;
        bool cur_tab = false;
        Keys cks;
        cks.n = 0;
        int ent[4] = {0, 0, 0, 0};
        for (int64_t t0b = sr.t0; t0b < sr.t_end; t0b += kBatch) {
            // the loads of kBatch elements are issued together
            uint8_t mb[kBatch];
            double ub[kBatch], vb[kBatch], wb[kBatch], wtb[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                const int64_t t = min(t0b + j, sr.t_end - 1);
                const int64_t r = t * g.P + sr.b;
                const int64_t e = r * g.n_chan + sr.c;
                mb[j] = (t0b + j < sr.t_end) ? mask[e] : 0;
                ub[j] = uvw[3 * r];
                vb[j] = uvw[3 * r + 1];
                wb[j] = uvw[3 * r + 2];
                wtb[j] = wts ? (F64W ? ((const double *)wts)[e] : (double)((const float *)wts)[e]) : 1.0;
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                Placed pl;
                uint32_t pk = kNoKey;
                if (mb[j] && place_vals(g, s, ub[j], vb[j], wb[j], sc, pl)) {
                    ++nu;
                    sw += wtb[j];
                    pk = pack_placed(g, img, pl);
                }
                if (pk != cur) {
                    // close the run of `cur`
                    if (run) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (i >= cks.n) continue;
                            if (cur_tab) s_tc[ent[i]][lane] += run;
                            else atomicAdd(&counts[cks.k[i]], run);
                        }
                    }
                    // open a run of `pk`: its bins in the table, added when missing
                    cur = pk;
                    run = 0;
                    unpack_keys(pk, g.NT, cks);
                    cur_tab = !ovf;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (i >= cks.n || !cur_tab) continue;
                        int f = -1;
                        for (int e = 0; e < n_ent; ++e)
                            if (s_tb[e][lane] == cks.k[i]) f = e;
                        if (f < 0) {
                            if (n_ent < kTab) {
                                f = n_ent++;
                                s_tb[f][lane] = cks.k[i];
                                s_tc[f][lane] = 0u;
                            } else {
                                ovf = true;
                                cur_tab = false;
                            }
                        }
                        ent[i] = f;
                    }
                }
                if (pk != kNoKey) ++run;
            }
        }
        if (run) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= cks.n) continue;
                if (cur_tab) s_tc[ent[i]][lane] += run;
                else atomicAdd(&counts[cks.k[i]], run);
            }
        }
        for (int e = 0; e < n_ent; ++e) {
            const uint32_t bin = s_tb[e][lane], n = s_tc[e][lane];
            if (n) atomicAdd(&counts[bin], n);
            tab[idx * kTab + e] = TabEntry{bin, n};
        }
        tab_n[idx] = ovf ? kTabOverflow : (uint32_t)n_ent;
    }
    if (n_img == 1) {
        for (int off = 32; off > 0; off >>= 1) {
            nu += __shfl_xor(nu, off);
            sw += __shfl_xor(sw, off);
        }
        if ((lane & 63) == 0) {
            atomicAdd(&s_used[0], nu);
            atomicAdd(&s_sumw[0], sw);
        }
    } else if (sr.ok) {
        atomicAdd(&s_used[img], nu);
        atomicAdd(&s_sumw[img], sw);
    }
    __syncthreads();
    for (int i = lane; i < n_img; i += blockDim.x) {
        if (s_used[i]) {
            atomicAdd(&st[i].n_used, s_used[i]);
            atomicAdd(&st[i].sum_w, s_sumw[i]);
        }
    }
}

// Scatter.  A thread reserves, for each (bin, records) pair its stretch left in
// the table, one range of slots (one atomic on the bin's cursor), then walks the
// stretch once more and writes each record into the next slot of its bin, so the
// records of one stretch are contiguous, in time order, inside every bin they
// reach.  An overflowed stretch reserves record by record.
template <typename VT>
__global__ __launch_bounds__(kBinThreads) void k_scatter(JobGeom g, const double *__restrict__ uvw,
                                                         const void *__restrict__ vis,
                                                         const void *__restrict__ wts,
                                                         const uint8_t *__restrict__ mask,
                                                         const ImgState *st, uint32_t *cls_cursor,
                                                         int n_cls, const TabEntry *__restrict__ tab,
                                                         const uint32_t *__restrict__ tab_n,
                                                         void *__restrict__ records, uint32_t capacity,
                                                         uint32_t *overflow) {
    __shared__ uint32_t s_tb[kTab][kBinThreads];
    __shared__ uint32_t s_tn[kTab][kBinThreads];   // next free slot of the entry's bin
    const int lane = threadIdx.x;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + lane;
    const Stretch sr = stretch_of(g, idx);
    if (!sr.ok) return;   // no barrier below
    const size_t n_bins = (size_t)g.n_img * g.n_pl << (2 * g.logNT);
    uint32_t *cursor = cls_cursor + (size_t)(blockIdx.x % (unsigned)n_cls) * n_bins;
    const int img = (g.n_img > 1) ? sr.c : 0;
    const ImgState s = st[img];
    const double sc = g.chan_scale[sr.c];
    const uint32_t tn = tab_n[idx];
    const bool ovf = tn == kTabOverflow;
    const int n_ent = ovf ? 0 : (int)tn;
    for (int e = 0; e < n_ent; ++e) {
        const TabEntry te = tab[idx * kTab + e];
        s_tb[e][lane] = te.bin;
        s_tn[e][lane] = te.n ? atomicAdd(&cursor[te.bin], te.n) : 0u;
    }
    uint32_t cur = kNoKey;
    Keys ks;
    ks.n = 0;
    int ent[4] = {-1, -1, -1, -1};
    for (int64_t t0b = sr.t0; t0b < sr.t_end; t0b += kBatch) {
        uint8_t m[kBatch];
        double u[kBatch], v[kBatch], w[kBatch], vr[kBatch], vi[kBatch], wt[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int64_t t = min(t0b + j, sr.t_end - 1);
            const int64_t r = t * g.P + sr.b;
            const int64_t e = r * g.n_chan + sr.c;
            m[j] = (t0b + j < sr.t_end) ? mask[e] : 0;
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
            if (pk != cur) {
                cur = pk;
                unpack_keys(pk, g.NT, ks);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int f = -1;
                    if (i < ks.n && !ovf)
                        for (int e = 0; e < n_ent; ++e)
                            if (s_tb[e][lane] == ks.k[i]) f = e;
                    ent[i] = f;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= ks.n) continue;
                uint32_t slot;
                if (ovf) {
                    slot = atomicAdd(&cursor[ks.k[i]], 1u);
                } else if (ent[i] >= 0) {
                    slot = s_tn[ent[i]][lane];
                    s_tn[ent[i]][lane] = slot + 1u;
                } else {
                    slot = capacity;   // the passes disagree: reported below
                }
                // the counting pass sized the buffer; a slot beyond it would mean the
                // two passes disagree: never write there, report it instead
                if (slot < capacity)
                    write_record<VT>(records, slot, g, pl, ks.k[i], vr[j], vi[j], wt[j]);
                else
                    atomicAdd(overflow, 1u);
            }
        }
    }
}

__global__ void k_class_totals(const uint32_t *__restrict__ cls_counts, int n_cls, size_t n_bins,
                               uint32_t *__restrict__ counts) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n_bins) return;
    uint32_t t = 0;
    if (i < n_bins)
        for (int c = 0; c < n_cls; ++c) t += cls_counts[(size_t)c * n_bins + i];
    counts[i] = t;   // the entry after the last bin stays 0: its offset is the total
}

__global__ void k_class_cursors(const uint32_t *__restrict__ cls_counts, int n_cls, size_t n_bins,
                                const uint32_t *__restrict__ offsets,
                                uint32_t *__restrict__ cls_cursor) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_bins) return;
    uint32_t run = offsets[i];
    for (int c = 0; c < n_cls; ++c) {
        cls_cursor[(size_t)c * n_bins + i] = run;
        run += cls_counts[(size_t)c * n_bins + i];
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

int64_t stretch_threads(int64_t n_chan, int64_t P, int64_t n_tb) { return n_chan * P * n_tb; }

int binning_classes(size_t n_bins) { return n_bins <= ((size_t)1 << 22) ? kMaxClasses : 1; }

void launch_count(const JobGeom &g, const double *uvw, const void *wts, bool f64,
                  const uint8_t *mask, ImgState *st, uint32_t *cls_counts, int n_cls,
                  TabEntry *tab, uint32_t *tab_n, hipStream_t s) {
    const int64_t n = stretch_threads(g.n_chan, g.P, g.n_tb);
    if (n == 0) return;
    const unsigned blocks = (unsigned)((n + kBinThreads - 1) / kBinThreads);
    if (f64)
        k_count<true><<<blocks, kBinThreads, 0, s>>>(g, uvw, wts, mask, st, cls_counts, n_cls, tab, tab_n);
    else
        k_count<false><<<blocks, kBinThreads, 0, s>>>(g, uvw, wts, mask, st, cls_counts, n_cls, tab, tab_n);
}

void launch_class_totals(const uint32_t *cls_counts, int n_cls, size_t n_bins, uint32_t *counts,
                         hipStream_t s) {
    k_class_totals<<<(unsigned)((n_bins + 1 + 255) / 256), 256, 0, s>>>(cls_counts, n_cls, n_bins, counts);
}

void launch_class_cursors(const uint32_t *cls_counts, int n_cls, size_t n_bins,
                          const uint32_t *offsets, uint32_t *cls_cursor, hipStream_t s) {
    if (n_bins == 0) return;
    k_class_cursors<<<(unsigned)((n_bins + 255) / 256), 256, 0, s>>>(cls_counts, n_cls, n_bins, offsets,
                                                                    cls_cursor);
}

void launch_scatter(const JobGeom &g, const double *uvw, const void *vis, const void *wts,
                    bool f64, const uint8_t *mask, const ImgState *st, uint32_t *cls_cursor,
                    int n_cls, const TabEntry *tab, const uint32_t *tab_n, void *records,
                    uint32_t capacity, uint32_t *overflow, hipStream_t s) {
    const int64_t n = stretch_threads(g.n_chan, g.P, g.n_tb);
    if (n == 0) return;
    const unsigned blocks = (unsigned)((n + kBinThreads - 1) / kBinThreads);
    if (f64)
        k_scatter<double><<<blocks, kBinThreads, 0, s>>>(g, uvw, vis, wts, mask, st, cls_cursor, n_cls,
                                                         tab, tab_n, records, capacity, overflow);
    else
        k_scatter<float><<<blocks, kBinThreads, 0, s>>>(g, uvw, vis, wts, mask, st, cls_cursor, n_cls,
                                                        tab, tab_n, records, capacity, overflow);
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
