// Binning of visibilities by (image, w-plane, uv tile): a counting sort.
//
// Sec. 2 of the paper groups the visibilities of each mesh slab into a bucket of
// their own before the convolution.  Here the buckets are
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
// the row period (baselines per time slice); a stretch is one (baseline,
// channel) track over kStretch consecutive time slices.  A workgroup first
// reads 16 stretches x 64 time slices with coalesced loads (consecutive
// threads, consecutive rows of one time slice) and places every element into
// an LDS table; then each wave takes whole stretches, one time slice per lane.
// A track moves slowly across the mesh, so consecutive lanes of a wave mostly
// hold the same bins: each run of lanes with the same bin takes one global
// atomic (the runs of a wave are found with shuffles and two ballots, and all
// of them issue their atomics together), and the scatter writes a run's
// records to consecutive slots.  This matters because the uv coverage is
// extremely uneven: the short baselines of a dense core all land in the few
// central tiles, where per-element atomics would serialise; the atomics are
// further spread over per-class copies of the counters (workgroup index mod
// the class count).  Records of one stretch stay contiguous inside their bin.
#include "wsg_internal.h"

#include <algorithm>

namespace wsg {

namespace {

constexpr int kThreads = 256;

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

__device__ __forceinline__ bool is_finite(double a) { return isfinite(a); }

// An empty statement that takes x and may change it: the compiler has to hold the
// loaded value here and cannot move its load into the branch that uses it.  Applied
// to every value of a thread's slots, it keeps all their loads in flight together
// instead of one slot's loads after another's.
__device__ __forceinline__ void pin(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(float &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(uint32_t &x) { asm volatile("" : "+v"(x)); }

// Every test but the flag and the w range (O2 of the method's reading), on the
// row's stored (u, v, w), the channel's scale, the visibility and its weight.
__device__ __forceinline__ bool valid_vals(const JobGeom &g, double um, double vm, double wm, double sc,
                                           double vr, double vi, double wt, double &w_out) {
    if (!(wt > 0.0) || !is_finite(wt)) return false;
    double u = um * sc, v = vm * sc, w = wm * sc;
    if (!is_finite(u) || !is_finite(v) || !is_finite(w)) return false;
    if (g.w_fold && wm < 0.0) {
        u = -u;
        v = -v;
        w = -w;
    }
    if (!is_finite(vr) || !is_finite(vi)) return false;
    int i0, j0;
    if (!footprint_fits(mesh_coord(u, g.scale, g.half), g.N, g.h, i0)) return false;
    if (!footprint_fits(mesh_coord(v, g.scale, g.half), g.N, g.h, j0)) return false;
    w_out = w;
    return true;
}


// elements a thread of the generic validity pass loads at once
constexpr int kPrepUnroll = 4;

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
    __shared__ unsigned long long s_min[256], s_max[256], s_flag[256], s_valid[256], s_used[256];
    __shared__ double s_sumw[256];
    const int n_img = g.n_img;
    for (int i = threadIdx.x; i < n_img; i += blockDim.x) {
        s_min[i] = ~0ull;
        s_max[i] = 0ull;
        s_flag[i] = 0;
        s_valid[i] = 0;
        s_used[i] = 0;
        s_sumw[i] = 0.0;
    }
    __syncthreads();
    const int64_t n_elem = g.n_rows * (int64_t)g.n_chan;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long kmin = ~0ull, kmax = 0ull, nf = 0, nv = 0, nu = 0;
    double sw = 0.0;
    const int c = (int)(e0 % g.n_chan);
    // the stride is a multiple of n_chan: the row advances by a constant
    const int64_t dr = stride / g.n_chan;
    int64_t r = e0 / g.n_chan;
    // kPrepUnroll elements per iteration, every load issued before any is used (a slot
    // past the data repeats the first element of the iteration and is skipped)
    constexpr int U = kPrepUnroll;
    const double sc = g.chan_scale[c];
    const VT *vsrc = (const VT *)vis;
    const VT *wsrc = wts ? (const VT *)wts : vsrc;   // without weights: read and replaced by 1
    for (int64_t e = e0; e < n_elem; e += U * stride, r += U * dr) {
        double um[U], vm[U], wm[U];
        VT vr[U], vi[U], wv[U];
        uint32_t fv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = e + u * stride < n_elem;
            const int64_t ee = in ? e + u * stride : e, rr = in ? r + u * dr : r;
            fv[u] = flags ? (uint32_t)flags[ee] : 0u;
            vr[u] = vsrc[2 * ee];
            vi[u] = vsrc[2 * ee + 1];
            wv[u] = wsrc[ee];
            um[u] = uvw[3 * rr];
            vm[u] = uvw[3 * rr + 1];
            wm[u] = uvw[3 * rr + 2];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pin(fv[u]);
            pin(vr[u]);
            pin(vi[u]);
            pin(wv[u]);
            pin(um[u]);
            pin(vm[u]);
            pin(wm[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
        if (e + u * stride >= n_elem) break;
        const bool fl = fv[u] != 0u;
        double w = 0.0;
        const double wt = wts ? (double)wv[u] : 1.0;
        const bool ok = !fl && valid_vals(g, um[u], vm[u], wm[u], sc, (double)vr[u], (double)vi[u], wt, w);
        mask[e + u * stride] = ok ? 1 : 0;
        nf += fl ? 1 : 0;
        if (ok) {
            ++nv;
            unsigned long long k = order_key(w);
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
            // used: valid and inside the w range (the data's own range holds every
            // valid visibility; a given range may not)
            if (!g.range_given || (w >= g.w_min_given && w <= g.w_max_given)) {
                ++nu;
                sw += wt;
            }
        }
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
            nu += __shfl_xor(nu, off);
            sw += __shfl_xor(sw, off);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin(&s_min[0], kmin);
            atomicMax(&s_max[0], kmax);
            atomicAdd(&s_flag[0], nf);
            atomicAdd(&s_valid[0], nv);
            atomicAdd(&s_used[0], nu);
            atomicAdd(&s_sumw[0], sw);
        }
    } else {
        atomicMin(&s_min[img], kmin);
        atomicMax(&s_max[img], kmax);
        atomicAdd(&s_flag[img], nf);
        atomicAdd(&s_valid[img], nv);
        atomicAdd(&s_used[img], nu);
        atomicAdd(&s_sumw[img], sw);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_img; i += blockDim.x) {
        if (s_valid[i]) {
            atomicMin(&st[i].wmin_key, s_min[i]);
            atomicMax(&st[i].wmax_key, s_max[i]);
            atomicAdd(&st[i].n_valid0, s_valid[i]);
        }
        if (s_used[i]) {
            atomicAdd(&st[i].n_used, s_used[i]);
            atomicAdd(&st[i].sum_w, s_sumw[i]);
        }
        if (s_flag[i]) atomicAdd(&st[i].n_flagged, s_flag[i]);
    }
}

// The validity pass of a single-image complex64 job with NC = 1, 2 or 4 channels, one
// thread per row: the row's (u, v, w) is loaded once for all its channels, and the
// channels' visibilities, weights, flags and mask bytes move in one vector access each.
template <int NC>
struct RowVec;
template <> struct RowVec<1> { using V = float2; using W = float; using F = uint8_t; };
template <> struct RowVec<2> { using V = float4; using W = float2; using F = uint16_t; };
template <> struct RowVec<4> { using V = float4; using W = float4; using F = uint32_t; };

template <int NC>
__global__ __launch_bounds__(kThreads) void k_prep_rows(JobGeom g, const double *__restrict__ uvw,
                                                        const float *__restrict__ vis,
                                                        const float *__restrict__ wts,
                                                        const uint8_t *__restrict__ flags,
                                                        uint8_t *__restrict__ mask, ImgState *st) {
    using RV = RowVec<NC>;
    __shared__ unsigned long long s_min, s_max, s_flag, s_valid, s_used;
    __shared__ double s_sumw;
    if (threadIdx.x == 0) {
        s_min = ~0ull;
        s_max = 0ull;
        s_flag = s_valid = s_used = 0ull;
        s_sumw = 0.0;
    }
    __syncthreads();
    unsigned long long kmin = ~0ull, kmax = 0ull, nf = 0, nv = 0, nu = 0;
    double sw = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < g.n_rows; r += stride) {
        const double um = uvw[3 * r], vm = uvw[3 * r + 1], wm = uvw[3 * r + 2];
        float vv[2 * NC], ww[NC];
        if constexpr (NC == 4) {
            const float4 a = ((const float4 *)vis)[2 * r], b = ((const float4 *)vis)[2 * r + 1];
            vv[0] = a.x; vv[1] = a.y; vv[2] = a.z; vv[3] = a.w;
            vv[4] = b.x; vv[5] = b.y; vv[6] = b.z; vv[7] = b.w;
        } else if constexpr (NC == 2) {
            const float4 a = ((const float4 *)vis)[r];
            vv[0] = a.x; vv[1] = a.y; vv[2] = a.z; vv[3] = a.w;
        } else {
            const float2 a = ((const float2 *)vis)[r];
            vv[0] = a.x; vv[1] = a.y;
        }
        if (wts) {
            const typename RV::W x = ((const typename RV::W *)wts)[r];
            if constexpr (NC == 4) { ww[0] = x.x; ww[1] = x.y; ww[2] = x.z; ww[3] = x.w; }
            else if constexpr (NC == 2) { ww[0] = x.x; ww[1] = x.y; }
            else { ww[0] = x; }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) ww[c] = 1.0f;
        }
        typename RV::F fl = 0;
        if (flags) fl = ((const typename RV::F *)flags)[r];
        typename RV::F m = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if ((fl >> (8 * c)) & 0xffu) {
                ++nf;
                continue;
            }
            double w;
            if (!valid_vals(g, um, vm, wm, g.chan_scale[c], (double)vv[2 * c], (double)vv[2 * c + 1],
                            (double)ww[c], w))
                continue;
            m |= (typename RV::F)(1u << (8 * c));
            ++nv;
            const unsigned long long k = order_key(w);
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
            if (!g.range_given || (w >= g.w_min_given && w <= g.w_max_given)) {
                ++nu;
                sw += (double)ww[c];
            }
        }
        ((typename RV::F *)mask)[r] = m;
    }
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long a = __shfl_xor(kmin, off);
        unsigned long long b = __shfl_xor(kmax, off);
        kmin = a < kmin ? a : kmin;
        kmax = b > kmax ? b : kmax;
        nf += __shfl_xor(nf, off);
        nv += __shfl_xor(nv, off);
        nu += __shfl_xor(nu, off);
        sw += __shfl_xor(sw, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&s_min, kmin);
        atomicMax(&s_max, kmax);
        atomicAdd(&s_flag, nf);
        atomicAdd(&s_valid, nv);
        atomicAdd(&s_used, nu);
        atomicAdd(&s_sumw, sw);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_valid) {
            atomicMin(&st[0].wmin_key, s_min);
            atomicMax(&st[0].wmax_key, s_max);
            atomicAdd(&st[0].n_valid0, s_valid);
        }
        if (s_used) {
            atomicAdd(&st[0].n_used, s_used);
            atomicAdd(&st[0].sum_w, s_sumw);
        }
        if (s_flag) atomicAdd(&st[0].n_flagged, s_flag);
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
    // with a kernel in w over 2 w_h + 1 planes the range covers the middle
    // N_w - 2 w_h planes, and w_h more on each side take the kernel's tails
    s.dw = (hi - lo) / (double)(g.n_w - 2 * g.w_h);
    s.w0 = lo - (double)g.w_h * s.dw;
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
    if (__builtin_expect(f < 1e-9 || f > 1.0 - 1e-9, 0)) q = d / dw;
    int k = (int)floor(q);
    return k > n_w - 1 ? n_w - 1 : k;
}

struct Placed {
    int k;
    int i0, j0;
    double x, y;
    double w;      // w in wavelengths (folded)
    bool flip;     // folded: the visibility is conjugated
};

// A valid element inside the w range: its plane, nearest cell and position, from
// the row's (u, v, w) as stored and the channel's scale.
__device__ __forceinline__ bool place_vals(const JobGeom &g, const ImgState &s, double um,
                                           double vm, double wm, double sc, Placed &pl) {
    // every product and difference rounded on its own (no contraction), so that both
    // binning passes, and the oracle, take the same decisions
#pragma clang fp contract(off)
    // w-folding: a row with w < 0 is the Hermitian mirror (-u, -v, -w), conj(V); the
    // negations are exact, so the decisions match those of the unfolded products
    pl.flip = g.w_fold && wm < 0.0;
    if (pl.flip) {
        um = -um;
        vm = -vm;
        wm = -wm;
    }
    double w = wm * sc;
    if (!(w >= s.w_min && w <= s.w_max)) return false;
    double u = um * sc, v = vm * sc;
    pl.x = mesh_coord(u, g.scale, g.half);
    pl.y = mesh_coord(v, g.scale, g.half);
    pl.i0 = (int)floor(pl.x + 0.5);
    pl.j0 = (int)floor(pl.y + 0.5);
    pl.k = plane_of(w, s.w0, s.dw, s.inv_dw, g.n_w);
    // a kernel in w needs its whole support inside the stack: a w at the very edge
    // of the range may round into the padding
    if (g.w_h && s.dw > 0.0) pl.k = min(max(pl.k, g.w_h), g.n_w - 1 - g.w_h);
    pl.w = w;
    return true;
}

__device__ __forceinline__ int64_t bin_base(const JobGeom &g, int img, int kl) {
    return ((int64_t)img * g.n_pl + kl) << (2 * g.logNT);
}

// Bins touched by one element's footprint (0, 1, 2 or 4), in a fixed order.
struct Keys {
    int n;
    uint32_t k[4];
};


constexpr uint32_t kNoKey = 0xffffffffu;
// bit 29 of a packed element: its visibility spreads over the planes of the kernel
// in w (set only where the image's plane width is not 0)
constexpr uint32_t kSpread = 1u << 29;

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

// Binning works on tiles of kBinStretches stretches (kStretch = 64 consecutive
// time slices of one (baseline, channel) track each) per workgroup.
//   Phase A reads the tile coalesced: consecutive threads take consecutive
//   stretches of one time slice, which are neighbouring elements in memory.
//   Each element leaves its packed bins (and, for the scatter, the parts of its
//   record that do not depend on the tile) in LDS.
//   Phase B gives each wave whole stretches, one time slice per lane: the
//   elements of a stretch that share a bin are counted with one ballot and get
//   one atomic, and their records take consecutive slots, in time order,
//   written by consecutive lanes.
// Consecutive workgroups run on one XCD, so rows they share meet in its L2.
constexpr int kBinThreads = 256;
constexpr int kBinStretches = 16;
constexpr int kPitch = kBinStretches + 1;              // LDS row pitch (no bank conflicts)
constexpr int kTileElems = kStretch * kPitch;
constexpr int kPerThread = kStretch * kBinStretches / kBinThreads;   // 4
constexpr int kPerWave = kBinStretches / (kBinThreads / 64);         // 4

__device__ __forceinline__ int64_t bin_block(int64_t bid, int64_t n_blocks) {
    // workgroups are dealt to the 8 XCDs round robin
    constexpr int kXcd = 8;
    if (n_blocks % kXcd) return bid;
    return (bid % kXcd) * (n_blocks / kXcd) + bid / kXcd;
}

// Row and element of one time slice of one stretch, in 32-bit arithmetic like the
// stretch position: a job holds at most 2^29 visibilities (the values of a slice past
// the data are not used)
struct Slice {
    int c;
    uint32_t r, e;
    bool ok;
};

// (channel, baseline, time block) of a stretch, in 32-bit arithmetic: a job holds
// at most 2^29 visibilities, so stretch indices stay far below 2^32 (64-bit
// division is a long software sequence on the GPU)
struct StretchPos {
    int c;
    uint32_t b, tb;
    bool ok;
};

__device__ __forceinline__ StretchPos stretch_pos(const JobGeom &g, uint32_t stretch) {
    StretchPos p;
    const uint32_t nc = (uint32_t)g.n_chan;
    p.c = (int)(stretch % nc);
    const uint32_t rest = stretch / nc;
    p.b = rest % (uint32_t)g.P;
    p.tb = rest / (uint32_t)g.P;
    p.ok = p.tb < (uint32_t)g.n_tb;
    return p;
}

__device__ __forceinline__ Slice slice_at(const JobGeom &g, const StretchPos &p, int t_in) {
    Slice sl;
    sl.c = p.c;
    const uint32_t t = p.tb * (uint32_t)kStretch + (uint32_t)t_in;
    sl.r = t * (uint32_t)g.P + p.b;
    sl.ok = p.ok && t < (uint32_t)g.n_t && sl.r < (uint32_t)g.n_rows;
    sl.e = sl.r * (uint32_t)g.n_chan + (uint32_t)sl.c;
    return sl;
}

// phase-A slot k of a thread: stretch s (the same for every k, as kBinThreads is a
// multiple of kBinStretches) and time slice t within the tile
__device__ __forceinline__ void tile_slot(int k, int &t, int &s) {
    const int q = threadIdx.x + k * kBinThreads;
    t = q / kBinStretches;
    s = q - t * kBinStretches;
}
static_assert(kBinThreads % kBinStretches == 0, "phase A keeps one stretch per thread");

// The keys of a wave, slot by slot (a lane's first key, then its second, ...), as
// runs of consecutive lanes (consecutive time slices of one track) holding the same
// key; where all lanes holding a slot hold one key, they are one run even with gaps
// (lanes without the slot between them).  f(key, len, head_lane, rank, head, mine) is called by every lane for every
// slot in use: `head` marks a run's first lane, `len` its length there, and `rank`
// is the lane's position in its run.  All runs of a slot are handled by the same
// instructions, so a wave takes one atomic round trip per slot, not per bin.  f also
// receives the slot index i first (a compile-time-unrolled constant).
template <typename F>
__device__ __forceinline__ void for_each_run(const Keys &ks, int lane, F &&f) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool has = i < ks.n;
        const unsigned long long hm = __ballot(has);
        if (hm == 0ull) break;   // slots are filled in order
        const uint32_t key = has ? ks.k[i] : kNoKey;
        // common case along a track: every lane holding slot i holds the same bin, and
        // those lanes (in time order, gaps allowed) form one run
        const int fl = __ffsll((long long)hm) - 1;
        const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, fl);   // fl is uniform
        if (__ballot(has && key != k0) == 0ull) {
            const uint32_t rank = (uint32_t)__popcll(hm & ((1ull << lane) - 1ull));
            const bool head = lane == fl;
            f(i, key, head ? (uint32_t)__popcll(hm) : 0u, fl, rank, head, has);
            continue;
        }
        const uint32_t prev = (uint32_t)__shfl_up((int)key, 1);
        const uint32_t next = (uint32_t)__shfl_down((int)key, 1);
        const bool head = has && (lane == 0 || prev != key);
        const bool tail = has && (lane == 63 || next != key);
        const unsigned long long heads = __ballot(head), tails = __ballot(tail);
        const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const unsigned long long from = ~((1ull << lane) - 1ull);
        const unsigned long long hu = heads & upto;
        const int hl = has && hu ? 63 - __clzll((long long)hu) : lane;
        const int tl = __ffsll((long long)(tails & from)) - 1;
        const uint32_t len = head ? (uint32_t)(tl - lane + 1) : 0u;
        f(i, key, len, hl, (uint32_t)(lane - hl), head, has);
    }
}

// sub-cell offset f in [-1/2, 1/2) as 24-bit fixed point
__device__ __forceinline__ uint32_t quant_frac(double f) {
    return (uint32_t)fmin((f + 0.5) * 16777216.0 + 0.5, 16777215.0);
}
// and, for the complex128 mesh, the 52 mantissa bits of f + 3/2 (the sum is exact
// where f has no bits below 2^-52)
__device__ __forceinline__ uint64_t quant_frac64(double f) {
    return (uint64_t)__double_as_longlong(f + 1.5) & kFracMask64;
}

// Counting pass: records per bin, into the workgroup's atomic class.
// Keys of plane offset dk: every bin of the element moved dk planes (a whole
// plane of tiles per step); none for dk != 0 unless the element spreads.
__device__ __forceinline__ Keys plane_keys(const Keys &ks, uint32_t pk, int dk, int logNT) {
    Keys kd = ks;
    if (dk != 0) {
        if (pk == kNoKey || !(pk & kSpread)) kd.n = 0;
        const uint32_t shift = (uint32_t)dk << (2 * logNT);
#pragma unroll
        for (int i = 0; i < 4; ++i) kd.k[i] = ks.k[i] + shift;
    }
    return kd;
}

template <bool WK>
__global__ __launch_bounds__(kBinThreads) void k_count(JobGeom g, const double *__restrict__ uvw,
                                                       const uint8_t *__restrict__ mask,
                                                       const ImgState *st,
                                                       uint32_t *__restrict__ cls_counts, int n_cls) {
    __shared__ uint32_t s_pk[kTileElems];
    const int64_t blk = bin_block(blockIdx.x, gridDim.x);
    const int64_t s0 = blk * kBinStretches;
    const StretchPos pos = stretch_pos(g, (uint32_t)(s0 + (int)threadIdx.x % kBinStretches));
    // every element of a thread belongs to its stretch: one channel, one image
    const int img = (g.n_img > 1) ? pos.c : 0;
    const ImgState sti = st[img];
    const double sc = g.chan_scale[pos.c];
    // phase A: all loads first, none of them conditional (a slot past the data reads
    // element 0 and is masked afterwards), so that they are all in flight together
    Slice sl[kPerThread];
    uint8_t mk[kPerThread];
    double u[kPerThread], v[kPerThread], w[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int t, s;
        tile_slot(k, t, s);
        sl[k] = slice_at(g, pos, t);
        const uint32_t r = sl[k].ok ? sl[k].r : 0u;
        const uint32_t e = sl[k].ok ? sl[k].e : 0u;
        mk[k] = mask[e];
        u[k] = uvw[3 * r];
        v[k] = uvw[3 * r + 1];
        w[k] = uvw[3 * r + 2];
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        uint32_t m = mk[k];
        pin(m);
        pin(u[k]);
        pin(v[k]);
        pin(w[k]);
        mk[k] = sl[k].ok ? (uint8_t)m : (uint8_t)0;
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int t, s;
        tile_slot(k, t, s);
        uint32_t pk = kNoKey;
        Placed pl;
        if (mk[k] && place_vals(g, sti, u[k], v[k], w[k], sc, pl)) {
            pk = pack_placed(g, img, pl);
            if (WK && pk != kNoKey && sti.dw > 0.0) pk |= kSpread;
        }
        s_pk[t * kPitch + s] = pk;
    }
    __syncthreads();
    // phase B
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t n_bins = (size_t)g.n_img * g.n_pl << (2 * g.logNT);
    uint32_t *counts = cls_counts + (size_t)(blk % n_cls) * n_bins;
    for (int j = 0; j < kPerWave; ++j) {
        const int s = wave * kPerWave + j;
        Keys ks;
        const uint32_t pk = s_pk[lane * kPitch + s];
        unpack_keys(pk, g.NT, ks);
        const int hw = WK ? g.w_h : 0;
        for (int dk = -hw; dk <= hw; ++dk) {
            const Keys kd = WK ? plane_keys(ks, pk, dk, g.logNT) : ks;
            for_each_run(kd, lane, [&](int, uint32_t bin, uint32_t len, int, uint32_t, bool head, bool) {
                if (head) atomicAdd(&counts[bin], len);
            });
        }
    }
}

// Scatter: each bin of a stretch reserves its records' slots with one atomic
// on the class cursor; the records go to consecutive slots in time order.
// The LDS holds, per element, the packed bins and the record without its tile:
// complex64 mesh: 24-bit sub-cell offsets with the cell relative to the lowest
// tile in the top byte, and W V; complex128 mesh: FP64 offsets, W V and the cell
// relative to the lowest tile.
template <typename VT>
struct ScatterLds;
template <>
struct ScatterLds<float> {
    uint32_t pk[kTileElems], a[kTileElems], b[kTileElems];
    float re[kTileElems], im[kTileElems];
};
template <>
struct ScatterLds<double> {
    uint32_t pk[kTileElems];
    uint64_t a[kTileElems], b[kTileElems];
    double re[kTileElems], im[kTileElems];
};

// with a kernel in w, also the element's w and its plane and image (k0 | img << 16)
template <typename VT, bool WK>
struct ScatterLdsW : ScatterLds<VT> {};
template <typename VT>
struct ScatterLdsW<VT, true> : ScatterLds<VT> {
    double wv[kTileElems];
    uint32_t kimg[kTileElems];
};

// Slot reservation per workgroup: each wave lists the runs of its stretches (bin and
// length) in its part of an LDS run list, the workgroup's threads then reserve the
// slots of every listed run with parallel atomics (one round trip for the whole
// workgroup instead of one per key slot of every stretch), and each wave finally walks
// its stretches again, in the same order, to write the records from the returned
// bases.  Runs beyond a wave's kWaveRuns entries reserve their slots on the spot.
constexpr int kWaveRuns = 32;
constexpr int kRunList = kWaveRuns * (kBinThreads / 64);
struct RunList {
    uint32_t bin[kRunList];
    uint32_t val[kRunList];    // run length, then the first slot reserved for it
    int n[kBinThreads / 64];   // listed runs per wave
};

// (w_k - w) / dw for plane k, each operation rounded on its own: the Kaiser-Bessel
// window is cut off at |d| = S_w / 2 with a non-zero value there, and the data's own
// extreme w values fall exactly on plane edges, so d must round as the method's
// reference rounds it
__device__ __forceinline__ double plane_offset(const ImgState &s, int k, double w) {
#pragma clang fp contract(off)
    const double wk = s.w0 + ((double)k + 0.5) * s.dw;
    return (wk - w) / s.dw;
}

// waves per SIMD to plan registers for: the complex64 scatter's LDS leaves room
// for 7 workgroups per CU, and more waves in flight hide the latency of its slot
// reservations (4.5 -> 3.95 ms on config 1 against the register count the
// compiler picks by itself)
template <typename VT, bool WK>
struct ScatterWaves { static constexpr int value = (sizeof(VT) == 4 && !WK) ? 7 : 1; };

template <typename VT, bool WK>
__global__ __launch_bounds__(kBinThreads) __attribute__((amdgpu_waves_per_eu(ScatterWaves<VT, WK>::value)))
void k_scatter(JobGeom g, const double *__restrict__ uvw,
                                                         const void *__restrict__ vis,
                                                         const void *__restrict__ wts,
                                                         const uint8_t *__restrict__ mask,
                                                         const ImgState *st, uint32_t *cls_cursor,
                                                         int n_cls, void *__restrict__ records,
                                                         uint32_t capacity, uint32_t *overflow) {
    __shared__ ScatterLdsW<VT, WK> L;
    __shared__ RunList R;
    const int64_t blk = bin_block(blockIdx.x, gridDim.x);
    const int64_t s0 = blk * kBinStretches;
    const StretchPos pos = stretch_pos(g, (uint32_t)(s0 + (int)threadIdx.x % kBinStretches));
    // every element of a thread belongs to its stretch: one channel, one image
    const int img = (g.n_img > 1) ? pos.c : 0;
    const ImgState sti = st[img];
    const double sc = g.chan_scale[pos.c];
    Slice sl[kPerThread];
    uint8_t mk[kPerThread];
    double u[kPerThread], v[kPerThread], w[kPerThread];
    VT vr[kPerThread], vi[kPerThread], wt[kPerThread];   // in the visibilities' own type
    // every load issued before any is used (a slot past the data reads element 0 and
    // is masked afterwards); without weights the load goes to the visibilities, which
    // hold at least as many elements, and is replaced by 1
    const VT *wsrc = wts ? (const VT *)wts : (const VT *)vis;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int t, s;
        tile_slot(k, t, s);
        sl[k] = slice_at(g, pos, t);
        const uint32_t r = sl[k].ok ? sl[k].r : 0u;
        const uint32_t e = sl[k].ok ? sl[k].e : 0u;
        mk[k] = mask[e];
        u[k] = uvw[3 * r];
        v[k] = uvw[3 * r + 1];
        w[k] = uvw[3 * r + 2];
        vr[k] = ((const VT *)vis)[2 * e];
        vi[k] = ((const VT *)vis)[2 * e + 1];
        wt[k] = wsrc[e];
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        uint32_t m = mk[k];
        pin(m);
        pin(u[k]);
        pin(v[k]);
        pin(w[k]);
        pin(vr[k]);
        pin(vi[k]);
        pin(wt[k]);
        if (!wts) wt[k] = VT(1);
        mk[k] = sl[k].ok ? (uint8_t)m : (uint8_t)0;
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        int t, s;
        tile_slot(k, t, s);
        uint32_t pk = kNoKey;
        Placed pl;
        if (mk[k] && place_vals(g, sti, u[k], v[k], w[k], sc, pl)) {
            pk = pack_placed(g, img, pl);
            if constexpr (WK) {
                if (pk != kNoKey && sti.dw > 0.0) {
                    pk |= kSpread;
                    L.wv[t * kPitch + s] = pl.w;
                    L.kimg[t * kPitch + s] = (uint32_t)pl.k | ((uint32_t)img << 16);
                }
            }
        }
        const int q = t * kPitch + s;
        L.pk[q] = pk;
        if (pk != kNoKey) {
            // cell relative to the lowest tile the footprint reaches
            const int li0 = pl.i0 - (((pl.i0 - g.h) >> g.logT) << g.logT);
            const int lj0 = pl.j0 - (((pl.j0 - g.h) >> g.logT) << g.logT);
            const double fx = pl.x - (double)pl.i0, fy = pl.y - (double)pl.j0;
            if constexpr (sizeof(VT) == 8) {
                L.a[q] = quant_frac64(fx) | ((uint64_t)li0 << kFracBits64);
                L.b[q] = quant_frac64(fy) | ((uint64_t)lj0 << kFracBits64);
                L.re[q] = wt[k] * vr[k];
                L.im[q] = pl.flip ? -(wt[k] * vi[k]) : wt[k] * vi[k];
            } else {
                L.a[q] = quant_frac(fx) | ((uint32_t)li0 << kFracBits);
                L.b[q] = quant_frac(fy) | ((uint32_t)lj0 << kFracBits);
                L.re[q] = wt[k] * vr[k];
                L.im[q] = pl.flip ? -(wt[k] * vi[k]) : wt[k] * vi[k];
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t n_bins = (size_t)g.n_img * g.n_pl << (2 * g.logNT);
    uint32_t *cursor = cls_cursor + (size_t)(blk % n_cls) * n_bins;
    const uint32_t tmask = (1u << (2 * g.logNT)) - 1u;
    // the record of element q in bin `bin` (plane weight gw) at `slot`
    auto put = [&](int q, uint32_t pk, uint32_t bin, uint32_t slot, double gw) {
        // the counting pass sized the buffer; a slot beyond it would mean the two
        // passes disagree: never write there, report it instead
        if (slot >= capacity) {
            atomicAdd(overflow, 1u);
            return;
        }
        const uint32_t tb0 = pk & tmask;   // lowest tile of the footprint
        const int tx0 = (int)(tb0 & (uint32_t)(g.NT - 1)), ty0 = (int)(tb0 >> g.logNT);
        const uint32_t tt = bin & tmask;
        const int dx = (int)(tt & (uint32_t)(g.NT - 1)) - tx0, dy = (int)(tt >> g.logNT) - ty0;
        if constexpr (sizeof(VT) == 8) {
            const uint64_t a = L.a[q], b = L.b[q];
            RecF64 rec;
            rec.px = (((a >> kFracBits64) - ((uint64_t)dx << g.logT) + (uint64_t)g.h) << kFracBits64) |
                     (a & kFracMask64);
            rec.py = (((b >> kFracBits64) - ((uint64_t)dy << g.logT) + (uint64_t)g.h) << kFracBits64) |
                     (b & kFracMask64);
            rec.re = WK ? L.re[q] * gw : L.re[q];
            rec.im = WK ? L.im[q] * gw : L.im[q];
            ((RecF64 *)records)[slot] = rec;
        } else {
            const uint32_t a = L.a[q], b = L.b[q];
            RecF32 rec;
            rec.px = (((a >> kFracBits) - ((uint32_t)dx << g.logT) + (uint32_t)g.h) << kFracBits) |
                     (a & 0xffffffu);
            rec.py = (((b >> kFracBits) - ((uint32_t)dy << g.logT) + (uint32_t)g.h) << kFracBits) |
                     (b & 0xffffffu);
            rec.re = WK ? L.re[q] * (float)gw : L.re[q];
            rec.im = WK ? L.im[q] * (float)gw : L.im[q];
            ((RecF32 *)records)[slot] = rec;
        }
    };
    const unsigned long long below = (1ull << lane) - 1ull;
    // list the runs of the wave's stretches (heads in lane order, slots in order)
    int nr = 0;
    for (int j = 0; j < kPerWave; ++j) {
        const int s = wave * kPerWave + j;
        const uint32_t pk = L.pk[lane * kPitch + s];
        Keys ks;
        unpack_keys(pk, g.NT, ks);
        const int hw = WK ? g.w_h : 0;
        for (int dk = -hw; dk <= hw; ++dk) {
            const Keys kd = WK ? plane_keys(ks, pk, dk, g.logNT) : ks;
            for_each_run(kd, lane, [&](int, uint32_t bin, uint32_t len, int, uint32_t, bool head, bool) {
                const unsigned long long heads = __ballot(head);
                const int e = nr + __popcll(heads & below);
                if (head && e < kWaveRuns) {
                    R.bin[wave * kWaveRuns + e] = bin;
                    R.val[wave * kWaveRuns + e] = len;
                }
                nr += __popcll(heads);
            });
        }
    }
    if (lane == 0) R.n[wave] = nr < kWaveRuns ? nr : kWaveRuns;
    __syncthreads();
    // reserve the slots of every listed run of the workgroup at once
    for (int e = threadIdx.x; e < kRunList; e += kBinThreads)
        if (e % kWaveRuns < R.n[e / kWaveRuns]) R.val[e] = atomicAdd(&cursor[R.bin[e]], R.val[e]);
    __syncthreads();
    // the same walk again: every lane's record goes to its run's first slot + its rank
    nr = 0;
    for (int j = 0; j < kPerWave; ++j) {
        const int s = wave * kPerWave + j;
        const int q = lane * kPitch + s;
        const uint32_t pk = L.pk[q];
        Keys ks;
        unpack_keys(pk, g.NT, ks);
        const int hw = WK ? g.w_h : 0;
        for (int dk = -hw; dk <= hw; ++dk) {
            // weight of plane k0 + dk under the kernel in w (1 without one)
            double gw = 1.0;
            if constexpr (WK)
                if (pk != kNoKey && (pk & kSpread)) {
                    const uint32_t ki = L.kimg[q];
                    gw = w_weight(g, plane_offset(st[ki >> 16], (int)(ki & 0xffffu) + dk, L.wv[q]));
                }
            const Keys kd = WK ? plane_keys(ks, pk, dk, g.logNT) : ks;
            for_each_run(kd, lane, [&](int, uint32_t bin, uint32_t len, int hl, uint32_t rank, bool head,
                                       bool mine) {
                const unsigned long long heads = __ballot(head);
                // list entry of the run this lane belongs to (its head's)
                const int eh = nr + __popcll(heads & ((1ull << hl) - 1ull));
                nr += __popcll(heads);
                const bool listed = eh < kWaveRuns;
                uint32_t late = 0u;
                if (head && !listed) late = atomicAdd(&cursor[bin], len);
                late = (uint32_t)__shfl((int)late, hl);
                if (!mine) return;
                const uint32_t base = listed ? R.val[wave * kWaveRuns + eh] : late;
                put(q, pk, bin, base + rank, gw);
            });
        }
    }
}

// size class of a work item of n >= 1 records: floor(log2(n))
__device__ __forceinline__ int item_class(uint32_t n) { return 31 - __clz((int)n); }

// pieces of a bin of cnt records: full pieces of kGridChunk, then the rest
__device__ __forceinline__ uint32_t bin_pieces(uint32_t cnt) {
    return (cnt + kGridChunk - 1u) / kGridChunk;
}

__global__ __launch_bounds__(256) void k_class_totals(const uint32_t *__restrict__ cls_counts,
                                                      int n_cls, size_t n_bins,
                                                      uint32_t *__restrict__ counts) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n_bins) return;
    uint32_t t = 0;
    if (i < n_bins)
        for (int c = 0; c < n_cls; ++c) t += cls_counts[(size_t)c * n_bins + i];
    counts[i] = t;   // the entry after the last bin stays 0: its offset is the total
}

// records of bin i if its plane lies in the stack window, else 0
__device__ __forceinline__ uint32_t window_count(const JobGeom &g, const uint32_t *__restrict__ counts,
                                                 size_t i, size_t n_bins) {
    if (i >= n_bins) return 0u;
    const int kl = (int)((i >> (2 * g.logNT)) % (uint32_t)g.n_pl);
    if (kl < g.stack_k0 || kl >= g.stack_k0 + g.stack_pl) return 0u;
    return counts[i];
}

__global__ __launch_bounds__(256) void k_item_hist(JobGeom g, const uint32_t *__restrict__ counts,
                                                   size_t n_bins, WorkTotals *wt) {
    __shared__ uint32_t s_hist[kItemClasses];
    if (threadIdx.x < kItemClasses) s_hist[threadIdx.x] = 0u;
    __syncthreads();
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t t = window_count(g, counts, i, n_bins);
    if (t) {
        const uint32_t np = bin_pieces(t);
        if (np > 1u) atomicAdd(&s_hist[kItemClasses - 1], np - 1u);
        atomicAdd(&s_hist[item_class(t - (np - 1u) * kGridChunk)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kItemClasses && s_hist[threadIdx.x])
        atomicAdd(&wt->cls_count[threadIdx.x], s_hist[threadIdx.x]);
}

// Class bases, largest class first; the cursors start at the bases.
__global__ void k_item_bases(const uint32_t *__restrict__ offsets, size_t n_bins, WorkTotals *wt) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0u;
    for (int c = kItemClasses - 1; c >= 0; --c) {
        wt->cls_cursor[c] = run;
        run += wt->cls_count[c];
    }
    wt->n_items = run;
    wt->n_records = offsets[n_bins];
    wt->next_item = 0u;
}

// Every piece of every non-empty bin takes a slot of its class: slots are reserved
// per workgroup (one global atomic per class) and dealt out through LDS.
__global__ __launch_bounds__(256) void k_item_place(JobGeom g, const uint32_t *__restrict__ counts,
                                                    size_t n_bins, WorkTotals *wt,
                                                    uint2 *__restrict__ items) {
    __shared__ uint32_t s_cnt[kItemClasses], s_base[kItemClasses];
    if (threadIdx.x < kItemClasses) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t t = window_count(g, counts, i, n_bins);
    const uint32_t np = t ? bin_pieces(t) : 0u;
    const int cl = t ? item_class(t - (np - 1u) * kGridChunk) : 0;
    uint32_t full_at = 0u, last_at = 0u;
    if (np > 1u) full_at = atomicAdd(&s_cnt[kItemClasses - 1], np - 1u);
    if (np) last_at = atomicAdd(&s_cnt[cl], 1u);
    __syncthreads();
    if (threadIdx.x < kItemClasses)
        s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(&wt->cls_cursor[threadIdx.x], s_cnt[threadIdx.x])
                                                 : 0u;
    __syncthreads();
    if (!np) return;
    const uint32_t b = (uint32_t)i;
    for (uint32_t c = 0; c + 1u < np; ++c)
        items[s_base[kItemClasses - 1] + full_at + c] = make_uint2(b, c);
    items[s_base[cl] + last_at] = make_uint2(b, np - 1u);
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct ScaleArgs {
    int n;
    double v[64];
};
__global__ void k_set_scales(double *__restrict__ dst, ScaleArgs a) {
    const int i = threadIdx.x;
    if (i < a.n) dst[i] = a.v[i];
}

__global__ void k_init_state(ImgState *st, int n_img) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_img) return;
    ImgState z{};
    z.wmin_key = ~0ull;
    z.wmax_key = 0ull;
    st[i] = z;
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
    // single complex64 image of 1, 2 or 4 channels with aligned rows: a thread per row
    const int nc = g.n_chan;
    const auto aligned = [](const void *p, size_t a) { return ((uintptr_t)p % a) == 0; };
    if (!f64 && g.n_img == 1 && (nc == 1 || nc == 2 || nc == 4) && aligned(vis, 8 * nc) &&
        aligned(wts, 4 * nc) && aligned(flags, nc) && aligned(mask, nc)) {
        const unsigned blocks = (unsigned)std::min<int64_t>((g.n_rows + kThreads - 1) / kThreads, 4096);
        const float *vf = (const float *)vis, *wf = (const float *)wts;
        if (nc == 4) k_prep_rows<4><<<blocks, kThreads, 0, s>>>(g, uvw, vf, wf, flags, mask, st);
        else if (nc == 2) k_prep_rows<2><<<blocks, kThreads, 0, s>>>(g, uvw, vf, wf, flags, mask, st);
        else k_prep_rows<1><<<blocks, kThreads, 0, s>>>(g, uvw, vf, wf, flags, mask, st);
        return;
    }
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

static unsigned binning_blocks(const JobGeom &g) {
    const int64_t n = stretch_threads(g.n_chan, g.P, g.n_tb);
    return (unsigned)((n + kBinStretches - 1) / kBinStretches);
}

void launch_count(const JobGeom &g, const double *uvw, const uint8_t *mask, const ImgState *st,
                  uint32_t *cls_counts, int n_cls, hipStream_t s) {
    const unsigned blocks = binning_blocks(g);
    if (blocks == 0) return;
    if (g.w_h > 0)
        k_count<true><<<blocks, kBinThreads, 0, s>>>(g, uvw, mask, st, cls_counts, n_cls);
    else
        k_count<false><<<blocks, kBinThreads, 0, s>>>(g, uvw, mask, st, cls_counts, n_cls);
}

void launch_class_totals(const uint32_t *cls_counts, int n_cls, size_t n_bins, uint32_t *counts,
                         hipStream_t s) {
    k_class_totals<<<(unsigned)((n_bins + 1 + 255) / 256), 256, 0, s>>>(cls_counts, n_cls, n_bins, counts);
}

void launch_work_list(const JobGeom &g, const uint32_t *counts, const uint32_t *offsets,
                      size_t n_bins, WorkTotals *wt, uint2 *items, hipStream_t s) {
    launch_fill_u32((uint32_t *)((char *)wt + offsetof(WorkTotals, cls_count)), kItemClasses, 0u, s);
    const unsigned blocks = (unsigned)std::max<size_t>((n_bins + 255) / 256, 1);
    k_item_hist<<<blocks, 256, 0, s>>>(g, counts, n_bins, wt);
    k_item_bases<<<1, 64, 0, s>>>(offsets, n_bins, wt);
    k_item_place<<<blocks, 256, 0, s>>>(g, counts, n_bins, wt, items);
}

void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    k_fill_u32<<<blocks, 256, 0, s>>>(p, n, v);
}

void launch_set_scales(double *dst, const double *vals, int n, hipStream_t s) {
    ScaleArgs a{};
    a.n = n < 64 ? n : 64;
    for (int i = 0; i < a.n; ++i) a.v[i] = vals[i];
    k_set_scales<<<1, 64, 0, s>>>(dst, a);
}

void launch_init_state(ImgState *st, int n_img, hipStream_t s) {
    if (n_img <= 0) return;
    k_init_state<<<(n_img + 63) / 64, 64, 0, s>>>(st, n_img);
}

void launch_class_cursors(const uint32_t *cls_counts, int n_cls, size_t n_bins,
                          const uint32_t *offsets, uint32_t *cls_cursor, hipStream_t s) {
    if (n_bins == 0) return;
    k_class_cursors<<<(unsigned)((n_bins + 255) / 256), 256, 0, s>>>(cls_counts, n_cls, n_bins, offsets,
                                                                    cls_cursor);
}

void launch_scatter(const JobGeom &g, const double *uvw, const void *vis, const void *wts,
                    bool f64, const uint8_t *mask, const ImgState *st, uint32_t *cls_cursor,
                    int n_cls, void *records, uint32_t capacity, uint32_t *overflow, hipStream_t s) {
    const unsigned blocks = binning_blocks(g);
    if (blocks == 0) return;
#define WSG_SCATTER(VT, WK)                                                                        \
    k_scatter<VT, WK><<<blocks, kBinThreads, 0, s>>>(g, uvw, vis, wts, mask, st, cls_cursor, n_cls, \
                                                     records, capacity, overflow)
    if (f64) {
        if (g.w_h > 0) WSG_SCATTER(double, true); else WSG_SCATTER(double, false);
    } else {
        if (g.w_h > 0) WSG_SCATTER(float, true); else WSG_SCATTER(float, false);
    }
#undef WSG_SCATTER
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

void launch_post_norm(int n_img, ImgState *st, bool normalize, hipStream_t s) {
    k_post_norm<<<(n_img + 63) / 64, 64, 0, s>>>(n_img, st, normalize ? 1 : 0);
}

}  // namespace wsg
