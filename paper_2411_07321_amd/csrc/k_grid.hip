// Convolutional gridding (Eq. 3 of the paper) of binned records.
//
// One work item = one non-empty (image, plane, tile) bin, or one chunk of a bin
// that holds more than `chunk` records.  The workgroup accumulates its records into
// an LDS copy of the T x T tile (every record adds W V G(i0+a-x) G(j0+b-y) to
// the cells of its S x S footprint that lie inside the tile), then writes the
// tile to the plane stack with coalesced stores.  A tile covered by a single
// chunk is stored (every cell of the stack is written exactly once, so the
// stack needs no clearing); the chunks of a split bin add their partial tiles
// with global atomics into a tile that k_zero_tiles cleared.  Empty bins get no
// work item: k_zero_tiles writes their tiles with plain stores, without LDS.
//
// G is separable: 2*S kernel values per record, S^2 multiply-adds.  KIND 0 is the
// Gaussian exp(-d^2 / (2 sigma^2)), KIND 1 the Kaiser-Bessel window
// I0(beta sqrt(1 - (2d/S)^2)) / I0(beta) that the paper's runs use (Sec. 2, after
// Eq. 3), from the tables described with KbTable.
#include "wsg_internal.h"

#include <algorithm>

namespace wsg {

namespace {

constexpr int kGridThreads = 256;
constexpr int kRunCap = 16;
constexpr int kFlushLanes = 60;

template <typename T>
struct RecTraits;

template <>
struct RecTraits<float> {
    using Rec = RecF32;
    static __device__ __forceinline__ void decode(const Rec &r, int h, int &li, int &lj, float &fx,
                                                  float &fy, float &re, float &im) {
        li = (int)(r.px >> kFracBits) - h;
        lj = (int)(r.py >> kFracBits) - h;
        fx = (float)(r.px & 0xffffffu) * (1.0f / kFracScale) - 0.5f;
        fy = (float)(r.py & 0xffffffu) * (1.0f / kFracScale) - 0.5f;
        re = r.re;
        im = r.im;
    }
    // exp(-d^2/(2 sigma^2)) as one hardware exp2 of -(d^2) * log2(e)/(2 sigma^2); the
    // argument's rounding gives a relative error of ~3e-7, far below the tolerance of
    // the FP32 mesh
    static __device__ __forceinline__ float gauss(float d, float inv2s2) {
        return __builtin_amdgcn_exp2f(-(d * d) * (inv2s2 * 1.4426950408889634f));
    }
};

template <>
struct RecTraits<double> {
    using Rec = RecF64;
    static __device__ __forceinline__ void decode(const Rec &r, int h, int &li, int &lj, double &fx,
                                                  double &fy, double &re, double &im) {
        li = (int)(r.px >> kFracBits64) - h;
        lj = (int)(r.py >> kFracBits64) - h;
        // f + 3/2 rebuilt from its mantissa bits; the difference is exact
        fx = __longlong_as_double((long long)((r.px & kFracMask64) | kOneBits64)) - 1.5;
        fy = __longlong_as_double((long long)((r.py & kFracMask64) | kOneBits64)) - 1.5;
        re = r.re;
        im = r.im;
    }
    static __device__ __forceinline__ double gauss(double d, double inv2s2) { return exp(-d * d * inv2s2); }
};

// G(k - f) for k = -H..H (g[H + k]) from three exponentials:
//   exp(-(k - f)^2 / (2 sigma^2)) = e^{-c f^2} * (e^{2 c f})^k * e^{-c k^2},  c = 1/(2 sigma^2)
// (cl2 = c log2(e), q[k] = e^{-c k^2}).  For |f| <= 1/2 the powers of e^{+-2cf} stay within
// [e^{-3c}, e^{3c}], and each value carries at most three more roundings than
// a direct evaluation, ~4e-7 relative in FP32.
template <int SS>
__device__ __forceinline__ void gauss_line(float f, float cl2, const float *q, float *g) {
    constexpr int H = (SS - 1) / 2;
    const float e0 = __builtin_amdgcn_exp2f(-(f * f) * cl2);
    const float r = __builtin_amdgcn_exp2f((2.0f * f) * cl2);
    const float ri = __builtin_amdgcn_exp2f((-2.0f * f) * cl2);
    g[H] = e0;
    float pp = e0, pm = e0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        pp *= r;
        pm *= ri;
        g[H + k] = pp * q[k];
        g[H - k] = pm * q[k];
    }
}

// The same recurrence in FP64 (q[k] = e^{-c k^2}, c = 1/(2 sigma^2)) without the taps'
// common factor e^{-c f^2}, which the caller takes for both axes at once
// (exp(-c (fx^2 + fy^2)), folded into W V): g[H + k] = r^k q[k] and g[H - k] = r^-k q[k],
// r = e^{2 c f} and its inverse by division, so a record takes three exponentials
// rather than six.  No tap exceeds 1 (2 c f k - c k^2 <= 0 for |f| <= 1/2, k >= 1).
template <int SS>
__device__ __forceinline__ void gauss_ratio_line64(double f, double c, const double *q, double *g) {
    constexpr int H = (SS - 1) / 2;
    const double r = exp((2.0 * f) * c);
    const double ri = 1.0 / r;
    g[H] = 1.0;
    double pp = 1.0, pm = 1.0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        pp *= r;
        pm *= ri;
        g[H + k] = pp * q[k];
        g[H - k] = pm * q[k];
    }
}

// Kaiser-Bessel taps g[a] = G((a - H) - f), a = 0..SS-1, on an FP32 mesh: tap a and
// tap SS-1-a are one fitted polynomial at x = 2f and at -x, E(x^2) +- x O(x^2).
template <int SS>
__device__ __forceinline__ void kb_line(float f, const float *__restrict__ poly, float *g) {
    constexpr int H = (SS - 1) / 2;
    const float x = 2.0f * f, x2 = x * x;
#pragma unroll
    for (int a = 0; a <= H; ++a) {
        const float *c = poly + a * kKbStride;
        float e = c[kKbEven - 1];
#pragma unroll
        for (int k = kKbEven - 2; k >= 0; --k) e = __builtin_fmaf(e, x2, c[k]);
        if (a == H) {
            g[H] = e;
        } else {
            float o = c[kKbStride - 1];
#pragma unroll
            for (int k = kKbOdd - 2; k >= 0; --k) o = __builtin_fmaf(o, x2, c[kKbEven + k]);
            o *= x;
            g[a] = e + o;
            g[SS - 1 - a] = e - o;
        }
    }
}

__device__ __forceinline__ void bin_coords(const JobGeom &g, uint32_t b, int &img, int &kl, int &ty,
                                           int &tx) {
    uint32_t per_plane = (uint32_t)g.NT * g.NT;
    uint32_t pl = b / per_plane;
    uint32_t t = b - pl * per_plane;
    ty = (int)(t / g.NT);
    tx = (int)(t - (uint32_t)ty * g.NT);
    img = (int)(pl / g.n_pl);
    kl = (int)(pl - (uint32_t)img * g.n_pl);
}

// cell (i, j) of plane kl (counted from plane_lo) of image img in the stack, which
// holds planes [stack_k0, stack_k0 + stack_pl) of every image
template <typename T>
__device__ __forceinline__ size_t cell_index(const JobGeom &g, int img, int kl, int i, int j,
                                             bool transposed) {
    size_t plane = ((size_t)img * g.stack_pl + (kl - g.stack_k0)) * (size_t)g.N * g.N;
    return plane + (transposed ? ((size_t)i * g.N + j) : ((size_t)j * g.N + i));
}

// LDS tile: separate real / imaginary FP64 arrays of T rows of TP = T + 8 cells, the
// last 8 of each row padding, and 8 more cells before the first row, so that every
// column from -8 to T + 7 of a row lies inside the arrays (columns outside the tile
// land in padding, which is never read).
//
// Each lane takes a contiguous stretch of the work item's records.  The
// binning pass keeps the records of one track (one baseline and channel over
// consecutive times) contiguous inside a bin, and a track moves slowly, so
// consecutive records of a lane have nearby nearest cells.  With ACC (complex64
// mesh, S <= 7) the lane sums the footprint values of such records in an
// (S+2) x (S+2) register window and adds it to the LDS tile only when a record's
// nearest cell leaves the 3 x 3 block around the run's first, or after kRunCap
// records (so an FP32 register sum never holds more than kRunCap terms);
// otherwise every record is added to the tile directly.
// (Variants that add the whole footprint from one base address, inside the tile
// or into an LDS apron, measured slower: bursts of 98 back-to-back FP64 LDS
// atomics, and an apron that leaves room for one workgroup per CU.)
//
// The launch is persistent: each workgroup takes the next item of the work list
// (largest items first) until the list is exhausted, so the count of items never
// has to come back to the host.
template <typename T, int TT, int SS, bool ACC, int KIND>
__global__ __launch_bounds__(kGridThreads) void k_grid(JobGeom g, const uint32_t *__restrict__ counts,
                                                        const uint32_t *__restrict__ offsets,
                                                        const uint2 *__restrict__ items,
                                                        WorkTotals *wt,
                                                        const typename RecTraits<T>::Rec *__restrict__ rec,
                                                        C2<T> *__restrict__ grid, int transposed,
                                                        int accumulate) {
    constexpr int TP = TT + 8;
    constexpr int L0 = 8;                  // cell (j, i) is element L0 + j * TP + i
    constexpr int H = (SS - 1) / 2;
    constexpr uint32_t chunk = kGridChunk;
    // the tile sums many contributions per cell: kept in FP64 for every mesh type,
    // rounded once when the cell is stored
    __shared__ double s_re[TT * TP + 2 * L0];
    __shared__ double s_im[TT * TP + 2 * L0];
    __shared__ uint32_t s_item;
    const uint32_t n_items = wt->n_items;
    for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&wt->next_item, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    if (item >= n_items) break;   // the same for every thread of the workgroup
    const uint2 it = items[item];
    const uint32_t b = it.x;
    const uint32_t c = it.y;
    const uint32_t cnt = counts[b];
    // add into the stack (a split bin, or a stack that holds earlier chunks)
    const bool split = accumulate || cnt > chunk;
    const uint32_t r0 = offsets[b] + c * chunk;
    const uint32_t r1 = offsets[b] + min(cnt, (c + 1) * chunk);

    for (int i = threadIdx.x; i < TT * TP + 2 * L0; i += blockDim.x) {
        s_re[i] = 0.0;
        s_im[i] = 0.0;
    }
    __syncthreads();

    const T inv2s2 = (T)g.inv2s2;
    const uint32_t n = r1 - r0;
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t q0 = r0 + min(n, threadIdx.x * per);
    const uint32_t q1 = r0 + min(n, (threadIdx.x + 1) * per);

    // register window of a run: W x W cells from the anchor (ax, ay) - H, the anchor
    // being one cell below and left of the run's first nearest cell; records whose
    // nearest cell lies at offset 0, 1 or 2 from the anchor in each axis join the
    // run, and [lx, hx] x [ly, hy] are the offsets used (the flush adds only the
    // window's columns lx .. hx + S - 1 and rows ly .. hy + S - 1)
    // (FP64 mesh: runs of one nearest cell, an S x S window of FP64 registers)
    constexpr bool RUN3 = ACC && sizeof(T) == 4;
    constexpr int W = ACC ? (RUN3 ? SS + 2 : SS) : 1;
    T ar[W][W], ai[W][W];
    int ax = 0, ay = 0, lx = 0, hx = 0, ly = 0, hy = 0, run = 0;
    // The flush adds the cells of the window the run used (rows ly .. hy + S - 1,
    // columns lx .. hx + S - 1) that lie in the tile rows.  Columns outside the tile
    // need no test (columns -7 .. T + 6 occur, the nearest cell lying within S/2 of the
    // tile, and fall into the padding), so the per-cell condition is the AND of a row
    // and a column condition, each evaluated once per flush.
    auto flush = [&]() {
        if constexpr (ACC) {
            bool col_used[W];
#pragma unroll
            for (int a = 0; a < W; ++a) col_used[a] = a >= lx && a < SS + hx;
#pragma unroll
            for (int bb = 0; bb < W; ++bb) {
                const int j = ay + bb - H;
                if (bb >= ly && bb < SS + hy && j >= 0 && j < TT) {
                    double *pr = s_re + (L0 + j * TP + ax - H);
                    double *pm = s_im + (L0 + j * TP + ax - H);
#pragma unroll
                    for (int a = 0; a < W; ++a) {
                        if (col_used[a]) {
                            atomicAdd(pr + a, (double)ar[bb][a]);
                            atomicAdd(pm + a, (double)ai[bb][a]);
                        }
                    }
                }
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    ar[bb][a] = T(0);
                    ai[bb][a] = T(0);
                }
            }
        }
    };
    if constexpr (ACC) {
#pragma unroll
        for (int bb = 0; bb < W; ++bb)
#pragma unroll
            for (int a = 0; a < W; ++a) {
                ar[bb][a] = T(0);
                ai[bb][a] = T(0);
            }
    }
    if constexpr (RUN3) {
        // exp(-k^2/(2 sigma^2)) for k = 1..H, for gauss_line
        const float cl2 = (float)g.inv2s2 * 1.4426950408889634f;
        float q[H + 1];
#pragma unroll
        for (int k = 0; k <= H; ++k) q[k] = __builtin_amdgcn_exp2f(-(float)(k * k) * cl2);
        const float *__restrict__ kbp = g.kb_poly;
        // A lane whose next record cannot join its run (its nearest cell leaves the
        // 3 x 3 block of cells around the run's first, or kRunCap records are summed)
        // parks until the wave flushes: the wave adds the register sums of all parked
        // lanes to the tile together once kFlushLanes lanes are parked, or when no
        // lane can go on, so each pass of LDS atomics serves many lanes rather than
        // the one or two whose run just ended.  A track moves about a cell per record
        // on long baselines; the block halves the runs of single cells.
        uint32_t pos = q0;
        bool pend = false;
        RecF32 nx{}, nn{};   // the lane's next two records, loaded ahead
        if (pos < q1) nx = rec[pos];
        if (pos + 1 < q1) nn = rec[pos + 1];
        for (;;) {
            if (pos < q1 && !pend) {
                const int li = (int)(nx.px >> kFracBits) - H;
                const int lj = (int)(nx.py >> kFracBits) - H;
                if (run == 0) {
                    ax = li - 1;
                    ay = lj - 1;
                    lx = hx = ly = hy = 1;
                }
                const int dx = li - ax, dy = lj - ay;
                if (run < kRunCap && dx >= 0 && dx <= 2 && dy >= 0 && dy <= 2) {
                    int li2, lj2;
                    T fx, fy, re, im;
                    RecTraits<T>::decode(nx, H, li2, lj2, fx, fy, re, im);
                    ++pos;
                    nx = nn;
                    if (pos + 1 < q1) nn = rec[pos + 1];
                    T gx[SS], gy[SS];
                    if constexpr (KIND == 0) {
                        gauss_line<SS>(fx, cl2, q, gx);
                        gauss_line<SS>(fy, cl2, q, gy);
                    } else {
                        kb_line<SS>(fx, kbp, gx);
                        kb_line<SS>(fy, kbp, gy);
                    }
                    // the footprint's weights placed in the window at offset (dx, dy)
                    T wx[W], wy[W];
#pragma unroll
                    for (int a = 0; a < W; ++a) {
                        const T x0 = a < SS ? gx[a] : T(0), x1 = (a >= 1 && a <= SS) ? gx[a - 1] : T(0),
                                x2 = a >= 2 ? gx[a - 2] : T(0);
                        const T y0 = a < SS ? gy[a] : T(0), y1 = (a >= 1 && a <= SS) ? gy[a - 1] : T(0),
                                y2 = a >= 2 ? gy[a - 2] : T(0);
                        wx[a] = dx == 0 ? x0 : (dx == 1 ? x1 : x2);
                        wy[a] = dy == 0 ? y0 : (dy == 1 ? y1 : y2);
                    }
#pragma unroll
                    for (int bb = 0; bb < W; ++bb) {
                        T wr = re * wy[bb], wi = im * wy[bb];
#pragma unroll
                        for (int a = 0; a < W; ++a) {
                            ar[bb][a] += wr * wx[a];
                            ai[bb][a] += wi * wx[a];
                        }
                    }
                    lx = min(lx, dx);
                    hx = max(hx, dx);
                    ly = min(ly, dy);
                    hy = max(hy, dy);
                    ++run;
                    if (pos == q1) pend = true;
                } else {
                    pend = true;
                }
            }
            const unsigned long long pm = __ballot(pend);
            const unsigned long long lm = __ballot(pos < q1 && !pend);
            if (pm == 0 && lm == 0) break;
            if (__popcll(pm) >= kFlushLanes || lm == 0) {
                if (pend) {
                    flush();
                    run = 0;
                    pend = false;
                }
            }
        }
    } else if constexpr (ACC) {
        // FP64 mesh: the same parking and wave-level flushes, with runs of records that
        // share one nearest cell summed in an S x S window of FP64 registers (a 3 x 3
        // block would need (S+2)^2 complex doubles).  Taps from the three-exponential
        // recurrence in FP64 (Gaussian) or the window's series (Kaiser-Bessel).
        double q[H + 1];
#pragma unroll
        for (int k = 0; k <= H; ++k) q[k] = exp(-(double)(k * k) * g.inv2s2);
        uint32_t pos = q0;
        bool pend = false;
        RecF64 nx{};   // the lane's next record, loaded ahead
        if (pos < q1) nx = rec[pos];
        for (;;) {
            if (pos < q1 && !pend) {
                const int li = (int)(nx.px >> kFracBits64) - H, lj = (int)(nx.py >> kFracBits64) - H;
                if (run == 0) {
                    ax = li;
                    ay = lj;
                }
                if (run < kRunCap && li == ax && lj == ay) {
                    int li2, lj2;
                    double fx, fy, re, im;
                    RecTraits<double>::decode(nx, H, li2, lj2, fx, fy, re, im);
                    ++pos;
                    if (pos < q1) nx = rec[pos];
                    double gx[SS], gy[SS];
                    if constexpr (KIND == 0) {
                        const double e0 = exp(-(fx * fx + fy * fy) * g.inv2s2);
                        re *= e0;
                        im *= e0;
                        gauss_ratio_line64<SS>(fx, g.inv2s2, q, gx);
                        gauss_ratio_line64<SS>(fy, g.inv2s2, q, gy);
                    } else {
#pragma unroll
                        for (int a = 0; a < SS; ++a) {
                            gx[a] = kb_series_value((double)(a - H) - fx, g.kb_series, g.kb_n, SS);
                            gy[a] = kb_series_value((double)(a - H) - fy, g.kb_series, g.kb_n, SS);
                        }
                    }
#pragma unroll
                    for (int bb = 0; bb < SS; ++bb) {
                        const double wr = re * gy[bb], wi = im * gy[bb];
#pragma unroll
                        for (int a = 0; a < SS; ++a) {
                            ar[bb][a] += wr * gx[a];
                            ai[bb][a] += wi * gx[a];
                        }
                    }
                    ++run;
                    if (pos == q1) pend = true;
                } else {
                    pend = true;
                }
            }
            const unsigned long long pm = __ballot(pend);
            const unsigned long long lm = __ballot(pos < q1 && !pend);
            if (pm == 0 && lm == 0) break;
            if (__popcll(pm) >= kFlushLanes || lm == 0) {
                if (pend) {
                    flush();
                    run = 0;
                    pend = false;
                }
            }
        }
    } else {
    for (uint32_t ri = q0; ri < q1; ++ri) {
        int li, lj;
        T fx, fy, re, im;
        RecTraits<T>::decode(rec[ri], H, li, lj, fx, fy, re, im);
        T gx[SS], gy[SS];
        if constexpr (KIND == 0) {
#pragma unroll
            for (int a = 0; a < SS; ++a) {
                gx[a] = RecTraits<T>::gauss((T)(a - H) - fx, inv2s2);
                gy[a] = RecTraits<T>::gauss((T)(a - H) - fy, inv2s2);
            }
        } else if constexpr (sizeof(T) == 4) {
            kb_line<SS>(fx, g.kb_poly, gx);
            kb_line<SS>(fy, g.kb_poly, gy);
        } else {
#pragma unroll
            for (int a = 0; a < SS; ++a) {
                gx[a] = kb_series_value((T)(a - H) - fx, g.kb_series, g.kb_n, SS);
                gy[a] = kb_series_value((T)(a - H) - fy, g.kb_series, g.kb_n, SS);
            }
        }
#pragma unroll
        for (int bb = 0; bb < SS; ++bb) {
            int j = lj + bb - H;
            if (j < 0 || j >= TT) continue;
            T wr = re * gy[bb], wi = im * gy[bb];
#pragma unroll
            for (int a = 0; a < SS; ++a) {
                int i = li + a - H;
                if (i < 0 || i >= TT) continue;
                atomicAdd(&s_re[L0 + j * TP + i], (double)(wr * gx[a]));
                atomicAdd(&s_im[L0 + j * TP + i], (double)(wi * gx[a]));
            }
        }
    }
    }
    __syncthreads();

    int img, kl, ty, tx;
    bin_coords(g, b, img, kl, ty, tx);
    const int gi0 = tx * TT, gj0 = ty * TT;
    for (int t = threadIdx.x; t < TT * TT; t += blockDim.x) {
        // fast index runs along the stored row of the plane
        int fast = t % TT, slow = t / TT;
        int i, j;
        if (transposed) { j = fast; i = slow; } else { i = fast; j = slow; }
        T vr = (T)s_re[L0 + j * TP + i], vi = (T)s_im[L0 + j * TP + i];
        size_t idx = cell_index<T>(g, img, kl, gi0 + i, gj0 + j, transposed != 0);
        if (split) {
            atomicAdd(&grid[idx].x, vr);
            atomicAdd(&grid[idx].y, vi);
        } else {
            grid[idx] = C2<T>{vr, vi};
        }
    }
    // every read of the tile and of s_item is done before the next item clears them
    __syncthreads();
    }
}

// Each workgroup checks kGridThreads consecutive bins (one per thread) and clears,
// together, the tiles of those that need it: split bins (their chunks add with
// atomics) and, with zero_empty, empty bins.  Few bins need it on the imaging path,
// so most workgroups only read their counts.
template <typename T, int TT>
__global__ __launch_bounds__(kGridThreads) void k_zero_tiles(JobGeom g, const uint32_t *__restrict__ counts,
                                                             size_t n_bins, uint32_t chunk, int zero_empty,
                                                             C2<T> *__restrict__ grid, int transposed) {
    __shared__ uint32_t s_bins[kGridThreads];
    __shared__ uint32_t s_n;
    if (threadIdx.x == 0) s_n = 0u;
    __syncthreads();
    const size_t b = (size_t)blockIdx.x * kGridThreads + threadIdx.x;
    if (b < n_bins) {
        const uint32_t c = counts[b];
        if (c > chunk || (zero_empty && c == 0)) {
            int img, kl, ty, tx;
            bin_coords(g, (uint32_t)b, img, kl, ty, tx);
            if (kl >= g.stack_k0 && kl < g.stack_k0 + g.stack_pl)   // in this pass
                s_bins[atomicAdd(&s_n, 1u)] = (uint32_t)b;
        }
    }
    __syncthreads();
    const uint32_t n = s_n;
    for (uint32_t k = 0; k < n; ++k) {
        int img, kl, ty, tx;
        bin_coords(g, s_bins[k], img, kl, ty, tx);
        const int gi0 = tx * TT, gj0 = ty * TT;
        for (int t = threadIdx.x; t < TT * TT; t += blockDim.x) {
            int fast = t % TT, slow = t / TT;
            int i, j;
            if (transposed) { j = fast; i = slow; } else { i = fast; j = slow; }
            grid[cell_index<T>(g, img, kl, gi0 + i, gj0 + j, transposed != 0)] = C2<T>{T(0), T(0)};
        }
    }
}

// One workgroup per plane: its tile bitmaps (in LDS), tile-row bitmap and the
// per-thread point masks of both transform passes.  Consecutive threads take
// consecutive tile columns tx, so the reads of counts (bin = (plane*NT + ty)*NT
// + tx) are contiguous.
__global__ __launch_bounds__(256) void k_occupancy(JobGeom g, const uint32_t *__restrict__ counts,
                                                   uint64_t *__restrict__ rows,
                                                   uint32_t *__restrict__ live1,
                                                   uint16_t *__restrict__ live2, ImgState *st,
                                                   int nw) {
    __shared__ unsigned long long s_tiles[256 * 4];   // [tx][word], NT <= 256
    __shared__ unsigned long long s_rows[4];
    const int pi = blockIdx.x;                         // plane of the stack
    const int img = pi / g.stack_pl;
    const int kl = g.stack_k0 + (pi - img * g.stack_pl);
    const int NT = g.NT, N = g.N, P = N / 16;
    if (threadIdx.x < 4) s_rows[threadIdx.x] = 0ull;
    __syncthreads();
    const uint32_t *c = counts + (((size_t)img * g.n_pl + kl) << (2 * g.logNT));
    for (int t = threadIdx.x; t < NT * nw; t += blockDim.x) {
        const int tx = t % NT, wd = t / NT;
        unsigned long long word = 0ull;
        for (int bit = 0; bit < 64; ++bit) {
            const int ty = wd * 64 + bit;
            if (ty < NT && c[(size_t)ty * NT + tx] != 0u) word |= 1ull << bit;
        }
        s_tiles[tx * nw + wd] = word;
        if (word) atomicOr(&s_rows[tx >> 6], 1ull << (tx & 63));
    }
    __syncthreads();
    if ((int)threadIdx.x < nw) rows[(size_t)pi * nw + threadIdx.x] = s_rows[threadIdx.x];
    if (threadIdx.x == 0) {
        unsigned long long nt = 0, nr = 0;
        for (int i = 0; i < NT * nw; ++i) nt += __popcll(s_tiles[i]);
        for (int i = 0; i < nw; ++i) nr += __popcll(s_rows[i]);
        if (nt) atomicAdd(&st[img].n_tiles, nt);
        if (nr) atomicAdd(&st[img].n_tile_rows, nr);
    }
    for (int idx = threadIdx.x; idx < NT * P; idx += blockDim.x) {
        const int tx = idx / P, t = idx - tx * P;
        uint32_t m1 = (uint32_t)((s_rows[tx >> 6] >> (tx & 63)) & 1ull) << 16;
        for (int m = 0; m < 16; ++m) {
            const int ty = (t + m * P) >> g.logT;
            m1 |= (uint32_t)((s_tiles[tx * nw + (ty >> 6)] >> (ty & 63)) & 1ull) << m;
        }
        live1[((size_t)pi * NT + tx) * P + t] = m1;
    }
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        uint32_t m2 = 0u;
        for (int m = 0; m < 16; ++m) {
            const int tx = (t + m * P) >> g.logT;
            m2 |= (uint32_t)((s_rows[tx >> 6] >> (tx & 63)) & 1ull) << m;
        }
        live2[(size_t)pi * P + t] = (uint16_t)m2;
    }
}

template <typename T, int TT, int SS>
void launch_tile(const JobGeom &g, unsigned n_wg, hipStream_t s, const uint32_t *counts,
                 const uint32_t *offsets, const uint2 *items, WorkTotals *wt,
                 const typename RecTraits<T>::Rec *r, C2<T> *gp, int tr, int acc) {
    constexpr bool ACC = SS <= 7;
    if (g.kernel == 1)
        k_grid<T, TT, SS, ACC, 1><<<n_wg, kGridThreads, 0, s>>>(g, counts, offsets, items, wt, r, gp, tr, acc);
    else
        k_grid<T, TT, SS, ACC, 0><<<n_wg, kGridThreads, 0, s>>>(g, counts, offsets, items, wt, r, gp, tr, acc);
}

template <typename T, int TT>
void launch_support(const JobGeom &g, unsigned n_wg, hipStream_t s, const uint32_t *counts,
                    const uint32_t *offsets, const uint2 *items, WorkTotals *wt,
                    const typename RecTraits<T>::Rec *r, C2<T> *gp, int tr, int acc) {
    switch (g.S) {
#define WSG_S(ss) case ss: launch_tile<T, TT, ss>(g, n_wg, s, counts, offsets, items, wt, r, gp, tr, acc); break;
    WSG_S(1) WSG_S(3) WSG_S(5) WSG_S(7) WSG_S(9) WSG_S(11) WSG_S(13) WSG_S(15)
#undef WSG_S
    default: break;
    }
}

template <typename T>
void dispatch_grid(const JobGeom &g, const uint32_t *counts, const uint32_t *offsets,
                   const uint2 *items, WorkTotals *wt, unsigned n_wg, const void *records,
                   void *grid, bool transposed, bool accumulate, hipStream_t s) {
    using Rec = typename RecTraits<T>::Rec;
    const Rec *r = (const Rec *)records;
    C2<T> *gp = (C2<T> *)grid;
    int tr = transposed ? 1 : 0, acc = accumulate ? 1 : 0;
    switch (g.T) {
    case 16: launch_support<T, 16>(g, n_wg, s, counts, offsets, items, wt, r, gp, tr, acc); break;
    case 32: launch_support<T, 32>(g, n_wg, s, counts, offsets, items, wt, r, gp, tr, acc); break;
    case 64: launch_support<T, 64>(g, n_wg, s, counts, offsets, items, wt, r, gp, tr, acc); break;
    default: break;
    }
}

template <typename T>
void dispatch_zero(const JobGeom &g, const uint32_t *counts, uint32_t chunk, int ze, void *grid,
                   bool transposed, hipStream_t s) {
    const size_t n_bins = (size_t)g.n_img * g.n_pl * g.NT * g.NT;
    const unsigned blocks = (unsigned)((n_bins + kGridThreads - 1) / kGridThreads);
    if (blocks == 0) return;
    C2<T> *gp = (C2<T> *)grid;
    int tr = transposed ? 1 : 0;
    switch (g.T) {
    case 16: k_zero_tiles<T, 16><<<blocks, kGridThreads, 0, s>>>(g, counts, n_bins, chunk, ze, gp, tr); break;
    case 32: k_zero_tiles<T, 32><<<blocks, kGridThreads, 0, s>>>(g, counts, n_bins, chunk, ze, gp, tr); break;
    case 64: k_zero_tiles<T, 64><<<blocks, kGridThreads, 0, s>>>(g, counts, n_bins, chunk, ze, gp, tr); break;
    default: break;
    }
}

}  // namespace

void launch_zero_tiles(const JobGeom &g, bool f64, const uint32_t *counts, uint32_t chunk,
                       bool zero_empty, void *grid, bool transposed, hipStream_t s) {
    const int ze = zero_empty ? 1 : 0;
    if (f64)
        dispatch_zero<double>(g, counts, chunk, ze, grid, transposed, s);
    else
        dispatch_zero<float>(g, counts, chunk, ze, grid, transposed, s);
}

int occupancy_words(int NT) { return (NT + 63) / 64; }

namespace {

// Fold one chunk of a chunked job into its accumulator: bins that received records
// (for the tile occupancy of the final stack), and the chunk's counts, weight sum
// and plane geometry (the w range is given, so every chunk has the same).
// Chunks are folded in call order, so the FP64 weight sum is deterministic.
__global__ void k_accum_chunk(const uint32_t *__restrict__ counts, uint32_t *__restrict__ seen,
                              size_t n_bins, const ImgState *__restrict__ st, ImgState *acc, int n_img,
                              const WorkTotals *__restrict__ wt, uint32_t *acc_totals) {
    for (size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_bins;
         b += (size_t)gridDim.x * blockDim.x)
        if (counts[b] != 0u) seen[b] = 1u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i < n_img; ++i) {
            acc[i].n_flagged += st[i].n_flagged;
            acc[i].n_valid0 += st[i].n_valid0;
            acc[i].n_used += st[i].n_used;
            acc[i].sum_w += st[i].sum_w;
            acc[i].w_min = st[i].w_min;
            acc[i].w_max = st[i].w_max;
            acc[i].dw = st[i].dw;
            acc[i].w0 = st[i].w0;
            acc[i].inv_dw = st[i].inv_dw;
        }
        // acc_totals: [0] scatter overflow, [1..2] records of all chunks (low, high word)
        acc_totals[0] += wt->overflow;
        const unsigned long long r =
            ((unsigned long long)acc_totals[2] << 32 | acc_totals[1]) + wt->n_records;
        acc_totals[1] = (uint32_t)r;
        acc_totals[2] = (uint32_t)(r >> 32);
    }
}

}  // namespace

void launch_occupancy(const JobGeom &g, const uint32_t *counts, uint64_t *rows, uint32_t *live1,
                      uint16_t *live2, ImgState *st, hipStream_t s) {
    const unsigned n_planes = (unsigned)(g.n_img * g.stack_pl);
    if (n_planes == 0) return;
    k_occupancy<<<n_planes, 256, 0, s>>>(g, counts, rows, live1, live2, st, occupancy_words(g.NT));
}

void launch_grid(const JobGeom &g, bool f64, const uint32_t *counts, const uint32_t *offsets,
                 const uint2 *items, WorkTotals *wt, unsigned n_wg, const void *records, void *grid,
                 bool transposed, bool accumulate, hipStream_t s) {
    if (n_wg == 0) return;
    if (f64)
        dispatch_grid<double>(g, counts, offsets, items, wt, n_wg, records, grid, transposed, accumulate, s);
    else
        dispatch_grid<float>(g, counts, offsets, items, wt, n_wg, records, grid, transposed, accumulate, s);
}

// Resident workgroups per CU: the FP64 LDS tile, 2 x (T (T+8) + 16) x 8 bytes, limits them
// (two for T = 64, eight for T <= 32, with four waves each); a launch of that many
// per CU keeps every CU busy until the list runs dry.
unsigned grid_workgroups(bool f64, int T, size_t max_items, int n_cu) {
    (void)f64;
    const size_t lds = 2u * ((size_t)T * (T + 8) + 16u) * 8u + 64u;
    size_t per_cu = std::min<size_t>((size_t)(160 * 1024) / lds, 8);
    per_cu = std::max<size_t>(per_cu, 1);
    const size_t want = per_cu * (size_t)std::max(n_cu, 1);
    return (unsigned)std::min(want, std::max<size_t>(max_items, 1));
}

void launch_accum_chunk(const uint32_t *counts, uint32_t *seen, size_t n_bins, const ImgState *st,
                        ImgState *acc, int n_img, const WorkTotals *wt, uint32_t *acc_totals,
                        hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<size_t>((n_bins + 255) / 256, 65535);
    k_accum_chunk<<<std::max(blocks, 1u), 256, 0, s>>>(counts, seen, n_bins, st, acc, n_img, wt,
                                                       acc_totals);
}

}  // namespace wsg
