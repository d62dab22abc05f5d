// Internal declarations of the w-stacking library: device types, per-job
// state, and the host-side launchers of each kernel family.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace wsg {

constexpr double kSpeedOfLight = 299792458.0;
constexpr int kMaxN = 16384;
constexpr int kMinN = 16;
constexpr int kMaxSupport = 15;

// ----------------------------------------------------------------------------
// complex arithmetic (interleaved re, im; layout-compatible with complex64/128)
// ----------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ----------------------------------------------------------------------------
// binning records: one per (visibility, tile its footprint touches)
// ----------------------------------------------------------------------------
// complex64 mesh: the cell inside the tile and the sub-cell offset f = x - i0
// in [-1/2, 1/2) as 24-bit fixed point share one word per axis.
struct RecF32 {
    uint32_t px, py;   // (local cell + h) << 24 | round((f + 1/2) * 2^24)
    float re, im;      // W * V
};
// complex128 mesh: the cell in the top 12 bits and the 52 mantissa bits of
// f + 3/2 (a double in [1, 2), so these bits are (f + 1/2) * 2^52) below them, in
// 32 bytes rather than 40.  Exact: f = x - i0 has no bits below ulp(x), and a mesh
// coordinate x >= 2 has none below 2^-52.
struct RecF64 {
    uint64_t px, py;   // (local cell + h) << 52 | mantissa of (f + 3/2)
    double re, im;     // W * V
};

constexpr uint32_t kFracBits = 24;
constexpr float kFracScale = 16777216.0f;        // 2^24
constexpr uint32_t kFracBits64 = 52;
constexpr uint64_t kFracMask64 = (1ull << 52) - 1ull;
constexpr uint64_t kOneBits64 = 0x3ff0000000000000ull;   // the bits of 1.0

// ----------------------------------------------------------------------------
// per-image device state: reductions of the validity pass and plane geometry
// ----------------------------------------------------------------------------
struct ImgState {
    unsigned long long wmin_key, wmax_key;   // order-preserving keys of w over valid rows
    unsigned long long n_flagged;
    unsigned long long n_valid0;             // pass every test but the w range
    unsigned long long n_used;
    double sum_w;
    double w_min, w_max, dw;                 // data (or given) range of w and plane width
    double w0;                               // planes sit at w0 + (k + 1/2) dw
    double inv_dw;                           // 1/dw (0 when dw = 0)
    double inv_norm;                         // 1/sum_w (or 1, or 0 for an empty image)
    unsigned long long n_tiles, n_tile_rows; // occupied (plane, tile) / (plane, tile-row)
};

// Kaiser-Bessel kernel tables.  FP64 meshes evaluate G(d) = I0(beta sqrt(u)) /
// I0(beta), u = 1 - (2d/S)^2, by its power series in u (every coefficient positive,
// so Horner's rule loses nothing to cancellation).  FP32 meshes take tap a of a
// footprint (d = (a - h) - f, f in [-1/2, 1/2)) from a degree-kKbDeg polynomial in
// x = 2f, fitted per tap by Chebyshev interpolation and split into its even part
// (kKbEven coefficients in x^2) and odd part (kKbOdd coefficients in x^2, times x):
// tap S-1-a is the same polynomial at -x, so the two share both parts.
constexpr int kKbMaxSeries = 128;

// Kaiser-Bessel value I0(beta sqrt(u)) / I0(beta), u = 1 - (2d/S)^2, by Horner's rule
// on its power series c[0 .. n) (0 outside the support, where u < 0).
__device__ __forceinline__ double kb_series_value(double d, const double *__restrict__ c, int n,
                                                  int S) {
    const double t = 2.0 * d / (double)S;
    const double u = 1.0 - t * t;
    if (u < 0.0) return 0.0;
    double acc = c[n - 1];
    for (int k = n - 2; k >= 0; --k) acc = fma(acc, u, c[k]);
    return acc;
}
constexpr int kKbDeg = 8;
constexpr int kKbEven = kKbDeg / 2 + 1;
constexpr int kKbOdd = (kKbDeg + 1) / 2;
constexpr int kKbStride = kKbEven + kKbOdd;

// Everything the binning and gridding kernels need about one job.
struct JobGeom {
    int64_t n_rows;
    int32_t n_chan;
    int32_t n_img;          // 1, or n_chan with one image per channel
    int32_t N;
    int32_t n_w;            // planes over [w_min, w_max]
    int32_t plane_lo, n_pl; // planes imaged: [plane_lo, plane_lo + n_pl)
    // the w-stack holds planes [stack_k0, stack_k0 + stack_pl) of the n_pl of every
    // image (planes counted from plane_lo): the whole range in one pass, or one pass
    // of several over the planes
    int32_t stack_k0, stack_pl;
    int32_t S, h;
    int32_t T, NT;          // tile edge and tiles per axis (powers of two)
    int32_t logT, logNT;
    double scale;           // N * cell_rad
    double half;            // N / 2
    int32_t kernel;         // WSG_KERNEL_GAUSSIAN or WSG_KERNEL_KAISER_BESSEL
    double inv2s2;          // Gaussian: 1 / (2 sigma^2)
    // Kaiser-Bessel, device tables of the context (see KbTable)
    const double *kb_series;  // G = sum_k kb_series[k] u^k, u = 1 - (2d/S)^2, k < kb_n
    int32_t kb_n;
    const float *kb_poly;     // per-tap polynomials in x = 2f, kKbStride floats per tap
    int32_t range_given;
    int32_t w_fold;         // rows with w < 0 placed at (-u, -v, -w), visibility conjugated
    // kernel in w over 2 w_h + 1 planes (w_h = 0: nearest plane only): Gaussian
    // exp(-d^2 w_inv2s2), or Kaiser-Bessel from the series kbw_series[0 .. kbw_n)
    int32_t w_h;
    double w_inv2s2;
    const double *kbw_series;
    int32_t kbw_n;
    double w_min_given, w_max_given;
    const double *chan_scale;  // device [n_chan]: f/c or 1
    // track traversal of the binning passes: rows are viewed as [n_t][P]
    // (P = row period, the baselines per time slice); a wave takes one
    // (baseline, channel) track through kStretch consecutive time slices, a
    // track having n_tb such stretches
    int64_t P, n_t, n_tb;
};

// Weight of plane offset d (in planes, w_k - w over dw) under the kernel in w.
__device__ __forceinline__ double w_weight(const JobGeom &g, double d) {
    if (g.kbw_series) return kb_series_value(d, g.kbw_series, g.kbw_n, 2 * g.w_h + 1);
    return exp(-d * d * g.w_inv2s2);
}

// Binning stretch: kStretch time slices of one (baseline, channel) track, one per
// lane of a binning wave (the wavefront size).
constexpr int kStretch = 64;
int64_t stretch_threads(int64_t n_chan, int64_t P, int64_t n_tb);
// The binning passes spread the atomics on one bin over n_cls classes (the
// workgroup index mod n_cls): class c counts into cls_counts[c][bin] and the
// scatter reserves from its own sub-range of the bin, starting at
// cls_cursor[c][bin].  Hot bins (the centre of the uv plane) otherwise take
// hundreds of thousands of atomics on one address.
constexpr int kMaxClasses = 8;
int binning_classes(size_t n_bins);

// ----------------------------------------------------------------------------
// launchers (each enqueues on `s`; no host synchronisation)
// ----------------------------------------------------------------------------
// validity pass: mask[e] = valid except w range; per-image w range, counts,
// n_used and sum_w
void launch_prep(const JobGeom &g, bool f64, const double *uvw, const void *vis,
                 const void *wts, const uint8_t *flags, uint8_t *mask, ImgState *st,
                 hipStream_t s);
void launch_finalize_range(const JobGeom &g, ImgState *st, hipStream_t s);
// records per (image, plane, tile) bin, per atomic class
void launch_count(const JobGeom &g, const double *uvw, const uint8_t *mask, const ImgState *st,
                  uint32_t *cls_counts, int n_cls, hipStream_t s);
// Gridding work list.  A work item is one non-empty bin, or one piece of `chunk`
// records of a bin holding more.  Items are listed largest first by size class
// (floor(log2(records of the item)), kItemClasses classes as items hold at most
// kGridChunk = 2^15 records), so that the persistent gridder starts the longest items
// first and the end of its launch is not held up by one late large tile.  Everything
// here is built on the device: the job needs no host round trip between binning and
// gridding.
constexpr uint32_t kGridChunk = 32768;
constexpr int kItemClasses = 16;
struct WorkTotals {
    uint32_t n_records;                  // records of the job (the last bin offset)
    uint32_t n_items;                    // work items in the list
    uint32_t next_item;                  // queue head of the persistent gridder
    uint32_t overflow;                   // scatter slots beyond the record buffer (must stay 0)
    uint32_t cls_count[kItemClasses];    // items per size class
    uint32_t cls_cursor[kItemClasses];   // placement cursors, then ends of the classes
};
// counts[bin] = sum over classes (counts[n_bins] = 0)
void launch_class_totals(const uint32_t *cls_counts, int n_cls, size_t n_bins, uint32_t *counts,
                         hipStream_t s);
// The work list of the bins whose plane lies in the stack window of g: the item count
// of every size class (wt->cls_count is cleared first), class bases (largest class
// first), n_items, n_records = offsets[n_bins] and queue head 0, then items[slot] =
// (bin, piece) for every piece of every non-empty bin of the window.
void launch_work_list(const JobGeom &g, const uint32_t *counts, const uint32_t *offsets,
                      size_t n_bins, WorkTotals *wt, uint2 *items, hipStream_t s);
// fill n words with v (a kernel, not a memset node, so the job can be captured in a graph)
void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
// dst[0 .. n) = vals[0 .. n), n <= 64, passed by value in the launch
void launch_set_scales(double *dst, const double *vals, int n, hipStream_t s);
// ImgState of n_img images at the start of a job: empty w range keys, zero counters
void launch_init_state(ImgState *st, int n_img, hipStream_t s);
// cls_cursor[c][bin] = offsets[bin] + records of classes < c in the bin
void launch_class_cursors(const uint32_t *cls_counts, int n_cls, size_t n_bins,
                          const uint32_t *offsets, uint32_t *cls_cursor, hipStream_t s);
// exclusive scan of n entries (u32) into out; tmp holds >= scan_tmp_elems(n) u32
size_t scan_tmp_elems(size_t n);
void launch_scan(const uint32_t *in, uint32_t *out, size_t n, uint32_t *tmp, hipStream_t s);
// records beyond `capacity` are not written; each such slot increments *overflow
void launch_scatter(const JobGeom &g, const double *uvw, const void *vis, const void *wts,
                    bool f64, const uint8_t *mask, const ImgState *st, uint32_t *cls_cursor,
                    int n_cls, void *records, uint32_t capacity, uint32_t *overflow, hipStream_t s);
void launch_post_norm(int n_img, ImgState *st, bool normalize, hipStream_t s);

// gridding of binned records into the plane stack [n_img][n_pl][N][N]
// transposed: store plane k as [i][j] (u index slow) instead of [j][i]
// Tile occupancy of the plane stack, so that the transform passes of the imaging
// path read only what the gridder wrote.  For plane pi (= img * stack_pl + kl -
// stack_k0) of the transposed stack G[i][j], tile-row tx (rows i in [tx*T, tx*T + T)), and the
// thread index t < P = N/16 of a length-N transform, whose points are
// t + m*P (m < 16):
//   rows[pi*nw + (tx >> 6)] bit (tx & 63): tile-row tx has a bin with records
//   live1[(pi*NT + tx)*P + t]: bit m: column t + m*P of row tile-row tx lies in
//       a tile with records (pass 1 reads it); bit 16: tile-row tx has records
//   live2[pi*P + t] bit m: row t + m*P lies in a tile-row with records (pass 2
//       reads it)
// with nw = ceil(NT / 64) <= 4.  rows == NULL: every cell of the stack is valid.
struct Occupancy {
    const uint64_t *rows = nullptr;
    const uint32_t *live1 = nullptr;
    const uint16_t *live2 = nullptr;
    int logT = 0;
    int nw = 0;
};
int occupancy_words(int NT);
void launch_occupancy(const JobGeom &g, const uint32_t *counts, uint64_t *rows, uint32_t *live1,
                      uint16_t *live2, ImgState *st, hipStream_t s);
// Clear the tiles of split bins (their chunks add with atomics) and, with
// zero_empty, those of empty bins (which have no work item).
void launch_zero_tiles(const JobGeom &g, bool f64, const uint32_t *counts, uint32_t chunk,
                       bool zero_empty, void *grid, bool transposed, hipStream_t s);
// accumulate: every tile is added into `grid` (which holds earlier chunks) instead
// of stored; otherwise single-item tiles are stored and split ones added.
// n_wg persistent workgroups take the items of the work list in order from
// wt->next_item until wt->n_items (both on the device).
void launch_grid(const JobGeom &g, bool f64, const uint32_t *counts, const uint32_t *offsets,
                 const uint2 *items, WorkTotals *wt, unsigned n_wg, const void *records,
                 void *grid, bool transposed, bool accumulate, hipStream_t s);
// workgroups of the persistent gridder worth launching for at most max_items items
unsigned grid_workgroups(bool f64, int T, size_t max_items, int n_cu);
// chunked jobs: seen[bin] = 1 where the chunk has records; counts, weight sum and
// plane geometry of the chunk's state folded into acc; overflow counters summed
void launch_accum_chunk(const uint32_t *counts, uint32_t *seen, size_t n_bins, const ImgState *st,
                        ImgState *acc, int n_img, const WorkTotals *wt, uint32_t *acc_totals,
                        hipStream_t s);

// transforms.  Pass 1: rows of planes [n][N][N] (in place) into the blocked
// layout [N/B][N][B]; pass 2: along the other axis.
// With occupancy, rows of empty tile-rows are neither read nor written and empty
// tiles read as zero.
void launch_fft_pass1(int N, bool f64, void *planes, int64_t n_planes, const void *twiddle,
                      const Occupancy &occ, hipStream_t s);
// pass 2 from the blocked layout `in` to row-major planes `out` (output row =
// the untransformed index), out of place
void launch_fft_pass2_store(int N, bool f64, const void *in, void *out, int64_t n_planes,
                            const void *twiddle, hipStream_t s);
// pass 2 fused with the phase screen, plane sum and post factors:
// image[img][q][p] = post(Re sum_k F_k[q][p] e^{2 pi i w_k (n-1)})
struct WcorrArgs {
    int N;
    int n_img;
    int n_pl;                // planes per image in the stack
    int plane_lo;            // absolute index of the first plane
    int accumulate;          // add to the image (a later pass over the planes) instead of
                             //   writing it
    int n_w;
    int phase32;             // FP32 phase screen
    int naive_nm1;           // FP32 phase with sqrt(1-eta)-1
    double cell;
    const ImgState *st;      // per image: w0, dw, inv_norm
    const double *inv_c;     // [N] 1/C(nu) or NULL for no grid correction
    Occupancy occ;           // what pass 1 wrote (live2 is used)
    // kernel in w: C_w(nu) = sum_j cw[2j+1] cos(2 pi nu cw[2j]) (quadrature nodes
    // and weights times the window), divided out at nu = dw (n - 1); NULL: none
    const double *cw;
    int n_cw;
};
void launch_fft_pass2_wcorr(const WcorrArgs &a, bool f64, const void *planes,
                            const void *twiddle, double *image, hipStream_t s);
// w-correction alone on row-major transformed planes
void launch_wcorrect(const WcorrArgs &a, bool f64, const void *planes, double *image,
                     hipStream_t s);
// transpose each N x N complex plane (for the row-major stage entry point)
void launch_transpose(int N, bool f64, const void *in, void *out, int64_t n_planes,
                      hipStream_t s);

// device probes (k_probe.hip)
void launch_probe_lds_add(int blocks, int iters, double *out, hipStream_t s);
int probe_lds_add_threads();
void launch_probe_copy(const void *in, void *out, size_t bytes, int n_cu, hipStream_t s);

}  // namespace wsg
