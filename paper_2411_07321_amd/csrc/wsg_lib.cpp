// Host side of the w-stacking library: the C ABI of include/wsg.h.
//
// A job runs as one chain of kernels on one stream, with no host wait inside:
//   [H2D of host inputs] -> prep -> finalize -> count -> scan -> work list ->
//   scatter -> grid (persistent, largest items first) -> transform pass 1 ->
//   transform pass 2 + w-correction + post -> [D2H]
// The record buffer is sized for the worst case (four tiles per visibility and
// plane), so nothing the counting pass finds has to come back to the host.
// Workspace lives in one device arena per context that only grows, so a steady
// stream of jobs allocates nothing after the first of its size.
#include "wsg_internal.h"
#include "../../include/wsg.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace wsg;

namespace {

constexpr uint32_t kChunk = kGridChunk;  // records per gridding work item
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Arena {
    void *ptr = nullptr;
    size_t size = 0;
};

struct DevBuf {
    void *ptr = nullptr;
    size_t size = 0;
};

}  // namespace

// Workspace of the no-allocation entry point (wsg_image_noalloc): a static device
// array, one copy on every GPU the library runs on, held until the process ends.
// Host code never uses its name as an address: the device address of each GPU's copy
// is looked up once per device (scratch_address) and kept.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxChan = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of the scratch array on `device`, which must be the current device.
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return hipSuccess;
}
}  // namespace

namespace {
// A job submitted to a context (wsg_submit): queued on the host, then enqueued on the
// context's stream, then finished.
struct AsyncJob;
// Pinned landing place of one enqueued job's totals and states, and its end event.
struct AsyncSlot {
    void *pin = nullptr;
    size_t size = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
};
constexpr int kAsyncDepth = 2;   // jobs of one context on the device at a time
}  // namespace

struct wsg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    uint64_t budget = 0;
    Arena fixed;
    int n_cu = 256;                      // compute units of the device
    void *scratch = nullptr;             // this device's copy of the static scratch array
    // cached tables
    std::map<std::pair<int, int>, DevBuf> twiddles;                       // (N, f64)
    std::map<std::tuple<int, int, int, double>, DevBuf> inv_c;            // (N, S, kernel, shape)
    std::map<std::pair<int, double>, DevBuf> kb;                          // (S, beta)
    std::map<std::tuple<int, int, double>, DevBuf> cw;                    // (S_w, kernel, shape)
    // device blocks of the last finished chunked job (w-stack block and the two
    // chunk slots), handed to the next one so that a stream of chunked jobs does
    // not allocate
    DevBuf acc_spare, slot_spare[2];
    std::map<std::tuple<int, int, int, int, int>, int> tuned;             // -> tile
    std::map<std::tuple<int, int, int, int, int>, int> tuned_ppp;         // -> planes per pass
    // pinned host staging
    void *pin = nullptr;
    size_t pin_size = 0;
    hipEvent_t pin_done = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // stage timing: events recorded at the stage boundaries of wsg_image
    int timing = 0;
    hipEvent_t tev[10] = {};
    // submitted jobs (wsg_submit), oldest first, until reported by wsg_poll / wsg_wait
    std::deque<std::shared_ptr<AsyncJob>> async_jobs;
    uint64_t next_ticket = 1;
    AsyncSlot aslot[kAsyncDepth];
    hipStream_t last_stream = nullptr;   // stream of the previous call (arena users);
    bool has_last = false;               // NULL is a real stream (the null stream)
};

namespace {

wsg_status fail(wsg_ctx *ctx, wsg_status s, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return s;
}

#define WSG_HIP(ctx, call)                                                               \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            wsg_status st_ = (e_ == hipErrorOutOfMemory) ? WSG_ENOMEM : WSG_EDEVICE;      \
            return fail(ctx, st_, std::string(#call) + ": " + hipGetErrorString(e_));    \
        }                                                                                \
    } while (0)

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

int n_images(const wsg_params *p, const wsg_vis *v) {
    return (p->flags & WSG_PER_CHANNEL) ? v->n_chan : 1;
}

bool f64_mode(const wsg_params *p) { return p->precision == WSG_PREC_F64; }

size_t cplx_size(const wsg_params *p) { return f64_mode(p) ? 16 : 8; }

bool range_given(const wsg_params *p) { return std::isfinite(p->w_min) && std::isfinite(p->w_max); }

// ---------------------------------------------------------------- Kaiser-Bessel
constexpr double kPi = 3.14159265358979323846;
constexpr double kKbMaxBeta = 64.0;
constexpr double kKbFitTol = 2e-7;   // largest |fitted - exact| tap value on an FP32 mesh

// I0(x) by its power series sum_k (x^2/4)^k / (k!)^2 (every term positive).
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 1000; ++k) {
        term *= q / ((double)k * k);
        const double next = sum + term;
        if (next == sum) break;
        sum = next;
    }
    return sum;
}

// beta = 0 in the parameters: pi sqrt((S/2)^2 1.5^2 - 0.8), Beatty, Nishimura and
// Pauly (2005) for a mesh oversampled twice over the image; undefined (NaN) for S = 1
double kb_beta(const wsg_params *p) {
    if (p->kernel_beta > 0.0) return p->kernel_beta;
    const double a = 0.75 * p->support;
    const double r = a * a - 0.8;
    return r > 0.0 ? kPi * std::sqrt(r) : std::nan("");
}

double kb_exact(int S, double beta, double i0b, double d) {
    const double t = 2.0 * d / S;
    const double u = 1.0 - t * t;
    return u < 0.0 ? 0.0 : bessel_i0(beta * std::sqrt(u)) / i0b;
}

// Host copy of the Kaiser-Bessel tables the gridder reads (see wsg_internal.h), and
// the largest error of the FP32 per-tap polynomials against the exact kernel.
struct KbHost {
    std::vector<double> series;
    std::vector<float> poly;
    double fit_err = 0.0;
};

KbHost make_kb(int S, double beta) {
    KbHost kb;
    const int H = (S - 1) / 2;
    // power series in u: c_k = (beta^2/4)^k / (k!)^2 / I0(beta), cut where the terms
    // have passed their peak and fall below 1e-18 of the sum
    const double q = 0.25 * beta * beta;
    std::vector<double> t(1, 1.0);
    double sum = 1.0;
    for (int k = 1; k < kKbMaxSeries; ++k) {
        t.push_back(t.back() * q / ((double)k * k));
        sum += t.back();
        if ((double)k * k > q && t.back() < 1e-18 * sum) break;
    }
    for (double v : t) kb.series.push_back(v / sum);
    const double i0b = bessel_i0(beta);
    // tap a of a footprint as a polynomial in x = 2f: Chebyshev interpolation at
    // kKbDeg + 1 nodes on [-1, 1], then the monomial coefficients through
    // T_{m+1} = 2x T_m - T_{m-1}
    constexpr int n = kKbDeg + 1;
    kb.poly.assign((size_t)(H + 1) * kKbStride, 0.0f);
    for (int a = 0; a <= H; ++a) {
        auto tap = [&](double x) { return kb_exact(S, beta, i0b, (double)(a - H) - 0.5 * x); };
        double fx[n], cheb[n];
        for (int j = 0; j < n; ++j) fx[j] = tap(std::cos(kPi * (j + 0.5) / n));
        for (int m = 0; m < n; ++m) {
            double c = 0.0;
            for (int j = 0; j < n; ++j) c += fx[j] * std::cos(kPi * m * (j + 0.5) / n);
            cheb[m] = (m == 0 ? 1.0 : 2.0) * c / n;
        }
        double mono[n] = {}, tm1[n] = {}, tm[n] = {};
        tm1[0] = 1.0;                      // T_0
        tm[1] = 1.0;                       // T_1
        mono[0] = cheb[0];
        for (int k = 0; k < n; ++k) mono[k] += cheb[1] * tm[k];
        for (int m = 2; m < n; ++m) {
            double tn[n] = {};
            for (int k = 0; k < n; ++k) tn[k] = (k ? 2.0 * tm[k - 1] : 0.0) - tm1[k];
            for (int k = 0; k < n; ++k) mono[k] += cheb[m] * tn[k];
            std::copy(tm, tm + n, tm1);
            std::copy(tn, tn + n, tm);
        }
        float *c = kb.poly.data() + (size_t)a * kKbStride;
        for (int k = 0; k < kKbEven; ++k) c[k] = (float)mono[2 * k];
        for (int k = 0; k < kKbOdd; ++k) c[kKbEven + k] = a == H ? 0.0f : (float)mono[2 * k + 1];
        // error of the stored (FP32-rounded) coefficients, for this tap (x) and its
        // mirror tap S-1-a (-x)
        for (int i = 0; i <= 1024; ++i) {
            const double x = -1.0 + i / 512.0, x2 = x * x;
            double e = 0.0, o = 0.0;
            for (int k = kKbEven - 1; k >= 0; --k) e = e * x2 + c[k];
            for (int k = kKbOdd - 1; k >= 0; --k) o = o * x2 + c[kKbEven + k];
            const double err = std::fabs(e + x * o - tap(x));
            const double err_m = std::fabs(e - x * o - tap(-x));
            kb.fit_err = std::max(kb.fit_err, std::max(err, a == H ? err : err_m));
        }
    }
    return kb;
}

// the tables for (S, beta), built once per process
const KbHost &kb_host(int S, double beta) {
    static std::mutex mu;
    static std::map<std::pair<int, double>, KbHost> memo;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(S, beta);
    auto it = memo.find(key);
    if (it == memo.end()) it = memo.emplace(key, make_kb(S, beta)).first;
    return it->second;
}

int w_half(const wsg_params *p) { return p->w_support > 1 ? (p->w_support - 1) / 2 : 0; }

// Worst-case binning records of n_elem visibilities: a footprint of S <= T + 1 cells
// touches at most two tiles per axis, on each of the 2 w_h + 1 planes of the kernel in w.
uint64_t max_records(const wsg_params *p, int64_t n_elem) {
    return (uint64_t)n_elem * 4u * (uint64_t)(2 * w_half(p) + 1);
}

// beta of the kernel in w: the given one, else the default for w_support
double kb_beta_w(const wsg_params *p) {
    wsg_params q = *p;
    q.support = p->w_support;
    return kb_beta(&q);
}

// smallest tile edge for a mesh of N cells: at most 256 tiles per axis
int min_tile(int N) { return std::max(16, N / 256); }

int default_tile(const wsg_params *p) {
    // 64: the FP64 LDS tile allows two workgroups per CU, as the registers do; the
    // FP64 Kaiser-Bessel gridder's registers allow one at 64, so it takes 32
    const bool kb64 = f64_mode(p) && p->kernel == WSG_KERNEL_KAISER_BESSEL;
    int t = std::max(kb64 ? 32 : 64, min_tile(p->grid_n));
    return std::min(t, p->grid_n);
}

wsg_status check_params(const wsg_params *p, std::string &why) {
    if (!p) { why = "params is NULL"; return WSG_EINVAL; }
    if (!is_pow2(p->grid_n) || p->grid_n < 4) { why = "grid_n must be a power of two"; return WSG_EINVAL; }
    if (p->grid_n < kMinN || p->grid_n > kMaxN) { why = "grid_n outside 16..16384"; return WSG_EUNSUPPORTED; }
    if (p->n_wplanes < 1) { why = "n_wplanes < 1"; return WSG_EINVAL; }
    if (p->support < 1 || (p->support % 2) == 0 || p->support > p->grid_n) {
        why = "support must be odd, >= 1 and <= grid_n";
        return WSG_EINVAL;
    }
    if (p->support > kMaxSupport) { why = "support above 15"; return WSG_EUNSUPPORTED; }
    // (every tile size here is >= 16 >= S - 1, so a footprint touches at most two
    // tiles per axis, which the binning passes rely on)
    if (p->precision < WSG_PREC_F64 || p->precision > WSG_PREC_F32_PHASE32) { why = "bad precision"; return WSG_EINVAL; }
    if (!(p->cell_rad > 0.0) || !std::isfinite(p->cell_rad)) { why = "cell_rad must be finite and > 0"; return WSG_EINVAL; }
    if (p->kernel == WSG_KERNEL_GAUSSIAN) {
        if (!(p->kernel_sigma > 0.0) || !std::isfinite(p->kernel_sigma)) { why = "kernel_sigma must be finite and > 0"; return WSG_EINVAL; }
    } else if (p->kernel == WSG_KERNEL_KAISER_BESSEL) {
        if (!(p->kernel_beta >= 0.0) || !std::isfinite(p->kernel_beta)) { why = "kernel_beta must be finite and >= 0"; return WSG_EINVAL; }
        if (p->kernel_beta > kKbMaxBeta) { why = "kernel_beta above 64"; return WSG_EUNSUPPORTED; }
        const double beta = kb_beta(p);
        if (!(beta > 0.0)) { why = "support 1 has no default kernel_beta: give one"; return WSG_EINVAL; }
        if (!f64_mode(p) && kb_host(p->support, beta).fit_err > kKbFitTol) {
            why = "kernel_beta too steep for the FP32 mesh's fitted kernel (use the FP64 mesh)";
            return WSG_EUNSUPPORTED;
        }
    } else {
        why = "unknown kernel";
        return WSG_EINVAL;
    }
    bool lo_nan = std::isnan(p->w_min), hi_nan = std::isnan(p->w_max);
    if (lo_nan != hi_nan) { why = "w_min and w_max must both be given or both NaN"; return WSG_EINVAL; }
    if (!lo_nan && (!std::isfinite(p->w_min) || !std::isfinite(p->w_max) || p->w_min > p->w_max)) {
        why = "w range must be finite with w_min <= w_max";
        return WSG_EINVAL;
    }
    int lo = p->plane_lo, hi = p->plane_hi;
    if (!(lo == 0 && hi == 0)) {
        if (lo < 0 || hi > p->n_wplanes || lo >= hi) { why = "plane range outside [0, n_wplanes)"; return WSG_EINVAL; }
        if (!(lo == 0 && hi == p->n_wplanes) && lo_nan) {
            why = "a plane range needs a given w range";
            return WSG_EINVAL;
        }
    }
    if (p->w_support < 0 || (p->w_support > 1 && p->w_support % 2 == 0)) {
        why = "w_support must be 0, 1 or odd";
        return WSG_EINVAL;
    }
    if (p->w_support > kMaxSupport) { why = "w_support above 15"; return WSG_EUNSUPPORTED; }
    if (p->w_support > 1) {
        if (p->n_wplanes < p->w_support) { why = "a kernel in w needs n_wplanes >= w_support"; return WSG_EINVAL; }
        if (!(lo == 0 && hi == 0) && !(lo == 0 && hi == p->n_wplanes)) {
            why = "a kernel in w needs the full plane range";
            return WSG_EUNSUPPORTED;
        }
        if (p->kernel == WSG_KERNEL_KAISER_BESSEL && !(kb_beta_w(p) > 0.0)) {
            why = "w_support has no default kernel_beta";
            return WSG_EINVAL;
        }
    }
    if (p->flags & ~(uint32_t)(WSG_GRID_CORRECT | WSG_NORMALIZE | WSG_PER_CHANNEL | WSG_NAIVE_NM1 |
                               WSG_W_FOLD)) {
        why = "unknown flag bits";
        return WSG_EINVAL;
    }
    if (p->planes_per_pass < 0) { why = "planes_per_pass < 0"; return WSG_EINVAL; }
    if (p->tile != 0) {
        if (!(p->tile == 16 || p->tile == 32 || p->tile == 64 || p->tile == 128) || p->tile > p->grid_n) {
            why = "tile must be 16, 32, 64 or 128 and <= grid_n";
            return WSG_EINVAL;
        }
        // the LDS tile holds FP64 sums: 64 x 64 cells is the largest that fits
        if (p->tile == 128) { why = "tile 128 does not fit the FP64 LDS tile"; return WSG_EUNSUPPORTED; }
        // the tile bitmaps of a plane hold at most 256 x 256 tiles
        if (p->tile < min_tile(p->grid_n)) { why = "tile below grid_n / 256"; return WSG_EUNSUPPORTED; }
    }
    return WSG_OK;
}

wsg_status check_vis(const wsg_params *p, const wsg_vis *v, std::string &why) {
    if (!v) { why = "vis is NULL"; return WSG_EINVAL; }
    if (v->n_rows < 0 || v->n_chan < 1) { why = "n_rows < 0 or n_chan < 1"; return WSG_EINVAL; }
    if (v->mem != WSG_MEM_HOST && v->mem != WSG_MEM_DEVICE) { why = "bad memory space"; return WSG_EINVAL; }
    if (v->n_rows > 0 && (!v->uvw || !v->vis)) { why = "uvw or vis is NULL"; return WSG_EINVAL; }
    int64_t n_elem = v->n_rows * (int64_t)v->n_chan;
    if (n_elem > (int64_t)1 << 29) { why = "more than 2^29 visibilities per call"; return WSG_EUNSUPPORTED; }
    // binning records are addressed with 32-bit offsets: a visibility makes at most
    // four (one per uv tile its footprint touches) on each of the w_support planes
    // it spreads over, and the worst case must stay below 2^32
    if (max_records(p, n_elem) > (uint64_t)UINT32_MAX) {
        why = "more than 2^32 - 1 binning records possible (4 x w_support per visibility): split "
              "the visibilities into chunks";
        return WSG_EUNSUPPORTED;
    }
    if ((p->flags & WSG_PER_CHANNEL) && v->n_chan > 256) { why = "more than 256 channels per cube"; return WSG_EUNSUPPORTED; }
    if (v->n_chan > 4096) { why = "more than 4096 channels"; return WSG_EUNSUPPORTED; }
    if (v->freq_hz) {
        for (int c = 0; c < v->n_chan; ++c)
            if (!(v->freq_hz[c] > 0.0) || !std::isfinite(v->freq_hz[c])) { why = "freq_hz must be finite and > 0"; return WSG_EINVAL; }
    }
    int n_img = n_images(p, v);
    int n_pl = (p->plane_hi > p->plane_lo) ? p->plane_hi - p->plane_lo : p->n_wplanes;
    if ((size_t)n_img * n_pl > 65535) { why = "more than 65535 planes in one stack"; return WSG_EUNSUPPORTED; }
    int tile = p->tile ? p->tile : default_tile(p);
    size_t nt = (size_t)(p->grid_n / tile);
    if ((size_t)n_img * n_pl * nt * nt > ((size_t)1 << 27)) { why = "more than 2^27 (plane, tile) bins"; return WSG_EUNSUPPORTED; }
    return WSG_OK;
}


int decade(int64_t n) {
    int d = 0;
    while (n >= 10) { n /= 10; ++d; }
    return d;
}

// ---------------------------------------------------------------- job plan
struct Plan {
    int N, n_w, n_pl, plane_lo, n_img, S, T, NT;
    bool f64;
    int64_t n_rows, n_elem;
    size_t n_bins;
    size_t vis_sz, wt_sz;
    // byte offsets in the fixed arena
    size_t o_uvw, o_vis, o_wts, o_flags, o_scale, o_mask, o_state, o_counts, o_offsets,
        o_cursor, o_scan, o_wt, o_items, o_records, o_occ_rows, o_occ_live1, o_occ_live2,
        o_stack, o_image,
        o_aux, fixed_bytes;
    size_t max_records, max_items;
    int ppp;                           // planes of each image held in the stack per pass
    int64_t P, n_t, n_tb, n_stretch;   // binning traversal (see JobGeom)
    int n_cls;                         // atomic classes of the binning passes
    size_t o_cls_counts;
};

// with_stack false: binning workspace only (chunks of a chunked job, whose stack,
// occupancy and image live in the accumulator)
Plan make_plan(const wsg_params *p, const wsg_vis *v, int tile, bool with_stack,
               bool host_out_image, int ppp = 0) {
    Plan pl{};
    pl.N = p->grid_n;
    pl.n_w = p->n_wplanes;
    pl.plane_lo = (p->plane_hi > p->plane_lo) ? p->plane_lo : 0;
    pl.n_pl = (p->plane_hi > p->plane_lo) ? p->plane_hi - p->plane_lo : p->n_wplanes;
    pl.n_img = n_images(p, v);
    pl.S = p->support;
    pl.T = tile;
    pl.NT = pl.N / tile;
    pl.f64 = f64_mode(p);
    pl.n_rows = v->n_rows;
    pl.n_elem = v->n_rows * (int64_t)v->n_chan;
    pl.n_bins = (size_t)pl.n_img * pl.n_pl * pl.NT * pl.NT;
    pl.ppp = (ppp > 0 && ppp < pl.n_pl) ? ppp : pl.n_pl;
    pl.vis_sz = pl.f64 ? 16 : 8;
    pl.wt_sz = pl.f64 ? 8 : 4;
    bool host_in = v->mem == WSG_MEM_HOST;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    pl.o_uvw = take(host_in ? (size_t)pl.n_rows * 24 : 0);
    pl.o_vis = take(host_in ? (size_t)pl.n_elem * pl.vis_sz : 0);
    pl.o_wts = take(host_in && v->weights ? (size_t)pl.n_elem * pl.wt_sz : 0);
    pl.o_flags = take(host_in && v->flags ? (size_t)pl.n_elem : 0);
    pl.o_scale = take((size_t)v->n_chan * 8);
    pl.o_mask = take((size_t)pl.n_elem);
    pl.o_state = take((size_t)pl.n_img * sizeof(ImgState));
    size_t nb1 = pl.n_bins + 1;
    pl.o_counts = take(nb1 * 4);
    pl.o_offsets = take(nb1 * 4);
    pl.n_cls = binning_classes(pl.n_bins);
    pl.o_cls_counts = take((size_t)pl.n_cls * pl.n_bins * 4);
    pl.o_cursor = take((size_t)pl.n_cls * pl.n_bins * 4);
    pl.o_scan = take(scan_tmp_elems(nb1) * 4);
    pl.o_wt = take(sizeof(WorkTotals));
    // worst case: every visibility touches four tiles on each plane of the kernel in w
    pl.max_records = (size_t)max_records(p, pl.n_elem);
    pl.max_items = pl.n_bins + pl.max_records / kChunk + 1;
    pl.o_items = take(pl.max_items * sizeof(uint2));
    pl.o_records = take(pl.max_records * (pl.f64 ? sizeof(RecF64) : sizeof(RecF32)));
    pl.P = (v->row_period > 1 && v->row_period <= pl.n_rows) ? v->row_period : 1;
    pl.n_t = pl.n_rows > 0 ? (pl.n_rows + pl.P - 1) / pl.P : 0;
    pl.n_tb = (pl.n_t + kStretch - 1) / kStretch;
    pl.n_stretch = stretch_threads(v->n_chan, pl.P, pl.n_tb);
    {
        const size_t nw = (size_t)occupancy_words(pl.NT), np = (size_t)pl.n_img * pl.ppp;
        const size_t k = with_stack ? 1 : 0;
        pl.o_occ_rows = take(k * np * nw * 8);
        pl.o_occ_live1 = take(k * np * pl.NT * (pl.N / 16) * 4);
        pl.o_occ_live2 = take(k * np * (pl.N / 16) * 2);
        pl.o_stack = take(k * np * pl.N * pl.N * (pl.f64 ? 16 : 8));
        pl.o_image = take(host_out_image ? (size_t)pl.n_img * pl.N * pl.N * 8 : 0);
    }
    pl.o_aux = take(0);
    pl.fixed_bytes = off;
    return pl;
}

// Grow an arena (never shrinks here).  The old block is released and the new one
// allocated in stream order on `s`, so other contexts' work is not waited for;
// work of this context on other streams is finished first.
wsg_status ensure_arena(wsg_ctx *ctx, Arena &a, size_t bytes, hipStream_t s) {
    if (bytes <= a.size) return WSG_OK;
    if (ctx->budget && bytes > ctx->budget)
        return fail(ctx, WSG_ENOMEM, "workspace of " + std::to_string(bytes) +
                                         " bytes exceeds the context budget");
    if (ctx->has_last && ctx->last_stream != s) WSG_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
    if (a.ptr) {
        WSG_HIP(ctx, hipFreeAsync(a.ptr, s));
        a.ptr = nullptr;
        a.size = 0;
    }
    size_t sz = align_up(bytes + bytes / 16);
    WSG_HIP(ctx, hipMallocAsync(&a.ptr, sz, s));
    a.size = sz;
    return WSG_OK;
}

wsg_status ensure_pin(wsg_ctx *ctx, size_t bytes) {
    if (ctx->pin_done) WSG_HIP(ctx, hipEventSynchronize(ctx->pin_done));
    if (bytes <= ctx->pin_size) return WSG_OK;
    if (ctx->pin) WSG_HIP(ctx, hipHostFree(ctx->pin));
    ctx->pin = nullptr;
    ctx->pin_size = 0;
    size_t sz = std::max<size_t>(align_up(bytes), 65536);
    WSG_HIP(ctx, hipHostMalloc(&ctx->pin, sz, hipHostMallocDefault));
    ctx->pin_size = sz;
    return WSG_OK;
}

// ---------------------------------------------------------------- tables
// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Host copies of the device tables, built once per process and kept until it ends
// (both the context caches and the no-allocation entry point copy from them).
template <typename K>
const std::vector<char> &memo_table(std::map<K, std::vector<char>> &memo, const K &key,
                                    std::vector<char> (*build)(const K &)) {
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    auto it = memo.find(key);
    if (it == memo.end()) it = memo.emplace(key, build(key)).first;
    return it->second;
}

// 1/C(nu_i), i = 0..N-1, nu_i = (i - N/2)/N, with C(nu) = int_{-S/2}^{S/2} G(d)
// cos(2 pi nu d) dd by 64-point Gauss-Legendre quadrature (both kernels are analytic
// on the support).  Key: (N, S, kernel, sigma or beta).
using InvCKey = std::tuple<int, int, int, double>;
std::vector<char> build_inv_c(const InvCKey &k) {
    const int N = std::get<0>(k), S = std::get<1>(k);
    const bool kb = std::get<2>(k) == WSG_KERNEL_KAISER_BESSEL;
    const double shape = std::get<3>(k);
    std::vector<double> xs, ws;
    gauss_legendre(64, xs, ws);
    const double a = S / 2.0, s2 = 2.0 * shape * shape;
    const double i0b = kb ? bessel_i0(shape) : 1.0;
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<double> gk(xs.size());
    for (size_t j = 0; j < xs.size(); ++j) {
        const double d = a * xs[j];
        gk[j] = kb ? kb_exact(S, shape, i0b, d) : std::exp(-d * d / s2);
    }
    std::vector<char> out((size_t)N * sizeof(double));
    double *h = (double *)out.data();
    for (int i = 0; i < N; ++i) {
        const double nu = (double)(i - N / 2) / N;
        double c = 0.0;
        for (size_t j = 0; j < xs.size(); ++j) c += ws[j] * gk[j] * std::cos(two_pi * nu * a * xs[j]);
        h[i] = 1.0 / (a * c);
    }
    return out;
}

// Quadrature table of the kernel in w for its grid correction: C_w(nu) =
// sum_j cw[2j+1] cos(2 pi nu cw[2j]) by kCwNodes-point Gauss-Legendre over the
// support (the window is analytic there).  Key: (w_support, kernel, sigma or beta).
constexpr int kCwNodes = 32;
using CwKey = std::tuple<int, int, double>;
std::vector<char> build_cw(const CwKey &k) {
    const int Sw = std::get<0>(k);
    const bool kb = std::get<1>(k) == WSG_KERNEL_KAISER_BESSEL;
    const double shape = std::get<2>(k);
    std::vector<double> xs, ws;
    gauss_legendre(kCwNodes, xs, ws);
    const double a = Sw / 2.0, i0b = kb ? bessel_i0(shape) : 1.0;
    const double s2 = 2.0 * shape * shape;
    std::vector<char> out(2 * kCwNodes * sizeof(double));
    double *t = (double *)out.data();
    for (int j = 0; j < kCwNodes; ++j) {
        const double d = a * xs[j];
        const double gv = kb ? kb_exact(Sw, shape, i0b, d) : std::exp(-d * d / s2);
        t[2 * j] = d;
        t[2 * j + 1] = a * ws[j] * gv;
    }
    return out;
}

// Twiddles e^{+2 pi i m / N}, m < N, in the mesh's complex type.  Key: (N, f64).
using TwKey = std::pair<int, int>;
std::vector<char> build_twiddle(const TwKey &k) {
    const int N = k.first;
    const bool f64 = k.second != 0;
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<char> out((size_t)2 * N * (f64 ? 8 : 4));
    for (int m = 0; m < N; ++m) {
        const double c = std::cos(two_pi * m / N), sn = std::sin(two_pi * m / N);
        if (f64) {
            ((double *)out.data())[2 * m] = c;
            ((double *)out.data())[2 * m + 1] = sn;
        } else {
            ((float *)out.data())[2 * m] = (float)c;
            ((float *)out.data())[2 * m + 1] = (float)sn;
        }
    }
    return out;
}

// Kaiser-Bessel tables as the kernels read them: kKbMaxSeries doubles of the power
// series, then the per-tap polynomials.  Key: (S, beta).
constexpr size_t kKbPolyOffset = kKbMaxSeries * sizeof(double);
using KbKey = std::pair<int, double>;
std::vector<char> build_kb_bytes(const KbKey &k) {
    const KbHost &h = kb_host(k.first, k.second);
    std::vector<char> out(kKbPolyOffset + h.poly.size() * sizeof(float), 0);
    std::memcpy(out.data(), h.series.data(), h.series.size() * sizeof(double));
    std::memcpy(out.data() + kKbPolyOffset, h.poly.data(), h.poly.size() * sizeof(float));
    return out;
}

InvCKey inv_c_key(const wsg_params *p) {
    const bool kb = p->kernel == WSG_KERNEL_KAISER_BESSEL;
    return InvCKey(p->grid_n, p->support, (int)p->kernel, kb ? kb_beta(p) : p->kernel_sigma);
}
CwKey cw_key(const wsg_params *p) {
    const bool kb = p->kernel == WSG_KERNEL_KAISER_BESSEL;
    return CwKey(p->w_support, (int)p->kernel, kb ? kb_beta_w(p) : p->kernel_sigma);
}

const std::vector<char> &host_inv_c(const wsg_params *p) {
    static std::map<InvCKey, std::vector<char>> memo;
    return memo_table(memo, inv_c_key(p), build_inv_c);
}
const std::vector<char> &host_cw(const wsg_params *p) {
    static std::map<CwKey, std::vector<char>> memo;
    return memo_table(memo, cw_key(p), build_cw);
}
const std::vector<char> &host_twiddle(int N, bool f64) {
    static std::map<TwKey, std::vector<char>> memo;
    return memo_table(memo, TwKey(N, f64 ? 1 : 0), build_twiddle);
}
const std::vector<char> &host_kb(int S, double beta) {
    static std::map<KbKey, std::vector<char>> memo;
    return memo_table(memo, KbKey(S, beta), build_kb_bytes);
}

bool needs_inv_c(const wsg_params *p) { return (p->flags & WSG_GRID_CORRECT) != 0; }
bool needs_cw(const wsg_params *p) { return (p->flags & WSG_GRID_CORRECT) && w_half(p) > 0; }

// device copy of a host table, cached in the context under `key`
template <typename M, typename K>
wsg_status cached_device(wsg_ctx *ctx, M &cache, const K &key, const std::vector<char> &host,
                         const void **out) {
    auto it = cache.find(key);
    if (it == cache.end()) {
        DevBuf b;
        WSG_HIP(ctx, hipMalloc(&b.ptr, host.size()));
        b.size = host.size();
        WSG_HIP(ctx, hipMemcpy(b.ptr, host.data(), b.size, hipMemcpyHostToDevice));
        it = cache.emplace(key, b).first;
    }
    *out = it->second.ptr;
    return WSG_OK;
}

wsg_status get_inv_c(wsg_ctx *ctx, const wsg_params *p, hipStream_t s, const double **out) {
    (void)s;
    *out = nullptr;
    if (!needs_inv_c(p)) return WSG_OK;
    return cached_device(ctx, ctx->inv_c, inv_c_key(p), host_inv_c(p), (const void **)out);
}

wsg_status kb_tables(wsg_ctx *ctx, int S, double beta, const double **series, int32_t *n,
                     const float **poly) {
    const void *d = nullptr;
    wsg_status rc = cached_device(ctx, ctx->kb, std::make_pair(S, beta), host_kb(S, beta), &d);
    if (rc) return rc;
    *series = (const double *)d;
    *n = (int32_t)kb_host(S, beta).series.size();
    *poly = (const float *)((const char *)d + kKbPolyOffset);
    return WSG_OK;
}

// Kernel tables of a job: the uv kernel's Kaiser-Bessel tables, and the kernel in w
wsg_status kernel_tables(wsg_ctx *ctx, const wsg_params *p, JobGeom *g) {
    const float *poly = nullptr;
    if (p->kernel == WSG_KERNEL_KAISER_BESSEL) {
        wsg_status rc = kb_tables(ctx, p->support, kb_beta(p), &g->kb_series, &g->kb_n, &g->kb_poly);
        if (rc) return rc;
    }
    if (g->w_h > 0 && p->kernel == WSG_KERNEL_KAISER_BESSEL) {
        wsg_status rc = kb_tables(ctx, p->w_support, kb_beta_w(p), &g->kbw_series, &g->kbw_n, &poly);
        if (rc) return rc;
    }
    return WSG_OK;
}

// NULL without a kernel in w or a grid correction
wsg_status get_cw(wsg_ctx *ctx, const wsg_params *p, const double **out, int *n_out) {
    *out = nullptr;
    *n_out = 0;
    if (!needs_cw(p)) return WSG_OK;
    wsg_status rc = cached_device(ctx, ctx->cw, cw_key(p), host_cw(p), (const void **)out);
    if (rc) return rc;
    *n_out = kCwNodes;
    return WSG_OK;
}

wsg_status get_twiddle(wsg_ctx *ctx, int N, bool f64, const void **out) {
    return cached_device(ctx, ctx->twiddles, std::make_pair(N, f64 ? 1 : 0), host_twiddle(N, f64), out);
}

// planes of each image per pass over the w-stack: the parameter, else the tuned choice
// for this job's shape, else all of them (0)
int choose_ppp(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v) {
    if (p->planes_per_pass > 0) return p->planes_per_pass;
    auto key = std::make_tuple(p->grid_n, p->n_wplanes, p->support, p->precision,
                               decade(v->n_rows * (int64_t)v->n_chan));
    auto it = ctx->tuned_ppp.find(key);
    return it != ctx->tuned_ppp.end() ? it->second : 0;
}

int choose_tile(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v) {
    if (p->tile) return p->tile;
    auto key = std::make_tuple(p->grid_n, p->n_wplanes, p->support, p->precision,
                               decade(v->n_rows * (int64_t)v->n_chan));
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return std::min(std::max(it->second, min_tile(p->grid_n)), p->grid_n);
    return default_tile(p);
}

// stage boundary marks (no-ops unless timing is on)
enum {
    kMarkStart = 0, kMarkPrep, kMarkCount, kMarkScatterStart, kMarkScatter, kMarkZero, kMarkGrid,
    kMarkOcc, kMarkFft1, kMarkEnd, kMarks
};

void mark(wsg_ctx *ctx, int i, hipStream_t s) {
    if (ctx->timing) (void)hipEventRecord(ctx->tev[i], s);
}

hipStream_t pick_stream(wsg_ctx *ctx, void *stream) {
    // NULL is HIP's null stream, as everywhere in HIP; the context's own stream is
    // passed explicitly (wsg_context_stream)
    hipStream_t s = (hipStream_t)stream;
    if (ctx->has_last && ctx->last_stream != s) (void)hipStreamSynchronize(ctx->last_stream);
    ctx->last_stream = s;
    ctx->has_last = true;
    return s;
}

// ---------------------------------------------------------------- the binned grid
struct Binned {
    Plan pl;
    JobGeom g;
    char *fx;              // fixed arena base
    const double *uvw;
    const void *vis, *wts;
    const uint8_t *flags;
    ImgState *st;
    uint32_t *counts, *offsets, *cursor;
    WorkTotals *wt;        // record and item totals, work queue head, overflow counter
    uint2 *items;          // gridding work list
    void *records;
};

wsg_status bin_device(wsg_ctx *ctx, const wsg_params *p, Binned &b, uint8_t *mask,
                      uint32_t *scan_tmp, hipStream_t s);

// Geometry of a job: everything the binning and gridding kernels need except the
// device pointers (inputs, workspace, kernel tables).
void job_geom(const wsg_params *p, const wsg_vis *v, const Plan &pl, JobGeom &g) {
    g = JobGeom{};
    g.n_rows = pl.n_rows;
    g.n_chan = v->n_chan;
    g.n_img = pl.n_img;
    g.N = pl.N;
    g.n_w = pl.n_w;
    g.plane_lo = pl.plane_lo;
    g.n_pl = pl.n_pl;
    g.stack_k0 = 0;
    g.stack_pl = pl.n_pl;
    g.S = pl.S;
    g.h = (pl.S - 1) / 2;
    g.T = pl.T;
    g.NT = pl.NT;
    while ((1 << g.logT) < g.T) ++g.logT;
    while ((1 << g.logNT) < g.NT) ++g.logNT;
    g.scale = (double)pl.N * p->cell_rad;
    g.half = 0.5 * (double)pl.N;
    g.kernel = p->kernel;
    g.inv2s2 = p->kernel == WSG_KERNEL_GAUSSIAN ? 1.0 / (2.0 * p->kernel_sigma * p->kernel_sigma) : 0.0;
    g.w_h = w_half(p);
    g.w_inv2s2 = 1.0 / (2.0 * p->kernel_sigma * p->kernel_sigma);
    g.range_given = range_given(p) ? 1 : 0;
    g.w_fold = (p->flags & WSG_W_FOLD) ? 1 : 0;
    g.w_min_given = p->w_min;
    g.w_max_given = p->w_max;
    // track traversal: P = row period (1 without the hint), kStretch time slices
    // per thread
    g.P = pl.P;
    g.n_t = pl.n_t;
    g.n_tb = pl.n_tb;
}

// Workspace pointers of a job laid out by its plan from `base`; device inputs are
// used in place, host inputs from their staging areas in the workspace.
void bind_workspace(Binned &b, char *base, const wsg_vis *v) {
    const Plan &pl = b.pl;
    b.fx = base;
    if (v->mem == WSG_MEM_HOST) {
        b.uvw = (const double *)(base + pl.o_uvw);
        b.vis = base + pl.o_vis;
        b.wts = v->weights ? base + pl.o_wts : nullptr;
        b.flags = v->flags ? (const uint8_t *)(base + pl.o_flags) : nullptr;
    } else {
        b.uvw = v->uvw;
        b.vis = v->vis;
        b.wts = v->weights;
        b.flags = v->flags;
    }
    b.g.chan_scale = (const double *)(base + pl.o_scale);
    b.st = (ImgState *)(base + pl.o_state);
    b.counts = (uint32_t *)(base + pl.o_counts);
    b.offsets = (uint32_t *)(base + pl.o_offsets);
    b.cursor = (uint32_t *)(base + pl.o_cursor);
    b.wt = (WorkTotals *)(base + pl.o_wt);
    b.items = (uint2 *)(base + pl.o_items);
    b.records = base + pl.o_records;
}

// Stage inputs, validity pass, counting sort and record scatter.  Ends with
// the records binned; the grid kernel is launched by the caller.
wsg_status bin_job(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, hipStream_t s, bool image_host,
                   Binned &b, int tile_fixed = 0, bool with_stack = true) {
    int tile = tile_fixed ? tile_fixed : choose_tile(ctx, p, v);
    b.pl = make_plan(p, v, tile, with_stack, image_host, with_stack ? choose_ppp(ctx, p, v) : 0);
    Plan &pl = b.pl;
    if (pl.n_bins > ((size_t)1 << 27)) return fail(ctx, WSG_EUNSUPPORTED, "more than 2^27 (plane, tile) bins");
    if (ctx->budget && pl.fixed_bytes > ctx->budget)
        return fail(ctx, WSG_ENOMEM, "job footprint " + std::to_string(pl.fixed_bytes) +
                                         " bytes exceeds the context budget");
    wsg_status rc = ensure_arena(ctx, ctx->fixed, pl.fixed_bytes, s);
    if (rc) return rc;
    char *fx = (char *)ctx->fixed.ptr;
    job_geom(p, v, pl, b.g);
    bind_workspace(b, fx, v);
    if (v->mem == WSG_MEM_HOST && pl.n_rows > 0) {
        WSG_HIP(ctx, hipMemcpyAsync(fx + pl.o_uvw, v->uvw, (size_t)pl.n_rows * 24, hipMemcpyHostToDevice, s));
        WSG_HIP(ctx, hipMemcpyAsync(fx + pl.o_vis, v->vis, (size_t)pl.n_elem * pl.vis_sz, hipMemcpyHostToDevice, s));
        if (v->weights)
            WSG_HIP(ctx, hipMemcpyAsync(fx + pl.o_wts, v->weights, (size_t)pl.n_elem * pl.wt_sz, hipMemcpyHostToDevice, s));
        if (v->flags)
            WSG_HIP(ctx, hipMemcpyAsync(fx + pl.o_flags, v->flags, (size_t)pl.n_elem, hipMemcpyHostToDevice, s));
    }
    rc = kernel_tables(ctx, p, &b.g);
    if (rc) return rc;
    // per-channel scale through the pinned staging block (ensure_pin first waits for
    // the previous copy out of it); state and counters are set by kernels
    rc = ensure_pin(ctx, (size_t)v->n_chan * 8 + 64);
    if (rc) return rc;
    double *hs = (double *)ctx->pin;
    for (int c = 0; c < v->n_chan; ++c) hs[c] = v->freq_hz ? v->freq_hz[c] / kSpeedOfLight : 1.0;
    WSG_HIP(ctx, hipMemcpyAsync(fx + pl.o_scale, hs, (size_t)v->n_chan * 8, hipMemcpyHostToDevice, s));
    WSG_HIP(ctx, hipEventRecord(ctx->pin_done, s));
    return bin_device(ctx, p, b, (uint8_t *)(fx + pl.o_mask), (uint32_t *)(fx + pl.o_scan), s);
}

// The binning chain on the device: validity, counting sort, work list, scatter.
// Enqueue only; every size it needs is the plan's worst case.
wsg_status bin_device(wsg_ctx *ctx, const wsg_params *p, Binned &b, uint8_t *mask,
                      uint32_t *scan_tmp, hipStream_t s) {
    const Plan &pl = b.pl;
    const JobGeom &g = b.g;
    uint32_t *cls_counts = (uint32_t *)(b.fx + pl.o_cls_counts);
    launch_init_state(b.st, pl.n_img, s);
    launch_fill_u32(cls_counts, (size_t)pl.n_cls * pl.n_bins, 0u, s);
    launch_fill_u32((uint32_t *)b.wt, sizeof(WorkTotals) / 4, 0u, s);
    launch_prep(g, pl.f64, b.uvw, b.vis, b.wts, b.flags, mask, b.st, s);
    launch_finalize_range(g, b.st, s);
    mark(ctx, kMarkPrep, s);
    launch_count(g, b.uvw, mask, b.st, cls_counts, pl.n_cls, s);
    launch_class_totals(cls_counts, pl.n_cls, pl.n_bins, b.counts, s);
    launch_post_norm(pl.n_img, b.st, (p->flags & WSG_NORMALIZE) != 0, s);
    // offsets over n_bins + 1 entries: the last one is the record total
    launch_scan(b.counts, b.offsets, pl.n_bins + 1, scan_tmp, s);
    launch_class_cursors(cls_counts, pl.n_cls, pl.n_bins, b.offsets, b.cursor, s);
    mark(ctx, kMarkCount, s);
    mark(ctx, kMarkScatterStart, s);
    launch_scatter(g, b.uvw, b.vis, b.wts, pl.f64, mask, b.st, b.cursor, pl.n_cls, b.records,
                   (uint32_t)pl.max_records, &b.wt->overflow, s);
    mark(ctx, kMarkScatter, s);
    WSG_HIP(ctx, hipGetLastError());
    return WSG_OK;
}

// dense: every cell of `grid` is written (the stage entry point); otherwise only
// the tiles of non-empty bins, and the occupancy bitmaps say which those are
// The planes of the stack window of b.g: work list, clearing, gridding, occupancy.
// marks: record the stage events (the first pass over the planes only).
wsg_status grid_binned(wsg_ctx *ctx, Binned &b, void *grid, bool transposed, bool dense,
                       hipStream_t s, bool marks = true) {
    launch_work_list(b.g, b.counts, b.offsets, b.pl.n_bins, b.wt, b.items, s);
    launch_zero_tiles(b.g, b.pl.f64, b.counts, kChunk, dense, grid, transposed, s);
    if (marks) mark(ctx, kMarkZero, s);
    launch_grid(b.g, b.pl.f64, b.counts, b.offsets, b.items, b.wt,
                grid_workgroups(b.pl.f64, b.pl.T, b.pl.max_items, ctx->n_cu), b.records, grid,
                transposed, false, s);
    if (marks) mark(ctx, kMarkGrid, s);
    if (!dense)
        launch_occupancy(b.g, b.counts, (uint64_t *)(b.fx + b.pl.o_occ_rows),
                         (uint32_t *)(b.fx + b.pl.o_occ_live1), (uint16_t *)(b.fx + b.pl.o_occ_live2),
                         b.st, s);
    if (marks) mark(ctx, kMarkOcc, s);
    WSG_HIP(ctx, hipGetLastError());
    return WSG_OK;
}

// Per-image stats from the job's totals and states read back to the host.
wsg_status fill_stats(wsg_ctx *ctx, const Binned &b, const wsg_vis *v, const WorkTotals &ht,
                      const ImgState *hs, wsg_stats *stats, bool timed) {
    if (ht.overflow != 0)
        return fail(ctx, WSG_EDEVICE, "internal error: binning passes disagree on record counts");
    float t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (timed) {
        WSG_HIP(ctx, hipEventSynchronize(ctx->tev[kMarkEnd]));
        const int pairs[9][2] = {{kMarkStart, kMarkPrep}, {kMarkPrep, kMarkCount},
                                 {kMarkScatterStart, kMarkScatter}, {kMarkScatter, kMarkZero},
                                 {kMarkZero, kMarkGrid}, {kMarkGrid, kMarkOcc},
                                 {kMarkOcc, kMarkFft1}, {kMarkFft1, kMarkEnd},
                                 {kMarkStart, kMarkEnd}};
        for (int i = 0; i < 9; ++i)
            WSG_HIP(ctx, hipEventElapsedTime(&t[i], ctx->tev[pairs[i][0]], ctx->tev[pairs[i][1]]));
    }
    int64_t per_img = (b.pl.n_img > 1) ? v->n_rows : v->n_rows * (int64_t)v->n_chan;
    for (int i = 0; i < b.pl.n_img; ++i) {
        stats[i].n_used = (int64_t)hs[i].n_used;
        stats[i].n_flagged = (int64_t)hs[i].n_flagged;
        stats[i].n_dropped = per_img - stats[i].n_used - stats[i].n_flagged;
        stats[i].n_records = (int64_t)ht.n_records;
        stats[i].n_tiles = (int64_t)hs[i].n_tiles;
        stats[i].n_tile_rows = (int64_t)hs[i].n_tile_rows;
        stats[i].sum_w = hs[i].sum_w;
        stats[i].w_min = hs[i].w_min;
        stats[i].w_max = hs[i].w_max;
        stats[i].ms_prep = t[0];
        stats[i].ms_count = t[1];
        stats[i].ms_scatter = t[2];
        stats[i].ms_zero = t[3];
        stats[i].ms_grid = t[4];
        stats[i].ms_occupancy = t[5];
        stats[i].ms_fft1 = t[6];
        stats[i].ms_fft2_wcorr = t[7];
        stats[i].ms_total = t[8];
    }
    return WSG_OK;
}

// Waits for the job and fills stats (NULL: returns at once), through the pinned block.
wsg_status read_stats(wsg_ctx *ctx, const Binned &b, const wsg_vis *v, hipStream_t s,
                      wsg_stats *stats, bool timed) {
    if (!stats) return WSG_OK;
    const size_t o_st = align_up(sizeof(WorkTotals));
    const size_t bytes = (size_t)b.pl.n_img * sizeof(ImgState);
    wsg_status rc = ensure_pin(ctx, o_st + bytes);
    if (rc) return rc;
    WSG_HIP(ctx, hipMemcpyAsync(ctx->pin, b.wt, sizeof(WorkTotals), hipMemcpyDeviceToHost, s));
    WSG_HIP(ctx, hipMemcpyAsync((char *)ctx->pin + o_st, b.st, bytes, hipMemcpyDeviceToHost, s));
    WSG_HIP(ctx, hipStreamSynchronize(s));
    return fill_stats(ctx, b, v, *(const WorkTotals *)ctx->pin,
                      (const ImgState *)((const char *)ctx->pin + o_st), stats, timed);
}

bool async_pending(const wsg_ctx *ctx);

wsg_status common_checks(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v) {
    if (!ctx) return WSG_EINVAL;
    if (async_pending(ctx))
        return fail(ctx, WSG_EBUSY, "the context has submitted jobs that are not finished");
    std::string why;
    wsg_status rc = check_params(p, why);
    if (rc) return fail(ctx, rc, why);
    if (v) {
        rc = check_vis(p, v, why);
        if (rc) return fail(ctx, rc, why);
    }
    WSG_HIP(ctx, hipSetDevice(ctx->device));
    return WSG_OK;
}

// Gridding, both transform passes and the w-correction of a binned job, into the
// device image img_dev [n_img][N][N].
// Device tables of the transform and the w-correction.
struct Tables {
    const void *tw = nullptr;          // twiddles of length N
    const double *inv_c = nullptr;     // 1/C(nu) or NULL (no grid correction)
    const double *cw = nullptr;        // kernel-in-w quadrature or NULL
    int n_cw = 0;
};

wsg_status ctx_tables(wsg_ctx *ctx, const wsg_params *p, hipStream_t s, Tables &t) {
    wsg_status rc = get_twiddle(ctx, p->grid_n, f64_mode(p), &t.tw);
    if (rc) return rc;
    rc = get_inv_c(ctx, p, s, &t.inv_c);
    if (rc) return rc;
    return get_cw(ctx, p, &t.cw, &t.n_cw);
}

// Gridding, both transform passes and the w-correction of a binned job, into the
// device image img_dev [n_img][N][N], in passes of pl.ppp planes per image over the
// w-stack (one pass holds them all unless fewer are asked for): each pass grids its
// planes into the stack, transforms them and adds their w-corrected sum to the image.
// With several passes the stage events cover the first pass (ms_total the whole job).
wsg_status image_binned(wsg_ctx *ctx, const wsg_params *p, Binned &b, double *img_dev,
                        const Tables &t, hipStream_t s) {
    const Plan &pl = b.pl;
    void *stack = b.fx + pl.o_stack;
    Occupancy occ;
    occ.rows = (const uint64_t *)(b.fx + pl.o_occ_rows);
    occ.live1 = (const uint32_t *)(b.fx + pl.o_occ_live1);
    occ.live2 = (const uint16_t *)(b.fx + pl.o_occ_live2);
    occ.logT = b.g.logT;
    occ.nw = occupancy_words(pl.NT);
    const int n_pass = (pl.n_pl + pl.ppp - 1) / pl.ppp;
    for (int ps = 0; ps < n_pass; ++ps) {
        b.g.stack_k0 = ps * pl.ppp;
        b.g.stack_pl = std::min(pl.ppp, pl.n_pl - b.g.stack_k0);
        wsg_status rc = grid_binned(ctx, b, stack, true, false, s, ps == 0);
        if (rc) return rc;
        launch_fft_pass1(pl.N, pl.f64, stack, (int64_t)pl.n_img * b.g.stack_pl, t.tw, occ, s);
        if (ps == 0) mark(ctx, kMarkFft1, s);
        WcorrArgs a{};
        a.N = pl.N;
        a.n_img = pl.n_img;
        a.n_pl = b.g.stack_pl;
        a.plane_lo = pl.plane_lo + b.g.stack_k0;
        a.accumulate = ps > 0;
        a.n_w = pl.n_w;
        a.phase32 = p->precision == WSG_PREC_F32_PHASE32;
        a.naive_nm1 = (p->flags & WSG_NAIVE_NM1) ? 1 : 0;
        a.cell = p->cell_rad;
        a.st = b.st;
        a.inv_c = t.inv_c;
        a.occ = occ;
        a.cw = t.cw;
        a.n_cw = t.n_cw;
        launch_fft_pass2_wcorr(a, pl.f64, stack, t.tw, img_dev, s);
    }
    b.g.stack_k0 = 0;
    b.g.stack_pl = pl.n_pl;
    WSG_HIP(ctx, hipGetLastError());
    return WSG_OK;
}

// The whole method for one job, enqueued on `s` (no host wait except for a host
// image, whose copy out waits for the job).
wsg_status enqueue_image(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, double *image,
                         int32_t image_mem, hipStream_t s, Binned &b) {
    if (!image) return fail(ctx, WSG_EINVAL, "image is NULL");
    if (image_mem != WSG_MEM_HOST && image_mem != WSG_MEM_DEVICE) return fail(ctx, WSG_EINVAL, "bad image memory space");
    const bool host_img = image_mem == WSG_MEM_HOST;
    mark(ctx, kMarkStart, s);
    wsg_status rc = bin_job(ctx, p, v, s, host_img, b);
    if (rc) return rc;
    const Plan &pl = b.pl;
    double *img_dev = host_img ? (double *)(b.fx + pl.o_image) : image;
    Tables tb;
    rc = ctx_tables(ctx, p, s, tb);
    if (rc) return rc;
    rc = image_binned(ctx, p, b, img_dev, tb, s);
    if (rc) return rc;
    if (host_img)
        WSG_HIP(ctx, hipMemcpyAsync(image, img_dev, (size_t)pl.n_img * pl.N * pl.N * 8, hipMemcpyDeviceToHost, s));
    mark(ctx, kMarkEnd, s);
    return WSG_OK;
}

// ---------------------------------------------------------------- submitted jobs
struct AsyncJob {
    uint64_t ticket = 0;
    enum { kQueued, kOnDevice, kFinished } state = kQueued;
    wsg_params p{};
    wsg_vis v{};
    std::vector<double> freq;        // the job's own copy of freq_hz
    double *image = nullptr;
    int32_t image_mem = WSG_MEM_DEVICE;
    int slot = -1;
    Binned b{};
    wsg_status status = WSG_OK;
    std::vector<wsg_stats> stats;
};

bool async_pending(const wsg_ctx *ctx) {
    for (const auto &j : ctx->async_jobs)
        if (j->state != AsyncJob::kFinished) return true;
    return false;
}

std::shared_ptr<AsyncJob> find_job(wsg_ctx *ctx, uint64_t ticket) {
    for (auto &j : ctx->async_jobs)
        if (j->ticket == ticket) return j;
    return nullptr;
}

// A job on the device has ended (its event has completed): fill its stats.
void finish_async(wsg_ctx *ctx, AsyncJob &j) {
    AsyncSlot &sl = ctx->aslot[j.slot];
    const size_t o_st = align_up(sizeof(WorkTotals));
    j.stats.assign((size_t)std::max(1, j.b.pl.n_img), wsg_stats{});
    j.status = fill_stats(ctx, j.b, &j.v, *(const WorkTotals *)sl.pin,
                          (const ImgState *)((const char *)sl.pin + o_st), j.stats.data(), false);
    sl.busy = false;
    j.slot = -1;
    j.state = AsyncJob::kFinished;
}

// Enqueue queued jobs while the device holds fewer than kAsyncDepth of this context's.
void pump_async(wsg_ctx *ctx) {
    for (auto &jp : ctx->async_jobs) {
        AsyncJob &j = *jp;
        if (j.state != AsyncJob::kQueued) continue;
        int k = -1;
        for (int i = 0; i < kAsyncDepth; ++i)
            if (!ctx->aslot[i].busy) { k = i; break; }
        if (k < 0) return;
        AsyncSlot &sl = ctx->aslot[k];
        const size_t o_st = align_up(sizeof(WorkTotals));
        const int n_img = n_images(&j.p, &j.v);
        const size_t need = o_st + (size_t)n_img * sizeof(ImgState);
        hipStream_t s = pick_stream(ctx, ctx->stream);
        wsg_status rc = WSG_OK;
        if (need > sl.size) {
            if (sl.pin) (void)hipHostFree(sl.pin);
            sl.pin = nullptr;
            sl.size = 0;
            if (hipHostMalloc(&sl.pin, need, hipHostMallocDefault) != hipSuccess)
                rc = fail(ctx, WSG_ENOMEM, "pinned stats block");
            else
                sl.size = need;
        }
        if (rc == WSG_OK) rc = enqueue_image(ctx, &j.p, &j.v, j.image, j.image_mem, s, j.b);
        if (rc == WSG_OK &&
            (hipMemcpyAsync(sl.pin, j.b.wt, sizeof(WorkTotals), hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipMemcpyAsync((char *)sl.pin + o_st, j.b.st, (size_t)n_img * sizeof(ImgState),
                            hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipEventRecord(sl.done, s) != hipSuccess))
            rc = fail(ctx, WSG_EDEVICE, "enqueueing the stats of a submitted job");
        if (rc != WSG_OK) {
            j.status = rc;
            j.state = AsyncJob::kFinished;
            continue;
        }
        sl.busy = true;
        j.slot = k;
        j.state = AsyncJob::kOnDevice;
    }
}

// Finish every job on the device whose work has ended (wait: the oldest one at least).
wsg_status progress_async(wsg_ctx *ctx, bool wait_oldest) {
    for (auto &jp : ctx->async_jobs) {
        if (jp->state != AsyncJob::kOnDevice) continue;
        hipEvent_t e = ctx->aslot[jp->slot].done;
        if (wait_oldest) {
            WSG_HIP(ctx, hipEventSynchronize(e));
            wait_oldest = false;
        } else {
            const hipError_t q = hipEventQuery(e);
            if (q == hipErrorNotReady) break;   // later jobs of the stream are not done either
            if (q != hipSuccess) return fail(ctx, WSG_EDEVICE, hipGetErrorString(q));
        }
        finish_async(ctx, *jp);
    }
    pump_async(ctx);
    return WSG_OK;
}

// Report a finished job once, then forget it.
wsg_status report_async(wsg_ctx *ctx, const std::shared_ptr<AsyncJob> &j, wsg_stats *stats) {
    if (stats && j->status == WSG_OK)
        std::memcpy(stats, j->stats.data(), j->stats.size() * sizeof(wsg_stats));
    for (auto it = ctx->async_jobs.begin(); it != ctx->async_jobs.end(); ++it)
        if (*it == j) {
            ctx->async_jobs.erase(it);
            break;
        }
    if (j->status != WSG_OK && j->status != WSG_ECANCELED) ctx->last_error = "submitted job failed";
    return j->status;
}

// ---------------------------------------------------------------- chunked jobs
// The accumulator's own device block: state, bins seen, overflow counter,
// occupancy bitmaps, the w-stack and (for host images) the image.
struct AccumLayout {
    size_t o_state, o_seen, o_overflow, o_rows, o_live1, o_live2, o_stack, o_image, bytes;
};

AccumLayout accum_layout(const wsg_params *p, int n_img, int tile) {
    AccumLayout L{};
    const int N = p->grid_n, NT = N / tile;
    const int n_pl = (p->plane_hi > p->plane_lo) ? p->plane_hi - p->plane_lo : p->n_wplanes;
    const size_t np = (size_t)n_img * n_pl, n_bins = np * NT * NT;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.o_state = take((size_t)n_img * sizeof(ImgState));
    L.o_seen = take(n_bins * 4);
    L.o_overflow = take(16);   // overflow counter, records of all chunks (64 bits)
    L.o_rows = take(np * occupancy_words(NT) * 8);
    L.o_live1 = take(np * NT * (N / 16) * 4);
    L.o_live2 = take(np * (N / 16) * 2);
    L.o_stack = take(np * N * N * (f64_mode(p) ? 16 : 8));
    L.o_image = take((size_t)n_img * N * N * 8);
    L.bytes = off;
    return L;
}

wsg_status check_accum(const wsg_params *p, int32_t n_chan, std::string &why) {
    wsg_status rc = check_params(p, why);
    if (rc) return rc;
    if (n_chan < 1 || n_chan > 4096) { why = "n_chan must be 1 .. 4096"; return WSG_EINVAL; }
    if ((p->flags & WSG_PER_CHANNEL) && n_chan > 256) { why = "more than 256 channels per cube"; return WSG_EUNSUPPORTED; }
    if (!range_given(p)) { why = "chunked imaging needs a given w range (w_min, w_max)"; return WSG_EINVAL; }
    return WSG_OK;
}

}  // namespace

struct wsg_accum {
    wsg_ctx *ctx = nullptr;
    wsg_params p{};
    int32_t n_chan = 0;
    int n_img = 0, tile = 0;
    bool per_channel = false, broken = false, finished = false;
    JobGeom g{};                   // mesh geometry for the occupancy pass
    size_t n_bins = 0;
    AccumLayout L{};
    char *mem = nullptr;
    size_t mem_size = 0;
    int64_t per_img_elems = 0;     // elements offered to each image, over all chunks
    // host chunks: two device slots filled on the copy stream
    hipStream_t copy = nullptr;
    void *slot[2] = {nullptr, nullptr};
    size_t slot_size[2] = {0, 0};
    hipEvent_t copied[2] = {nullptr, nullptr}, slot_free[2] = {nullptr, nullptr};
    int next_slot = 0;
};

namespace {

// Device copy of a host chunk in the accumulator's next slot, on its copy stream,
// ordered after the last job that read the slot; the compute stream waits for it.
wsg_status stage_chunk(wsg_accum *a, const wsg_vis *v, hipStream_t s, wsg_vis *dv, int *used) {
    wsg_ctx *ctx = a->ctx;
    const bool f64 = f64_mode(&a->p);
    const size_t n_elem = (size_t)v->n_rows * v->n_chan;
    const size_t b_uvw = align_up((size_t)v->n_rows * 24), b_vis = align_up(n_elem * (f64 ? 16 : 8));
    const size_t b_wts = v->weights ? align_up(n_elem * (f64 ? 8 : 4)) : 0;
    const size_t b_fl = v->flags ? align_up(n_elem) : 0;
    const size_t need = b_uvw + b_vis + b_wts + b_fl;
    const int k = a->next_slot;
    if (need > a->slot_size[k]) {
        WSG_HIP(ctx, hipEventSynchronize(a->slot_free[k]));
        if (a->slot[k]) WSG_HIP(ctx, hipFree(a->slot[k]));
        a->slot[k] = nullptr;
        a->slot_size[k] = 0;
        WSG_HIP(ctx, hipMalloc(&a->slot[k], need));
        a->slot_size[k] = need;
    }
    char *d = (char *)a->slot[k];
    WSG_HIP(ctx, hipStreamWaitEvent(a->copy, a->slot_free[k], 0));
    WSG_HIP(ctx, hipMemcpyAsync(d, v->uvw, (size_t)v->n_rows * 24, hipMemcpyHostToDevice, a->copy));
    WSG_HIP(ctx, hipMemcpyAsync(d + b_uvw, v->vis, n_elem * (f64 ? 16 : 8), hipMemcpyHostToDevice, a->copy));
    if (v->weights)
        WSG_HIP(ctx, hipMemcpyAsync(d + b_uvw + b_vis, v->weights, n_elem * (f64 ? 8 : 4),
                                    hipMemcpyHostToDevice, a->copy));
    if (v->flags)
        WSG_HIP(ctx, hipMemcpyAsync(d + b_uvw + b_vis + b_wts, v->flags, n_elem, hipMemcpyHostToDevice,
                                    a->copy));
    WSG_HIP(ctx, hipEventRecord(a->copied[k], a->copy));
    WSG_HIP(ctx, hipStreamWaitEvent(s, a->copied[k], 0));
    *dv = *v;
    dv->mem = WSG_MEM_DEVICE;
    dv->uvw = (const double *)d;
    dv->vis = d + b_uvw;
    dv->weights = v->weights ? d + b_uvw + b_vis : nullptr;
    dv->flags = v->flags ? (const uint8_t *)(d + b_uvw + b_vis + b_wts) : nullptr;
    *used = k;
    a->next_slot = k ^ 1;
    return WSG_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

wsg_status wsg_create(int device, wsg_ctx **out) {
    if (!out) return WSG_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return WSG_EDEVICE;
    if (device < 0 || device >= n) return WSG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return WSG_EDEVICE;
    wsg_ctx *ctx = new (std::nothrow) wsg_ctx();
    if (!ctx) return WSG_ENOMEM;
    ctx->device = device;
    if (scratch_address(device, &ctx->scratch) != hipSuccess) {
        delete ctx;
        return WSG_EDEVICE;
    }
    {
        int n_cu = 0;
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            n_cu > 0)
            ctx->n_cu = n_cu;
    }
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->pin_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        [&] {
            for (auto &e : ctx->tev)
                if (hipEventCreate(&e) != hipSuccess) return true;
            return false;
        }()) {
        wsg_destroy(ctx);
        return WSG_EDEVICE;
    }
    *out = ctx;
    return WSG_OK;
}

void wsg_destroy(wsg_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->has_last && ctx->last_stream != ctx->stream) (void)hipStreamSynchronize(ctx->last_stream);
    ctx->async_jobs.clear();   // queued jobs are dropped; the device has finished the others
    for (auto &sl : ctx->aslot) {
        if (sl.pin) (void)hipHostFree(sl.pin);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (ctx->fixed.ptr) (void)hipFreeAsync(ctx->fixed.ptr, ctx->stream);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->twiddles) (void)hipFree(kv.second.ptr);
    for (auto &kv : ctx->inv_c) (void)hipFree(kv.second.ptr);
    for (auto &kv : ctx->kb) (void)hipFree(kv.second.ptr);
    for (auto &kv : ctx->cw) (void)hipFree(kv.second.ptr);
    for (DevBuf *d : {&ctx->acc_spare, &ctx->slot_spare[0], &ctx->slot_spare[1]})
        if (d->ptr) (void)hipFree(d->ptr);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    if (ctx->pin_done) (void)hipEventDestroy(ctx->pin_done);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (auto &e : ctx->tev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *wsg_strerror(wsg_status s) {
    switch (s) {
    case WSG_OK: return "ok";
    case WSG_EINVAL: return "invalid argument";
    case WSG_ENOMEM: return "out of memory (workspace budget or device memory)";
    case WSG_EDEVICE: return "HIP device error";
    case WSG_EBUSY: return "context busy";
    case WSG_EUNSUPPORTED: return "unsupported by the library";
    case WSG_ECANCELED: return "job canceled before it started";
    default: return "unknown status";
    }
}

void *wsg_context_stream(const wsg_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

const char *wsg_last_error(const wsg_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

wsg_status wsg_set_budget(wsg_ctx *ctx, uint64_t bytes) {
    if (!ctx) return WSG_EINVAL;
    ctx->budget = bytes;
    return WSG_OK;
}

wsg_status wsg_trim(wsg_ctx *ctx) {
    if (!ctx) return WSG_EINVAL;
    WSG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->has_last ? ctx->last_stream : ctx->stream;
    if (ctx->fixed.ptr) WSG_HIP(ctx, hipFreeAsync(ctx->fixed.ptr, s));
    ctx->fixed = Arena{};
    WSG_HIP(ctx, hipStreamSynchronize(s));
    for (DevBuf *d : {&ctx->acc_spare, &ctx->slot_spare[0], &ctx->slot_spare[1]}) {
        if (d->ptr) WSG_HIP(ctx, hipFree(d->ptr));
        *d = DevBuf{};
    }
    return WSG_OK;
}

wsg_status wsg_set_timing(wsg_ctx *ctx, int32_t on) {
    if (!ctx) return WSG_EINVAL;
    ctx->timing = on ? 1 : 0;
    return WSG_OK;
}

wsg_status wsg_check(const wsg_params *p, const wsg_vis *v) {
    std::string why;
    wsg_status rc = check_params(p, why);
    if (rc) return rc;
    if (v) return check_vis(p, v, why);
    return WSG_OK;
}

int32_t wsg_n_images(const wsg_params *p, const wsg_vis *v) {
    if (!p || !v) return 0;
    return n_images(p, v);
}

wsg_status wsg_footprint(const wsg_params *p, const wsg_vis *v, uint64_t *bytes) {
    if (!bytes) return WSG_EINVAL;
    std::string why;
    wsg_status rc = check_params(p, why);
    if (rc) return rc;
    rc = check_vis(p, v, why);
    if (rc) return rc;
    int tile = p->tile ? p->tile : default_tile(p);
    Plan pl = make_plan(p, v, tile, true, false, p->planes_per_pass);
    *bytes = pl.fixed_bytes;
    return WSG_OK;
}

wsg_status wsg_image(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, double *image,
                     int32_t image_mem, void *stream, wsg_stats *stats) {
    wsg_status rc = common_checks(ctx, p, v);
    if (rc) return rc;
    hipStream_t s = pick_stream(ctx, stream);
    Binned b;
    rc = enqueue_image(ctx, p, v, image, image_mem, s, b);
    if (rc) return rc;
    if (!stats && image_mem == WSG_MEM_HOST) WSG_HIP(ctx, hipStreamSynchronize(s));
    return read_stats(ctx, b, v, s, stats, ctx->timing != 0);
}

wsg_status wsg_submit(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, double *image,
                      int32_t image_mem, uint64_t *ticket) {
    if (!ctx || !ticket) return WSG_EINVAL;
    *ticket = 0;
    std::string why;
    wsg_status rc = check_params(p, why);
    if (!rc) rc = check_vis(p, v, why);
    if (rc) return fail(ctx, rc, why);
    if (!image) return fail(ctx, WSG_EINVAL, "image is NULL");
    if (image_mem != WSG_MEM_HOST && image_mem != WSG_MEM_DEVICE) return fail(ctx, WSG_EINVAL, "bad image memory space");
    WSG_HIP(ctx, hipSetDevice(ctx->device));
    for (auto &sl : ctx->aslot)
        if (!sl.done) WSG_HIP(ctx, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    auto j = std::make_shared<AsyncJob>();
    j->ticket = ctx->next_ticket++;
    j->p = *p;
    j->v = *v;
    if (v->freq_hz) {
        j->freq.assign(v->freq_hz, v->freq_hz + v->n_chan);
        j->v.freq_hz = j->freq.data();
    }
    j->image = image;
    j->image_mem = image_mem;
    ctx->async_jobs.push_back(j);
    pump_async(ctx);
    *ticket = j->ticket;
    return WSG_OK;
}

wsg_status wsg_poll(wsg_ctx *ctx, uint64_t ticket, int32_t *done, wsg_stats *stats) {
    if (!ctx || !done) return WSG_EINVAL;
    *done = 0;
    std::shared_ptr<AsyncJob> j = find_job(ctx, ticket);
    if (!j) return fail(ctx, WSG_EINVAL, "unknown ticket");
    WSG_HIP(ctx, hipSetDevice(ctx->device));
    wsg_status rc = progress_async(ctx, false);
    if (rc) return rc;
    if (j->state != AsyncJob::kFinished) return WSG_OK;
    *done = 1;
    return report_async(ctx, j, stats);
}

wsg_status wsg_wait(wsg_ctx *ctx, uint64_t ticket, wsg_stats *stats) {
    if (!ctx) return WSG_EINVAL;
    std::shared_ptr<AsyncJob> j = find_job(ctx, ticket);
    if (!j) return fail(ctx, WSG_EINVAL, "unknown ticket");
    WSG_HIP(ctx, hipSetDevice(ctx->device));
    while (j->state != AsyncJob::kFinished) {
        wsg_status rc = progress_async(ctx, true);
        if (rc) return rc;
    }
    return report_async(ctx, j, stats);
}

wsg_status wsg_cancel(wsg_ctx *ctx, uint64_t ticket) {
    if (!ctx) return WSG_EINVAL;
    std::shared_ptr<AsyncJob> j = find_job(ctx, ticket);
    if (!j) return fail(ctx, WSG_EINVAL, "unknown ticket");
    if (j->state == AsyncJob::kOnDevice)
        return fail(ctx, WSG_EBUSY, "the job is already on the device");
    if (j->state == AsyncJob::kQueued) {
        j->status = WSG_ECANCELED;
        j->state = AsyncJob::kFinished;
    }
    return WSG_OK;
}

wsg_status wsg_stage_grid(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, void *grid,
                          int32_t mem, void *stream, wsg_stats *stats) {
    wsg_status rc = common_checks(ctx, p, v);
    if (rc) return rc;
    if (!grid) return fail(ctx, WSG_EINVAL, "grid is NULL");
    if (mem != WSG_MEM_HOST && mem != WSG_MEM_DEVICE) return fail(ctx, WSG_EINVAL, "bad grid memory space");
    hipStream_t s = pick_stream(ctx, stream);
    Binned b;
    rc = bin_job(ctx, p, v, s, false, b);
    if (rc) return rc;
    const Plan &pl = b.pl;
    void *dst = (mem == WSG_MEM_HOST) ? (void *)(b.fx + pl.o_stack) : grid;
    rc = grid_binned(ctx, b, dst, false, true, s);
    if (rc) return rc;
    if (mem == WSG_MEM_HOST) {
        size_t bytes = (size_t)pl.n_img * pl.n_pl * pl.N * pl.N * cplx_size(p);
        WSG_HIP(ctx, hipMemcpyAsync(grid, dst, bytes, hipMemcpyDeviceToHost, s));
        WSG_HIP(ctx, hipStreamSynchronize(s));
    }
    return read_stats(ctx, b, v, s, stats, false);
}

wsg_status wsg_stage_fft(wsg_ctx *ctx, const wsg_params *p, void *planes, int64_t n_planes,
                         int32_t mem, void *stream) {
    wsg_status rc = common_checks(ctx, p, nullptr);
    if (rc) return rc;
    if (!planes || n_planes < 0) return fail(ctx, WSG_EINVAL, "planes is NULL or n_planes < 0");
    if (mem != WSG_MEM_HOST && mem != WSG_MEM_DEVICE) return fail(ctx, WSG_EINVAL, "bad memory space");
    if (n_planes > 65535) return fail(ctx, WSG_EUNSUPPORTED, "more than 65535 planes");
    if (n_planes == 0) return WSG_OK;
    hipStream_t s = pick_stream(ctx, stream);
    int N = p->grid_n;
    bool f64 = f64_mode(p);
    size_t bytes = (size_t)n_planes * N * N * cplx_size(p);
    size_t need = (mem == WSG_MEM_HOST ? 2 : 1) * align_up(bytes);
    rc = ensure_arena(ctx, ctx->fixed, need, s);
    if (rc) return rc;
    char *fx = (char *)ctx->fixed.ptr;
    void *src = planes;
    void *work = fx;
    if (mem == WSG_MEM_HOST) {
        src = fx + align_up(bytes);
        WSG_HIP(ctx, hipMemcpyAsync(src, planes, bytes, hipMemcpyHostToDevice, s));
    }
    const void *tw = nullptr;
    rc = get_twiddle(ctx, N, f64, &tw);
    if (rc) return rc;
    launch_transpose(N, f64, src, work, n_planes, s);
    launch_fft_pass1(N, f64, work, n_planes, tw, Occupancy(), s);
    launch_fft_pass2_store(N, f64, work, src, n_planes, tw, s);
    WSG_HIP(ctx, hipGetLastError());
    if (mem == WSG_MEM_HOST) {
        WSG_HIP(ctx, hipMemcpyAsync(planes, src, bytes, hipMemcpyDeviceToHost, s));
        WSG_HIP(ctx, hipStreamSynchronize(s));
    }
    return WSG_OK;
}

wsg_status wsg_stage_wcorrect(wsg_ctx *ctx, const wsg_params *p, const void *planes,
                              int64_t n_planes, double w_min, double w_max, double sum_w,
                              double *image, int32_t mem, void *stream) {
    wsg_status rc = common_checks(ctx, p, nullptr);
    if (rc) return rc;
    if (!planes || !image || n_planes < 0) return fail(ctx, WSG_EINVAL, "NULL buffer or n_planes < 0");
    if (mem != WSG_MEM_HOST && mem != WSG_MEM_DEVICE) return fail(ctx, WSG_EINVAL, "bad memory space");
    if (!std::isfinite(w_min) || !std::isfinite(w_max) || w_min > w_max || !std::isfinite(sum_w))
        return fail(ctx, WSG_EINVAL, "bad w range or sum_w");
    int lo = (p->plane_hi > p->plane_lo) ? p->plane_lo : 0;
    if (lo + n_planes > p->n_wplanes) return fail(ctx, WSG_EINVAL, "planes beyond n_wplanes");
    hipStream_t s = pick_stream(ctx, stream);
    int N = p->grid_n;
    size_t pbytes = (size_t)n_planes * N * N * cplx_size(p);
    size_t ibytes = (size_t)N * N * 8;
    size_t need = align_up(sizeof(ImgState)) + (mem == WSG_MEM_HOST ? align_up(pbytes) + align_up(ibytes) : 0);
    rc = ensure_arena(ctx, ctx->fixed, need, s);
    if (rc) return rc;
    char *fx = (char *)ctx->fixed.ptr;
    ImgState *st = (ImgState *)fx;
    const void *src = planes;
    double *dst = image;
    if (mem == WSG_MEM_HOST) {
        src = fx + align_up(sizeof(ImgState));
        dst = (double *)(fx + align_up(sizeof(ImgState)) + align_up(pbytes));
        WSG_HIP(ctx, hipMemcpyAsync((void *)src, planes, pbytes, hipMemcpyHostToDevice, s));
    }
    rc = ensure_pin(ctx, sizeof(ImgState));
    if (rc) return rc;
    ImgState *hs = (ImgState *)ctx->pin;
    std::memset(hs, 0, sizeof(ImgState));
    hs->w_min = w_min;
    hs->w_max = w_max;
    hs->dw = (w_max - w_min) / (double)(p->n_wplanes - 2 * w_half(p));
    hs->w0 = w_min - (double)w_half(p) * hs->dw;
    hs->sum_w = sum_w;
    hs->inv_norm = (p->flags & WSG_NORMALIZE) ? (sum_w > 0.0 ? 1.0 / sum_w : 0.0) : 1.0;
    WSG_HIP(ctx, hipMemcpyAsync(st, hs, sizeof(ImgState), hipMemcpyHostToDevice, s));
    WSG_HIP(ctx, hipEventRecord(ctx->pin_done, s));
    const double *inv_c = nullptr;
    rc = get_inv_c(ctx, p, s, &inv_c);
    if (rc) return rc;
    WcorrArgs a{};
    a.N = N;
    a.n_img = 1;
    a.n_pl = (int)n_planes;
    a.plane_lo = lo;
    a.n_w = p->n_wplanes;
    a.phase32 = p->precision == WSG_PREC_F32_PHASE32;
    a.naive_nm1 = (p->flags & WSG_NAIVE_NM1) ? 1 : 0;
    a.cell = p->cell_rad;
    a.st = st;
    a.inv_c = inv_c;
    rc = get_cw(ctx, p, &a.cw, &a.n_cw);
    if (rc) return rc;
    launch_wcorrect(a, f64_mode(p), src, dst, s);
    WSG_HIP(ctx, hipGetLastError());
    if (mem == WSG_MEM_HOST) {
        WSG_HIP(ctx, hipMemcpyAsync(image, dst, ibytes, hipMemcpyDeviceToHost, s));
        WSG_HIP(ctx, hipStreamSynchronize(s));
    }
    return WSG_OK;
}

wsg_status wsg_autotune(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, const char *cache_path,
                        int32_t *best_tile, int32_t *best_ppp) {
    wsg_status rc = common_checks(ctx, p, v);
    if (rc) return rc;
    const auto key = std::make_tuple(p->grid_n, p->n_wplanes, p->support, p->precision,
                                     decade(v->n_rows * (int64_t)v->n_chan));
    const int n_pl = (p->plane_hi > p->plane_lo) ? p->plane_hi - p->plane_lo : p->n_wplanes;
    auto choose = [&](int tile, int ppp) {
        ctx->tuned[key] = tile;
        ctx->tuned_ppp[key] = ppp;
        if (best_tile) *best_tile = tile;
        if (best_ppp) *best_ppp = ppp;
    };
    // a stored choice for this job shape (the last line that matches) is taken as it is
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            int n, nw, sup, prec, dec, tile, ppp, found = 0, ft = 0, fp = 0;
            float ms;
            char line[256];
            while (std::fgets(line, sizeof line, f)) {
                if (std::sscanf(line, "%d %d %d %d %d %d %d %f", &n, &nw, &sup, &prec, &dec, &tile, &ppp,
                                &ms) == 8 &&
                    std::make_tuple(n, nw, sup, prec, dec) == key && (tile == 16 || tile == 32 || tile == 64) &&
                    tile >= min_tile(n) && ppp >= 0) {
                    found = 1;
                    ft = tile;
                    fp = ppp;
                }
            }
            std::fclose(f);
            if (found) {
                choose(ft, fp);
                return WSG_OK;
            }
        }
    }
    hipStream_t s = pick_stream(ctx, ctx->stream);
    float best_ms = 1e30f;
    int best_t = default_tile(p), best_p = 0;
    std::vector<int> ppps{0};
    for (int d : {2, 4})
        if ((n_pl + d - 1) / d < n_pl) ppps.push_back((n_pl + d - 1) / d);
    for (int t : {16, 32, 64}) {
        if (t > p->grid_n || t < min_tile(p->grid_n)) continue;
        for (int ppp : ppps) {
            wsg_params q = *p;
            q.tile = t;
            q.planes_per_pass = ppp;
            uint64_t fp = 0;
            if (ctx->budget && wsg_footprint(&q, v, &fp) == WSG_OK && fp > ctx->budget) continue;
            float acc = 0.f;
            for (int rep = 0; rep < 3; ++rep) {
                WSG_HIP(ctx, hipEventRecord(ctx->ev0, s));
                // the whole path: the tile also sets how much of the stack the
                // transform passes skip, the passes how much of it is held at once
                Binned b;
                rc = bin_job(ctx, &q, v, s, true, b);
                if (rc) return rc;
                Tables tb;
                rc = ctx_tables(ctx, &q, s, tb);
                if (rc) return rc;
                rc = image_binned(ctx, &q, b, (double *)(b.fx + b.pl.o_image), tb, s);
                if (rc) return rc;
                WSG_HIP(ctx, hipEventRecord(ctx->ev1, s));
                WSG_HIP(ctx, hipEventSynchronize(ctx->ev1));
                float ms = 0.f;
                WSG_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
                if (rep > 0) acc += ms;   // first repetition warms the arena
            }
            if (acc < best_ms) {
                best_ms = acc;
                best_t = t;
                best_p = ppp;
            }
        }
    }
    choose(best_t, best_p);
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%d %d %d %d %d %d %d %.4f\n", p->grid_n, p->n_wplanes, p->support, p->precision,
                         decade(v->n_rows * (int64_t)v->n_chan), best_t, best_p, best_ms / 2);
            std::fclose(f);
        }
    }
    return WSG_OK;
}

// ---------------------------------------------------------------- no allocation
// wsg_image on the static scratch array: device inputs and image, workspace and
// tables in the scratch of this GPU, nothing allocated (device or pinned host memory).
wsg_status wsg_image_noalloc(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, double *image,
                             void *stream, wsg_stats *stats) {
    wsg_status rc = common_checks(ctx, p, v);
    if (rc) return rc;
    if (!image) return fail(ctx, WSG_EINVAL, "image is NULL");
    if (v->mem != WSG_MEM_DEVICE)
        return fail(ctx, WSG_EINVAL, "wsg_image_noalloc takes device inputs only (nothing is staged)");
    if (v->n_chan > kNoAllocMaxChan)
        return fail(ctx, WSG_EUNSUPPORTED, "wsg_image_noalloc takes at most 64 channels");
    if (!ctx->scratch) return fail(ctx, WSG_EDEVICE, "no scratch array on this device");
    Binned b;
    b.pl = make_plan(p, v, choose_tile(ctx, p, v), true, false, choose_ppp(ctx, p, v));
    const Plan &pl = b.pl;
    if (pl.n_bins > ((size_t)1 << 27)) return fail(ctx, WSG_EUNSUPPORTED, "more than 2^27 (plane, tile) bins");
    // tables after the job's workspace, copied from host tables that live as long as
    // the process (so the copies may complete after this call returns)
    const bool kbk = p->kernel == WSG_KERNEL_KAISER_BESSEL;
    const std::vector<char> *tab[5] = {
        &host_twiddle(pl.N, pl.f64), needs_inv_c(p) ? &host_inv_c(p) : nullptr,
        needs_cw(p) ? &host_cw(p) : nullptr, kbk ? &host_kb(p->support, kb_beta(p)) : nullptr,
        (kbk && w_half(p) > 0) ? &host_kb(p->w_support, kb_beta_w(p)) : nullptr};
    size_t o_tab[5], off = pl.fixed_bytes;
    for (int i = 0; i < 5; ++i) {
        o_tab[i] = off;
        off = align_up(off + (tab[i] ? tab[i]->size() : 0));
    }
    if (off > kScratchBytes)
        return fail(ctx, WSG_ENOMEM, "job needs " + std::to_string(off) +
                                         " bytes of workspace; wsg_image_noalloc has " +
                                         std::to_string(kScratchBytes));
    hipStream_t s = pick_stream(ctx, stream);
    char *base = (char *)ctx->scratch;
    job_geom(p, v, pl, b.g);
    bind_workspace(b, base, v);
    for (int i = 0; i < 5; ++i)
        if (tab[i])
            WSG_HIP(ctx, hipMemcpyAsync(base + o_tab[i], tab[i]->data(), tab[i]->size(),
                                        hipMemcpyHostToDevice, s));
    if (tab[3]) {
        b.g.kb_series = (const double *)(base + o_tab[3]);
        b.g.kb_n = (int32_t)kb_host(p->support, kb_beta(p)).series.size();
        b.g.kb_poly = (const float *)(base + o_tab[3] + kKbPolyOffset);
    }
    if (tab[4]) {
        b.g.kbw_series = (const double *)(base + o_tab[4]);
        b.g.kbw_n = (int32_t)kb_host(p->w_support, kb_beta_w(p)).series.size();
    }
    double sc[kNoAllocMaxChan];
    for (int c = 0; c < v->n_chan; ++c) sc[c] = v->freq_hz ? v->freq_hz[c] / kSpeedOfLight : 1.0;
    launch_set_scales((double *)(base + pl.o_scale), sc, v->n_chan, s);
    mark(ctx, kMarkStart, s);
    rc = bin_device(ctx, p, b, (uint8_t *)(base + pl.o_mask), (uint32_t *)(base + pl.o_scan), s);
    if (rc) return rc;
    Tables t;
    t.tw = base + o_tab[0];
    t.inv_c = tab[1] ? (const double *)(base + o_tab[1]) : nullptr;
    t.cw = tab[2] ? (const double *)(base + o_tab[2]) : nullptr;
    t.n_cw = tab[2] ? kCwNodes : 0;
    rc = image_binned(ctx, p, b, image, t, s);
    if (rc) return rc;
    mark(ctx, kMarkEnd, s);
    if (!stats) return WSG_OK;
    // stats through pageable host memory: no pinned staging block either
    WorkTotals ht;
    ImgState hs[kNoAllocMaxChan];
    WSG_HIP(ctx, hipMemcpyAsync(&ht, b.wt, sizeof(WorkTotals), hipMemcpyDeviceToHost, s));
    WSG_HIP(ctx, hipMemcpyAsync(hs, b.st, (size_t)pl.n_img * sizeof(ImgState), hipMemcpyDeviceToHost, s));
    WSG_HIP(ctx, hipStreamSynchronize(s));
    return fill_stats(ctx, b, v, ht, hs, stats, ctx->timing != 0);
}

// ---------------------------------------------------------------- device probes
wsg_status wsg_probe_rates(int device, uint64_t copy_bytes, double *lds_f64_adds_per_s,
                           double *copy_bytes_per_s) {
    if (lds_f64_adds_per_s) *lds_f64_adds_per_s = 0.0;
    if (copy_bytes_per_s) *copy_bytes_per_s = 0.0;
    if (hipSetDevice(device) != hipSuccess) return WSG_EDEVICE;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n_cu <= 0)
        return WSG_EDEVICE;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *a = nullptr, *b = nullptr;
    wsg_status rc = WSG_OK;
    auto best_ms = [&](auto launch) -> float {
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
            (void)hipEventRecord(e0, s);
            launch();
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) best = std::min(best, ms);   // the first launch warms up
        }
        return best;
    };
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = WSG_EDEVICE;
    } else {
        // LDS: 8 workgroups per CU, 4 x 2048 adds per lane
        const int blocks = n_cu * 8, iters = 2048, thr = probe_lds_add_threads();
        if (hipMalloc(&a, (size_t)blocks * thr * sizeof(double)) != hipSuccess) {
            rc = WSG_ENOMEM;
        } else {
            const float ms = best_ms([&] { launch_probe_lds_add(blocks, iters, (double *)a, s); });
            if (hipGetLastError() != hipSuccess) rc = WSG_EDEVICE;
            else if (lds_f64_adds_per_s) *lds_f64_adds_per_s = (double)blocks * thr * 4.0 * iters / (ms * 1e-3);
            (void)hipFree(a);
            a = nullptr;
        }
        const size_t bytes = (size_t)copy_bytes & ~(size_t)255;
        if (rc == WSG_OK && bytes > 0) {
            if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess ||
                hipMemsetAsync(a, 0, bytes, s) != hipSuccess) {
                rc = WSG_ENOMEM;
            } else {
                const float ms = best_ms([&] { launch_probe_copy(a, b, bytes, n_cu, s); });
                if (hipGetLastError() != hipSuccess) rc = WSG_EDEVICE;
                else if (copy_bytes_per_s) *copy_bytes_per_s = 2.0 * (double)bytes / (ms * 1e-3);
            }
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    return rc;
}

// ---------------------------------------------------------------- chunked jobs
wsg_status wsg_accum_footprint(const wsg_params *p, int32_t n_chan, uint64_t *bytes) {
    if (!p || !bytes) return WSG_EINVAL;
    std::string why;
    wsg_status rc = check_accum(p, n_chan, why);
    if (rc) return rc;
    const int n_img = (p->flags & WSG_PER_CHANNEL) ? n_chan : 1;
    *bytes = accum_layout(p, n_img, p->tile ? p->tile : default_tile(p)).bytes;
    return WSG_OK;
}

wsg_status wsg_accum_begin(wsg_ctx *ctx, const wsg_params *p, int32_t n_chan, void *stream,
                           wsg_accum **out) {
    if (!out) return WSG_EINVAL;
    *out = nullptr;
    wsg_status rc = common_checks(ctx, p, nullptr);
    if (rc) return rc;
    std::string why;
    rc = check_accum(p, n_chan, why);
    if (rc) return fail(ctx, rc, why);
    hipStream_t s = pick_stream(ctx, stream);
    wsg_accum *a = new (std::nothrow) wsg_accum();
    if (!a) return fail(ctx, WSG_ENOMEM, "accumulator");
    a->ctx = ctx;
    a->p = *p;
    a->n_chan = n_chan;
    a->per_channel = (p->flags & WSG_PER_CHANNEL) != 0;
    a->n_img = a->per_channel ? n_chan : 1;
    a->tile = p->tile ? p->tile : default_tile(p);
    a->L = accum_layout(p, a->n_img, a->tile);
    JobGeom &g = a->g;
    g.N = p->grid_n;
    g.n_img = a->n_img;
    g.n_w = p->n_wplanes;
    g.plane_lo = (p->plane_hi > p->plane_lo) ? p->plane_lo : 0;
    g.n_pl = (p->plane_hi > p->plane_lo) ? p->plane_hi - p->plane_lo : p->n_wplanes;
    g.stack_k0 = 0;
    g.stack_pl = g.n_pl;
    g.S = p->support;
    g.h = (p->support - 1) / 2;
    g.T = a->tile;
    g.NT = g.N / g.T;
    while ((1 << g.logT) < g.T) ++g.logT;
    while ((1 << g.logNT) < g.NT) ++g.logNT;
    a->n_bins = (size_t)a->n_img * g.n_pl * g.NT * g.NT;
    auto undo = [&](wsg_status st) {
        wsg_accum_destroy(a);
        return st;
    };
    if (ctx->budget && ctx->fixed.size + a->L.bytes > ctx->budget)
        return undo(fail(ctx, WSG_ENOMEM, "accumulator of " + std::to_string(a->L.bytes) +
                                              " bytes exceeds the context budget"));
    if (hipStreamCreateWithFlags(&a->copy, hipStreamNonBlocking) != hipSuccess)
        return undo(fail(ctx, WSG_EDEVICE, "copy stream"));
    for (int k = 0; k < 2; ++k)
        if (hipEventCreateWithFlags(&a->copied[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&a->slot_free[k], hipEventDisableTiming) != hipSuccess)
            return undo(fail(ctx, WSG_EDEVICE, "accumulator events"));
    for (int k = 0; k < 2; ++k) {
        a->slot[k] = ctx->slot_spare[k].ptr;
        a->slot_size[k] = ctx->slot_spare[k].size;
        ctx->slot_spare[k] = DevBuf{};
    }
    if (ctx->acc_spare.ptr && ctx->acc_spare.size >= a->L.bytes) {
        a->mem = (char *)ctx->acc_spare.ptr;
        a->mem_size = ctx->acc_spare.size;
        ctx->acc_spare = DevBuf{};
    } else {
        if (ctx->acc_spare.ptr) {
            (void)hipFree(ctx->acc_spare.ptr);
            ctx->acc_spare = DevBuf{};
        }
        hipError_t e = hipMalloc((void **)&a->mem, a->L.bytes);
        if (e != hipSuccess) {
            a->mem = nullptr;
            return undo(fail(ctx, e == hipErrorOutOfMemory ? WSG_ENOMEM : WSG_EDEVICE,
                             std::string("accumulator: ") + hipGetErrorString(e)));
        }
        a->mem_size = a->L.bytes;
    }
    // everything starts at zero except the plane geometry of the state, which the
    // chunks overwrite with their own (identical) values; here it only keeps an
    // accumulator without chunks finite
    std::vector<ImgState> init(a->n_img);
    for (auto &x : init) {
        std::memset(&x, 0, sizeof(x));
        x.w_min = p->w_min;
        x.w_max = p->w_max;
        x.dw = (p->w_max - p->w_min) / (p->n_wplanes - 2 * w_half(p));
        x.w0 = p->w_min - (double)w_half(p) * x.dw;
    }
    if (hipMemsetAsync(a->mem, 0, a->L.bytes, s) != hipSuccess ||
        hipMemcpyAsync(a->mem + a->L.o_state, init.data(), init.size() * sizeof(ImgState),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return undo(fail(ctx, WSG_EDEVICE, "accumulator initialisation"));
    *out = a;
    return WSG_OK;
}

wsg_status wsg_accum_add(wsg_accum *a, const wsg_vis *v, void *stream) {
    if (!a) return WSG_EINVAL;
    wsg_ctx *ctx = a->ctx;
    if (a->broken || a->finished) return fail(ctx, WSG_EINVAL, "accumulator finished or failed");
    wsg_status rc = common_checks(ctx, &a->p, v);
    if (rc) return rc;
    if (a->per_channel && v->n_chan != a->n_chan)
        return fail(ctx, WSG_EINVAL, "a chunk of a cube must have the accumulator's n_chan");
    hipStream_t s = pick_stream(ctx, stream);
    a->per_img_elems += a->per_channel ? v->n_rows : v->n_rows * (int64_t)v->n_chan;
    if (v->n_rows == 0) return WSG_OK;
    wsg_vis dv;
    const wsg_vis *vd = v;
    int slot = -1;
    if (v->mem == WSG_MEM_HOST) {
        rc = stage_chunk(a, v, s, &dv, &slot);
        if (rc) { a->broken = true; return rc; }
        vd = &dv;
    }
    Binned b;
    rc = bin_job(ctx, &a->p, vd, s, false, b, a->tile, false);
    if (rc) { a->broken = true; return rc; }
    launch_work_list(b.g, b.counts, b.offsets, b.pl.n_bins, b.wt, b.items, s);
    launch_grid(b.g, b.pl.f64, b.counts, b.offsets, b.items, b.wt,
                grid_workgroups(b.pl.f64, b.pl.T, b.pl.max_items, ctx->n_cu), b.records,
                a->mem + a->L.o_stack, true, true, s);
    launch_accum_chunk(b.counts, (uint32_t *)(a->mem + a->L.o_seen), a->n_bins, b.st,
                       (ImgState *)(a->mem + a->L.o_state), a->n_img, b.wt,
                       (uint32_t *)(a->mem + a->L.o_overflow), s);
    if (slot >= 0) {
        hipError_t e = hipEventRecord(a->slot_free[slot], s);
        if (e != hipSuccess) { a->broken = true; return fail(ctx, WSG_EDEVICE, "slot event"); }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { a->broken = true; return fail(ctx, WSG_EDEVICE, hipGetErrorString(e)); }
    return WSG_OK;
}

wsg_status wsg_accum_finish(wsg_accum *a, double *image, int32_t image_mem, void *stream,
                            wsg_stats *stats) {
    if (!a) return WSG_EINVAL;
    wsg_ctx *ctx = a->ctx;
    if (a->broken || a->finished) return fail(ctx, WSG_EINVAL, "accumulator finished or failed");
    if (!image) return fail(ctx, WSG_EINVAL, "image is NULL");
    if (image_mem != WSG_MEM_HOST && image_mem != WSG_MEM_DEVICE) return fail(ctx, WSG_EINVAL, "bad image memory space");
    WSG_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    a->finished = true;
    const wsg_params *p = &a->p;
    const bool f64 = f64_mode(p), host_img = image_mem == WSG_MEM_HOST;
    ImgState *st = (ImgState *)(a->mem + a->L.o_state);
    void *stack = a->mem + a->L.o_stack;
    double *img_dev = host_img ? (double *)(a->mem + a->L.o_image) : image;
    const void *tw = nullptr;
    wsg_status rc = get_twiddle(ctx, p->grid_n, f64, &tw);
    if (rc) return rc;
    const double *inv_c = nullptr;
    rc = get_inv_c(ctx, p, s, &inv_c);
    if (rc) return rc;
    launch_post_norm(a->n_img, st, (p->flags & WSG_NORMALIZE) != 0, s);
    Occupancy occ;
    occ.rows = (const uint64_t *)(a->mem + a->L.o_rows);
    occ.live1 = (const uint32_t *)(a->mem + a->L.o_live1);
    occ.live2 = (const uint16_t *)(a->mem + a->L.o_live2);
    occ.logT = a->g.logT;
    occ.nw = occupancy_words(a->g.NT);
    launch_occupancy(a->g, (const uint32_t *)(a->mem + a->L.o_seen), (uint64_t *)occ.rows,
                     (uint32_t *)occ.live1, (uint16_t *)occ.live2, st, s);
    launch_fft_pass1(p->grid_n, f64, stack, (int64_t)a->n_img * a->g.n_pl, tw, occ, s);
    WcorrArgs w{};
    w.N = p->grid_n;
    w.n_img = a->n_img;
    w.n_pl = a->g.n_pl;
    w.plane_lo = a->g.plane_lo;
    w.n_w = p->n_wplanes;
    w.phase32 = p->precision == WSG_PREC_F32_PHASE32;
    w.naive_nm1 = (p->flags & WSG_NAIVE_NM1) ? 1 : 0;
    w.cell = p->cell_rad;
    w.st = st;
    w.inv_c = inv_c;
    w.occ = occ;
    rc = get_cw(ctx, p, &w.cw, &w.n_cw);
    if (rc) return rc;
    launch_fft_pass2_wcorr(w, f64, stack, tw, img_dev, s);
    WSG_HIP(ctx, hipGetLastError());
    if (host_img) {
        WSG_HIP(ctx, hipMemcpyAsync(image, img_dev, (size_t)a->n_img * p->grid_n * p->grid_n * 8,
                                    hipMemcpyDeviceToHost, s));
        WSG_HIP(ctx, hipStreamSynchronize(s));
    }
    if (!stats) return WSG_OK;
    rc = ensure_pin(ctx, align_up(16) + (size_t)a->n_img * sizeof(ImgState));
    if (rc) return rc;
    char *h = (char *)ctx->pin;
    WSG_HIP(ctx, hipMemcpyAsync(h, a->mem + a->L.o_overflow, 16, hipMemcpyDeviceToHost, s));
    WSG_HIP(ctx, hipMemcpyAsync(h + align_up(16), st, (size_t)a->n_img * sizeof(ImgState),
                                hipMemcpyDeviceToHost, s));
    WSG_HIP(ctx, hipStreamSynchronize(s));
    const uint32_t *tot = (const uint32_t *)h;
    if (tot[0] != 0)
        return fail(ctx, WSG_EDEVICE, "internal error: binning passes disagree on record counts");
    const int64_t n_records = (int64_t)((uint64_t)tot[2] << 32 | tot[1]);
    const ImgState *hs = (const ImgState *)(h + align_up(16));
    for (int i = 0; i < a->n_img; ++i) {
        std::memset(&stats[i], 0, sizeof(wsg_stats));
        stats[i].n_used = (int64_t)hs[i].n_used;
        stats[i].n_flagged = (int64_t)hs[i].n_flagged;
        stats[i].n_dropped = a->per_img_elems - stats[i].n_used - stats[i].n_flagged;
        stats[i].n_records = n_records;
        stats[i].n_tiles = (int64_t)hs[i].n_tiles;
        stats[i].n_tile_rows = (int64_t)hs[i].n_tile_rows;
        stats[i].sum_w = hs[i].sum_w;
        stats[i].w_min = hs[i].w_min;
        stats[i].w_max = hs[i].w_max;
    }
    return WSG_OK;
}

void wsg_accum_destroy(wsg_accum *a) {
    if (!a) return;
    (void)hipSetDevice(a->ctx->device);
    if (a->ctx->has_last) (void)hipStreamSynchronize(a->ctx->last_stream);
    if (a->copy) (void)hipStreamSynchronize(a->copy);
    wsg_ctx *ctx = a->ctx;
    for (int k = 0; k < 2; ++k) {
        if (a->slot_free[k]) (void)hipEventSynchronize(a->slot_free[k]);
        if (a->slot[k]) {
            if (!ctx->slot_spare[k].ptr)
                ctx->slot_spare[k] = DevBuf{a->slot[k], a->slot_size[k]};
            else
                (void)hipFree(a->slot[k]);
        }
        if (a->copied[k]) (void)hipEventDestroy(a->copied[k]);
        if (a->slot_free[k]) (void)hipEventDestroy(a->slot_free[k]);
    }
    if (a->mem) {
        if (!ctx->acc_spare.ptr)
            ctx->acc_spare = DevBuf{a->mem, a->mem_size};
        else
            (void)hipFree(a->mem);
    }
    if (a->copy) (void)hipStreamDestroy(a->copy);
    delete a;
}

}  // extern "C"

// device bytes held by a context (its arenas and cached tables), for the server
uint64_t wsg_ctx_device_bytes(const wsg_ctx *ctx) {
    uint64_t b = ctx->fixed.size;
    for (auto &kv : ctx->twiddles) b += kv.second.size;
    for (auto &kv : ctx->inv_c) b += kv.second.size;
    for (auto &kv : ctx->kb) b += kv.second.size;
    for (auto &kv : ctx->cw) b += kv.second.size;
    b += ctx->acc_spare.size + ctx->slot_spare[0].size + ctx->slot_spare[1].size;
    return b;
}
