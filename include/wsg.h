/*
 * wsg.h -- w-stacking gridder/imager for AMD MI355X (gfx950), C ABI.
 *
 * The library images radio-interferometer visibilities with the w-stacking
 * method described in Sec. 2 of De Rubeis et al., "Accelerating radio
 * astronomy imaging with RICK" (arXiv 2411.07321):
 *
 *   1. every visibility (u,v,w in wavelengths, Eq. 1) goes to the closest of
 *      N_w w-planes and is convolved onto the N x N (u,v) mesh of that plane
 *      with a kernel G of support S (Eq. 3);
 *   2. every plane is inverse Fourier transformed (2D, complex-to-complex);
 *   3. each plane is multiplied by the phase screen exp(2 pi i w_k (n - 1)),
 *      n = sqrt(1 - l^2 - m^2), and the planes are summed (Eq. 2); the real
 *      part is the dirty image.
 *
 * Conventions (readings of points the paper leaves open):
 *   - mesh cell i has u_i = (i - N/2) du, du = 1/(N * cell_rad); image pixel p
 *     has l_p = (p - N/2) * cell_rad; arrays are row-major with the u / l
 *     index fastest: grid[k][j][i], image[q][p];
 *   - a visibility sits at x = u * (N * cell_rad) + N/2 (no fused multiply-
 *     add), nearest cell i0 = floor(x + 1/2), footprint i0-h .. i0+h with
 *     h = (S-1)/2; G is separable in u and v: the Gaussian
 *     G(d) = exp(-d^2 / (2 sigma^2)), or the Kaiser-Bessel window the paper's
 *     runs use (Sec. 2, after Eq. 3) G(d) = I0(beta sqrt(1 - (2d/S)^2)) / I0(beta)
 *     on |d| <= S/2 (beta = 0 in wsg_params: pi sqrt((S/2)^2 1.5^2 - 0.8), the
 *     choice of Beatty et al. 2005 for a mesh twice oversampled);
 *   - planes are N_w cells of width dw = (w_max - w_min)/N_w over [w_min,
 *     w_max]; k = min(N_w-1, floor((w - w_min)/dw)), w_k = w_min + (k+1/2) dw;
 *     dw = 0 puts everything on plane 0 at w_0 = w_min;
 *   - the transform is F[q][p] = sum g[j][i] exp(+2 pi i ((i-N/2)(p-N/2) +
 *     (j-N/2)(q-N/2))/N), unnormalised;
 *   - n - 1 is formed as -eta / (1 + sqrt(1 - eta)), eta = l^2 + m^2; pixels
 *     with eta >= 1 are 0;
 *   - image = Re(A) / (sum W * C(nu_p) * C(nu_q)), C the continuous transform
 *     of the truncated kernel, nu_p = (p - N/2)/N; each factor is switched by
 *     WSG_GRID_CORRECT / WSG_NORMALIZE; sum W = 0 gives a zero image.
 *
 * Validity: a visibility is used iff it is unflagged, its weight is finite
 * and > 0, u, v, w and V are finite, its footprint lies inside the mesh and
 * w lies in [w_min, w_max].  Anything else is skipped and counted, never an
 * error.
 *
 * Ownership: the caller owns every input and output buffer; the library never
 * frees or keeps a caller pointer after the call returns (an enqueue-only call
 * reads them until the stream reaches the end of its work).  The library owns
 * its workspace (bins, records, plane stack, tables), keeps it in the context
 * between calls and frees it in wsg_destroy.
 *
 * Errors: no C++ exception crosses this interface.  On error the outputs are
 * unspecified and *stats is not written.  wsg_last_error() gives detail.
 *
 * Threads: a context is used by one host thread at a time; several contexts
 * per device may be used concurrently from different threads.
 */
#ifndef WSG_H
#define WSG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wsg_ctx wsg_ctx;
typedef int32_t wsg_status;

enum {
    WSG_OK = 0,
    WSG_EINVAL = -1,        /* bad parameter, NULL required pointer, bad memory space      */
    WSG_ENOMEM = -2,        /* workspace above the context's budget or device memory        */
    WSG_EDEVICE = -3,       /* HIP runtime error (no device, launch failure, ...)           */
    WSG_EBUSY = -4,         /* the context still has enqueued work it must not overlap      */
    WSG_EUNSUPPORTED = -5,  /* valid but outside what the library supports (e.g. N > 16384) */
    WSG_ECANCELED = -6      /* a submitted job was canceled before it reached the device    */
};

/* Arithmetic of the mesh, the transform and the phase screen. */
enum {
    WSG_PREC_F64 = 0,          /* complex128 mesh and transform, FP64 phase, FP64 image      */
    WSG_PREC_F32_PHASE64 = 1,  /* complex64 mesh and transform, FP64 phase and image sum     */
    WSG_PREC_F32_PHASE32 = 2   /* complex64 mesh and transform, FP32 phase, FP64 image sum   */
};

enum { WSG_MEM_HOST = 0, WSG_MEM_DEVICE = 1 };

/* Gridding kernel G. */
enum { WSG_KERNEL_GAUSSIAN = 0, WSG_KERNEL_KAISER_BESSEL = 1 };

enum {
    WSG_GRID_CORRECT = 1u,   /* divide by C(nu_p) C(nu_q)                                    */
    WSG_NORMALIZE = 2u,      /* divide by sum W                                              */
    WSG_PER_CHANNEL = 4u,    /* one image per channel (a cube) instead of one image          */
    WSG_NAIVE_NM1 = 8u,      /* FP32 phase only: sqrt(1-eta)-1 instead of the stable form    */
    WSG_W_FOLD = 16u         /* rows with w < 0 are gridded at (-u,-v,-w) with conj(V): the   */
                             /*   visibilities of a real sky are Hermitian (Eq. 1), so the    */
                             /*   real image is unchanged and the planes span w >= 0 only    */
};

typedef struct {
    int32_t grid_n;        /* N: power of two, 16 .. 16384                                     */
    int32_t n_wplanes;     /* N_w >= 1                                                         */
    int32_t support;       /* S: odd, 1 .. 15, S <= N                                          */
    int32_t precision;     /* WSG_PREC_*                                                       */
    double cell_rad;       /* image pixel size dl in radians (> 0, finite)                     */
    double kernel_sigma;   /* Gaussian width in cells (> 0); 0.9 is the reading for S = 7;     */
                           /*   not used by the Kaiser-Bessel kernel                          */
    double w_min, w_max;   /* plane range; both NaN: taken from the data                       */
    int32_t plane_lo;      /* image only planes [plane_lo, plane_hi) of N_w (both 0: all);    */
    int32_t plane_hi;      /*   needs a given w range, so that every shard agrees             */
    uint32_t flags;        /* WSG_GRID_CORRECT | WSG_NORMALIZE | ...                           */
    int32_t tile;          /* uv tile edge for binning: 0 = library choice, else 16/32/64,    */
                           /*   at least grid_n / 256                                         */
    int32_t kernel;        /* WSG_KERNEL_*                                                     */
    double kernel_beta;    /* Kaiser-Bessel beta (0 .. 64; 0: the default for S, which S = 1  */
                           /*   lacks: WSG_EINVAL).  FP32 meshes take each tap from a fitted   */
                           /*   degree-8 polynomial; a beta it cannot follow within 2e-7 is    */
                           /*   WSG_EUNSUPPORTED there (the FP64 mesh takes any beta)          */
    int32_t w_support;     /* planes a visibility spreads over (Eq. 3's G in w): 0 or 1 = its */
                           /*   nearest plane only; odd 3 .. 15: the kernel's kind over that  */
                           /*   many planes (Gaussian: the same sigma in planes; Kaiser-      */
                           /*   Bessel: beta, or the default for w_support), the w range       */
                           /*   covering the middle N_w - 2 h_w planes, and WSG_GRID_CORRECT   */
                           /*   also divides by its transform at dw (n - 1).  Needs N_w >=    */
                           /*   w_support and the full plane range                             */
    int32_t planes_per_pass; /* planes of each image held in the w-stack at a time: 0 = all   */
                           /*   (or the choice wsg_autotune stored); fewer make several passes */
                           /*   over the planes, each gridding, transforming and w-correcting  */
                           /*   its planes into the image, with that fraction of the stack's   */
                           /*   memory (wsg_image and wsg_image_noalloc)                       */
} wsg_params;

typedef struct {
    int64_t n_rows;          /* rows (baseline x time samples)                                */
    int32_t n_chan;          /* channels per row (>= 1)                                       */
    int32_t mem;             /* WSG_MEM_* of uvw, vis, weights and flags                      */
    int64_t row_period;      /* performance hint, results do not depend on it: rows of one    */
                             /*   baseline recur every row_period rows (the baselines per     */
                             /*   time slice of time-major data); 0 or 1 = no such structure  */
    const double *uvw;       /* [n_rows][3]; wavelengths if freq_hz is NULL, else metres      */
    const double *freq_hz;   /* HOST array [n_chan] or NULL                                   */
    const void *vis;         /* [n_rows][n_chan] interleaved (re, im): complex128 if F64,    */
                             /*   else complex64                                               */
    const void *weights;     /* [n_rows][n_chan]: double if F64 else float; NULL = all 1     */
    const uint8_t *flags;    /* [n_rows][n_chan]: nonzero = skip; NULL = none                 */
} wsg_vis;

typedef struct {
    int64_t n_used, n_flagged, n_dropped;
    int64_t n_records;       /* binning records of the whole job: one per (visibility, uv     */
                             /*   tile its footprint touches)                                 */
    int64_t n_tiles;         /* wsg_image: (plane, uv tile) cells of this image's w-stack     */
                             /*   that received visibilities; the rest are never written or   */
                             /*   read (0 from the stage entry points)                        */
    int64_t n_tile_rows;     /* wsg_image: (plane, tile row) pairs with such a tile           */
    double sum_w, w_min, w_max;
    /* device time in ms between hipEvents recorded on the job's stream, filled when
     * timing is on (wsg_set_timing); all 0 otherwise.  The stages are: staging of
     * host inputs and the validity pass; counting and scans; record scatter;
     * clearing of split tiles; gridding (the gridding kernel alone); the tile
     * occupancy pass; transform pass 1; transform pass 2 with w-correction and
     * plane sum.  ms_total spans the whole call, host waits included. */
    float ms_prep, ms_count, ms_scatter, ms_zero, ms_grid, ms_occupancy, ms_fft1, ms_fft2_wcorr,
        ms_total;
} wsg_stats;

/* ---------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------- */
/* Bind a context to HIP device `device`.  *out is NULL on error. */
wsg_status wsg_create(int device, wsg_ctx **out);
/* Wait for the context's work, free its workspace and the context.  NULL is a no-op. */
void wsg_destroy(wsg_ctx *ctx);
const char *wsg_strerror(wsg_status s);
/* Detail of the last failure on this context (never NULL). */
const char *wsg_last_error(const wsg_ctx *ctx);
/* The context's own hipStream_t (non-blocking, default priority), for callers that
 * want the library's work off the null stream; NULL for a NULL context.  Valid
 * until wsg_destroy. */
void *wsg_context_stream(const wsg_ctx *ctx);
/* Limit the context's workspace to `bytes` (0 = no limit); larger jobs fail with ENOMEM. */
wsg_status wsg_set_budget(wsg_ctx *ctx, uint64_t bytes);
/* Record hipEvents between the stages of wsg_image and report their durations in
 * wsg_stats (on = 1) or not (on = 0, the default). */
wsg_status wsg_set_timing(wsg_ctx *ctx, int32_t on);

/* ---------------------------------------------------------------------------
 * Host-side checks (no device needed)
 * ------------------------------------------------------------------------- */
/* Validate parameters and input description (pointers need not be dereferenceable). */
wsg_status wsg_check(const wsg_params *p, const wsg_vis *v);
/* Device workspace in bytes that wsg_image needs for this job (inputs staged
 * from host memory included), for admission control. */
wsg_status wsg_footprint(const wsg_params *p, const wsg_vis *v, uint64_t *bytes);
/* Number of images the job produces: n_chan with WSG_PER_CHANNEL, else 1. */
int32_t wsg_n_images(const wsg_params *p, const wsg_vis *v);

/* ---------------------------------------------------------------------------
 * The method, end to end (Sec. 2: gridding, transform, w-correction and sum)
 * ------------------------------------------------------------------------- */
/*
 * image: [n_images][N][N] double, row-major (p fastest), in memory space
 *        image_mem; written completely.
 * stream: hipStream_t to run on; NULL is HIP's null stream, which is ordered
 *         after the work of every blocking stream of the device (torch's default
 *         stream is this stream).  The calls on one context must not overlap:
 *         switching streams waits for the previous stream.
 * stats:  NULL, or an array of n_images entries; when given, the call waits
 *         for the device and fills it.  With stats NULL and a device image the
 *         call may return before the work is done; synchronise `stream`.
 */
wsg_status wsg_image(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v,
                     double *image, int32_t image_mem, void *stream, wsg_stats *stats);

/* ---------------------------------------------------------------------------
 * The method, asynchronously: jobs submitted to a context
 * ------------------------------------------------------------------------- */
/*
 * wsg_submit validates the job (errors of wsg_check are returned at once) and queues
 * it; the context runs its submitted jobs one after another, in submission order, on
 * its own stream (wsg_context_stream), with at most two of them on the device at a
 * time, so that the host side of the next job overlaps the device work of the
 * previous one.  Jobs reach the device from wsg_submit, wsg_poll and wsg_wait; nothing
 * runs in the background.  A job's buffers (inputs, freq_hz excepted: it is copied,
 * and image) must stay valid until the job is reported done.  A host image makes the
 * call that puts the job on the device wait for it (the copy out is synchronous).
 *   wsg_poll: *done = 0 while the job runs; once finished, *done = 1 and the return
 *             value is the job's own status (stats, NULL or n_images entries, filled
 *             on success); the ticket is then forgotten.
 *   wsg_wait: waits for the job, then as wsg_poll with *done = 1.
 *   wsg_cancel: a job still queued on the host is dropped; wsg_poll / wsg_wait then
 *             report WSG_ECANCELED.  A job already on the device cannot be canceled
 *             (WSG_EBUSY); a finished one is left as it is.
 * Stage times are not measured for submitted jobs (the ms_* fields are 0).  While any
 * submitted job is unfinished, the other calls on the context (wsg_image, the stages,
 * the chunked calls, wsg_autotune) fail with WSG_EBUSY.  wsg_destroy drops queued jobs
 * and waits for those on the device.  An unknown or already reported ticket is
 * WSG_EINVAL.
 */
wsg_status wsg_submit(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, double *image,
                      int32_t image_mem, uint64_t *ticket);
wsg_status wsg_poll(wsg_ctx *ctx, uint64_t ticket, int32_t *done, wsg_stats *stats);
wsg_status wsg_wait(wsg_ctx *ctx, uint64_t ticket, wsg_stats *stats);
wsg_status wsg_cancel(wsg_ctx *ctx, uint64_t ticket);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): wsg_image without any
 * allocation.  The workspace (binning state, records, work list, the w-stack) and the
 * transform tables live in one static device array of 64 MiB per GPU that the library
 * holds from its first wsg_create on that GPU until the process ends; nothing else is
 * allocated (no device memory, no pinned host memory).
 *   - uvw, vis, weights, flags and image must be device buffers (v->mem =
 *     WSG_MEM_DEVICE); at most 64 channels;
 *   - a job whose workspace exceeds 64 MiB fails with WSG_ENOMEM before any device
 *     work (roughly: N_w x N^2 x 8 bytes of complex64 stack plus 64 bytes per
 *     visibility, e.g. N = 512 with 8 planes and 500,000 visibilities);
 *   - every call on one GPU uses that GPU's one array, whatever the context: calls
 *     that overlap in time on one GPU (two host threads, or two streams whose work
 *     interleaves) race and give wrong results; order them on one stream or wait;
 *   - the result equals wsg_image's up to the order of floating-point sums.
 * stream and stats as for wsg_image (stats are read back through pageable host
 * memory, so a call with stats waits for the device).
 */
wsg_status wsg_image_noalloc(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v, double *image,
                             void *stream, wsg_stats *stats);

/* ---------------------------------------------------------------------------
 * Stages, separately (for checking each step)
 * ------------------------------------------------------------------------- */
/* Eq. 3 on the nearest plane: grid [n_images][hi-lo][N][N] complex (complex128
 * for F64, else complex64), overwritten. */
wsg_status wsg_stage_grid(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v,
                          void *grid, int32_t mem, void *stream, wsg_stats *stats);
/* Centred unnormalised inverse transform of n_planes N x N planes, in place. */
wsg_status wsg_stage_fft(wsg_ctx *ctx, const wsg_params *p, void *planes, int64_t n_planes,
                         int32_t mem, void *stream);
/* w-correction and plane sum of n_planes transformed planes that hold planes
 * plane_lo .. plane_lo+n_planes-1 of the range [w_min, w_max] (Eq. 2), then
 * the post factors with sum_w: image [N][N] double. */
wsg_status wsg_stage_wcorrect(wsg_ctx *ctx, const wsg_params *p, const void *planes,
                              int64_t n_planes, double w_min, double w_max, double sum_w,
                              double *image, int32_t mem, void *stream);

/* ---------------------------------------------------------------------------
 * Chunked imaging: data larger than one call, loaded chunk after chunk by time
 * or by frequency (the paper's Discussion, Sec. 5), onto one resident w-stack
 * ------------------------------------------------------------------------- */
/*
 * An accumulator owns the w-stack of one imaging job (n_images x planes x N x N,
 * complex64 or complex128; wsg_accum_footprint says how much) plus small state.
 * Each wsg_accum_add bins and grids one chunk of visibilities (Eq. 3) into it;
 * wsg_accum_finish transforms, w-corrects and sums the planes (Eq. 2) into the
 * image.  The result equals wsg_image over the concatenated chunks (up to the
 * order of floating-point sums).
 *
 * Rules:
 *   - the w range must be given (w_min, w_max finite): planes are fixed before
 *     the data are seen; a plane range [plane_lo, plane_hi) is allowed;
 *   - n_chan: with WSG_PER_CHANNEL every chunk has n_chan channels (a chunk of
 *     time of a cube); without it (one image) chunks may differ in n_chan and
 *     freq_hz (chunks of frequency);
 *   - the tile size is fixed by the parameters at begin (0: the library choice
 *     for N and S);
 *   - the calls on one accumulator and its context must not overlap; the
 *     context may run other jobs between them (each chunk's binning workspace
 *     is the context's).
 * Host chunks are copied to the device on a copy stream of the accumulator:
 * the copy of one chunk overlaps the scatter and gridding of the previous one
 * (from pinned host memory the copy runs at full rate).  A chunk's host
 * buffers may be reused when wsg_accum_add returns.
 * Errors: WSG_EINVAL (bad parameters, w range not given, n_chan mismatch),
 * WSG_ENOMEM (stack allocation), WSG_EDEVICE.  An error during add leaves the
 * accumulator unusable (finish returns WSG_EINVAL); destroy it.
 */
typedef struct wsg_accum wsg_accum;
/* Allocate and clear the w-stack on `stream`.  *out is NULL on error. */
wsg_status wsg_accum_begin(wsg_ctx *ctx, const wsg_params *p, int32_t n_chan, void *stream,
                           wsg_accum **out);
/* Device bytes the accumulator itself holds (stack, occupancy, state). */
wsg_status wsg_accum_footprint(const wsg_params *p, int32_t n_chan, uint64_t *bytes);
/* Bin and grid one chunk (may be empty).  Returns once the chunk's work is
 * enqueued on `stream` (the chunk's record count is read back on the way). */
wsg_status wsg_accum_add(wsg_accum *a, const wsg_vis *chunk, void *stream);
/* Transform, w-correct, sum and post-process into image (as wsg_image); stats
 * (NULL or n_images entries) cover every chunk added: n_records is their sum,
 * the stage times are 0.  The accumulator can be finished once. */
wsg_status wsg_accum_finish(wsg_accum *a, double *image, int32_t image_mem, void *stream,
                            wsg_stats *stats);
/* Wait for the accumulator's work and free it.  NULL is a no-op. */
void wsg_accum_destroy(wsg_accum *a);

/* ---------------------------------------------------------------------------
 * Tuning
 * ------------------------------------------------------------------------- */
/* Time the whole imaging path on this job's data, on the context's own stream, at each
 * binning tile size (16, 32, 64, at least grid_n / 256) and each number of planes per
 * pass over the w-stack (all, half, a quarter; candidates whose footprint exceeds the
 * context's budget are skipped), and store the fastest pair per (N, N_w, S, precision,
 * visibility-count decade) in the context: later calls with tile = 0 and
 * planes_per_pass = 0 use it.  With cache_path, a line for this job shape already in the
 * file (the last one) is taken without timing; otherwise the choice is appended as
 * "N N_w S precision decade tile planes_per_pass ms".  *best_tile and *best_ppp (0 = all
 * planes at once) receive the choice (each may be NULL).  Waits for the device. */
wsg_status wsg_autotune(wsg_ctx *ctx, const wsg_params *p, const wsg_vis *v,
                        const char *cache_path, int32_t *best_tile, int32_t *best_ppp);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent imaging jobs on one device
 * ------------------------------------------------------------------------- */
/*
 * A server owns n_slots worker threads, each with its own context (stream and
 * workspace).  Submitted jobs wait in a FIFO queue and are admitted while a
 * slot is free and the device memory held by all slots stays within
 * hbm_budget bytes (0 = no limit): the first queued job that fits is started,
 * so a large job does not block smaller ones behind it.  Admitted jobs run
 * concurrently on their slots' streams; their staging copies, kernels and
 * read-back overlap on the device.  A job that fails (bad parameters, a device
 * error) completes with its error status; the other jobs are unaffected.  (For
 * checks of that isolation, the environment variable WSG_SERVER_FAIL_GRID_N, read
 * when the server is created, makes every job of that mesh size fail in its slot
 * with WSG_EDEVICE before any device work.)
 * Buffers of a job (inputs, freq_hz, image) must stay valid until it is
 * reported done.  A job whose footprint alone exceeds the budget fails with
 * WSG_ENOMEM.
 */
typedef struct wsg_server wsg_server;

typedef struct {
    wsg_status status;       /* result of the job                                            */
    double t_submit, t_start, t_end;   /* seconds on a monotonic clock                       */
    uint64_t footprint;      /* bytes accounted for admission                                */
    wsg_stats stats;         /* stats of the (first) image                                   */
} wsg_job_info;

wsg_status wsg_server_create(int device, int32_t n_slots, uint64_t hbm_budget, wsg_server **out);
/* Wait for every job, then stop the workers and free their workspace. */
void wsg_server_destroy(wsg_server *srv);
wsg_status wsg_server_submit(wsg_server *srv, const wsg_params *p, const wsg_vis *v, double *image,
                             int32_t image_mem, uint64_t *ticket);
/* *done = 1 and *info filled once the job has finished (either way). */
wsg_status wsg_server_poll(wsg_server *srv, uint64_t ticket, int32_t *done, wsg_job_info *info);
wsg_status wsg_server_wait(wsg_server *srv, uint64_t ticket, wsg_job_info *info);
/* Drop a job that is still queued (not yet admitted): it is then reported done with
 * status WSG_ECANCELED.  WSG_EBUSY if a slot already runs it; a finished job is left
 * as it is. */
wsg_status wsg_server_cancel(wsg_server *srv, uint64_t ticket);
/* Current and peak device bytes held by the slots (their workspaces). */
wsg_status wsg_server_memory(wsg_server *srv, uint64_t *held, uint64_t *peak);
/* Release the workspace of every idle slot. */
wsg_status wsg_trim(wsg_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Device probes (measurement of the roofline's peaks; not part of the method)
 * ------------------------------------------------------------------------- */
/* Measured on `device` with this library's own kernels, best of three timed launches:
 *   *lds_f64_adds_per_s: FP64 atomic adds into LDS without a returned value, one
 *       double per lane, no bank conflicts (the operation of the gridder's flushes);
 *   *copy_bytes_per_s: bytes read plus written per second by a 16-byte streaming copy
 *       of copy_bytes bytes (0 skips it; two buffers of that size are allocated).
 * Outputs may be NULL.  Waits for the device.  WSG_ENOMEM if the buffers do not fit. */
wsg_status wsg_probe_rates(int device, uint64_t copy_bytes, double *lds_f64_adds_per_s,
                           double *copy_bytes_per_s);

/* LDS atomic add rate on `device` (adds per second, best of three timed launches, no
 * returned value), by kind: 0 FP64 with every lane on its own bank pair (as in
 * wsg_probe_rates), 1 FP32 with every lane on its own bank, 2 FP64 with two lanes per
 * bank pair, 3 FP64 with sixteen lanes per bank pair.  The gridder's flushes are FP64
 * adds at positions that collide on banks; kind 1 is the rate an FP32 tile would see.
 * WSG_EINVAL for another kind or a NULL output; waits for the device. */
wsg_status wsg_probe_lds(int device, int32_t kind, double *adds_per_s);

#ifdef __cplusplus
}
#endif

#endif /* WSG_H */
