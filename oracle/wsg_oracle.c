/*
 * FP64 CPU oracle of the w-stacking imager -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the slow, plain reference against which the HIP library is
 * checked.  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline may load it; the product path never does.  It shares no code,
 * header or table with the HIP library.
 *
 * Paper: De Rubeis et al., "Accelerating radio astronomy imaging with RICK"
 * (arXiv 2411.07321).  Sec. 2 defines the method:
 *   - visibilities V(u,v,w), (u,v,w) in wavelengths (Eq. 1 and the text below it);
 *   - each visibility goes to the closest w-plane (Sec. 2, w-stacking paragraph);
 *   - it is convolved onto the (u,v) mesh of its plane with a kernel G (Eq. 3);
 *   - each plane is inverse-Fourier transformed, phase-corrected with
 *     exp(+2 pi i w (sqrt(1-l^2-m^2) - 1)) and the planes are summed (Eq. 2,
 *     and the description of the third and fourth algorithmic components).
 *
 * Readings of points the paper leaves open (listed in the design notes):
 *   - G is separable in u and v, support S odd, h = (S-1)/2 cells on each
 *     side of the nearest cell i0 = floor(x + 1/2); either a Gaussian
 *     G(d) = exp(-d^2 / (2 sigma^2)) or the Kaiser-Bessel window the paper's
 *     runs use (Sec. 2, after Eq. 3; Jackson et al. 1991)
 *     G(d) = I0(beta sqrt(1 - (2d/S)^2)) / I0(beta) for |d| <= S/2;
 *   - x = u * (N * dl) + N/2 with no fused multiply-add, so that the cell and
 *     plane decisions are reproducible bit for bit;
 *   - N_w cell-centred planes over [w_min, w_max]: dw = (w_max - w_min)/N_w,
 *     k = min(N_w - 1, floor((w - w_min)/dw)), w_k = w_min + (k + 1/2) dw;
 *     dw = 0 puts everything on plane 0 at w_0 = w_min;
 *   - a measurement is used iff it is unflagged, its weight is finite and > 0,
 *     u, v, w and V are finite, its footprint lies inside the grid and its w
 *     lies inside [w_min, w_max]; everything else is skipped and counted.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the parallel loops below (n > 0 sets them); returns the count in use. */
int oracle_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

typedef struct {
    int64_t n_used;     /* measurements that enter the image (all planes)      */
    int64_t n_flagged;  /* flag != 0                                           */
    int64_t n_dropped;  /* unflagged but unused (bad value, off-grid, off-w)   */
    double  sum_w;      /* sum of weights of used measurements                 */
} oracle_counts;

/* Position of one measurement on the mesh (Eq. 3 support placement). */
static void position(double u, double v, double scale, int n, double *x, double *y)
{
    double half = 0.5 * (double)n;
    double ux = u * scale;          /* one rounding for the product ... */
    double vy = v * scale;
    *x = ux + half;                 /* ... and one for the sum          */
    *y = vy + half;
}

/* Footprint test: i0 = floor(x + 1/2) must satisfy h <= i0 <= N-1-h. */
static int fits(double x, int n, int h, int64_t *i0)
{
    double f = floor(x + 0.5);
    if (!(f >= (double)h && f <= (double)(n - 1 - h))) return 0;
    *i0 = (int64_t)f;
    return 1;
}

static int is_valid0(const double *uvw_row, double sc, const double *vis_rc, double wt,
                     uint8_t flag, double scale, int n, int h)
{
    if (flag) return 0;
    if (!(wt > 0.0) || !isfinite(wt)) return 0;
    double u = uvw_row[0] * sc, v = uvw_row[1] * sc, w = uvw_row[2] * sc;
    if (!isfinite(u) || !isfinite(v) || !isfinite(w)) return 0;
    if (!isfinite(vis_rc[0]) || !isfinite(vis_rc[1])) return 0;
    double x, y;
    int64_t i0, j0;
    position(u, v, scale, n, &x, &y);
    return fits(x, n, h, &i0) && fits(y, n, h, &j0);
}

/*
 * Range of w over the measurements that pass every test except the w-range
 * cut (the "from the data" default of the plane placement).
 * chan < 0: all channels; else only that channel.
 * Returns the number of such measurements; *w_lo/*w_hi untouched if none.
 */
int64_t oracle_w_range(int64_t n_rows, int n_chan, const double *uvw, const double *chan_scale,
                       const double *vis, const double *weights, const uint8_t *flags,
                       int n, int support, double cell, int chan,
                       double *w_lo, double *w_hi)
{
    int h = (support - 1) / 2;
    double scale = (double)n * cell;
    int64_t cnt = 0;
    double lo = 0.0, hi = 0.0;
    for (int64_t r = 0; r < n_rows; ++r) {
        for (int c = 0; c < n_chan; ++c) {
            if (chan >= 0 && c != chan) continue;
            int64_t rc = r * n_chan + c;
            double wt = weights ? weights[rc] : 1.0;
            uint8_t fl = flags ? flags[rc] : 0;
            if (!is_valid0(uvw + 3 * r, chan_scale[c], vis + 2 * rc, wt, fl, scale, n, h))
                continue;
            double w = uvw[3 * r + 2] * chan_scale[c];
            if (cnt == 0) { lo = w; hi = w; }
            if (w < lo) lo = w;
            if (w > hi) hi = w;
            ++cnt;
        }
    }
    if (cnt) { *w_lo = lo; *w_hi = hi; }
    return cnt;
}

/* Nearest w-plane (cell-centred planes over [w_min, w_max]). */
static int plane_of(double w, double w_min, double dw, int n_w)
{
    if (dw == 0.0) return 0;
    double t = floor((w - w_min) / dw);
    int k = (int)t;
    if (k > n_w - 1) k = n_w - 1;
    return k;
}

/* Modified Bessel function of the first kind, order 0, by its power series
 * sum_k (x^2/4)^k / (k!)^2 (every term positive), summed until a term no
 * longer changes the sum. */
double oracle_bessel_i0(double x)
{
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        double next = sum + term;
        if (next == sum) break;
        sum = next;
    }
    return sum;
}

/* The gridding kernel at offset d (cells): kind 0 Gaussian with par = sigma,
 * kind 1 Kaiser-Bessel with par = beta over the support S.  0 outside |d| <= S/2. */
double oracle_kernel_value(int kind, double par, int support, double d)
{
    if (kind == 0) return exp(-d * d / (2.0 * par * par));
    double t = 2.0 * d / (double)support;
    double u = 1.0 - t * t;
    if (u < 0.0) return 0.0;
    return oracle_bessel_i0(par * sqrt(u)) / oracle_bessel_i0(par);
}

/*
 * Plane geometry.  Without a kernel in w (w_support 1) the N_w planes are cells
 * of width dw = (w_max - w_min)/N_w from w0 = w_min.  With a kernel of
 * w_support = 2 h_w + 1 planes, the data range [w_min, w_max] covers the middle
 * N_w - 2 h_w planes and h_w more on each side take the kernel's tails:
 * dw = (w_max - w_min)/(N_w - 2 h_w), w0 = w_min - h_w dw.  Plane k sits at
 * w_k = w0 + (k + 1/2) dw (w0 when dw = 0).
 */
void oracle_plane_geometry(double w_min, double w_max, int n_w, int w_support, double *w0,
                           double *dw)
{
    int hw = (w_support - 1) / 2;
    *dw = (w_max - w_min) / (double)(n_w - 2 * hw);
    *w0 = w_min - (double)hw * *dw;
}

/*
 * Eq. 3:
 *   g_k[j0+b][i0+a] += W V G(i0+a-x) G(j0+b-y) G_w((w_k - w)/dw),
 * a, b in [-h, h], k = k0 - h_w .. k0 + h_w around the plane k0 whose cell holds
 * w; G_w is the kernel of the same kind over w_support planes (shape wpar), and
 * 1 for w_support 1 or dw = 0 (every plane then at w0: the visibility stays on k0).
 * grid: complex128 interleaved [plane_hi-plane_lo][N][N] (row j, column i),
 * accumulated into (the caller zeroes it).  Only planes in [plane_lo,
 * plane_hi) are gridded; the counts cover every plane.
 * Threads: the mesh rows are split into one band per thread; every thread walks
 * all measurements in their order and adds only the footprint rows of its band,
 * so each cell receives its terms in the same order as with one thread and the
 * result does not depend on the thread count.
 */
int oracle_grid(int64_t n_rows, int n_chan, const double *uvw, const double *chan_scale,
                const double *vis, const double *weights, const uint8_t *flags,
                int n, int n_w, int support, double cell, int kernel, double kpar,
                int w_support, double wpar,
                double w_min, double w_max, int plane_lo, int plane_hi, int chan,
                double *grid, oracle_counts *counts)
{
    int h = (support - 1) / 2;
    double scale = (double)n * cell;
    double w0, dw;
    oracle_plane_geometry(w_min, w_max, n_w, w_support, &w0, &dw);
    int hw = dw == 0.0 ? 0 : (w_support - 1) / 2;
    if (support > 63) return -1;
#pragma omp parallel
    {
    int band = 0, n_band = 1;
#ifdef _OPENMP
    band = omp_get_thread_num();
    n_band = omp_get_num_threads();
#endif
    const int64_t j_lo = (int64_t)n * band / n_band, j_hi = (int64_t)n * (band + 1) / n_band;
    double gx[64], gy[64];
    oracle_counts cnt = {0, 0, 0, 0.0};
    for (int64_t r = 0; r < n_rows; ++r) {
        for (int c = 0; c < n_chan; ++c) {
            if (chan >= 0 && c != chan) continue;
            int64_t rc = r * n_chan + c;
            double wt = weights ? weights[rc] : 1.0;
            uint8_t fl = flags ? flags[rc] : 0;
            if (fl) { cnt.n_flagged++; continue; }
            if (!is_valid0(uvw + 3 * r, chan_scale[c], vis + 2 * rc, wt, fl, scale, n, h)) {
                cnt.n_dropped++;
                continue;
            }
            double u = uvw[3 * r + 0] * chan_scale[c];
            double v = uvw[3 * r + 1] * chan_scale[c];
            double w = uvw[3 * r + 2] * chan_scale[c];
            if (!(w >= w_min && w <= w_max)) { cnt.n_dropped++; continue; }
            cnt.n_used++;
            cnt.sum_w += wt;
            int k0 = plane_of(w, w0, dw, n_w);
            /* the kernel's planes must exist: a w at the edge of the range can round
             * into the padding planes */
            if (hw > 0) {
                if (k0 < hw) k0 = hw;
                if (k0 > n_w - 1 - hw) k0 = n_w - 1 - hw;
            }
            double x, y;
            int64_t i0, j0;
            position(u, v, scale, n, &x, &y);
            fits(x, n, h, &i0);
            fits(y, n, h, &j0);
            if (j0 + h < j_lo || j0 - h >= j_hi) continue;   /* no row of this band */
            for (int a = -h; a <= h; ++a)
                gx[a + h] = oracle_kernel_value(kernel, kpar, support, (double)(i0 + a) - x);
            for (int b = -h; b <= h; ++b)
                gy[b + h] = oracle_kernel_value(kernel, kpar, support, (double)(j0 + b) - y);
            for (int k = k0 - hw; k <= k0 + hw; ++k) {
                if (k < plane_lo || k >= plane_hi) continue;
                double gw = 1.0;
                if (hw > 0) {
                    double wk = w0 + ((double)k + 0.5) * dw;
                    gw = oracle_kernel_value(kernel, wpar, w_support, (wk - w) / dw);
                }
                double wv_re = wt * vis[2 * rc + 0] * gw;
                double wv_im = wt * vis[2 * rc + 1] * gw;
                double *plane = grid + (size_t)(k - plane_lo) * (size_t)n * (size_t)n * 2;
                for (int b = -h; b <= h; ++b) {
                    if (j0 + b < j_lo || j0 + b >= j_hi) continue;
                    double *row = plane + ((size_t)(j0 + b) * (size_t)n) * 2;
                    for (int a = -h; a <= h; ++a) {
                        double g = gx[a + h] * gy[b + h];
                        size_t i = (size_t)(i0 + a) * 2;
                        row[i + 0] += wv_re * g;
                        row[i + 1] += wv_im * g;
                    }
                }
            }
        }
    }
    if (band == 0 && counts) *counts = cnt;   /* every band counts every measurement */
    }
    return 0;
}

/*
 * The raw image A(q,p) at a list of pixels, evaluated directly from the
 * measurements instead of through the mesh (the same discrete sum, taken in
 * the other order):
 *   A(q,p) = sum_used W V [sum_a G(i0+a-x) e^{2 pi i (i0+a-N/2)(p-N/2)/N}]
 *                        [sum_b G(j0+b-y) e^{2 pi i (j0+b-N/2)(q-N/2)/N}]
 *                        e^{2 pi i w_k (n_pq - 1)},
 * with n_pq - 1 = -eta/(1 + sqrt(1 - eta)), eta = l_p^2 + m_q^2, and A = 0
 * where eta >= 1.  The integer product (i0+a-N/2)(p-N/2) is reduced mod N
 * exactly before the exponential is taken.
 * Used for sampled checks at sizes where the full mesh is too large.
 * out: complex128 interleaved [n_pix].  Deterministic: partial sums per
 * thread block of rows are added in block order.
 */
int oracle_pixels(int64_t n_rows, int n_chan, const double *uvw, const double *chan_scale,
                  const double *vis, const double *weights, const uint8_t *flags,
                  int n, int n_w, int support, double cell, int kernel, double kpar,
                  double w_min, double w_max, int chan,
                  int n_pix, const int32_t *pix_q, const int32_t *pix_p, double *out)
{
    const double two_pi = 6.283185307179586476925286766559;
    int h = (support - 1) / 2;
    double scale = (double)n * cell;
    double dw = (w_max - w_min) / (double)n_w;
    if (support > 63 || n_pix <= 0) return n_pix < 0 ? -1 : 0;

    double *ct = (double *)malloc(sizeof(double) * (size_t)n);
    double *st = (double *)malloc(sizeof(double) * (size_t)n);
    double *wk = (double *)malloc(sizeof(double) * 2 * (size_t)n_pix * (size_t)n_w);
    for (int t = 0; t < n; ++t) {
        ct[t] = cos(two_pi * (double)t / (double)n);
        st[t] = sin(two_pi * (double)t / (double)n);
    }
    for (int ip = 0; ip < n_pix; ++ip) {
        double l = (double)(pix_p[ip] - n / 2) * cell;
        double m = (double)(pix_q[ip] - n / 2) * cell;
        double eta = l * l + m * m;
        for (int k = 0; k < n_w; ++k) {
            double *e = wk + 2 * ((size_t)ip * n_w + k);
            if (eta >= 1.0) { e[0] = 0.0; e[1] = 0.0; continue; }
            double nm1 = -eta / (1.0 + sqrt(1.0 - eta));
            double wkk = (dw == 0.0) ? w_min : w_min + ((double)k + 0.5) * dw;
            double ph = two_pi * wkk * nm1;
            e[0] = cos(ph);
            e[1] = sin(ph);
        }
    }

    const int64_t block = 1 << 16;
    int64_t n_blocks = (n_rows + block - 1) / block;
    double *part = (double *)calloc((size_t)(n_blocks > 0 ? n_blocks : 1) * 2 * (size_t)n_pix,
                                    sizeof(double));

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bi = 0; bi < n_blocks; ++bi) {
        double gx[64], gy[64];
        double *acc = part + (size_t)bi * 2 * (size_t)n_pix;
        int64_t r1 = (bi + 1) * block < n_rows ? (bi + 1) * block : n_rows;
        for (int64_t r = bi * block; r < r1; ++r) {
            for (int c = 0; c < n_chan; ++c) {
                if (chan >= 0 && c != chan) continue;
                int64_t rc = r * n_chan + c;
                double wt = weights ? weights[rc] : 1.0;
                uint8_t fl = flags ? flags[rc] : 0;
                if (!is_valid0(uvw + 3 * r, chan_scale[c], vis + 2 * rc, wt, fl, scale, n, h))
                    continue;
                double u = uvw[3 * r + 0] * chan_scale[c];
                double v = uvw[3 * r + 1] * chan_scale[c];
                double w = uvw[3 * r + 2] * chan_scale[c];
                if (!(w >= w_min && w <= w_max)) continue;
                int k = plane_of(w, w_min, dw, n_w);
                double x, y;
                int64_t i0, j0;
                position(u, v, scale, n, &x, &y);
                fits(x, n, h, &i0);
                fits(y, n, h, &j0);
                for (int a = -h; a <= h; ++a)
                    gx[a + h] = oracle_kernel_value(kernel, kpar, support, (double)(i0 + a) - x);
                for (int b = -h; b <= h; ++b)
                    gy[b + h] = oracle_kernel_value(kernel, kpar, support, (double)(j0 + b) - y);
                double wv_re = wt * vis[2 * rc + 0];
                double wv_im = wt * vis[2 * rc + 1];
                for (int ip = 0; ip < n_pix; ++ip) {
                    /* (i0+a-N/2)(p-N/2) mod N, stepped exactly in a */
                    int64_t pp = ((int64_t)(pix_p[ip] - n / 2) % n + n) % n;
                    int64_t qq = ((int64_t)(pix_q[ip] - n / 2) % n + n) % n;
                    double kx_re = 0.0, kx_im = 0.0, ky_re = 0.0, ky_im = 0.0;
                    int64_t t = (((i0 - h - n / 2) * pp) % n + n) % n;
                    for (int a = -h; a <= h; ++a) {
                        kx_re += gx[a + h] * ct[t];
                        kx_im += gx[a + h] * st[t];
                        t += pp;
                        if (t >= n) t -= n;
                    }
                    t = (((j0 - h - n / 2) * qq) % n + n) % n;
                    for (int b = -h; b <= h; ++b) {
                        ky_re += gy[b + h] * ct[t];
                        ky_im += gy[b + h] * st[t];
                        t += qq;
                        if (t >= n) t -= n;
                    }
                    const double *e = wk + 2 * ((size_t)ip * n_w + k);
                    double k_re = kx_re * ky_re - kx_im * ky_im;
                    double k_im = kx_re * ky_im + kx_im * ky_re;
                    double z_re = k_re * e[0] - k_im * e[1];
                    double z_im = k_re * e[1] + k_im * e[0];
                    acc[2 * ip + 0] += wv_re * z_re - wv_im * z_im;
                    acc[2 * ip + 1] += wv_re * z_im + wv_im * z_re;
                }
            }
        }
    }
    for (int ip = 0; ip < n_pix; ++ip) { out[2 * ip] = 0.0; out[2 * ip + 1] = 0.0; }
    for (int64_t bi = 0; bi < n_blocks; ++bi)
        for (int ip = 0; ip < n_pix; ++ip) {
            out[2 * ip + 0] += part[(size_t)bi * 2 * n_pix + 2 * ip + 0];
            out[2 * ip + 1] += part[(size_t)bi * 2 * n_pix + 2 * ip + 1];
        }
    free(part);
    free(wk);
    free(st);
    free(ct);
    return 0;
}
