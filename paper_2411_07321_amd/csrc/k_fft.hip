// 2D inverse transform of every w-plane and the w-correction (Eq. 2).
//
// The centred transform F[q][p] = sum g[j][i] e^{+2 pi i ((i-N/2)(p-N/2) +
// (j-N/2)(q-N/2))/N} equals (-1)^(p+q) * IDFT2((-1)^(i+j) g) exactly when N is
// a multiple of 4 (every supported N is), so both passes are plain
// unnormalised inverse DFTs with sign flips folded into their loads / outputs.
//
// Each 1D transform is a Stockham autosort FFT: every thread keeps E = 16
// points in registers, runs radix-16 (the first stage may use radix 2, 4 or 8)
// butterflies there and exchanges through LDS between stages.
//
// Layout between the passes ("blocked"): pass 1 transforms B consecutive rows
// of a plane X[a][b] along b and writes them back into the same region as
// Y[a/B][b'][a%B], so pass 2, which transforms along a for B' consecutive
// b', reads runs of B*B' contiguous elements (128 bytes for complex64) and
// every HBM access of both passes is a full 128-byte run.
//
// In the imaging pipeline the gridder stores each plane transposed (G[i][j],
// u index slow), pass 1 transforms along v (j -> q) and pass 2 along u
// (i -> p) while it walks the planes of a strip of image rows q, multiplies by
// the phase screen e^{2 pi i w_k (n-1)} and accumulates Re in FP64 registers;
// the strip of the image is written once, with the post factors applied.
//
// The imaging path passes the tile occupancy of the stack: pass 1 then reads
// only the tiles the gridder wrote and skips rows of empty tile-rows altogether,
// and pass 2 skips those rows and planes without records.
#include "wsg_internal.h"

#include <type_traits>

namespace wsg {

namespace {

constexpr int E = 16;

template <typename T> struct BlockRows;
template <> struct BlockRows<float> { static constexpr int value = 4; };
template <> struct BlockRows<double> { static constexpr int value = 2; };

// Rows of N >= kBigN points: a workgroup holds at most 1024 threads (one or two
// rows), and the LDS exchange between stages moves one component at a time (the
// real parts, then the imaginary ones) through one buffer, as a whole row of
// complex points would not fit in LDS.
constexpr int kBigN = 8192;

// Extra words at the end of each LDS row.  A wave holds points of several rows (the
// lowest lane bits pick the row), and rows whose pitch is a multiple of the bank count
// would put the same point of every row on one bank; these offsets, chosen by counting
// the conflicts of every exchange of fft_line for 32 and 64 four-byte banks, spread
// the rows over the banks (pass 1: 4x fewer conflicted cycles at N = 4096).
template <typename T, int N, bool PASS2>
__host__ __device__ constexpr int row_pad() {
    if (N >= kBigN) return 0;
    if constexpr (sizeof(T) == 4) {
        if (!PASS2) return N == 64 ? 1 : N == 4096 ? 8 : N >= 512 ? 16 : 0;
        return N == 64 ? 1 : N == 128 || N == 256 ? 4 : N == 512 ? 8 : N >= 1024 ? 16 : 0;
    } else {
        if (!PASS2) return N == 64 ? 1 : N == 4096 ? 8 : N >= 512 ? 16 : 0;
        return N == 64 || N == 128 || N == 256 ? 2 : N == 512 ? 4 : N == 1024 ? 5 : N == 2048 ? 16 : 0;
    }
}

// transforms per workgroup: at least B, enough threads for 4 waves when N is small,
// at most 1024 threads
// B, the rows of a block of the intermediate layout, is BlockRows unless fewer rows
// fit in one workgroup: pass 1 rewrites a block in place, so all of its rows must be
// read by one workgroup before any of them is overwritten.
template <typename T, int N>
struct Shape {
    static constexpr int P = N / E;                  // threads per transform
    static constexpr int want = 256 / P;
    static constexpr int B0 = BlockRows<T>::value;
    static constexpr int NTR0 = want > B0 ? want : B0;
    static constexpr int NTR1 = NTR0 > N ? N : NTR0;
    static constexpr int NTR = NTR1 * P > 1024 ? 1024 / P : NTR1;  // transforms per workgroup
    static constexpr int B = B0 < NTR ? B0 : NTR;
    static constexpr int THREADS = NTR * P;
    static constexpr int NPAD = N + N / 16 + row_pad<T, N, false>();   // LDS row length
    static constexpr bool SPLIT = N >= kBigN;         // exchange one component at a time
    static constexpr int LDS_ROWS = SPLIT ? NTR : 2 * NTR;
};

// pass 2: fewer transforms per workgroup where the FP64 plane sums would not fit in
// registers next to the points (at most 512 threads for complex64, 256 for complex128,
// and one row of any N)
template <typename T, int N>
struct Shape2 {
    static constexpr int B = Shape<T, N>::B;
    static constexpr int P = N / E;
    static constexpr int cap = (sizeof(T) == 4 ? 512 : 256) / P;
    static constexpr int NTR = Shape<T, N>::NTR < cap ? Shape<T, N>::NTR : (cap > 0 ? cap : 1);
    static constexpr int THREADS = NTR * P;
    static constexpr int NPAD = N + N / 16 + row_pad<T, N, true>();
    static constexpr bool SPLIT = N >= kBigN;
    static constexpr int LDS_ROWS = SPLIT ? NTR : 2 * NTR;
};

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// first-stage radix: N = R0 * E^k
template <int N>
struct FirstRadix {
    static constexpr int L = ilog2(N);
    static constexpr int r = (L % 4 == 0) ? 16 : (1 << (L % 4));
    static constexpr int stages = (L - ilog2(r)) / 4 + 1;
};

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

// e^{+2 pi i idx / 16} times b, specialised for the trivial angles
template <typename T>
__device__ __forceinline__ C2<T> rot16(C2<T> b, int idx) {
    const T r2 = (T)0.70710678118654752440084436210485;
    const T c1 = (T)0.92387953251128675612818318939679;   // cos(pi/8)
    const T s1 = (T)0.38268343236508977172845998403040;   // sin(pi/8)
    switch (idx & 15) {
    case 0: return b;
    case 4: return C2<T>{-b.y, b.x};
    case 8: return C2<T>{-b.x, -b.y};
    case 12: return C2<T>{b.y, -b.x};
    case 2: return C2<T>{(b.x - b.y) * r2, (b.x + b.y) * r2};
    case 6: return C2<T>{(-b.x - b.y) * r2, (b.x - b.y) * r2};
    case 10: return C2<T>{(b.y - b.x) * r2, (-b.x - b.y) * r2};
    case 14: return C2<T>{(b.x + b.y) * r2, (b.y - b.x) * r2};
    case 1: return cmul(b, C2<T>{c1, s1});
    case 3: return cmul(b, C2<T>{s1, c1});
    case 5: return cmul(b, C2<T>{-s1, c1});
    case 7: return cmul(b, C2<T>{-c1, s1});
    case 9: return cmul(b, C2<T>{-c1, -s1});
    case 11: return cmul(b, C2<T>{-s1, -c1});
    case 13: return cmul(b, C2<T>{s1, -c1});
    default: return cmul(b, C2<T>{c1, -s1});   // 15
    }
}

__host__ __device__ constexpr int bitrev(int i, int bits) {
    int r = 0;
    for (int k = 0; k < bits; ++k) r |= ((i >> k) & 1) << (bits - 1 - k);
    return r;
}

// In-register inverse DFT of R points v[base + stride*s], s = 0..R-1 (R <= 16),
// natural order in and out.
template <typename T, int R, int STRIDE>
__device__ __forceinline__ void dft_reg(C2<T> *v, int base) {
    constexpr int LG = ilog2(R);
    C2<T> x[R];
#pragma unroll
    for (int s = 0; s < R; ++s) x[bitrev(s, LG)] = v[base + STRIDE * s];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len / 2;
#pragma unroll
        for (int i0 = 0; i0 < R; i0 += len) {
#pragma unroll
            for (int k = 0; k < half; ++k) {
                C2<T> a = x[i0 + k];
                C2<T> b = rot16(x[i0 + k + half], k * (16 / len));
                x[i0 + k] = cadd(a, b);
                x[i0 + k + half] = csub(a, b);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < R; ++s) v[base + STRIDE * s] = x[s];
}

// One length-N inverse transform, cooperatively by the P threads of a row.
// In:  v[m] = X[t + m*P] (m < E).  Out: v[s] = Y[t + s*P].
// lre/lim: this transform's LDS rows (NPAD elements each).  Every thread of
// the workgroup must call this together (it contains barriers when N > E).
// SPLIT: lre and lim are one buffer; the components pass through it one after the other.
template <typename T, int N, bool SPLIT = false>
__device__ __forceinline__ void fft_line(C2<T> *v, T *lre, T *lim, int t, const C2<T> *__restrict__ tw) {
    constexpr int P = N / E;
    constexpr int R0 = FirstRadix<N>::r;
    constexpr int NST = FirstRadix<N>::stages;
    // ---- stage 1 (Ns = 1): E/R0 butterflies of radix R0 over m = u + s*(E/R0)
#pragma unroll
    for (int u = 0; u < E / R0; ++u) dft_reg<T, R0, E / R0>(v, u);
    if constexpr (NST == 1) return;
    // butterfly j = t + u*P writes Y[j*R0 + s]
    int ns = R0;
#pragma unroll
    for (int st = 1; st < NST; ++st) {
#pragma unroll
        for (int comp = 0; comp < (SPLIT ? 2 : 1); ++comp) {
        // component mask: both at once, or the real (comp 0) then the imaginary parts
        const bool wr = !SPLIT || comp == 0, wi = !SPLIT || comp == 1;
        __syncthreads();
        if (st == 1) {
#pragma unroll
            for (int u = 0; u < E / R0; ++u) {
                int j = t + u * P;
#pragma unroll
                for (int s = 0; s < R0; ++s) {
                    int idx = lds_pad(j * R0 + s);
                    if (wr) lre[idx] = v[u + s * (E / R0)].x;
                    if (wi) lim[idx] = v[u + s * (E / R0)].y;
                }
            }
        } else {
            // previous radix-E stage with span ns/E: j = t
            int nsp = ns / E;
            int jm = t % nsp;
            int o = (t / nsp) * nsp * E + jm;
#pragma unroll
            for (int s = 0; s < E; ++s) {
                int idx = lds_pad(o + s * nsp);
                if (wr) lre[idx] = v[s].x;
                if (wi) lim[idx] = v[s].y;
            }
        }
        __syncthreads();
        if constexpr (SPLIT) {
            // the first round replaces the real parts by their exchanged values; the
            // imaginary parts stay in their registers, in the old order, for the second
#pragma unroll
            for (int s = 0; s < E; ++s) {
                int idx = lds_pad(t + s * P);
                if (comp == 0) v[s].x = lre[idx];
                else v[s].y = lim[idx];
            }
        } else {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                int idx = lds_pad(t + s * P);
                v[s] = C2<T>{lre[idx], lim[idx]};
            }
        }
        }
        // twiddles e^{+2 pi i (t mod ns) s / (ns E)} = W_N[(t mod ns) * s * N/(ns E)]
        int step = (t % ns) * (N / (ns * E));
#pragma unroll
        for (int s = 1; s < E; ++s) v[s] = cmul(v[s], tw[step * s]);
        dft_reg<T, E, 1>(v, 0);
        ns *= E;
    }
}

// Planes whose bytes fit 32-bit offsets: their point loads take a 32-bit byte offset
// from the plane's (workgroup-uniform) base instead of a 64-bit address per point.
template <typename T, int N>
struct PlaneOff {
    static constexpr bool ok = (uint64_t)N * N * sizeof(C2<T>) <= (1ull << 32);
};

// ---------------------------------------------------------------- pass 1
template <typename T, int N>
__global__ __launch_bounds__((Shape<T, N>::THREADS)) void k_pass1(C2<T> *__restrict__ planes,
                                                                 const C2<T> *__restrict__ tw,
                                                                 Occupancy occ) {
    using SH = Shape<T, N>;
    constexpr int B = SH::B, P = SH::P, NTR = SH::NTR;
    __shared__ __align__(16) T lds[SH::LDS_ROWS * SH::NPAD];
    const int tid = threadIdx.x;
    const int r_lo = tid % B;
    const int t = (tid / B) % P;
    const int r_hi = tid / (B * P);
    const int r = r_hi * B + r_lo;
    const int grp = blockIdx.x;
    const int a = grp * NTR + r;
    const int pi = blockIdx.y;
    C2<T> *X = planes + (size_t)pi * N * N;
    // sparse stack: a row of an empty tile-row is neither read nor written (pass 2
    // skips it too), and an empty tile of a live row reads as zero
    bool row_live = true;
    uint32_t on = 0xffffu;
    if (occ.rows) {
        const int NT = N >> occ.logT;
        const int txr = a >> occ.logT;
        const uint32_t lm = occ.live1[((size_t)pi * NT + txr) * P + t];
        const uint64_t *rows = occ.rows + (size_t)pi * occ.nw;
        const int a0 = grp * NTR;
        bool any = false;
        for (int tx = a0 >> occ.logT; tx <= (a0 + NTR - 1) >> occ.logT; ++tx)
            any = any || ((rows[tx >> 6] >> (tx & 63)) & 1ull);
        if (!any) return;   // the same for every thread of the workgroup
        row_live = (lm >> 16) & 1u;
        on = lm & 0xffffu;
    }
    C2<T> v[E];
    if constexpr (PlaneOff<T, N>::ok) {
        // 32-bit byte offsets from the plane; a dead point reads the thread's first
        // point (a cached line) and is zeroed, so no load is branched around
        const char *base = (const char *)X;
        const uint32_t off0 = (uint32_t)(a * N + t) * (uint32_t)sizeof(C2<T>);
        constexpr uint32_t step = (uint32_t)P * (uint32_t)sizeof(C2<T>);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const bool live = (on >> m) & 1u;
            C2<T> z = *(const C2<T> *)(base + (live ? off0 + (uint32_t)m * step : off0));
            z = live ? z : C2<T>{T(0), T(0)};
            if ((a + t + m * P) & 1) z = C2<T>{-z.x, -z.y};
            v[m] = z;
        }
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            int b = t + m * P;
            C2<T> z = C2<T>{T(0), T(0)};
            if ((on >> m) & 1u) z = X[(size_t)a * N + b];
            if ((a + b) & 1) z = C2<T>{-z.x, -z.y};
            v[m] = z;
        }
    }
    T *lre = lds + (size_t)r * SH::NPAD;
    T *lim = SH::SPLIT ? lre : lds + (size_t)(NTR + r) * SH::NPAD;
    fft_line<T, N, SH::SPLIT>(v, lre, lim, t, tw);
    __syncthreads();   // every load of this region is done before it is overwritten
    C2<T> *Y = X + (size_t)(a / B) * B * N;
    if (row_live) {
#pragma unroll
        for (int s = 0; s < E; ++s) Y[(size_t)(t + s * P) * B + r_lo] = v[s];
    }
}

// ---------------------------------------------------------------- pass 2
// Workgroups are dealt to the 8 XCDs round robin.  Strip s of pass 2 goes to the
// workgroup that makes consecutive strips run side by side on one XCD, so two
// strips whose reads share 128-byte lines (B x NTR elements of 8 bytes = 64 bytes
// each) meet in that XCD's L2 and every line is fetched from HBM once.
__device__ __forceinline__ int xcd_strip(int bid, int n_strips) {
    constexpr int kXcd = 8;
    if (n_strips % kXcd) return bid;
    return (bid % kXcd) * (n_strips / kXcd) + bid / kXcd;
}

// thread -> (t_lo, r, t_hi): reads of 16 consecutive lanes form one 128-byte run
template <typename T, int N>
struct P2Index {
    using SH = Shape2<T, N>;
    int t, r;
    __device__ __forceinline__ P2Index(int tid) {
        constexpr int TB = SH::B < SH::P ? SH::B : SH::P;
        constexpr int NTR = SH::NTR;
        int t_lo = tid % TB;
        r = (tid / TB) % NTR;
        int t_hi = tid / (TB * NTR);
        t = t_hi * TB + t_lo;
    }
};

template <typename T, int N>
__device__ __forceinline__ void load_blocked(C2<T> *v, const C2<T> *__restrict__ Y, int t, int bcol) {
    constexpr int B = Shape<T, N>::B, P = N / E;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        int a = t + m * P;
        v[m] = Y[((size_t)(a / B) * N + bcol) * B + (a % B)];
    }
}

// the same for the points m whose bit is set in `live`; the others read as zero.
// Their loads go to `dummy` (one cached line) instead of being branched around,
// so that all E loads are issued together.
template <typename T, int N>
__device__ __forceinline__ void load_blocked_live(C2<T> *v, const C2<T> *__restrict__ Y, int t,
                                                  int bcol, uint32_t live,
                                                  const C2<T> *__restrict__ dummy) {
    constexpr int B = Shape<T, N>::B, P = N / E;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        int a = t + m * P;
        const bool on = (live >> m) & 1u;
        const C2<T> *src = on ? Y + ((size_t)(a / B) * N + bcol) * B + (a % B) : dummy;
        const C2<T> z = *src;
        v[m] = on ? z : C2<T>{T(0), T(0)};
    }
}

template <typename T, int N>
__global__ __launch_bounds__((Shape2<T, N>::THREADS)) void k_pass2_store(const C2<T> *__restrict__ in,
                                                                        C2<T> *__restrict__ out,
                                                                        const C2<T> *__restrict__ tw) {
    using SH = Shape2<T, N>;
    constexpr int P = SH::P, NTR = SH::NTR;
    __shared__ __align__(16) T lds[SH::LDS_ROWS * SH::NPAD];
    P2Index<T, N> ix(threadIdx.x);
    const int strip = xcd_strip(blockIdx.x, N / NTR);
    const int bcol = strip * NTR + ix.r;
    const C2<T> *Y = in + (size_t)blockIdx.y * N * N;
    C2<T> v[E];
    load_blocked<T, N>(v, Y, ix.t, bcol);
    T *lre = lds + (size_t)ix.r * SH::NPAD;
    fft_line<T, N, SH::SPLIT>(v, lre, SH::SPLIT ? lre : lds + (size_t)(NTR + ix.r) * SH::NPAD, ix.t, tw);
    if constexpr (SH::SPLIT) {
        // one row per workgroup: consecutive threads hold consecutive points, so the
        // row-major writes are contiguous as they are
        C2<T> *Z = out + (size_t)blockIdx.y * N * N + (size_t)bcol * N;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            int ap = ix.t + s * P;
            C2<T> z = v[s];
            if ((ap + bcol) & 1) z = C2<T>{-z.x, -z.y};
            Z[ap] = z;
        }
        return;
    }
    // stage through LDS so that the row-major writes are contiguous
    __syncthreads();
    C2<T> *st = (C2<T> *)lds;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        int ap = ix.t + s * P;
        C2<T> z = v[s];
        if ((ap + bcol) & 1) z = C2<T>{-z.x, -z.y};
        st[ix.r * N + ap] = z;
    }
    __syncthreads();
    C2<T> *Z = out + (size_t)blockIdx.y * N * N + (size_t)strip * NTR * N;
    for (int i = threadIdx.x; i < NTR * N; i += blockDim.x) Z[i] = st[i];
}

// phase screen of one pixel for plane w: e^{2 pi i w (n-1)}
//   MODE 0 (FP64 mesh):      argument and sin/cos in FP64
//   MODE 1 (FP32 mesh):      argument w (n-1) in turns formed in FP64 and reduced
//                            exactly to [-1/2, 1/2]; sin/cos of the reduced angle by
//                            the hardware's FP32 functions (error <= 1.3e-7)
//   MODE 2 (FP32 phase):     argument and sin/cos in FP32 (the precision study)
template <int MODE>
struct Phase;

// sin and cos of 2 pi t (t in turns) in FP64.  The reduction is exact: r = t - rint(t)
// lies in [-1/2, 1/2], and with q = rint(4 r) the octant remainder f = r - q/4 lies in
// [-1/8, 1/8] (both differences are exact in binary floating point).  With
// x = 2 pi f in [-pi/4, pi/4], the Taylor series of sin to x^15 and of cos to x^16
// leave remainders below |x|^17/17! < 5e-17 and |x|^18/18! < 3e-18; the quarter turns
// q pi/2 are then applied by exchanging and negating the two.
__device__ __forceinline__ void sincos_turns(double t, double &s, double &c) {
    const double r = t - rint(t);
    const double q = rint(4.0 * r);
    const double f = r - 0.25 * q;
    const double x = f * 6.283185307179586476925286766559;
    const double x2 = x * x;
    // 1/n! for n = 3, 5, ..., 15 and n = 2, 4, ..., 16, alternating in sign
    double ps = -7.6471637318198164759e-13;                 // -1/15!
    ps = fma(ps, x2, 1.6059043836821614599e-10);             //  1/13!
    ps = fma(ps, x2, -2.5052108385441718775e-08);            // -1/11!
    ps = fma(ps, x2, 2.7557319223985890653e-06);             //  1/9!
    ps = fma(ps, x2, -1.9841269841269841270e-04);            // -1/7!
    ps = fma(ps, x2, 8.3333333333333333333e-03);             //  1/5!
    ps = fma(ps, x2, -1.6666666666666666667e-01);            // -1/3!
    const double sx = fma(ps * x2, x, x);
    double pc = 4.7794773323873852974e-14;                  //  1/16!
    pc = fma(pc, x2, -1.1470745597729724714e-11);            // -1/14!
    pc = fma(pc, x2, 2.0876756987868098979e-09);             //  1/12!
    pc = fma(pc, x2, -2.7557319223985890653e-07);            // -1/10!
    pc = fma(pc, x2, 2.4801587301587301587e-05);             //  1/8!
    pc = fma(pc, x2, -1.3888888888888888889e-03);            // -1/6!
    pc = fma(pc, x2, 4.1666666666666666667e-02);             //  1/4!
    pc = fma(pc, x2, -0.5);                                  // -1/2!
    const double cx = fma(pc, x2, 1.0);
    // 2 pi r = x + q pi/2, q in {-2, -1, 0, 1, 2}
    //   q = 0: (sin x, cos x); 1: (cos x, -sin x); +-2: (-sin x, -cos x); -1: (-cos x, sin x)
    const int qi = (int)q;
    const bool odd = qi & 1;
    const double so = odd ? cx : sx, co = odd ? sx : cx;
    s = (qi == 0 || qi == 1) ? so : -so;
    c = (qi == 0 || qi == -1) ? co : -co;
}

template <>
struct Phase<0> {
    using R = double;
    static __device__ __forceinline__ R nm1(double l, double m, int /*naive*/, bool &inside) {
        double eta = l * l + m * m;
        inside = eta < 1.0;
        if (!inside) return 0.0;
        return -eta / (1.0 + sqrt(1.0 - eta));
    }
    static __device__ __forceinline__ void screen(R nm1v, double w, double &c, double &s) {
        sincos_turns(w * nm1v, s, c);
    }
};

template <>
struct Phase<1> {
    using R = double;
    // -eta/(1 + sqrt(1 - eta)) to ~1e-14 relative: FP32 seeds for the square root
    // and the reciprocal, each refined by one Newton step in FP64
    static __device__ __forceinline__ R nm1(double l, double m, int /*naive*/, bool &inside) {
        double eta = l * l + m * m;
        inside = eta < 1.0;
        if (!inside) return 0.0;
        double x = 1.0 - eta;
        float yf = sqrtf((float)x);
        float rf = 1.0f / yf;
        double y = (double)yf;
        y = y + (x - y * y) * (0.5 * (double)rf);
        double d = 1.0 + y;
        double rd = (double)(1.0f / (float)d);
        double q = -eta * rd;
        q = q + (-eta - q * d) * rd;
        return q;
    }
    static __device__ __forceinline__ void screen(R nm1v, double w, float &c, float &s) {
        double t = w * nm1v;             // turns
        double r = t - rint(t);          // exact: |r| <= 1/2
        // hardware sine and cosine of an argument in turns: max error 1.3e-7 over
        // [-1/2, 1/2] (measured against FP64), about twice the FP32 mesh rounding
        s = __builtin_amdgcn_sinf((float)r);
        c = __builtin_amdgcn_cosf((float)r);
    }
};

template <>
struct Phase<2> {
    using R = float;
    static __device__ __forceinline__ R nm1(double l, double m, int naive, bool &inside) {
        float lf = (float)l, mf = (float)m;
        float eta = lf * lf + mf * mf;
        inside = eta < 1.0f;
        if (!inside) return 0.0f;
        if (naive) return sqrtf(1.0f - eta) - 1.0f;
        return -eta / (1.0f + sqrtf(1.0f - eta));
    }
    static __device__ __forceinline__ void screen(R nm1v, double w, float &c, float &s) {
        sincospif(2.0f * ((float)w * nm1v), &s, &c);
    }
};

template <typename T, bool PH32>
struct PhaseMode {
    static constexpr int value = PH32 ? 2 : (sizeof(T) == 8 ? 0 : 1);
};

// acc += Re(z * (c + i s)), in the arithmetic of the screen
template <typename T>
__device__ __forceinline__ void acc_re(double &acc, C2<T> z, double c, double s) {
    acc += (double)z.x * c - (double)z.y * s;
}
template <typename T>
__device__ __forceinline__ void acc_re(double &acc, C2<T> z, float c, float s) {
    acc += (double)(z.x * c - z.y * s);
}

// C_w(nu) of the kernel in w by its quadrature table; FP64 cosines for the FP64
// mode, else the hardware's of the exactly reduced argument in turns
template <int PM>
__device__ __forceinline__ double w_transform(const double *__restrict__ cw, int n_cw, double nu) {
    double c = 0.0;
    for (int j = 0; j < n_cw; ++j) {
        const double t = nu * cw[2 * j];
        if constexpr (PM == 0) {
            c += cw[2 * j + 1] * cospi(2.0 * t);
        } else {
            const double r = t - rint(t);
            c += cw[2 * j + 1] * (double)__builtin_amdgcn_cosf((float)r);
        }
    }
    return c;
}

// Layout choices of pass 2 with the w-correction: n - 1 of the workgroup's pixels is
// kept in an LDS table where it fits next to the exchange buffer, else recomputed per
// plane; the next plane's points are loaded during the current plane's transform
// (software pipeline) where the registers allow it (at most 512 threads, N < kBigN).
template <typename T, int N, int PM>
struct Wc2 {
    using SH = Shape2<T, N>;
    using PR = typename Phase<PM>::R;
    static constexpr size_t LDS_BYTES = (size_t)SH::LDS_ROWS * SH::NPAD * sizeof(T);
    static constexpr bool NM1_TABLE = LDS_BYTES + (size_t)SH::NTR * N * sizeof(PR) <= 150 * 1024;
    static constexpr int NM1_LEN = NM1_TABLE ? SH::NTR * N : 1;
    static constexpr bool PIPE = SH::THREADS <= 512 && N < kBigN;
};

template <typename T, int N, bool PH32>
__global__ __launch_bounds__((Shape2<T, N>::THREADS)) void k_pass2_wcorr(const C2<T> *__restrict__ stack,
                                                                        const C2<T> *__restrict__ tw,
                                                                        WcorrArgs a,
                                                                        double *__restrict__ image) {
    using SH = Shape2<T, N>;
    constexpr int PM = PhaseMode<T, PH32>::value;
    using PR = typename Phase<PM>::R;
    using WC = Wc2<T, N, PM>;
    constexpr int P = SH::P, NTR = SH::NTR;
    __shared__ __align__(16) T lds[SH::LDS_ROWS * SH::NPAD];
    // n - 1 of this workgroup's pixels, computed once and read for every plane
    __shared__ PR s_nm1[WC::NM1_LEN];
    P2Index<T, N> ix(threadIdx.x);
    const int img = blockIdx.y;
    const int strip = xcd_strip(blockIdx.x, N / NTR);
    const int q = strip * NTR + ix.r;                 // image row handled by this thread
    const ImgState &st = a.st[img];
    const double m = (double)(q - N / 2) * a.cell;
    auto nm1_of = [&](int s) -> PR {
        if constexpr (WC::NM1_TABLE) {
            return s_nm1[ix.r * N + ix.t + s * P];
        } else {
            bool in;
            return Phase<PM>::nm1((double)(ix.t + s * P - N / 2) * a.cell, m, a.naive_nm1, in);
        }
    };
    if constexpr (WC::NM1_TABLE) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
            bool in;
            const double l = (double)(ix.t + s * P - N / 2) * a.cell;
            s_nm1[ix.r * N + ix.t + s * P] = Phase<PM>::nm1(l, m, a.naive_nm1, in);
        }
    }
    double acc[E];
#pragma unroll
    for (int s = 0; s < E; ++s) acc[s] = 0.0;
    const double w0 = st.w0, dw = st.dw;
    // points of rows that pass 1 wrote (all of them for a dense stack; none of a plane
    // without records, whose transform then only adds zeros), per plane
    auto live_of = [&](int kl) -> uint32_t {
        return a.occ.live2 ? (uint32_t)a.occ.live2[((size_t)img * a.n_pl + kl) * P + ix.t] : 0xffffu;
    };
    T *lre = lds + (size_t)ix.r * SH::NPAD;
    T *lim = SH::SPLIT ? lre : lds + (size_t)(NTR + ix.r) * SH::NPAD;
    // software pipeline: the points of plane kl + 1 are loaded while plane kl is
    // transformed (the loads count on the vector-memory counter, the exchanges of the
    // transform on the LDS counter, so neither waits for the other); the mask of plane
    // kl + 2 is fetched one step earlier still
    C2<T> vn[WC::PIPE ? E : 1];
    uint32_t live_next = a.n_pl > 1 ? live_of(1) : 0u;
    if constexpr (WC::PIPE)
        if (a.n_pl > 0) load_blocked_live<T, N>(vn, stack + (size_t)img * a.n_pl * N * N, ix.t, q, live_of(0), tw);
    for (int kl = 0; kl < a.n_pl; ++kl) {
        const int k = a.plane_lo + kl;
        const double wk = (dw == 0.0) ? w0 : w0 + ((double)k + 0.5) * dw;
        const size_t pi = (size_t)img * a.n_pl + kl;
        C2<T> v[E];
        if constexpr (WC::PIPE) {
#pragma unroll
            for (int mm = 0; mm < E; ++mm) v[mm] = vn[mm];
            if (kl + 1 < a.n_pl) {
                const uint32_t live = live_next;
                if (kl + 2 < a.n_pl) live_next = live_of(kl + 2);
                load_blocked_live<T, N>(vn, stack + (pi + 1) * N * N, ix.t, q, live, tw);
            }
        } else {
            load_blocked_live<T, N>(v, stack + pi * N * N, ix.t, q, live_of(kl), tw);
        }
        fft_line<T, N, SH::SPLIT>(v, lre, lim, ix.t, tw);
        // (n - 1 comes from LDS or is recomputed: holding it for all E pixels in
        // registers would not fit next to the points and the FP64 sums)
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const PR nm1 = nm1_of(s);
            typename std::conditional<PM == 0, double, float>::type c, sn;
            Phase<PM>::screen(nm1, wk, c, sn);
            acc_re(acc[s], v[s], c, sn);
        }
    }
    // post factors and the output sign (-1)^(p+q); stage through LDS for contiguous
    // row writes (with one row per workgroup, consecutive threads already hold
    // consecutive pixels)
    const double inv_row = st.inv_norm * (a.inv_c ? a.inv_c[q] : 1.0);
    constexpr bool STAGE = WC::LDS_BYTES >= (size_t)NTR * N * sizeof(double) && NTR > 1;
    if constexpr (STAGE) __syncthreads();
    double *stg = (double *)lds;
    double *D = image + (size_t)img * N * N + (size_t)strip * NTR * N;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        int p = ix.t + s * P;
        const double l = (double)(p - N / 2) * a.cell;
        const bool inside = l * l + m * m < 1.0;
        double d = inside ? acc[s] * inv_row * (a.inv_c ? a.inv_c[p] : 1.0) : 0.0;
        if (a.cw && inside && dw > 0.0) d /= w_transform<PM>(a.cw, a.n_cw, dw * (double)nm1_of(s));
        if ((p + q) & 1) d = -d;
        if constexpr (STAGE) stg[ix.r * N + p] = d;
        else D[(size_t)ix.r * N + p] = a.accumulate ? D[(size_t)ix.r * N + p] + d : d;
    }
    if constexpr (STAGE) {
        __syncthreads();
        for (int i = threadIdx.x; i < NTR * N; i += blockDim.x) D[i] = a.accumulate ? D[i] + stg[i] : stg[i];
    }
}

// ---------------------------------------------------------------- w-correction alone
template <typename T, bool PH32>
__global__ __launch_bounds__(256) void k_wcorrect(const C2<T> *__restrict__ F, WcorrArgs a,
                                                  double *__restrict__ image) {
    constexpr int PM = PhaseMode<T, PH32>::value;
    using PR = typename Phase<PM>::R;
    const int N = a.N;
    const size_t n2 = (size_t)N * N;
    size_t pix = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= n2) return;
    const int q = (int)(pix / N), p = (int)(pix % N);
    const ImgState &st = a.st[0];
    bool inside;
    PR nm1 = Phase<PM>::nm1((double)(p - N / 2) * a.cell, (double)(q - N / 2) * a.cell,
                            a.naive_nm1, inside);
    double acc = 0.0;
    for (int kl = 0; kl < a.n_pl; ++kl) {
        const int k = a.plane_lo + kl;
        const double wk = (st.dw == 0.0) ? st.w0 : st.w0 + ((double)k + 0.5) * st.dw;
        C2<T> z = F[(size_t)kl * n2 + pix];
        typename std::conditional<PM == 0, double, float>::type c, s;
        Phase<PM>::screen(nm1, wk, c, s);
        acc_re(acc, z, c, s);
    }
    double d = inside ? acc * st.inv_norm * (a.inv_c ? a.inv_c[p] * a.inv_c[q] : 1.0) : 0.0;
    if (a.cw && inside && st.dw > 0.0) d /= w_transform<PM>(a.cw, a.n_cw, st.dw * (double)nm1);
    image[pix] = d;
}

// ---------------------------------------------------------------- transpose
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const C2<T> *__restrict__ in, C2<T> *__restrict__ out, int N) {
    __shared__ C2<T> tile[32][33];
    const size_t plane = (size_t)blockIdx.z * N * N;
    int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += 8)
        if (y0 + k < N && x0 + (int)threadIdx.x < N)
            tile[k][threadIdx.x] = in[plane + (size_t)(y0 + k) * N + x0 + threadIdx.x];
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8)
        if (x0 + k < N && y0 + (int)threadIdx.x < N)
            out[plane + (size_t)(x0 + k) * N + y0 + threadIdx.x] = tile[threadIdx.x][k];
}

template <typename T, int N>
void pass1_n(void *planes, int64_t n_planes, const void *tw, const Occupancy &occ, hipStream_t s) {
    using SH = Shape<T, N>;
    dim3 grid(N / SH::NTR, (unsigned)n_planes);
    k_pass1<T, N><<<grid, SH::THREADS, 0, s>>>((C2<T> *)planes, (const C2<T> *)tw, occ);
}

template <typename T, int N>
void pass2_store_n(const void *in, void *out, int64_t n_planes, const void *tw, hipStream_t s) {
    using SH = Shape2<T, N>;
    dim3 grid(N / SH::NTR, (unsigned)n_planes);
    k_pass2_store<T, N><<<grid, SH::THREADS, 0, s>>>((const C2<T> *)in, (C2<T> *)out, (const C2<T> *)tw);
}

template <typename T, int N>
void pass2_wcorr_n(const WcorrArgs &a, const void *stack, const void *tw, double *image, hipStream_t s) {
    using SH = Shape2<T, N>;
    dim3 grid(N / SH::NTR, (unsigned)a.n_img);
    if (a.phase32)
        k_pass2_wcorr<T, N, true><<<grid, SH::THREADS, 0, s>>>((const C2<T> *)stack, (const C2<T> *)tw, a, image);
    else
        k_pass2_wcorr<T, N, false><<<grid, SH::THREADS, 0, s>>>((const C2<T> *)stack, (const C2<T> *)tw, a, image);
}

#define WSG_FOR_EACH_N(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(16384)

}  // namespace


void launch_fft_pass1(int N, bool f64, void *planes, int64_t n_planes, const void *twiddle,
                      const Occupancy &occ, hipStream_t s) {
    if (n_planes <= 0) return;
#define X(n)                                                                     \
    case n:                                                                      \
        if (f64) pass1_n<double, n>(planes, n_planes, twiddle, occ, s);          \
        else pass1_n<float, n>(planes, n_planes, twiddle, occ, s);               \
        break;
    switch (N) { WSG_FOR_EACH_N(X) default: break; }
#undef X
}

void launch_fft_pass2_store(int N, bool f64, const void *in, void *out, int64_t n_planes,
                            const void *twiddle, hipStream_t s) {
    if (n_planes <= 0) return;
#define X(n)                                                                     \
    case n:                                                                      \
        if (f64) pass2_store_n<double, n>(in, out, n_planes, twiddle, s);        \
        else pass2_store_n<float, n>(in, out, n_planes, twiddle, s);             \
        break;
    switch (N) { WSG_FOR_EACH_N(X) default: break; }
#undef X
}

void launch_fft_pass2_wcorr(const WcorrArgs &a, bool f64, const void *planes, const void *twiddle,
                            double *image, hipStream_t s) {
    if (a.n_img <= 0) return;
#define X(n)                                                                     \
    case n:                                                                      \
        if (f64) pass2_wcorr_n<double, n>(a, planes, twiddle, image, s);         \
        else pass2_wcorr_n<float, n>(a, planes, twiddle, image, s);              \
        break;
    switch (a.N) { WSG_FOR_EACH_N(X) default: break; }
#undef X
}

void launch_wcorrect(const WcorrArgs &a, bool f64, const void *planes, double *image, hipStream_t s) {
    size_t n2 = (size_t)a.N * a.N;
    unsigned blocks = (unsigned)((n2 + 255) / 256);
    if (f64) {
        if (a.phase32) k_wcorrect<double, true><<<blocks, 256, 0, s>>>((const C2<double> *)planes, a, image);
        else k_wcorrect<double, false><<<blocks, 256, 0, s>>>((const C2<double> *)planes, a, image);
    } else {
        if (a.phase32) k_wcorrect<float, true><<<blocks, 256, 0, s>>>((const C2<float> *)planes, a, image);
        else k_wcorrect<float, false><<<blocks, 256, 0, s>>>((const C2<float> *)planes, a, image);
    }
}

void launch_transpose(int N, bool f64, const void *in, void *out, int64_t n_planes, hipStream_t s) {
    if (n_planes <= 0) return;
    dim3 grid((N + 31) / 32, (N + 31) / 32, (unsigned)n_planes);
    dim3 block(32, 8);
    if (f64) k_transpose<double><<<grid, block, 0, s>>>((const C2<double> *)in, (C2<double> *)out, N);
    else k_transpose<float><<<grid, block, 0, s>>>((const C2<float> *)in, (C2<float> *)out, N);
}

}  // namespace wsg
