// Complex analytic fringe signal (paper Sec. 2, Eq. 1) by an exact DFT mask,
// plus the tiled transposes that turn the y direction into lines.
//
// analytic_kernel: one block per pair of lines (256 threads for transforms up
// to 2048 samples, 1024 above).  The pair is decoded to FP32 as z = x_a + i x_b,
// run through a mixed-radix (4, 2, 3, 5, 7, 11, 13) Stockham FFT ping-ponged
// between two LDS buffers, multiplied by -i sgn(k) (the one-sided mask H[0] =
// 0, H[k] = 2 for 0 < 2k < n, 0 otherwise, applied to the imaginary part: DC
// and Nyquist removed, carrier kept) and transformed back with the same
// forward FFT applied to the conjugate; the real parts are the samples with
// their DC and Nyquist components removed.  Two transforms per pair of lines.  Twiddles come from per-pass tables of each length,
// contiguous in the butterfly index, computed in FP64 on the host and
// rounded once; they are read through the caches (staging them in LDS cost
// more in blocks per CU than it saved in latency).  A length with a prime factor above 13 takes each DFT
// by Bluestein's identity jk = (j^2 + k^2 - (k-j)^2) / 2: with the chirp
// w_j = e^{-i pi j^2 / n}, X_k = w_k sum_j (x_j w_j) conj(w_{k-j}), a linear
// convolution done as a circular one of 5-smooth length m >= 2n - 1 (two
// length-m FFTs against the precomputed transform of the conjugate chirp).
#include "bm_internal.h"

namespace bm {
namespace {

constexpr int kTrThreads = 256;


__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i and +i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }

// One forward Stockham pass of radix R over the whole line: src -> dst.
// tw is the pass's own table: tw[(r-1) Ns + k] = e^{-2 pi i r k / (Ns R)} for
// 0 < r < R, k < Ns (contiguous in k, so neighbouring lanes read neighbouring
// entries), then tw[(R-1) Ns + r - 1] = e^{-2 pi i r / R}, the butterfly's own.
template <int R, int T>
__device__ __forceinline__ void stockham_pass(const float2* __restrict__ src, float2* __restrict__ dst, int n,
                                              int Ns, const float2* __restrict__ tw) {
    const int nR = n / R;
    // j / Ns by a float reciprocal: (j + 1/2) / Ns is at least 1/(2 Ns) from an
    // integer and its rounding error stays below (n / Ns) 2^-22, so the
    // truncation is exact for n <= 8192 (an integer division costs ~30 instructions)
    const float inv_ns = 1.0f / (float)Ns;
    // odd prime radices: cos and sin of 2 pi r / R from the length's own table
    float cs[R], sn[R];
    if constexpr (R >= 7) {
        cs[0] = 1.f;
        sn[0] = 0.f;
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const float2 w = tw[(R - 1) * Ns + r - 1];          // e^{-2 pi i r / R}
            cs[r] = w.x;
            sn[r] = -w.y;
        }
    }
    for (int j = threadIdx.x; j < nR; j += T) {
        const int g = (int)(((float)j + 0.5f) * inv_ns);
        const int k = j - g * Ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[j + r * nR];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(r - 1) * Ns + k]);
        float2 y[R];
        if constexpr (R == 2) {
            y[0] = cadd(v[0], v[1]);
            y[1] = csub(v[0], v[1]);
        } else if constexpr (R == 4) {
            const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
            const float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
            y[0] = cadd(t0, t2);
            y[2] = csub(t0, t2);
            y[1] = cadd(t1, mul_mi(t3));
            y[3] = cadd(t1, mul_pi(t3));
        } else if constexpr (R == 3) {
            constexpr float h = 0.866025403784438647f;  // sin(2 pi / 3)
            const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
            const float2 base = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
            const float2 rot = make_float2(h * d.y, -h * d.x);   // -i h d
            y[0] = cadd(v[0], s);
            y[1] = cadd(base, rot);
            y[2] = csub(base, rot);
        } else if constexpr (R >= 7) {
            // odd prime radix: pair the inputs r and R-r (in place: v[r] = sum,
            // v[R-r] = difference), write each output pair as it is formed,
            // y[q], y[R-q] = v0 + sum_r s_r cos(2 pi r q / R) -/+ i sum_r d_r sin(2 pi r q / R)
            constexpr int h = (R - 1) / 2;
            const int idx = g * Ns * R + k;
            float2 y0 = v[0];
#pragma unroll
            for (int r = 1; r <= h; ++r) {
                const float2 sr = cadd(v[r], v[R - r]);
                v[R - r] = csub(v[r], v[R - r]);
                v[r] = sr;
                y0 = cadd(y0, sr);
            }
            dst[idx] = y0;
#pragma unroll
            for (int q = 1; q <= h; ++q) {
                float2 a = v[0], b = make_float2(0.f, 0.f);
#pragma unroll
                for (int r = 1; r <= h; ++r) {
                    const int e = (r * q) % R;
                    a.x = fmaf(v[r].x, cs[e], a.x);
                    a.y = fmaf(v[r].y, cs[e], a.y);
                    b.x = fmaf(v[R - r].x, sn[e], b.x);
                    b.y = fmaf(v[R - r].y, sn[e], b.y);
                }
                dst[idx + q * Ns] = cadd(a, mul_mi(b));
                dst[idx + (R - q) * Ns] = cadd(a, mul_pi(b));
            }
            continue;
        } else if constexpr (R == 5) {
            constexpr float c1 = 0.309016994374947424f, c2 = -0.809016994374947424f;
            constexpr float s1 = 0.951056516295153572f, s2 = 0.587785252292473129f;
            const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
            const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
            y[0] = cadd(v[0], cadd(a1, a2));
            const float2 p1 = make_float2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
            const float2 q1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
            const float2 p2 = make_float2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
            const float2 q2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
            y[1] = cadd(p1, mul_mi(q1));
            y[4] = cadd(p1, mul_pi(q1));
            y[2] = cadd(p2, mul_mi(q2));
            y[3] = cadd(p2, mul_pi(q2));
        }
        const int idx = g * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[idx + r * Ns] = y[r];
    }
}

template <int R, int T>
__device__ __forceinline__ void stockham_pass_odd(const float2* __restrict__ src, float2* __restrict__ dst, int n, int Ns,
                                               const float2* __restrict__ tw) {
    stockham_pass<R, T>(src, dst, n, Ns, tw);
}

// Forward DFT of the line held in `a` (scratch `b`); returns the buffer that
// holds the result in natural order.  MAXR bounds the radices compiled in: the
// radix-7/11/13 butterflies need several times the registers of the others,
// so plans without them run in a kernel that does not carry them.
template <int MAXR, int T>
__device__ __forceinline__ float2* fft_forward(float2* a, float2* b, int n, const FftPlan& plan, const float2* tw) {
    int Ns = 1;
    for (int ps = 0; ps < plan.passes; ++ps) {
        const int R = plan.radix[ps];
        const float2* twp = tw;                 // this pass's table, then the next one's
        tw += (R - 1) * (Ns + 1);
        if (R == 4) stockham_pass<4, T>(a, b, n, Ns, twp);
        else if (R == 2) stockham_pass<2, T>(a, b, n, Ns, twp);
        else if (R == 3) stockham_pass<3, T>(a, b, n, Ns, twp);
        else if (MAXR <= 5 || R == 5) stockham_pass<5, T>(a, b, n, Ns, twp);
        else if (R == 7) stockham_pass_odd<7, T>(a, b, n, Ns, twp);
        else if (R == 11) stockham_pass_odd<11, T>(a, b, n, Ns, twp);
        else stockham_pass_odd<13, T>(a, b, n, Ns, twp);
        __syncthreads();
        float2* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// DFT of the n samples at a[0..n): a direct mixed-radix FFT, or Bluestein's
// chirp-z route through length plan.n = m.  a and b hold m elements each;
// returns the buffer holding X[0..n) in natural order.
template <int MAXR, int T>
__device__ __forceinline__ float2* dft_line(float2* a, float2* b, const FftJob& J, const float2* tw) {
    const int n = J.n, m = J.plan.n;
    if (!J.chirp) return fft_forward<MAXR, T>(a, b, n, J.plan, tw);
    for (int i = threadIdx.x; i < m; i += T)
        a[i] = i < n ? cmul(a[i], J.chirp[i]) : make_float2(0.f, 0.f);
    __syncthreads();
    float2* P = fft_forward<MAXR, T>(a, b, m, J.plan, tw);
    float2* Q = (P == a) ? b : a;
    // circular convolution with conj(w): inverse DFT as the conjugate of a forward one
    for (int k = threadIdx.x; k < m; k += T) {
        const float2 v = cmul(P[k], J.kern[k]);
        P[k] = make_float2(v.x, -v.y);
    }
    __syncthreads();
    float2* Y = fft_forward<MAXR, T>(P, Q, m, J.plan, tw);
    for (int k = threadIdx.x; k < n; k += T) {
        const float2 v = Y[k];
        Y[k] = cmul(make_float2(v.x, -v.y), J.chirp[k]);
    }
    __syncthreads();
    return Y;
}

// Index of the job that owns work item w: prefix[j] <= w < prefix[j+1].
__device__ __forceinline__ int find_job(const int* prefix, int njobs, int w) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float load_real(const void* base, int64_t idx, int elem) {
    if (elem == (int)Elem::F16) return (float)static_cast<const _Float16*>(base)[idx];
    if (elem == (int)Elem::F64) return (float)static_cast<const double*>(base)[idx];
    if (elem == (int)Elem::U8) return (float)static_cast<const unsigned char*>(base)[idx];
    return static_cast<const float*>(base)[idx];
}

__device__ __forceinline__ float2 conjf2(float2 v) { return make_float2(v.x, -v.y); }

// Gamma is stored with streaming (nontemporal) stores: a later launch reads it,
// long after it has left the caches, while the samples that the analytic
// kernels read a second time should stay there.
typedef float f2v __attribute__((ext_vector_type(2)));

// One block per pair of lines (2i, 2i+1; a lone last line pairs with zeros).
// With z = x_a + i x_b and Z = DFT(z), the analytic signal of each real line
// is Gamma = IFFT(H X) (reading of Sec. 2 / Eq. 1: H[0] = 0, H[k] = 2 for
// 0 < 2k < n, 0 above), whose two parts are
//   Re Gamma = x - X[0]/n - X[n/2] (-1)^i / n      (DC and Nyquist removed)
//   Im Gamma = IFFT(-i sgn(k) X[k])                (the Hilbert transform)
// with sgn(k) = +1 for 0 < 2k < n, -1 for 2k > n, 0 at k = 0 and 2k = n.  The
// Hilbert transform is real-linear, so one inverse DFT of -i sgn(k) Z[k]
// gives h_a + i h_b, the imaginary parts of both lines, and X_a[0] + i X_b[0]
// = Z[0] (and so at n/2).  A pair costs two transforms instead of the three
// that splitting the spectra and inverting H X_a and H X_b take (four for two
// lines alone), and needs two line buffers of LDS.  The real parts are the
// samples themselves, read again at the end (from the cache: holding them in
// registers instead took the 1024-thread kernel from two blocks per CU to one).
template <int MAXR, int T>
__global__ __launch_bounds__(T) void analytic_kernel(FftBatch B, int item0) {
    extern __shared__ float2 lds[];
    const int w = item0 + blockIdx.x;
    const int j = find_job(B.prefix, B.njobs, w);
    const FftJob& J = B.jobs[j];
    const int item = w - B.prefix[j];
    const int n = J.n, m = J.plan.n;
    const int elem = J.elem;
    const int la = 2 * item;
    const bool two = la + 1 < J.nlines;
    float2* a = lds;
    float2* b = lds + m;
    const float2* tw = J.tw;
    const int64_t off = (int64_t)la * J.src_ls;
    for (int i = threadIdx.x; i < n; i += T)
        a[i] = make_float2(load_real(J.src, off + i, elem), two ? load_real(J.src, off + J.src_ls + i, elem) : 0.f);
    __syncthreads();
    float2* X = dft_line<MAXR, T>(a, b, J, tw);
    float2* V = (X == a) ? b : a;
    const float inv_n = 1.0f / (float)n;
    const float2 z0 = X[0];
    const float2 zh = (n & 1) ? make_float2(0.f, 0.f) : X[n >> 1];
    // V = conj(-i sgn(k) Z[k]) / n = sgn(k) (Im Z, Re Z) / n, so that the forward DFT
    // of V, conjugated, is IFFT(-i sgn Z)
    for (int k = threadIdx.x; k < n; k += T) {
        const float2 v = X[k];
        const float sg = (k == 0 || 2 * k == n) ? 0.f : (2 * k < n ? inv_n : -inv_n);
        V[k] = make_float2(sg * v.y, sg * v.x);
    }
    __syncthreads();
    float2* Y = dft_line<MAXR, T>(V, X, J, tw);
    // h_a + i h_b = conj(Y): Im Gamma_a = Y.x, Im Gamma_b = -Y.y
    const float dca = z0.x * inv_n, dcb = z0.y * inv_n, nqa = zh.x * inv_n, nqb = zh.y * inv_n;
    float2* out = J.dst + (int64_t)la * n;
    for (int i = threadIdx.x; i < n; i += T) {
        const float sgn = (i & 1) ? -1.f : 1.f;
        const float2 y = Y[i];
        __builtin_nontemporal_store(f2v{load_real(J.src, off + i, elem) - dca - sgn * nqa, y.x},
                                    reinterpret_cast<f2v*>(out + i));
        if (two)
            __builtin_nontemporal_store(f2v{load_real(J.src, off + J.src_ls + i, elem) - dcb - sgn * nqb, -y.y},
                                        reinterpret_cast<f2v*>(out + n + i));
    }
}

// ---- power-of-two lines of 512 ... 4096 samples: register-resident passes ----
//
// n = R0 * 256 with R0 in {2, 4, 8, 16} takes three Stockham passes of radices
// R0, 16, 16 (the pass formulas of stockham_pass).  A line pair is n/16
// threads, and in every pass thread j holds the 16 elements j + s n/16,
// s < 16, of the transform in registers: the first pass reads them straight
// from the frame, the last leaves X[j + s n/16] in natural order, which is
// where the spectrum is multiplied and the inverse transform's first pass
// starts, so only four exchanges per line pair go through LDS (one buffer of
// 4096 elements, read fully before it is rewritten).  A block of 256 threads
// takes 4096/n pairs.  LDS index i lives at i ^ ((i >> 5) & 31): the strided
// writes of the first two passes then meet at most two lanes per bank.

__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 5) & 31); }

// forward DFT4 in place: x_k = sum_n x_n e^{-2 pi i n k / 4}
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = csub(x1, x3);
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, mul_mi(t3));
    x3 = cadd(t1, mul_pi(t3));
}

// a e^{-2 pi i m / 16}
template <int M>
__device__ __forceinline__ float2 w16(float2 a) {
    constexpr int m = M & 15;
    constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f, h = 0.707106781186547524f;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return mul_mi(a);
    else if constexpr (m == 8) return make_float2(-a.x, -a.y);
    else if constexpr (m == 12) return mul_pi(a);
    else {
        constexpr float c = m == 1 ? c1 : m == 2 ? h : m == 3 ? s1 : m == 5 ? -s1 : m == 6 ? -h : m == 7 ? -c1
                          : m == 9 ? -c1 : m == 10 ? -h : m == 11 ? -s1 : m == 13 ? s1 : m == 14 ? h : c1;
        constexpr float sn = m == 1 ? s1 : m == 2 ? h : m == 3 ? c1 : m == 5 ? c1 : m == 6 ? h : m == 7 ? s1
                           : m == 9 ? -s1 : m == 10 ? -h : m == 11 ? -c1 : m == 13 ? -c1 : m == 14 ? -h : -s1;
        // (a.x + i a.y)(c - i sn)
        return make_float2(fmaf(a.x, c, a.y * sn), fmaf(a.y, c, -a.x * sn));
    }
}

// forward DFT16 in place, as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);   // v[4 k1 + n2]
    v[5] = w16<1>(v[5]);
    v[6] = w16<2>(v[6]);
    v[7] = w16<3>(v[7]);
    v[9] = w16<2>(v[9]);
    v[10] = w16<4>(v[10]);
    v[11] = w16<6>(v[11]);
    v[13] = w16<3>(v[13]);
    v[14] = w16<6>(v[14]);
    v[15] = w16<9>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);  // v[4 k1 + k2]
    float2 o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = o[k];
}

// forward DFT8 of v[i0 + r st], r < 8, in place, as 2 x 4: n = 2 n1 + n2, k = k1 + 4 k2
template <int I0, int ST>
__device__ __forceinline__ void dft8s(float2 (&v)[16]) {
    float2 a[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = v[I0 + r * ST];
    dft4(a[0], a[2], a[4], a[6]);    // a[2 k1]     = A[0][k1]
    dft4(a[1], a[3], a[5], a[7]);    // a[2 k1 + 1] = A[1][k1]
    a[3] = w16<2>(a[3]);
    a[5] = w16<4>(a[5]);
    a[7] = w16<6>(a[7]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        v[I0 + k1 * ST] = cadd(a[2 * k1], a[2 * k1 + 1]);
        v[I0 + (k1 + 4) * ST] = csub(a[2 * k1], a[2 * k1 + 1]);
    }
}

// First pass (radix R0, Ns = 1) on the registers of thread j: butterfly
// j + T q (q < 16/R0) takes z[q + r 16/R0], r < R0, and writes element
// (j + T q) R0 + r of the line pair's buffer.
template <int R0, int T>
__device__ __forceinline__ void pow2_first_pass(float2 (&z)[16], float2* buf, int base, int j) {
    constexpr int Q = 16 / R0;
    if constexpr (R0 == 16) {
        dft16(z);
    } else if constexpr (R0 == 8) {
        dft8s<0, 2>(z);
        dft8s<1, 2>(z);
    } else if constexpr (R0 == 4) {
#pragma unroll
        for (int q = 0; q < Q; ++q) dft4(z[q], z[q + Q], z[q + 2 * Q], z[q + 3 * Q]);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float2 a = z[q], b = z[q + Q];
            z[q] = cadd(a, b);
            z[q + Q] = csub(a, b);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int r = 0; r < R0; ++r) buf[swz(base + (j + T * q) * R0 + r)] = z[q + r * Q];
}

// A radix-16 pass with stride Ns (power of two) on the registers of thread j:
// twiddles w^s = tw[(s - 1) Ns + k], k = j mod Ns, of which six are read
// (s = 1, 2, 3, 4, 8, 12) and the others formed as w^{4a} w^b (one more
// rounding: fewer live registers than fifteen loads); the DFT16 result stays in v.
__device__ __forceinline__ void pow2_pass16(float2 (&v)[16], const float2* __restrict__ tw, int Ns, int j) {
    const int k = j & (Ns - 1);
    const float2 wb[4] = {make_float2(1.f, 0.f), tw[k], tw[Ns + k], tw[2 * Ns + k]};
    const float2 wa[4] = {make_float2(1.f, 0.f), tw[3 * Ns + k], tw[7 * Ns + k], tw[11 * Ns + k]};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int s = 4 * a + b;
            if (s == 0) continue;
            const float2 w = (a == 0) ? wb[b] : (b == 0 ? wa[a] : cmul(wa[a], wb[b]));
            v[s] = cmul(v[s], w);
        }
    dft16(v);
}

// Forward transform of the pair held in z (thread j, pair buffer at base):
// on return z[s] = Z[j + s T].  Starts and ends without a pending barrier.
template <int R0>
__device__ __forceinline__ void pow2_fft(float2 (&z)[16], float2* buf, int base, int j, const float2* tw) {
    constexpr int T = R0 * 16;           // threads per line pair = n / 16
    pow2_first_pass<R0, T>(z, buf, base, j);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) z[s] = buf[swz(base + j + s * T)];
    __syncthreads();
    const float2* tw1 = tw + 2 * (R0 - 1);
    pow2_pass16(z, tw1, R0, j);
    const int g = j / R0, k = j & (R0 - 1);
#pragma unroll
    for (int s = 0; s < 16; ++s) buf[swz(base + g * 16 * R0 + k + s * R0)] = z[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) z[s] = buf[swz(base + j + s * T)];
    const float2* tw2 = tw1 + 15 * (R0 + 1);
    pow2_pass16(z, tw2, T, j);
}

// The analytic signal of analytic_kernel for n = 256 R0, per line pair:
// Z = DFT(x_a + i x_b), V = sgn(k) (Im Z, Re Z) / n, Y = DFT(V); Im Gamma_a =
// Y.x, Im Gamma_b = -Y.y, Re Gamma = x - DC - Nyquist (-1)^i.
template <int R0>
__global__ __launch_bounds__(256) void analytic_pow2_kernel(FftBatch B, int item0) {
    constexpr int n = 256 * R0, T = 16 * R0, P = 4096 / n;
    __shared__ float2 buf[4096];
    const int w = item0 + blockIdx.x;
    const int jb = find_job(B.prefix, B.njobs, w);
    const FftJob& J = B.jobs[jb];
    const int item = w - B.prefix[jb];
    const int t = threadIdx.x, p = t / T, j = t - p * T;
    const int base = p * n;
    const int la = 2 * (item * P + p);
    const bool has_a = la < J.nlines, has_b = la + 1 < J.nlines;
    const int elem = J.elem;
    const int64_t off = (int64_t)la * J.src_ls;
    float2 z[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int i = j + s * T;
        z[s] = make_float2(has_a ? load_real(J.src, off + i, elem) : 0.f,
                           has_b ? load_real(J.src, off + J.src_ls + i, elem) : 0.f);
    }
    pow2_fft<R0>(z, buf, base, j, J.tw);
    // z[s] = Z[j + s T]; DC at (j, s) = (0, 0), Nyquist at (0, 8)
    const float2 z0 = z[0], zh = z[8];
    constexpr float inv_n = 1.0f / (float)n;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int k = j + s * T;
        const float sg = (k == 0 || 2 * k == n) ? 0.f : (2 * k < n ? inv_n : -inv_n);
        z[s] = make_float2(sg * z[s].y, sg * z[s].x);
    }
    __syncthreads();
    pow2_fft<R0>(z, buf, base, j, J.tw);
    // the pair's DC and Nyquist terms, from thread 0 of the pair
    __syncthreads();
    if (j == 0) {
        buf[base] = z0;
        buf[base + 1] = zh;
    }
    __syncthreads();
    const float2 dc = buf[base], ny = buf[base + 1];
    const float dca = dc.x * inv_n, dcb = dc.y * inv_n, nqa = ny.x * inv_n, nqb = ny.y * inv_n;
    float2* out = J.dst + (int64_t)la * n;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int i = j + s * T;
        const float sgn = (i & 1) ? -1.f : 1.f;
        if (has_a) __builtin_nontemporal_store(f2v{load_real(J.src, off + i, elem) - dca - sgn * nqa, z[s].x},
                                               reinterpret_cast<f2v*>(out + i));
        if (has_b) __builtin_nontemporal_store(f2v{load_real(J.src, off + J.src_ls + i, elem) - dcb - sgn * nqb, -z[s].y},
                                               reinterpret_cast<f2v*>(out + n + i));
    }
}

// One block of 256 threads per tile of any job: 64 x 64 for real input
// (decoded to FP32, 16 elements per thread) and 32 x 32 float2 for C32 input
// (4 per thread), both in the same LDS words.  Tiles are padded by one
// element per row so that the column reads hit distinct banks.  (32 x 32
// float2 tiles for real data too were 1.45x slower on the 1024^2 frames.)
__global__ __launch_bounds__(kTrThreads) void transpose_kernel(TrBatch B) {
    __shared__ __align__(16) float smem[kTrTile * (kTrTile + 1)];
    const int j = find_job(B.prefix, B.njobs, blockIdx.x);
    const TrJob& J = B.jobs[j];
    const int tid = blockIdx.x - B.prefix[j];
    const int rows = J.rows, cols = J.cols, elem = J.elem;
    if (elem == (int)Elem::C32) {
        constexpr int T = kTrTileC, S = kTrThreads / kTrTileC;
        float2 (*tile)[T + 1] = reinterpret_cast<float2 (*)[T + 1]>(smem);
        const int bx = (tid % J.tiles_x) * T, by = (tid / J.tiles_x) * T;
        const int tx = threadIdx.x % T, ty = threadIdx.x / T;
#pragma unroll
        for (int jj = 0; jj < T; jj += S) {
            const int r = by + ty + jj, c = bx + tx;
            if (r < rows && c < cols) tile[ty + jj][tx] = static_cast<const float2*>(J.src)[(int64_t)r * J.src_ls + c];
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < T; jj += S) {
            const int c = bx + ty + jj, r = by + tx;
            if (r < rows && c < cols) static_cast<float2*>(J.dst)[(int64_t)c * rows + r] = tile[tx][ty + jj];
        }
        return;
    }
    constexpr int T = kTrTile, S = kTrThreads / kTrTile;
    float (*tile)[T + 1] = reinterpret_cast<float (*)[T + 1]>(smem);
    const int bx = (tid % J.tiles_x) * T, by = (tid / J.tiles_x) * T;
    // Whole FP32/FP16 tiles with 16-byte aligned rows on both sides: each thread
    // moves four runs of four elements (one 16- or 8-byte load, one 16-byte
    // store each) instead of sixteen single elements.
    const bool vec = (elem == (int)Elem::F32 || elem == (int)Elem::F16) && bx + T <= cols && by + T <= rows &&
                     (J.src_ls & 3) == 0 && (rows & 3) == 0 && ((uintptr_t)J.src & 15) == 0 &&
                     ((uintptr_t)J.dst & 15) == 0;
    if (vec) {
        constexpr int G = T / 4, RS = kTrThreads / G;        // 16 groups of four columns, 16 rows a round
        const int c4 = (threadIdx.x % G) * 4, r0 = threadIdx.x / G;
#pragma unroll
        for (int jj = 0; jj < T; jj += RS) {
            const int64_t idx = (int64_t)(by + r0 + jj) * J.src_ls + bx + c4;
            float4 v;
            if (elem == (int)Elem::F32) {
                v = *reinterpret_cast<const float4*>(static_cast<const float*>(J.src) + idx);
            } else {
                typedef _Float16 h4 __attribute__((ext_vector_type(4)));
                const h4 h = *reinterpret_cast<const h4*>(static_cast<const _Float16*>(J.src) + idx);
                v = make_float4((float)h[0], (float)h[1], (float)h[2], (float)h[3]);
            }
            tile[r0 + jj][c4] = v.x;
            tile[r0 + jj][c4 + 1] = v.y;
            tile[r0 + jj][c4 + 2] = v.z;
            tile[r0 + jj][c4 + 3] = v.w;
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < T; jj += RS) {
            const int c = r0 + jj;                             // destination row bx + c, elements by + c4 ..
            const float4 v = make_float4(tile[c4][c], tile[c4 + 1][c], tile[c4 + 2][c], tile[c4 + 3][c]);
            *reinterpret_cast<float4*>(static_cast<float*>(J.dst) + (int64_t)(bx + c) * rows + by + c4) = v;
        }
        return;
    }
    const int tx = threadIdx.x % T, ty = threadIdx.x / T;
#pragma unroll
    for (int jj = 0; jj < T; jj += S) {
        const int r = by + ty + jj, c = bx + tx;
        if (r < rows && c < cols) tile[ty + jj][tx] = load_real(J.src, (int64_t)r * J.src_ls + c, elem);
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < T; jj += S) {
        const int c = bx + ty + jj, r = by + tx;
        if (r < rows && c < cols) static_cast<float*>(J.dst)[(int64_t)c * rows + r] = tile[tx][ty + jj];
    }
}

}  // namespace

hipError_t analytic_set_attributes() {
    const int bytes = kFftLdsElems * (int)sizeof(float2);
    const void* k[4] = {(const void*)analytic_kernel<5, 256>, (const void*)analytic_kernel<13, 256>,
                                  (const void*)analytic_kernel<5, 1024>, (const void*)analytic_kernel<13, 1024>};
    for (const void* f : k) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_analytic(const FftBatch& b, hipStream_t s) {
    for (int c = 0; c < kFftClasses; ++c) {
        const int i0 = b.cls_from[c], cnt = b.cls_from[c + 1] - i0;
        if (cnt <= 0) continue;
        const size_t shmem = (size_t)b.lds[c] * sizeof(float2);
        switch (c) {
            case 0: hipLaunchKernelGGL((analytic_kernel<5, 256>), dim3(cnt), dim3(256), shmem, s, b, i0); break;
            case 1: hipLaunchKernelGGL((analytic_kernel<13, 256>), dim3(cnt), dim3(256), shmem, s, b, i0); break;
            case 2: hipLaunchKernelGGL((analytic_kernel<5, 1024>), dim3(cnt), dim3(1024), shmem, s, b, i0); break;
            case 3: hipLaunchKernelGGL((analytic_kernel<13, 1024>), dim3(cnt), dim3(1024), shmem, s, b, i0); break;
            case 4: hipLaunchKernelGGL((analytic_pow2_kernel<2>), dim3(cnt), dim3(256), 0, s, b, i0); break;
            case 5: hipLaunchKernelGGL((analytic_pow2_kernel<4>), dim3(cnt), dim3(256), 0, s, b, i0); break;
            case 6: hipLaunchKernelGGL((analytic_pow2_kernel<8>), dim3(cnt), dim3(256), 0, s, b, i0); break;
            default: hipLaunchKernelGGL((analytic_pow2_kernel<16>), dim3(cnt), dim3(256), 0, s, b, i0); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_transpose(const TrBatch& b, hipStream_t s) {
    if (b.total <= 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_kernel, dim3(b.total), dim3(kTrThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace bm

namespace bm {
namespace {

// Deterministic test signal for the autotuner: a complex tone of frequency
// w0 plus hashed uniform noise of amplitude `noise`.
__global__ void synth_kernel(float2* g, int64_t n, float w0, float noise) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    const float u1 = (float)(h & 0xffff) * (1.f / 65536.f) - 0.5f;
    const float u2 = (float)(h >> 16) * (1.f / 65536.f) - 0.5f;
    float s, c;
    sincosf(w0 * (float)(i % 4096), &s, &c);
    g[i] = make_float2(c + noise * u1, s + noise * u2);
}

}  // namespace

hipError_t launch_synth(float2* g, int64_t n, float w0, float noise, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, n, w0, noise);
    return hipGetLastError();
}

}  // namespace bm
