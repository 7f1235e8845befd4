// Per-window root-MUSIC local-frequency kernel for gfx950.
//
// One lane owns one window (one output pixel of one direction).  A block of
// BLOCK lanes (128 or 256) covers BLOCK-(L-1) consecutive window positions of one line; the
// overlapping windows are staged once in LDS with coalesced loads.  Steps:
//
//   lag sums    S_d(m) = sum_k g[m+k] conj(g[m+k+d]), d < L, one start m per
//               lane, shared through LDS: the covariance of the window that
//               starts at s is R_ij = S_{j-i}(s+i)             (paper Eq. 4)
//   FB average + unitary real transform: T = Q^H R_fb Q is real symmetric
//               (Q the sparse centro-symmetric unitary matrix), built in
//               closed form from R without forming R_fb
//   eigen-split the eigenvector v of the largest eigenvalue of T gives the
//               signal subspace u1 = Q v (paper Eq. 6-11, one-dimensional
//               signal subspace).  Default solver: Householder reduction to
//               tridiagonal form, Newton's method from above on the
//               characteristic polynomial (monotone for real-rooted
//               polynomials) for the largest eigenvalue, one shifted inverse
//               iteration for its eigenvector, back-transformation.  The
//               cyclic Jacobi solver is kept as a selectable alternative.
//   polynomial  c_k = sum_i C[i,i+k] with C = I - u1 u1^H = Un Un^H
//               (paper Eq. 12-14)
//   roots       Aberth-Ehrlich simultaneous iteration in FP32 from the roots
//               of the noise-free single-tone polynomial rotated to the
//               window's frequency guess; evaluation at 1/conj(z) for roots
//               outside the unit circle keeps Horner free of overflow
//   selection   the root nearest the unit circle and its mate nearest
//               1/conj(z_sel) (the paper's rule, Sec. 3, applied to the
//               conjugate-reciprocal root pairs)
//   polish      FP64 Newton iteration on the pair's quadratic factor
//               z^2 - r z - s (Bairstow's method with complex coefficients),
//               which is well conditioned even when the pair is a
//               near-double root
//   omega       arg(r) = arg(z_sel + z_mate)  (paper Eq. 15)
#include "bm_internal.h"

#include <cmath>

namespace bm {
namespace {

// Tunables (overridable at compile time for tuning sweeps).
#ifndef BM_JACOBI_TOL2
#define BM_JACOBI_TOL2 1e-12f   // squared off-diagonal mass of the trace-normalised matrix
#endif
#ifndef BM_ROOT_TOL2
#define BM_ROOT_TOL2 1e-4f      // squared relative root step that ends the root iteration
#endif
#ifndef BM_MAX_ROOT_ITERS
#define BM_MAX_ROOT_ITERS 16
#endif
#ifndef BM_POLISH_ITERS
#define BM_POLISH_ITERS 3
#endif
#ifndef BM_NEWTON_ITERS
#define BM_NEWTON_ITERS 12
#endif
#ifndef BM_INVERSE_ITERS
#define BM_INVERSE_ITERS 2
#endif

constexpr int kMaxJacobiSweeps = 10;
constexpr float kJacobiTol2 = BM_JACOBI_TOL2;
constexpr int kMaxRootIters = BM_MAX_ROOT_ITERS;
constexpr float kRootTol2 = BM_ROOT_TOL2;
constexpr int kPolishIters = BM_POLISH_ITERS;
constexpr int kNewtonIters = BM_NEWTON_ITERS;
constexpr int kInverseIters = BM_INVERSE_ITERS;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

// Symmetric L x L matrix, upper triangle stored (compile-time indices only).
template <int L>
struct Sym {
    float a[L][L];
    __device__ __forceinline__ float& at(int i, int j) { return i <= j ? a[i][j] : a[j][i]; }
};

// Hermitian covariance, upper triangle stored.
template <int L>
struct Cov {
    float re[L][L];
    float im[L][L];
    __device__ __forceinline__ float gr(int i, int j) const { return i <= j ? re[i][j] : re[j][i]; }
    __device__ __forceinline__ float gi(int i, int j) const { return i <= j ? im[i][j] : -im[j][i]; }
};

// T = Q^H R_fb Q, real symmetric.  With F = R + J conj(R) J = 2 R_fb, m = L/2,
// o = L - m, and i, j < m:
//   T[i][j]     = Re(F[i][j] + F[i][L-1-j])
//   T[i][o+j]   = Im F[i][L-1-j] - Im F[i][j]
//   T[o+i][o+j] = Re(F[i][j] - F[i][L-1-j])
// and for odd L: T[i][m] = sqrt2 Re F[i][m], T[m][m] = Re F[m][m],
// T[m][o+j] = -sqrt2 Im F[m][j].
template <int L>
__device__ __forceinline__ void build_T(const Cov<L>& R, Sym<L>& T) {
    constexpr int m = L / 2;
    constexpr int o = L - m;
    constexpr float kSqrt2 = 1.41421356237309515f;
    auto Fr = [&](int i, int j) { return R.gr(i, j) + R.gr(L - 1 - i, L - 1 - j); };
    auto Fi = [&](int i, int j) { return R.gi(i, j) - R.gi(L - 1 - i, L - 1 - j); };
#pragma unroll
    for (int i = 0; i < m; ++i) {
#pragma unroll
        for (int j = 0; j < m; ++j) {
            if (j >= i) {
                T.a[i][j] = Fr(i, j) + Fr(i, L - 1 - j);
                T.a[o + i][o + j] = Fr(i, j) - Fr(i, L - 1 - j);
            }
            T.a[i][o + j] = Fi(i, L - 1 - j) - Fi(i, j);
        }
        if (L & 1) T.a[i][m] = kSqrt2 * Fr(i, m);
    }
    if (L & 1) {
        T.a[m][m] = Fr(m, m);
#pragma unroll
        for (int j = 0; j < m; ++j) T.a[m][o + j] = -kSqrt2 * Fi(m, j);
    }
}

// Eigenvector of the largest eigenvalue of the trace-normalised symmetric T:
// Householder tridiagonalisation, Newton from above on det(xI - T_tri),
// shifted inverse iteration on the tridiagonal matrix, back-transformation.
template <int L>
__device__ __forceinline__ void top_eigvec_tridiag(Sym<L>& T, float (&v)[L], int& its) {
    float hv[L][L];   // reflector k lives in hv[k][k+1 .. L-1]
    float hb[L];
    float e[L];
#pragma unroll
    for (int k = 0; k < L - 2; ++k) {
        float nrm2 = 0.f;
#pragma unroll
        for (int j = k + 1; j < L; ++j) {
            hv[k][j] = T.at(j, k);
            nrm2 = fmaf(hv[k][j], hv[k][j], nrm2);
        }
        const float nrm = fsqrt(nrm2);
        const float alpha = hv[k][k + 1] >= 0.f ? -nrm : nrm;
        hv[k][k + 1] -= alpha;
        float vtv = 0.f;
#pragma unroll
        for (int j = k + 1; j < L; ++j) vtv = fmaf(hv[k][j], hv[k][j], vtv);
        const float beta = vtv > 0.f ? 2.f * frcp(vtv) : 0.f;
        hb[k] = beta;
        e[k] = alpha;
        float p[L];
#pragma unroll
        for (int i = k + 1; i < L; ++i) {
            float acc = 0.f;
#pragma unroll
            for (int j = k + 1; j < L; ++j) acc = fmaf(T.at(i, j), hv[k][j], acc);
            p[i] = beta * acc;
        }
        float pv = 0.f;
#pragma unroll
        for (int i = k + 1; i < L; ++i) pv = fmaf(p[i], hv[k][i], pv);
        const float Kf = 0.5f * beta * pv;
#pragma unroll
        for (int i = k + 1; i < L; ++i) p[i] = fmaf(-Kf, hv[k][i], p[i]);   // w
#pragma unroll
        for (int i = k + 1; i < L; ++i)
#pragma unroll
            for (int j = i; j < L; ++j) T.a[i][j] -= fmaf(hv[k][i], p[j], p[i] * hv[k][j]);
    }
    float d[L];
#pragma unroll
    for (int i = 0; i < L; ++i) d[i] = T.a[i][i];
    e[L - 2] = T.a[L - 2][L - 1];
    float e2[L];
#pragma unroll
    for (int i = 0; i < L - 1; ++i) e2[i] = e[i] * e[i];
    // start above the largest eigenvalue: T is positive semidefinite with trace 1
    float g = 0.f;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        float r = d[i];
        if (i > 0) r += fabsf(e[i - 1]);
        if (i < L - 1) r += fabsf(e[i]);
        g = fmaxf(g, r);
    }
    float x = fminf(g, 1.f) * 1.000001f + 1e-30f;
    for (int it = 0; it < kNewtonIters; ++it) {
        ++its;
        float q0 = 1.f, q1 = x - d[0], dq0 = 0.f, dq1 = 1.f;
#pragma unroll
        for (int i = 1; i < L; ++i) {
            const float xi = x - d[i];
            const float q2 = fmaf(xi, q1, -e2[i - 1] * q0);
            const float dq2 = fmaf(xi, dq1, fmaf(-e2[i - 1], dq0, q1));
            q0 = q1; q1 = q2; dq0 = dq1; dq1 = dq2;
        }
        const float step = q1 * frcp(dq1);
        if (!finitef(step)) break;
        x -= step;
        if (!(fabsf(step) > 1e-7f * x)) break;
    }
    // (sigma I - T_tri) y = y_prev, LDL^T without pivoting; sigma just above lambda_1
    const float sigma = x * 1.000002f + 1e-30f;
    float y[L];
#pragma unroll
    for (int i = 0; i < L; ++i) y[i] = 1.f;
    float Dg[L], l[L];
    Dg[0] = sigma - d[0];
#pragma unroll
    for (int i = 0; i < L - 1; ++i) {
        const float Di = Dg[i] != 0.f ? Dg[i] : 1e-30f;
        l[i] = -e[i] * frcp(Di);
        Dg[i + 1] = fmaf(-l[i] * l[i], Di, sigma - d[i + 1]);
    }
    float Dinv[L];
#pragma unroll
    for (int i = 0; i < L; ++i) Dinv[i] = frcp(Dg[i] != 0.f ? Dg[i] : 1e-30f);
#pragma unroll
    for (int it = 0; it < kInverseIters; ++it) {
#pragma unroll
        for (int i = 1; i < L; ++i) y[i] = fmaf(-l[i - 1], y[i - 1], y[i]);
#pragma unroll
        for (int i = 0; i < L; ++i) y[i] *= Dinv[i];
#pragma unroll
        for (int i = L - 2; i >= 0; --i) y[i] = fmaf(-l[i], y[i + 1], y[i]);
        float n2 = 0.f;
#pragma unroll
        for (int i = 0; i < L; ++i) n2 = fmaf(y[i], y[i], n2);
        const float in = frsq(n2);
#pragma unroll
        for (int i = 0; i < L; ++i) y[i] *= in;
    }
#pragma unroll
    for (int k = L - 3; k >= 0; --k) {
        float sp = 0.f;
#pragma unroll
        for (int j = k + 1; j < L; ++j) sp = fmaf(hv[k][j], y[j], sp);
        sp *= hb[k];
#pragma unroll
        for (int j = k + 1; j < L; ++j) y[j] = fmaf(-sp, hv[k][j], y[j]);
    }
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] = y[i];
}

// Same eigenvector by cyclic Jacobi rotations (selectable alternative).
template <int L>
__device__ __forceinline__ void top_eigvec_jacobi(Sym<L>& T, float (&v)[L], int& sweeps) {
    float V[L][L];
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = 0; j < L; ++j) V[i][j] = (i == j) ? 1.f : 0.f;
    for (int sw = 0; sw < kMaxJacobiSweeps; ++sw) {
        float off = 0.f;
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int j = i + 1; j < L; ++j) off = fmaf(T.a[i][j], T.a[i][j], off);
        if (!(off > kJacobiTol2)) break;
        ++sweeps;
#pragma unroll
        for (int pp = 0; pp < L - 1; ++pp) {
#pragma unroll
            for (int qq = pp + 1; qq < L; ++qq) {
                const float apq = T.a[pp][qq];
                const float th = T.a[qq][qq] - T.a[pp][pp];
                const float sgn = th >= 0.f ? 1.f : -1.f;
                const float den = fabsf(th) + fsqrt(fmaf(th, th, 4.f * apq * apq));
                const float tt = den > 0.f ? 2.f * apq * sgn * frcp(den) : 0.f;
                const float c = frsq(fmaf(tt, tt, 1.f));
                const float s = tt * c;
                T.a[pp][pp] = fmaf(-tt, apq, T.a[pp][pp]);
                T.a[qq][qq] = fmaf(tt, apq, T.a[qq][qq]);
                T.a[pp][qq] = 0.f;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    if (k == pp || k == qq) continue;
                    const float akp = T.at(k, pp), akq = T.at(k, qq);
                    T.at(k, pp) = c * akp - s * akq;
                    T.at(k, qq) = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    const float vkp = V[k][pp], vkq = V[k][qq];
                    V[k][pp] = c * vkp - s * vkq;
                    V[k][qq] = s * vkp + c * vkq;
                }
            }
        }
    }
    float best = T.a[0][0];
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] = V[i][0];
#pragma unroll
    for (int k = 1; k < L; ++k) {
        const bool b = T.a[k][k] > best;
        best = b ? T.a[k][k] : best;
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = b ? V[i][k] : v[i];
    }
}

// Counters a lane accumulates over the windows it owns.
struct LaneStats {
    int counted = 0, eig_its = 0, iters = 0, pfail = 0;
};

// One block of windows: BLOCK-(L-1) consecutive pixels p0.. of one line of job J.
template <int L, int BLOCK, bool JACOBI>
__device__ __forceinline__ void rootmusic_block(const RmJob& J, int line, int p0, float2* sg, float2 (*sS)[BLOCK],
                                                const RootTemplate& tmpl, LaneStats& ls) {
    constexpr int n = 2 * L - 2;            // polynomial degree
    constexpr int m = L / 2;
    constexpr int o = L - m;
    constexpr int WPB = BLOCK - (L - 1);
    const int t = threadIdx.x;
    const int N = J.N;
    const int half = N >> 1;
    const int K = N - L + 1;
    const float2* g = J.gamma + (int64_t)line * J.gamma_ls;
    const int len = J.len;

    // window of pixel p0+t starts at base+t
    const int base = p0 - half;
    for (int i = t; i < BLOCK + N - 1; i += BLOCK) {
        const int q = base + i;
        sg[i] = (q >= 0 && q < len) ? g[q] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // ---- lag sums S_d(base+t), d < L (every lane) -------------------------
    {
        float sr[L], si[L];
#pragma unroll
        for (int d = 0; d < L; ++d) { sr[d] = 0.f; si[d] = 0.f; }
        float2 win[L];
#pragma unroll
        for (int d = 0; d < L - 1; ++d) win[d + 1] = sg[t + d];
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int d = 0; d < L - 1; ++d) win[d] = win[d + 1];
            win[L - 1] = sg[t + k + L - 1];
            // products g[k] conj(g[k+d]) with g[k] = win[0]
#pragma unroll
            for (int d = 0; d < L; ++d) {
                sr[d] = fmaf(win[0].x, win[d].x, fmaf(win[0].y, win[d].y, sr[d]));
                si[d] = fmaf(win[0].y, win[d].x, fmaf(-win[0].x, win[d].y, si[d]));
            }
        }
#pragma unroll
        for (int d = 0; d < L; ++d) sS[d][t] = make_float2(sr[d], si[d]);
    }
    __syncthreads();

    const int p = p0 + t;
    const bool inside_line = (t < WPB) && (p < len);
    const bool valid = inside_line && (p - half >= 0) && (p - half + N <= len);

    float omega = __builtin_nanf("");
    unsigned flag = 0;
    int eig_its = 0, iters = 0, pfail = 0, counted = 0;

    if (valid) {
        // ---- covariance R_ij = S_{j-i}(s+i) (Eq. 4, up to the 1/K scale) ---
        Cov<L> R;
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int j = i; j < L; ++j) {
                const float2 v = sS[j - i][t + i];
                R.re[i][j] = v.x;
                R.im[i][j] = (i == j) ? 0.f : v.y;
            }
        Sym<L> T;
        build_T<L>(R, T);
        float tr = 0.f;
#pragma unroll
        for (int i = 0; i < L; ++i) tr += T.a[i][i];

        if (tr > 0.f && finitef(tr)) {
            counted = 1;
            const float itr = frcp(tr);
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
                for (int j = i; j < L; ++j) T.a[i][j] *= itr;

            // ---- signal subspace (Eq. 6-11) ------------------------------
            float v[L];
            if (JACOBI) top_eigvec_jacobi<L>(T, v, eig_its);
            else top_eigvec_tridiag<L>(T, v, eig_its);
            // u1 = Q v
            float ur[L], ui[L];
            constexpr float kS = 0.70710678118654752f;
#pragma unroll
            for (int i = 0; i < m; ++i) {
                ur[i] = kS * v[i];
                ui[i] = kS * v[o + i];
                ur[L - 1 - i] = kS * v[i];
                ui[L - 1 - i] = -kS * v[o + i];
            }
            if (L & 1) { ur[m] = v[m]; ui[m] = 0.f; }

            // ---- polynomial coefficients (Eq. 12-14) -------------------------
            // c_k = L delta_k - sum_i u[i] conj(u[i+k]),  k = 0..L-1
            float cr[L], ci[L];
#pragma unroll
            for (int k = 0; k < L; ++k) {
                float sr = 0.f, si = 0.f;
#pragma unroll
                for (int i = 0; i + k < L; ++i) {
                    sr = fmaf(ur[i], ur[i + k], fmaf(ui[i], ui[i + k], sr));
                    si = fmaf(ui[i], ur[i + k], fmaf(-ur[i], ui[i + k], si));
                }
                cr[k] = -sr;
                ci[k] = -si;
            }
            cr[0] += (float)L;
            ci[0] = 0.f;
            // ascending coefficients: a_j = c_{j-(L-1)}, c_{-k} = conj(c_k)
            float ar[n + 1], ai[n + 1];
#pragma unroll
            for (int j = 0; j <= n; ++j) {
                const int k = j - (L - 1);
                ar[j] = k >= 0 ? cr[k] : cr[-k];
                ai[j] = k >= 0 ? ci[k] : -ci[-k];
            }

            // ---- Aberth-Ehrlich in FP32 ---------------------------------------
            // frequency guess: u1[i+1]/u1[i] ~ e^{j w}, so c_1 ~ -((L-1)/L) e^{-j w}
            const float w0 = atan2f(ci[1], -cr[1]);
            float sw0, cw0;
            sincosf(w0, &sw0, &cw0);
            float zr[n], zi[n];
#pragma unroll
            for (int i = 0; i < n; ++i) {
                zr[i] = tmpl.re[i] * cw0 - tmpl.im[i] * sw0;
                zi[i] = tmpl.re[i] * sw0 + tmpl.im[i] * cw0;
            }
            for (int it = 0; it < kMaxRootIters; ++it) {
                ++iters;
                float Nr[n], Ni[n];
#pragma unroll
                for (int i = 0; i < n; ++i) {
                    const float m2 = zr[i] * zr[i] + zi[i] * zi[i];
                    const bool outer = m2 > 1.f;
                    const float im2 = frcp(m2);
                    const float er = outer ? zr[i] * im2 : zr[i];
                    const float ei = outer ? zi[i] * im2 : zi[i];
                    float Pr = ar[n], Pi = ai[n], Dr = 0.f, Di = 0.f;
#pragma unroll
                    for (int j = n - 1; j >= 0; --j) {
                        const float nDr = fmaf(Dr, er, fmaf(-Di, ei, Pr));
                        const float nDi = fmaf(Dr, ei, fmaf(Di, er, Pi));
                        const float nPr = fmaf(Pr, er, fmaf(-Pi, ei, ar[j]));
                        const float nPi = fmaf(Pr, ei, fmaf(Pi, er, ai[j]));
                        Dr = nDr; Di = nDi; Pr = nPr; Pi = nPi;
                    }
                    // inside:  N = P / D
                    // outside: N = z conj(P) / (n conj(P) - conj(D zeta))
                    const float Xr = Dr * er - Di * ei, Xi = Dr * ei + Di * er;
                    const float numr = outer ? (zr[i] * Pr + zi[i] * Pi) : Pr;
                    const float numi = outer ? (zi[i] * Pr - zr[i] * Pi) : Pi;
                    const float denr = outer ? ((float)n * Pr - Xr) : Dr;
                    const float deni = outer ? (-(float)n * Pi + Xi) : Di;
                    const float q = frcp(denr * denr + deni * deni);
                    Nr[i] = (numr * denr + numi * deni) * q;
                    Ni[i] = (numi * denr - numr * deni) * q;
                }
                float Sr[n], Si[n];
#pragma unroll
                for (int i = 0; i < n; ++i) { Sr[i] = 0.f; Si[i] = 0.f; }
#pragma unroll
                for (int i = 0; i < n; ++i)
#pragma unroll
                    for (int j = i + 1; j < n; ++j) {
                        const float dr = zr[i] - zr[j], di = zi[i] - zi[j];
                        const float q = frcp(dr * dr + di * di);
                        const float ir = dr * q, ii = -di * q;
                        Sr[i] += ir; Si[i] += ii;
                        Sr[j] -= ir; Si[j] -= ii;
                    }
                float maxstep = 0.f;
#pragma unroll
                for (int i = 0; i < n; ++i) {
                    // W = N / (1 - N S)
                    const float dr = 1.f - (Nr[i] * Sr[i] - Ni[i] * Si[i]);
                    const float di = -(Nr[i] * Si[i] + Ni[i] * Sr[i]);
                    const float q = frcp(dr * dr + di * di);
                    float Wr = (Nr[i] * dr + Ni[i] * di) * q;
                    float Wi = (Ni[i] * dr - Nr[i] * di) * q;
                    const bool ok = finitef(Wr) && finitef(Wi);
                    Wr = ok ? Wr : 0.f;
                    Wi = ok ? Wi : 0.f;
                    zr[i] -= Wr;
                    zi[i] -= Wi;
                    const float m2 = zr[i] * zr[i] + zi[i] * zi[i];
                    const float st = (Wr * Wr + Wi * Wi) * frcp(fmaxf(1.f, m2));
                    maxstep = fmaxf(maxstep, st);
                }
                if (!(maxstep >= kRootTol2)) break;
            }

            // ---- pair selection -----------------------------------------------
            float bestd = INFINITY, zsr = zr[0], zsi = zi[0];
            int sel = 0;
#pragma unroll
            for (int i = 0; i < n; ++i) {
                const float d = fabsf(fsqrt(zr[i] * zr[i] + zi[i] * zi[i]) - 1.f);
                const bool b = d < bestd;
                bestd = b ? d : bestd;
                zsr = b ? zr[i] : zsr;
                zsi = b ? zi[i] : zsi;
                sel = b ? i : sel;
            }
            const float sm2 = frcp(zsr * zsr + zsi * zsi);
            const float mir = zsr * sm2, mii = zsi * sm2;     // 1/conj(z_sel)
            float bestm = INFINITY, zmr = zr[0], zmi = zi[0];
#pragma unroll
            for (int i = 0; i < n; ++i) {
                const float dr = zr[i] - mir, di = zi[i] - mii;
                const float d = dr * dr + di * di;
                const bool b = (i != sel) && (d < bestm);
                bestm = b ? d : bestm;
                zmr = b ? zr[i] : zmr;
                zmi = b ? zi[i] : zmi;
            }

            // ---- FP64 polish of the quadratic factor z^2 - r z - s ----------
            double rr = (double)zsr + (double)zmr, ri = (double)zsi + (double)zmi;
            double s_r = -((double)zsr * zmr - (double)zsi * zmi);
            double s_i = -((double)zsr * zmi + (double)zsi * zmr);
            bool pok = true;
            double lastc = 0.0;
            for (int it = 0; it < kPolishIters; ++it) {
                double b1r = 0, b1i = 0, b2r = 0, b2i = 0;     // b_{k+1}, b_{k+2}
                double c1r = 0, c1i = 0, c2r = 0, c2i = 0;     // c_{k+1}, c_{k+2}
                double B0r = 0, B0i = 0, B1r = 0, B1i = 0;
                double C1r = 0, C1i = 0, C2r = 0, C2i = 0, C3r = 0, C3i = 0;
#pragma unroll
                for (int k = n; k >= 0; --k) {
                    const double bkr = (double)ar[k] + (rr * b1r - ri * b1i) + (s_r * b2r - s_i * b2i);
                    const double bki = (double)ai[k] + (rr * b1i + ri * b1r) + (s_r * b2i + s_i * b2r);
                    if (k == 0) { B0r = bkr; B0i = bki; }
                    if (k == 1) { B1r = bkr; B1i = bki; }
                    if (k >= 1) {
                        const double ckr = bkr + (rr * c1r - ri * c1i) + (s_r * c2r - s_i * c2i);
                        const double cki = bki + (rr * c1i + ri * c1r) + (s_r * c2i + s_i * c2r);
                        if (k == 1) { C1r = ckr; C1i = cki; }
                        if (k == 2) { C2r = ckr; C2i = cki; }
                        if (k == 3) { C3r = ckr; C3i = cki; }
                        c2r = c1r; c2i = c1i; c1r = ckr; c1i = cki;
                    }
                    b2r = b1r; b2i = b1i; b1r = bkr; b1i = bki;
                }
                // [C2 C3; C1 C2] [dr; ds] = -[B1; B0]
                const double detr = (C2r * C2r - C2i * C2i) - (C1r * C3r - C1i * C3i);
                const double deti = 2.0 * C2r * C2i - (C1r * C3i + C1i * C3r);
                const double nr1 = -(B1r * C2r - B1i * C2i) + (B0r * C3r - B0i * C3i);
                const double ni1 = -(B1r * C2i + B1i * C2r) + (B0r * C3i + B0i * C3r);
                const double nr2 = -(B0r * C2r - B0i * C2i) + (B1r * C1r - B1i * C1i);
                const double ni2 = -(B0r * C2i + B0i * C2r) + (B1r * C1i + B1i * C1r);
                const double id = 1.0 / (detr * detr + deti * deti);
                const double drr = (nr1 * detr + ni1 * deti) * id;
                const double dri = (ni1 * detr - nr1 * deti) * id;
                const double dsr = (nr2 * detr + ni2 * deti) * id;
                const double dsi = (ni2 * detr - nr2 * deti) * id;
                if (!(__builtin_isfinite(drr) && __builtin_isfinite(dri) &&
                      __builtin_isfinite(dsr) && __builtin_isfinite(dsi))) {
                    pok = false;
                    break;
                }
                rr += drr; ri += dri; s_r += dsr; s_i += dsi;
                lastc = fabs(drr) + fabs(dri);
            }
            const double rmag = fabs(rr) + fabs(ri);
            if (!(pok && lastc <= 1e-6 * rmag)) {
                pok = false;
                rr = (double)zsr + (double)zmr;
                ri = (double)zsi + (double)zmi;
            }
            pfail = pok ? 0 : 1;
            if (!pok) flag |= BM_FLAG_NO_POLISH;
            omega = atan2f((float)ri, (float)rr);
        } else {
            flag |= BM_FLAG_UNDEFINED;
        }
    } else {
        flag |= BM_FLAG_UNDEFINED;
    }

    if (inside_line) {
        const int64_t oidx = (int64_t)p * J.out_es + (int64_t)line * J.out_ls;
        J.out[oidx] = omega;
        if (J.flags) {
            const uint8_t f = (uint8_t)(flag << J.flag_shift);
            if (J.flag_or) J.flags[oidx] |= f;
            else J.flags[oidx] = f;
        }
    }
    ls.counted += counted;
    ls.eig_its += eig_its;
    ls.iters += iters;
    ls.pfail += pfail;
}

// Grid-stride loop over the work items of every job of one L: item w is
// block (w - prefix[j]) of job j, i.e. line (w - prefix[j]) / bpl and window
// block (w - prefix[j]) % bpl.  A grid of one block per item runs each item
// once; a smaller (persistent) grid walks the list.
template <int L, int BLOCK, bool STATS, bool JACOBI>
__global__ __launch_bounds__(BLOCK) void rootmusic_kernel(RmBatch B) {
    constexpr int WPB = BLOCK - (L - 1);
    __shared__ float2 sg[BLOCK + kMaxN];
    __shared__ float2 sS[L][BLOCK];
    LaneStats ls;
    for (int w = blockIdx.x; w < B.total; w += gridDim.x) {
        int lo = 0, hi = B.njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B.prefix[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const RmJob J = B.jobs[lo];
        const int local = w - B.prefix[lo];
        const int line = local / J.bpl;
        const int bx = local - line * J.bpl;
        rootmusic_block<L, BLOCK, JACOBI>(J, line, bx * WPB, sg, sS, B.tmpl, ls);
        __syncthreads();
    }
    if (STATS) {
        unsigned long long a0 = ls.counted, a1 = ls.eig_its, a2 = ls.iters, a3 = ls.pfail;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off);
            a1 += __shfl_xor(a1, off);
            a2 += __shfl_xor(a2, off);
            a3 += __shfl_xor(a3, off);
        }
        if ((threadIdx.x & 63) == 0) {
            // spread the counters over kStatSlots slots to avoid one hot address
            unsigned long long* sl = B.stats + 4 * ((blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6)) % kStatSlots);
            atomicAdd(sl + 0, a0);
            atomicAdd(sl + 1, a1);
            atomicAdd(sl + 2, a2);
            atomicAdd(sl + 3, a3);
        }
    }
}

template <int L, int BLOCK, bool JACOBI>
hipError_t launch_LBJ(const RmBatch& b, int grid, hipStream_t s) {
    if (b.stats)
        hipLaunchKernelGGL((rootmusic_kernel<L, BLOCK, true, JACOBI>), dim3(grid), dim3(BLOCK), 0, s, b);
    else
        hipLaunchKernelGGL((rootmusic_kernel<L, BLOCK, false, JACOBI>), dim3(grid), dim3(BLOCK), 0, s, b);
    return hipGetLastError();
}

template <int L>
hipError_t launch_L(const RmBatch& b, int block, int grid, hipStream_t s) {
    if (block == 128)
        return b.jacobi ? launch_LBJ<L, 128, true>(b, grid, s) : launch_LBJ<L, 128, false>(b, grid, s);
    return b.jacobi ? launch_LBJ<L, 256, true>(b, grid, s) : launch_LBJ<L, 256, false>(b, grid, s);
}

}  // namespace

int rootmusic_windows_per_block(int L, int block) { return block - (L - 1); }

hipError_t launch_rootmusic(int L, const RmBatch& b, int block, int grid, hipStream_t s) {
    if (b.total <= 0 || b.njobs <= 0) return hipSuccess;
    if (block != 128 && block != 256) return hipErrorInvalidValue;
    if (grid <= 0 || grid > b.total) grid = b.total;
    switch (L) {
        case 2: return launch_L<2>(b, block, grid, s);
        case 3: return launch_L<3>(b, block, grid, s);
        case 4: return launch_L<4>(b, block, grid, s);
        case 5: return launch_L<5>(b, block, grid, s);
        case 6: return launch_L<6>(b, block, grid, s);
        case 7: return launch_L<7>(b, block, grid, s);
        case 8: return launch_L<8>(b, block, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bm
