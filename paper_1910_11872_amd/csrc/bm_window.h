// Per-window arithmetic shared by the root-MUSIC kernels: covariance to the
// real symmetric T, its top eigenvector, the root-MUSIC polynomial, the
// simultaneous root iteration, pair selection and the quadratic-factor polish.
// Device code only; included by the kernel translation units.
#pragma once

#include "bm_internal.h"

#include <cmath>

namespace bm {


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
constexpr int kCertIters32 = 6;   // at most this many FP32 Newton steps towards the signal root
constexpr int kCertIters = 8;     // then at most this many FP64 Newton steps before the pair certificate
// Newton with the mate divided out converges quadratically once the error is
// small against the distance |z - 1/conj z| to the mate: iterating stops at
// the first step below 1e-4 |z| and below 1e-2 |z - 1/conj z| (the error
// after it is then of order 1e-8 |z| or less, under the FP32 resolution of
// omega; without the second bound, windows whose pair lies within 1e-4 of
// the circle stopped with errors up to 2e-5 in numpy trials), and a root that
// has not met both within the step limit is not trusted.  With such a root
// the division by the pair's factor leaves a remainder of order 1e-7 of the
// coefficients' size (1e-6 at most in the same trials over L, N and SNR), so
// the remainder test allows 1e-5; a lone root on the circle leaves O(1).
constexpr double kPairStepTol = 1e-4;
constexpr double kPairMateTol = 1e-2;
constexpr double kCertRemTol = 1e-5;
// The same test with the division in FP32 (line windows of L <= 8): its own
// rounding leaves up to 2.2e-5 of the coefficients' size at L = 8 (numpy
// trials over 0-30 dB, N = 16-32; 1e-6 at the median), against remainders
// of the roots that pass in FP64 below 1e-5 and O(1e-2 .. 1) for one that is
// not a root, so FP32 allows 1e-4.
constexpr float kCertRemTol32 = 1e-4f;
constexpr int kNewtonIters = BM_NEWTON_ITERS;
constexpr int kInverseIters = BM_INVERSE_ITERS;
// The one-dimensional signal subspace of Eq. 6-11 needs lambda_1 to stand
// apart: a window with lambda_2 >= lambda_1 / (1 + kDegenRel) has no
// determined signal eigenvector (two tones of equal power, say) and gets
// NaN with BM_FLAG_DEGENERATE.  1e-5 is above the resolution of eigenvalues
// computed in FP32 (a few 1e-7 of the trace).
constexpr float kDegenRel = 1e-5f;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

// Symmetric L x L matrix, upper triangle stored (compile-time indices only).
template <int L>
struct Sym {
    float a[L][L];
    __device__ __forceinline__ float& at(int i, int j) { return i <= j ? a[i][j] : a[j][i]; }
    __device__ __forceinline__ float at(int i, int j) const { return i <= j ? a[i][j] : a[j][i]; }
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

// Number of eigenvalues of the symmetric tridiagonal matrix (diagonal d,
// squared off-diagonal e2) above p: the sign changes of the leading principal
// minors of p I - T (Sturm).
template <int L>
__device__ __forceinline__ int sturm_above(const float (&d)[L], const float (&e2)[L], float p) {
    float q0 = 1.f, q1 = p - d[0];
    int changes = q1 < 0.f ? 1 : 0;
#pragma unroll
    for (int i = 1; i < L; ++i) {
        const float q2 = fmaf(p - d[i], q1, -e2[i - 1] * q0);
        changes += ((q2 < 0.f) != (q1 < 0.f)) ? 1 : 0;
        q0 = q1;
        q1 = q2;
    }
    return changes;
}

// Eigenvector of the largest eigenvalue of the trace-normalised symmetric T:
// Householder tridiagonalisation, Newton from above on det(xI - T_tri),
// shifted inverse iteration on the tridiagonal matrix, back-transformation.
template <int L>
__device__ __forceinline__ void top_eigvec_tridiag(Sym<L>& T, float (&v)[L], int& its, float& lam, bool& degen) {
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
    // start above the largest eigenvalue: T is positive semidefinite with
    // trace 1, so lambda_1 <= 1; Gerschgorin's bound; and the trace bound of
    // Wolkowicz and Styan (1980), lambda_1 <= mu + s sqrt(L - 1) with mu the
    // mean eigenvalue and s^2 their variance, here sum (d_i - mu)^2 / L +
    // 2 sum e_i^2 / L from the tridiagonal form (sums of squares, so no
    // cancellation; the similarity keeps tr T^2).  The last is near lambda_1
    // whenever the other eigenvalues are alike, the usual signal-plus-noise
    // spectrum, and saves most Newton steps.
    float g = 0.f, mu = 0.f;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        float r = d[i];
        if (i > 0) r += fabsf(e[i - 1]);
        if (i < L - 1) r += fabsf(e[i]);
        g = fmaxf(g, r);
        mu += d[i];
    }
    mu *= 1.f / (float)L;
    float var = 0.f;
#pragma unroll
    for (int i = 0; i < L; ++i) var = fmaf(d[i] - mu, d[i] - mu, var);
#pragma unroll
    for (int i = 0; i < L - 1; ++i) var = fmaf(2.f * e[i], e[i], var);
    const float ws = mu + fsqrt(var * ((float)(L - 1) / (float)L));
    float x = fminf(fminf(g, 1.f), ws) * 1.00001f + 1e-30f;
    float last_step = x;                  // no step taken: lambda_1 >= 0 is all that is known
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
        last_step = step;
        // quadratic convergence: a step below 1e-5 x leaves an error of order 1e-10 x
        if (!(fabsf(step) > 1e-5f * x)) break;
    }
    lam = x;
    // Degenerate signal subspace?  Every eigenvalue is below the Newton iterate,
    // so its step at x was q/q' = 1 / sum_i 1/(x - lambda_i) >= (x - lambda_1)/L:
    // lambda_1 >= lo = x_new - (L - 1) |last step|, a bound that also holds when
    // the iteration stopped on its step limit short of a (nearly) double top
    // eigenvalue; lambda_1 <= hi = x.  T has trace 1 and no negative
    // eigenvalue, so lambda_2 <= 1 - lambda_1, and lo (2 + d) > 1 + d already
    // proves lambda_2 < lambda_1 / (1 + d).  Otherwise Sturm counts decide: at
    // most one eigenvalue above lo / (1 + d) proves the gap, two above
    // hi / (1 + d) disprove it, and in between bisection narrows [lo, hi]
    // around lambda_1 until one of the two holds.
    degen = false;
    float lo = x - (float)(L - 1) * fabsf(last_step), hi = x;
    if (!(lo * (2.f + kDegenRel) > 1.f + kDegenRel)) {
        constexpr float kInv = 1.f / (1.f + kDegenRel);
        degen = true;                                 // if 24 halvings cannot decide
        for (int b = 0; b < 24; ++b) {
            if (sturm_above<L>(d, e2, lo * kInv) <= 1) { degen = false; break; }
            if (sturm_above<L>(d, e2, hi * kInv) >= 2) break;
            const float mid = 0.5f * (lo + hi);
            if (sturm_above<L>(d, e2, mid) >= 1) lo = mid;
            else hi = mid;
        }
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
__device__ __forceinline__ void top_eigvec_jacobi(Sym<L>& T, float (&v)[L], int& sweeps, float& lam, bool& degen) {
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
    float best = T.a[0][0], second = -INFINITY;
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] = V[i][0];
#pragma unroll
    for (int k = 1; k < L; ++k) {
        const bool b = T.a[k][k] > best;
        second = b ? best : fmaxf(second, T.a[k][k]);
        best = b ? T.a[k][k] : best;
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = b ? V[i][k] : v[i];
    }
    lam = best;
    degen = second * (1.f + kDegenRel) >= best;
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

// Store omega (and the flag nibble) of pixel p of `line` of job J.
__device__ __forceinline__ void store_omega(const RmJob& J, int line, int p, float omega, unsigned flag) {
    J.out[(int64_t)p * J.out_es + (int64_t)line * J.out_ls] = omega;
    if (J.flags) {
        const int64_t fidx = (int64_t)p * J.flag_es + (int64_t)line * J.flag_ls;
        const uint8_t f = (uint8_t)(flag << J.flag_shift);
        if (J.flag_or) J.flags[fidx] |= f;
        else J.flags[fidx] = f;
    }
}

// Counters a lane accumulates over the windows it owns.
struct LaneStats {
    int counted = 0, eig_its = 0, iters = 0, pfail = 0, accepted = 0, rejected = 0, pair_its = 0, pair_its32 = 0,
        power = 0;
};

// u1 = Q v for the unitary transform used by build_T.
template <int L>
__device__ __forceinline__ void signal_vector(const float (&v)[L], float (&ur)[L], float (&ui)[L]) {
    constexpr int m = L / 2;
    constexpr int o = L - m;
    constexpr float kS = 0.70710678118654752f;
#pragma unroll
    for (int i = 0; i < m; ++i) {
        ur[i] = kS * v[i];
        ui[i] = kS * v[o + i];
        ur[L - 1 - i] = kS * v[i];
        ui[L - 1 - i] = -kS * v[o + i];
    }
    if (L & 1) { ur[m] = v[m]; ui[m] = 0.f; }
}

// Root-MUSIC polynomial of Eq. 12 from the signal vector (C = I - u1 u1^H):
// c_k = L delta_k - sum_i u[i] conj(u[i+k]); ascending a_j = c_{j-(L-1)},
// c_{-k} = conj(c_k).
template <int L>
__device__ __forceinline__ void poly_coeffs(const float (&ur)[L], const float (&ui)[L], float (&ar)[2 * L - 1],
                                            float (&ai)[2 * L - 1]) {
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
#pragma unroll
    for (int j = 0; j <= 2 * L - 2; ++j) {
        const int k = j - (L - 1);
        ar[j] = k >= 0 ? cr[k] : cr[-k];
        ai[j] = k >= 0 ? ci[k] : -ci[-k];
    }
}

// Newton iterations on the quadratic factor z^2 - r z - s of the polynomial
// (complex Bairstow), in precision T: at most `iters` steps, fewer once a
// step is below tol |r|.  Returns false when a step is not finite; `lastc`
// receives |dr| of the last step; *its (optional) counts the steps.
template <typename Tp, int n>
__device__ __forceinline__ bool bairstow(const float (&ar)[n + 1], const float (&ai)[n + 1], Tp& rr, Tp& ri, Tp& s_r,
                                         Tp& s_i, int iters, Tp& lastc, Tp tol = 0, int* its = nullptr) {
    for (int it = 0; it < iters; ++it) {
        if (its) ++*its;
        Tp b1r = 0, b1i = 0, b2r = 0, b2i = 0;     // b_{k+1}, b_{k+2}
        Tp c1r = 0, c1i = 0, c2r = 0, c2i = 0;     // c_{k+1}, c_{k+2}
        Tp B0r = 0, B0i = 0, B1r = 0, B1i = 0;
        Tp C1r = 0, C1i = 0, C2r = 0, C2i = 0, C3r = 0, C3i = 0;
#pragma unroll
        for (int k = n; k >= 0; --k) {
            const Tp tr = fma(s_r, b2r, fma(-s_i, b2i, (Tp)ar[k]));
            const Tp ti = fma(s_r, b2i, fma(s_i, b2r, (Tp)ai[k]));
            const Tp bkr = fma(rr, b1r, fma(-ri, b1i, tr));
            const Tp bki = fma(rr, b1i, fma(ri, b1r, ti));
            if (k == 0) { B0r = bkr; B0i = bki; }
            if (k == 1) { B1r = bkr; B1i = bki; }
            if (k >= 1) {
                const Tp ur = fma(s_r, c2r, fma(-s_i, c2i, bkr));
                const Tp ui = fma(s_r, c2i, fma(s_i, c2r, bki));
                const Tp ckr = fma(rr, c1r, fma(-ri, c1i, ur));
                const Tp cki = fma(rr, c1i, fma(ri, c1r, ui));
                if (k == 1) { C1r = ckr; C1i = cki; }
                if (k == 2) { C2r = ckr; C2i = cki; }
                if (k == 3) { C3r = ckr; C3i = cki; }
                c2r = c1r; c2i = c1i; c1r = ckr; c1i = cki;
            }
            b2r = b1r; b2i = b1i; b1r = bkr; b1i = bki;
        }
        // [C2 C3; C1 C2] [dr; ds] = -[B1; B0]
        const Tp detr = (C2r * C2r - C2i * C2i) - (C1r * C3r - C1i * C3i);
        const Tp deti = (Tp)2 * C2r * C2i - (C1r * C3i + C1i * C3r);
        const Tp nr1 = -(B1r * C2r - B1i * C2i) + (B0r * C3r - B0i * C3i);
        const Tp ni1 = -(B1r * C2i + B1i * C2r) + (B0r * C3i + B0i * C3r);
        const Tp nr2 = -(B0r * C2r - B0i * C2i) + (B1r * C1r - B1i * C1i);
        const Tp ni2 = -(B0r * C2i + B0i * C2r) + (B1r * C1i + B1i * C1r);
        const Tp id = (Tp)1 / (detr * detr + deti * deti);
        const Tp drr = (nr1 * detr + ni1 * deti) * id;
        const Tp dri = (ni1 * detr - nr1 * deti) * id;
        const Tp dsr = (nr2 * detr + ni2 * deti) * id;
        const Tp dsi = (ni2 * detr - nr2 * deti) * id;
        if (!(__builtin_isfinite(drr) && __builtin_isfinite(dri) && __builtin_isfinite(dsr) &&
              __builtin_isfinite(dsi)))
            return false;
        rr += drr; ri += dri; s_r += dsr; s_i += dsi;
        lastc = (drr < 0 ? -drr : drr) + (dri < 0 ? -dri : dri);
        if (lastc <= tol * ((rr < 0 ? -rr : rr) + (ri < 0 ? -ri : ri))) break;
    }
    return true;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rcp_est(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_est(double x) { return __builtin_amdgcn_rcp(x); }

// Number of zeros of f(z) = sum_i (fr[i] + j fi[i]) z^i (formal degree m)
// strictly inside the unit disk, by the Schur-Cohn recursion
//     T f = conj(a_0) f - a_m f*,   f*(z) = z^m conj(f(1/conj(z))),
// whose constant term gamma = |a_0|^2 - |a_m|^2 decides the count: when
// gamma > 0, T f has as many zeros inside as f; when gamma < 0, as many as
// f*, i.e. m minus those of f (Henrici, Applied and Computational Complex
// Analysis I, Sec. 6.8).  Returns -1 when some |gamma| is not above
// `margin` (|a_0|^2 + |a_m|^2), which is the case of a zero on or very near
// the unit circle.  From the second step on a_0 is that real gamma, which
// takes a quarter of the products out of every coefficient update.
template <int m, typename T>
__device__ __forceinline__ int schur_cohn_count(T (&fr)[m + 1], T (&fi)[m + 1], T margin) {
    unsigned neg = 0;
    bool ok = true;
#pragma unroll
    for (int d = m; d >= 1; --d) {
        const T a0r = fr[0], adr = fr[d], adi = fi[d];
        const T a0i = d == m ? fi[0] : (T)0;
        const T p0 = fma_t(a0r, a0r, a0i * a0i), pd = fma_t(adr, adr, adi * adi);
        const T g = p0 - pd;
        ok = ok && ((g < (T)0 ? -g : g) > margin * (p0 + pd));
        neg |= (g < (T)0 ? 1u : 0u) << d;
        // any positive scale keeps the signs that are read; folded into a0 and a_d
        const T sc = rcp_est(p0 + pd);
        const T br = a0r * sc, cr = adr * sc, ci = adi * sc;
        // new_i = conj(a0) a_i - a_d conj(a_{d-i}) (times sc), in place over the pairs (i, d-i)
        if (d == m) {
            const T bi = a0i * sc;
#pragma unroll
            for (int i = 1; 2 * i <= d; ++i) {
                const int k = d - i;
                const T xr = fr[i], xi = fi[i], yr = fr[k], yi = fi[k];
                fr[i] = fma_t(br, xr, fma_t(bi, xi, -fma_t(cr, yr, ci * yi)));
                fi[i] = fma_t(br, xi, fma_t(-bi, xr, -fma_t(ci, yr, -cr * yi)));
                fr[k] = fma_t(br, yr, fma_t(bi, yi, -fma_t(cr, xr, ci * xi)));
                fi[k] = fma_t(br, yi, fma_t(-bi, yr, -fma_t(ci, xr, -cr * xi)));
            }
        } else {
#pragma unroll
            for (int i = 1; 2 * i < d; ++i) {
                const int k = d - i;
                const T xr = fr[i], xi = fi[i], yr = fr[k], yi = fi[k];
                fr[i] = fma_t(br, xr, -fma_t(cr, yr, ci * yi));
                fi[i] = fma_t(br, xi, -fma_t(ci, yr, -cr * yi));
                fr[k] = fma_t(br, yr, -fma_t(cr, xr, ci * xi));
                fi[k] = fma_t(br, yi, -fma_t(ci, xr, -cr * xi));
            }
            if (d % 2 == 0) {                         // the middle coefficient is its own partner
                const int i = d / 2;
                const T xr = fr[i], xi = fi[i];
                fr[i] = fma_t(br, xr, -fma_t(cr, xr, ci * xi));
                fi[i] = fma_t(br, xi, -fma_t(ci, xr, -cr * xi));
            }
        }
        fr[0] = g * sc;
        fi[0] = (T)0;
    }
    int count = 0;
#pragma unroll
    for (int d = 1; d <= m; ++d)
        if ((neg >> d) & 1u) count = d - count;
    return ok ? count : -1;
}

template <int m>
__device__ __forceinline__ int zeros_inside_unit_disk(double (&fr)[m + 1], double (&fi)[m + 1]) {
    return schur_cohn_count<m, double>(fr, fi, 1e-9);
}

constexpr double kCertMargin = 1e-6;  // relative radius margin of the nearest-pair certificate

__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * fma(-x, r, 2.0);              // two Newton steps on the hardware estimate
    return r * fma(-x, r, 2.0);
}

// z^N for N >= 0 by squaring (N is a compile-time constant).
template <int N, typename T>
__device__ __forceinline__ void cpow(T xr, T xi, T& pr, T& pi) {
    if constexpr (N == 0) {
        pr = (T)1;
        pi = (T)0;
    } else if constexpr (N == 1) {
        pr = xr;
        pi = xi;
    } else if constexpr (N % 2 == 0) {
        T hr, hi;
        cpow<N / 2, T>(xr, xi, hr, hi);
        pr = fma_t(hr, hr, -hi * hi);
        pi = (T)2 * hr * hi;
    } else {
        T hr, hi;
        cpow<N - 1, T>(xr, xi, hr, hi);
        pr = fma_t(hr, xr, -hi * xi);
        pi = fma_t(hr, xi, hi * xr);
    }
}

// The root-MUSIC polynomial and its derivative at z from the signal vector
// itself.  With u conjugate-symmetric (u_{L-1-i} = conj(u_i), u = Q v) the
// diagonal sums of u u^H are the coefficients of B(z)^2, B(z) = sum_i
// conj(u_i) z^i, so P(z) = L z^{L-1} - B(z)^2 and P'(z) = L (L-1) z^{L-2} -
// 2 B(z) B'(z): Horner over the L coefficients of B instead of the 2L - 1 of
// P (the same polynomial; its rounded FP32 coefficients serve the
// certificate and the all-roots path).
template <int L, typename T>
__device__ __forceinline__ void music_poly_eval(const float (&ur)[L], const float (&ui)[L], T xr, T xi, T& Pr, T& Pi,
                                                T& Dr, T& Di) {
    T Br = (T)ur[L - 1], Bi = -(T)ui[L - 1], Er = (T)0, Ei = (T)0;   // B and B'
#pragma unroll
    for (int j = L - 2; j >= 0; --j) {
        const T nEr = fma_t(Er, xr, fma_t(-Ei, xi, Br)), nEi = fma_t(Er, xi, fma_t(Ei, xr, Bi));
        const T nBr = fma_t(Br, xr, fma_t(-Bi, xi, (T)ur[j]));
        const T nBi = fma_t(Br, xi, fma_t(Bi, xr, -(T)ui[j]));
        Er = nEr; Ei = nEi; Br = nBr; Bi = nBi;
    }
    T qr, qi;                                          // z^{L-2}
    cpow<L - 2, T>(xr, xi, qr, qi);
    const T wr = fma_t(qr, xr, -qi * xi), wi = fma_t(qr, xi, qi * xr);   // z^{L-1}
    // P = L z^{L-1} - B^2,  P' = L (L-1) z^{L-2} - 2 B B'
    Pr = fma_t((T)L, wr, -fma_t(Br, Br, -Bi * Bi));
    Pi = fma_t((T)L, wi, -(T)2 * Br * Bi);
    Dr = fma_t((T)(L * (L - 1)), qr, -(T)2 * fma_t(Br, Er, -Bi * Ei));
    Di = fma_t((T)(L * (L - 1)), qi, -(T)2 * fma_t(Br, Ei, Bi * Er));
}

// Newton's iteration for a root z of the root-MUSIC polynomial (paper
// Eq. 12) whose mate 1/conj(z) is a root as well -- every root of this
// polynomial has its mate, c_{-k} = conj(c_k) -- with the mate divided out
// (Maehly's correction), which keeps the convergence quadratic although the
// two roots nearly coincide near the unit circle:
//   z <- z - P(z) / (P'(z) - P(z) / (z - 1/conj(z)))
// FP32 approach to the same root: at most `iters` steps of the iteration
// above in FP32, ending at the first step below 1e-3 |z|.  Per-phase counters
// of this kernel show its FP64 phases taking about twice the cycles per
// instruction of its FP32 phases, and from the point reached here the FP64
// steps below stop after about one step (numpy trials: FP64 steps of a
// wave's slowest lane 3.4 -> 1.3 at 10 dB, plus 2.5 FP32 steps).  A
// non-finite step leaves z at the last finite iterate.
template <int L>
__device__ __forceinline__ void pair_newton32(const float (&ur)[L], const float (&ui)[L], double& zr, double& zi,
                                              int iters, int* its) {
    float xr = (float)zr, xi = (float)zi;
    for (int it = 0; it < iters; ++it) {
        if (its) ++*its;
        float Pr, Pi, Dr, Di;
        music_poly_eval<L, float>(ur, ui, xr, xi, Pr, Pi, Dr, Di);
        const float f = 1.f - frcp(fmaf(xr, xr, xi * xi));
        const float ur_ = xr * f, ui_ = xi * f;
        const float nr = fmaf(Pr, ur_, -Pi * ui_), ni = fmaf(Pr, ui_, Pi * ur_);
        const float dr = fmaf(Dr, ur_, -Di * ui_) - Pr, di = fmaf(Dr, ui_, Di * ur_) - Pi;
        const float q = frcp(fmaf(dr, dr, di * di));
        const float sr = fmaf(nr, dr, ni * di) * q, si = fmaf(ni, dr, -nr * di) * q;
        if (!(finitef(sr) && finitef(si))) break;
        xr -= sr;
        xi -= si;
        if (fabsf(sr) + fabsf(si) <= 1e-3f * (fabsf(xr) + fabsf(xi))) break;
    }
    if (finitef(xr) && finitef(xi)) {
        zr = (double)xr;
        zi = (double)xi;
    }
}

// At most `iters` steps; true once a step meets the stop rule above, false
// when none did or a step is not finite.
template <int L>
__device__ __forceinline__ bool pair_newton(const float (&ur)[L], const float (&ui)[L], double& zr, double& zi,
                                            int iters, int* its) {
    for (int it = 0; it < iters; ++it) {
        if (its) ++*its;
        double Pr64, Pi64, Dr64, Di64;
        music_poly_eval<L, double>(ur, ui, zr, zi, Pr64, Pi64, Dr64, Di64);
        // The residual P (and P') needs FP64; the step formed from them does not: its
        // relative rounding in FP32 (1e-7) only scales the error left after the step,
        // and z itself is updated in FP64.  u = z - 1/conj(z) = z (|z|^2 - 1)/|z|^2,
        // the difference taken in FP64; step = P u / (P' u - P).
        const double m2 = fma(zr, zr, zi * zi);
        const float m2f = (float)m2;
        const float f = (float)(m2 - 1.0) * frcp(m2f);
        const float xr = (float)zr, xi = (float)zi;
        const float ur_ = xr * f, ui_ = xi * f;
        const float Pr = (float)Pr64, Pi = (float)Pi64, Dr = (float)Dr64, Di = (float)Di64;
        const float nr = fmaf(Pr, ur_, -Pi * ui_), ni = fmaf(Pr, ui_, Pi * ur_);
        const float dr = fmaf(Dr, ur_, -Di * ui_) - Pr, di = fmaf(Dr, ui_, Di * ur_) - Pi;
        const float q = frcp(fmaf(dr, dr, di * di));
        const float sr = fmaf(nr, dr, ni * di) * q, si = fmaf(ni, dr, -nr * di) * q;
        if (!(finitef(sr) && finitef(si))) return false;
        zr -= (double)sr;
        zi -= (double)si;
        const float st = fabsf(sr) + fabsf(si);
        if (st <= (float)kPairStepTol * (float)(fabs(zr) + fabs(zi)) && st <= (float)kPairMateTol * (fabsf(ur_) + fabsf(ui_)))
            return true;
    }
    return false;
}

// The same count in FP32, decided only when every |gamma| exceeds
// kCount32Margin of |a_0|^2 + |a_d|^2: -1 otherwise.  In numpy trials of the
// certificate's polynomials (L = 4, 6, 8 at 0-30 dB, radius 0.8) the FP32
// gamma of the windows so decided stayed within 1e-4 of the FP64 value, two
// orders under the margin, and the counts agreed on every window.
constexpr float kCount32Margin = 1e-2f;

template <int m>
__device__ __forceinline__ int zeros_inside_unit_disk32(float (&fr)[m + 1], float (&fi)[m + 1]) {
    return schur_cohn_count<m, float>(fr, fi, kCount32Margin);
}

// Quotient q_0 .. q_{n-2} of P (degree n) by z^2 - r z - s, in FP64,
// stored as Q; returns the size |b_1| + |b_0| of the remainder b_1 (z - r) + b_0.
template <int n, typename Q>
__device__ __forceinline__ double pair_quotient(const float (&ar)[n + 1], const float (&ai)[n + 1], double rr, double ri,
                                                double s_r, double s_i, Q (&fr)[n - 1], Q (&fi)[n - 1]) {
    double b1r = 0.0, b1i = 0.0, b2r = 0.0, b2i = 0.0;
#pragma unroll
    for (int k = n; k >= 0; --k) {
        // the s b_{k+2} part first: only two dependent FMAs per step wait for b_{k+1}
        const double tr = fma(s_r, b2r, fma(-s_i, b2i, (double)ar[k]));
        const double ti = fma(s_r, b2i, fma(s_i, b2r, (double)ai[k]));
        const double bkr = fma(rr, b1r, fma(-ri, b1i, tr));
        const double bki = fma(rr, b1i, fma(ri, b1r, ti));
        if (k >= 2) {
            fr[k - 2] = (Q)bkr;
            fi[k - 2] = (Q)bki;
        }
        b2r = b1r; b2i = b1i; b1r = bkr; b1i = bki;
    }
    // here b2 = b_1 and b1 = b_0
    return fabs(b2r) + fabs(b2i) + fabs(b1r) + fabs(b1i);
}

// The same division in FP32 (the pair's factor rounded to FP32), for the FP32 root count.
template <int n>
__device__ __forceinline__ float pair_quotient32(const float (&ar)[n + 1], const float (&ai)[n + 1], float rr, float ri,
                                                 float s_r, float s_i, float (&fr)[n - 1], float (&fi)[n - 1]) {
    float b1r = 0.f, b1i = 0.f, b2r = 0.f, b2i = 0.f;
#pragma unroll
    for (int k = n; k >= 0; --k) {
        const float tr = fmaf(s_r, b2r, fmaf(-s_i, b2i, ar[k]));
        const float ti = fmaf(s_r, b2i, fmaf(s_i, b2r, ai[k]));
        const float bkr = fmaf(rr, b1r, fmaf(-ri, b1i, tr));
        const float bki = fmaf(rr, b1i, fmaf(ri, b1r, ti));
        if (k >= 2) {
            fr[k - 2] = bkr;
            fi[k - 2] = bki;
        }
        b2r = b1r; b2i = b1i; b1r = bkr; b1i = bki;
    }
    return fabsf(b2r) + fabsf(b2i) + fabsf(b1r) + fabsf(b1i);
}

// Q is self-inversive (P and the pair's factor are), q_{m-k} = conj(q_k) q_m / conj(q_0)
// with m = 2L - 4, so the first Schur-Cohn step on f(z) = Q(rho z) has the closed form
// T f = conj(q_0) sum_{k<m} q_k (rho^k - rho^{2m-k}) z^k, with a positive constant term:
// f and T f have equally many zeros inside the unit disk.  rho^k - rho^{2m-k} =
// rho^k (1 - rho^{2(m-k)}): ascending powers first, then the factor descending.
// The conj(q_0) factor does not move zeros and is left out.
template <int m, typename T>
__device__ __forceinline__ void first_schur_step(const T (&fr)[m + 1], const T (&fi)[m + 1], T rho, T (&gr)[m],
                                                 T (&gi)[m]) {
    T pk = (T)1;
#pragma unroll
    for (int k = 0; k < m; ++k) {
        gr[k] = pk;
        pk *= rho;
    }
    const T rho2 = rho * rho;
    T a = rho2;                                       // rho^{2(m-k)} at k = m - 1
#pragma unroll
    for (int k = m - 1; k >= 0; --k) {
        const T w = gr[k] * ((T)1 - a);
        gr[k] = fr[k] * w;
        gi[k] = fi[k] * w;
        a *= rho2;
    }
}

// The L - 2 inner roots of the quotient (FP64 coefficients) strictly inside
// |z| < |z_in| (1 - margin), by Schur-Cohn on Q(rho z).
template <int L>
__device__ __forceinline__ bool inner_roots_inside(const double (&fr)[2 * L - 3], const double (&fi)[2 * L - 3],
                                                   double rin) {
    constexpr int m = 2 * L - 4;
    double gr[m], gi[m];
    first_schur_step<m, double>(fr, fi, rin * (1.0 - kCertMargin), gr, gi);
    return zeros_inside_unit_disk<m - 1>(gr, gi) == L - 2;
}

// Line-window sizes whose certificate first counts in FP32 at the fixed radius
// kCertKappa: the other roots of the root-MUSIC polynomial of a window with a
// tone sit well inside it (numpy trials, L = 4-8, N = 2L + 8 to 32, 0-30 dB:
// the largest inner one at radius 0.58 at the median, 0.76 at most), where the
// count is well conditioned; all inside kCertKappa <= rho means all inside rho.
// Larger sizes (block windows, few snapshots) count at rho in FP64 only.
constexpr int kCert32MaxL = 8;
constexpr float kCertKappa = 0.8f;

// True when the root z0 (with its mate 1/conj(z0)) is the root pair nearest
// the unit circle, i.e. the pair the selection rule of Sec. 3 picks from all
// roots.  Every root pair (z, 1/conj z) has its inner member at radius < 1,
// and the nearest pair is the one with the largest inner radius, so with
// z_in the inner member of z0's pair: (z - z_in)(z - 1/conj z_in) must divide
// P (remainder below kCertRemTol of the coefficients' size, kCertRemTol32 with the
// division in FP32 for L <= 8; a root on the circle,
// its own mirror, fails here), and the quotient Q must have all its L - 2
// inner roots strictly inside |z| < |z_in| (1 - margin) = rho.  For L <= 8 a
// decided FP32 count of L - 2 zeros of Q inside kCertKappa <= rho settles it;
// otherwise Schur-Cohn on Q(rho z) in FP64 decides.  On success (rr, ri) =
// z_in + 1/conj(z_in).
template <int L>
__device__ __forceinline__ bool certified_root(const float (&ar)[2 * L - 1], const float (&ai)[2 * L - 1], double z0r,
                                               double z0i, double& rr, double& ri) {
    constexpr int n = 2 * L - 2;
    double m2 = fma(z0r, z0r, z0i * z0i);
    if (!(m2 > 0.0) || !__builtin_isfinite(m2)) return false;
    if (m2 > 1.0) {                                   // take the inner member
        const double im = rcp64(m2);
        z0r *= im;
        z0i *= im;
        m2 = fma(z0r, z0r, z0i * z0i);
    }
    constexpr double kInnerMax2 = (1.0 - 1e-9) * (1.0 - 1e-9);
    if (!(m2 < kInnerMax2)) return false;             // |z_in| within 1e-9 of the circle
    const double im2 = rcp64(m2);
    const double z1r = z0r * im2, z1i = z0i * im2;   // 1/conj(z_in)
    rr = z0r + z1r;
    ri = z0i + z1i;
    // z^2 - r z - s with s = -z_in / conj(z_in)
    const double s_r = -(z0r * z1r - z0i * z1i), s_i = -(z0r * z1i + z0i * z1r);
    float scale = 0.f;                                // size of the (FP32) coefficients
#pragma unroll
    for (int k = n; k >= 0; --k) scale += fabsf(ar[k]) + fabsf(ai[k]);
    if constexpr (L == 2) {
        double fr[1], fi[1];
        return pair_quotient<n, double>(ar, ai, rr, ri, s_r, s_i, fr, fi) <= kCertRemTol * (double)scale;  // no other roots
    } else if constexpr (L <= kCert32MaxL) {
        constexpr int m = n - 2;
        float qr[n - 1], qi[n - 1];
        if (!(pair_quotient32<n>(ar, ai, (float)rr, (float)ri, (float)s_r, (float)s_i, qr, qi) <=
              kCertRemTol32 * scale))
            return false;
        constexpr double kKappaIn = (double)kCertKappa / (1.0 - kCertMargin);
        if (m2 >= kKappaIn * kKappaIn) {              // rho = |z_in| (1 - margin) >= kappa
            float gr[m], gi[m];
            first_schur_step<m, float>(qr, qi, kCertKappa, gr, gi);
            if (zeros_inside_unit_disk32<m - 1>(gr, gi) == L - 2) return true;
        }
        double fr[n - 1], fi[n - 1];                  // undecided: the quotient again, in FP64
        pair_quotient<n, double>(ar, ai, rr, ri, s_r, s_i, fr, fi);
        return inner_roots_inside<L>(fr, fi, sqrt(m2));
    } else {
        double fr[n - 1], fi[n - 1];
        if (!(pair_quotient<n, double>(ar, ai, rr, ri, s_r, s_i, fr, fi) <= kCertRemTol * (double)scale)) return false;
        return inner_roots_inside<L>(fr, fi, sqrt(m2));
    }
}

// Direction of the frequency guess from the lag-1 coefficient: u1[i+1]/u1[i]
// ~ e^{j w}, so c_1 ~ -((L-1)/L) e^{-j w} and e^{j w} = -conj(c_1) / |c_1|
// (no trigonometric functions needed); (1, 0) when c_1 vanishes.
__device__ __forceinline__ void guess_direction(float c1r, float c1i, float& cw, float& sw) {
    const float m2 = c1r * c1r + c1i * c1i;
    const bool ok = m2 > 0.f && finitef(m2);
    const float im = ok ? frsq(m2) : 0.f;
    cw = ok ? -c1r * im : 1.f;
    sw = ok ? c1i * im : 0.f;
}

// g(w) = e^{-j w (L-1)/2} B(e^{j w}) and its first two derivatives, where
// B(z) = sum_i conj(u_i) z^i: on the unit circle the root-MUSIC polynomial is
// z^{L-1} (L - g(w)^2) (with u = Q v conjugate-symmetric, u_{L-1-i} =
// conj(u_i), P(z) = L z^{L-1} - B(z)^2), and g is real:
// g(w) = sqrt2 sum_{i<m} (v_i cos(w s_i) + v_{o+i} sin(w s_i)) (+ v_m for odd L),
// s_i = i - (L-1)/2, from the real eigenvector v of T.  (hc, hs) = e^{j w / 2}.
template <int L>
__device__ __forceinline__ void spectral_g(const float (&v)[L], float hc, float hs, float& g, float& g1, float& g2) {
    constexpr int m = L / 2;
    constexpr int o = L - m;
    // e^{j w s_0}, s_0 = -(L-1)/2, then steps of e^{j w}
    float er = 1.f, ei = 0.f;
#pragma unroll
    for (int k = 0; k < L - 1; ++k) {
        const float t = er * hc + ei * hs;             // times e^{-j w/2}
        ei = ei * hc - er * hs;
        er = t;
    }
    const float sr = hc * hc - hs * hs, si = 2.f * hc * hs;   // e^{j w}
    float a = 0.f, b = 0.f, c = 0.f;
#pragma unroll
    for (int i = 0; i < m; ++i) {
        const float s = (float)i - 0.5f * (float)(L - 1);
        const float x = fmaf(v[i], er, v[o + i] * ei);         // v_i cos + v_{o+i} sin
        const float y = fmaf(v[o + i], er, -v[i] * ei);        // d/d(ws) of it
        a += x;
        b = fmaf(s, y, b);
        c = fmaf(-s * s, x, c);
        const float t = er * sr - ei * si;
        ei = er * si + ei * sr;
        er = t;
    }
    constexpr float kSqrt2 = 1.41421356237309515f;
    g = kSqrt2 * a;
    g1 = kSqrt2 * b;
    g2 = kSqrt2 * c;
    if (L & 1) g += v[m];
}

// Start of the signal-root iteration.  The signal root pair straddles the
// unit circle where |g(w)|^2 nearly reaches L, i.e. at the peak of g^2: one
// Newton step on (g^2)' = 0 from the guessed direction (cw, sw) moves w to
// the peak, and there the quadratic model L - g^2 + (g'^2 + g g'') t^2 = 0 of
// the polynomial at w + j t puts the root at radius e^{-t}.  From this start
// the FP32 Newton stage of a window at 10 dB usually needs one step and the
// FP64 stage one more (numpy trials, L = 6 and 8: FP32 steps of a wave's
// slowest lane 2.9 -> 1.0, FP64 1.7 -> 1.0, against the lag-1 direction at a
// radius fitted to lambda_1 and K).  Any start is safe: the certificate
// judges the root found.
template <int L>
__device__ __forceinline__ void pair_start(const float (&v)[L], float cw, float sw, double& zr, double& zi) {
    // e^{j w/2} from e^{j w} (cos(w/2) >= 0)
    float hc = fsqrt(fmaxf(0.5f * (1.f + cw), 0.f));
    float hs = hc > 1e-3f ? 0.5f * sw * frcp(hc) : 1.f;
    if (!(hc > 1e-3f)) hc = 0.f;
    float g, g1, g2;
    spectral_g<L>(v, hc, hs, g, g1, g2);
    // Newton step towards the peak of g^2: d = -(g g') / (g'^2 + g g'')
    const float h2 = fmaf(g1, g1, g * g2);
    float d = h2 < 0.f ? -g * g1 * frcp(h2) : 0.f;
    d = fminf(0.25f, fmaxf(-0.25f, finitef(d) ? d : 0.f));
    // rotate by e^{j d/2} (|d/2| <= 1/8: two Taylor terms each)
    const float x = 0.5f * d, x2 = x * x;
    const float rc = fmaf(x2, fmaf(x2, 1.f / 24.f, -0.5f), 1.f), rs = x * fmaf(x2, -1.f / 6.f, 1.f);
    const float nc = hc * rc - hs * rs, ns = hs * rc + hc * rs;
    spectral_g<L>(v, nc, ns, g, g1, g2);
    const float hh = fmaf(g1, g1, g * g2);
    const float dep = fmaxf((float)L - g * g, 0.f);
    float t = hh < 0.f ? fsqrt(dep * frcp(-hh)) : 0.01f;
    t = fminf(0.1f, fmaxf(1e-4f, finitef(t) ? t : 0.01f));
    const float r0 = __expf(-t);
    zr = (double)(r0 * (nc * nc - ns * ns));
    zi = (double)(r0 * 2.f * nc * ns);
}

// Lag sums at start t: S_d = sum_{k<K} g[t+k] conj(g[t+k+d]), d < L, from the
// staged signal g, into registers.  The last L samples live in a circular
// register buffer indexed by k mod L, unrolled L steps at a time so that no
// register moves are needed.
template <int L>
__device__ __forceinline__ void lag_sum_regs(const float2* g, int t, int K, float (&sr)[L], float (&si)[L]) {
#pragma unroll
    for (int d = 0; d < L; ++d) { sr[d] = 0.f; si[d] = 0.f; }
    float2 win[L];                      // win[m mod L] = g[t + m]
#pragma unroll
    for (int d = 0; d < L - 1; ++d) win[d] = g[t + d];
    int k0 = 0;
    for (; k0 + L <= K; k0 += L) {
#pragma unroll
        for (int u = 0; u < L; ++u) {
            win[(u + L - 1) % L] = g[t + k0 + u + L - 1];
#pragma unroll
            for (int d = 0; d < L; ++d) {
                const float2 a = win[u], b = win[(u + d) % L];
                sr[d] = fmaf(a.x, b.x, fmaf(a.y, b.y, sr[d]));
                if (d > 0) si[d] = fmaf(a.y, b.x, fmaf(-a.x, b.y, si[d]));   // S_0 is real
            }
        }
    }
#pragma unroll
    for (int u = 0; u < L - 1; ++u) {
        if (k0 + u < K) {
            win[(u + L - 1) % L] = g[t + k0 + u + L - 1];
#pragma unroll
            for (int d = 0; d < L; ++d) {
                const float2 a = win[u], b = win[(u + d) % L];
                sr[d] = fmaf(a.x, b.x, fmaf(a.y, b.y, sr[d]));
                if (d > 0) si[d] = fmaf(a.y, b.x, fmaf(-a.x, b.y, si[d]));   // S_0 is real
            }
        }
    }
}

// Lag sums of lane t stored to sS[d][t].
template <int L, int STRIDE>
__device__ __forceinline__ void lag_sums(const float2* g, int t, int K, float2 (*sS)[STRIDE]) {
    float sr[L], si[L];
    lag_sum_regs<L>(g, t, K, sr, si);
#pragma unroll
    for (int d = 0; d < L; ++d) sS[d][t] = make_float2(sr[d], si[d]);
}

// Lag sums at the two starts q and q+1 (q even), the second slid from the
// first: S_d(q+1) = S_d(q) - g[q] conj(g[q+d]) + g[q+K] conj(g[q+K+d]).
// Stored as one 16-byte pair per lag to sS[d][q .. q+1] (16-byte aligned rows).
template <int L, int STRIDE>
__device__ __forceinline__ void lag_sums_pair(const float2* g, int q, int K, float2 (*sS)[STRIDE]) {
    float sr[L], si[L];
    lag_sum_regs<L>(g, q, K, sr, si);
    const float2 a0 = g[q], a1 = g[q + K];
#pragma unroll
    for (int d = 0; d < L; ++d) {
        const float2 b0 = g[q + d], b1 = g[q + K + d];
        const float tr = fmaf(a1.x, b1.x, fmaf(a1.y, b1.y, fmaf(-a0.x, b0.x, fmaf(-a0.y, b0.y, sr[d]))));
        const float ti = d == 0 ? 0.f : fmaf(a1.y, b1.x, fmaf(-a1.x, b1.y, fmaf(-a0.y, b0.x, fmaf(a0.x, b0.y, si[d]))));
        *reinterpret_cast<float4*>(&sS[d][q]) = make_float4(sr[d], si[d], tr, ti);
    }
}

// Staged line samples in LDS, de-interleaved by index mod 4: sample i sits in
// slot (i & 3) Q + (i >> 2), Q = the quarter length.  The lane pairs below
// read samples four starts apart; in a plain layout a wave's 32 distinct
// addresses would fall on a quarter of the LDS banks, de-interleaved they are
// consecutive slots.
constexpr int sg_quarter(int n) { return (n + 3) / 4; }
__device__ __forceinline__ int sg_slot(int i, int quarter) { return (i & 3) * quarter + (i >> 2); }

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

// Lag sums S_d(q) = sum_{k<K} g[q+k] conj(g[q+k+d]), d < L, of the four
// window starts q .. q+3, q = 4 (t / 2), computed by the lane pair (t, t ^ 1):
// lane h = t & 1 takes the lags d0 .. d0 + LH - 1, d0 = h LH, LH = ceil(L/2)
// (for odd L the second lane's last lag is a dummy, not stored; its sums read
// one sample past the last window's, which is staged as well).  The first
// start's sums are direct over its K snapshots, with the b-samples g[q+k+d]
// in a circular register buffer indexed by k mod LH (unrolled lcm(LH, 4)
// steps at a time, so that neither register moves nor run-time slot
// arithmetic are needed); the next three are slid by one sample each,
//   S_d(s+1) = S_d(s) - g[s] conj(g[s+d]) + g[s+K] conj(g[s+K+d]),
// so each start costs about a quarter of a direct sum over all lags.  Blocks
// start at multiples of four pixels, so which starts are summed directly
// depends on the start alone, not on the tile size.  g is in the
// de-interleaved layout above (quarter length QUARTER): the slot of sample
// q + off + 4a + r is base[r] + a for per-lane bases of the offsets 0, d0, K
// and K + d0.  Stored as two 16-byte pairs per lag to sS[d][q .. q+3]
// (16-byte aligned rows).  S_0's imaginary part is not meaningful (readers
// take the zero lag as real).
template <int L, int STRIDE, int QUARTER>
__device__ __forceinline__ void lag_sums_quad(const float2* g, int t, int K, float2 (*sS)[STRIDE]) {
    constexpr int LH = (L + 1) / 2;
    constexpr int U = LH * 4 / gcd_int(LH, 4);
    const int jq = t >> 1;                               // q / 4
    const int q = 4 * jq;
    const int d0 = (t & 1) * LH;
    int ba[4], bb[4], bk[4], bkd[4];                      // slot bases of q + {0, d0, K, K + d0} + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ba[r] = r * QUARTER + jq;
        bb[r] = ((d0 + r) & 3) * QUARTER + jq + ((d0 + r) >> 2);
        bk[r] = ((K + r) & 3) * QUARTER + jq + ((K + r) >> 2);
        bkd[r] = ((K + d0 + r) & 3) * QUARTER + jq + ((K + d0 + r) >> 2);
    }
    float sr[LH], si[LH];
#pragma unroll
    for (int e = 0; e < LH; ++e) { sr[e] = 0.f; si[e] = 0.f; }
    float2 win[LH];                      // win[(k + e) mod LH] = g[q + d0 + k + e]
#pragma unroll
    for (int e = 0; e < LH - 1; ++e) win[e] = g[bb[e & 3] + (e >> 2)];
    // k = k0 + u with k0 a multiple of U: every slot index below is a base plus a constant
    auto term = [&](int a4, int u) {
        const int c = u + LH - 1;
        win[(u + LH - 1) % LH] = g[bb[c & 3] + a4 + (c >> 2)];
        const float2 a = g[ba[u & 3] + a4 + (u >> 2)];
#pragma unroll
        for (int e = 0; e < LH; ++e) {
            const float2 b = win[(u + e) % LH];
            sr[e] = fmaf(a.x, b.x, fmaf(a.y, b.y, sr[e]));
            si[e] = fmaf(a.y, b.x, fmaf(-a.x, b.y, si[e]));
        }
    };
    int k0 = 0;
    for (; k0 + U <= K; k0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) term(k0 >> 2, u);
    }
#pragma unroll
    for (int u = 0; u < U - 1; ++u)
        if (k0 + u < K) term(k0 >> 2, u);
    auto slide = [&](int st) {                          // S(q + st) -> S(q + st + 1), st compile-time
        const float2 a0 = g[ba[st & 3] + (st >> 2)], a1 = g[bk[st & 3] + (st >> 2)];
#pragma unroll
        for (int e = 0; e < LH; ++e) {
            const int c = st + e;
            const float2 b0 = g[bb[c & 3] + (c >> 2)], b1 = g[bkd[c & 3] + (c >> 2)];
            sr[e] = fmaf(a1.x, b1.x, fmaf(a1.y, b1.y, fmaf(-a0.x, b0.x, fmaf(-a0.y, b0.y, sr[e]))));
            si[e] = fmaf(a1.y, b1.x, fmaf(-a1.x, b1.y, fmaf(-a0.y, b0.x, fmaf(a0.x, b0.y, si[e]))));
        }
    };
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float pr[LH], pi[LH];
#pragma unroll
        for (int e = 0; e < LH; ++e) { pr[e] = sr[e]; pi[e] = si[e]; }
        slide(2 * h);
#pragma unroll
        for (int e = 0; e < LH; ++e)
            if (d0 + e < L)
                *reinterpret_cast<float4*>(&sS[d0 + e][q + 2 * h]) = make_float4(pr[e], pi[e], sr[e], si[e]);
        if (h == 0) slide(1);
    }
}

// Divide T by its trace; false when the trace is zero or not finite (no
// signal subspace).
template <int L>
__device__ __forceinline__ bool trace_normalise(Sym<L>& T) {
    float tr = 0.f;
#pragma unroll
    for (int i = 0; i < L; ++i) tr += T.a[i][i];
    if (!(tr > 0.f && finitef(tr))) return false;
    const float itr = frcp(tr);
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = i; j < L; ++j) T.a[i][j] *= itr;
    return true;
}

// Trace-normalised T = Q^H R_fb Q from the covariance; false when R is zero
// or not finite (no signal subspace).
template <int L>
__device__ __forceinline__ bool normalised_T(const Cov<L>& R, Sym<L>& T) {
    build_T<L>(R, T);
    return trace_normalise<L>(T);
}

// T = Q^H R_fb Q summed straight from the snapshots s_k (Eq. 4), without the
// complex covariance.  Q satisfies J conj(Q) = Q, so Q^H J conj(R) J Q =
// conj(Q^H R Q) and T = Re(Q^H R Q) = sum_k (a_k a_k^T + b_k b_k^T) with
// a_k + j b_k = Q^H s_k: for i < m = L/2, (Q^H s)_i = (s_i + s_{L-1-i})/sqrt2,
// (Q^H s)_{o+i} = -j (s_i - s_{L-1-i})/sqrt2, o = L - m, and for odd L
// (Q^H s)_m = s_m.  The common factor sqrt2 is left in (y = sqrt2 Q^H s), which
// scales T by 2; the trace normalisation removes it.  `snap(k, i)` returns
// s_k[i].  About half the work of the complex upper triangle plus build_T,
// and no complex L x L array in registers.  (c1r, c1i) receives the lag-1
// sum sum_k sum_i conj(s_k[i]) s_k[i+1], whose phase starts the power iteration.
template <int L, typename F>
__device__ __forceinline__ void T_from_snapshots(int K, F snap, Sym<L>& T, float& c1r, float& c1i) {
    constexpr int m = L / 2;
    constexpr int o = L - m;
    constexpr float kSqrt2 = 1.41421356237309515f;
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = i; j < L; ++j) T.a[i][j] = 0.f;
    c1r = 0.f;
    c1i = 0.f;
    // one snapshot at a time: unrolled, the loads of all snapshots would be
    // hoisted and held in registers
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        float2 v[L];
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = snap(k, i);
        // lag-1 sum: sum_i conj(s[i]) s[i+1]
#pragma unroll
        for (int i = 0; i + 1 < L; ++i) {
            c1r = fmaf(v[i].x, v[i + 1].x, fmaf(v[i].y, v[i + 1].y, c1r));
            c1i = fmaf(v[i].x, v[i + 1].y, fmaf(-v[i].y, v[i + 1].x, c1i));
        }
        float a[L], b[L];
#pragma unroll
        for (int i = 0; i < m; ++i) {
            const float2 p = v[i], q = v[L - 1 - i];
            a[i] = p.x + q.x;
            b[i] = p.y + q.y;
            a[o + i] = p.y - q.y;         // -j (p - q) = (p.y - q.y) - j (p.x - q.x)
            b[o + i] = q.x - p.x;
        }
        if (L & 1) {
            a[m] = kSqrt2 * v[m].x;
            b[m] = kSqrt2 * v[m].y;
        }
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int j = i; j < L; ++j) T.a[i][j] = fmaf(a[i], a[j], fmaf(b[i], b[j], T.a[i][j]));
    }
}

// Top eigenvector of the trace-normalised T by power iteration from the real
// form of the steering vector of a predicted frequency w, (hc, hs) = e^{j w/2}
// (v0 = Q^H a(w) e^{-j w (L-1)/2} / sqrt L: sqrt(2/L) (cos w s_i, sin w s_i)
// with s_i = i - (L-1)/2, and 1/sqrt L for the middle of odd L).  The iterate
// is accepted once an a-posteriori bound proves it within `tol` of the top
// eigenvector.  With the Rayleigh quotient rho and residual r of the vector
// v a step is taken from: lambda_1 >= rho; every other eigenvalue has
// |lambda_i| <= l2 = sqrt(tr T^2 - rho^2), since their squares sum to
// tr T^2 - lambda_1^2; so sin(angle of v) <= sb = |r| / (|v| (rho - l2))
// (the residual bound for symmetric matrices), and the step multiplies
// tan(angle) by at most l2 / rho.  The result of the step is accepted when
// (l2 / rho) tan <= tol, with tan <= sb / sqrt(1 - sb^2) <= sb sqrt(4/3) for
// sb <= 1/2, and rho - l2 > 1e-5 rho is required too: that proves
// lambda_1 > lambda_2 (1 + 1e-5), so an accepted window is never degenerate.  Returns false (v undefined) when no step
// within max_steps is accepted; *steps counts the steps taken.  *nu receives
// the MUSIC null spectrum 1 - (v^T v0)^2 at the prediction.
template <int L>
__device__ __forceinline__ bool power_top_eigvec(const Sym<L>& T, float hc, float hs, int min_steps, int max_steps,
                                                 float tol, float (&v)[L], int& steps, float& nu) {
    constexpr int m = L / 2;
    constexpr int o = L - m;
    float v0[L];
    {
        float er = 1.f, ei = 0.f;
#pragma unroll
        for (int k = 0; k < L - 1; ++k) {                  // e^{j w s_0}
            const float t = er * hc + ei * hs;
            ei = ei * hc - er * hs;
            er = t;
        }
        const float sr = hc * hc - hs * hs, si = 2.f * hc * hs;
        const float sc = 1.41421356237309515f * frsq((float)L);
#pragma unroll
        for (int a = 0; a < m; ++a) {
            v0[a] = sc * er;
            v0[o + a] = sc * ei;
            const float t = er * sr - ei * si;
            ei = er * si + ei * sr;
            er = t;
        }
        if (L & 1) v0[m] = frsq((float)L);
    }
    float t2 = 0.f;                                         // tr T^2
#pragma unroll
    for (int i = 0; i < L; ++i) {
        t2 = fmaf(T.a[i][i], T.a[i][i], t2);
#pragma unroll
        for (int j = i + 1; j < L; ++j) t2 = fmaf(2.f * T.a[i][j], T.a[i][j], t2);
    }
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] = v0[i];
    // Unnormalised steps: the trace is 1, so lambda_1 >= 1/L and max_steps
    // steps shrink the iterate by at most L^-max_steps, far inside FP32's range.
    bool ok = false;
    for (int it = 0; it < max_steps; ++it) {
        ++steps;
        float y[L];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < L; ++j) acc = fmaf(T.at(i, j), v[j], acc);
            y[i] = acc;
        }
        if (it + 1 >= min_steps) {
            float vy = 0.f, vv = 0.f;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                vy = fmaf(v[i], y[i], vy);
                vv = fmaf(v[i], v[i], vv);
            }
            const float ivv = frcp(vv);
            const float rho = vy * ivv;                     // Rayleigh quotient of v
            float r2 = 0.f;                                 // |T v - rho v|^2, summed from its terms
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const float r = fmaf(-rho, v[i], y[i]);
                r2 = fmaf(r, r, r2);
            }
            // |lambda_i| <= l2 for every i >= 2 (Frobenius), sin(theta) of v <= sb,
            // and the step contracts tan(theta) by at least l2 / rho
            const float l2 = fsqrt(fmaxf(fmaf(-rho, rho, t2), 0.f));
            const float gap = rho - l2;
            const float sb2 = r2 * ivv * frcp(gap * gap);
            const float c2 = l2 * l2 * frcp(rho * rho);
            ok = gap > kDegenRel * rho && sb2 <= 0.25f && sb2 * c2 * (4.f / 3.f) <= tol * tol && finitef(ivv);
            // give up early where even the remaining steps at the proven
            // contraction cannot reach tol (low SNR: the plain solver is cheaper)
            const float left = (float)(max_steps - it);
            const bool hopeless = !(gap > 0.f) || !finitef(ivv) ||
                                  fminf(sb2, 0.25f) * (4.f / 3.f) *
                                          __builtin_amdgcn_exp2f(left * __builtin_amdgcn_logf(c2)) > tol * tol;
            if (!ok && hopeless) break;
        }
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = y[i];
        if (ok) break;
    }
    float n2 = 0.f, dot = 0.f;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        n2 = fmaf(v[i], v[i], n2);
        dot = fmaf(v[i], v0[i], dot);
    }
    const float in = frsq(n2);
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] *= in;
    dot *= in;
    nu = 1.f - dot * dot;
    return ok;
}

// Plain root-MUSIC frequency of one window from its covariance (paper
// Sec. 3, Eq. 6-15): eigen-split, polynomial, the certified pair or all
// roots, pair selection, FP64 pair polish.  omega stays NaN with
// BM_FLAG_UNDEFINED when the covariance is zero or not finite, and with
// BM_FLAG_DEGENERATE when its signal subspace is not determined.
template <int L>
__device__ __forceinline__ void window_omega_v(const float (&v)[L], const RootTemplate& tmpl, bool full_roots,
                                               float wprev, float& omega, unsigned& flag, LaneStats& ls);

// e^{j w / 2} of the lag-1 direction of the covariance, w = arg sum_i
// R[i][i+1]^* (the phase of the mean lag-1 product), for a power-iteration start.
// e^{j w / 2} for w = arg(sr + j si) (w = 0 when that is zero or not finite).
__device__ __forceinline__ void half_angle_of(float sr, float si, float& hc, float& hs) {
    const float m2 = sr * sr + si * si;
    const bool ok = m2 > 0.f && finitef(m2);
    const float im = ok ? frsq(m2) : 0.f;
    const float cw = ok ? sr * im : 1.f, sw = ok ? si * im : 0.f;
    hc = fsqrt(fmaxf(0.5f * (1.f + cw), 0.f));
    hs = hc > 1e-3f ? 0.5f * sw * frcp(hc) : 1.f;
    if (!(hc > 1e-3f)) hc = 0.f;
}

template <int L>
__device__ __forceinline__ void lag1_half_angle(const Cov<L>& R, float& hc, float& hs) {
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int i = 0; i + 1 < L; ++i) {
        sr += R.re[i][i + 1];
        si -= R.im[i][i + 1];
    }
    half_angle_of(sr, si, hc, hs);
}

// Power iteration of the windows: a start at the lag-1 direction, the
// first test after two steps, at most eight, and a proven angle below 1e-5.
constexpr int kPowerMinSteps = 2;
constexpr int kPowerMaxSteps = 8;
constexpr float kPowerTol = 1e-5f;

// The signal eigenvector of T by the tridiagonal solver (Jacobi with
// JACOBI); false, with BM_FLAG_DEGENERATE, when the subspace is not determined.
template <int L, bool JACOBI>
__device__ __forceinline__ bool signal_eigvec_T(Sym<L>& T, float (&v)[L], unsigned& flag, LaneStats& ls) {
    float lam = 1.f;
    bool degen = false;
    if (JACOBI) top_eigvec_jacobi<L>(T, v, ls.eig_its, lam, degen);
    else top_eigvec_tridiag<L>(T, v, ls.eig_its, lam, degen);
    if (degen) flag |= BM_FLAG_DEGENERATE;
    return !degen;
}

// The window from its trace-normalised T and a start e^{j w/2} = (hc, hs) at
// the window's lag-1 phase: the signal eigenvector first by power iteration
// (power_top_eigvec: accepted only with a proven angle below 1e-5 rad and a
// proven gap), else by the tridiagonal solver (Jacobi alone with JACOBI);
// then the polynomial, the root pair and omega.
template <int L, bool JACOBI>
__device__ __forceinline__ void window_omega_Ts(Sym<L>& T, float hc, float hs, const RootTemplate& tmpl,
                                                bool full_roots, float wprev, float& omega, unsigned& flag,
                                                LaneStats& ls) {
    ls.counted += 1;
    // ---- signal subspace (Eq. 6-11) ------------------------------------
    float v[L];
    bool have = false;
    if (!JACOBI) {
        float nu;
        int steps = 0;
        have = power_top_eigvec<L>(T, hc, hs, kPowerMinSteps, kPowerMaxSteps, kPowerTol, v, steps, nu);
        if (have) {
            ls.power += 1;
            ls.eig_its += steps;
        }
    }
    if (!have && !signal_eigvec_T<L, JACOBI>(T, v, flag, ls)) return;
    window_omega_v<L>(v, tmpl, full_roots, wprev, omega, flag, ls);
}

// The window from its covariance (line windows).
template <int L, bool JACOBI>
__device__ __forceinline__ void window_omega(const Cov<L>& R, const RootTemplate& tmpl, bool full_roots, int K,
                                             float wprev, float& omega, unsigned& flag, LaneStats& ls) {
    float hc = 1.f, hs = 0.f;
    if (!JACOBI) lag1_half_angle<L>(R, hc, hs);
    Sym<L> T;
    if (!normalised_T<L>(R, T)) {
        flag |= BM_FLAG_UNDEFINED;
        return;
    }
    window_omega_Ts<L, JACOBI>(T, hc, hs, tmpl, full_roots, wprev, omega, flag, ls);
}

// The rest of the window from the top eigenvector v of T (unit, real form of
// u1 = Q v): polynomial, the certified pair or all roots, omega.
template <int L>
__device__ __forceinline__ void window_omega_v(const float (&v)[L], const RootTemplate& tmpl, bool full_roots,
                                               float wprev, float& omega, unsigned& flag, LaneStats& ls) {
    constexpr int n = 2 * L - 2;
    float ur[L], ui[L];
    signal_vector<L>(v, ur, ui);
    // ---- polynomial coefficients (Eq. 12-14) -----------------------------
    float ar[n + 1], ai[n + 1];
    poly_coeffs<L>(ur, ui, ar, ai);

    // frequency guess from the lag-1 coefficient c_1, or, with the temporal
    // warm start, the previous frame's frequency at this pixel
    float sw0, cw0;
    if (finitef(wprev)) __sincosf(wprev, &sw0, &cw0);
    else guess_direction(ar[L], ai[L], cw0, sw0);

    // ---- certified pair ---------------------------------------------------
    // FP64 Newton (with the mate divided out) for the signal root from the
    // guess w0; when its pair is certified as the pair nearest the unit
    // circle it is the pair the selection rule picks from all roots, and its
    // sum gives omega exactly as below.  Otherwise every root is found.
    bool cert = false;
    if (!full_roots) {
        double zr0, zi0, rr = 0.0, ri = 0.0;
        pair_start<L>(v, cw0, sw0, zr0, zi0);
        pair_newton32<L>(ur, ui, zr0, zi0, kCertIters32, &ls.pair_its32);
        cert = pair_newton<L>(ur, ui, zr0, zi0, kCertIters, &ls.pair_its) && certified_root<L>(ar, ai, zr0, zi0, rr, ri);
        if (cert) omega = atan2f((float)ri, (float)rr);
    }
    ls.accepted += cert ? 1 : 0;
    ls.rejected += (!full_roots && !cert) ? 1 : 0;
    if (cert) return;

    // ---- Aberth-Ehrlich in FP32 -------------------------------------------
    float zr[n], zi[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        zr[i] = tmpl.re[i] * cw0 - tmpl.im[i] * sw0;
        zi[i] = tmpl.re[i] * sw0 + tmpl.im[i] * cw0;
    }
    for (int it = 0; it < kMaxRootIters; ++it) {
        ++ls.iters;
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

    // ---- pair selection -------------------------------------------------
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

    // ---- FP64 polish of the quadratic factor z^2 - r z - s --------------
    double rr = (double)zsr + (double)zmr, ri = (double)zsi + (double)zmi;
    double s_r = -((double)zsr * zmr - (double)zsi * zmi);
    double s_i = -((double)zsr * zmi + (double)zsi * zmr);
    double lastc = 0.0;
    bool pok = bairstow<double, n>(ar, ai, rr, ri, s_r, s_i, kPolishIters, lastc);
    const double rmag = fabs(rr) + fabs(ri);
    if (!(pok && lastc <= 1e-6 * rmag)) {
        pok = false;
        rr = (double)zsr + (double)zmr;
        ri = (double)zsi + (double)zmi;
    }
    ls.pfail += pok ? 0 : 1;
    if (!pok) flag |= BM_FLAG_NO_POLISH;
    omega = atan2f((float)ri, (float)rr);
}

}  // namespace bm
