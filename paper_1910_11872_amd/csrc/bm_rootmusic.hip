// Per-window root-MUSIC local-frequency kernel for gfx950.
//
// One lane owns one window (one output pixel of one direction).  A block of
// 256 lanes covers 256 consecutive window positions of one line; the
// overlapping windows are staged once in LDS with coalesced loads.  Per lane,
// entirely in registers:
//
//   covariance  R_ij = sum_k g[k+i] conj(g[k+j])          (paper Eq. 4)
//   FB average + unitary real transform: T = Q^H R_fb Q is real symmetric
//               (Q the sparse centro-symmetric unitary matrix), built in
//               closed form from R without forming R_fb
//   eigen-split cyclic Jacobi on T; the eigenvector of the largest
//               eigenvalue v gives the signal subspace u1 = Q v
//               (paper Eq. 6-11, one-dimensional signal subspace)
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

constexpr int kBlock = 256;
constexpr int kMaxJacobiSweeps = 10;
constexpr float kJacobiTol2 = 1e-12f;   // squared off-diagonal mass, trace-normalised
constexpr int kMaxRootIters = 16;
constexpr float kRootTol2 = 1e-6f;     // squared relative root step
constexpr int kPolishIters = 3;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

// Hermitian accessor of the upper-triangle covariance store.
template <int L>
struct Cov {
    float re[L][L];
    float im[L][L];
    __device__ __forceinline__ float gr(int i, int j) const { return i <= j ? re[i][j] : re[j][i]; }
    __device__ __forceinline__ float gi(int i, int j) const { return i <= j ? im[i][j] : -im[j][i]; }
};

template <int L>
struct Sym {
    float a[L][L];
    __device__ __forceinline__ float& at(int i, int j) { return i <= j ? a[i][j] : a[j][i]; }
};

template <int L, bool STATS>
__global__ __launch_bounds__(kBlock) void rootmusic_kernel(RootMusicArgs A) {
    constexpr int n = 2 * L - 2;            // polynomial degree
    constexpr int m = L / 2;
    constexpr int o = L - m;                // first column of the imaginary block of Q
    __shared__ float2 sg[kBlock + kMaxN];

    const int line = blockIdx.y;
    const int p0 = blockIdx.x * kBlock;
    const int t = threadIdx.x;
    const int N = A.N;
    const int half = N >> 1;
    const int K = N - L + 1;
    const float2* g = A.gamma + (int64_t)line * A.gamma_ls;

    const int base = p0 - half;
    for (int i = t; i < kBlock + N - 1; i += kBlock) {
        const int q = base + i;
        sg[i] = (q >= 0 && q < A.len) ? g[q] : make_float2(0.f, 0.f);
    }
    __syncthreads();

    const int p = p0 + t;
    const bool inside_line = p < A.len;
    const bool valid = inside_line && (p - half >= 0) && (p - half + N <= A.len);

    float omega = __builtin_nanf("");
    unsigned flag = 0;
    int sweeps = 0, iters = 0, pfail = 0, counted = 0;

    if (valid) {
        const float2* w = sg + t;
        // ---- covariance of the sub-snapshots (Eq. 4), upper triangle -------
        Cov<L> R;
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int j = i; j < L; ++j) { R.re[i][j] = 0.f; R.im[i][j] = 0.f; }
        for (int k = 0; k < K; ++k) {
            float2 s[L];
#pragma unroll
            for (int i = 0; i < L; ++i) s[i] = w[k + i];
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
                for (int j = i; j < L; ++j) {
                    R.re[i][j] = fmaf(s[i].x, s[j].x, fmaf(s[i].y, s[j].y, R.re[i][j]));
                    if (i != j) R.im[i][j] = fmaf(s[i].y, s[j].x, fmaf(-s[i].x, s[j].y, R.im[i][j]));
                }
        }
        // ---- T = Q^H R_fb Q (real symmetric), with F = 2 R_fb --------------
        // F(i,j) = R(i,j) + conj(R(L-1-i, L-1-j))
        auto Fr = [&](int i, int j) { return R.gr(i, j) + R.gr(L - 1 - i, L - 1 - j); };
        auto Fi = [&](int i, int j) { return R.gi(i, j) - R.gi(L - 1 - i, L - 1 - j); };
        Sym<L> T;
        constexpr float kSqrt2 = 1.41421356237309515f;
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

            // ---- cyclic Jacobi on T (eigen-split, Eq. 6-11) ----------------
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
            // eigenvector of the largest eigenvalue
            float v[L];
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
                zr[i] = A.tmpl.re[i] * cw0 - A.tmpl.im[i] * sw0;
                zi[i] = A.tmpl.re[i] * sw0 + A.tmpl.im[i] * cw0;
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
        const int64_t oidx = (int64_t)p * A.out_es + (int64_t)line * A.out_ls;
        A.out[oidx] = omega;
        if (A.flags) {
            const uint8_t f = (uint8_t)(flag << A.flag_shift);
            if (A.flag_or) A.flags[oidx] |= f;
            else A.flags[oidx] = f;
        }
    }
    if (STATS) {
        unsigned long long a0 = counted, a1 = sweeps, a2 = iters, a3 = pfail;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off);
            a1 += __shfl_xor(a1, off);
            a2 += __shfl_xor(a2, off);
            a3 += __shfl_xor(a3, off);
        }
        if ((t & 63) == 0) {
            atomicAdd(A.stats + 0, a0);
            atomicAdd(A.stats + 1, a1);
            atomicAdd(A.stats + 2, a2);
            atomicAdd(A.stats + 3, a3);
        }
    }
}

template <int L>
hipError_t launch_L(const RootMusicArgs& a, hipStream_t s) {
    dim3 grid((a.len + kBlock - 1) / kBlock, a.nlines);
    if (a.stats)
        hipLaunchKernelGGL((rootmusic_kernel<L, true>), grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((rootmusic_kernel<L, false>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rootmusic(int L, const RootMusicArgs& a, hipStream_t s) {
    if (a.len <= 0 || a.nlines <= 0) return hipSuccess;
    switch (L) {
        case 2: return launch_L<2>(a, s);
        case 3: return launch_L<3>(a, s);
        case 4: return launch_L<4>(a, s);
        case 5: return launch_L<5>(a, s);
        case 6: return launch_L<6>(a, s);
        case 7: return launch_L<7>(a, s);
        case 8: return launch_L<8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bm
