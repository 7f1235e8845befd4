// Per-window root-MUSIC local-frequency kernels for gfx950 (device code and
// launch templates, shared by bm_rootmusic.hip and bm_bigblock.hip).
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
//               signal subspace).  Power iteration on T from
//               the steering vector of the window's lag-1 phase, kept when
//               an a-posteriori bound proves it within 1e-5 rad of the top
//               eigenvector (2-3 steps at 10 dB).  Otherwise: Householder
//               reduction to tridiagonal form, Newton's
//               method from above on the characteristic polynomial
//               (monotone for real-rooted polynomials) for the largest
//               eigenvalue, one shifted inverse iteration for its
//               eigenvector, back-transformation.  The cyclic Jacobi solver
//               is kept as a selectable alternative.
//   polynomial  c_k = sum_i C[i,i+k] with C = I - u1 u1^H = Un Un^H
//               (paper Eq. 12-14)
//   certified pair  FP64 Newton for the signal root with its mate
//               1/conj(z) divided out, started just inside the unit circle
//               at the phase of c_1; accepted when the polynomial divides by
//               the pair's factor and a Schur-Cohn count on the quotient
//               puts every other inner root strictly inside |z_in|: that
//               pair is the one the selection below would pick.  Windows
//               that fail this (about 1 in 10^4 at 8 dB) take the path below.
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
#pragma once

#include "bm_window.h"

namespace bm {
namespace {

// Line windows per lane (two window starts per lane).  For L <= 6 a lane sums
// the lags of its two starts, the second slid from the first (lag_sums_pair);
// for L >= 7 a lane pair sums the lags of four consecutive starts, one half of
// the lags each, the first start directly and the next three slid by one
// sample (lag_sums_quad), so each start costs about a quarter of a direct sum
// over all lags while the block keeps the same 2 x 256 starts in LDS.  (At
// L = 6 the quarter-cost form measured 3-6% slower: with three lags per lane
// its two LDS reads per snapshot weigh more than the FMAs it saves.)  Blocks
// start at multiples of two (four) pixels, so which window starts are summed
// directly and which are slid depends on the start alone, not on the tile
// size: results are the same for every tiling.  (Four starts per lane, each
// lane with all lags, double the lag sums a block keeps in LDS, which halves
// the blocks resident per CU: twice slower on 1024-wide lines.)
constexpr int kLineSpan = 2;

constexpr bool line_quad(int L) { return L >= 7; }
constexpr int line_windows_per_block(int L, int block) {
    return (kLineSpan * block - (L - 1)) & (line_quad(L) ? ~3 : ~1);
}

template <int L, int BLOCK>
struct LineSpan {
    static constexpr int span = kLineSpan * BLOCK;                  // window starts per block
    static constexpr int wpb = line_windows_per_block(L, BLOCK);    // output pixels per block (even; L >= 7: x4)
    static constexpr bool quad = line_quad(L);                      // lag_sums_quad (else lag_sums_pair)
    static constexpr int row = span + 8;                            // lag-sum row: >= span, 16-byte multiple
    static constexpr int quarter = sg_quarter(span + kMaxN);        // staged samples, de-interleaved
};

// One block of windows: SPAN-(L-1) consecutive pixels p0.. of one line of job J.
template <int L, int BLOCK, bool JACOBI, bool WARM>
__device__ __forceinline__ void rootmusic_block(const RmJob& J, int line, int p0, float2* sg,
                                                float2 (*sS)[LineSpan<L, BLOCK>::row], const RootTemplate& tmpl,
                                                bool full_roots, LaneStats& ls) {
    constexpr int SPAN = LineSpan<L, BLOCK>::span;
    constexpr int WPB = LineSpan<L, BLOCK>::wpb;
    const int t = threadIdx.x;
    const int N = J.N;
    const int half = N >> 1;
    const int K = N - L + 1;
    const float2* g = J.gamma + (int64_t)line * J.gamma_ls;
    const int len = J.len;

    // window of pixel p0+s starts at base+s
    const int base = p0 - half;
    // ---- lag sums S_d(base + s), s < SPAN, d < L -----------------------------
    if constexpr (LineSpan<L, BLOCK>::quad) {
        for (int i = t; i < SPAN + N; i += BLOCK) {        // one sample more for the odd-L dummy lag
            const int q = base + i;
            sg[sg_slot(i, LineSpan<L, BLOCK>::quarter)] = (q >= 0 && q < len) ? g[q] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        lag_sums_quad<L, LineSpan<L, BLOCK>::row, LineSpan<L, BLOCK>::quarter>(sg, t, K, sS);
    } else {
        for (int i = t; i < SPAN + N - 1; i += BLOCK) {
            const int q = base + i;
            sg[i] = (q >= 0 && q < len) ? g[q] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        lag_sums_pair<L, LineSpan<L, BLOCK>::row>(sg, kLineSpan * t, K, sS);
    }
    __syncthreads();

#pragma unroll 1
    for (int r = 0; r < kLineSpan; ++r) {
        const int s = r * BLOCK + t;
        const int p = p0 + s;
        const bool inside_line = (s < WPB) && (p < len);
        const bool valid = inside_line && (p - half >= 0) && (p - half + N <= len);
        float omega = __builtin_nanf("");
        unsigned flag = 0;
        if (valid) {
            // covariance R_ij = S_{j-i}(s+i) (Eq. 4, up to the 1/K scale)
            Cov<L> R;
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
                for (int j = i; j < L; ++j) {
                    const float2 v = sS[j - i][s + i];
                    R.re[i][j] = v.x;
                    R.im[i][j] = (i == j) ? 0.f : v.y;
                }
            const float wprev = (WARM && J.prev) ? J.prev[(int64_t)p * J.prev_es + (int64_t)line * J.prev_ls]
                                                 : __builtin_nanf("");
            window_omega<L, JACOBI>(R, tmpl, full_roots, K, wprev, omega, flag, ls);
        } else {
            flag |= BM_FLAG_UNDEFINED;
        }
        if (inside_line) store_omega(J, line, p, omega, flag);
    }
}


// One block of pixels p0 .. p0+BLOCK-L of line `line` in block mode (the
// paper's L x L moving window, Sec. 3): the rows line-h .. line-h+L-1 of the
// window columns p0-h .. are staged in LDS; each lane sums its block's real
// symmetric T straight from the block's rows (omega_x) and from its columns
// (omega_y) as snapshots, s_k[i] = G[k][t+i] or G[i][t+k] (Eq. 4).
// With the snapshots read in increasing x (or y), omega = +arg of the
// selected root in both directions -- the paper's -arg(z_x) for its
// E{Gamma^H Gamma} form.  With both frequencies, the block phase (Eq. 15's
// alpha, block coordinates measured from the pixel) is
// arg sum_{i,j} G[i][j] e^{-j(omega_x (j-h) + omega_y (i-h))}.
template <int L, int BLOCK, bool JACOBI>
__device__ __forceinline__ void rootmusic_block2d(const RmJob& J, int line, int p0, float2 (*sR)[BLOCK + L],
                                                  const RootTemplate& tmpl, bool full_roots, LaneStats& ls) {
    constexpr int WPB = BLOCK - (L - 1);
    constexpr int h = L / 2;
    const int t = threadIdx.x;
    const int len = J.len, nl = J.nlines;
    const int c0 = p0 - h, r0 = line - h;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int r = r0 + i;
        const bool rin = r >= 0 && r < nl;
        const float2* g = J.gamma + (int64_t)(rin ? r : 0) * J.gamma_ls;
        for (int c = t; c < BLOCK + L - 1; c += BLOCK) {
            const int q = c0 + c;
            sR[i][c] = (rin && q >= 0 && q < len) ? g[q] : make_float2(0.f, 0.f);
        }
    }
    __syncthreads();
    const int p = p0 + t;
    const bool inside_line = (t < WPB) && (p < len);
    const bool valid = inside_line && (c0 + t >= 0) && (c0 + t + L <= len) && (r0 >= 0) && (r0 + L <= nl);
    float wx = __builtin_nanf(""), wy = __builtin_nanf(""), ph = __builtin_nanf("");
    unsigned fx = 0, fy = 0;
    if (valid) {
        if (J.bdirs & BM_DIR_X) {
            Sym<L> T;
            float c1r, c1i, hc, hs;
            T_from_snapshots<L>(L, [&](int k, int i) { return sR[k][t + i]; }, T, c1r, c1i);
            half_angle_of(c1r, c1i, hc, hs);
            if (trace_normalise<L>(T))
                window_omega_Ts<L, JACOBI>(T, hc, hs, tmpl, full_roots, __builtin_nanf(""), wx, fx, ls);
            else fx |= BM_FLAG_UNDEFINED;
        }
        if (J.bdirs & BM_DIR_Y) {
            Sym<L> T;
            float c1r, c1i, hc, hs;
            T_from_snapshots<L>(L, [&](int k, int i) { return sR[i][t + k]; }, T, c1r, c1i);
            half_angle_of(c1r, c1i, hc, hs);
            if (trace_normalise<L>(T))
                window_omega_Ts<L, JACOBI>(T, hc, hs, tmpl, full_roots, __builtin_nanf(""), wy, fy, ls);
            else fy |= BM_FLAG_UNDEFINED;
        }
        if (J.phase && finitef(wx) && finitef(wy)) {
            // the hardware sine and cosine: arguments stay within |w| (L/2) <= 4 pi,
            // where their error (~1e-6) is far below the phase tolerance, and the
            // library's large-argument reduction would hold registers the whole
            // kernel pays for (two waves per SIMD instead of three or four)
            float exr[L], exi[L];
#pragma unroll
            for (int j = 0; j < L; ++j) {
                float sn, cs;
                __sincosf(wx * (float)(j - h), &sn, &cs);
                exr[j] = cs;
                exi[j] = -sn;
            }
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                float rr = 0.f, ri = 0.f;     // sum_j G[i][j] e^{-j wx (j-h)}
#pragma unroll
                for (int j = 0; j < L; ++j) {
                    const float2 v = sR[i][t + j];
                    rr = fmaf(v.x, exr[j], fmaf(-v.y, exi[j], rr));
                    ri = fmaf(v.x, exi[j], fmaf(v.y, exr[j], ri));
                }
                float sn, cs;
                __sincosf(wy * (float)(i - h), &sn, &cs);   // times e^{-j wy (i-h)}
                ar = fmaf(rr, cs, fmaf(ri, sn, ar));
                ai = fmaf(ri, cs, fmaf(-rr, sn, ai));
            }
            ph = atan2f(ai, ar);
        }
    } else {
        fx = fy = BM_FLAG_UNDEFINED;
    }
    if (inside_line) {
        const int64_t o = (int64_t)p * J.out_es + (int64_t)line * J.out_ls;
        if (J.bdirs & BM_DIR_X) J.out[o] = wx;
        if (J.bdirs & BM_DIR_Y) J.out_y[o] = wy;
        if (J.phase) J.phase[o] = ph;
        if (J.flags)
            J.flags[(int64_t)p * J.flag_es + (int64_t)line * J.flag_ls] =
                (uint8_t)(((J.bdirs & BM_DIR_X) ? fx : 0u) | (((J.bdirs & BM_DIR_Y) ? fy : 0u) << 4));
    }
}

template <int BLOCK>
__device__ __forceinline__ void flush_stats(const LaneStats& ls, unsigned long long* stats) {
    unsigned long long a[kStatFields] = {(unsigned long long)ls.counted, (unsigned long long)ls.eig_its,
                                         (unsigned long long)ls.iters, (unsigned long long)ls.pfail,
                                         (unsigned long long)ls.accepted, (unsigned long long)ls.rejected,
                                         (unsigned long long)ls.pair_its, (unsigned long long)ls.pair_its32,
                                         (unsigned long long)ls.power};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < kStatFields; ++c) a[c] += __shfl_xor(a[c], off);
    if ((threadIdx.x & 63) == 0) {
        // spread the counters over kStatSlots slots to avoid one hot address
        unsigned long long* sl =
            stats + kStatFields * ((blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6)) % kStatSlots);
#pragma unroll
        for (int c = 0; c < kStatFields; ++c)
            if (a[c]) atomicAdd(sl + c, a[c]);
    }
}

// Grid-stride loop over the work items of every job of one L: item w is
// block (w - prefix[j]) of job j, i.e. line (w - prefix[j]) / bpl and window
// block (w - prefix[j]) % bpl.  A grid of one block per item runs each item
// once; a smaller (persistent) grid walks the list.
// Without the statistics counters the L <= 6 line kernels fit five waves per
// SIMD (96 VGPRs, a few spilled), 1.3% faster on L = 6 than the four that 119
// VGPRs allow, and the L = 7, 8 ones four (128 VGPRs; L = 8 spills seven and
// runs 3% faster than at the three waves of its 151).  The block-window
// kernels run four too (L = 7: 143 -> 128 VGPRs with no spill, 11% faster;
// L = 8: 160 -> 128 with 14 spilled, 8% faster).
// Block windows above 8 x 8 (odd sizes to 17 x 17) run 128 lanes per block at
// one wave per SIMD: the per-lane T, the degree 2L-2 polynomial and the FP64
// certificate need up to 512 VGPRs.
// WARM: line windows may read a previous-frame map (the other build folds the
// warm-start branch away: four fewer spilled registers at L = 8).
// LOOP = false (line windows): one block per work item (grid = total), no
// grid-stride loop; the loop keeps values live across items that cost the
// L = 6 and 8 line kernels 40-50 spilled registers.
template <int L, int BLOCK, bool STATS, bool JACOBI, bool BLOCKWIN, bool WARM = false, bool LOOP = true>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu((!STATS && L <= kMaxL) ? (BLOCKWIN ? 4 : (L <= 6 ? 5 : 4)) : 1)))
void rootmusic_kernel(RmBatch B) {
    // line windows: staged signal + lag sums; block windows: the block's staged rows
    constexpr int ROW = BLOCKWIN ? BLOCK + L : LineSpan<L, BLOCK>::row;
    constexpr int WPB = BLOCKWIN ? BLOCK - (L - 1) : LineSpan<L, BLOCK>::wpb;
    __shared__ float2 sg[BLOCKWIN ? 1 : 4 * LineSpan<L, BLOCK>::quarter];
    __shared__ __align__(16) float2 sS[L][ROW];
    LaneStats ls;
    // LOOP = false: exactly one item, blockIdx.x (a trip count of one the compiler sees)
    const int wend = LOOP ? B.total : (int)blockIdx.x + 1;
    const int wstep = LOOP ? (int)gridDim.x : 1;
    for (int w = blockIdx.x; w < wend; w += wstep) {
        const int j = find_job(B.prefix, B.njobs, w);
        const RmJob J = B.jobs[j];
        const int local = w - B.prefix[j];
        const int line = local / J.bpl;
        const int bx = local - line * J.bpl;
        // line and block windows are separate instantiations, so that neither
        // pays the other's registers
        if constexpr (BLOCKWIN)
            rootmusic_block2d<L, BLOCK, JACOBI>(J, line, bx * WPB, sS, B.tmpl, B.full_roots != 0, ls);
        else
            rootmusic_block<L, BLOCK, JACOBI, WARM>(J, line, bx * WPB, sg, sS, B.tmpl, B.full_roots != 0, ls);
        __syncthreads();
    }
    if (STATS) flush_stats<BLOCK>(ls, B.stats);
}

// Plain root-MUSIC on a list of windows (job, line, pixel), one lane each,
// with the covariance summed directly from the analytic signal.
template <int L, bool STATS, bool JACOBI>
__global__ __launch_bounds__(kGatherBlock) void rootmusic_gather_kernel(RmBatch B, const int2* list,
                                                                        const unsigned long long* count) {
    const unsigned long long cnt = *count;
    LaneStats ls;
    for (unsigned long long e = (unsigned long long)blockIdx.x * kGatherBlock + threadIdx.x; e < cnt;
         e += (unsigned long long)gridDim.x * kGatherBlock) {
        const int2 en = list[e];
        const RmJob J = B.jobs[en.x];
        const int line = (int)((unsigned)en.y >> 16), p = en.y & 0xFFFF;
        const int N = J.N;
        const int K = N - L + 1;
        const float2* g = J.gamma + (int64_t)line * J.gamma_ls + (p - (N >> 1));
        Cov<L> R;
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int j = i; j < L; ++j) { R.re[i][j] = 0.f; R.im[i][j] = 0.f; }
        float2 win[L];
#pragma unroll
        for (int d = 0; d < L - 1; ++d) win[d + 1] = g[d];
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int d = 0; d < L - 1; ++d) win[d] = win[d + 1];
            win[L - 1] = g[k + L - 1];
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
                for (int jj = i; jj < L; ++jj) {
                    R.re[i][jj] = fmaf(win[i].x, win[jj].x, fmaf(win[i].y, win[jj].y, R.re[i][jj]));
                    if (i != jj) R.im[i][jj] = fmaf(win[i].y, win[jj].x, fmaf(-win[i].x, win[jj].y, R.im[i][jj]));
                }
        }
        float omega = __builtin_nanf("");
        unsigned flag = 0;
        window_omega<L, JACOBI>(R, B.tmpl, B.full_roots != 0, K, __builtin_nanf(""), omega, flag, ls);
        store_omega(J, line, p, omega, flag);
    }
    if (STATS) flush_stats<kGatherBlock>(ls, B.stats);
}

template <int L, int BLOCK, bool JACOBI, bool WARM>
hipError_t launch_LBJW(const RmBatch& b, int grid, hipStream_t s) {
    if (b.stats)
        hipLaunchKernelGGL((rootmusic_kernel<L, BLOCK, true, JACOBI, false, WARM>), dim3(grid), dim3(BLOCK), 0, s, b);
    else if (grid < b.total)
        hipLaunchKernelGGL((rootmusic_kernel<L, BLOCK, false, JACOBI, false, WARM>), dim3(grid), dim3(BLOCK), 0, s,
                           b);
    else
        hipLaunchKernelGGL((rootmusic_kernel<L, BLOCK, false, JACOBI, false, WARM, false>), dim3(b.total),
                           dim3(BLOCK), 0, s, b);
    return hipGetLastError();
}

template <int L, int BLOCK, bool JACOBI>
hipError_t launch_LBJ(const RmBatch& b, int grid, hipStream_t s) {
    return b.warm ? launch_LBJW<L, BLOCK, JACOBI, true>(b, grid, s) : launch_LBJW<L, BLOCK, JACOBI, false>(b, grid, s);
}

// Block windows: 256 lanes per block (128 above 8 x 8).
template <int L, bool JACOBI>
hipError_t launch_block_LJ(const RmBatch& b, int grid, hipStream_t s) {
    constexpr int BL = block_window_lanes(L);
    if (b.stats)
        hipLaunchKernelGGL((rootmusic_kernel<L, BL, true, JACOBI, true>), dim3(grid), dim3(BL), 0, s, b);
    else
        hipLaunchKernelGGL((rootmusic_kernel<L, BL, false, JACOBI, true>), dim3(grid), dim3(BL), 0, s, b);
    return hipGetLastError();
}

// Block windows above 8 x 8: the tridiagonal solver only.
template <int L>
hipError_t launch_big_block(const RmBatch& b, int grid, hipStream_t s) {
    if (!b.block_windows) return hipErrorInvalidValue;
    return launch_block_LJ<L, false>(b, grid, s);
}

// Line and block windows up to 8 x 8 of one eigen solver (JACOBI or the
// default route), one translation unit each.
template <int L, bool JACOBI>
hipError_t launch_LJ(const RmBatch& b, int block, int grid, hipStream_t s) {
    if (b.block_windows) return launch_block_LJ<L, JACOBI>(b, grid, s);
    if (block == 128) return launch_LBJ<L, 128, JACOBI>(b, grid, s);
    return launch_LBJ<L, 256, JACOBI>(b, grid, s);
}

template <bool JACOBI>
hipError_t launch_rootmusic_J(int L, const RmBatch& b, int block, int grid, hipStream_t s) {
    switch (L) {
        case 2: return launch_LJ<2, JACOBI>(b, block, grid, s);
        case 3: return launch_LJ<3, JACOBI>(b, block, grid, s);
        case 4: return launch_LJ<4, JACOBI>(b, block, grid, s);
        case 5: return launch_LJ<5, JACOBI>(b, block, grid, s);
        case 6: return launch_LJ<6, JACOBI>(b, block, grid, s);
        case 7: return launch_LJ<7, JACOBI>(b, block, grid, s);
        case 8: return launch_LJ<8, JACOBI>(b, block, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <int L, bool JACOBI>
hipError_t launch_gather_LJ(const RmBatch& b, const int2* list, const unsigned long long* count, int grid, hipStream_t s) {
    if (b.stats)
        hipLaunchKernelGGL((rootmusic_gather_kernel<L, true, JACOBI>), dim3(grid), dim3(kGatherBlock), 0, s, b, list,
                           count);
    else
        hipLaunchKernelGGL((rootmusic_gather_kernel<L, false, JACOBI>), dim3(grid), dim3(kGatherBlock), 0, s, b,
                           list, count);
    return hipGetLastError();
}



}  // namespace
}  // namespace bm
