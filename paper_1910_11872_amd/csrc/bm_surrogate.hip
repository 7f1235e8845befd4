// Learned surrogate of the per-window frequency estimate (an addition to the
// paper's method), with the paper's root-MUSIC as the check and the fallback.
//
// surrogate_kernel: the plain line kernel's blocks (two window starts per
// lane, lag sums shared through LDS), with a cheaper route to the signal
// subspace where the network's estimate allows it:
//   1. stage the analytic signal of the block in LDS;
//   2. features of every 8th window: 16 central samples, de-rotated by the
//      phase of the central sample, divided by the window's RMS magnitude, as
//      bfloat16 [Re(16), Im(16)];
//   3. MLP 32 -> GELU 64 -> GELU 64 -> 2 on the matrix cores: every GEMM is
//      a set of v_mfma_f32_16x16x32_bf16 tiles with FP32 accumulation, in
//      transposed form (W^T X^T) so that the bfloat16 weights are the A
//      operand and each layer's output tile is the next layer's B operand
//      after one LDS round trip; omega_hat = atan2 of the two outputs;
//   4. lag sums, covariance and the real symmetric T = Q^H R_fb Q as in the
//      plain kernel; the top eigenvector by power iteration from the steering
//      vector of omega_hat, accepted once an a-posteriori bound proves it
//      within 1e-5 of the eigenvector and the MUSIC null spectrum at
//      omega_hat is below tau; otherwise the plain eigen-split (Householder,
//      Newton, inverse iteration);
//   5. the plain path's polynomial, certified root pair (or all roots) and
//      omega = arg(z1 + z2) either way.
// A better prediction needs fewer power steps; a window the prediction does
// not serve is computed by the plain path in the same lane.
#include "bm_rootmusic_kernels.h"

#include <algorithm>

namespace bm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kSurBlock = 256;
constexpr int kPredictStride = 32;    // one network prediction per this many windows
// predictions per block, in 16-window MLP tiles
constexpr int kPredictions = (2 * kSurBlock / kPredictStride + 15) / 16 * 16;
constexpr int kPredictTiles = kPredictions / 16;
static_assert(kPredictions <= 16 * (kSurBlock / 64), "at most one output tile per wave");
static_assert(kSurBlock % kPredictions == 0 && 16 % (kSurBlock / kPredictions) == 0,
              "lanes per prediction: a power of two that divides the 16 feature samples");

// C(16 x 16) += A(16 x 32) B(32 x 16) on one wave.  A(i, k) = a[i*lda + k],
// B(k, j) = b[j*ldb + k]; both 16-byte aligned with k contiguous.  Lane l
// supplies row l%16 of A and column l%16 of B for k = 8(l/16) .. 8(l/16)+7;
// the result holds column l%16, rows 4(l/16) .. 4(l/16)+3.
__device__ __forceinline__ floatx4 mfma_tile(const __bf16* a, int lda, const __bf16* b, int ldb, floatx4 c) {
    const int l = threadIdx.x & 63;
    const int i = l & 15, kg = (l >> 4) * 8;
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + i * lda + kg);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(b + i * ldb + kg);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

// erf by Abramowitz and Stegun, Handbook of Mathematical Functions, 7.1.26:
// erf(x) = 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x), x >= 0,
// absolute error below 1.5e-7 (plus the hardware reciprocal and exp2
// roundings), extended as an odd function.  A GELU evaluated with it is
// exact to well under one bfloat16 unit, the precision of the activations.
__device__ __forceinline__ float erf_as(float x) {
    const float a = fabsf(x);
    const float t = frcp(fmaf(0.3275911f, a, 1.f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    p *= t;
    const float e = __builtin_amdgcn_exp2f(-1.44269504088896341f * a * a);
    return copysignf(fmaf(-p, e, 1.f), x);
}

__device__ __forceinline__ float gelu(float x) {
    const float h = 0.5f * x;
    return fmaf(h, erf_as(x * 0.70710678118654752f), h);
}

struct alignas(16) MlpSmem {
    __bf16 w1t[kMlpHidden * kMlpIn];
    __bf16 w2t[kMlpHidden * kMlpHidden];
    __bf16 w3t[16 * kMlpHidden];
    float b1[kMlpHidden], b2[kMlpHidden], b3[4];
};

// 16-byte copies (n16 of them); both pointers 16-byte aligned.
__device__ __forceinline__ void copy16(const __bf16* src, __bf16* dst, int n16, int nthreads) {
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    for (int i = threadIdx.x; i < n16; i += nthreads) d4[i] = s4[i];
}

// The weights into LDS (the bfloat16 matrices 16-byte aligned in device memory).
__device__ void load_weights(const MlpWeights& w, MlpSmem& s, int nthreads) {
    copy16(w.w1t, s.w1t, kMlpHidden * kMlpIn / 8, nthreads);
    copy16(w.w2t, s.w2t, kMlpHidden * kMlpHidden / 8, nthreads);
    // W3^T: its two rows, and zeros for the padding rows of the 16-row tile
    copy16(w.w3t, s.w3t, kMlpOut * kMlpHidden / 8, nthreads);
    for (int i = threadIdx.x; i < (16 - kMlpOut) * kMlpHidden / 8; i += nthreads)
        reinterpret_cast<uint4*>(s.w3t + kMlpOut * kMlpHidden)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int i = threadIdx.x; i < kMlpHidden; i += nthreads) {
        s.b1[i] = w.b1[i];
        s.b2[i] = w.b2[i];
    }
    if (threadIdx.x < 2) s.b3[threadIdx.x] = w.b3[threadIdx.x];
}

// LDS written by this wave is visible to all its lanes: the workgroup-scope
// fence waits for the wave's own LDS stores; no other wave is waited for.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// MLP on one tile of 16 rows of x ([row][32] bf16, written by this wave or
// before a block barrier); h1, h2 are this wave's [16][64] bf16 scratch
// tiles.  Wave-local: no block barrier.  Lanes 0..15 return (y0, y1) of row l.
__device__ __forceinline__ float2 mlp_tile(const MlpSmem& s, const __bf16* x, __bf16* h1, __bf16* h2) {
    const int l = threadIdx.x & 63;
    const int col = l & 15, rq = (l >> 4) * 4;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma_tile(s.w1t + 16 * rb * kMlpIn, kMlpIn, x, kMlpIn, c);
        // this lane's four outputs are adjacent hidden units: one 8-byte store
        const int hid = 16 * rb + rq;
        bf16x4 hv;
#pragma unroll
        for (int q = 0; q < 4; ++q) hv[q] = (__bf16)gelu(c[q] + s.b1[hid + q]);
        *reinterpret_cast<bf16x4*>(h1 + col * kMlpHidden + hid) = hv;
    }
    wave_lds_sync();
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            c = mfma_tile(s.w2t + 16 * rb * kMlpHidden + 32 * kb, kMlpHidden, h1 + 32 * kb, kMlpHidden, c);
        const int hid = 16 * rb + rq;
        bf16x4 hv;
#pragma unroll
        for (int q = 0; q < 4; ++q) hv[q] = (__bf16)gelu(c[q] + s.b2[hid + q]);
        *reinterpret_cast<bf16x4*>(h2 + col * kMlpHidden + hid) = hv;
    }
    wave_lds_sync();
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) c = mfma_tile(s.w3t + 32 * kb, kMlpHidden, h2 + 32 * kb, kMlpHidden, c);
    return make_float2(c[0] + s.b3[0], c[1] + s.b3[1]);
}

// MLP on T tiles of 16 rows of x ([row][32] bf16, LDS) by the block's four
// waves together: wave w computes hidden units 16w .. 16w+15 of every tile in
// both hidden layers, so each wave takes a quarter of the GELUs and needs only
// its own 16 rows of W1^T and W2^T, read as MFMA A operands straight from
// device memory (the 14 KiB of weights stay in the caches); the output layer
// runs on the first T waves.  h1, h2: [T][16][64] bf16 in LDS.  Lanes 0..15
// of wave j < T write what[16 j + l] = atan2(y1, y0) of row 16 j + l.
template <int T>
__device__ __forceinline__ void mlp_block(const MlpWeights& w, const __bf16* x, __bf16* h1, __bf16* h2, float* what) {
    static_assert(kSurBlock / 64 * 16 == kMlpHidden, "one 16-unit slice of each hidden layer per wave");
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = l & 15, hid = 16 * wv + (l >> 4) * 4;
    const float4 b1 = *reinterpret_cast<const float4*>(w.b1 + hid);
    const float4 b2 = *reinterpret_cast<const float4*>(w.b2 + hid);
#pragma unroll
    for (int j = 0; j < T; ++j) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma_tile(w.w1t + 16 * wv * kMlpIn, kMlpIn, x + 16 * j * kMlpIn, kMlpIn, c);
        bf16x4 hv;
        hv[0] = (__bf16)gelu(c[0] + b1.x);
        hv[1] = (__bf16)gelu(c[1] + b1.y);
        hv[2] = (__bf16)gelu(c[2] + b1.z);
        hv[3] = (__bf16)gelu(c[3] + b1.w);
        *reinterpret_cast<bf16x4*>(h1 + (16 * j + col) * kMlpHidden + hid) = hv;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < T; ++j) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            c = mfma_tile(w.w2t + 16 * wv * kMlpHidden + 32 * kb, kMlpHidden, h1 + 16 * j * kMlpHidden + 32 * kb,
                          kMlpHidden, c);
        bf16x4 hv;
        hv[0] = (__bf16)gelu(c[0] + b2.x);
        hv[1] = (__bf16)gelu(c[1] + b2.y);
        hv[2] = (__bf16)gelu(c[2] + b2.z);
        hv[3] = (__bf16)gelu(c[3] + b2.w);
        *reinterpret_cast<bf16x4*>(h2 + (16 * j + col) * kMlpHidden + hid) = hv;
    }
    __syncthreads();
    if (wv < T) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            c = mfma_tile(w.w3t + 32 * kb, kMlpHidden, h2 + 16 * wv * kMlpHidden + 32 * kb, kMlpHidden, c);
        if (l < 16) what[16 * wv + l] = atan2f(c[1] + w.b3[1], c[0] + w.b3[0]);
    }
}

template <int L, bool STATS>
__global__ __launch_bounds__(kSurBlock)
__attribute__((amdgpu_waves_per_eu(STATS ? 1 : 4)))
void surrogate_kernel(SurBatch S) {
    constexpr int BLOCK = kSurBlock;
    constexpr int SPAN = LineSpan<L, BLOCK>::span;
    constexpr int WPB = LineSpan<L, BLOCK>::wpb;
    constexpr int ROW = LineSpan<L, BLOCK>::row;
    constexpr int NP = kPredictions;
    static_assert(NP * kPredictStride >= SPAN, "the predictions cover the block's windows");
    __shared__ float2 sg[SPAN + kMaxN];
    __shared__ float what[NP];
    // the MLP's features and hidden tiles, later the lag sums
    constexpr int kXBytes = NP * kMlpIn * 2, kHBytes = 2 * NP * kMlpHidden * 2;
    constexpr int kSBytes = L * ROW * 8;
    constexpr int kMBytes = kXBytes + kHBytes;
    __shared__ alignas(16) unsigned char ubuf[kMBytes > kSBytes ? kMBytes : kSBytes];
    __bf16* xs = reinterpret_cast<__bf16*>(ubuf);
    float2 (*sS)[ROW] = reinterpret_cast<float2 (*)[ROW]>(ubuf);
    const int t = threadIdx.x;
    __bf16* h1 = reinterpret_cast<__bf16*>(ubuf + kXBytes);
    __bf16* h2 = h1 + NP * kMlpHidden;

    const RmBatch& B = S.rm;
    const int j = find_job(B.prefix, B.njobs, blockIdx.x);
    const RmJob J = B.jobs[j];
    const int local = blockIdx.x - B.prefix[j];
    const int line = local / J.bpl;
    const int p0 = (local - line * J.bpl) * WPB;
    const int N = J.N, half = N >> 1, K = N - L + 1, len = J.len;
    const float2* g = J.gamma + (int64_t)line * J.gamma_ls;
    const int base = p0 - half;
    for (int i = t; i < SPAN + N - 1; i += BLOCK) {
        const int q = base + i;
        sg[i] = (q >= 0 && q < len) ? g[q] : make_float2(0.f, 0.f);
    }
    __syncthreads();

    // ---- features and the MLP ------------------------------------------
    // The local frequency varies slowly along a line and the prediction only
    // seeds the power iteration, so the network runs on every
    // kPredictStride-th window: prediction k is made at window
    // kPredictStride k + kPredictStride/2 (moved inside the block's valid
    // windows) and serves windows kPredictStride k .. kPredictStride (k+1) - 1.
    // LPW lanes make the features of one prediction (a share of the energy
    // sum and 16/LPW of the 16 samples each); the whole block runs the MLP.
    if (S.predictor == 0) {
        constexpr int LPW = BLOCK / NP, SPL = 16 / LPW;
        const int lo = max(0, half - p0);
        const int hi = min(min(WPB - 1, len - 1 - p0), len - N + half - p0);
        const int k = t / LPW, q = t % LPW;
        const int pos = min(max(kPredictStride * k + kPredictStride / 2, lo), max(hi, lo));
        const float2* w = sg + pos;
        float e = 0.f;
        for (int i = q; i < N; i += LPW) e = fmaf(w[i].x, w[i].x, fmaf(w[i].y, w[i].y, e));
#pragma unroll
        for (int off = 1; off < LPW; off <<= 1) e += __shfl_xor(e, off);
        const float2 gc = w[half];
        const float mc = fsqrt(gc.x * gc.x + gc.y * gc.y);
        const bool ok = hi >= lo && mc > 0.f && e > 0.f;
        const float sc = ok ? frcp(mc) * frsq(e / (float)N) : 0.f;
        const float rc = gc.x * sc, rs = -gc.y * sc;               // conj(gc)/|gc|/rms
#pragma unroll
        for (int m = 0; m < SPL; ++m) {
            const int i = q * SPL + m;
            const float2 v = w[half - 8 + i];
            xs[k * kMlpIn + i] = (__bf16)(v.x * rc - v.y * rs);
            xs[k * kMlpIn + 16 + i] = (__bf16)(v.x * rs + v.y * rc);
        }
        __syncthreads();
        mlp_block<kPredictTiles>(S.w, xs, h1, h2, what);
    }
    __syncthreads();
    // ---- lag sums (the MLP scratch is dead: every wave passed the barrier) ---
    lag_sums_pair<L, ROW>(sg, 2 * t, K, sS);
    __syncthreads();

    LaneStats ls;
#pragma unroll 1
    for (int r = 0; r < 2; ++r) {
        const int s = r * BLOCK + t;
        const int p = p0 + s;
        const bool inside_line = (s < WPB) && (p < len);
        const bool valid = inside_line && (p - half >= 0) && (p - half + N <= len);
        float omega = __builtin_nanf("");
        unsigned flag = 0;
        if (valid) {
            Cov<L> R;
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
                for (int jj = i; jj < L; ++jj) {
                    const float2 v = sS[jj - i][s + i];
                    R.re[i][jj] = v.x;
                    R.im[i][jj] = (i == jj) ? 0.f : v.y;
                }
            // the prediction's e^{j w_hat / 2}
            float hc, hs;
            if (S.predictor == 0) __sincosf(0.5f * what[min(NP - 1, s / kPredictStride)], &hs, &hc);
            else lag1_half_angle<L>(R, hc, hs);
            Sym<L> T;
            if (!normalised_T<L>(R, T)) {
                flag |= BM_FLAG_UNDEFINED;
            } else {
                ls.counted += 1;
                float v[L], nu = 1.f;
                int steps = 0;
                const bool good =
                    power_top_eigvec<L>(T, hc, hs, kPowerMinSteps, kPowerMaxSteps, kPowerTol, v, steps, nu) &&
                    nu <= S.tau;
                if (good) {
                    ls.power += 1;
                    ls.eig_its += steps;
                }
                // the surrogate's own counters: windows the prediction served, and the rest
                const int a0 = ls.accepted, r0 = ls.rejected;
                if (good || signal_eigvec_T<L, false>(T, v, flag, ls))
                    window_omega_v<L>(v, B.tmpl, B.full_roots != 0, __builtin_nanf(""), omega, flag, ls);
                ls.accepted = a0 + (good ? 1 : 0);
                ls.rejected = r0 + (good ? 0 : 1);
            }
        } else {
            flag |= BM_FLAG_UNDEFINED;
        }
        if (inside_line) store_omega(J, line, p, omega, flag);
    }
    if (STATS) flush_stats<BLOCK>(ls, B.stats);
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpWeights w, const float* X, float* Y, int M) {
    __shared__ MlpSmem sm;
    __shared__ alignas(16) __bf16 xs[64 * kMlpIn];
    __shared__ alignas(16) __bf16 hs[4][2][16 * kMlpHidden];
    load_weights(w, sm, 256);
    const int t = threadIdx.x, wv = t >> 6;
    const int r0 = blockIdx.x * 64;
    for (int i = t; i < 64 * kMlpIn; i += 256) {
        const int r = r0 + i / kMlpIn;
        xs[i] = (__bf16)(r < M ? X[(int64_t)r0 * kMlpIn + i] : 0.f);
    }
    __syncthreads();
    const float2 y = mlp_tile(sm, xs + wv * 16 * kMlpIn, hs[wv][0], hs[wv][1]);
    const int r = r0 + wv * 16 + (t & 15);
    if ((t & 63) < 16 && r < M) {
        Y[2 * (int64_t)r] = y.x;
        Y[2 * (int64_t)r + 1] = y.y;
    }
}


// ===========================================================================
// Training: data generation, forward/backward on the matrix cores, Adam
// ===========================================================================

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): words 0 and
// 2 are multiplied by the round constants, the high halves are crossed with
// words 1 and 3 and the key, and the key is bumped by the Weyl constants
// between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

__device__ __forceinline__ float u01(uint32_t u) { return ((float)u + 0.5f) * 2.3283064365386963e-10f; }

// Training line id (first + blockIdx.x): 0.5 + 0.4 cos(w n + theta) + noise,
// parameters from counter (id, 0, 0, 0), noise of samples 4b..4b+3 from
// counter (id, b+1, 0, 0) by two Box-Muller pairs.  One block of 32 lanes per line.
__global__ __launch_bounds__(32) void gen_lines_kernel(float* lines, long long first, unsigned long long seed) {
    const uint32_t id = (uint32_t)(first + blockIdx.x);
    const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
    const uint4 pr = philox4x32_10(make_uint4(id, 0u, 0u, 0u), key);
    const float kTwoPi = 6.28318530717958648f;
    const float w = kTwoPi / 16.f + u01(pr.x) * (kTwoPi / 4.f - kTwoPi / 16.f);
    const float th = kTwoPi * u01(pr.y);
    const float snr = 30.f * u01(pr.z);
    const float sig = sqrtf(0.08f * exp10f(-0.1f * snr));
    const int b = threadIdx.x;
    const uint4 q = philox4x32_10(make_uint4(id, (uint32_t)b + 1u, 0u, 0u), key);
    const float r0 = sqrtf(-2.f * logf(u01(q.x))), r1 = sqrtf(-2.f * logf(u01(q.z)));
    float s0, c0, s1, c1;
    sincosf(kTwoPi * u01(q.y), &s0, &c0);
    sincosf(kTwoPi * u01(q.w), &s1, &c1);
    const float z[4] = {r0 * c0, r0 * s0, r1 * c1, r1 * s1};
    float* out = lines + (int64_t)blockIdx.x * 128;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int n = 4 * b + i;
        out[n] = 0.5f + 0.4f * cosf(w * (float)n + th) + sig * z[i];
    }
}

// Entries {job, line << 16 | 64} of the label windows (centre of each line),
// 65536 lines per job.
__global__ void label_entries_kernel(int2* list, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) list[i] = make_int2(i >> 16, (int)(((unsigned)(i & 0xFFFF) << 16) | 64u));
}

// Features of the 32-sample window centred on sample 64 of each line, and the
// target (cos w, sin w) of its label.
__global__ void train_features_kernel(const float2* gamma, int count, const float* labels, float* X, float* T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float2* w = gamma + (int64_t)i * 128 + 48;
    float e = 0.f;
    for (int k = 0; k < 32; ++k) e = fmaf(w[k].x, w[k].x, fmaf(w[k].y, w[k].y, e));
    const float2 gc = w[16];
    const float mc = sqrtf(gc.x * gc.x + gc.y * gc.y);
    const float sc = (mc > 0.f && e > 0.f) ? 1.f / (mc * sqrtf(e / 32.f)) : 0.f;
    const float rc = gc.x * sc, rs = -gc.y * sc;
    float* x = X + (int64_t)i * kMlpIn;
    for (int k = 0; k < 16; ++k) {
        const float2 v = w[8 + k];
        x[k] = v.x * rc - v.y * rs;
        x[16 + k] = v.x * rs + v.y * rc;
    }
    float sw, cw;
    sincosf(labels[i], &sw, &cw);
    T[2 * (int64_t)i] = cw;
    T[2 * (int64_t)i + 1] = sw;
}

constexpr int kTrainChunk = 64;     // samples per block iteration (4 waves x 16)
// per-block partial layout: dW1^T [64][32], db1 [64], dW2^T [64][64], db2 [64], dW3^T [2][64], db3 [2], loss
constexpr int kPartDW1 = 0, kPartDB1 = 2048, kPartDW2 = 2112, kPartDB2 = 6208, kPartDW3 = 6272, kPartDB3 = 6400,
              kPartLoss = 6402, kPartStride = 6404;

__device__ __forceinline__ float gelu_grad(float x) {
    return fmaf(0.5f, erf_as(x * 0.70710678118654752f), 0.5f) +
           x * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x);
}

struct alignas(16) TrainSmem {
    __bf16 w1t[64 * 32], w2t[64 * 64], w3t[16 * 64], w2[64 * 64];
    float b1[64], b2[64], b3[4];
    __bf16 x[64 * 32], xT[32 * 64];
    __bf16 h1[64 * 64], h1T[64 * 64], h2[64 * 64], h2T[64 * 64];
    __bf16 dz2[64 * 64], dz2T[64 * 64], dz1T[64 * 64];
    __bf16 dyT[16 * 64];
    float dy[64 * 2];
    float red[4][2 * 64 + 2 + 1];
};

// Forward and backward of M samples (M a multiple of 64), gradients of the
// mean squared error summed per block into `part` (kPartStride floats per block).
__global__ __launch_bounds__(256) void mlp_train_kernel(MlpWeights w, const __bf16* w2, const float* X, const float* T,
                                                         int M, float* part) {
    __shared__ TrainSmem sm;
    const int t = threadIdx.x, wv = t >> 6, l = t & 63, col = l & 15, rq = (l >> 4) * 4;
    for (int i = t; i < 64 * 32; i += 256) { sm.w1t[i] = w.w1t[i]; }
    for (int i = t; i < 64 * 64; i += 256) { sm.w2t[i] = w.w2t[i]; sm.w2[i] = w2[i]; }
    for (int i = t; i < 16 * 64; i += 256) { sm.w3t[i] = w.w3t[i]; sm.dyT[i] = (__bf16)0.f; }
    if (t < 64) { sm.b1[t] = w.b1[t]; sm.b2[t] = w.b2[t]; }
    if (t < 2) sm.b3[t] = w.b3[t];
    const float inv = 2.f / (float)M;
    floatx4 acc[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) acc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
    float db1[16], db2[16], db3[2] = {0.f, 0.f}, lsum = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) { db1[k] = 0.f; db2[k] = 0.f; }
    __syncthreads();
    const int r0 = wv * 16;     // this wave's rows in the chunk
    for (int c0 = blockIdx.x * kTrainChunk; c0 < M; c0 += gridDim.x * kTrainChunk) {
        for (int i = t; i < 64 * 32; i += 256) {
            const __bf16 v = (__bf16)X[(int64_t)c0 * 32 + i];
            sm.x[i] = v;
            sm.xT[(i % 32) * 64 + i / 32] = v;
        }
        __syncthreads();
        // ---- forward ----------------------------------------------------
        float z1[4][4], z2[4][4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            floatx4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma_tile(sm.w1t + 16 * rb * 32, 32, sm.x + r0 * 32, 32, c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int hid = 16 * rb + rq + q, win = r0 + col;
                z1[rb][q] = c[q] + sm.b1[hid];
                const __bf16 hv = (__bf16)gelu(z1[rb][q]);
                sm.h1[win * 64 + hid] = hv;
                sm.h1T[hid * 64 + win] = hv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                c = mfma_tile(sm.w2t + 16 * rb * 64 + 32 * kb, 64, sm.h1 + r0 * 64 + 32 * kb, 64, c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int hid = 16 * rb + rq + q, win = r0 + col;
                z2[rb][q] = c[q] + sm.b2[hid];
                const __bf16 hv = (__bf16)gelu(z2[rb][q]);
                sm.h2[win * 64 + hid] = hv;
                sm.h2T[hid * 64 + win] = hv;
            }
        }
        __syncthreads();
        {
            floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                c = mfma_tile(sm.w3t + 32 * kb, 64, sm.h2 + r0 * 64 + 32 * kb, 64, c);
            if (l < 16) {
                const int win = r0 + l;
                const int64_t gi = (int64_t)(c0 + win) * 2;
                const float e0 = c[0] + sm.b3[0] - T[gi], e1 = c[1] + sm.b3[1] - T[gi + 1];
                lsum += e0 * e0 + e1 * e1;
                sm.dy[win * 2] = inv * e0;
                sm.dy[win * 2 + 1] = inv * e1;
                sm.dyT[0 * 64 + win] = (__bf16)(inv * e0);
                sm.dyT[1 * 64 + win] = (__bf16)(inv * e1);
                db3[0] += inv * e0;
                db3[1] += inv * e1;
            }
        }
        __syncthreads();
        // ---- backward: dZ2 = (dY W3^T) * gelu'(Z2) on the vector units ---------
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int hid = 16 * rb + rq + q, win = r0 + col;
                const float dh = sm.dy[win * 2] * (float)sm.w3t[hid] + sm.dy[win * 2 + 1] * (float)sm.w3t[64 + hid];
                const float dz = dh * gelu_grad(z2[rb][q]);
                db2[rb * 4 + q] += dz;
                const __bf16 dv = (__bf16)dz;
                sm.dz2[win * 64 + hid] = dv;
                sm.dz2T[hid * 64 + win] = dv;
            }
        __syncthreads();
        // dH1^T = W2 dZ2^T (A = W2 [in][out], k = out contiguous), dZ1 = dH1 * gelu'(Z1)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                c = mfma_tile(sm.w2 + 16 * rb * 64 + 32 * kb, 64, sm.dz2 + r0 * 64 + 32 * kb, 64, c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int hid = 16 * rb + rq + q, win = r0 + col;
                const float dz = c[q] * gelu_grad(z1[rb][q]);
                db1[rb * 4 + q] += dz;
                sm.dz1T[hid * 64 + win] = (__bf16)dz;
            }
        }
        __syncthreads();
        // ---- weight gradients over the 64 samples: 28 tiles, 7 per wave -----
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const int tile = wv + 4 * k;
            const __bf16 *a, *b;
            if (tile < 8) {            // dW1^T [64 out][32 in]
                a = sm.dz1T + 16 * (tile >> 1) * 64;
                b = sm.xT + 16 * (tile & 1) * 64;
            } else if (tile < 24) {    // dW2^T [64 out][64 in]
                a = sm.dz2T + 16 * ((tile - 8) >> 2) * 64;
                b = sm.h1T + 16 * ((tile - 8) & 3) * 64;
            } else {                   // dW3^T [16 (2) out][64 in]
                a = sm.dyT;
                b = sm.h2T + 16 * (tile - 24) * 64;
            }
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) acc[k] = mfma_tile(a + 32 * kb, 64, b + 32 * kb, 64, acc[k]);
        }
        __syncthreads();
    }
    // ---- per-block partial sums ---------------------------------------------
    float* P = part + (int64_t)blockIdx.x * kPartStride;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int tile = wv + 4 * k;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rq + q;     // within the 16-row tile
            if (tile < 8) P[kPartDW1 + (16 * (tile >> 1) + row) * 32 + 16 * (tile & 1) + col] = acc[k][q];
            else if (tile < 24)
                P[kPartDW2 + (16 * ((tile - 8) >> 2) + row) * 64 + 16 * ((tile - 8) & 3) + col] = acc[k][q];
            else if (row < 2)
                P[kPartDW3 + row * 64 + 16 * (tile - 24) + col] = acc[k][q];
        }
    }
    // bias sums: reduce over the 16 lanes sharing rq (different samples), then over waves
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            db1[k] += __shfl_xor(db1[k], off);
            db2[k] += __shfl_xor(db2[k], off);
        }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
        db3[0] += __shfl_xor(db3[0], off);
        db3[1] += __shfl_xor(db3[1], off);
        lsum += __shfl_xor(lsum, off);
    }
    if (col == 0) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sm.red[wv][16 * rb + rq + q] = db1[rb * 4 + q];
                sm.red[wv][64 + 16 * rb + rq + q] = db2[rb * 4 + q];
            }
    }
    if (l == 0) {
        sm.red[wv][128] = db3[0];
        sm.red[wv][129] = db3[1];
        sm.red[wv][130] = lsum;
    }
    __syncthreads();
    if (t < 131) {
        const float v = ((sm.red[0][t] + sm.red[1][t]) + sm.red[2][t]) + sm.red[3][t];
        if (t < 64) P[kPartDB1 + t] = v;
        else if (t < 128) P[kPartDB2 + t - 64] = v;
        else if (t < 130) P[kPartDB3 + t - 128] = v;
        else P[kPartLoss] = v / (float)M;
    }
}

// Gradient sums over the blocks in a fixed order, then (adam != 0) one Adam
// step on the FP32 master parameters and fresh bfloat16 copies.
// Gradient sums over the blocks, in the partials' own layout so that the
// loads are coalesced: a block of 256 lanes owns 64 partial entries, four
// lanes per entry sum every fourth block, and the four sums are added in a
// fixed order.  Then (adam != 0) one Adam step on the FP32 master parameter
// the entry belongs to, and fresh bfloat16 copies.
constexpr int kReduceItems = 64;

__global__ __launch_bounds__(256) void mlp_reduce_adam_kernel(const float* part, int nblocks, float* master, float* m,
                                                             float* v, float* grad, float* loss, __bf16* wts,
                                                             int adam, float lr, float c1, float c2) {
    __shared__ float red[4][kReduceItems];
    const int t = threadIdx.x, col = t & (kReduceItems - 1), slice = t / kReduceItems;
    const int q = blockIdx.x * kReduceItems + col;     // partial-layout index, kPartLoss included
    float g = 0.f;
    if (part && q <= kPartLoss)
        for (int b = slice; b < nblocks; b += 4) g += part[(int64_t)b * kPartStride + q];
    red[slice][col] = g;
    __syncthreads();
    if (slice != 0 || q > kPartLoss) return;
    g = ((red[0][col] + red[1][col]) + red[2][col]) + red[3][col];
    if (q == kPartLoss) {
        if (loss && part) *loss = g;
        return;
    }
    // partial layout -> master layout (W1 [32][64], b1, W2 [64][64], b2, W3 [64][2], b3)
    int p, kind, i = 0, o = 0;
    if (q < kPartDB1) { o = q / 32; i = q % 32; p = i * 64 + o; kind = 1; }
    else if (q < kPartDW2) { p = q; kind = 0; }
    else if (q < kPartDB2) { const int r = q - kPartDW2; o = r / 64; i = r % 64; p = kPartDW2 + i * 64 + o; kind = 2; }
    else if (q < kPartDW3) { p = q; kind = 0; }
    else if (q < kPartDB3) { const int r = q - kPartDW3; o = r / 64; i = r % 64; p = kPartDW3 + i * 2 + o; kind = 3; }
    else { p = q; kind = 0; }
    if (part) {
        if (grad) grad[p] = g;
    } else {
        g = grad[p];
    }
    if (!adam) return;
    const float mm = 0.9f * m[p] + 0.1f * g;
    const float vv = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mm;
    v[p] = vv;
    const float val = master[p] - lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
    master[p] = val;
    const __bf16 bv = (__bf16)val;
    if (kind == 1) wts[o * 32 + i] = bv;                                  // W1^T
    else if (kind == 2) {
        wts[2048 + o * 64 + i] = bv;                                      // W2^T
        wts[2048 + 4096 + 1024 + i * 64 + o] = bv;                        // W2
    } else if (kind == 3) wts[2048 + 4096 + o * 64 + i] = bv;             // W3^T
}

__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

template <int L>
hipError_t launch_sur_L(const SurBatch& b, hipStream_t s) {
    const dim3 grid(b.rm.total), block(kSurBlock);
    if (b.rm.stats) hipLaunchKernelGGL((surrogate_kernel<L, true>), grid, block, 0, s, b);
    else hipLaunchKernelGGL((surrogate_kernel<L, false>), grid, block, 0, s, b);
    return hipGetLastError();
}

hipError_t launch_surrogate(int L, const SurBatch& b, hipStream_t s) {
    if (b.rm.total <= 0) return hipSuccess;
    switch (L) {
        case 2: return launch_sur_L<2>(b, s);
        case 3: return launch_sur_L<3>(b, s);
        case 4: return launch_sur_L<4>(b, s);
        case 5: return launch_sur_L<5>(b, s);
        case 6: return launch_sur_L<6>(b, s);
        case 7: return launch_sur_L<7>(b, s);
        case 8: return launch_sur_L<8>(b, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mlp_forward(const MlpWeights& w, const float* X, float* Y, int M, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((M + 63) / 64), dim3(256), 0, s, w, X, Y, M);
    return hipGetLastError();
}


hipError_t launch_gen_lines(float* lines, long long first, int count, unsigned long long seed, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(gen_lines_kernel, dim3(count), dim3(32), 0, s, lines, first, seed);
    return hipGetLastError();
}

hipError_t launch_label_entries(int2* list, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(label_entries_kernel, dim3((count + 255) / 256), dim3(256), 0, s, list, count);
    return hipGetLastError();
}

hipError_t launch_train_features(const float2* gamma, int count, const float* labels, float* X, float* T,
                                 hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(train_features_kernel, dim3((count + 255) / 256), dim3(256), 0, s, gamma, count, labels, X, T);
    return hipGetLastError();
}

int mlp_train_blocks(int M) { return std::max(1, std::min(256, M / kTrainChunk)); }
int mlp_partial_stride() { return kPartStride; }

hipError_t launch_mlp_train(const MlpWeights& w, const __bf16* w2, const float* X, const float* T, int M, float* part,
                            int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(mlp_train_kernel, dim3(nblocks), dim3(256), 0, s, w, w2, X, T, M, part);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce_adam(const float* part, int nblocks, float* master, float* m, float* v, float* grad,
                                  float* loss, __bf16* wts, int adam, float lr, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kPartLoss + 1 + kReduceItems - 1) / kReduceItems), dim3(256), 0, s,
                       part, nblocks, master, m, v, grad, loss, wts, adam, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace bm
