// Complex analytic fringe signal (paper Sec. 2, Eq. 1) by an exact DFT mask,
// plus the tiled transposes that turn the y direction into lines.
//
// analytic_kernel: one block per line.  The line is decoded to FP32, run
// through a mixed-radix (4, 2, 3, 5) Stockham FFT ping-ponged between two LDS
// buffers, multiplied by the one-sided mask H (H[0] = 0, H[k] = 2 for
// 0 < 2k < n, 0 otherwise, so DC and Nyquist are removed and the carrier is
// kept), and transformed back with the same forward FFT applied to the
// conjugate.  Twiddles come from a per-length table computed in FP64 on the
// host and rounded once.
#include "bm_internal.h"

namespace bm {
namespace {

constexpr int kFftThreads = 256;
constexpr int kTile = 32;

__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(double v) { return (float)v; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i and +i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }

// One forward Stockham pass of radix R over the whole line: src -> dst.
template <int R>
__device__ __forceinline__ void stockham_pass(const float2* __restrict__ src, float2* __restrict__ dst, int n,
                                              int Ns, const float2* __restrict__ tw) {
    const int nR = n / R;
    const int tws = n / (Ns * R);
    for (int j = threadIdx.x; j < nR; j += kFftThreads) {
        const int k = j % Ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[j + r * nR];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * tws]);
        float2 y[R];
        if (R == 2) {
            y[0] = cadd(v[0], v[1]);
            y[1] = csub(v[0], v[1]);
        } else if (R == 4) {
            const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
            const float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
            y[0] = cadd(t0, t2);
            y[2] = csub(t0, t2);
            y[1] = cadd(t1, mul_mi(t3));
            y[3] = cadd(t1, mul_pi(t3));
        } else if (R == 3) {
            constexpr float h = 0.866025403784438647f;  // sin(2 pi / 3)
            const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
            const float2 base = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
            const float2 rot = make_float2(h * d.y, -h * d.x);   // -i h d
            y[0] = cadd(v[0], s);
            y[1] = cadd(base, rot);
            y[2] = csub(base, rot);
        } else if (R == 5) {
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
        const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[idx + r * Ns] = y[r];
    }
}

// Forward DFT of the line held in `a` (scratch `b`); returns the buffer that
// holds the result in natural order.
__device__ float2* fft_forward(float2* a, float2* b, int n, const FftPlan& plan, const float2* tw) {
    int Ns = 1;
    for (int ps = 0; ps < plan.passes; ++ps) {
        const int R = plan.radix[ps];
        if (R == 4) stockham_pass<4>(a, b, n, Ns, tw);
        else if (R == 2) stockham_pass<2>(a, b, n, Ns, tw);
        else if (R == 3) stockham_pass<3>(a, b, n, Ns, tw);
        else stockham_pass<5>(a, b, n, Ns, tw);
        __syncthreads();
        float2* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

template <typename Tin>
__global__ __launch_bounds__(kFftThreads) void analytic_kernel(const Tin* __restrict__ src, int64_t src_ls,
                                                               FftPlan plan, const float2* __restrict__ tw,
                                                               float2* __restrict__ dst) {
    extern __shared__ float2 lds[];
    const int n = plan.n;
    float2* a = lds;
    float2* b = lds + n;
    const Tin* x = src + (int64_t)blockIdx.x * src_ls;
    for (int i = threadIdx.x; i < n; i += kFftThreads) a[i] = make_float2(to_f32(x[i]), 0.f);
    __syncthreads();
    float2* X = fft_forward(a, b, n, plan, tw);
    float2* other = (X == a) ? b : a;
    // one-sided mask and 1/n, then conjugate so that a forward DFT inverts
    const float sc = 2.0f / (float)n;
    for (int k = threadIdx.x; k < n; k += kFftThreads) {
        const float2 v = X[k];
        const bool keep = (k >= 1) && (2 * k < n);
        X[k] = keep ? make_float2(v.x * sc, -v.y * sc) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    float2* Y = fft_forward(X, other, n, plan, tw);
    float2* out = dst + (int64_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += kFftThreads) {
        const float2 v = Y[i];
        out[i] = make_float2(v.x, -v.y);
    }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kTile * 8) void transpose_kernel(const Tin* __restrict__ src, int64_t src_ls, int rows,
                                                              int cols, Tout* __restrict__ dst) {
    __shared__ Tout tile[kTile][kTile + 1];
    const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
#pragma unroll
    for (int j = 0; j < kTile; j += 8) {
        const int r = by + ty + j, c = bx + tx;
        if (r < rows && c < cols) {
            if constexpr (__is_same(Tout, float2))
                tile[ty + j][tx] = src[(int64_t)r * src_ls + c];
            else
                tile[ty + j][tx] = to_f32(src[(int64_t)r * src_ls + c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTile; j += 8) {
        const int c = bx + ty + j, r = by + tx;
        if (r < rows && c < cols) dst[(int64_t)c * rows + r] = tile[tx][ty + j];
    }
}

template <typename Tin>
hipError_t launch_analytic_t(const void* src, int64_t ls, int nlines, const FftPlan& plan, const float2* tw,
                             float2* dst, hipStream_t s) {
    const size_t shmem = 2u * (size_t)plan.n * sizeof(float2);
    hipLaunchKernelGGL(analytic_kernel<Tin>, dim3(nlines), dim3(kFftThreads), shmem, s,
                       (const Tin*)src, ls, plan, tw, dst);
    return hipGetLastError();
}

template <typename Tin>
hipError_t set_attr() {
    return hipFuncSetAttribute((const void*)analytic_kernel<Tin>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               2 * kMaxFFT * (int)sizeof(float2));
}

}  // namespace

hipError_t analytic_set_attributes() {
    hipError_t e = set_attr<_Float16>();
    if (e == hipSuccess) e = set_attr<float>();
    if (e == hipSuccess) e = set_attr<double>();
    return e;
}

hipError_t launch_analytic(Elem e, const void* src, int64_t src_ls, int nlines, const FftPlan& plan,
                           const float2* twiddle, float2* dst, hipStream_t s) {
    if (nlines <= 0) return hipSuccess;
    switch (e) {
        case Elem::F16: return launch_analytic_t<_Float16>(src, src_ls, nlines, plan, twiddle, dst, s);
        case Elem::F32: return launch_analytic_t<float>(src, src_ls, nlines, plan, twiddle, dst, s);
        case Elem::F64: return launch_analytic_t<double>(src, src_ls, nlines, plan, twiddle, dst, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transpose(Elem e, const void* src, int64_t src_ls, int rows, int cols, void* dst,
                            hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((cols + kTile - 1) / kTile, (rows + kTile - 1) / kTile);
    dim3 block(kTile * 8);
    switch (e) {
        case Elem::F16:
            hipLaunchKernelGGL((transpose_kernel<_Float16, float>), grid, block, 0, s, (const _Float16*)src, src_ls,
                               rows, cols, (float*)dst);
            break;
        case Elem::F32:
            hipLaunchKernelGGL((transpose_kernel<float, float>), grid, block, 0, s, (const float*)src, src_ls, rows,
                               cols, (float*)dst);
            break;
        case Elem::F64:
            hipLaunchKernelGGL((transpose_kernel<double, float>), grid, block, 0, s, (const double*)src, src_ls,
                               rows, cols, (float*)dst);
            break;
        case Elem::C32:
            hipLaunchKernelGGL((transpose_kernel<float2, float2>), grid, block, 0, s, (const float2*)src, src_ls,
                               rows, cols, (float2*)dst);
            break;
    }
    return hipGetLastError();
}

}  // namespace bm
