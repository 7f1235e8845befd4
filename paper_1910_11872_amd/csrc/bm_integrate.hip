// FP64 trapezoid integration of the local-frequency maps to phase.
//
// The paper recovers the global phase from the per-window estimates
// (Sec. 3, after Eq. 15); here the phase is the path integral of the
// frequency maps on the window-centre grid:
//   anchor column xa = floor(Nx/2), anchor row ya = floor(Ny/2), phi(ya,xa) = 0,
//   phi(y+1, xa) = phi(y, xa) + (wy(y,xa) + wy(y+1,xa))/2 - cy,
//   phi(y, x+1)  = phi(y, x)  + (wx(y,x)  + wx(y,x+1))/2  - cx.
// Both scans are block-wide prefix sums in FP64: each thread scans a
// contiguous chunk held in LDS, the chunk totals are scanned across the
// block, and the offsets are added back before a coalesced store.
#include "bm_internal.h"

namespace bm {
namespace {

constexpr int kAnchorThreads = 1024;
constexpr int kRowThreads = 256;
constexpr int kRowsPerBlock = 4;

// Exclusive block scan of one double per thread: a shuffle scan within each
// wave, then the totals of the waves before it.
template <int T>
__device__ double block_scan_exclusive(double v, double* sh) {
    static_assert(T % 64 == 0 && T <= 64 * 64, "whole waves");
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    double x = v;                                  // inclusive scan within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;                    // wave totals
    __syncthreads();
    double base = 0.0;
    for (int k = 0; k < wv; ++k) base += sh[k];
    __syncthreads();                               // sh is free for the next scan
    return base + x - v;
}

__global__ __launch_bounds__(kAnchorThreads) void anchor_kernel(const float* __restrict__ wy, int W, int xa, int y0,
                                                                int y1, double cy, double* __restrict__ anchor) {
    __shared__ double sh[kAnchorThreads / 64];
    const int nsteps = y1 - y0;
    const int chunk = (nsteps + kAnchorThreads - 1) / kAnchorThreads;
    const int t = threadIdx.x;
    const int i0 = t * chunk, i1 = min(nsteps, i0 + chunk);
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double a = wy[(int64_t)(y0 + i) * W + xa], b = wy[(int64_t)(y0 + i + 1) * W + xa];
        acc += 0.5 * (a + b) - cy;
        anchor[y0 + i + 1] = acc;  // local prefix, offset added below
    }
    const double off = block_scan_exclusive<kAnchorThreads>(acc, sh);
    for (int i = i0; i < i1; ++i) anchor[y0 + i + 1] += off;
    if (t == 0) anchor[y0] = 0.0;
}

// One block per row.  LDS: row of omega (float, W) + local prefixes (double, W).
__global__ __launch_bounds__(kRowThreads) void rows_kernel(const float* __restrict__ wx, int W, int H, int x0, int x1,
                                                           int y0, int y1, double cx, const double* __restrict__ anchor,
                                                           double* __restrict__ phi) {
    extern __shared__ double dyn[];
    __shared__ double sh[kRowThreads / 64];
    double* sp = dyn;                              // W doubles
    float* sw = reinterpret_cast<float*>(dyn + W);  // W floats
    const int y = blockIdx.x;
    double* out = phi + (int64_t)y * W;
    const double nan = __builtin_nan("");
    if (y < y0 || y > y1 || x1 < x0) {
        for (int x = threadIdx.x; x < W; x += kRowThreads) out[x] = nan;
        return;
    }
    const float* row = wx + (int64_t)y * W;
    for (int x = threadIdx.x; x < W; x += kRowThreads) sw[x] = row[x];
    __syncthreads();
    const int nsteps = x1 - x0;
    const int chunk = (nsteps + kRowThreads - 1) / kRowThreads;
    const int t = threadIdx.x;
    const int i0 = t * chunk, i1 = min(nsteps, i0 + chunk);
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) {
        acc += 0.5 * ((double)sw[x0 + i] + (double)sw[x0 + i + 1]) - cx;
        sp[x0 + i + 1] = acc;
    }
    const double off = block_scan_exclusive<kRowThreads>(acc, sh);
    const double base = anchor ? anchor[y] : 0.0;
    for (int i = i0; i < i1; ++i) sp[x0 + i + 1] += off;
    __syncthreads();
    for (int x = threadIdx.x; x < W; x += kRowThreads) {
        double v = nan;
        if (x == x0) v = base;
        else if (x > x0 && x <= x1) v = base + sp[x];
        out[x] = v;
    }
}

// Batched forms: job j = blockIdx.x for the anchors; rows of all jobs in one grid.
__global__ __launch_bounds__(kAnchorThreads) void anchor_many_kernel(const IntJob* __restrict__ jobs, int njobs,
                                                                     double* __restrict__ anchors) {
    __shared__ double sh[kAnchorThreads / 64];
    const IntJob& J = jobs[blockIdx.x];
    if (!J.wy || J.y1 < J.y0 || J.x1 < J.x0) return;
    double* anchor = anchors + J.anchor_off;
    const int nsteps = J.y1 - J.y0;
    const int chunk = (nsteps + kAnchorThreads - 1) / kAnchorThreads;
    const int t = threadIdx.x;
    const int i0 = t * chunk, i1 = min(nsteps, i0 + chunk);
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double a = J.wy[(int64_t)(J.y0 + i) * J.W + J.x0], b = J.wy[(int64_t)(J.y0 + i + 1) * J.W + J.x0];
        acc += 0.5 * (a + b) - J.cy;
        anchor[J.y0 + i + 1] = acc;
    }
    const double off = block_scan_exclusive<kAnchorThreads>(acc, sh);
    for (int i = i0; i < i1; ++i) anchor[J.y0 + i + 1] += off;
    if (t == 0) anchor[J.y0] = 0.0;
}

// kRowsPerBlock consecutive rows of the job list per block (one job lookup
// for all of them), T threads per row.
template <int T>
__global__ __launch_bounds__(T) void rows_many_kernel(const IntJob* __restrict__ jobs, const int* __restrict__ prefix,
                                                      int njobs, int total_rows, const double* __restrict__ anchors) {
    extern __shared__ double dyn[];
    __shared__ double sh[T / 64];
    const int w0 = blockIdx.x * kRowsPerBlock;
    int lo = 0, hi = njobs - 1;              // job of row w0: last j with prefix[j] <= w0
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= w0) lo = mid;
        else hi = mid - 1;
    }
    int jb = lo;
    const double nan = __builtin_nan("");
    for (int q = 0; q < kRowsPerBlock; ++q) {
        const int w = w0 + q;
        if (w >= total_rows) break;
        while (w >= prefix[jb + 1]) ++jb;        // the next (non-empty) job
        const IntJob& J = jobs[jb];
        const int W = J.W;
        const int y = w - prefix[jb];
        double* sp = dyn;                              // W doubles
        float* sw = reinterpret_cast<float*>(dyn + W);  // W floats
        double* out = J.phi + (int64_t)y * W;
        if (y < J.y0 || y > J.y1 || J.x1 < J.x0) {
            for (int x = threadIdx.x; x < W; x += T) out[x] = nan;
            continue;
        }
        __syncthreads();                         // the previous row is out of LDS
        const float* row = J.wx + (int64_t)y * W;
        for (int x = threadIdx.x; x < W; x += T) sw[x] = row[x];
        __syncthreads();
        const int x0 = J.x0, nsteps = J.x1 - J.x0;
        const int chunk = (nsteps + T - 1) / T;
        const int t = threadIdx.x;
        const int i0 = t * chunk, i1 = min(nsteps, i0 + chunk);
        double acc = 0.0;
        for (int i = i0; i < i1; ++i) {
            acc += 0.5 * ((double)sw[x0 + i] + (double)sw[x0 + i + 1]) - J.cx;
            sp[x0 + i + 1] = acc;
        }
        const double off = block_scan_exclusive<T>(acc, sh);
        const double base = J.wy ? anchors[J.anchor_off + y] : 0.0;
        for (int i = i0; i < i1; ++i) sp[x0 + i + 1] += off;
        __syncthreads();
        for (int x = threadIdx.x; x < W; x += T) {
            double v = nan;
            if (x == x0) v = base;
            else if (x > x0 && x <= J.x1) v = base + sp[x];
            out[x] = v;
        }
    }
}

}  // namespace

hipError_t launch_integrate_many(const IntJob* jobs, const int* prefix, int njobs, int total_rows, int max_w,
                                 double* anchors, hipStream_t s) {
    if (njobs <= 0 || total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(anchor_many_kernel, dim3(njobs), dim3(kAnchorThreads), 0, s, jobs, njobs, anchors);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t shmem = (size_t)max_w * (sizeof(double) + sizeof(float));
    const dim3 grid((total_rows + kRowsPerBlock - 1) / kRowsPerBlock);
    if (max_w > 2048)          // wide rows: more waves per block, four samples per thread at 4096
        hipLaunchKernelGGL(rows_many_kernel<1024>, grid, dim3(1024), shmem, s, jobs, prefix, njobs, total_rows, anchors);
    else
        hipLaunchKernelGGL(rows_many_kernel<kRowThreads>, grid, dim3(kRowThreads), shmem, s, jobs, prefix, njobs,
                           total_rows, anchors);
    return hipGetLastError();
}

hipError_t launch_integrate(const float* wx, const float* wy, int W, int H, int Nx, int Ny, double cx, double cy,
                            double* anchor_ws, double* phi, hipStream_t s) {
    const int x0 = Nx / 2, x1 = W - Nx + Nx / 2;
    int y0 = 0, y1 = H - 1;
    const double* anchor = nullptr;
    if (wy) {
        y0 = Ny / 2;
        y1 = H - Ny + Ny / 2;
        if (y1 >= y0 && x1 >= x0) {
            hipLaunchKernelGGL(anchor_kernel, dim3(1), dim3(kAnchorThreads), 0, s, wy, W, x0, y0, y1, cy, anchor_ws);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        anchor = anchor_ws;
    }
    const size_t shmem = (size_t)W * (sizeof(double) + sizeof(float));
    hipLaunchKernelGGL(rows_kernel, dim3(H), dim3(kRowThreads), shmem, s, wx, W, H, x0, x1, y0, y1, cx, anchor, phi);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free entry point: the anchor column of one
// integration, kNoAllocMaxHeight doubles, held on every device the library
// runs on until the process ends.  In host code `noalloc_anchor` names a
// host-side stand-in, not device memory: host code uses only the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double noalloc_anchor[kNoAllocMaxHeight];

hipError_t noalloc_anchor_address(double** ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_anchor));
    if (e != hipSuccess) return e;
    *ptr = static_cast<double*>(p);
    return hipSuccess;
}

hipError_t integrate_set_attributes() {
    hipError_t e = hipFuncSetAttribute((const void*)rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kMaxFFT * (int)(sizeof(double) + sizeof(float)));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)rows_many_kernel<kRowThreads>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kMaxFFT * (int)(sizeof(double) + sizeof(float)));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)rows_many_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kMaxFFT * (int)(sizeof(double) + sizeof(float)));
}

}  // namespace bm
