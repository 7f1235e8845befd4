// FP64 trapezoid integration of the local-frequency maps to phase.
//
// The paper recovers the global phase from the per-window estimates
// (Sec. 3, after Eq. 15); here the phase is the path integral of the
// frequency maps on the window-centre grid:
//   anchor column xa = floor(Nx/2), anchor row ya = floor(Ny/2), phi(ya,xa) = 0,
//   phi(y+1, xa) = phi(y, xa) + (wy(y,xa) + wy(y+1,xa))/2 - cy,
//   phi(y, x+1)  = phi(y, x)  + (wx(y,x)  + wx(y,x+1))/2  - cx.
// Both scans are block-wide prefix sums in FP64: each thread sums a
// contiguous chunk, the chunk totals are scanned across the block, and the
// offsets are added back before the store.
#include "bm_internal.h"

namespace bm {
namespace {

constexpr int kAnchorThreads = 1024;
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

// One row of phi, by one block of T threads.  Thread t sums the trapezoid
// increments of its E = row_elems(W) samples x = E t .. E t + E - 1 in
// registers, the block scan adds the totals of the threads before it, and
// the row's anchor comes last: the arithmetic depends on the row's width
// alone, so a single call and a batched call give the same bits whatever
// block size (at least W / E threads) and data path each takes.  The data
// path: vec rows (W a multiple of 4, at most 4096, omega_x and phi 16-byte
// aligned) load their four samples with one 16-byte load (and the sample
// before them) and store two 16-byte pairs; other rows stage omega in LDS and
// store single doubles.
constexpr int row_elems(int W) { return W <= 4096 ? 4 : 8; }

template <int T>
__device__ __forceinline__ void integrate_row(const float* __restrict__ row, int W, int x0, int x1, double cx,
                                              double base, double* __restrict__ out, bool vec, float* sw,
                                              double* sh) {
    const double nan = __builtin_nan("");
    const int t = threadIdx.x;
    const int E = row_elems(W);
    const int x = E * t;
    float v[8], prev = 0.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = 0.f;
    if (vec) {                                     // E = 4
        if (x < W) {
            const float4 r4 = *reinterpret_cast<const float4*>(row + x);
            v[0] = r4.x; v[1] = r4.y; v[2] = r4.z; v[3] = r4.w;
            if (x > 0) prev = row[x - 1];
        }
    } else {
        __syncthreads();                           // a previous row is out of LDS
        for (int i = t; i < W; i += T) sw[i] = row[i];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (m < E && x + m < W) v[m] = sw[x + m];
        if (x > 0 && x - 1 < W) prev = sw[x - 1];
    }
    // increment of sample xx (from xx - 1), x0 < xx <= x1
    double a[8], acc = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int xx = x + m;
        const double inc = 0.5 * ((double)(m == 0 ? prev : v[m - 1]) + (double)v[m]) - cx;
        if (m < E && xx > x0 && xx <= x1) acc += inc;
        a[m] = acc;
    }
    const double off = block_scan_exclusive<T>(acc, sh);
    double o[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int xx = x + m;
        o[m] = (xx >= x0 && xx <= x1) ? base + (a[m] + off) : nan;
    }
    if (vec) {
        if (x < W) {
            double2* out2 = reinterpret_cast<double2*>(out + x);
            out2[0] = make_double2(o[0], o[1]);
            out2[1] = make_double2(o[2], o[3]);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (m < E && x + m < W) out[x + m] = o[m];
    }
}

// One block per row of one map.
template <int T>
__global__ __launch_bounds__(T) void rows_kernel(const float* __restrict__ wx, int W, int H, int x0, int x1, int y0,
                                                 int y1, double cx, const double* __restrict__ anchor,
                                                 double* __restrict__ phi, int vec) {
    extern __shared__ double dyn[];
    __shared__ double sh[T / 64];
    const int y = blockIdx.x;
    double* out = phi + (int64_t)y * W;
    if (y < y0 || y > y1 || x1 < x0) {
        const double nan = __builtin_nan("");
        for (int x = threadIdx.x; x < W; x += T) out[x] = nan;
        return;
    }
    integrate_row<T>(wx + (int64_t)y * W, W, x0, x1, cx, anchor ? anchor[y] : 0.0, out, vec != 0,
                     reinterpret_cast<float*>(dyn), sh);
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
        double* out = J.phi + (int64_t)y * W;
        if (y < J.y0 || y > J.y1 || J.x1 < J.x0) {
            for (int x = threadIdx.x; x < W; x += T) out[x] = nan;
            continue;
        }
        integrate_row<T>(J.wx + (int64_t)y * W, W, J.x0, J.x1, J.cx, J.wy ? anchors[J.anchor_off + y] : 0.0, out,
                         J.vec != 0, reinterpret_cast<float*>(dyn), sh);
    }
}

}  // namespace

hipError_t launch_integrate_many(const IntJob* jobs, const int* prefix, int njobs, int total_rows, int threads,
                                 int lds_w, double* anchors, hipStream_t s) {
    if (njobs <= 0 || total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(anchor_many_kernel, dim3(njobs), dim3(kAnchorThreads), 0, s, jobs, njobs, anchors);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t shmem = (size_t)lds_w * sizeof(float);
    const dim3 grid((total_rows + kRowsPerBlock - 1) / kRowsPerBlock);
    if (threads <= 256)
        hipLaunchKernelGGL(rows_many_kernel<256>, grid, dim3(256), shmem, s, jobs, prefix, njobs, total_rows, anchors);
    else if (threads <= 512)
        hipLaunchKernelGGL(rows_many_kernel<512>, grid, dim3(512), shmem, s, jobs, prefix, njobs, total_rows, anchors);
    else
        hipLaunchKernelGGL(rows_many_kernel<1024>, grid, dim3(1024), shmem, s, jobs, prefix, njobs, total_rows,
                           anchors);
    return hipGetLastError();
}

int integrate_row_threads(int W) {
    const int n = (W + row_elems(W) - 1) / row_elems(W);
    return n <= 256 ? 256 : (n <= 512 ? 512 : 1024);
}

bool integrate_row_vec(int W, const void* wx, const void* phi) {
    return W % 4 == 0 && W <= 4096 && ((uintptr_t)wx & 15) == 0 && ((uintptr_t)phi & 15) == 0;
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
    const bool vec = integrate_row_vec(W, wx, phi);
    const int T = integrate_row_threads(W);
    const size_t shmem = vec ? 0 : (size_t)W * sizeof(float);
    if (T <= 256)
        hipLaunchKernelGGL(rows_kernel<256>, dim3(H), dim3(256), shmem, s, wx, W, H, x0, x1, y0, y1, cx, anchor, phi,
                           (int)vec);
    else if (T <= 512)
        hipLaunchKernelGGL(rows_kernel<512>, dim3(H), dim3(512), shmem, s, wx, W, H, x0, x1, y0, y1, cx, anchor, phi,
                           (int)vec);
    else
        hipLaunchKernelGGL(rows_kernel<1024>, dim3(H), dim3(1024), shmem, s, wx, W, H, x0, x1, y0, y1, cx, anchor,
                           phi, (int)vec);
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
    const int bytes = kMaxFFT * (int)sizeof(float);
    const void* k[6] = {(const void*)rows_kernel<256>, (const void*)rows_kernel<512>, (const void*)rows_kernel<1024>,
                        (const void*)rows_many_kernel<256>, (const void*)rows_many_kernel<512>,
                        (const void*)rows_many_kernel<1024>};
    for (const void* f : k) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace bm
