// Internal interfaces between the host runtime (bm_runtime.cpp) and the
// kernel translation units.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/bosmusic.h"

namespace bm {

constexpr int kMaxL = 8;
constexpr int kMaxN = 64;
constexpr int kMaxFFT = 8192;
constexpr int kMaxRadixPasses = 20;
constexpr int kStatSlots = 64;   // counter slots of the statistics buffer (4 counters each)

// Mixed-radix plan of one DFT length (radices 4, 2, 3, 5 in pass order).
struct FftPlan {
    int n;                       // transform length
    int passes;                  // number of radix passes
    int radix[kMaxRadixPasses];  // radix of each pass
};

// Input element types of the analytic / transpose kernels.
enum class Elem : int { F16 = 1, F32 = 2, F64 = 3, C32 = 4 };

// Starting points of the simultaneous root iteration: the roots of the
// noise-free root-MUSIC polynomial of a single tone at frequency 0, with its
// double root at 1 split radially into (rho, 1/rho).  Rotated by the
// frequency guess of each window at run time.
struct RootTemplate {
    float re[2 * kMaxL - 2];
    float im[2 * kMaxL - 2];
};

// One direction of one frame for the root-MUSIC kernel: `nlines` lines of
// `len` complex samples, `bpl` window blocks per line.
struct RmJob {
    const float2* gamma;   // line-major complex signal
    int64_t gamma_ls;      // complex elements between line starts
    float* out;            // omega
    int64_t out_es;        // output stride along the line (elements)
    int64_t out_ls;        // output stride between lines (elements)
    uint8_t* flags;        // optional per-pixel flags
    int len;
    int nlines;
    int N;                 // window length
    int bpl;               // window blocks per line
    int flag_shift;        // 0 for x, 4 for y
    int flag_or;           // 1: OR into existing flags, 0: overwrite
};

// All root-MUSIC work of one L: jobs[j] owns work items prefix[j] .. prefix[j+1)-1.
struct RmBatch {
    const RmJob* jobs;
    const int* prefix;     // njobs + 1 entries
    int njobs;
    int total;             // prefix[njobs]
    int jacobi;            // 1: cyclic Jacobi eigen-split instead of the tridiagonal solver
    unsigned long long* stats;  // kStatSlots x 4 counters, or nullptr
    RootTemplate tmpl;
};

// Lines of one frame direction for the analytic-signal kernel (one block per line).
struct FftJob {
    const void* src;       // real lines, src_ls elements apart
    int64_t src_ls;
    float2* dst;           // complex lines, plan.n apart
    const float2* tw;      // twiddles e^{-2 pi i m / n}, m < n
    int elem;              // Elem of src
    int nlines;
    FftPlan plan;
};

struct FftBatch {
    const FftJob* jobs;
    const int* prefix;     // lines: njobs + 1 entries
    int njobs;
    int total;
    int max_n;
};

// Transpose of one frame (rows x cols, src_ls elements per row) to cols x rows.
struct TrJob {
    const void* src;
    int64_t src_ls;
    void* dst;             // float (real input) or float2 (C32)
    int rows, cols;
    int tiles_x;           // 32-wide tiles along cols
    int elem;
};

struct TrBatch {
    const TrJob* jobs;
    const int* prefix;     // tiles: njobs + 1 entries
    int njobs;
    int total;
};

// Launchers (enqueue only; return the launch error).  `block` is 128 or 256
// threads; `grid` is the number of blocks of the grid-stride loop (<= 0: one
// block per work item).
hipError_t launch_rootmusic(int L, const RmBatch& b, int block, int grid, hipStream_t s);
int rootmusic_windows_per_block(int L, int block);
hipError_t launch_transpose(const TrBatch& b, hipStream_t s);
hipError_t launch_analytic(const FftBatch& b, hipStream_t s);

hipError_t launch_synth(float2* g, int64_t n, float w0, float noise, hipStream_t s);

hipError_t launch_integrate(const float* wx, const float* wy, int W, int H, int Nx, int Ny,
                            double cx, double cy, double* anchor_ws, double* phi, hipStream_t s);

// Raise the dynamic-LDS limit of the kernels that need more than 64 KiB; call
// once per device with that device current.
hipError_t analytic_set_attributes();
hipError_t integrate_set_attributes();

}  // namespace bm
