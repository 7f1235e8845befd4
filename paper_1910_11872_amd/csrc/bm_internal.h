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

struct RootMusicArgs {
    const float2* gamma;   // line-major complex signal
    int64_t gamma_ls;      // complex elements between line starts
    int len;               // samples per line (window positions)
    int nlines;
    int N;                 // window length
    float* out;            // omega
    int64_t out_es;        // output stride along the line (elements)
    int64_t out_ls;        // output stride between lines (elements)
    uint8_t* flags;        // optional per-pixel flags
    int flag_shift;        // 0 for x, 4 for y
    int flag_or;           // 1: OR into existing flags, 0: overwrite
    unsigned long long* stats;  // kStatSlots x 4 counters, or nullptr
    int jacobi;            // 1: cyclic Jacobi eigen-split instead of the tridiagonal solver
    RootTemplate tmpl;
};

// Launchers (enqueue only; return the launch error).
hipError_t launch_rootmusic(int L, const RootMusicArgs& a, hipStream_t s);

hipError_t launch_transpose(Elem e, const void* src, int64_t src_ls, int rows, int cols,
                            void* dst, hipStream_t s);

hipError_t launch_analytic(Elem e, const void* src, int64_t src_ls, int nlines, const FftPlan& plan,
                           const float2* twiddle, float2* dst, hipStream_t s);

hipError_t launch_integrate(const float* wx, const float* wy, int W, int H, int Nx, int Ny,
                            double cx, double cy, double* anchor_ws, double* phi, hipStream_t s);

// Raise the dynamic-LDS limit of the kernels that need more than 64 KiB; call
// once per device with that device current.
hipError_t analytic_set_attributes();
hipError_t integrate_set_attributes();

}  // namespace bm
