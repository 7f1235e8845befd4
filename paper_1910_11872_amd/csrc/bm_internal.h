// Internal interfaces between the host runtime (bm_runtime.cpp) and the
// kernel translation units.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/bosmusic.h"

namespace bm {

constexpr int kMaxL = 8;        // covariance size of line windows
// Block windows (the paper's (2L+1) x (2L+1) window, Sec. 3) go up to 17 x 17, the
// largest of the paper's window-size table; above kMaxL only odd sizes.
constexpr int kMaxBlockL = 17;
constexpr bool block_size_supported(int L) { return L >= 2 && (L <= kMaxL || (L <= kMaxBlockL && (L & 1))); }
constexpr int kMaxN = 64;
constexpr int kMaxFFT = 8192;
constexpr int kMaxRadixPasses = 20;
constexpr int kStatSlots = 64;   // counter slots of the statistics buffer
constexpr int kStatFields = 9;   // counters per slot
constexpr int kGatherBlock = 256;

// Mixed-radix plan of one DFT length (radices 4, 2, 3, 5, 7, 11, 13 in pass order).
struct FftPlan {
    int n;                       // transform length
    int passes;                  // number of radix passes
    int radix[kMaxRadixPasses];  // radix of each pass
};

// Input element types of the analytic / transpose kernels.
enum class Elem : int { F16 = 1, F32 = 2, F64 = 3, C32 = 4, U8 = 5 };

// Starting points of the simultaneous root iteration: the roots of the
// noise-free root-MUSIC polynomial of a single tone at frequency 0, with its
// double root at 1 split radially into (rho, 1/rho).  Rotated by the
// frequency guess of each window at run time.
struct RootTemplate {
    float re[2 * kMaxBlockL - 2];
    float im[2 * kMaxBlockL - 2];
};

// Window kinds of a root-MUSIC job.
enum RmKind : int {
    RM_LINE = 0,      // N samples along the line, length-L sub-snapshots
    RM_BLOCK = 1,     // L x L block around the pixel: its rows (omega_x) and columns (omega_y)
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
    int64_t flag_es;       // flag strides along the line and between lines (elements)
    int64_t flag_ls;
    int len;
    int nlines;
    int N;                 // window length
    int bpl;               // window blocks per line
    int flag_shift;        // 0 for x, 4 for y
    int flag_or;           // 1: OR into existing flags, 0: overwrite
    int kind;              // RmKind
    // RM_BLOCK only: `out` is omega_x; both maps and the phase share out_es / out_ls
    int bdirs;             // BM_DIR_X | BM_DIR_Y
    float* out_y;          // omega_y
    float* phase;          // wrapped block phase, or nullptr
    // RM_LINE, optional temporal warm start: the previous frame's omega at
    // prev[p * prev_es + line * prev_ls] (nullptr: none)
    const float* prev;
    int64_t prev_es, prev_ls;
};

// All root-MUSIC work of one L: jobs[j] owns work items prefix[j] .. prefix[j+1)-1.
struct RmBatch {
    const RmJob* jobs;
    const int* prefix;     // njobs + 1 entries
    int njobs;
    int total;             // prefix[njobs]
    int jacobi;            // 1: cyclic Jacobi eigen-split instead of the tridiagonal solver
    int full_roots;        // 1: always find every root (no certified-pair shortcut)
    int block_windows;     // 1: every job is RM_BLOCK (256-lane blocks); 0: every job is RM_LINE
    int warm;              // 1: some job has a previous-frame map (line windows: the warm-start kernels)
    unsigned long long* stats;  // kStatSlots x kStatFields counters, or nullptr
    RootTemplate tmpl;
};

// Lines of one frame direction for the analytic-signal kernel (one block per line).
// A length n with a prime factor above 13 takes the DFT by Bluestein's chirp-z
// identity through a circular convolution of 5-smooth length m = plan.n >= 2n-1.
struct FftJob {
    const void* src;       // real lines, src_ls elements apart
    int64_t src_ls;
    float2* dst;           // complex lines, n apart
    const float2* tw;      // per-pass twiddle tables of plan.n (read from global memory: cached,
                           // and leaving LDS to more blocks measured faster than staging them)
    const float2* chirp;   // Bluestein only: e^{-i pi j^2 / n}, j < n
    const float2* kern;    // Bluestein only: DFT_m of the conjugate chirp, wrapped, divided by m
    int elem;              // Elem of src
    int nlines;
    int n;                 // line length
    FftPlan plan;          // plan of n, or of m under Bluestein (chirp != nullptr)
    int pow2;              // R0 of the register-resident path (n = 256 R0, R0 in 2, 4, 8, 16;
                           // plan = R0, 16, 16), 0 for the LDS Stockham path
};

// The register-resident path takes n = 256 R0, R0 in {2, 4, 8, 16}.
inline int fft_pow2_r0(int n) { return (n == 512 || n == 1024 || n == 2048 || n == 4096) ? n / 256 : 0; }

// LDS of the analytic kernel's block, in complex elements (132 KiB): two
// buffers of up to 8192 samples (or of a Bluestein transform length).
constexpr int kFftLdsElems = 16896;

// Transform lengths above this run 1024 threads per block, shorter ones 256.
constexpr int kFftWideMin = 2049;

// Work items (blocks) of one job: pairs of lines, 4096/n pairs per block on
// the register-resident path.
inline int fft_items(const FftJob& j) {
    const int pairs = (j.nlines + 1) / 2;
    if (!j.pow2) return pairs;
    const int per = 16 / j.pow2;
    return (pairs + per - 1) / per;
}

// Entries of the per-pass twiddle tables of a plan: (R - 1)(Ns + 1) per pass,
// at most plan.n + 64.
inline int fft_tw_len(const FftPlan& p) {
    int len = 0, ns = 1;
    for (int i = 0; i < p.passes; ++i) {
        len += (p.radix[i] - 1) * (ns + 1);
        ns *= p.radix[i];
    }
    return len;
}

// Dynamic LDS of one job's block, in complex elements (the register-resident
// path has its own static buffer).
inline int fft_lds_elems(const FftJob& j) { return j.pow2 ? 0 : 2 * j.plan.n; }

// True when the job's plan has a radix above 5.
inline bool fft_big_radix(const FftJob& j) {
    for (int p = 0; p < j.plan.passes; ++p)
        if (j.plan.radix[p] > 5) return true;
    return false;
}

// Kernel variant of a job: radices up to 5, or up to 13; 256 or 1024 threads;
// or the register-resident path of R0 = 2, 4, 8, 16 (classes 4 .. 7).
constexpr int kFftClasses = 8;
// A job of the 1024-thread kernel variants (classes 2 and 3).
inline bool fft_wide(const FftJob& j) { return !j.pow2 && j.plan.n >= kFftWideMin; }

inline int fft_class(const FftJob& j) {
    if (j.pow2) return j.pow2 == 2 ? 4 : j.pow2 == 4 ? 5 : j.pow2 == 8 ? 6 : 7;
    return (fft_big_radix(j) ? 1 : 0) + (j.plan.n >= kFftWideMin ? 2 : 0);
}

// Jobs are ordered by class: items [cls_from[c], cls_from[c+1]) run in the
// kernel variant of class c, with lds[c] complex elements of LDS per block.
struct FftBatch {
    const FftJob* jobs;
    const int* prefix;     // work items (fft_items): njobs + 1 entries
    int njobs;
    int total;
    int cls_from[kFftClasses + 1];
    int lds[kFftClasses];
};

// Transpose of one frame (rows x cols, src_ls elements per row) to cols x rows.
// Square tile of the batched transpose (elements per side).
constexpr int kTrTile = 64;       // real elements: 64 x 64 FP32 tiles
constexpr int kTrTileC = 32;      // complex (C32) elements: 32 x 32 tiles of float2

struct TrJob {
    const void* src;
    int64_t src_ls;
    void* dst;             // float (real input) or float2 (C32)
    int rows, cols;
    int tiles_x;           // tr_tile()-wide tiles along cols
    int elem;
};

// Tile side of a transpose job: float2 tiles of complex elements are half as wide.
inline int tr_tile(const TrJob& j) { return j.elem == (int)Elem::C32 ? kTrTileC : kTrTile; }

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
// Lanes per block of the block-window kernels: 256, or 128 above 8 x 8.
constexpr int block_window_lanes(int L) { return L <= kMaxL ? 256 : 128; }
// Block windows above 8 x 8 (odd sizes to kMaxBlockL), in their own translation unit.
hipError_t launch_big_block_window(int L, const RmBatch& b, int grid, hipStream_t s);
hipError_t launch_big_block_window_15_17(int L, const RmBatch& b, int grid, hipStream_t s);
// The same launch with the cyclic Jacobi eigen-split (L <= 8).
hipError_t launch_rootmusic_jacobi(int L, const RmBatch& b, int block, int grid, hipStream_t s);
// Output pixels per work item of a line: the line-window root-MUSIC kernel
// (line_kernel) covers two starts per lane, the block-window and surrogate
// kernels one.
int rootmusic_windows_per_block(int L, int block, bool line_kernel);
// Plain root-MUSIC on the *count windows of `list` ({job, line << 16 | pixel};
// lines and pixels are below 65536 because frame sides are), grid-stride over
// `grid` blocks of kGatherBlock lanes.
hipError_t launch_rootmusic_gather(int L, const RmBatch& b, const int2* list, const unsigned long long* count,
                                   int grid, hipStream_t s);

// Surrogate MLP 32 -> 64 -> 64 -> 2 (GELU), bfloat16 weights stored
// transposed (out x in) for the MFMA A operand, FP32 biases.
struct MlpWeights {
    const __bf16* w1t;     // [64][32]
    const __bf16* w2t;     // [64][64]
    const __bf16* w3t;     // [16][64], rows 2..15 zero
    const float* b1;       // [64]
    const float* b2;       // [64]
    const float* b3;       // [2]
};
constexpr int kMlpIn = 32, kMlpHidden = 64, kMlpOut = 2;
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden * kMlpOut + kMlpOut;   // 6402

struct SurBatch {
    RmBatch rm;            // the windows (jobs of one L)
    MlpWeights w;
    int predictor;         // 0: MLP, 1: lag-1 phase of the covariance (no learning)
    float tau;             // acceptance bound on the MUSIC null spectrum at the prediction
};

// Surrogate pass over every window of b.rm: the line kernel's blocks (256
// lanes, line_windows_per_block windows, one block per work item); windows
// the prediction does not serve are finished by the plain eigen-split.
hipError_t launch_surrogate(int L, const SurBatch& b, hipStream_t s);
// Y[M x 2] = MLP(X[M x 32]) with the kernel's bfloat16 arithmetic.
hipError_t launch_mlp_forward(const MlpWeights& w, const float* X, float* Y, int M, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s);

// Surrogate training.  Lines of 128 samples drawn by counter (Philox4x32-10)
// for ids first .. first+count-1; label windows {job = i >> 16, line = i & 0xFFFF,
// pixel 64}; features and targets of the centre window of each line.
hipError_t launch_gen_lines(float* lines, long long first, int count, unsigned long long seed, hipStream_t s);
hipError_t launch_label_entries(int2* list, int count, hipStream_t s);
hipError_t launch_train_features(const float2* gamma, int count, const float* labels, float* X, float* T,
                                 hipStream_t s);
int mlp_train_blocks(int M);
int mlp_partial_stride();
// Per-block gradient partials of the mean squared error over M samples (M % 64 == 0).
hipError_t launch_mlp_train(const MlpWeights& w, const __bf16* w2, const float* X, const float* T, int M, float* part,
                            int nblocks, hipStream_t s);
// Fixed-order sums of the partials into grad (optional) and loss (optional),
// then with adam != 0 one Adam step (bias corrections c1 = 1/(1-b1^t),
// c2 = 1/(1-b2^t)) on master with bfloat16 copies written to wts
// (W1^T | W2^T | W3^T | W2).
hipError_t launch_mlp_reduce_adam(const float* part, int nblocks, float* master, float* m, float* v, float* grad,
                                  float* loss, __bf16* wts, int adam, float lr, float c1, float c2, hipStream_t s);
hipError_t launch_transpose(const TrBatch& b, hipStream_t s);
hipError_t launch_analytic(const FftBatch& b, hipStream_t s);

hipError_t launch_synth(float2* g, int64_t n, float w0, float noise, hipStream_t s);

hipError_t launch_integrate(const float* wx, const float* wy, int W, int H, int Nx, int Ny,
                            double cx, double cy, double* anchor_ws, double* phi, hipStream_t s);

// One map of a batched integration: valid columns x0..x1, rows y0..y1 (the
// whole height without omega_y), anchor column at anchors + anchor_off.
struct IntJob {
    const float* wx;
    const float* wy;       // or nullptr
    double* phi;
    double cx, cy;
    int64_t anchor_off;
    int W, H, x0, x1, y0, y1;
    int vec;               // 16-byte loads and stores (integrate_row_vec)
};
// Anchors of every job (one block each), then every row of every job (rows
// job j own prefix[j] .. prefix[j+1]-1) by blocks of `threads` (at least
// integrate_row_threads of every job); lds_w sizes the row LDS (the widest
// job whose rows go through LDS, 0 if none).
hipError_t launch_integrate_many(const IntJob* jobs, const int* prefix, int njobs, int total_rows, int threads,
                                 int lds_w, double* anchors, hipStream_t s);
// Whether a map's rows load and store 16 bytes at a time (width a multiple of
// 4, at most 4096, omega_x and phi 16-byte aligned), and the threads a row
// needs; neither changes the arithmetic.
bool integrate_row_vec(int W, const void* wx, const void* phi);
int integrate_row_threads(int W);

// Allocation-free integration: the anchor column lives in a fixed device array
// of kNoAllocMaxHeight doubles (512 KiB); its address on the current device.
constexpr int kNoAllocMaxHeight = BOSMUSIC_NOALLOC_MAX_HEIGHT;
hipError_t noalloc_anchor_address(double** ptr);

// Raise the dynamic-LDS limit of the kernels that need more than 64 KiB; call
// once per device with that device current.
hipError_t analytic_set_attributes();
hipError_t integrate_set_attributes();

}  // namespace bm
