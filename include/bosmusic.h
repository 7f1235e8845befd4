/*
 * bosmusic -- sliding-window root-MUSIC fringe demodulation on AMD Instinct
 * MI355X (gfx950).
 *
 * The library computes, for every pixel of every frame of a time-lapsed
 * fringe image stack (paper, Sec. 2: the recorded frames form an image stack,
 * each a carrier-modulated cosinusoidal intensity), the local fringe
 * frequency along x and/or y by root-MUSIC over a moving window (paper,
 * Sec. 3, Eq. 2-15), and integrates the frequency maps to a phase map
 * (the paper recovers the global phase from the per-window estimates,
 * Sec. 3 after Eq. 15).
 *
 * Per pixel and direction the steps are:
 *   - complex analytic fringe signal Gamma of Eq. 1 along the window
 *     direction (exact one-sided DFT mask, DC and Nyquist removed, carrier
 *     kept); complex input is used as Gamma directly;
 *   - window of N samples starting at x - floor(N/2) (valid iff it fits);
 *   - L x L sample autocorrelation of the K = N-L+1 length-L sub-snapshots
 *     (Eq. 4), forward-backward averaged;
 *   - signal/noise eigen-split with a one-dimensional signal subspace
 *     (Eq. 6-11);
 *   - root-MUSIC polynomial a(z)^H Un Un^H a(z) (Eq. 12) from the diagonal
 *     sums of the noise projector, degree 2L-2, and all its roots;
 *   - the root pair nearest the unit circle; omega = arg of the pair sum,
 *     equal to arg of the inner root (Eq. 15) in exact arithmetic.
 *
 * Conventions
 *   - Every call returns a bm_status; nothing throws or aborts across this
 *     boundary.  Arguments are validated before anything is enqueued; on a
 *     validation error nothing is enqueued and outputs are untouched.
 *   - All frame and map pointers are DEVICE pointers owned by the caller and
 *     must stay valid until the work enqueued on `stream` has completed.
 *     `stream` is a hipStream_t (NULL = the default stream); calls only
 *     enqueue work and return without synchronising, except where noted.
 *   - omega is in rad/px in [-pi, pi]; border pixels whose window does not
 *     fit, and windows whose covariance is identically zero or non-finite,
 *     are NaN.  phi is in rad, FP64, NaN outside the integrated region.
 *   - A handle owns its workspace and serves one stream at a time; it is not
 *     thread-safe.  Separate handles are independent.
 */
#ifndef BOSMUSIC_H
#define BOSMUSIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BOSMUSIC_VERSION 1

typedef struct bosmusic_s* bosmusic_t;

typedef int32_t bm_status;
enum {
    BM_OK = 0,
    BM_E_INVALID_ARG = -1, /* bad pointer, size, L/N, dtype or direction */
    BM_E_UNSUPPORTED = -2, /* valid request this build does not implement */
    BM_E_NOMEM = -3,       /* device or host allocation failed */
    BM_E_DEVICE = -4,      /* HIP runtime error (no device, launch failure) */
};

/* element type of a frame */
enum {
    BM_F16 = 1, /* real IEEE half   */
    BM_F32 = 2, /* real float       */
    BM_F64 = 3, /* real double      */
    BM_C32 = 4, /* interleaved complex float: Gamma of Eq. 1 given directly */
};

/* directions */
enum { BM_DIR_X = 1u, BM_DIR_Y = 2u };

/* demodulation modes */
enum { BM_PLAIN = 0, BM_SURROGATE = 1 };

/* handle options */
enum {
    BM_OPT_STATS = 1u,  /* count Jacobi sweeps and root iterations per call */
    BM_OPT_TIMING = 2u, /* time every root-MUSIC kernel launch with HIP events on its stream */
    BM_OPT_JACOBI = 4u, /* signal subspace by cyclic Jacobi instead of the tridiagonal solver */
    BM_OPT_GRAPH = 8u,  /* capture each distinct batch once into a hipGraph and replay it;
                           ignored when BM_OPT_TIMING is set */
};

/* per-pixel flag bits (optional output); bits 0-3 for x, 4-7 for y */
enum {
    BM_FLAG_UNDEFINED = 1u, /* border pixel, zero/non-finite covariance: omega is NaN */
    BM_FLAG_NO_POLISH = 2u, /* the FP64 pair polish failed; the FP32 pair sum was kept */
};

typedef struct {
    int32_t device;           /* HIP device ordinal */
    int32_t max_width;        /* frames wider or taller than this are rejected */
    int32_t max_height;
    uint32_t options;         /* BM_OPT_* */
    int64_t max_batch_pixels; /* workspace: pixels of frames processed together in one
                                 launch group (20 B each); 0 = max_width * max_height.
                                 Larger batches are split into groups that fit. */
    const char* tune_cache;   /* autotuner cache file (JSON lines) or NULL: no cache */
} bosmusic_config;

typedef struct {
    const void* data;   /* device pointer to height rows of row_stride elements */
    int32_t dtype;      /* BM_F16 / BM_F32 / BM_F64 / BM_C32 */
    int32_t width;      /* pixels per row  (1 .. max_width)  */
    int32_t height;     /* number of rows  (1 .. max_height) */
    int64_t row_stride; /* elements between row starts, >= width */
    int32_t L;          /* covariance size, 2 <= L <= 8 */
    int32_t N;          /* window length, L <= N <= 64 */
    uint32_t dirs;      /* BM_DIR_X | BM_DIR_Y, nonzero */
    float* omega_x;     /* width*height, row stride = width; required iff BM_DIR_X */
    float* omega_y;     /* width*height, row stride = width; required iff BM_DIR_Y */
    uint8_t* flags;     /* optional width*height flag bytes (BM_FLAG_*), or NULL */
} bosmusic_frame;

typedef struct {
    uint64_t windows;       /* windows demodulated since the last reset */
    uint64_t eig_iters;     /* sum over windows of Newton steps (Jacobi sweeps with BM_OPT_JACOBI) */
    uint64_t root_iters;    /* sum over windows of simultaneous root iterations */
    uint64_t polish_fail;   /* windows whose FP64 pair polish did not converge */
    uint64_t rm_launches;   /* root-MUSIC kernel launches timed (BM_OPT_TIMING) */
    uint64_t rm_time_ns;    /* their summed duration between HIP events, ns */
} bosmusic_stats;

/* Create a handle on cfg->device, allocating the workspace for frames up to
 * max_width x max_height.  *out receives the handle (NULL on failure). */
bm_status bosmusic_create(const bosmusic_config* cfg, bosmusic_t* out);

/* Release the handle and its workspace (synchronises its device). NULL is OK. */
bm_status bosmusic_destroy(bosmusic_t h);

/* Demodulate n_frames frames (paper Sec. 3, Eq. 2-15, per pixel and per
 * requested direction) into their omega maps, enqueued on `stream`.
 * Frames may differ in size, dtype, L and N.  Frames are grouped so that each
 * group fits the workspace; per group the work runs as one batched transpose
 * launch, one batched analytic-signal launch and one root-MUSIC launch per
 * distinct L (with BM_OPT_GRAPH: one replay of a cached hipGraph holding them,
 * the per-L launches on forked streams).  The job tables of a group are
 * uploaded from pinned host memory on `stream`; the call may wait for the
 * previous call's upload to finish before reusing that buffer.
 * mode: BM_PLAIN (BM_SURROGATE returns BM_E_UNSUPPORTED in this build).
 * Requirements per frame: 2 <= L <= 8, L <= N <= 64, width/height within
 * the handle's maximum, row_stride >= width; for real dtypes the length of
 * every requested direction must factor into 2, 3 and 5 and be <= 8192
 * (exact DFT analytic step).  A window longer than the frame is not an error:
 * the whole map is NaN. */
bm_status bosmusic_demodulate(bosmusic_t h, const bosmusic_frame* frames, int32_t n_frames,
                              int32_t mode, void* stream);

/* Integrate omega maps to phase (FP64 trapezoid rule on the window-centre
 * grid), enqueued on `stream`.  Anchor phi = 0 at column floor(Nx/2) and,
 * when omega_y is given, row floor(Ny/2): first down the anchor column with
 * omega_y - carrier_y, then along every row with omega_x - carrier_x.
 * Without omega_y (NULL) every row starts at 0 in the anchor column.  phi is
 * width*height doubles (row stride = width), NaN outside columns
 * [floor(Nx/2), width-Nx+floor(Nx/2)] and, with omega_y, rows
 * [floor(Ny/2), height-Ny+floor(Ny/2)].  width <= 8192. */
bm_status bosmusic_integrate(bosmusic_t h, const float* omega_x, const float* omega_y,
                             int32_t width, int32_t height, int32_t Nx, int32_t Ny,
                             double carrier_x, double carrier_y, double* phi, void* stream);

/* Copy the handle's counters (BM_OPT_STATS, BM_OPT_TIMING) after
 * synchronising `stream`; reset = 1 zeroes them afterwards.  Counters of an
 * option that is not set read zero. */
bm_status bosmusic_get_stats(bosmusic_t h, bosmusic_stats* out, int32_t reset, void* stream);

/* Autotune the root-MUSIC launch for covariance size L and window N on the
 * handle's device: times every candidate tile shape (128 or 256 lanes per
 * block) and grid size (one block per work item, or 1..16 resident blocks
 * per compute unit walking the work list) with HIP events on a synthetic
 * line set of `lines` lines x `width` samples, keeps the fastest for later
 * bosmusic_demodulate calls with this (L, N), and appends it to the handle's
 * tune cache file if one was given.  Results do not depend on the choice.
 * Synchronises `stream`.  *best_us (optional) receives the best time. */
bm_status bosmusic_autotune(bosmusic_t h, int32_t L, int32_t N, int32_t width, int32_t lines,
                            double* best_us, void* stream);

/* Static text for a status code. */
const char* bosmusic_status_string(bm_status s);

/* Detail of the last error on this handle (or of the last failed create when
 * h is NULL); empty string if none.  Valid until the next call on h. */
const char* bosmusic_last_error(bosmusic_t h);

/* BOSMUSIC_VERSION of the built library. */
int32_t bosmusic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BOSMUSIC_H */
