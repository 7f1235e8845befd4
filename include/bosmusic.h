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
 *     (Eq. 6-11): the top eigenvector of the real form of the covariance,
 *     by power iteration where an a-posteriori bound proves it within
 *     1e-5 rad, else by a tridiagonal solver (the power iteration starts
 *     at a line window's lag-1 phase, at a block window's summed lag-1
 *     phase, or at the surrogate's prediction);
 *   - root-MUSIC polynomial a(z)^H Un Un^H a(z) (Eq. 12) from the diagonal
 *     sums of the noise projector, degree 2L-2;
 *   - the root pair nearest the unit circle (Sec. 3, selection rule): found
 *     alone by Newton's method for the signal root and proven nearest by a
 *     root-count certificate, or, where that proof fails (or with
 *     BM_OPT_FULL_ROOTS), selected from all 2L-2 roots; omega = arg of the
 *     pair sum, equal to arg of the inner root (Eq. 15) in exact arithmetic.
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
 *     fit, windows whose covariance is identically zero or non-finite, and
 *     windows whose signal subspace is not determined (BM_FLAG_DEGENERATE)
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
    BM_U8 = 5,  /* real unsigned 8-bit, the camera's own samples (Sec. 4) */
};

/* directions, and the window shape */
enum {
    BM_DIR_X = 1u,
    BM_DIR_Y = 2u,
    /* The paper's own window (Sec. 3): the L x L block of the row-wise analytic
     * signal around the pixel (rows and columns y-floor(L/2) .., x-floor(L/2) ..,
     * valid iff it fits), whose L columns are the snapshots for omega_y and whose
     * L rows are the snapshots for omega_x (Eq. 4, 12-15; omega_x = -arg(z_x) of
     * the paper's E{Gamma^H Gamma} form).  Requires N == L; only BM_PLAIN. */
    BM_BLOCK = 4u,
};

/* demodulation modes */
enum { BM_PLAIN = 0, BM_SURROGATE = 1 };

/* handle options */
enum {
    BM_OPT_STATS = 1u,  /* count Jacobi sweeps and root iterations per call */
    BM_OPT_TIMING = 2u, /* time every root-MUSIC kernel launch with HIP events on its stream
                           (each launch alone on the device: no two-stream pipelining) */
    BM_OPT_JACOBI = 4u, /* signal subspace by cyclic Jacobi for every window (no power
                           iteration, no tridiagonal solver) */
    BM_OPT_GRAPH = 8u,  /* capture each distinct batch once into a hipGraph and replay it;
                           ignored when BM_OPT_TIMING is set */
    BM_OPT_FULL_ROOTS = 16u, /* always find every root of the polynomial, never the
                                certified-pair shortcut (same results up to rounding) */
};

/* per-pixel flag bits (optional output); bits 0-3 for x, 4-7 for y */
enum {
    BM_FLAG_UNDEFINED = 1u, /* border pixel, zero/non-finite covariance: omega is NaN */
    BM_FLAG_NO_POLISH = 2u, /* the FP64 pair polish failed; the FP32 pair sum was kept */
    BM_FLAG_DEGENERATE = 4u, /* the two largest eigenvalues of the covariance are within a
                                relative 1e-5 (lambda_1 <= lambda_2 (1 + 1e-5)): the
                                one-dimensional signal subspace of Eq. 6-11 is not
                                determined, e.g. two tones of equal power; omega is NaN */
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
    int32_t dtype;      /* BM_F16 / BM_F32 / BM_F64 / BM_C32 / BM_U8 */
    int32_t width;      /* pixels per row  (1 .. max_width)  */
    int32_t height;     /* number of rows  (1 .. max_height) */
    int64_t row_stride; /* elements between row starts, >= width */
    int32_t L;          /* covariance size, 2 <= L <= 8 */
    int32_t N;          /* window length, L <= N <= 64 */
    uint32_t dirs;      /* BM_DIR_X and/or BM_DIR_Y, optionally | BM_BLOCK */
    float* omega_x;     /* width*height, row stride = width; required iff BM_DIR_X */
    float* omega_y;     /* width*height, row stride = width; required iff BM_DIR_Y */
    uint8_t* flags;     /* optional width*height flag bytes (BM_FLAG_*), or NULL */
    float* phase;       /* optional, BM_BLOCK with both directions only: width*height, the
                           wrapped phase of the block's linear model at the pixel, i.e.
                           Eq. 15's alpha = arg(mean(Gamma_w e^{-j(omega_x x + omega_y y)}))
                           with x, y measured from the pixel; NaN where omega is; or NULL */
    /* Temporal warm start (optional; line windows; ignored by BM_SURROGATE): the omega maps of
     * the previous frame of a time-lapsed series, the same size, row stride =
     * width (the paper's premise that the phase changes little between
     * successive frames, Sec. 1 and 4).  Where the previous frequency at the
     * pixel is finite, the Newton iteration for the window's signal root
     * starts in its direction instead of the window's own lag-1 direction.
     * The certified pair, hence omega, is the same either way (up to
     * rounding); only the iteration counts change.  NULL: no warm start. */
    const float* prev_omega_x;
    const float* prev_omega_y;
} bosmusic_frame;

typedef struct {
    uint64_t windows;       /* windows demodulated since the last reset (in BM_PLAIN:
                               sur_accepted + sur_rejected + the BM_FLAG_DEGENERATE ones;
                               in BM_SURROGATE: sur_accepted + sur_rejected) */
    uint64_t eig_iters;     /* sum over windows of eigen-split iterations: power steps of the
                               power_windows, Newton steps of the tridiagonal solver for the
                               rest (Jacobi sweeps with BM_OPT_JACOBI) */
    uint64_t root_iters;    /* sum over windows of simultaneous root iterations (all-roots windows) */
    uint64_t polish_fail;   /* windows whose FP64 pair polish did not converge */
    uint64_t sur_accepted;  /* BM_SURROGATE: windows whose signal eigenvector came from the
                               prediction (proven converged, null spectrum at the
                               prediction <= tau);
                               BM_PLAIN: windows finished by the certified pair */
    uint64_t sur_rejected;  /* BM_SURROGATE: windows finished by the plain eigen-split;
                               BM_PLAIN: windows whose roots were all found */
    uint64_t pair_iters;    /* sum over windows of FP64 Newton steps for the signal root
                               (its mate divided out) before the certificate */
    uint64_t rm_launches;   /* root-MUSIC kernel launches timed (BM_OPT_TIMING) */
    uint64_t rm_time_ns;    /* their summed duration between HIP events, ns */
    uint64_t pair_iters32;  /* sum over windows of FP32 Newton steps for the signal root,
                               taken before the FP64 ones */
    uint64_t power_windows; /* windows whose signal eigenvector came from the verified power
                               iteration (the rest took the tridiagonal solver); eig_iters
                               holds their power steps */
} bosmusic_stats;

/* Create a handle on cfg->device, allocating the workspace for frames up to
 * max_width x max_height.  *out receives the handle (NULL on failure).
 * Test hooks read here from the environment: BOSMUSIC_FAULT=alloc makes the
 * workspace allocation fail (BM_E_NOMEM after the clean-up), BOSMUSIC_LOG=1
 * makes the handle write one line per create, planned group and graph
 * capture or replay to stderr. */
bm_status bosmusic_create(const bosmusic_config* cfg, bosmusic_t* out);

/* Release the handle and its workspace (synchronises its device). NULL is OK. */
bm_status bosmusic_destroy(bosmusic_t h);

/* Demodulate n_frames frames (paper Sec. 3, Eq. 2-15, per pixel and per
 * requested direction) into their omega maps, enqueued on `stream`.
 * Frames may differ in size, dtype, L and N.  Frames are grouped so that each
 * group fits the workspace; per group the work runs as one batched transpose
 * launch, one batched analytic-signal launch and one root-MUSIC launch per
 * distinct L (with BM_OPT_GRAPH: one replay of a cached hipGraph holding them,
 * the per-L launches on forked streams).  Without BM_OPT_GRAPH and
 * BM_OPT_TIMING, a group of two or more frames runs as two halves on
 * `stream` and a second stream of the handle: the second half's transpose
 * and analytic launches run beside the first half's root-MUSIC launch, its
 * root-MUSIC launch after the first half's; `stream` waits for the second
 * stream before the call returns, so every output is ordered on `stream`
 * as if the work had been enqueued there alone.  (Not when the second half
 * has a real line longer than 2048 samples whose length is not a power of
 * two: the analytic step's 1024-thread blocks for it cannot run beside a
 * root-MUSIC launch, so the group runs in `stream` alone.)  The job tables of a group are
 * uploaded from pinned host memory on `stream`; the call may wait for the
 * previous call's upload to finish before reusing that buffer.
 * mode: BM_PLAIN, or BM_SURROGATE (needs loaded parameters unless the
 * lag-1 predictor is configured, and N >= 16 for every frame).
 * Requirements per frame: 2 <= L <= 8, L <= N <= 64, width/height within
 * the handle's maximum, row_stride >= width; for real dtypes the length of
 * every requested direction must either factor into 2, 3, 5, 7, 11 and 13
 * and be <= 8192, or be <= 4096 (any factors: the exact DFT of the analytic
 * step then goes through Bluestein's chirp-z identity at a 5-smooth length
 * >= 2n - 1, about four times the transform work).  A window longer than the
 * frame is not an error: the whole map is NaN. */
bm_status bosmusic_demodulate(bosmusic_t h, const bosmusic_frame* frames, int32_t n_frames,
                              int32_t mode, void* stream);

/* Integrate omega maps to phase (FP64 trapezoid rule on the window-centre
 * grid), enqueued on `stream`.  This replaces the paper's route from the
 * frequencies to the phase (Sec. 3 after Eq. 15: the per-window offset alpha
 * of Eq. 15, then phase unwrapping): the local frequencies are the phase
 * derivatives, so their running sums give the unwrapped phase directly.  Anchor phi = 0 at column floor(Nx/2) and,
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

/* ---- learned surrogate (BM_SURROGATE) -------------------------------------
 * An MLP 32 -> 64 -> 64 -> 2 (exact-erf GELU) maps the normalised window (16
 * central samples de-rotated by the central sample's phase, divided by the
 * window's RMS magnitude, [Re(16), Im(16)]) to (cos w, sin w); it runs on
 * one window in 32 of a line and its estimate w_hat serves those 32.  w_hat
 * seeds a power iteration on the window's FB-averaged covariance (in its
 * real form, paper Eq. 6-11) for the signal eigenvector u1, accepted once an
 * a-posteriori bound proves it within 1e-5 rad of the top eigenvector and
 * the MUSIC null spectrum 1 - |u1^H a(w_hat)|^2 / L at the prediction is at
 * most tau.  Any other window takes the plain eigen-split.  From u1 on every
 * window follows the plain path (polynomial, Eq. 12-14; certified pair or
 * all roots; w = arg(z1 + z2), Eq. 15), so the output equals the plain
 * output up to the eigenvector bound and rounding.  Line windows with
 * L <= 8 and N >= 16 only.
 * Parameters are FP32, in this order, row-major: W1[32][64], b1[64],
 * W2[64][64], b2[64], W3[64][2], b3[2] (6402 floats); the kernels use
 * bfloat16 copies (round to nearest even) and FP32 accumulation. */
#define BOSMUSIC_MLP_PARAMS 6402

/* Load FP32 parameters from host memory (n must be BOSMUSIC_MLP_PARAMS).
 * Synchronous. */
bm_status bosmusic_surrogate_load(bosmusic_t h, const float* params, int64_t n);

/* Copy the current FP32 parameters to host memory. Synchronous. */
bm_status bosmusic_surrogate_save(bosmusic_t h, float* params, int64_t n);

/* Training checkpoint for an exact resume: state[3 * BOSMUSIC_MLP_PARAMS]
 * (host) = the FP32 parameters, then Adam's first and second moments, in
 * the parameter order; *adam_step = the Adam step count.  A handle given
 * the same state by bosmusic_surrogate_set_state and then the same training
 * calls (same data, batch, steps, lr) reaches the same parameters bit for
 * bit: the minibatches follow from those arguments, the training data from
 * (first_line, seed) of bosmusic_surrogate_dataset, and the gradient sums
 * are in a fixed order.  Both calls synchronise the device.  n must be
 * 3 * BOSMUSIC_MLP_PARAMS; set_state refuses non-finite values, a negative
 * second moment or a negative step count (BM_E_INVALID_ARG) before it
 * changes anything. */
bm_status bosmusic_surrogate_get_state(bosmusic_t h, float* state, int64_t n, int64_t* adam_step);
bm_status bosmusic_surrogate_set_state(bosmusic_t h, const float* state, int64_t n, int64_t adam_step);

/* Bound tau on the null spectrum at the prediction (default 0.25) and predictor:
 * 0 = the MLP, 1 = the lag-1 phase of the covariance (a non-learned
 * predictor, for comparison). */
bm_status bosmusic_surrogate_config(bosmusic_t h, float tau, int32_t predictor);

/* Y[M][2] = MLP(X[M][32]) on the device (X, Y device pointers, FP32), with
 * the same bfloat16 arithmetic as BM_SURROGATE.  Enqueued on `stream`. */
bm_status bosmusic_surrogate_forward(bosmusic_t h, const float* X, float* Y, int32_t M, void* stream);

/* ---- surrogate training ----------------------------------------------------
 * The network is trained on windows and labels the method produces itself.
 * Training line i (0 <= i < 2^32) has 128 samples
 *     0.5 + 0.4 cos(w n + theta) + sqrt(0.08 * 10^(-SNR/10)) z_n,
 * w = 2 pi/16 + u0 (2 pi/4 - 2 pi/16), theta = 2 pi u1, SNR = 30 u2 dB, with
 * (u0, u1, u2) from Philox4x32-10 (Salmon et al., SC'11) at counter
 * (i, 0, 0, 0) and key (seed low, seed high), u = (x + 0.5) / 2^32, and the
 * Gaussian noise z of samples 4b..4b+3 from counter (i, b+1, 0, 0) by two
 * Box-Muller pairs (r cos, r sin of words 0,1 and of words 2,3).  Its label is
 * the plain root-MUSIC frequency (Sec. 3, Eq. 15) of the window N = 32,
 * L = 8 centred on sample 64 of the line's analytic signal (Eq. 1); its
 * features are those of that window, its target (cos, sin) of the label. */

/* Generate lines first_line .. first_line+count-1: X[count][32] features,
 * T[count][2] targets and, when omega is not NULL, omega[count] labels, all
 * device pointers (FP32) owned by the caller.  Works on `stream` and
 * returns after synchronising it. */
bm_status bosmusic_surrogate_dataset(bosmusic_t h, int64_t first_line, int64_t count, uint64_t seed, float* X,
                                     float* T, float* omega, void* stream);

/* Gradient of the mean over the M samples (M a positive multiple of 64) of
 * the squared error |MLP(X_m) - T_m|^2 with respect to the parameters at the
 * current weights (bfloat16 operands, FP32 accumulation, the bfloat16
 * roundings taken as identity).  grad[BOSMUSIC_MLP_PARAMS] in the parameter
 * order and loss[1] (may be NULL) are device pointers.  Enqueued on `stream`;
 * the result does not depend on scheduling (fixed summation order). */
bm_status bosmusic_surrogate_grad(bosmusic_t h, const float* X, const float* T, int32_t M, float* grad, float* loss,
                                  void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * count since the last bosmusic_surrogate_load) on the FP32 parameters with
 * the device gradient grad[BOSMUSIC_MLP_PARAMS]; refreshes the bfloat16
 * copies.  Enqueued on `stream`. */
bm_status bosmusic_surrogate_step(bosmusic_t h, const float* grad, float lr, void* stream);

/* `steps` Adam steps of minibatch training over X[M][32], T[M][2] (device):
 * step s uses the batch of `batch` samples (a multiple of 64) starting at
 * ((s mod (M / batch)) * batch), continuing the handle's step count.  With
 * `losses` (host, `steps` floats) non-NULL, receives the loss of each step
 * before its update and returns after synchronising `stream`; otherwise
 * only enqueues. */
bm_status bosmusic_surrogate_train(bosmusic_t h, const float* X, const float* T, int64_t M, int32_t batch,
                                   int32_t steps, float lr, float* losses, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * integration of bosmusic_integrate, with the same arguments and results
 * (the same kernels), but without a handle and without allocating anything.
 * It runs on the current HIP device; the anchor column it needs lives in a
 * fixed device array of BOSMUSIC_NOALLOC_MAX_HEIGHT doubles (512 KiB) that the
 * library keeps on every device it runs on until the process ends, looked up
 * on the first call on each device.  height > BOSMUSIC_NOALLOC_MAX_HEIGHT, or
 * any other argument bosmusic_integrate would refuse, returns
 * BM_E_INVALID_ARG before anything is enqueued; the detail is in
 * bosmusic_last_error(NULL).  Every call on one device uses that device's one
 * array (each call writes the rows it reads, nothing carries over): calls that
 * overlap on one device, on different streams or threads, race on it and
 * must be ordered by the caller. */
#define BOSMUSIC_NOALLOC_MAX_HEIGHT 65536
bm_status bosmusic_integrate_noalloc(const float* omega_x, const float* omega_y, int32_t width, int32_t height,
                                     int32_t Nx, int32_t Ny, double carrier_x, double carrier_y, double* phi,
                                     void* stream);

/* One map of a batched integration: the arguments of bosmusic_integrate. */
typedef struct {
    const float* omega_x;   /* width*height, required */
    const float* omega_y;   /* width*height, or NULL (every row then starts at 0) */
    int32_t width, height;  /* width <= 8192 */
    int32_t Nx, Ny;         /* window lengths the maps were made with (Ny ignored without omega_y) */
    double carrier_x, carrier_y;
    double* phi;            /* width*height FP64 output */
} bosmusic_integrate_job;

/* bosmusic_integrate for n maps in two launches (all anchor columns, then
 * every row of every map), results identical to n single calls.  The job
 * table is uploaded from pinned host memory on `stream`; the call may wait
 * for its previous upload before reusing that buffer.  Maps must not overlap
 * another job's phi. */
bm_status bosmusic_integrate_many(bosmusic_t h, const bosmusic_integrate_job* jobs, int32_t n, void* stream);

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
