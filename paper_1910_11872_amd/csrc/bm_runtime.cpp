// Host runtime behind the bosmusic C ABI: handle, workspace, validation,
// batch planning (job tables for the batched transpose, analytic-signal and
// root-MUSIC kernels), hipGraph capture and replay, the autotuner and its
// cache, DFT plans and twiddle tables, and root templates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bm_internal.h"

namespace {

struct Tune {
    int block = 256;       // lanes per block
    int grid_per_cu = 0;   // 0: one block per work item; k: k * CU-count resident blocks
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* blob = nullptr;  // device job tables referenced by the graph's kernels
    uint64_t last_use = 0;
};

constexpr int kMaxGraphs = 8;
constexpr int kMaxForks = bm::kMaxL;   // one capture stream per distinct L

}  // namespace

struct bosmusic_s {
    int device = 0;
    int max_w = 0, max_h = 0;
    uint32_t options = 0;
    int cu_count = 1;
    std::string arch;
    char* ws = nullptr;           // workspace: analytic signals and transposed frames
    size_t ws_bytes = 0;
    double* anchor = nullptr;     // integration anchor column (max_h)
    unsigned long long* stats = nullptr;
    std::map<int, float2*> twiddles;
    std::map<int, float2*> bluestein;   // line length -> chirp (n) then kernel (m) in one allocation
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;
    uint64_t rm_launches = 0, rm_time_ns = 0;
    bm::RootTemplate tmpl[bm::kMaxBlockL + 1];
    Tune tune[bm::kMaxL + 1][bm::kMaxN + 1];
    std::string tune_path;
    // eager job-table upload
    char* pin = nullptr;
    size_t pin_bytes = 0;
    void* djobs = nullptr;
    size_t djobs_bytes = 0;
    hipEvent_t pin_ev = nullptr;
    bool pin_pending = false;
    // graphs
    std::map<std::string, GraphEntry> graphs;
    uint64_t tick = 0;
    hipStream_t cap[kMaxForks] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kMaxForks] = {};
    hipEvent_t pipe_ev[3] = {};    // eager two-stream pipeline of a group's halves
    hipStream_t last_graph_stream = nullptr;
    // surrogate
    float* sur_master = nullptr;   // FP32 parameters (BOSMUSIC_MLP_PARAMS)
    __bf16* sur_w = nullptr;       // bfloat16 W1^T [64][32] | W2^T [64][64] | W3^T [16][64] | W2 [64][64]
    bool sur_loaded = false;
    float sur_tau = 0.25f;
    int sur_predictor = 0;
    bool log = false;              // BOSMUSIC_LOG=1 at create
    // surrogate training
    float* adam_m = nullptr;       // Adam moments (BOSMUSIC_MLP_PARAMS each)
    float* adam_v = nullptr;
    int64_t adam_t = 0;            // Adam steps since the last load
    float* part = nullptr;         // per-block gradient partials
    int part_blocks = 0;
    float* losses = nullptr;       // per-step losses of a train call
    int losses_cap = 0;
    char* ds = nullptr;            // dataset generation buffers
    size_t ds_bytes = 0;
    // batched integration: job tables (pinned staging + device copy) and anchor columns
    char* int_pin = nullptr;
    void* int_dev = nullptr;
    size_t int_bytes = 0;
    hipEvent_t int_ev = nullptr;
    bool int_pending = false;
    double* int_anchor = nullptr;
    size_t int_anchor_cap = 0;
    std::string err;
};

namespace {

// Detail of the last failed handle-less call on this thread (create, the
// allocation-free integration): a fixed buffer, so that reporting allocates nothing.
thread_local char g_create_error[512];

bm_status fail(bosmusic_s* h, bm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else std::memcpy(g_create_error, buf, sizeof(buf));
    return st;
}

// Test hooks read from the environment at each create: BOSMUSIC_FAULT=alloc makes
// the workspace allocation of bosmusic_create fail after its first buffer is
// allocated (the clean-up path, BM_E_NOMEM); BOSMUSIC_LOG=1 writes one line per
// create, call plan and graph capture or replay to stderr.
bool env_is(const char* name, const char* value) {
    const char* v = std::getenv(name);
    return v && std::strcmp(v, value) == 0;
}

void log_line(const bosmusic_s* h, const char* fmt, ...);

bm_status check(bosmusic_s* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return BM_OK;
    return fail(h, BM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void log_line(const bosmusic_s* h, const char* fmt, ...) {
    if (!h || !h->log) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[bosmusic] %s\n", buf);
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    hipError_t status = hipSuccess;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        status = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool plan_fft(int n, bm::FftPlan& p) {
    if (n < 1 || n > bm::kMaxFFT) return false;
    p.n = n;
    p.passes = 0;
    int r = n;
    const int order[7] = {4, 2, 3, 5, 7, 11, 13};
    for (int f : order) {
        while (r % f == 0) {
            if (p.passes >= bm::kMaxRadixPasses) return false;
            p.radix[p.passes++] = f;
            r /= f;
        }
    }
    return r == 1;
}

// The mixed-radix FFT takes n directly (factors 2, 3, 5, 7, 11, 13 only).
bool fft_direct(int n) {
    bm::FftPlan p;
    return plan_fft(n, p);
}

// Transform length of Bluestein's route for a line of n samples: the least
// 5-smooth m >= 2n - 1 (radix 2-5 passes only), or 0 when that exceeds the
// largest FFT.
int bluestein_len(int n) {
    for (int m = std::max(2 * n - 1, 1); m <= bm::kMaxFFT; ++m) {
        int r = m;
        for (int f : {2, 3, 5})
            while (r % f == 0) r /= f;
        if (r == 1) return m;
    }
    return 0;
}

// A line of n samples has an exact DFT here: directly or by Bluestein.
bool dft_supported(int n) { return n >= 1 && (fft_direct(n) || bluestein_len(n) > 0); }

// In-place FP64 DFT (recursive decimation in time by the smallest prime factor).
void dft64(std::vector<std::complex<double>>& x) {
    const int n = (int)x.size();
    if (n == 1) return;
    int p = 2;
    while (n % p) ++p;
    const int q = n / p;
    std::vector<std::vector<std::complex<double>>> sub(p, std::vector<std::complex<double>>(q));
    for (int r = 0; r < p; ++r)
        for (int k = 0; k < q; ++k) sub[r][k] = x[(size_t)k * p + r];
    for (auto& s : sub) dft64(s);
    for (int k = 0; k < n; ++k) {
        std::complex<double> acc = 0.0;
        for (int r = 0; r < p; ++r) {
            const double a = -2.0 * M_PI * (double)(((int64_t)r * k) % n) / (double)n;
            acc += sub[r][k % q] * std::complex<double>(std::cos(a), std::sin(a));
        }
        x[k] = acc;
    }
}

// Roots of the noise-free root-MUSIC polynomial of a tone at frequency 0.
// With u1 = a(0)/sqrt(L), sum_k c_k w^{k+L-1} = L w^{L-1} - (1/L) (sum_{i<L} w^i)^2.
// Its double root at w = 1 is divided out and replaced by (rho, 1/rho); the
// remaining 2L-4 roots are found by Durand-Kerner in double precision.
void make_template(int L, bm::RootTemplate& t) {
    using cd = std::complex<double>;
    const int n = 2 * L - 2;
    std::vector<double> p(n + 1, 0.0);  // ascending
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) p[i + j] -= 1.0 / L;
    p[L - 1] += L;
    for (int rep = 0; rep < 2; ++rep) {  // divide by (w - 1), highest power first
        const int deg = (int)p.size() - 1;
        std::vector<double> q(deg, 0.0);
        double carry = 0.0;
        for (int k = deg; k >= 1; --k) {
            carry = p[k] + carry;
            q[k - 1] = carry;
        }
        p = q;
    }
    const int m = (int)p.size() - 1;  // 2L-4
    std::vector<cd> z(m);
    for (int i = 0; i < m; ++i) z[i] = std::polar(1.3, 2.0 * M_PI * (i + 0.25) / std::max(m, 1) + 0.4);
    for (int it = 0; it < 2000 && m > 0; ++it) {
        double mx = 0.0;
        for (int i = 0; i < m; ++i) {
            cd v = p[m];
            for (int k = m - 1; k >= 0; --k) v = v * z[i] + p[k];
            cd d = p[m];
            for (int j = 0; j < m; ++j)
                if (j != i) d *= (z[i] - z[j]);
            const cd step = v / d;
            z[i] -= step;
            mx = std::max(mx, std::abs(step));
        }
        if (mx < 1e-15) break;
    }
    const double rho = 0.9;
    t.re[0] = (float)rho;
    t.im[0] = 0.f;
    t.re[1] = (float)(1.0 / rho);
    t.im[1] = 0.f;
    for (int i = 0; i < m; ++i) {
        t.re[2 + i] = (float)z[i].real();
        t.im[2 + i] = (float)z[i].imag();
    }
    for (int i = n; i < 2 * bm::kMaxBlockL - 2; ++i) t.re[i] = t.im[i] = 0.f;
}

// Per-pass twiddle tables of the mixed-radix plan of n: for pass p with
// radix R and stride Ns, e^{-2 pi i r k / (Ns R)} at (r - 1) Ns + k (0 < r < R,
// k < Ns), then the butterfly constants e^{-2 pi i r / R} (0 < r < R); the
// angle is reduced exactly (r k mod Ns R) and evaluated in FP64, rounded once.
// The register-resident path's plan R0, 16, 16 has its own tables, cached
// under -n.
bm_status get_twiddles(bosmusic_s* h, int n, const float2** out, int pow2 = 0) {
    bm::FftPlan plan;
    if (pow2) {
        plan.n = n;
        plan.passes = 3;
        plan.radix[0] = pow2;
        plan.radix[1] = plan.radix[2] = 16;
    } else if (!plan_fft(n, plan)) {
        return fail(h, BM_E_UNSUPPORTED, "twiddles of %d", n);
    }
    const int key = pow2 ? -n : n;
    auto it = h->twiddles.find(key);
    if (it != h->twiddles.end()) {
        *out = it->second;
        return BM_OK;
    }
    std::vector<float2> tw;
    tw.reserve(bm::fft_tw_len(plan));
    auto put = [&](int64_t num, int64_t den) {
        const double a = -2.0 * M_PI * (double)(num % den) / (double)den;
        tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
    };
    int ns = 1;
    for (int p = 0; p < plan.passes; ++p) {
        const int R = plan.radix[p];
        for (int r = 1; r < R; ++r)
            for (int k = 0; k < ns; ++k) put((int64_t)r * k, (int64_t)ns * R);
        for (int r = 1; r < R; ++r) put(r, R);
        ns *= R;
    }
    float2* d = nullptr;
    if (hipMalloc(&d, sizeof(float2) * tw.size()) != hipSuccess) return fail(h, BM_E_NOMEM, "twiddle table of %d", n);
    if (hipMemcpy(d, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return fail(h, BM_E_DEVICE, "twiddle upload failed");
    }
    h->twiddles[key] = d;
    *out = d;
    return BM_OK;
}

// Chirp w_j = e^{-i pi j^2 / n} (j < n) and the length-m DFT of the wrapped
// conjugate chirp c_t = conj(w_t), |t| < n, divided by m; computed in FP64
// (the angle reduced exactly as j^2 mod 2n) and rounded once.
bm_status get_bluestein(bosmusic_s* h, int n, int m, const float2** chirp, const float2** kern) {
    auto it = h->bluestein.find(n);
    if (it == h->bluestein.end()) {
        using cd = std::complex<double>;
        std::vector<cd> w(n), c(m, cd(0.0, 0.0));
        for (int j = 0; j < n; ++j) {
            const int64_t r = ((int64_t)j * j) % (2 * (int64_t)n);
            const double a = -M_PI * (double)r / (double)n;
            w[j] = cd(std::cos(a), std::sin(a));
        }
        for (int t = 0; t < n; ++t) {
            c[t] = std::conj(w[t]);
            if (t > 0) c[m - t] = std::conj(w[t]);
        }
        dft64(c);
        std::vector<float2> host((size_t)n + m);
        for (int j = 0; j < n; ++j) host[j] = make_float2((float)w[j].real(), (float)w[j].imag());
        for (int k = 0; k < m; ++k)
            host[(size_t)n + k] = make_float2((float)(c[k].real() / m), (float)(c[k].imag() / m));
        float2* d = nullptr;
        if (hipMalloc(&d, sizeof(float2) * host.size()) != hipSuccess)
            return fail(h, BM_E_NOMEM, "Bluestein tables of %d", n);
        if (hipMemcpy(d, host.data(), sizeof(float2) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return fail(h, BM_E_DEVICE, "Bluestein table upload failed");
        }
        it = h->bluestein.emplace(n, d).first;
    }
    *chirp = it->second;
    *kern = it->second + n;
    return BM_OK;
}

// Plan, twiddles and (when n is not 13-smooth) Bluestein tables of a line length.
bm_status make_fft_job(bosmusic_s* h, int n, bm::FftJob& fj) {
    fj.n = n;
    fj.chirp = fj.kern = nullptr;
    fj.pow2 = bm::fft_pow2_r0(n);
    if (fj.pow2) {
        fj.plan.n = n;
        fj.plan.passes = 3;
        fj.plan.radix[0] = fj.pow2;
        fj.plan.radix[1] = fj.plan.radix[2] = 16;
        return get_twiddles(h, n, &fj.tw, fj.pow2);
    }
    if (plan_fft(n, fj.plan)) return get_twiddles(h, n, &fj.tw);
    const int m = bluestein_len(n);
    if (m == 0 || !plan_fft(m, fj.plan)) return fail(h, BM_E_UNSUPPORTED, "line length %d", n);
    bm_status st = get_twiddles(h, m, &fj.tw);
    if (st != BM_OK) return st;
    return get_bluestein(h, n, m, &fj.chirp, &fj.kern);
}

bm_status validate_frame(bosmusic_s* h, const bosmusic_frame& f, int idx) {
    if (!f.data) return fail(h, BM_E_INVALID_ARG, "frame %d: data is NULL", idx);
    if (f.dtype < BM_F16 || f.dtype > BM_U8) return fail(h, BM_E_INVALID_ARG, "frame %d: dtype %d", idx, f.dtype);
    if (f.width < 1 || f.height < 1 || f.width > h->max_w || f.height > h->max_h)
        return fail(h, BM_E_INVALID_ARG, "frame %d: size %dx%d outside 1..%dx%d", idx, f.width, f.height, h->max_w,
                    h->max_h);
    if (f.row_stride < f.width) return fail(h, BM_E_INVALID_ARG, "frame %d: row_stride < width", idx);
    if (f.dirs & BM_BLOCK) {
        if (!bm::block_size_supported(f.L))
            return fail(h, BM_E_INVALID_ARG, "frame %d: block window %d x %d: 2..8, or odd up to %d", idx, f.L, f.L,
                        bm::kMaxBlockL);
        if (f.L > bm::kMaxL && f.width < f.L)
            return fail(h, BM_E_INVALID_ARG, "frame %d: block window wider than the frame", idx);
    } else if (f.L < 2 || f.L > bm::kMaxL) {
        return fail(h, BM_E_INVALID_ARG, "frame %d: L=%d outside 2..8", idx, f.L);
    }
    if (f.N < f.L || f.N > bm::kMaxN) return fail(h, BM_E_INVALID_ARG, "frame %d: N=%d outside L..64", idx, f.N);
    if ((f.dirs & 3u) == 0 || (f.dirs & ~(3u | BM_BLOCK)))
        return fail(h, BM_E_INVALID_ARG, "frame %d: dirs=%u", idx, f.dirs);
    if ((f.dirs & BM_BLOCK) && f.N != f.L)
        return fail(h, BM_E_INVALID_ARG, "frame %d: block windows need N == L (got L=%d, N=%d)", idx, f.L, f.N);
    if (f.phase && ((f.dirs & (BM_BLOCK | 3u)) != (BM_BLOCK | 3u)))
        return fail(h, BM_E_INVALID_ARG, "frame %d: phase needs BM_BLOCK with both directions", idx);
    if ((f.prev_omega_x || f.prev_omega_y) && (f.dirs & BM_BLOCK))
        return fail(h, BM_E_UNSUPPORTED, "frame %d: the temporal warm start is for line windows", idx);
    if ((f.dirs & BM_DIR_X) && !f.omega_x) return fail(h, BM_E_INVALID_ARG, "frame %d: omega_x is NULL", idx);
    if ((f.dirs & BM_DIR_Y) && !f.omega_y) return fail(h, BM_E_INVALID_ARG, "frame %d: omega_y is NULL", idx);
    if (f.dtype != BM_C32) {
        // block windows use the row-wise analytic signal for both directions
        if (((f.dirs & BM_DIR_X) || (f.dirs & BM_BLOCK)) && !dft_supported(f.width))
            return fail(h, BM_E_UNSUPPORTED, "frame %d: width %d is neither 13-smooth and <= %d nor <= %d", idx,
                        f.width, bm::kMaxFFT, bm::kMaxFFT / 2);
        if ((f.dirs & BM_DIR_Y) && !(f.dirs & BM_BLOCK) && !dft_supported(f.height))
            return fail(h, BM_E_UNSUPPORTED, "frame %d: height %d is neither 13-smooth and <= %d nor <= %d", idx,
                        f.height, bm::kMaxFFT, bm::kMaxFFT / 2);
    }
    return BM_OK;
}

size_t frame_ws_bytes(const bosmusic_frame& f) {
    const size_t px = (size_t)f.width * (size_t)f.height;
    if (f.dirs & BM_BLOCK) return f.dtype != BM_C32 ? align_up(px * sizeof(float2), 256) : 0;
    size_t b = 0;
    if ((f.dirs & BM_DIR_X) && f.dtype != BM_C32) b += align_up(px * sizeof(float2), 256);
    if (f.dirs & BM_DIR_Y) {
        b += align_up(px * sizeof(float2), 256);
        b += align_up(px * sizeof(float), 256);   // transposed real frame, then the omega_y scratch
    }
    return b;
}

// ---------------------------------------------------------------------------
// Batch planning: the job tables of one group of frames, laid out in one blob
// ---------------------------------------------------------------------------
struct RmSet {
    int L = 0;
    bool y_pass = false;            // second launch for y jobs (flags are OR-ed after x)
    bool block_win = false;         // block-window jobs (their own kernel instantiation)
    std::vector<bm::RmJob> jobs;
    std::vector<int> prefix;
    size_t jobs_off = 0, prefix_off = 0;
    bm::RmBatch batch{};
    Tune tune;
};

struct GroupPlan {
    int mode = BM_PLAIN;
    std::vector<bm::TrJob> tr;
    std::vector<int> tr_prefix;
    std::vector<bm::FftJob> fft;
    std::vector<int> fft_prefix;
    int fft_cls_from[bm::kFftClasses + 1] = {};
    int fft_lds[bm::kFftClasses] = {};
    std::vector<RmSet> rm;          // one (or two, with flags) per distinct L
    std::vector<bm::TrJob> back;    // omega_y from its line-major scratch to the caller's row-major map
    std::vector<int> back_prefix;
    size_t tr_off = 0, trp_off = 0, fft_off = 0, fftp_off = 0, back_off = 0, backp_off = 0;
    std::vector<char> blob;
    bm::TrBatch trb{};
    bm::FftBatch fftb{};
    bm::TrBatch backb{};
};

template <typename T>
size_t append(std::vector<char>& blob, const std::vector<T>& v) {
    const size_t off = align_up(blob.size(), 64);
    blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

bm_status plan_group(bosmusic_s* h, const bosmusic_frame* frames, int i0, int i1, int mode, GroupPlan& gp,
                     size_t ws_base = 0) {
    size_t cur = ws_base;   // the group's workspace starts here
    std::map<std::pair<int, int>, RmSet> sets;   // (L, pass + 2 * block) -> set
    bool any_flags = false;
    for (int i = i0; i < i1; ++i) any_flags |= frames[i].flags != nullptr;
    auto add_rm = [&](int L, bool ypass, const bm::RmJob& jb) {
        const bool blk = jb.kind != bm::RM_LINE;
        RmSet& s = sets[{L, (ypass ? 1 : 0) + (blk ? 2 : 0)}];
        s.L = L;
        s.y_pass = ypass;
        s.block_win = blk;
        s.jobs.push_back(jb);
    };
    for (int i = i0; i < i1; ++i) {
        const bosmusic_frame& f = frames[i];
        const bm::Elem e = (bm::Elem)f.dtype;
        const int W = f.width, H = f.height;
        const size_t px = (size_t)W * (size_t)H;
        bm_status st;
        if (f.dirs & BM_BLOCK) {
            // the paper's block window: one row-wise analytic signal serves both directions
            const float2* gam = (const float2*)f.data;
            int64_t gls = f.row_stride;
            if (e != bm::Elem::C32) {
                float2* gx = (float2*)(h->ws + cur);
                cur += align_up(px * sizeof(float2), 256);
                bm::FftJob fj{};
                if ((st = make_fft_job(h, W, fj)) != BM_OK) return st;
                fj.src = f.data;
                fj.src_ls = f.row_stride;
                fj.dst = gx;
                fj.elem = f.dtype;
                fj.nlines = H;
                gp.fft.push_back(fj);
                gam = gx;
                gls = W;
            }
            bm::RmJob j{};
            j.gamma = gam;
            j.gamma_ls = gls;
            j.out = f.omega_x;
            j.out_y = f.omega_y;
            j.phase = f.phase;
            j.bdirs = (int)(f.dirs & 3u);
            j.out_es = 1;
            j.out_ls = W;
            j.flags = f.flags;
            j.flag_es = 1;
            j.flag_ls = W;
            j.len = W;
            j.nlines = H;
            j.N = f.N;
            j.kind = bm::RM_BLOCK;
            add_rm(f.L, false, j);
            continue;
        }
        if (f.dirs & BM_DIR_X) {
            bm::RmJob j{};
            if (e == bm::Elem::C32) {
                j.gamma = (const float2*)f.data;
                j.gamma_ls = f.row_stride;
            } else {
                float2* gx = (float2*)(h->ws + cur);
                cur += align_up(px * sizeof(float2), 256);
                bm::FftJob fj{};
                if ((st = make_fft_job(h, W, fj)) != BM_OK) return st;
                fj.src = f.data;
                fj.src_ls = f.row_stride;
                fj.dst = gx;
                fj.elem = f.dtype;
                fj.nlines = H;
                gp.fft.push_back(fj);
                j.gamma = gx;
                j.gamma_ls = W;
            }
            j.out = f.omega_x;
            j.out_es = 1;
            j.out_ls = W;
            j.prev = f.prev_omega_x;
            j.prev_es = 1;
            j.prev_ls = W;
            j.flags = f.flags;
            j.flag_es = 1;
            j.flag_ls = W;
            j.len = W;
            j.nlines = H;
            j.N = f.N;
            j.flag_shift = 0;
            j.flag_or = 0;
            add_rm(f.L, false, j);
        }
        if (f.dirs & BM_DIR_Y) {
            float2* gy = (float2*)(h->ws + cur);
            cur += align_up(px * sizeof(float2), 256);
            bm::TrJob tj{};
            tj.src = f.data;
            tj.src_ls = f.row_stride;
            tj.rows = H;
            tj.cols = W;
            tj.elem = f.dtype;
            tj.tiles_x = (W + bm::tr_tile(tj) - 1) / bm::tr_tile(tj);
            if (e == bm::Elem::C32) {
                tj.dst = gy;
            } else {
                // (decoded to FP32: an FP16 transposed frame halves the transpose's
                // writes but made the analytic step's reads of it slower, 2.9 -> 3.4 ms on cfg4)
                float* tr = (float*)(h->ws + cur);
                cur += align_up(px * sizeof(float), 256);
                tj.dst = tr;
                bm::FftJob fj{};
                if ((st = make_fft_job(h, H, fj)) != BM_OK) return st;
                fj.src = tr;
                fj.src_ls = H;
                fj.dst = gy;
                fj.elem = BM_F32;
                fj.nlines = W;
                gp.fft.push_back(fj);
            }
            gp.tr.push_back(tj);
            // omega_y is written line-major (coalesced) into a scratch map, then
            // transposed into the caller's map; for real input the scratch is the
            // transposed frame, dead once the analytic step has read it
            float* oy = (e == bm::Elem::C32) ? (float*)(h->ws + cur) : (float*)tj.dst;
            if (e == bm::Elem::C32) cur += align_up(px * sizeof(float), 256);
            bm::TrJob bj{};
            bj.src = oy;
            bj.src_ls = H;
            bj.dst = f.omega_y;
            bj.rows = W;
            bj.cols = H;
            bj.elem = BM_F32;
            bj.tiles_x = (H + bm::tr_tile(bj) - 1) / bm::tr_tile(bj);
            gp.back.push_back(bj);
            bm::RmJob j{};
            j.gamma = gy;
            j.gamma_ls = H;
            j.out = oy;
            j.out_es = 1;
            j.out_ls = H;
            j.prev = f.prev_omega_y;     // the caller's row-major map: along the line (y) W apart
            j.prev_es = W;
            j.prev_ls = 1;
            j.flags = f.flags;
            j.flag_es = W;
            j.flag_ls = 1;
            j.len = H;
            j.nlines = W;
            j.N = f.N;
            j.flag_shift = 4;
            j.flag_or = (f.dirs & BM_DIR_X) ? 1 : 0;
            // with flags, y jobs OR into bytes the x jobs store: run them in a later launch
            add_rm(f.L, any_flags && (f.dirs & BM_DIR_X), j);
        }
    }
    if (cur > h->ws_bytes) return fail(h, BM_E_INVALID_ARG, "group exceeds the workspace");
    gp.tr_prefix.assign(1, 0);
    for (auto& t : gp.tr)
        gp.tr_prefix.push_back(gp.tr_prefix.back() + t.tiles_x * ((t.rows + bm::tr_tile(t) - 1) / bm::tr_tile(t)));
    // jobs ordered by kernel variant (radix range, twiddles in LDS or not): one launch per variant
    std::stable_sort(gp.fft.begin(), gp.fft.end(),
                     [](const bm::FftJob& x, const bm::FftJob& y) { return bm::fft_class(x) < bm::fft_class(y); });
    gp.fft_prefix.assign(1, 0);
    for (int c = 0; c < bm::kFftClasses; ++c) gp.fft_lds[c] = 0;
    int cls = 0;
    gp.fft_cls_from[0] = 0;
    for (auto& f : gp.fft) {
        const int c = bm::fft_class(f);
        while (cls < c) gp.fft_cls_from[++cls] = gp.fft_prefix.back();
        gp.fft_lds[c] = std::max(gp.fft_lds[c], bm::fft_lds_elems(f));
        gp.fft_prefix.push_back(gp.fft_prefix.back() + bm::fft_items(f));
    }
    while (cls < bm::kFftClasses) gp.fft_cls_from[++cls] = gp.fft_prefix.back();
    gp.back_prefix.assign(1, 0);
    for (auto& t : gp.back)
        gp.back_prefix.push_back(gp.back_prefix.back() + t.tiles_x * ((t.rows + bm::tr_tile(t) - 1) / bm::tr_tile(t)));
    for (auto& kv : sets) {
        RmSet s = kv.second;
        int nmax = 0;
        for (auto& j : s.jobs) nmax = std::max(nmax, j.N);
        // the surrogate and block-window kernels run 256 lanes (128 for block windows
        // above 8 x 8), one block per item; plain line windows take the tuned tile
        if (mode == BM_SURROGATE || s.block_win) s.tune = Tune{};
        else s.tune = h->tune[s.L][nmax];
        if (s.block_win) s.tune.block = bm::block_window_lanes(s.L);
        const int wpb = bm::rootmusic_windows_per_block(s.L, s.tune.block, !s.block_win);
        s.prefix.assign(1, 0);
        for (auto& j : s.jobs) {
            j.bpl = (j.len + wpb - 1) / wpb;
            s.prefix.push_back(s.prefix.back() + j.bpl * j.nlines);
        }
        gp.rm.push_back(s);
    }
    gp.mode = mode;
    gp.blob.clear();
    gp.tr_off = append(gp.blob, gp.tr);
    gp.trp_off = append(gp.blob, gp.tr_prefix);
    gp.fft_off = append(gp.blob, gp.fft);
    gp.fftp_off = append(gp.blob, gp.fft_prefix);
    gp.back_off = append(gp.blob, gp.back);
    gp.backp_off = append(gp.blob, gp.back_prefix);
    for (auto& s : gp.rm) {
        s.jobs_off = append(gp.blob, s.jobs);
        s.prefix_off = append(gp.blob, s.prefix);
    }
    return BM_OK;
}

// Point the batch descriptors at a device copy of the blob.
void bind_group(bosmusic_s* h, GroupPlan& gp, const char* dev) {
    gp.trb.jobs = (const bm::TrJob*)(dev + gp.tr_off);
    gp.trb.prefix = (const int*)(dev + gp.trp_off);
    gp.trb.njobs = (int)gp.tr.size();
    gp.trb.total = gp.tr_prefix.back();
    gp.fftb.jobs = (const bm::FftJob*)(dev + gp.fft_off);
    gp.fftb.prefix = (const int*)(dev + gp.fftp_off);
    gp.fftb.njobs = (int)gp.fft.size();
    gp.fftb.total = gp.fft_prefix.back();
    for (int c = 0; c <= bm::kFftClasses; ++c) gp.fftb.cls_from[c] = gp.fft_cls_from[c];
    for (int c = 0; c < bm::kFftClasses; ++c) gp.fftb.lds[c] = gp.fft_lds[c];
    gp.backb.jobs = (const bm::TrJob*)(dev + gp.back_off);
    gp.backb.prefix = (const int*)(dev + gp.backp_off);
    gp.backb.njobs = (int)gp.back.size();
    gp.backb.total = gp.back_prefix.back();
    for (auto& s : gp.rm) {
        s.batch.jobs = (const bm::RmJob*)(dev + s.jobs_off);
        s.batch.prefix = (const int*)(dev + s.prefix_off);
        s.batch.njobs = (int)s.jobs.size();
        s.batch.total = s.prefix.back();
        s.batch.jacobi = (h->options & BM_OPT_JACOBI) ? 1 : 0;
        s.batch.full_roots = (h->options & BM_OPT_FULL_ROOTS) ? 1 : 0;
        s.batch.block_windows = s.block_win ? 1 : 0;
        s.batch.warm = 0;
        for (auto& jb : s.jobs) s.batch.warm |= jb.prev ? 1 : 0;
        s.batch.stats = (h->options & BM_OPT_STATS) ? h->stats : nullptr;
        s.batch.tmpl = h->tmpl[s.L];
    }
}

int grid_for(const bosmusic_s* h, const Tune& t, int total) {
    if (t.grid_per_cu <= 0) return total;
    return std::min(total, t.grid_per_cu * h->cu_count);
}

bm::MlpWeights mlp_weights(const bosmusic_s* h) {
    bm::MlpWeights w;
    w.w1t = h->sur_w;
    w.w2t = h->sur_w + bm::kMlpHidden * bm::kMlpIn;
    w.w3t = h->sur_w + bm::kMlpHidden * bm::kMlpIn + bm::kMlpHidden * bm::kMlpHidden;
    w.b1 = h->sur_master + bm::kMlpIn * bm::kMlpHidden;
    w.b2 = h->sur_master + bm::kMlpIn * bm::kMlpHidden + bm::kMlpHidden + bm::kMlpHidden * bm::kMlpHidden;
    w.b3 = h->sur_master + bm::kMlpParams - bm::kMlpOut;
    return w;
}

// Surrogate pass over a set: every window is finished in the surrogate
// kernel, by the plain eigen-split where the prediction does not serve.
bm_status launch_sur(bosmusic_s* h, const RmSet& s, hipStream_t st) {
    bm::SurBatch sb;
    sb.rm = s.batch;
    sb.w = mlp_weights(h);
    sb.predictor = h->sur_predictor;
    sb.tau = h->sur_tau;
    return check(h, bm::launch_surrogate(s.L, sb, st), "surrogate");
}

// Root-MUSIC launch, bracketed by HIP events on the same stream when timing.
bm_status launch_rm(bosmusic_s* h, const RmSet& s, hipStream_t st, bool timing, int mode) {
    const int grid = grid_for(h, s.tune, s.batch.total);
    if (!timing) {
        if (mode == BM_SURROGATE) return launch_sur(h, s, st);
        return check(h, bm::launch_rootmusic(s.L, s.batch, s.tune.block, grid, st), "rootmusic");
    }
    std::pair<hipEvent_t, hipEvent_t> ev;
    bm_status r;
    if (!h->ev_free.empty()) {
        ev = h->ev_free.back();
        h->ev_free.pop_back();
    } else {
        if ((r = check(h, hipEventCreate(&ev.first), "event"))) return r;
        if ((r = check(h, hipEventCreate(&ev.second), "event"))) {
            (void)hipEventDestroy(ev.first);
            return r;
        }
    }
    h->ev_pending.push_back(ev);
    if ((r = check(h, hipEventRecord(ev.first, st), "event record"))) return r;
    if (mode == BM_SURROGATE) {
        if ((r = launch_sur(h, s, st))) return r;
    } else if ((r = check(h, bm::launch_rootmusic(s.L, s.batch, s.tune.block, grid, st), "rootmusic"))) {
        return r;
    }
    return check(h, hipEventRecord(ev.second, st), "event record");
}

// Transpose and analytic steps of a bound group on `st`.
bm_status launch_front(bosmusic_s* h, const GroupPlan& gp, hipStream_t st) {
    bm_status r;
    if ((r = check(h, bm::launch_transpose(gp.trb, st), "transpose"))) return r;
    return check(h, bm::launch_analytic(gp.fftb, st), "analytic");
}

// omega_y maps from their line-major scratch into the caller's maps.
bm_status launch_back(bosmusic_s* h, const GroupPlan& gp, hipStream_t st) {
    return check(h, bm::launch_transpose(gp.backb, st), "omega_y transpose");
}

bm_status ensure_upload_buffers(bosmusic_s* h, size_t bytes, hipStream_t st) {
    if (bytes <= h->pin_bytes && bytes <= h->djobs_bytes) return BM_OK;
    bm_status r;
    // the old buffers may still be read by enqueued work
    if ((r = check(h, hipStreamSynchronize(st), "sync before growing job buffers"))) return r;
    if (h->pin_pending && (r = check(h, hipEventSynchronize(h->pin_ev), "upload wait"))) return r;
    h->pin_pending = false;
    const size_t nb = align_up(std::max(bytes, (size_t)1 << 16) * 2, 4096);
    (void)hipHostFree(h->pin);
    (void)hipFree(h->djobs);
    h->pin = nullptr;
    h->djobs = nullptr;
    h->pin_bytes = h->djobs_bytes = 0;
    if (hipHostMalloc((void**)&h->pin, nb, hipHostMallocDefault) != hipSuccess) return fail(h, BM_E_NOMEM, "pinned");
    if (hipMalloc(&h->djobs, nb) != hipSuccess) return fail(h, BM_E_NOMEM, "job tables");
    h->pin_bytes = h->djobs_bytes = nb;
    return BM_OK;
}

bm_status run_group_eager(bosmusic_s* h, GroupPlan& gp, hipStream_t st) {
    bm_status r;
    if ((r = ensure_upload_buffers(h, gp.blob.size(), st))) return r;
    if (h->pin_pending && (r = check(h, hipEventSynchronize(h->pin_ev), "upload wait"))) return r;
    std::memcpy(h->pin, gp.blob.data(), gp.blob.size());
    if ((r = check(h, hipMemcpyAsync(h->djobs, h->pin, gp.blob.size(), hipMemcpyHostToDevice, st), "job upload")))
        return r;
    if ((r = check(h, hipEventRecord(h->pin_ev, st), "upload event"))) return r;
    h->pin_pending = true;
    bind_group(h, gp, (const char*)h->djobs);
    if ((r = launch_front(h, gp, st))) return r;
    const bool timing = (h->options & BM_OPT_TIMING) != 0;
    for (auto& s : gp.rm)
        if ((r = launch_rm(h, s, st, timing, gp.mode))) return r;
    return launch_back(h, gp, st);
}

// `to` waits for the work enqueued on `from` so far.
bm_status stream_after(bosmusic_s* h, hipEvent_t ev, hipStream_t from, hipStream_t to) {
    bm_status r;
    if ((r = check(h, hipEventRecord(ev, from), "pipeline event"))) return r;
    return check(h, hipStreamWaitEvent(to, ev, 0), "pipeline wait");
}

// A group in two halves a, b (disjoint frames and workspace) on two streams,
// so that one half's transposes and analytic step, bound by memory latency,
// run beside the other half's root-MUSIC launch, bound by VALU issue.  st runs
// a's front, a's root-MUSIC, a's back; the second stream runs b's front once
// a's front is done, b's root-MUSIC once a's is done (the two root-MUSIC
// launches never share the chip), then b's back; st waits for the second
// stream before this returns, so the caller sees one stream-ordered call.
bm_status run_pair_eager(bosmusic_s* h, GroupPlan& a, GroupPlan& b, hipStream_t st) {
    bm_status r;
    const size_t boff = align_up(a.blob.size(), 256);
    const size_t bytes = boff + b.blob.size();
    if ((r = ensure_upload_buffers(h, bytes, st))) return r;
    if (h->pin_pending && (r = check(h, hipEventSynchronize(h->pin_ev), "upload wait"))) return r;
    std::memcpy(h->pin, a.blob.data(), a.blob.size());
    std::memcpy(h->pin + boff, b.blob.data(), b.blob.size());
    if ((r = check(h, hipMemcpyAsync(h->djobs, h->pin, bytes, hipMemcpyHostToDevice, st), "job upload"))) return r;
    if ((r = check(h, hipEventRecord(h->pin_ev, st), "upload event"))) return r;
    h->pin_pending = true;
    bind_group(h, a, (const char*)h->djobs);
    bind_group(h, b, (const char*)h->djobs + boff);
    hipStream_t s1 = h->cap[1];
    const bool timing = (h->options & BM_OPT_TIMING) != 0;
    if ((r = launch_front(h, a, st)) || (r = stream_after(h, h->pipe_ev[0], st, s1))) return r;
    // from here on the second stream holds work: join it on every return
    if (!(r = launch_front(h, b, s1)))
        for (auto& s : a.rm)
            if ((r = launch_rm(h, s, st, timing, a.mode))) break;
    if (!r && !(r = stream_after(h, h->pipe_ev[1], st, s1))) {
        for (auto& s : b.rm)
            if ((r = launch_rm(h, s, s1, timing, b.mode))) break;
        if (!r) r = launch_back(h, b, s1);
    }
    if (!r) r = launch_back(h, a, st);
    const bm_status j = stream_after(h, h->pipe_ev[2], s1, st);
    return r ? r : j;
}

// Signature of a call: every frame field, mode-relevant options and tuning.
std::string signature(const bosmusic_s* h, const bosmusic_frame* frames, int n, int mode) {
    std::string key;
    key.append((const char*)&mode, sizeof(mode));
    if (mode == BM_SURROGATE) {
        key.append((const char*)&h->sur_tau, sizeof(h->sur_tau));
        key.append((const char*)&h->sur_predictor, sizeof(h->sur_predictor));
    }
    key.append((const char*)frames, (size_t)n * sizeof(bosmusic_frame));
    key.append((const char*)&h->options, sizeof(h->options));
    for (int i = 0; i < n; ++i)
        if (frames[i].L <= bm::kMaxL) key.append((const char*)&h->tune[frames[i].L][frames[i].N], sizeof(Tune));
    return key;
}

void destroy_graph(GraphEntry& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    (void)hipFree(g.blob);
    g = GraphEntry{};
}

bm_status build_graph(bosmusic_s* h, const bosmusic_frame* frames, int n,
                      const std::vector<std::pair<int, int>>& groups, int mode, hipStream_t st, GraphEntry& ge) {
    bm_status r;
    std::vector<GroupPlan> plans(groups.size());
    size_t total = 0;
    std::vector<size_t> offs;
    for (size_t g = 0; g < groups.size(); ++g) {
        if ((r = plan_group(h, frames, groups[g].first, groups[g].second, mode, plans[g]))) return r;
        offs.push_back(align_up(total, 256));
        total = offs.back() + plans[g].blob.size();
    }
    if (hipMalloc(&ge.blob, std::max<size_t>(total, 256)) != hipSuccess) return fail(h, BM_E_NOMEM, "graph tables");
    for (size_t g = 0; g < groups.size(); ++g) {
        if ((r = check(h, hipMemcpy((char*)ge.blob + offs[g], plans[g].blob.data(), plans[g].blob.size(),
                                    hipMemcpyHostToDevice), "graph table upload")))
            return r;
        bind_group(h, plans[g], (const char*)ge.blob + offs[g]);
    }
    hipStream_t c0 = h->cap[0];
    if ((r = check(h, hipStreamBeginCapture(c0, hipStreamCaptureModeThreadLocal), "begin capture"))) return r;
    bm_status lr = BM_OK;
    for (auto& gp : plans) {
        if ((lr = launch_front(h, gp, c0))) break;
        if (gp.rm.size() == 1) {
            if ((lr = launch_rm(h, gp.rm[0], c0, false, mode))) break;
            if ((lr = launch_back(h, gp, c0))) break;
            continue;
        }
        // fork: each distinct L on its own capture stream; a y pass stays on
        // the stream of the x pass of the same L, after it
        if ((lr = check(h, hipEventRecord(h->fork_ev, c0), "fork"))) break;
        // (more distinct sizes than capture streams, possible with block windows,
        // share streams and run one after another on them)
        std::map<int, int> lane_of_L;
        for (auto& s : gp.rm)
            if (!lane_of_L.count(s.L)) {
                const int k = (int)lane_of_L.size() % kMaxForks;
                lane_of_L[s.L] = k;
            }
        for (auto& kv : lane_of_L)
            if (kv.second > 0 && (lr = check(h, hipStreamWaitEvent(h->cap[kv.second], h->fork_ev, 0), "fork wait")))
                break;
        if (lr) break;
        for (auto& s : gp.rm)
            if ((lr = launch_rm(h, s, h->cap[lane_of_L[s.L]], false, mode))) break;
        if (lr) break;
        for (auto& kv : lane_of_L) {
            if (kv.second == 0) continue;
            if ((lr = check(h, hipEventRecord(h->join_ev[kv.second], h->cap[kv.second]), "join"))) break;
            if ((lr = check(h, hipStreamWaitEvent(c0, h->join_ev[kv.second], 0), "join wait"))) break;
        }
        if (lr) break;
        if ((lr = launch_back(h, gp, c0))) break;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c0, &graph);
    if (lr) {
        if (graph) (void)hipGraphDestroy(graph);
        return lr;
    }
    if ((r = check(h, ec, "end capture"))) return r;
    ge.graph = graph;
    if ((r = check(h, hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0), "graph instantiate"))) return r;
    return BM_OK;
}

bm_status run_graph(bosmusic_s* h, const bosmusic_frame* frames, int n,
                    const std::vector<std::pair<int, int>>& groups, int mode, hipStream_t st) {
    const std::string key = signature(h, frames, n, mode);
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        if ((int)h->graphs.size() >= kMaxGraphs) {
            auto victim = h->graphs.begin();
            for (auto g = h->graphs.begin(); g != h->graphs.end(); ++g)
                if (g->second.last_use < victim->second.last_use) victim = g;
            // a replay of the victim may still be running
            if (h->last_graph_stream) (void)hipStreamSynchronize(h->last_graph_stream);
            (void)hipStreamSynchronize(st);
            destroy_graph(victim->second);
            h->graphs.erase(victim);
        }
        GraphEntry ge;
        bm_status r = build_graph(h, frames, n, groups, mode, st, ge);
        if (r != BM_OK) {
            destroy_graph(ge);
            return r;
        }
        it = h->graphs.emplace(key, ge).first;
        log_line(h, "graph captured: %d frames, %zu groups, mode %d (%zu cached)", n, groups.size(), mode,
                 h->graphs.size());
    } else {
        log_line(h, "graph replayed: %d frames, mode %d", n, mode);
    }
    it->second.last_use = ++h->tick;
    h->last_graph_stream = st;
    return check(h, hipGraphLaunch(it->second.exec, st), "graph launch");
}

// ---------------------------------------------------------------------------
// Tune cache: one JSON object per line
//   {"arch":"gfx950","L":6,"N":32,"block":256,"grid_per_cu":0,"us":123.4}
// ---------------------------------------------------------------------------
void load_tune_cache(bosmusic_s* h) {
    if (h->tune_path.empty()) return;
    FILE* fp = std::fopen(h->tune_path.c_str(), "r");
    if (!fp) return;
    char line[512];
    while (std::fgets(line, sizeof(line), fp)) {
        char arch[64] = {0};
        int L = 0, N = 0, block = 0, gpc = 0;
        double us = 0;
        if (std::sscanf(line, " {\"arch\":\"%63[^\"]\",\"L\":%d,\"N\":%d,\"block\":%d,\"grid_per_cu\":%d,\"us\":%lf",
                        arch, &L, &N, &block, &gpc, &us) == 6 &&
            h->arch == arch && L >= 2 && L <= bm::kMaxL && N >= L && N <= bm::kMaxN &&
            (block == 128 || block == 256) && gpc >= 0 && gpc <= 64) {
            h->tune[L][N].block = block;
            h->tune[L][N].grid_per_cu = gpc;
        }
    }
    std::fclose(fp);
}


// bfloat16 of an FP32 value, round to nearest even.
uint16_t to_bf16_bits(float f) {
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Upload FP32 parameters and their bfloat16 copies (W1^T | W2^T | W3^T | W2);
// the device is synchronised first (enqueued work may still read the old ones).
bm_status upload_params(bosmusic_s* h, const float* params) {
    const int64_t n = bm::kMlpParams;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return fail(h, BM_E_INVALID_ARG, "parameter %lld is not finite", (long long)i);
    const int H = bm::kMlpHidden, I = bm::kMlpIn;
    const float* W1 = params;
    const float* W2 = params + I * H + H;
    const float* W3 = W2 + H * H + H;
    std::vector<uint16_t> w((size_t)H * I + 2 * (size_t)H * H + 16 * (size_t)H, 0);
    for (int i = 0; i < I; ++i)
        for (int o = 0; o < H; ++o) w[(size_t)o * I + i] = to_bf16_bits(W1[i * H + o]);
    uint16_t* w2t = w.data() + (size_t)H * I;
    for (int i = 0; i < H; ++i)
        for (int o = 0; o < H; ++o) w2t[(size_t)o * H + i] = to_bf16_bits(W2[i * H + o]);
    uint16_t* w3t = w2t + (size_t)H * H;
    for (int i = 0; i < H; ++i)
        for (int o = 0; o < bm::kMlpOut; ++o) w3t[(size_t)o * H + i] = to_bf16_bits(W3[i * bm::kMlpOut + o]);
    uint16_t* w2 = w3t + 16 * (size_t)H;
    for (int i = 0; i < H * H; ++i) w2[i] = to_bf16_bits(W2[i]);
    bm_status r;
    if ((r = check(h, hipDeviceSynchronize(), "sync")) ||
        (r = check(h, hipMemcpy(h->sur_master, params, n * sizeof(float), hipMemcpyHostToDevice), "load")) ||
        (r = check(h, hipMemcpy(h->sur_w, w.data(), w.size() * 2, hipMemcpyHostToDevice), "load")))
        return r;
    return BM_OK;
}

}  // namespace

extern "C" {

bm_status bosmusic_surrogate_load(bosmusic_t h, const float* params, int64_t n) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (!params || n != bm::kMlpParams) return fail(h, BM_E_INVALID_ARG, "need %d parameters", bm::kMlpParams);
        DeviceGuard dg(h->device);
        bm_status r;
        if ((r = upload_params(h, params)) ||
            (r = check(h, hipMemset(h->adam_m, 0, n * sizeof(float)), "load")) ||
            (r = check(h, hipMemset(h->adam_v, 0, n * sizeof(float)), "load")))
            return r;
        h->adam_t = 0;
        h->sur_loaded = true;
        return BM_OK;
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in surrogate_load");
    }
}

bm_status bosmusic_surrogate_get_state(bosmusic_t h, float* state, int64_t n, int64_t* adam_step) {
    if (!h) return BM_E_INVALID_ARG;
    h->err.clear();
    if (!state || !adam_step || n != 3 * (int64_t)bm::kMlpParams)
        return fail(h, BM_E_INVALID_ARG, "need a state of %d floats and a step pointer", 3 * bm::kMlpParams);
    DeviceGuard dg(h->device);
    const size_t b = bm::kMlpParams * sizeof(float);
    bm_status r;
    if ((r = check(h, hipDeviceSynchronize(), "sync")) ||
        (r = check(h, hipMemcpy(state, h->sur_master, b, hipMemcpyDeviceToHost), "state")) ||
        (r = check(h, hipMemcpy(state + bm::kMlpParams, h->adam_m, b, hipMemcpyDeviceToHost), "state")) ||
        (r = check(h, hipMemcpy(state + 2 * bm::kMlpParams, h->adam_v, b, hipMemcpyDeviceToHost), "state")))
        return r;
    *adam_step = h->adam_t;
    return BM_OK;
}

bm_status bosmusic_surrogate_set_state(bosmusic_t h, const float* state, int64_t n, int64_t adam_step) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (!state || n != 3 * (int64_t)bm::kMlpParams || adam_step < 0)
            return fail(h, BM_E_INVALID_ARG, "need a state of %d floats and a step count >= 0", 3 * bm::kMlpParams);
        for (int64_t i = bm::kMlpParams; i < n; ++i)
            if (!std::isfinite(state[i]) || (i >= 2 * bm::kMlpParams && state[i] < 0.f))
                return fail(h, BM_E_INVALID_ARG, "Adam moment %lld is not valid", (long long)i);
        DeviceGuard dg(h->device);
        const size_t b = bm::kMlpParams * sizeof(float);
        bm_status r;
        if ((r = upload_params(h, state)) ||
            (r = check(h, hipMemcpy(h->adam_m, state + bm::kMlpParams, b, hipMemcpyHostToDevice), "state")) ||
            (r = check(h, hipMemcpy(h->adam_v, state + 2 * bm::kMlpParams, b, hipMemcpyHostToDevice), "state")))
            return r;
        h->adam_t = adam_step;
        h->sur_loaded = true;
        return BM_OK;
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in surrogate_set_state");
    }
}

bm_status bosmusic_surrogate_save(bosmusic_t h, float* params, int64_t n) {
    if (!h) return BM_E_INVALID_ARG;
    if (!params || n != bm::kMlpParams) return fail(h, BM_E_INVALID_ARG, "need %d parameters", bm::kMlpParams);
    DeviceGuard dg(h->device);
    bm_status r;
    if ((r = check(h, hipDeviceSynchronize(), "sync"))) return r;
    return check(h, hipMemcpy(params, h->sur_master, n * sizeof(float), hipMemcpyDeviceToHost), "save");
}

bm_status bosmusic_surrogate_config(bosmusic_t h, float tau, int32_t predictor) {
    if (!h) return BM_E_INVALID_ARG;
    if (!(tau > 0.f && tau <= 1.f) || (predictor != 0 && predictor != 1))
        return fail(h, BM_E_INVALID_ARG, "tau in (0, 1], predictor 0 or 1");
    h->sur_tau = tau;
    h->sur_predictor = predictor;
    return BM_OK;
}

bm_status bosmusic_surrogate_dataset(bosmusic_t h, int64_t first_line, int64_t count, uint64_t seed, float* X,
                                     float* T, float* omega, void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (!X || !T || count < 0 || first_line < 0 || first_line + count > ((int64_t)1 << 32))
            return fail(h, BM_E_INVALID_ARG, "X/T/count/first_line");
        if (count == 0) return BM_OK;
        DeviceGuard dg(h->device);
        hipStream_t st = (hipStream_t)stream;
        bm_status r;
        constexpr int kLen = 128, kLabelL = 8, kLabelN = 32, kPerJob = 65536;
        constexpr int64_t kChunk = (int64_t)1 << 18;
        constexpr int kMaxJobs = (int)(kChunk / kPerJob);
        const int64_t chunk = std::min(count, kChunk);
        size_t off = 0;
        auto carve = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes, 256); return o; };
        const size_t o_lines = carve((size_t)chunk * kLen * sizeof(float));
        const size_t o_gamma = carve((size_t)chunk * kLen * sizeof(float2));
        const size_t o_labels = carve((size_t)chunk * sizeof(float));
        const size_t o_list = carve((size_t)chunk * sizeof(int2));
        const size_t o_count = carve(sizeof(unsigned long long));
        const size_t o_fj = carve(sizeof(bm::FftJob));
        const size_t o_fp = carve(2 * sizeof(int));
        const size_t o_rj = carve(kMaxJobs * sizeof(bm::RmJob));
        const size_t o_rp = carve((kMaxJobs + 1) * sizeof(int));
        if (off > h->ds_bytes) {
            if ((r = check(h, hipStreamSynchronize(st), "sync"))) return r;
            (void)hipFree(h->ds);
            h->ds = nullptr;
            h->ds_bytes = 0;
            if (hipMalloc(&h->ds, off) != hipSuccess) return fail(h, BM_E_NOMEM, "dataset buffers (%zu bytes)", off);
            h->ds_bytes = off;
        }
        bm::FftJob fj{};
        if ((r = make_fft_job(h, kLen, fj))) return r;
        float* lines = (float*)(h->ds + o_lines);
        float2* gamma = (float2*)(h->ds + o_gamma);
        for (int64_t c0 = 0; c0 < count; c0 += chunk) {
            const int n = (int)std::min(chunk, count - c0);
            float* labels = omega ? omega + c0 : (float*)(h->ds + o_labels);
            fj.src = lines;
            fj.src_ls = kLen;
            fj.dst = gamma;
            fj.elem = BM_F32;
            fj.nlines = n;
            const int fprefix[2] = {0, bm::fft_items(fj)};
            std::vector<bm::RmJob> rj;
            std::vector<int> rp(1, 0);
            for (int j = 0; j * kPerJob < n; ++j) {
                bm::RmJob J{};
                J.gamma = gamma + (int64_t)j * kPerJob * kLen;
                J.gamma_ls = kLen;
                J.out = labels + (int64_t)j * kPerJob;
                J.out_es = 0;
                J.out_ls = 1;
                J.len = kLen;
                J.nlines = std::min(kPerJob, n - j * kPerJob);
                J.N = kLabelN;
                J.bpl = 1;
                rj.push_back(J);
                rp.push_back(rp.back() + J.nlines);
            }
            // the tables are read by this chunk's kernels: finish the previous chunk first
            if ((r = check(h, hipStreamSynchronize(st), "sync")) ||
                (r = check(h, hipMemcpy(h->ds + o_fj, &fj, sizeof(fj), hipMemcpyHostToDevice), "tables")) ||
                (r = check(h, hipMemcpy(h->ds + o_fp, fprefix, sizeof(fprefix), hipMemcpyHostToDevice), "tables")) ||
                (r = check(h, hipMemcpy(h->ds + o_rj, rj.data(), rj.size() * sizeof(bm::RmJob), hipMemcpyHostToDevice),
                           "tables")) ||
                (r = check(h, hipMemcpy(h->ds + o_rp, rp.data(), rp.size() * sizeof(int), hipMemcpyHostToDevice),
                           "tables")))
                return r;
            bm::FftBatch fb;
            fb.jobs = (const bm::FftJob*)(h->ds + o_fj);
            fb.prefix = (const int*)(h->ds + o_fp);
            fb.njobs = 1;
            fb.total = fprefix[1];
            for (int c = 0; c <= bm::kFftClasses; ++c) fb.cls_from[c] = c <= bm::fft_class(fj) ? 0 : fb.total;
            for (int c = 0; c < bm::kFftClasses; ++c) fb.lds[c] = bm::fft_lds_elems(fj);
            bm::RmBatch rb{};
            rb.jobs = (const bm::RmJob*)(h->ds + o_rj);
            rb.prefix = (const int*)(h->ds + o_rp);
            rb.njobs = (int)rj.size();
            rb.total = n;
            rb.jacobi = (h->options & BM_OPT_JACOBI) ? 1 : 0;
            rb.full_roots = (h->options & BM_OPT_FULL_ROOTS) ? 1 : 0;
            rb.stats = nullptr;
            rb.tmpl = h->tmpl[kLabelL];
            int2* list = (int2*)(h->ds + o_list);
            unsigned long long* dcount = (unsigned long long*)(h->ds + o_count);
            const int grid = std::max(1, std::min(8 * h->cu_count, (n + bm::kGatherBlock - 1) / bm::kGatherBlock));
            if ((r = check(h, bm::launch_gen_lines(lines, first_line + c0, n, seed, st), "training lines")) ||
                (r = check(h, bm::launch_analytic(fb, st), "analytic")) ||
                (r = check(h, bm::launch_label_entries(list, n, st), "label windows")) ||
                (r = check(h, bm::launch_fill_u64(dcount, 1, (unsigned long long)n, st), "label count")) ||
                (r = check(h, bm::launch_rootmusic_gather(kLabelL, rb, list, dcount, grid, st), "labels")) ||
                (r = check(h, bm::launch_train_features(gamma, n, labels, X + c0 * bm::kMlpIn, T + c0 * bm::kMlpOut,
                                                        st),
                           "features")))
                return r;
        }
        return check(h, hipStreamSynchronize(st), "dataset");
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in surrogate_dataset");
    }
}

namespace {

bm_status ensure_partials(bosmusic_s* h, int blocks, hipStream_t st) {
    if (blocks <= h->part_blocks) return BM_OK;
    bm_status r;
    if ((r = check(h, hipStreamSynchronize(st), "sync"))) return r;
    (void)hipFree(h->part);
    h->part = nullptr;
    h->part_blocks = 0;
    if (hipMalloc(&h->part, (size_t)blocks * bm::mlp_partial_stride() * sizeof(float)) != hipSuccess)
        return fail(h, BM_E_NOMEM, "gradient partials");
    h->part_blocks = blocks;
    return BM_OK;
}

const __bf16* w2_plain(const bosmusic_s* h) {
    return h->sur_w + bm::kMlpHidden * bm::kMlpIn + bm::kMlpHidden * bm::kMlpHidden + 16 * bm::kMlpHidden;
}

// One Adam step from the partials of `blocks` blocks (or from grad when part is null).
bm_status adam_step(bosmusic_s* h, const float* part, int blocks, float* grad, float* loss, float lr, hipStream_t st) {
    ++h->adam_t;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)h->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)h->adam_t)));
    return check(h, bm::launch_mlp_reduce_adam(part, blocks, h->sur_master, h->adam_m, h->adam_v, grad, loss, h->sur_w,
                                               1, lr, c1, c2, st),
                 "adam");
}

}  // namespace

bm_status bosmusic_surrogate_grad(bosmusic_t h, const float* X, const float* T, int32_t M, float* grad, float* loss,
                                  void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    if (!X || !T || !grad || M <= 0 || M % 64) return fail(h, BM_E_INVALID_ARG, "X/T/grad, M a positive multiple of 64");
    DeviceGuard dg(h->device);
    hipStream_t st = (hipStream_t)stream;
    const int blocks = bm::mlp_train_blocks(M);
    bm_status r;
    if ((r = ensure_partials(h, blocks, st)) ||
        (r = check(h, bm::launch_mlp_train(mlp_weights(h), w2_plain(h), X, T, M, h->part, blocks, st), "mlp train")))
        return r;
    return check(h, bm::launch_mlp_reduce_adam(h->part, blocks, nullptr, nullptr, nullptr, grad, loss, nullptr, 0, 0.f,
                                               0.f, 0.f, st),
                 "gradient sum");
}

bm_status bosmusic_surrogate_step(bosmusic_t h, const float* grad, float lr, void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    if (!grad || !(lr > 0.f)) return fail(h, BM_E_INVALID_ARG, "grad/lr");
    DeviceGuard dg(h->device);
    return adam_step(h, nullptr, 0, const_cast<float*>(grad), nullptr, lr, (hipStream_t)stream);
}

bm_status bosmusic_surrogate_train(bosmusic_t h, const float* X, const float* T, int64_t M, int32_t batch,
                                   int32_t steps, float lr, float* losses, void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (!X || !T || batch <= 0 || batch % 64 || M < batch || steps < 0 || !(lr > 0.f))
            return fail(h, BM_E_INVALID_ARG, "X/T, batch a positive multiple of 64 and <= M, steps >= 0, lr > 0");
        DeviceGuard dg(h->device);
        hipStream_t st = (hipStream_t)stream;
        const int blocks = bm::mlp_train_blocks(batch);
        bm_status r;
        if ((r = ensure_partials(h, blocks, st))) return r;
        if (losses && steps > h->losses_cap) {
            if ((r = check(h, hipStreamSynchronize(st), "sync"))) return r;
            (void)hipFree(h->losses);
            h->losses = nullptr;
            h->losses_cap = 0;
            if (hipMalloc(&h->losses, (size_t)steps * sizeof(float)) != hipSuccess)
                return fail(h, BM_E_NOMEM, "loss buffer");
            h->losses_cap = steps;
        }
        const int64_t nb = M / batch;   // whole batches per pass over the data
        for (int s = 0; s < steps; ++s) {
            const int64_t b0 = (int64_t)(s % nb) * batch;
            if ((r = check(h, bm::launch_mlp_train(mlp_weights(h), w2_plain(h), X + b0 * bm::kMlpIn,
                                                   T + b0 * bm::kMlpOut, batch, h->part, blocks, st),
                           "mlp train")) ||
                (r = adam_step(h, h->part, blocks, nullptr, losses ? h->losses + s : nullptr, lr, st)))
                return r;
        }
        if (losses && steps > 0) {
            if ((r = check(h, hipMemcpyAsync(losses, h->losses, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, st),
                           "losses")))
                return r;
            return check(h, hipStreamSynchronize(st), "train");
        }
        return BM_OK;
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in surrogate_train");
    }
}

bm_status bosmusic_surrogate_forward(bosmusic_t h, const float* X, float* Y, int32_t M, void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    if (!X || !Y || M < 0) return fail(h, BM_E_INVALID_ARG, "X/Y/M");
    DeviceGuard dg(h->device);
    return check(h, bm::launch_mlp_forward(mlp_weights(h), X, Y, M, (hipStream_t)stream), "mlp forward");
}

}  // extern "C"

namespace {

void release(bosmusic_s* h) {
    if (!h) return;
    for (auto& kv : h->graphs) destroy_graph(kv.second);
    h->graphs.clear();
    (void)hipFree(h->ws);
    (void)hipFree(h->anchor);
    (void)hipFree(h->stats);
    (void)hipFree(h->djobs);
    (void)hipFree(h->sur_master);
    (void)hipFree(h->sur_w);
    (void)hipFree(h->adam_m);
    (void)hipFree(h->adam_v);
    (void)hipFree(h->part);
    (void)hipFree(h->losses);
    (void)hipFree(h->ds);
    (void)hipFree(h->int_dev);
    (void)hipFree(h->int_anchor);
    if (h->int_pin) (void)hipHostFree(h->int_pin);
    if (h->int_ev) (void)hipEventDestroy(h->int_ev);
    if (h->pin) (void)hipHostFree(h->pin);
    for (auto& kv : h->twiddles) (void)hipFree(kv.second);
    for (auto& kv : h->bluestein) (void)hipFree(kv.second);
    for (auto* v : {&h->ev_free, &h->ev_pending})
        for (auto& e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    for (auto& e : h->pipe_ev)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < kMaxForks; ++i) {
        if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
        if (h->cap[i]) (void)hipStreamDestroy(h->cap[i]);
    }
    delete h;
}

}  // namespace

extern "C" {

int32_t bosmusic_version(void) { return BOSMUSIC_VERSION; }

const char* bosmusic_status_string(bm_status s) {
    switch (s) {
        case BM_OK: return "ok";
        case BM_E_INVALID_ARG: return "invalid argument";
        case BM_E_UNSUPPORTED: return "unsupported";
        case BM_E_NOMEM: return "out of memory";
        case BM_E_DEVICE: return "device error";
        default: return "unknown status";
    }
}

const char* bosmusic_last_error(bosmusic_t h) { return h ? h->err.c_str() : g_create_error; }

bm_status bosmusic_create(const bosmusic_config* cfg, bosmusic_t* out) {
    try {
        if (!out) return fail(nullptr, BM_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!cfg) return fail(nullptr, BM_E_INVALID_ARG, "cfg is NULL");
        if (cfg->max_width < 1 || cfg->max_height < 1 || cfg->max_width > 65536 || cfg->max_height > 65536)
            return fail(nullptr, BM_E_INVALID_ARG, "max size %dx%d", cfg->max_width, cfg->max_height);
        if (cfg->options & ~(uint32_t)(BM_OPT_STATS | BM_OPT_TIMING | BM_OPT_JACOBI | BM_OPT_GRAPH | BM_OPT_FULL_ROOTS))
            return fail(nullptr, BM_E_INVALID_ARG, "options %u", cfg->options);
        if (cfg->max_batch_pixels < 0) return fail(nullptr, BM_E_INVALID_ARG, "max_batch_pixels < 0");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
            return fail(nullptr, BM_E_DEVICE, "no HIP device available");
        if (cfg->device < 0 || cfg->device >= ndev)
            return fail(nullptr, BM_E_INVALID_ARG, "device %d of %d", cfg->device, ndev);
        DeviceGuard dg(cfg->device);
        if (dg.status != hipSuccess) return fail(nullptr, BM_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(dg.status));
        bosmusic_s* h = new (std::nothrow) bosmusic_s();
        if (!h) return fail(nullptr, BM_E_NOMEM, "handle");
        h->device = cfg->device;
        h->max_w = cfg->max_width;
        h->max_h = cfg->max_height;
        h->options = cfg->options;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) {
            release(h);
            return fail(nullptr, BM_E_DEVICE, "device properties");
        }
        h->cu_count = std::max(1, prop.multiProcessorCount);
        h->arch = prop.gcnArchName;
        h->arch = h->arch.substr(0, h->arch.find(':'));
        const int64_t frame_px = (int64_t)cfg->max_width * cfg->max_height;
        const int64_t ws_px = std::max<int64_t>(cfg->max_batch_pixels, frame_px);
        // per pixel: x analytic (8) + y analytic (8) + transposed real (4), plus alignment slack
        h->ws_bytes = (size_t)ws_px * 20 + (size_t)3 * 256 * 1024;
        if (hipMalloc(&h->ws, h->ws_bytes) != hipSuccess || env_is("BOSMUSIC_FAULT", "alloc") ||
            hipMalloc(&h->anchor, (size_t)cfg->max_height * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->stats, bm::kStatFields * bm::kStatSlots * sizeof(unsigned long long)) != hipSuccess) {
            release(h);
            (void)hipGetLastError();
            return fail(nullptr, BM_E_NOMEM, "workspace for %lld pixels", (long long)ws_px);
        }
        bool ok = hipMemset(h->stats, 0, bm::kStatFields * bm::kStatSlots * sizeof(unsigned long long)) == hipSuccess &&
                  bm::analytic_set_attributes() == hipSuccess && bm::integrate_set_attributes() == hipSuccess &&
                  hipEventCreateWithFlags(&h->pin_ev, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&h->int_ev, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; ok && i < 3; ++i)
            ok = hipEventCreateWithFlags(&h->pipe_ev[i], hipEventDisableTiming) == hipSuccess;
        for (int i = 0; ok && i < kMaxForks; ++i)
            ok = hipStreamCreateWithFlags(&h->cap[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            release(h);
            return fail(nullptr, BM_E_DEVICE, "device set-up failed");
        }
        const size_t nw = (size_t)bm::kMlpHidden * bm::kMlpIn + 2 * (size_t)bm::kMlpHidden * bm::kMlpHidden +
                          16 * (size_t)bm::kMlpHidden;
        if (hipMalloc(&h->sur_master, bm::kMlpParams * sizeof(float)) != hipSuccess ||
            hipMalloc(&h->adam_m, bm::kMlpParams * sizeof(float)) != hipSuccess ||
            hipMalloc(&h->adam_v, bm::kMlpParams * sizeof(float)) != hipSuccess ||
            hipMemset(h->adam_m, 0, bm::kMlpParams * sizeof(float)) != hipSuccess ||
            hipMemset(h->adam_v, 0, bm::kMlpParams * sizeof(float)) != hipSuccess ||
            hipMalloc(&h->sur_w, nw * sizeof(__bf16)) != hipSuccess ||
            hipMemset(h->sur_master, 0, bm::kMlpParams * sizeof(float)) != hipSuccess ||
            hipMemset(h->sur_w, 0, nw * sizeof(__bf16)) != hipSuccess) {
            release(h);
            return fail(nullptr, BM_E_NOMEM, "surrogate parameters");
        }
        for (int L = 2; L <= bm::kMaxBlockL; ++L) make_template(L, h->tmpl[L]);
        if (cfg->tune_cache) h->tune_path = cfg->tune_cache;
        load_tune_cache(h);
        h->log = env_is("BOSMUSIC_LOG", "1");
        log_line(h, "create: device %d (%s, %d CUs), frames up to %dx%d, workspace %zu bytes, options 0x%x",
                 cfg->device, h->arch.c_str(), h->cu_count, cfg->max_width, cfg->max_height, h->ws_bytes,
                 cfg->options);
        *out = h;
        return BM_OK;
    } catch (...) {
        return fail(nullptr, BM_E_NOMEM, "host exception in create");
    }
}

bm_status bosmusic_destroy(bosmusic_t h) {
    if (!h) return BM_OK;
    try {
        DeviceGuard dg(h->device);
        (void)hipDeviceSynchronize();
        release(h);
        return BM_OK;
    } catch (...) {
        return BM_E_DEVICE;
    }
}

bm_status bosmusic_demodulate(bosmusic_t h, const bosmusic_frame* frames, int32_t n_frames, int32_t mode,
                              void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (n_frames < 0 || (n_frames > 0 && !frames)) return fail(h, BM_E_INVALID_ARG, "frames/n_frames");
        if (mode != BM_PLAIN && mode != BM_SURROGATE) return fail(h, BM_E_INVALID_ARG, "mode %d", mode);
        if (mode == BM_SURROGATE && !h->sur_loaded && h->sur_predictor == 0)
            return fail(h, BM_E_UNSUPPORTED, "surrogate mode needs loaded parameters");
        for (int i = 0; i < n_frames; ++i) {
            bm_status st = validate_frame(h, frames[i], i);
            if (st != BM_OK) return st;
            if (mode == BM_SURROGATE && frames[i].N < 16)
                return fail(h, BM_E_UNSUPPORTED, "frame %d: surrogate mode needs N >= 16", i);
            if (mode == BM_SURROGATE && (frames[i].dirs & BM_BLOCK))
                return fail(h, BM_E_UNSUPPORTED, "frame %d: surrogate mode needs line windows", i);
        }
        if (n_frames == 0) return BM_OK;
        DeviceGuard dg(h->device);
        if (dg.status != hipSuccess) return check(h, dg.status, "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        // group frames so that each group fits the workspace
        std::vector<std::pair<int, int>> groups;
        size_t used = 0;
        int g0 = 0;
        for (int i = 0; i < n_frames; ++i) {
            const size_t b = frame_ws_bytes(frames[i]) + 3 * 256;
            if (i > g0 && used + b > h->ws_bytes) {
                groups.push_back({g0, i});
                g0 = i;
                used = 0;
            }
            used += b;
        }
        groups.push_back({g0, n_frames});
        const bool graph = (h->options & BM_OPT_GRAPH) && !(h->options & BM_OPT_TIMING);
        if (graph) return run_graph(h, frames, n_frames, groups, mode, s);
        for (auto& g : groups) {
            if (g.second - g.first >= 2 && !(h->options & BM_OPT_TIMING)) {
                // two halves pipelined on two streams (results do not depend on the split);
                // with BM_OPT_TIMING each root-MUSIC launch runs alone, timed by its events
                const int mid = g.first + (g.second - g.first + 1) / 2;
                GroupPlan ga, gb;
                size_t used_a = 0;
                for (int i = g.first; i < mid; ++i) used_a += frame_ws_bytes(frames[i]) + 3 * 256;
                bm_status st = plan_group(h, frames, g.first, mid, mode, ga);
                if (st == BM_OK) st = plan_group(h, frames, mid, g.second, mode, gb, align_up(used_a, 256));
                if (st != BM_OK) return st;
                // a 1024-thread analytic block needs a whole CU's wave slots, so it waits
                // for the root-MUSIC launch to drain (measured slower on the 19-frame
                // 1850 x 700 series): a second half with such lines runs after the first
                bool wide = false;
                for (auto& f : gb.fft) wide |= bm::fft_wide(f);
                if (!wide) {
                    log_line(h, "group frames %d..%d, mode %d: halves %d..%d and %d..%d on two streams", g.first,
                             g.second - 1, mode, g.first, mid - 1, mid, g.second - 1);
                    if ((st = run_pair_eager(h, ga, gb, s)) != BM_OK) return st;
                    continue;
                }
            }
            GroupPlan gp;
            bm_status st = plan_group(h, frames, g.first, g.second, mode, gp);
            if (st == BM_OK && h->log) {
                std::string sets;
                for (auto& rs : gp.rm)
                    sets += " L" + std::to_string(rs.L) + (rs.block_win ? "b" : "") + ":" +
                            std::to_string(rs.prefix.back()) + "x" + std::to_string(rs.tune.block);
                log_line(h, "group frames %d..%d, mode %d: %d analytic items, root-MUSIC sets (items x lanes)%s",
                         g.first, g.second - 1, mode, gp.fft_prefix.back(), sets.c_str());
            }
            if (st == BM_OK) st = run_group_eager(h, gp, s);
            if (st != BM_OK) return st;
        }
        return BM_OK;
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in demodulate");
    }
}

bm_status bosmusic_integrate(bosmusic_t h, const float* omega_x, const float* omega_y, int32_t width,
                             int32_t height, int32_t Nx, int32_t Ny, double carrier_x, double carrier_y, double* phi,
                             void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (!omega_x || !phi) return fail(h, BM_E_INVALID_ARG, "omega_x/phi is NULL");
        if (width < 1 || height < 1 || width > bm::kMaxFFT || height > h->max_h)
            return fail(h, BM_E_INVALID_ARG, "size %dx%d (width <= %d, height <= %d)", width, height, bm::kMaxFFT,
                        h->max_h);
        if (Nx < 1 || Nx > bm::kMaxN || (omega_y && (Ny < 1 || Ny > bm::kMaxN)))
            return fail(h, BM_E_INVALID_ARG, "Nx/Ny");
        if (!std::isfinite(carrier_x) || !std::isfinite(carrier_y)) return fail(h, BM_E_INVALID_ARG, "carrier");
        DeviceGuard dg(h->device);
        if (dg.status != hipSuccess) return check(h, dg.status, "hipSetDevice");
        return check(h, bm::launch_integrate(omega_x, omega_y, width, height, Nx, Ny, carrier_x, carrier_y, h->anchor,
                                             phi, (hipStream_t)stream),
                     "integrate");
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in integrate");
    }
}

}  // extern "C"

namespace {

// Per device: the address of the fixed anchor scratch, looked up once with that
// device current (each device holds its own copy of the array at its own address).
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_anchor[kNoAllocDevices] = {};

}  // namespace

extern "C" {

bm_status bosmusic_integrate_noalloc(const float* omega_x, const float* omega_y, int32_t width, int32_t height,
                                     int32_t Nx, int32_t Ny, double carrier_x, double carrier_y, double* phi,
                                     void* stream) {
    g_create_error[0] = 0;
    if (!omega_x || !phi) return fail(nullptr, BM_E_INVALID_ARG, "omega_x/phi is NULL");
    if (width < 1 || height < 1 || width > bm::kMaxFFT)
        return fail(nullptr, BM_E_INVALID_ARG, "size %dx%d (1 <= width <= %d)", width, height, bm::kMaxFFT);
    if (height > bm::kNoAllocMaxHeight)
        return fail(nullptr, BM_E_INVALID_ARG, "height %d exceeds the fixed scratch of %d rows", height,
                    bm::kNoAllocMaxHeight);
    if (Nx < 1 || Nx > bm::kMaxN || (omega_y && (Ny < 1 || Ny > bm::kMaxN)))
        return fail(nullptr, BM_E_INVALID_ARG, "Nx/Ny");
    if (!std::isfinite(carrier_x) || !std::isfinite(carrier_y)) return fail(nullptr, BM_E_INVALID_ARG, "carrier");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, BM_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoAllocDevices) return fail(nullptr, BM_E_UNSUPPORTED, "device %d", dev);
    double* anchor = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_anchor[dev]) {
            // set-up on the first call on this device (the current one)
            double* p = nullptr;
            if ((e = bm::noalloc_anchor_address(&p)) != hipSuccess || !p)
                return fail(nullptr, BM_E_DEVICE, "hipGetSymbolAddress of the scratch: %s", hipGetErrorString(e));
            if ((e = bm::integrate_set_attributes()) != hipSuccess)
                return fail(nullptr, BM_E_DEVICE, "kernel attributes: %s", hipGetErrorString(e));
            g_noalloc_anchor[dev] = p;
        }
        anchor = g_noalloc_anchor[dev];
    }
    e = bm::launch_integrate(omega_x, omega_y, width, height, Nx, Ny, carrier_x, carrier_y, anchor, phi,
                             (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, BM_E_DEVICE, "integrate: %s", hipGetErrorString(e));
    return BM_OK;
}

bm_status bosmusic_integrate_many(bosmusic_t h, const bosmusic_integrate_job* jobs, int32_t n, void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (n < 0 || (n > 0 && !jobs)) return fail(h, BM_E_INVALID_ARG, "jobs/n");
        std::vector<bm::IntJob> tab((size_t)n);
        std::vector<int> prefix(1, 0);
        int64_t anchors = 0;
        int threads = 1, lds_w = 0;
        for (int i = 0; i < n; ++i) {
            const bosmusic_integrate_job& q = jobs[i];
            if (!q.omega_x || !q.phi) return fail(h, BM_E_INVALID_ARG, "job %d: omega_x/phi is NULL", i);
            if (q.width < 1 || q.height < 1 || q.width > bm::kMaxFFT || q.height > 65536)
                return fail(h, BM_E_INVALID_ARG, "job %d: size %dx%d", i, q.width, q.height);
            if (q.Nx < 1 || q.Nx > bm::kMaxN || (q.omega_y && (q.Ny < 1 || q.Ny > bm::kMaxN)))
                return fail(h, BM_E_INVALID_ARG, "job %d: Nx/Ny", i);
            if (!std::isfinite(q.carrier_x) || !std::isfinite(q.carrier_y))
                return fail(h, BM_E_INVALID_ARG, "job %d: carrier", i);
            if ((int64_t)prefix.back() + q.height > INT32_MAX) return fail(h, BM_E_INVALID_ARG, "too many rows");
            bm::IntJob& J = tab[i];
            J.wx = q.omega_x;
            J.wy = q.omega_y;
            J.phi = q.phi;
            J.cx = q.carrier_x;
            J.cy = q.carrier_y;
            J.W = q.width;
            J.H = q.height;
            J.x0 = q.Nx / 2;
            J.x1 = q.width - q.Nx + q.Nx / 2;
            J.y0 = q.omega_y ? q.Ny / 2 : 0;
            J.y1 = q.omega_y ? q.height - q.Ny + q.Ny / 2 : q.height - 1;
            J.anchor_off = anchors;
            anchors += q.height;
            J.vec = bm::integrate_row_vec(q.width, q.omega_x, q.phi) ? 1 : 0;
            threads = std::max(threads, bm::integrate_row_threads(q.width));
            if (!J.vec) lds_w = std::max(lds_w, q.width);
            prefix.push_back(prefix.back() + q.height);
        }
        if (n == 0) return BM_OK;
        DeviceGuard dg(h->device);
        if (dg.status != hipSuccess) return check(h, dg.status, "hipSetDevice");
        hipStream_t st = (hipStream_t)stream;
        bm_status r;
        const size_t toff = 0, poff = align_up(tab.size() * sizeof(bm::IntJob), 256);
        const size_t bytes = poff + prefix.size() * sizeof(int);
        if (bytes > h->int_bytes || (size_t)anchors > h->int_anchor_cap) {
            // the old buffers may still be read by enqueued work
            if ((r = check(h, hipStreamSynchronize(st), "sync before growing integration buffers"))) return r;
            if (h->int_pending && (r = check(h, hipEventSynchronize(h->int_ev), "upload wait"))) return r;
            h->int_pending = false;
            if (bytes > h->int_bytes) {
                const size_t nb = align_up(std::max<size_t>(bytes, 1 << 14) * 2, 4096);
                (void)hipHostFree(h->int_pin);
                (void)hipFree(h->int_dev);
                h->int_pin = nullptr;
                h->int_dev = nullptr;
                h->int_bytes = 0;
                if (hipHostMalloc((void**)&h->int_pin, nb, hipHostMallocDefault) != hipSuccess ||
                    hipMalloc(&h->int_dev, nb) != hipSuccess)
                    return fail(h, BM_E_NOMEM, "integration job tables");
                h->int_bytes = nb;
            }
            if ((size_t)anchors > h->int_anchor_cap) {
                (void)hipFree(h->int_anchor);
                h->int_anchor = nullptr;
                h->int_anchor_cap = 0;
                if (hipMalloc(&h->int_anchor, (size_t)anchors * 2 * sizeof(double)) != hipSuccess)
                    return fail(h, BM_E_NOMEM, "integration anchors");
                h->int_anchor_cap = (size_t)anchors * 2;
            }
        }
        if (h->int_pending && (r = check(h, hipEventSynchronize(h->int_ev), "upload wait"))) return r;
        std::memcpy(h->int_pin + toff, tab.data(), tab.size() * sizeof(bm::IntJob));
        std::memcpy(h->int_pin + poff, prefix.data(), prefix.size() * sizeof(int));
        if ((r = check(h, hipMemcpyAsync(h->int_dev, h->int_pin, bytes, hipMemcpyHostToDevice, st), "upload")) ||
            (r = check(h, hipEventRecord(h->int_ev, st), "upload event")))
            return r;
        h->int_pending = true;
        const char* dev = (const char*)h->int_dev;
        return check(h, bm::launch_integrate_many((const bm::IntJob*)(dev + toff), (const int*)(dev + poff), n,
                                                  prefix.back(), threads, lds_w, h->int_anchor, st),
                     "integrate_many");
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in integrate_many");
    }
}

bm_status bosmusic_autotune(bosmusic_t h, int32_t L, int32_t N, int32_t width, int32_t lines, double* best_us,
                            void* stream) {
    if (!h) return BM_E_INVALID_ARG;
    try {
        h->err.clear();
        if (L < 2 || L > bm::kMaxL || N < L || N > bm::kMaxN) return fail(h, BM_E_INVALID_ARG, "L/N");
        if (width < N || width > 65536 || lines < 1 || (int64_t)width * lines > ((int64_t)1 << 28))
            return fail(h, BM_E_INVALID_ARG, "width/lines");
        DeviceGuard dg(h->device);
        if (dg.status != hipSuccess) return check(h, dg.status, "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        const int64_t px = (int64_t)width * lines;
        float2* g = nullptr;
        float* o = nullptr;
        void* tab = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto cleanup = [&]() {
            (void)hipStreamSynchronize(s);
            (void)hipFree(g);
            (void)hipFree(o);
            (void)hipFree(tab);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        };
        if (hipMalloc(&g, px * sizeof(float2)) != hipSuccess || hipMalloc(&o, px * sizeof(float)) != hipSuccess ||
            hipMalloc(&tab, 4096) != hipSuccess) {
            cleanup();
            return fail(h, BM_E_NOMEM, "autotune buffers");
        }
        bm_status r = BM_OK;
        if ((r = check(h, hipEventCreate(&e0), "event")) || (r = check(h, hipEventCreate(&e1), "event")) ||
            (r = check(h, bm::launch_synth(g, px, 0.7f, 0.6f, s), "synth")) ||
            (r = check(h, hipStreamSynchronize(s), "sync"))) {
            cleanup();
            return r;
        }
        Tune best;
        double best_t = 1e30;
        const int blocks[2] = {128, 256};
        const int gpcs[6] = {0, 1, 2, 4, 8, 16};
        for (int bi = 0; bi < 2 && r == BM_OK; ++bi) {
            bm::RmJob j{};
            j.gamma = g;
            j.gamma_ls = width;
            j.out = o;
            j.out_es = 1;
            j.out_ls = width;
            j.len = width;
            j.nlines = lines;
            j.N = N;
            const int wpb = bm::rootmusic_windows_per_block(L, blocks[bi], true);
            j.bpl = (width + wpb - 1) / wpb;
            int prefix[2] = {0, j.bpl * lines};
            // the previous candidate's launches read the table: wait before rewriting it
            if ((r = check(h, hipStreamSynchronize(s), "sync")) ||
                (r = check(h, hipMemcpy(tab, &j, sizeof(j), hipMemcpyHostToDevice), "table")) ||
                (r = check(h, hipMemcpy((char*)tab + 1024, prefix, sizeof(prefix), hipMemcpyHostToDevice), "table")))
                break;
            bm::RmBatch b{};
            b.jobs = (const bm::RmJob*)tab;
            b.prefix = (const int*)((char*)tab + 1024);
            b.njobs = 1;
            b.total = prefix[1];
            b.jacobi = (h->options & BM_OPT_JACOBI) ? 1 : 0;
            b.tmpl = h->tmpl[L];
            for (int gi = 0; gi < 6 && r == BM_OK; ++gi) {
                Tune t;
                t.block = blocks[bi];
                t.grid_per_cu = gpcs[gi];
                const int grid = grid_for(h, t, b.total);
                if ((r = check(h, bm::launch_rootmusic(L, b, t.block, grid, s), "warm-up"))) break;
                const int reps = 3;
                if ((r = check(h, hipEventRecord(e0, s), "event"))) break;
                for (int k = 0; k < reps && r == BM_OK; ++k)
                    r = check(h, bm::launch_rootmusic(L, b, t.block, grid, s), "timed launch");
                if (r || (r = check(h, hipEventRecord(e1, s), "event")) ||
                    (r = check(h, hipEventSynchronize(e1), "event sync")))
                    break;
                float ms = 0.f;
                if ((r = check(h, hipEventElapsedTime(&ms, e0, e1), "event time"))) break;
                const double us = 1e3 * ms / reps;
                if (us < best_t) {
                    best_t = us;
                    best = t;
                }
            }
        }
        cleanup();
        if (r != BM_OK) return r;
        h->tune[L][N] = best;
        if (best_us) *best_us = best_t;
        if (!h->tune_path.empty()) {
            FILE* fp = std::fopen(h->tune_path.c_str(), "a");
            if (fp) {
                std::fprintf(fp, "{\"arch\":\"%s\",\"L\":%d,\"N\":%d,\"block\":%d,\"grid_per_cu\":%d,\"us\":%.3f}\n",
                             h->arch.c_str(), L, N, best.block, best.grid_per_cu, best_t);
                std::fclose(fp);
            }
        }
        return BM_OK;
    } catch (...) {
        return fail(h, BM_E_NOMEM, "host exception in autotune");
    }
}

bm_status bosmusic_get_stats(bosmusic_t h, bosmusic_stats* out, int32_t reset, void* stream) {
    if (!h || !out) return BM_E_INVALID_ARG;
    try {
        DeviceGuard dg(h->device);
        hipStream_t s = (hipStream_t)stream;
        unsigned long long slots[bm::kStatFields * bm::kStatSlots];
        unsigned long long v[bm::kStatFields] = {};
        bm_status st;
        if ((st = check(h, hipStreamSynchronize(s), "sync"))) return st;
        if ((st = check(h, hipMemcpy(slots, h->stats, sizeof(slots), hipMemcpyDeviceToHost), "stats copy")))
            return st;
        for (int i = 0; i < bm::kStatFields * bm::kStatSlots; ++i) v[i % bm::kStatFields] += slots[i];
        if (reset && (st = check(h, hipMemset(h->stats, 0, sizeof(slots)), "stats reset"))) return st;
        for (auto& e : h->ev_pending) {
            float ms = 0.f;
            if ((st = check(h, hipEventElapsedTime(&ms, e.first, e.second), "event time"))) return st;
            h->rm_time_ns += (uint64_t)((double)ms * 1e6 + 0.5);
            h->rm_launches += 1;
            h->ev_free.push_back(e);
        }
        h->ev_pending.clear();
        out->windows = v[0];
        out->eig_iters = v[1];
        out->root_iters = v[2];
        out->polish_fail = v[3];
        out->sur_accepted = v[4];
        out->sur_rejected = v[5];
        out->pair_iters = v[6];
        out->pair_iters32 = v[7];
        out->power_windows = v[8];
        out->rm_launches = h->rm_launches;
        out->rm_time_ns = h->rm_time_ns;
        if (reset) h->rm_launches = h->rm_time_ns = 0;
        return BM_OK;
    } catch (...) {
        return BM_E_DEVICE;
    }
}

}  // extern "C"
