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
#include <cstring>
#include <map>
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
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;
    uint64_t rm_launches = 0, rm_time_ns = 0;
    bm::RootTemplate tmpl[bm::kMaxL + 1];
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
    hipStream_t last_graph_stream = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_create_error;

bm_status fail(bosmusic_s* h, bm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_create_error = buf;
    return st;
}

bm_status check(bosmusic_s* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return BM_OK;
    return fail(h, BM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
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
    const int order[4] = {4, 2, 3, 5};
    for (int f : order) {
        while (r % f == 0) {
            if (p.passes >= bm::kMaxRadixPasses) return false;
            p.radix[p.passes++] = f;
            r /= f;
        }
    }
    return r == 1;
}

bool factors_235(int n) {
    bm::FftPlan p;
    return plan_fft(n, p);
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
    for (int i = n; i < 2 * bm::kMaxL - 2; ++i) t.re[i] = t.im[i] = 0.f;
}

bm_status get_twiddles(bosmusic_s* h, int n, const float2** out) {
    auto it = h->twiddles.find(n);
    if (it != h->twiddles.end()) {
        *out = it->second;
        return BM_OK;
    }
    std::vector<float2> tw(n);
    for (int m = 0; m < n; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)n;
        tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    float2* d = nullptr;
    if (hipMalloc(&d, sizeof(float2) * n) != hipSuccess) return fail(h, BM_E_NOMEM, "twiddle table of %d", n);
    if (hipMemcpy(d, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return fail(h, BM_E_DEVICE, "twiddle upload failed");
    }
    h->twiddles[n] = d;
    *out = d;
    return BM_OK;
}

bm_status validate_frame(bosmusic_s* h, const bosmusic_frame& f, int idx) {
    if (!f.data) return fail(h, BM_E_INVALID_ARG, "frame %d: data is NULL", idx);
    if (f.dtype < BM_F16 || f.dtype > BM_C32) return fail(h, BM_E_INVALID_ARG, "frame %d: dtype %d", idx, f.dtype);
    if (f.width < 1 || f.height < 1 || f.width > h->max_w || f.height > h->max_h)
        return fail(h, BM_E_INVALID_ARG, "frame %d: size %dx%d outside 1..%dx%d", idx, f.width, f.height, h->max_w,
                    h->max_h);
    if (f.row_stride < f.width) return fail(h, BM_E_INVALID_ARG, "frame %d: row_stride < width", idx);
    if (f.L < 2 || f.L > bm::kMaxL) return fail(h, BM_E_INVALID_ARG, "frame %d: L=%d outside 2..8", idx, f.L);
    if (f.N < f.L || f.N > bm::kMaxN) return fail(h, BM_E_INVALID_ARG, "frame %d: N=%d outside L..64", idx, f.N);
    if (f.dirs == 0 || (f.dirs & ~3u)) return fail(h, BM_E_INVALID_ARG, "frame %d: dirs=%u", idx, f.dirs);
    if ((f.dirs & BM_DIR_X) && !f.omega_x) return fail(h, BM_E_INVALID_ARG, "frame %d: omega_x is NULL", idx);
    if ((f.dirs & BM_DIR_Y) && !f.omega_y) return fail(h, BM_E_INVALID_ARG, "frame %d: omega_y is NULL", idx);
    if (f.dtype != BM_C32) {
        if ((f.dirs & BM_DIR_X) && !factors_235(f.width))
            return fail(h, BM_E_UNSUPPORTED, "frame %d: width %d is not 2^a 3^b 5^c <= %d", idx, f.width,
                        bm::kMaxFFT);
        if ((f.dirs & BM_DIR_Y) && !factors_235(f.height))
            return fail(h, BM_E_UNSUPPORTED, "frame %d: height %d is not 2^a 3^b 5^c <= %d", idx, f.height,
                        bm::kMaxFFT);
    }
    return BM_OK;
}

size_t frame_ws_bytes(const bosmusic_frame& f) {
    const size_t px = (size_t)f.width * (size_t)f.height;
    size_t b = 0;
    if ((f.dirs & BM_DIR_X) && f.dtype != BM_C32) b += align_up(px * sizeof(float2), 256);
    if (f.dirs & BM_DIR_Y) {
        b += align_up(px * sizeof(float2), 256);
        if (f.dtype != BM_C32) b += align_up(px * sizeof(float), 256);
    }
    return b;
}

// ---------------------------------------------------------------------------
// Batch planning: the job tables of one group of frames, laid out in one blob
// ---------------------------------------------------------------------------
struct RmSet {
    int L = 0;
    bool y_pass = false;            // second launch for y jobs (flags are OR-ed after x)
    std::vector<bm::RmJob> jobs;
    std::vector<int> prefix;
    size_t jobs_off = 0, prefix_off = 0;
    bm::RmBatch batch{};
    Tune tune;
};

struct GroupPlan {
    std::vector<bm::TrJob> tr;
    std::vector<int> tr_prefix;
    std::vector<bm::FftJob> fft;
    std::vector<int> fft_prefix;
    int max_n = 0;
    std::vector<RmSet> rm;          // one (or two, with flags) per distinct L
    size_t tr_off = 0, trp_off = 0, fft_off = 0, fftp_off = 0;
    std::vector<char> blob;
    bm::TrBatch trb{};
    bm::FftBatch fftb{};
};

template <typename T>
size_t append(std::vector<char>& blob, const std::vector<T>& v) {
    const size_t off = align_up(blob.size(), 64);
    blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

bm_status plan_group(bosmusic_s* h, const bosmusic_frame* frames, int i0, int i1, GroupPlan& gp) {
    size_t cur = 0;
    std::map<std::pair<int, int>, RmSet> sets;   // (L, pass) -> set
    bool any_flags = false;
    for (int i = i0; i < i1; ++i) any_flags |= frames[i].flags != nullptr;
    auto add_rm = [&](int L, bool ypass, const bm::RmJob& jb) {
        RmSet& s = sets[{L, ypass ? 1 : 0}];
        s.L = L;
        s.y_pass = ypass;
        s.jobs.push_back(jb);
    };
    for (int i = i0; i < i1; ++i) {
        const bosmusic_frame& f = frames[i];
        const bm::Elem e = (bm::Elem)f.dtype;
        const int W = f.width, H = f.height;
        const size_t px = (size_t)W * (size_t)H;
        bm_status st;
        if (f.dirs & BM_DIR_X) {
            bm::RmJob j{};
            if (e == bm::Elem::C32) {
                j.gamma = (const float2*)f.data;
                j.gamma_ls = f.row_stride;
            } else {
                float2* gx = (float2*)(h->ws + cur);
                cur += align_up(px * sizeof(float2), 256);
                bm::FftJob fj{};
                if (!plan_fft(W, fj.plan)) return fail(h, BM_E_UNSUPPORTED, "width %d", W);
                if ((st = get_twiddles(h, W, &fj.tw)) != BM_OK) return st;
                fj.src = f.data;
                fj.src_ls = f.row_stride;
                fj.dst = gx;
                fj.elem = f.dtype;
                fj.nlines = H;
                gp.fft.push_back(fj);
                gp.max_n = std::max(gp.max_n, W);
                j.gamma = gx;
                j.gamma_ls = W;
            }
            j.out = f.omega_x;
            j.out_es = 1;
            j.out_ls = W;
            j.flags = f.flags;
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
            tj.tiles_x = (W + 31) / 32;
            tj.elem = f.dtype;
            if (e == bm::Elem::C32) {
                tj.dst = gy;
            } else {
                float* tr = (float*)(h->ws + cur);
                cur += align_up(px * sizeof(float), 256);
                tj.dst = tr;
                bm::FftJob fj{};
                if (!plan_fft(H, fj.plan)) return fail(h, BM_E_UNSUPPORTED, "height %d", H);
                if ((st = get_twiddles(h, H, &fj.tw)) != BM_OK) return st;
                fj.src = tr;
                fj.src_ls = H;
                fj.dst = gy;
                fj.elem = BM_F32;
                fj.nlines = W;
                gp.fft.push_back(fj);
                gp.max_n = std::max(gp.max_n, H);
            }
            gp.tr.push_back(tj);
            bm::RmJob j{};
            j.gamma = gy;
            j.gamma_ls = H;
            j.out = f.omega_y;
            j.out_es = W;
            j.out_ls = 1;
            j.flags = f.flags;
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
    for (auto& t : gp.tr) gp.tr_prefix.push_back(gp.tr_prefix.back() + t.tiles_x * ((t.rows + 31) / 32));
    gp.fft_prefix.assign(1, 0);
    for (auto& f : gp.fft) gp.fft_prefix.push_back(gp.fft_prefix.back() + f.nlines);
    for (auto& kv : sets) {
        RmSet s = kv.second;
        int nmax = 0;
        for (auto& j : s.jobs) nmax = std::max(nmax, j.N);
        s.tune = h->tune[s.L][nmax];
        const int wpb = bm::rootmusic_windows_per_block(s.L, s.tune.block);
        s.prefix.assign(1, 0);
        for (auto& j : s.jobs) {
            j.bpl = (j.len + wpb - 1) / wpb;
            s.prefix.push_back(s.prefix.back() + j.bpl * j.nlines);
        }
        gp.rm.push_back(s);
    }
    gp.blob.clear();
    gp.tr_off = append(gp.blob, gp.tr);
    gp.trp_off = append(gp.blob, gp.tr_prefix);
    gp.fft_off = append(gp.blob, gp.fft);
    gp.fftp_off = append(gp.blob, gp.fft_prefix);
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
    gp.fftb.max_n = gp.max_n;
    for (auto& s : gp.rm) {
        s.batch.jobs = (const bm::RmJob*)(dev + s.jobs_off);
        s.batch.prefix = (const int*)(dev + s.prefix_off);
        s.batch.njobs = (int)s.jobs.size();
        s.batch.total = s.prefix.back();
        s.batch.jacobi = (h->options & BM_OPT_JACOBI) ? 1 : 0;
        s.batch.stats = (h->options & BM_OPT_STATS) ? h->stats : nullptr;
        s.batch.tmpl = h->tmpl[s.L];
    }
}

int grid_for(const bosmusic_s* h, const Tune& t, int total) {
    if (t.grid_per_cu <= 0) return total;
    return std::min(total, t.grid_per_cu * h->cu_count);
}

// Root-MUSIC launch, bracketed by HIP events on the same stream when timing.
bm_status launch_rm(bosmusic_s* h, const RmSet& s, hipStream_t st, bool timing) {
    const int grid = grid_for(h, s.tune, s.batch.total);
    if (!timing) return check(h, bm::launch_rootmusic(s.L, s.batch, s.tune.block, grid, st), "rootmusic");
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
    if ((r = check(h, bm::launch_rootmusic(s.L, s.batch, s.tune.block, grid, st), "rootmusic"))) return r;
    return check(h, hipEventRecord(ev.second, st), "event record");
}

// Transpose and analytic steps of a bound group on `st`.
bm_status launch_front(bosmusic_s* h, const GroupPlan& gp, hipStream_t st) {
    bm_status r;
    if ((r = check(h, bm::launch_transpose(gp.trb, st), "transpose"))) return r;
    return check(h, bm::launch_analytic(gp.fftb, st), "analytic");
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
        if ((r = launch_rm(h, s, st, timing))) return r;
    return BM_OK;
}

// Signature of a call: every frame field, mode-relevant options and tuning.
std::string signature(const bosmusic_s* h, const bosmusic_frame* frames, int n) {
    std::string key;
    key.append((const char*)frames, (size_t)n * sizeof(bosmusic_frame));
    key.append((const char*)&h->options, sizeof(h->options));
    for (int i = 0; i < n; ++i) key.append((const char*)&h->tune[frames[i].L][frames[i].N], sizeof(Tune));
    return key;
}

void destroy_graph(GraphEntry& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    (void)hipFree(g.blob);
    g = GraphEntry{};
}

bm_status build_graph(bosmusic_s* h, const bosmusic_frame* frames, int n,
                      const std::vector<std::pair<int, int>>& groups, GraphEntry& ge) {
    bm_status r;
    std::vector<GroupPlan> plans(groups.size());
    size_t total = 0;
    std::vector<size_t> offs;
    for (size_t g = 0; g < groups.size(); ++g) {
        if ((r = plan_group(h, frames, groups[g].first, groups[g].second, plans[g]))) return r;
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
            if ((lr = launch_rm(h, gp.rm[0], c0, false))) break;
            continue;
        }
        // fork: each distinct L on its own capture stream; a y pass stays on
        // the stream of the x pass of the same L, after it
        if ((lr = check(h, hipEventRecord(h->fork_ev, c0), "fork"))) break;
        std::map<int, int> lane_of_L;
        for (auto& s : gp.rm)
            if (!lane_of_L.count(s.L)) {
                const int k = (int)lane_of_L.size();
                lane_of_L[s.L] = k;
            }
        for (auto& kv : lane_of_L)
            if (kv.second > 0 && (lr = check(h, hipStreamWaitEvent(h->cap[kv.second], h->fork_ev, 0), "fork wait")))
                break;
        if (lr) break;
        for (auto& s : gp.rm)
            if ((lr = launch_rm(h, s, h->cap[lane_of_L[s.L]], false))) break;
        if (lr) break;
        for (auto& kv : lane_of_L) {
            if (kv.second == 0) continue;
            if ((lr = check(h, hipEventRecord(h->join_ev[kv.second], h->cap[kv.second]), "join"))) break;
            if ((lr = check(h, hipStreamWaitEvent(c0, h->join_ev[kv.second], 0), "join wait"))) break;
        }
        if (lr) break;
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
                    const std::vector<std::pair<int, int>>& groups, hipStream_t st) {
    const std::string key = signature(h, frames, n);
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
        bm_status r = build_graph(h, frames, n, groups, ge);
        if (r != BM_OK) {
            destroy_graph(ge);
            return r;
        }
        it = h->graphs.emplace(key, ge).first;
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

void release(bosmusic_s* h) {
    if (!h) return;
    for (auto& kv : h->graphs) destroy_graph(kv.second);
    h->graphs.clear();
    (void)hipFree(h->ws);
    (void)hipFree(h->anchor);
    (void)hipFree(h->stats);
    (void)hipFree(h->djobs);
    if (h->pin) (void)hipHostFree(h->pin);
    for (auto& kv : h->twiddles) (void)hipFree(kv.second);
    for (auto* v : {&h->ev_free, &h->ev_pending})
        for (auto& e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
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

const char* bosmusic_last_error(bosmusic_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

bm_status bosmusic_create(const bosmusic_config* cfg, bosmusic_t* out) {
    try {
        if (!out) return fail(nullptr, BM_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!cfg) return fail(nullptr, BM_E_INVALID_ARG, "cfg is NULL");
        if (cfg->max_width < 1 || cfg->max_height < 1 || cfg->max_width > 65536 || cfg->max_height > 65536)
            return fail(nullptr, BM_E_INVALID_ARG, "max size %dx%d", cfg->max_width, cfg->max_height);
        if (cfg->options & ~(uint32_t)(BM_OPT_STATS | BM_OPT_TIMING | BM_OPT_JACOBI | BM_OPT_GRAPH))
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
        if (hipMalloc(&h->ws, h->ws_bytes) != hipSuccess ||
            hipMalloc(&h->anchor, (size_t)cfg->max_height * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->stats, 4 * bm::kStatSlots * sizeof(unsigned long long)) != hipSuccess) {
            release(h);
            (void)hipGetLastError();
            return fail(nullptr, BM_E_NOMEM, "workspace for %lld pixels", (long long)ws_px);
        }
        bool ok = hipMemset(h->stats, 0, 4 * bm::kStatSlots * sizeof(unsigned long long)) == hipSuccess &&
                  bm::analytic_set_attributes() == hipSuccess && bm::integrate_set_attributes() == hipSuccess &&
                  hipEventCreateWithFlags(&h->pin_ev, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; ok && i < kMaxForks; ++i)
            ok = hipStreamCreateWithFlags(&h->cap[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            release(h);
            return fail(nullptr, BM_E_DEVICE, "device set-up failed");
        }
        for (int L = 2; L <= bm::kMaxL; ++L) make_template(L, h->tmpl[L]);
        if (cfg->tune_cache) h->tune_path = cfg->tune_cache;
        load_tune_cache(h);
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
        if (mode == BM_SURROGATE) return fail(h, BM_E_UNSUPPORTED, "surrogate mode is not built");
        if (mode != BM_PLAIN) return fail(h, BM_E_INVALID_ARG, "mode %d", mode);
        for (int i = 0; i < n_frames; ++i) {
            bm_status st = validate_frame(h, frames[i], i);
            if (st != BM_OK) return st;
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
        if (graph) return run_graph(h, frames, n_frames, groups, s);
        for (auto& g : groups) {
            GroupPlan gp;
            bm_status st = plan_group(h, frames, g.first, g.second, gp);
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
            const int wpb = bm::rootmusic_windows_per_block(L, blocks[bi]);
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
        unsigned long long slots[4 * bm::kStatSlots];
        unsigned long long v[4] = {0, 0, 0, 0};
        bm_status st;
        if ((st = check(h, hipStreamSynchronize(s), "sync"))) return st;
        if ((st = check(h, hipMemcpy(slots, h->stats, sizeof(slots), hipMemcpyDeviceToHost), "stats copy")))
            return st;
        for (int i = 0; i < 4 * bm::kStatSlots; ++i) v[i % 4] += slots[i];
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
        out->rm_launches = h->rm_launches;
        out->rm_time_ns = h->rm_time_ns;
        if (reset) h->rm_launches = h->rm_time_ns = 0;
        return BM_OK;
    } catch (...) {
        return BM_E_DEVICE;
    }
}

}  // extern "C"
