// Host runtime behind the bosmusic C ABI: handle, workspace, validation,
// DFT plans and twiddle tables, root templates, and the per-frame dispatch of
// the analytic, transpose, root-MUSIC and integration kernels.
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

struct bosmusic_s {
    int device = 0;
    int max_w = 0, max_h = 0;
    uint32_t options = 0;
    float2* gx = nullptr;       // analytic signal, x lines (max_w * max_h)
    float2* gy = nullptr;       // analytic signal, y lines (transposed)
    float* treal = nullptr;     // transposed real frame
    double* anchor = nullptr;   // integration anchor column (max_h)
    unsigned long long* stats = nullptr;
    std::map<int, float2*> twiddles;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;
    uint64_t rm_launches = 0, rm_time_ns = 0;
    bm::RootTemplate tmpl[bm::kMaxL + 1];
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
    // divide twice by (w - 1): synthetic division, highest power first
    for (int rep = 0; rep < 2; ++rep) {
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

bool factors_235(int n) {
    bm::FftPlan p;
    return plan_fft(n, p);
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

bm_status check(bosmusic_s* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return BM_OK;
    return fail(h, BM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Root-MUSIC launch, bracketed by HIP events on the same stream when timing.
bm_status rootmusic(bosmusic_s* h, int L, const bm::RootMusicArgs& a, hipStream_t s, const char* what) {
    if (!(h->options & BM_OPT_TIMING)) return check(h, bm::launch_rootmusic(L, a, s), what);
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!h->ev_free.empty()) {
        ev = h->ev_free.back();
        h->ev_free.pop_back();
    } else {
        bm_status st;
        if ((st = check(h, hipEventCreate(&ev.first), "event"))) return st;
        if ((st = check(h, hipEventCreate(&ev.second), "event"))) {
            (void)hipEventDestroy(ev.first);
            return st;
        }
    }
    h->ev_pending.push_back(ev);
    bm_status st;
    if ((st = check(h, hipEventRecord(ev.first, s), "event record"))) return st;
    if ((st = check(h, bm::launch_rootmusic(L, a, s), what))) return st;
    return check(h, hipEventRecord(ev.second, s), "event record");
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

bm_status run_frame(bosmusic_s* h, const bosmusic_frame& f, hipStream_t s) {
    const bm::Elem e = (bm::Elem)f.dtype;
    const int W = f.width, H = f.height;
    bm::RootMusicArgs a{};
    a.N = f.N;
    a.flags = f.flags;
    a.stats = (h->options & BM_OPT_STATS) ? h->stats : nullptr;
    a.jacobi = (h->options & BM_OPT_JACOBI) ? 1 : 0;
    a.tmpl = h->tmpl[f.L];
    bm_status st;
    if (f.dirs & BM_DIR_X) {
        const float2* g;
        int64_t gls;
        if (e == bm::Elem::C32) {
            g = (const float2*)f.data;
            gls = f.row_stride;
        } else {
            bm::FftPlan plan;
            plan_fft(W, plan);
            const float2* tw;
            if ((st = get_twiddles(h, W, &tw)) != BM_OK) return st;
            if ((st = check(h, bm::launch_analytic(e, f.data, f.row_stride, H, plan, tw, h->gx, s), "analytic x")))
                return st;
            g = h->gx;
            gls = W;
        }
        a.gamma = g;
        a.gamma_ls = gls;
        a.len = W;
        a.nlines = H;
        a.out = f.omega_x;
        a.out_es = 1;
        a.out_ls = W;
        a.flag_shift = 0;
        a.flag_or = 0;
        if ((st = rootmusic(h, f.L, a, s, "rootmusic x"))) return st;
    }
    if (f.dirs & BM_DIR_Y) {
        if (e == bm::Elem::C32) {
            if ((st = check(h, bm::launch_transpose(e, f.data, f.row_stride, H, W, h->gy, s), "transpose y")))
                return st;
        } else {
            bm::FftPlan plan;
            plan_fft(H, plan);
            const float2* tw;
            if ((st = get_twiddles(h, H, &tw)) != BM_OK) return st;
            if ((st = check(h, bm::launch_transpose(e, f.data, f.row_stride, H, W, h->treal, s), "transpose y")))
                return st;
            if ((st = check(h, bm::launch_analytic(bm::Elem::F32, h->treal, H, W, plan, tw, h->gy, s),
                            "analytic y")))
                return st;
        }
        a.gamma = h->gy;
        a.gamma_ls = H;
        a.len = H;
        a.nlines = W;
        a.out = f.omega_y;
        a.out_es = W;
        a.out_ls = 1;
        a.flag_shift = 4;
        a.flag_or = (f.dirs & BM_DIR_X) ? 1 : 0;
        if ((st = rootmusic(h, f.L, a, s, "rootmusic y"))) return st;
    }
    return BM_OK;
}

void release(bosmusic_s* h) {
    if (!h) return;
    (void)hipFree(h->gx);
    (void)hipFree(h->gy);
    (void)hipFree(h->treal);
    (void)hipFree(h->anchor);
    (void)hipFree(h->stats);
    for (auto& kv : h->twiddles) (void)hipFree(kv.second);
    for (auto* v : {&h->ev_free, &h->ev_pending})
        for (auto& e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
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
        if (cfg->options & ~(uint32_t)(BM_OPT_STATS | BM_OPT_TIMING | BM_OPT_JACOBI)) return fail(nullptr, BM_E_INVALID_ARG, "options %u", cfg->options);
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
        const size_t px = (size_t)cfg->max_width * (size_t)cfg->max_height;
        if (hipMalloc(&h->gx, px * sizeof(float2)) != hipSuccess || hipMalloc(&h->gy, px * sizeof(float2)) != hipSuccess ||
            hipMalloc(&h->treal, px * sizeof(float)) != hipSuccess ||
            hipMalloc(&h->anchor, (size_t)cfg->max_height * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->stats, 4 * bm::kStatSlots * sizeof(unsigned long long)) != hipSuccess) {
            release(h);
            (void)hipGetLastError();
            return fail(nullptr, BM_E_NOMEM, "workspace for %dx%d", cfg->max_width, cfg->max_height);
        }
        if (hipMemset(h->stats, 0, 4 * bm::kStatSlots * sizeof(unsigned long long)) != hipSuccess ||
            bm::analytic_set_attributes() != hipSuccess || bm::integrate_set_attributes() != hipSuccess) {
            release(h);
            return fail(nullptr, BM_E_DEVICE, "device set-up failed");
        }
        for (int L = 2; L <= bm::kMaxL; ++L) make_template(L, h->tmpl[L]);
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
        DeviceGuard dg(h->device);
        if (dg.status != hipSuccess) return check(h, dg.status, "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        for (int i = 0; i < n_frames; ++i) {
            bm_status st = run_frame(h, frames[i], s);
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
