// C ABI of libkaze: argument validation, the level schedule (Eqs. 6-7),
// workspace layout and the launch sequence of the scale space (Sec. II-A,
// Sec. III-A), detector response (Eq. 8) and extrema (Sec. II-B).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "kaze.h"
#include "kaze_internal.h"

namespace {

using namespace kaze;

thread_local char g_err[512] = "";

kaze_status fail(kaze_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

// ---------------------------------------------------------------- profiling
const char* const kKernelNames[K_COUNT] = {
    "gauss", "grad",        "hist",        "kselect", "cond", "aos_reduce",
    "aos_iface", "aos_recover", "det", "nms",     "fill", "copy"};

struct Profiler {
    unsigned mask = 0;  // bit i: record launches of kernel i
    std::vector<hipEvent_t> ev;  // pairs: start, stop
    int used = 0;
    static constexpr int kMaxPairs = 65536;
} g_prof;

struct ProfScope {
    int id;
    hipStream_t s;
    bool on;
    ProfScope(int id_, hipStream_t s_) : id(id_), s(s_), on(false) {
        if (!(g_prof.mask & (1u << id)) || g_prof.used >= Profiler::kMaxPairs) return;
        const size_t need = 2 * (size_t)(g_prof.used + 1);
        while (g_prof.ev.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            g_prof.ev.push_back(e);
        }
        on = hipEventRecord(g_prof.ev[2 * g_prof.used], s) == hipSuccess;
    }
    ~ProfScope() {
        if (!on) return;
        if (hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s) == hipSuccess) ++g_prof.used;
    }
};

#define KZ_LAUNCH(id, stream, call)                                                   \
    do {                                                                              \
        hipError_t e_;                                                                \
        {                                                                             \
            ProfScope ps_(id, stream);                                                \
            e_ = (call);                                                              \
        }                                                                             \
        if (e_ != hipSuccess)                                                         \
            return fail(KAZE_ERR_HIP, "%s launch failed: %s", kKernelNames[id],       \
                        hipGetErrorString(e_));                                       \
    } while (0)

// ---------------------------------------------------------------- parameters
int gauss_radius(double sigma) { return (int)ceil(3.0 * sigma); }

Taps gauss_taps(double sigma) {
    Taps t;
    memset(&t, 0, sizeof(t));
    t.r = gauss_radius(sigma);
    double w[2 * kMaxRadius + 1];
    double sum = 0.0;
    for (int j = -t.r; j <= t.r; ++j) {
        w[j + t.r] = exp(-(double)(j * j) / (2.0 * sigma * sigma));
        sum += w[j + t.r];
    }
    for (int j = 0; j <= 2 * t.r; ++j) t.w[j] = (float)(w[j] / sum);
    return t;
}

struct Level {
    double sigma, t, tau, sigma_n;
    int step;
};

kaze_status check_params(const kaze_params* p) {
    if (!p) return fail(KAZE_ERR_INVALID_ARG, "params pointer is NULL");
    if (p->octaves < 1 || p->sublevels < 1)
        return fail(KAZE_ERR_INVALID_ARG, "octaves and sublevels must be >= 1");
    if ((long long)p->octaves * p->sublevels > kMaxLevels)
        return fail(KAZE_ERR_UNSUPPORTED, "at most %d levels", kMaxLevels);
    if (!(p->sigma0 > 0.0) || !(p->sigma_cond > 0.0))
        return fail(KAZE_ERR_INVALID_ARG, "sigma0 and sigma_cond must be > 0");
    if (gauss_radius(p->sigma0) > kMaxRadius)
        return fail(KAZE_ERR_UNSUPPORTED, "sigma0 radius ceil(3 sigma) must be <= %d", kMaxRadius);
    if (gauss_radius(p->sigma_cond) > kMaxCondRadius)
        return fail(KAZE_ERR_UNSUPPORTED, "sigma_cond radius ceil(3 sigma) must be <= %d",
                    kMaxCondRadius);
    if (p->diffusivity != KAZE_G1 && p->diffusivity != KAZE_G2)
        return fail(KAZE_ERR_INVALID_ARG, "diffusivity must be KAZE_G1 or KAZE_G2");
    if (!(p->k_override > 0.0)) {
        if (!(p->k_percentile >= 1e-6 && p->k_percentile <= 1.0))
            return fail(KAZE_ERR_INVALID_ARG, "k_percentile must be in [1e-6, 1]");
        if (p->k_bins < 1 || p->k_bins > 4096)
            return fail(KAZE_ERR_INVALID_ARG, "k_bins must be in [1, 4096]");
    }
    if (!isfinite(p->det_threshold))
        return fail(KAZE_ERR_INVALID_ARG, "det_threshold must be finite");
    return KAZE_OK;
}

void schedule(const kaze_params* p, std::vector<Level>& lv) {
    const int N = p->octaves * p->sublevels;
    lv.resize(N);
    for (int i = 0; i < N; ++i) {
        const int o = i / p->sublevels, s = i % p->sublevels;
        Level& L = lv[i];
        L.sigma = p->sigma0 * pow(2.0, o + (double)s / p->sublevels);
        L.t = 0.5 * L.sigma * L.sigma;
        L.tau = i == 0 ? 0.0 : L.t - lv[i - 1].t;
        L.sigma_n = L.sigma / pow(2.0, o);
        const int st = (int)floor(L.sigma_n + 0.5);
        L.step = st < 1 ? 1 : st;
    }
}

kaze_status check_size(int W, int H) {
    if (W < 8 || H < 8) return fail(KAZE_ERR_INVALID_ARG, "image must be at least 8x8");
    if (W > kTile * kWave || H > kTile * kWave)
        return fail(KAZE_ERR_UNSUPPORTED, "image larger than %dx%d (got %dx%d)", kTile * kWave,
                    kTile * kWave, W, H);
    return KAZE_OK;
}

kaze_status check_steps(const kaze_params* p) {
    std::vector<Level> lv;
    schedule(p, lv);
    for (const Level& L : lv)
        if (L.step > kMaxStep)
            return fail(KAZE_ERR_UNSUPPORTED, "Scharr step %d exceeds %d", L.step, kMaxStep);
    return KAZE_OK;
}

// ---------------------------------------------------------------- workspace
struct Workspace {
    size_t g, rrow, rcol, zrow, zcol, hist, hmax, total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Workspace layout(int W, int H, const kaze_params* p) {
    Workspace w;
    const size_t ncx = (W + kTile - 1) / kTile, ncy = (H + kTile - 1) / kTile;
    const int nbins = p->k_bins > 0 ? p->k_bins : 1;
    size_t off = 0;
    w.g = off;    off = align256(off + (size_t)W * H * sizeof(float));
    w.rrow = off; off = align256(off + (size_t)H * ncx * 8 * sizeof(float));
    w.rcol = off; off = align256(off + (size_t)W * ncy * 8 * sizeof(float));
    w.zrow = off; off = align256(off + (size_t)H * ncx * 2 * sizeof(float));
    w.zcol = off; off = align256(off + (size_t)W * ncy * 2 * sizeof(float));
    w.hist = off; off = align256(off + (size_t)nbins * sizeof(unsigned));
    w.hmax = off; off = align256(off + sizeof(unsigned));
    w.total = off;
    return w;
}

ImageDesc image_desc(int W, int H, void* ws, const Workspace& w) {
    char* base = static_cast<char*>(ws);
    ImageDesc d;
    d.L = nullptr;
    d.Lnext = nullptr;
    d.g = reinterpret_cast<float*>(base + w.g);
    d.rrow = reinterpret_cast<float*>(base + w.rrow);
    d.rcol = reinterpret_cast<float*>(base + w.rcol);
    d.zrow = reinterpret_cast<float*>(base + w.zrow);
    d.zcol = reinterpret_cast<float*>(base + w.zcol);
    d.k = nullptr;
    d.W = W;
    d.H = H;
    d.ncx = (W + kTile - 1) / kTile;
    d.ncy = (H + kTile - 1) / kTile;
    return d;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// exact binary fraction of the percentile: pct = mant * 2^-shift
void percentile_fraction(double pct, unsigned long long* mant, int* shift) {
    int e;
    const double f = frexp(pct, &e);  // pct = f * 2^e, f in [0.5, 1)
    unsigned long long m = (unsigned long long)ldexp(f, 53);
    int sh = 53 - e;
    while (sh > 0 && (m & 1ull) == 0) {
        m >>= 1;
        --sh;
    }
    *mant = m;
    *shift = sh;
}

// a3-a5: (conductivity +) chunk reduction, interface solves, recovery.
kaze_status aos_step(const ImageDesc& d, const Taps& tc, float tau, bool compute_g, int gmode,
                     float k_host, hipStream_t s) {
    const WorkList none{nullptr, nullptr, 0};
    KZ_LAUNCH(K_AOS_REDUCE, s,
              launch_aos_reduce(d, none, tc, tau, compute_g, gmode, k_host, 0, s));
    KZ_LAUNCH(K_AOS_IFACE, s, launch_aos_iface(d, none, 0, s));
    KZ_LAUNCH(K_AOS_RECOVER, s, launch_aos_recover(d, none, tau, 0, s));
    return KAZE_OK;
}

}  // namespace

extern "C" {

kaze_status kaze_default_params(kaze_params* p) {
    if (!p) return fail(KAZE_ERR_INVALID_ARG, "params pointer is NULL");
    p->octaves = 4;
    p->sublevels = 4;
    p->sigma0 = 1.6;
    p->sigma_cond = 1.0;
    p->diffusivity = KAZE_G2;
    p->k_percentile = 0.7;
    p->k_bins = 300;
    p->k_override = 0.0;
    p->det_threshold = 0.001;
    return KAZE_OK;
}

int kaze_num_levels(const kaze_params* p) {
    const kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    return p->octaves * p->sublevels;
}

kaze_status kaze_schedule(const kaze_params* p, double* sigma, double* t, double* tau,
                          double* sigma_norm, int* deriv_step) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    std::vector<Level> lv;
    schedule(p, lv);
    for (size_t i = 0; i < lv.size(); ++i) {
        if (sigma) sigma[i] = lv[i].sigma;
        if (t) t[i] = lv[i].t;
        if (tau) tau[i] = lv[i].tau;
        if (sigma_norm) sigma_norm[i] = lv[i].sigma_n;
        if (deriv_step) deriv_step[i] = lv[i].step;
    }
    return KAZE_OK;
}

size_t kaze_workspace_bytes(int W, int H, const kaze_params* p) {
    if (check_params(p) != KAZE_OK || check_size(W, H) != KAZE_OK) return 0;
    return layout(W, H, p).total;
}

kaze_status kaze_build_scale_space(const float* img, int W, int H, int ld_img,
                                   const kaze_params* p, float* levels, float* k_out, void* ws,
                                   size_t ws_bytes, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if (!img || !levels || !k_out)
        return fail(KAZE_ERR_INVALID_ARG, "img, levels and k_out must be non-NULL");
    if (ld_img < W) return fail(KAZE_ERR_INVALID_ARG, "ld_img (%d) < W (%d)", ld_img, W);
    if (!aligned(img, 4) || !aligned(levels, 4) || !aligned(k_out, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    const Workspace w = layout(W, H, p);
    if (!ws || !aligned(ws, 256) || ws_bytes < w.total)
        return fail(KAZE_ERR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    w.total, ws_bytes);

    hipStream_t s = static_cast<hipStream_t>(stream);
    ImageDesc d = image_desc(W, H, ws, w);
    char* base = static_cast<char*>(ws);
    unsigned* hist = reinterpret_cast<unsigned*>(base + w.hist);
    unsigned* hmax = reinterpret_cast<unsigned*>(base + w.hmax);

    std::vector<Level> lv;
    schedule(p, lv);
    const int N = (int)lv.size();
    const size_t plane = (size_t)W * H;
    const Taps t0 = gauss_taps(p->sigma0);
    const Taps tc = gauss_taps(p->sigma_cond);
    const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;

    // a1: base image L_0 = G_sigma0 * img
    KZ_LAUNCH(K_GAUSS, s, launch_gauss(img, ld_img, levels, W, H, t0, s));

    // a2: contrast factor k from the gradient histogram of L_0
    if (!(p->k_override > 0.0)) {
        unsigned long long mant;
        int shift;
        percentile_fraction(p->k_percentile, &mant, &shift);
        KZ_LAUNCH(K_FILL, s, launch_fill_u32(hist, p->k_bins, 0u, s));
        KZ_LAUNCH(K_FILL, s, launch_fill_u32(hmax, 1, 0u, s));
        KZ_LAUNCH(K_GRAD, s, launch_cond(levels, d.g, W, H, tc, nullptr, 1.f, 2, hmax, s));
        KZ_LAUNCH(K_HIST, s, launch_hist(d.g, (int)plane, hmax, hist, p->k_bins, s));
        KZ_LAUNCH(K_KSELECT, s, launch_kselect(hist, p->k_bins, hmax, mant, shift, k_out, s));
    } else {
        KZ_LAUNCH(K_FILL, s, launch_fill_f32(k_out, 1, (float)p->k_override, s));
    }
    d.k = k_out;

    // a3-a5: one AOS step per level, conductivity from the previous level
    for (int i = 1; i < N; ++i) {
        d.L = levels + plane * (i - 1);
        d.Lnext = levels + plane * i;
        st = aos_step(d, tc, (float)lv[i].tau, true, gmode, 1.f, s);
        if (st != KAZE_OK) return st;
    }
    return KAZE_OK;
}

kaze_status kaze_conductivity(const float* L, int W, int H, const kaze_params* p, double k,
                              float* g, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if (!L || !g) return fail(KAZE_ERR_INVALID_ARG, "L and g must be non-NULL");
    if (!aligned(L, 4) || !aligned(g, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    if (!(k > 0.0) || !isfinite(k)) return fail(KAZE_ERR_INVALID_ARG, "k must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Taps tc = gauss_taps(p->sigma_cond);
    const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;
    KZ_LAUNCH(K_COND, s, launch_cond(L, g, W, H, tc, nullptr, (float)k, gmode, nullptr, s));
    return KAZE_OK;
}

kaze_status kaze_aos_step(const float* L, const float* g, int W, int H, double tau,
                          float* L_next, void* ws, size_t ws_bytes, void* stream) {
    kaze_status st = check_size(W, H);
    if (st != KAZE_OK) return st;
    if (!L || !g || !L_next) return fail(KAZE_ERR_INVALID_ARG, "L, g and L_next must be non-NULL");
    if (!aligned(L, 4) || !aligned(g, 4) || !aligned(L_next, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    if (!(tau > 0.0) || !isfinite(tau)) return fail(KAZE_ERR_INVALID_ARG, "tau must be > 0");
    kaze_params p;
    kaze_default_params(&p);
    const Workspace w = layout(W, H, &p);
    if (!ws || !aligned(ws, 256) || ws_bytes < w.total)
        return fail(KAZE_ERR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    w.total, ws_bytes);
    ImageDesc d = image_desc(W, H, ws, w);
    d.L = L;
    d.Lnext = L_next;
    d.g = const_cast<float*>(g);  // read only when the conductivity is given
    return aos_step(d, gauss_taps(p.sigma_cond), (float)tau, false, 0, 1.f,
                    static_cast<hipStream_t>(stream));
}

kaze_status kaze_detector_response(const float* levels, int W, int H, const kaze_params* p,
                                   float* det, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if ((st = check_steps(p)) != KAZE_OK) return st;
    if (!levels || !det) return fail(KAZE_ERR_INVALID_ARG, "levels and det must be non-NULL");
    if (!aligned(levels, 4) || !aligned(det, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    std::vector<Level> lv;
    schedule(p, lv);
    DetLevels dl;
    memset(&dl, 0, sizeof(dl));
    for (size_t i = 0; i < lv.size(); ++i) {
        dl.step[i] = lv[i].step;
        dl.sn2[i] = (float)(lv[i].sigma_n * lv[i].sigma_n);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    KZ_LAUNCH(K_DET, s, launch_det(levels, det, W, H, (int)lv.size(), dl, s));
    return KAZE_OK;
}

kaze_status kaze_find_extrema(const float* det, int W, int H, const kaze_params* p,
                              kaze_keypoint* kps, int capacity, int* count, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if (!det || !count) return fail(KAZE_ERR_INVALID_ARG, "det and count must be non-NULL");
    if (capacity < 0) return fail(KAZE_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && !kps) return fail(KAZE_ERR_INVALID_ARG, "kps is NULL with capacity > 0");
    if (!aligned(det, 4) || !aligned(count, 4) || (kps && !aligned(kps, 4)))
        return fail(KAZE_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = p->octaves * p->sublevels;
    KZ_LAUNCH(K_FILL, s, launch_fill_u32(reinterpret_cast<unsigned*>(count), 1, 0u, s));
    KZ_LAUNCH(K_NMS, s, launch_nms(det, W, H, N, (float)p->det_threshold, kps, capacity, count, s));
    return KAZE_OK;
}

const char* kaze_last_error(void) { return g_err; }

kaze_status kaze_profile_begin(const char* kernel_names) {
    if (!kernel_names) return fail(KAZE_ERR_INVALID_ARG, "kernel name list is NULL");
    unsigned mask = 0;
    const char* p = kernel_names;
    while (*p) {
        const char* e = strchr(p, ',');
        const size_t n = e ? (size_t)(e - p) : strlen(p);
        int found = -1;
        for (int i = 0; i < K_COUNT; ++i)
            if (strlen(kKernelNames[i]) == n && strncmp(p, kKernelNames[i], n) == 0) found = i;
        if (found < 0) return fail(KAZE_ERR_INVALID_ARG, "unknown kernel name in '%s'", kernel_names);
        mask |= 1u << found;
        p += n;
        if (*p == ',') ++p;
    }
    if (!mask) return fail(KAZE_ERR_INVALID_ARG, "empty kernel name list");
    g_prof.mask = mask;
    g_prof.used = 0;
    return KAZE_OK;
}

kaze_status kaze_profile_end(int* launches, double* total_ms) {
    double sum = 0.0;
    for (int i = 0; i < g_prof.used; ++i) {
        hipError_t e = hipEventSynchronize(g_prof.ev[2 * i + 1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
        if (e != hipSuccess) {
            g_prof.mask = 0;
            return fail(KAZE_ERR_HIP, "profiling events failed: %s", hipGetErrorString(e));
        }
        sum += ms;
    }
    if (launches) *launches = g_prof.used;
    if (total_ms) *total_ms = sum;
    g_prof.mask = 0;
    g_prof.used = 0;
    return KAZE_OK;
}

const char* kaze_kernel_names(void) {
    static char buf[512] = "";
    if (!buf[0]) {
        for (int i = 0; i < K_COUNT; ++i) {
            if (i) strcat(buf, ",");
            strcat(buf, kKernelNames[i]);
        }
    }
    return buf;
}

kaze_status kaze_copy_f32(const float* src, float* dst, size_t n, void* stream) {
    if (!src || !dst) return fail(KAZE_ERR_INVALID_ARG, "src and dst must be non-NULL");
    if (!aligned(src, 16) || !aligned(dst, 16))
        return fail(KAZE_ERR_INVALID_ARG, "src and dst must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KZ_LAUNCH(K_COPY, s, launch_copy(src, dst, n, s));
    return KAZE_OK;
}

}  // extern "C"
