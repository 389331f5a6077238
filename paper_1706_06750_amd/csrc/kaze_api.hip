// C ABI of libkaze: argument validation, the level schedule (Eqs. 6-7),
// workspace layout and the launch sequence of the scale space (Sec. II-A,
// Sec. III-A), detector response (Eq. 8) and extrema (Sec. II-B), for one
// image or for a batch of images replayed through a captured hipGraph.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "kaze.h"
#include "kaze_internal.h"
#include "fed_internal.h"
#include "kaze_surrogate.h"
#include "sg_internal.h"

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace kaze {
kaze_status set_error(kaze_status st, const char* fmt, va_list ap) {
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    return st;
}
}  // namespace kaze

namespace {

using namespace kaze;

kaze_status fail(kaze_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    set_error(st, fmt, ap);
    va_end(ap);
    return st;
}

// ---------------------------------------------------------------- profiling
const char* const kKernelNames[K_COUNT] = {
    "gauss", "grad", "hist", "kselect", "cond", "aos_reduce", "aos_iface", "aos_recover",
    "det",   "nms",  "fill", "copy",    "sg_pack", "sg_conv1", "sg_conv", "sg_conv6",
    "sg_probe", "fed", "refine", "deriv", "describe"};

struct Profiler {
    unsigned mask = 0;  // bit i: record launches of kernel i
    bool capturing = false;  // no pairs while a graph is captured
    bool in_segment = false; // a batch run's level segment has its own pair
    std::vector<hipEvent_t> ev;  // pairs: start, stop
    int used = 0;
    static constexpr int kMaxPairs = 65536;
} g_prof;

struct ProfScope {
    int id;
    hipStream_t s;
    bool on;
    ProfScope(int id_, hipStream_t s_) : id(id_), s(s_), on(false) {
        if (g_prof.capturing || g_prof.in_segment || !(g_prof.mask & (1u << id)) ||
            g_prof.used >= Profiler::kMaxPairs)
            return;
        const size_t need = 2 * (size_t)(g_prof.used + 1);
        while (g_prof.ev.size() < need) {
            hipEvent_t e;
            // timing only: no system-scope cache write-back at each record
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return;
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

#define KZ_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(KAZE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
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
        if (p->k_bins < 1 || p->k_bins > KAZE_MAX_K_BINS)
            return fail(KAZE_ERR_INVALID_ARG, "k_bins must be in [1, %d]", KAZE_MAX_K_BINS);
    }
    if (!isfinite(p->det_threshold))
        return fail(KAZE_ERR_INVALID_ARG, "det_threshold must be finite");
    if (p->scheme != KAZE_AOS && p->scheme != KAZE_FED)
        return fail(KAZE_ERR_INVALID_ARG, "scheme must be KAZE_AOS or KAZE_FED");
    if (p->extrema_window != KAZE_WINDOW_3X3 && p->extrema_window != KAZE_WINDOW_SIGMA)
        return fail(KAZE_ERR_INVALID_ARG, "extrema_window must be KAZE_WINDOW_3X3 or KAZE_WINDOW_SIGMA");
    if (p->substeps < 1 || p->substeps > kMaxSubsteps)
        return fail(KAZE_ERR_INVALID_ARG, "substeps must be in [1, %d]", kMaxSubsteps);
    return KAZE_OK;
}

void schedule(const kaze_params* p, std::vector<Level>& lv);

// Cross-level window half-sides: 1, or for the exact test the h whose side
// 2h + 1 is the odd number nearest sigma_i (half up), at least 1; capped at
// the largest image side (the window is clipped to the image anyway).
NmsRadii nms_radii(const kaze_params* p) {
    NmsRadii r;
    const int N = p->octaves * p->sublevels;
    for (int i = 0; i < kMaxLevels; ++i) {
        r.h[i] = 1;
        r.step[i] = 1;
    }
    std::vector<Level> lv;
    schedule(p, lv);
    for (int i = 0; i < N && i < kMaxLevels; ++i) r.step[i] = std::min(lv[i].step, kMaxStep);
    if (p->extrema_window == KAZE_WINDOW_SIGMA) {
        for (int i = 0; i < N; ++i) {
            const int o = i / p->sublevels, s = i % p->sublevels;
            const double sigma = p->sigma0 * pow(2.0, o + (double)s / p->sublevels);
            const double h = floor((sigma - 1.0) / 2.0 + 0.5);
            r.h[i] = h < 1.0 ? 1 : (h > kMaxSide ? kMaxSide : (int)h);
        }
    }
    return r;
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

static_assert(kAosShapes == KAZE_AOS_SHAPES, "the public shape count matches the kernels");

// Every AOS tile shape takes every image size the library accepts.
bool shape_fits(int W, int H, int shape) {
    (void)W;
    (void)H;
    return shape >= 0 && shape < kAosShapes;
}

// Every AOS shape serves the longest line in one wavefront: the interface
// solve spans at most 64 lanes of M chunks each (iface_lanes), which
// check_size guarantees for every accepted image.
constexpr bool shapes_fit_one_wavefront() {
    for (const AosShape& a : kAosShape)
        if ((kMaxSide + a.rc - 1) / a.rc > 64 * a.m || (kMaxSide + a.cc - 1) / a.cc > 64 * a.m)
            return false;
    return true;
}
static_assert(shapes_fit_one_wavefront(), "an AOS shape needs more than 64 interface lanes");

kaze_status check_size(int W, int H) {
    if (W < 8 || H < 8) return fail(KAZE_ERR_INVALID_ARG, "image must be at least 8x8");
    if (W > kMaxSide || H > kMaxSide)
        return fail(KAZE_ERR_UNSUPPORTED, "image larger than %dx%d (got %dx%d)", kMaxSide,
                    kMaxSide, W, H);
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

// Per-level detector constants; band: rows per detector band (det_band_for
// of the pixels of one run).
DetLevels det_levels(const std::vector<Level>& lv, int band) {
    DetLevels dl;
    memset(&dl, 0, sizeof(dl));
    dl.band = band;
    for (size_t i = 0; i < lv.size(); ++i) {
        dl.step[i] = lv[i].step;
        dl.sn2[i] = (float)(lv[i].sigma_n * lv[i].sigma_n);
        dl.sn[i] = (float)lv[i].sigma_n;
    }
    return dl;
}

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

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- workspace
// Per-image scratch: conductivity plane, interface equations and solutions
// of the AOS tile shape, histogram and hmax.
struct Scratch {
    size_t g, rrow, rcol, zrow, zcol, hist, hmax, tmp, sub, mask, total;
};

// fed: room for the second plane of the explicit steps (FED scheme only);
// sub: the plane between the sub-steps of a level (more than one sub-step);
// mask_levels: detector masks of that many levels (BatchImage::mask).
Scratch scratch_layout(int W, int H, int nbins, int shape, size_t base, bool fed = false,
                       bool sub = false, int mask_levels = 0) {
    Scratch w;
    const size_t ncx = aos_row_chunks(W, kAosShape[shape].rc);
    const size_t ncy = aos_col_chunks(H, kAosShape[shape].cc);
    size_t off = base;
    w.g = off;    off = align256(off + (size_t)W * H * sizeof(float));
    w.rrow = off; off = align256(off + (size_t)H * ncx * kEqFloats * sizeof(float));
    w.rcol = off; off = align256(off + (size_t)W * ncy * kEqFloats * sizeof(float));
    w.zrow = off; off = align256(off + (size_t)H * ncx * 2 * sizeof(float));
    w.zcol = off; off = align256(off + (size_t)W * ncy * 2 * sizeof(float));
    w.hist = off;
    off = align256(off + (size_t)(nbins > 0 ? nbins : 1) * kHistCopies * sizeof(unsigned));
    // one |grad| maximum per gradient tile (the smallest tile height, 32)
    w.hmax = off; off = align256(off + (size_t)aos_tiles_of(W, H, 32) * sizeof(unsigned));
    w.tmp = off;  off = align256(off + (fed ? (size_t)W * H * sizeof(float) : 0));
    w.sub = off;  off = align256(off + (sub ? (size_t)W * H * sizeof(float) : 0));
    w.mask = off;
    off = align256(off + (size_t)mask_levels * H * mask_words(W) * sizeof(unsigned long long));
    w.total = off - base;
    return w;
}

int hist_bins(const kaze_params* p) { return p->k_override > 0.0 ? 1 : p->k_bins; }

ImageDesc aos_desc(int W, int H, int shape, char* base, const Scratch& w, const float* k) {
    ImageDesc d;
    d.L = nullptr;
    d.Lnext = nullptr;
    d.g = reinterpret_cast<float*>(base + w.g);
    d.rrow = reinterpret_cast<float*>(base + w.rrow);
    d.rcol = reinterpret_cast<float*>(base + w.rcol);
    d.zrow = reinterpret_cast<float*>(base + w.zrow);
    d.zcol = reinterpret_cast<float*>(base + w.zcol);
    d.k = k;
    d.W = W;
    d.H = H;
    d.gate = nullptr;
    d.bound = 0.f;
    d.nchr = aos_row_chunks(W, kAosShape[shape].rc);
    d.nchc = aos_col_chunks(H, kAosShape[shape].cc);
    return d;
}

BatchImage batch_image(int W, int H) {
    BatchImage b;
    memset(&b, 0, sizeof(b));
    b.W = W;
    b.H = H;
    return b;
}

// a3-a5: (conductivity +) chunk reduction, interface solves, recovery, on
// the tiles, chunks and interface lanes of `shape`.
kaze_status aos_step(const ImageDesc& d, const AosWork& tiles, const AosWork& lines, int shape,
                     const Taps& tc, float tau, bool compute_g, int gmode, float k_host,
                     hipStream_t s) {
    KZ_LAUNCH(K_AOS_REDUCE, s,
              launch_aos_reduce(d, tiles, shape, tc, tau, compute_g, gmode, k_host, s));
    KZ_LAUNCH(K_AOS_IFACE, s, launch_aos_iface(d, lines, shape, s));
    KZ_LAUNCH(K_AOS_RECOVER, s, launch_aos_recover(d, tiles, shape, tau, s));
    return KAZE_OK;
}

// The shape of single-image calls: the default rule of the interface lanes.
int default_shape(int W, int H) { return default_shape_for(aos_line_groups(W, H, kAosShape[1])); }

// The default shape of a batch (aos_shape -1): the same rule over the
// interface wavefronts of all its images.
int default_batch_shape(const kaze_image_desc* im, int n) {
    if (!im || n < 1) return 0;
    long long groups = 0;
    for (int j = 0; j < n; ++j)
        if (im[j].W >= 1 && im[j].H >= 1) groups += aos_line_groups(im[j].W, im[j].H, kAosShape[1]);
    return default_shape_for(groups);
}

// One FED cycle of total time T (Eq. 5) from L into out with g fixed: the
// steps of fed_schedule(T) in launches of kFedS, alternating between out and
// tmp so that the last launch writes out.
kaze_status fed_cycle(const float* L, const float* g, float* out, float* tmp, int W, int H,
                      double T, hipStream_t s) {
    const std::vector<double> tau = fed_schedule(T);
    const int n = (int)tau.size();
    const int launches = (n + kFedS - 1) / kFedS;
    const float* src = L;
    for (int l = 0; l < launches; ++l) {
        float* dst = ((launches - 1 - l) % 2 == 0) ? out : tmp;
        FedSteps st;
        st.n = std::min(kFedS, n - l * kFedS);
        for (int j = 0; j < kFedS; ++j)
            st.half_tau[j] = j < st.n ? (float)(0.5 * tau[l * kFedS + j]) : 0.f;
        KZ_LAUNCH(K_FED, s, launch_fed(src, g, dst, W, H, st, s));
        src = dst;
    }
    return KAZE_OK;
}

// a1-a2: base image and contrast factor (or the given k) for one image or a
// batch (images / tiles / AOS tiles of height cty / hist items of hist_chunk
// pixels select the work).
kaze_status base_and_k(const BatchImage& b0, const ImgWork& images, const ImgWork& tiles,
                       const ImgWork& ctiles, int cty, const ImgWork& hist, int hist_chunk,
                       const kaze_params* p, hipStream_t s) {
    const Taps t0 = gauss_taps(p->sigma0);
    const Taps tc = gauss_taps(p->sigma_cond);
    const bool use_hist = !(p->k_override > 0.0);
    // the Gaussian's first tile of each image resets its counters
    KZ_LAUNCH(K_GAUSS, s,
              launch_gauss(b0, tiles, t0, hist_bins(p), use_hist ? 0.f : (float)p->k_override, s));
    if (use_hist) {
        unsigned long long mant;
        int shift;
        percentile_fraction(p->k_percentile, &mant, &shift);
        KZ_LAUNCH(K_GRAD, s, launch_cond(b0, ctiles, tc, 1.f, 2, cty, s));
        KZ_LAUNCH(K_HIST, s, launch_hist(b0, hist, p->k_bins, cty, hist_chunk, s));
        KZ_LAUNCH(K_KSELECT, s, launch_kselect(b0, images, p->k_bins, mant, shift, cty, s));
    }
    return KAZE_OK;
}

}  // namespace

// ============================================================================
// Batches: device tables, graph capture and replay.
// ============================================================================
namespace {
struct SgBatch;
}

struct kaze_batch {
    int n = 0;
    int N = 0;
    int shape = 0;
    bool with_det = false;
    bool with_nms = false;
    kaze_params p;
    std::vector<Level> lv;
    BatchImage* d_imgs = nullptr;
    ImageDesc* d_lvl = nullptr;  // (N-1) x m x n: sub-step q of level i at row (i-1) m + q
    int2 *d_items = nullptr, *d_tiles = nullptr, *d_aos = nullptr, *d_lines = nullptr,
         *d_hist = nullptr, *d_det = nullptr, *d_nms = nullptr;
    int n_tiles = 0, n_aos = 0, n_lines = 0, n_hist = 0, n_det = 0, n_nms = 0;
    // captured segments: 0 base image + k, 1 the N-1 AOS steps with the
    // detector response of each level on a forked stream, 2 extrema
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    hipStream_t side = nullptr;      // fork target while a segment is captured
    std::vector<hipEvent_t> ev;      // fork / join points (N + 1)
    bool fork_det = false;           // detector response beside the steps, per level
    int det_band = kDetBandShort;    // rows per detector band (det_band_for of the plan's pixels)
    int hist_chunk = kHistChunk;     // pixels per histogram block (hist_chunk_for of the same)
    SgBatch* sg = nullptr;           // surrogate steps (kaze_sg_batch_create), or none
};

// The detector response of every level runs beside the steps, on a second
// stream, only for batches of at least this many pixels.  Smaller batches
// run it after the steps: detector blocks beside the step kernels slowed the
// steps by more than the detector took after them (one 1920x1200 image:
// 24.2 -> 27.7 us per level; 8 x 1920x1200: 3260 against 3505 images/s),
// while batches of 67 and 295 Mpx gain 2.5% from the overlap.
constexpr double kForkDetPixels = 32e6;

extern "C" kaze_status kaze_batch_destroy(kaze_batch* b);

namespace {

// Surrogate steps of a batch (kaze_sg_batch_create); defined with the
// surrogate scale space below.
struct SgSpec {
    const kaze_sg_config* c;
    const void* packed;
    const int* probe_xy;  // (host) n x N x probes x 2
    float* err;           // (device) n x N
};
size_t sg_batch_bytes(const kaze_image_desc* im, int n, const kaze_params* p,
                      const kaze_sg_config* c);
kaze_status sg_batch_check(const kaze_image_desc* im, int n, const kaze_params* p,
                           const SgSpec& sp);
kaze_status sg_batch_build(kaze_batch* B, const kaze_image_desc* im, const SgSpec& sp,
                           char* base, size_t off, const std::vector<size_t>& scratch);
kaze_status sg_batch_levels(const kaze_batch& B, hipStream_t s);

struct BatchLayout {
    size_t imgs, lvl, items, tiles, aos, lines, hist, det, nms, tables_end;
    std::vector<size_t> scratch;  // per image
    size_t total;
    int n_tiles, n_aos, n_lines, n_hist, n_det, n_nms;
};

// Smallest and largest Scharr step of the detector levels.
void step_range(const kaze_params* p, int& smin, int& smax) {
    std::vector<Level> lv;
    schedule(p, lv);
    smin = 1 << 30;
    smax = 0;
    for (const Level& l : lv) {
        smin = std::min(smin, l.step);
        smax = std::max(smax, l.step);
    }
}

// Pixels of one run of a batch.
double batch_pixels(const kaze_image_desc* im, int n) {
    double px = 0;
    for (int j = 0; j < n; ++j) px += (double)im[j].W * im[j].H;
    return px;
}

BatchLayout batch_layout(const kaze_image_desc* im, int n, const kaze_params* p, int shape) {
    BatchLayout L;
    const int N = p->octaves * p->sublevels;
    int smin, smax;
    step_range(p, smin, smax);
    const int band = det_band_for(batch_pixels(im, n));
    const int hist_chunk = hist_chunk_for(batch_pixels(im, n));
    L.n_tiles = L.n_aos = L.n_lines = L.n_hist = L.n_det = L.n_nms = 0;
    for (int j = 0; j < n; ++j) {
        L.n_tiles += tiles_of(im[j].W, im[j].H);
        L.n_aos += aos_tiles_of(im[j].W, im[j].H, kAosShape[shape].ty);
        L.n_lines += aos_line_groups(im[j].W, im[j].H, kAosShape[shape]);
        L.n_hist += (im[j].W * im[j].H + hist_chunk - 1) / hist_chunk;
        L.n_det += det_tiles_of(im[j].W, im[j].H, smin, smax, band);
        L.n_nms += nms_blocks_of(im[j].W, im[j].H, true);
    }
    size_t off = 0;
    L.imgs = off;  off = align256(off + n * sizeof(BatchImage));
    L.lvl = off;
    off = align256(off + (size_t)(N > 1 ? N - 1 : 1) * p->substeps * n * sizeof(ImageDesc));
    L.items = off; off = align256(off + n * sizeof(int2));
    L.tiles = off; off = align256(off + L.n_tiles * sizeof(int2));
    L.aos = off;   off = align256(off + L.n_aos * sizeof(int2));
    L.lines = off; off = align256(off + L.n_lines * sizeof(int2));
    L.hist = off;  off = align256(off + L.n_hist * sizeof(int2));
    L.det = off;   off = align256(off + L.n_det * sizeof(int2));
    L.nms = off;   off = align256(off + L.n_nms * sizeof(int2));
    L.tables_end = off;
    L.scratch.resize(n);
    for (int j = 0; j < n; ++j) {
        L.scratch[j] = off;
        // detector masks when the batch finds extrema
        off += scratch_layout(im[j].W, im[j].H, hist_bins(p), shape, 0, false, p->substeps > 1,
                              im[0].count ? N : 0)
                   .total;
    }
    L.total = off;
    return L;
}

kaze_status check_batch(const kaze_image_desc* im, int n, const kaze_params* p, int shape) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if (p->scheme != KAZE_AOS)
        return fail(KAZE_ERR_UNSUPPORTED, "batches run the AOS scheme only");
    if ((st = check_steps(p)) != KAZE_OK) return st;
    if (!im || n < 1) return fail(KAZE_ERR_INVALID_ARG, "a batch needs at least one image");
    if (shape < 0 || shape >= kAosShapes) return fail(KAZE_ERR_INVALID_ARG, "bad AOS tile shape");
    const bool det0 = im[0].det != nullptr, cnt0 = im[0].count != nullptr;
    for (int j = 0; j < n; ++j) {
        const kaze_image_desc& d = im[j];
        if ((st = check_size(d.W, d.H)) != KAZE_OK) return st;
        if (!shape_fits(d.W, d.H, shape))
            return fail(KAZE_ERR_UNSUPPORTED, "image %d (%dx%d) does not fit tile shape %dx%d", j,
                        d.W, d.H, kAosTX, kAosShape[shape].ty);
        if (!d.img || !d.levels || !d.k)
            return fail(KAZE_ERR_INVALID_ARG, "image %d: img, levels and k must be non-NULL", j);
        if (d.ld_img < d.W) return fail(KAZE_ERR_INVALID_ARG, "image %d: ld_img < W", j);
        if ((d.det != nullptr) != det0 || (d.count != nullptr) != cnt0)
            return fail(KAZE_ERR_INVALID_ARG, "det and count must be given for all images or none");
        if (d.count && !d.det)
            return fail(KAZE_ERR_INVALID_ARG, "image %d: extrema need det", j);
        if (d.capacity < 0 || (d.capacity > 0 && !d.kps))
            return fail(KAZE_ERR_INVALID_ARG, "image %d: bad keypoint buffer", j);
        if (!aligned(d.img, 4) || !aligned(d.levels, 4) || !aligned(d.k, 4) ||
            (d.det && !aligned(d.det, 4)) || (d.count && !aligned(d.count, 4)) ||
            (d.kps && !aligned(d.kps, 4)))
            return fail(KAZE_ERR_INVALID_ARG, "image %d: buffers must be 4-byte aligned", j);
    }
    return KAZE_OK;
}

// The a1-a7 sequence of a batch, one launch per phase for all images, in
// three segments: 0 base image and contrast factor, 1 the AOS steps and the
// detector response, 2 extrema.  With a side stream the detector response of
// large batches forks off the step sequence level by level.
kaze_status enqueue_segment(const kaze_batch& B, int seg, hipStream_t s, hipStream_t side) {
    const kaze_params* p = &B.p;
    const BatchImage b0 = batch_image(0, 0);
    if (seg == 0) {
        const ImgWork images{B.d_imgs, B.d_items, B.n};
        const ImgWork tiles{B.d_imgs, B.d_tiles, B.n_tiles};
        const ImgWork ctiles{B.d_imgs, B.d_aos, B.n_aos};  // the plan's AOS tiles
        const ImgWork hist{B.d_imgs, B.d_hist, B.n_hist};
        return base_and_k(b0, images, tiles, ctiles, kAosShape[B.shape].ty, hist, B.hist_chunk, p,
                          s);
    }
    const ImgWork det{B.d_imgs, B.d_det, B.n_det};
    DetLevels dl = det_levels(B.lv, B.det_band);
    dl.thr = (float)p->det_threshold;  // of the masks the extrema kernel reads
    const bool fork = B.fork_det && side != nullptr;
    if (seg == 1 && B.sg) return sg_batch_levels(B, s);
    if (seg == 1) {
        // The detector response of level i needs level i only: in a large
        // batch (graph and eager runs) it runs on the side stream,
        // overlapping the later steps.
        const Taps tc = gauss_taps(p->sigma_cond);
        const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;
        hipStream_t ds = fork ? side : s;
        auto det_level = [&](int i) -> kaze_status {
            if (!fork) return KAZE_OK;
            {
                KZ_HIP(hipEventRecord(B.ev[i], s));
                KZ_HIP(hipStreamWaitEvent(ds, B.ev[i], 0));
            }
            KZ_LAUNCH(K_DET, ds, launch_det(b0, det, i, i + 1, dl, ds));
            return KAZE_OK;
        };
        kaze_status st = det_level(0);
        if (st != KAZE_OK) return st;
        ImageDesc a0;
        memset(&a0, 0, sizeof(a0));
        const int m = p->substeps;
        for (int i = 1; i < B.N; ++i) {
            for (int q = 0; q < m; ++q) {
                const ImageDesc* lvl = B.d_lvl + ((size_t)(i - 1) * m + q) * B.n;
                const AosWork at{lvl, B.d_aos, B.n_aos};
                const AosWork al{lvl, B.d_lines, B.n_lines};
                st = aos_step(a0, at, al, B.shape, tc, (float)(B.lv[i].tau / m), true, gmode, 1.f,
                              s);
                if (st != KAZE_OK) return st;
            }
            if ((st = det_level(i)) != KAZE_OK) return st;
        }
        if (fork) {  // join
            KZ_HIP(hipEventRecord(B.ev[B.N], ds));
            KZ_HIP(hipStreamWaitEvent(s, B.ev[B.N], 0));
        }
        return KAZE_OK;
    }
    if (B.with_det && !fork) KZ_LAUNCH(K_DET, s, launch_det(b0, det, 0, B.N, dl, s));
    if (B.with_nms) {
        const ImgWork nms{B.d_imgs, B.d_nms, B.n_nms};
        KZ_LAUNCH(K_NMS, s,
                  launch_nms(b0, nms, B.N, (float)p->det_threshold, nms_radii(p), s, true));
    }
    return KAZE_OK;
}

// Eager run of a batch plan: the same launches as its graphs, the per-level
// detector fork of large batches onto the plan's second stream (ordered
// through events), and under kaze_profile_begin("aos_reduce") one event pair
// around the level segment as in a graph run.
kaze_status enqueue_batch(const kaze_batch& B, hipStream_t s) {
    kaze_status st = enqueue_segment(B, 0, s, B.side);
    if (st != KAZE_OK) return st;
    {
        ProfScope ps(K_AOS_REDUCE, s);
        g_prof.in_segment = true;
        st = enqueue_segment(B, 1, s, B.side);
        g_prof.in_segment = false;
    }
    if (st != KAZE_OK) return st;
    return enqueue_segment(B, 2, s, B.side);
}

kaze_status batch_create(const kaze_image_desc* im, int n, const kaze_params* p, int shape,
                         void* ws, size_t ws_bytes, kaze_batch** out,
                         const SgSpec* sp = nullptr) {
    kaze_status st = check_batch(im, n, p, shape);
    if (st != KAZE_OK) return st;
    if (!out) return fail(KAZE_ERR_INVALID_ARG, "out pointer is NULL");
    if (sp && (st = sg_batch_check(im, n, p, *sp)) != KAZE_OK) return st;
    const BatchLayout L = batch_layout(im, n, p, shape);
    int smin, smax;
    step_range(p, smin, smax);
    const size_t total = L.total + (sp ? sg_batch_bytes(im, n, p, sp->c) : 0);
    if (!ws || !aligned(ws, 256) || ws_bytes < total)
        return fail(KAZE_ERR_WORKSPACE, "batch workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    total, ws_bytes);
    char* base = static_cast<char*>(ws);
    kaze_batch* B = new kaze_batch();
    B->n = n;
    B->p = *p;
    schedule(p, B->lv);
    B->N = (int)B->lv.size();
    B->shape = shape;
    B->with_det = im[0].det != nullptr;
    B->with_nms = im[0].count != nullptr;
    const double px = batch_pixels(im, n);
    B->det_band = det_band_for(px);
    B->hist_chunk = hist_chunk_for(px);
    // surrogate batches run the detector after the steps (no fork)
    B->fork_det = !sp && B->with_det && px >= kForkDetPixels;
    B->d_imgs = reinterpret_cast<BatchImage*>(base + L.imgs);
    B->d_lvl = reinterpret_cast<ImageDesc*>(base + L.lvl);
    B->d_items = reinterpret_cast<int2*>(base + L.items);
    B->d_tiles = reinterpret_cast<int2*>(base + L.tiles);
    B->d_aos = reinterpret_cast<int2*>(base + L.aos);
    B->d_lines = reinterpret_cast<int2*>(base + L.lines);
    B->d_hist = reinterpret_cast<int2*>(base + L.hist);
    B->d_det = reinterpret_cast<int2*>(base + L.det);
    B->d_nms = reinterpret_cast<int2*>(base + L.nms);
    B->n_tiles = L.n_tiles;
    B->n_aos = L.n_aos;
    B->n_lines = L.n_lines;
    B->n_hist = L.n_hist;
    B->n_det = L.n_det;
    B->n_nms = L.n_nms;

    // host image of the tables, uploaded once
    std::vector<char> host(L.tables_end, 0);
    BatchImage* himgs = reinterpret_cast<BatchImage*>(host.data() + L.imgs);
    ImageDesc* hlvl = reinterpret_cast<ImageDesc*>(host.data() + L.lvl);
    int2* hitems = reinterpret_cast<int2*>(host.data() + L.items);
    int2* ht = reinterpret_cast<int2*>(host.data() + L.tiles);
    int2* ha = reinterpret_cast<int2*>(host.data() + L.aos);
    int2* hl = reinterpret_cast<int2*>(host.data() + L.lines);
    int2* hh = reinterpret_cast<int2*>(host.data() + L.hist);
    int2* hd = reinterpret_cast<int2*>(host.data() + L.det);
    int2* hn = reinterpret_cast<int2*>(host.data() + L.nms);
    int it = 0, ia = 0, il = 0, ih = 0, idt = 0, inm = 0;
    const int nb = hist_bins(p);
    const int m = p->substeps;
    for (int j = 0; j < n; ++j) {
        const kaze_image_desc& d = im[j];
        const Scratch sc =
            scratch_layout(d.W, d.H, nb, shape, L.scratch[j], false, m > 1, B->with_nms ? B->N : 0);
        BatchImage b = batch_image(d.W, d.H);
        b.img = d.img;
        b.ld = d.ld_img;
        b.levels = d.levels;
        b.det = d.det;
        b.g = reinterpret_cast<float*>(base + sc.g);
        b.hist = reinterpret_cast<unsigned*>(base + sc.hist);
        b.hmax = reinterpret_cast<unsigned*>(base + sc.hmax);
        b.k = d.k;
        b.kps = d.kps;
        b.capacity = d.capacity;
        b.count = d.count;
        b.mask = B->with_nms ? reinterpret_cast<unsigned long long*>(base + sc.mask) : nullptr;
        himgs[j] = b;
        hitems[j] = make_int2(j, 0);
        const size_t plane = (size_t)d.W * d.H;
        float* mid = reinterpret_cast<float*>(base + sc.sub);
        for (int i = 1; i < B->N; ++i) {
            const float* src = d.levels + plane * (i - 1);
            for (int q = 0; q < m; ++q) {  // as in kaze_build_scale_space
                ImageDesc a = aos_desc(d.W, d.H, shape, base, sc, d.k);
                a.L = src;
                a.Lnext = ((m - 1 - q) % 2 == 0) ? d.levels + plane * i : mid;
                if (sp) {  // the exact step runs only where the surrogate was rejected
                    a.gate = sp->err + (size_t)j * B->N + i;
                    a.bound = (float)sp->c->bound;
                }
                hlvl[((size_t)(i - 1) * m + q) * n + j] = a;
                src = a.Lnext;
            }
        }
        for (int t = 0; t < tiles_of(d.W, d.H); ++t) ht[it++] = make_int2(j, t);
        for (int t = 0; t < aos_tiles_of(d.W, d.H, kAosShape[shape].ty); ++t)
            ha[ia++] = make_int2(j, t);
        for (int t = 0; t < aos_line_groups(d.W, d.H, kAosShape[shape]); ++t)
            hl[il++] = make_int2(j, t);
        for (int t = 0; t < (d.W * d.H + B->hist_chunk - 1) / B->hist_chunk; ++t)
            hh[ih++] = make_int2(j, t);
        for (int t = 0; t < det_tiles_of(d.W, d.H, smin, smax, B->det_band); ++t)
            hd[idt++] = make_int2(j, t);
        for (int t = 0; t < nms_blocks_of(d.W, d.H, true); ++t) hn[inm++] = make_int2(j, t);
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipMemcpy(base, host.data(), L.tables_end, hipMemcpyHostToDevice);
    if (e == hipSuccess && sp) {
        st = sg_batch_build(B, im, *sp, base, L.total, L.scratch);
        if (st != KAZE_OK) {
            kaze_batch_destroy(B);
            return st;
        }
    }
    // capture each segment once on a private stream (default priority); the
    // detector response forks to a second one
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking);
    for (int i = 0; i <= B->N && e == hipSuccess; ++i) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) B->ev.push_back(ev);
    }
    for (int seg = 0; seg < 3 && e == hipSuccess && st == KAZE_OK; ++seg) {
        hipGraph_t graph = nullptr;
        g_prof.capturing = true;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = enqueue_segment(*B, seg, cs, B->side);
            const hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (st == KAZE_OK && e2 != hipSuccess) e = e2;
        }
        g_prof.capturing = false;
        if (e == hipSuccess && st == KAZE_OK)
            e = hipGraphInstantiate(&B->exec[seg], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (st != KAZE_OK || e != hipSuccess) {
        kaze_batch_destroy(B);
        return st != KAZE_OK ? st : fail(KAZE_ERR_HIP, "batch graph setup failed: %s",
                                         hipGetErrorString(e));
    }
    *out = B;
    return KAZE_OK;
}

kaze_status run_graphs(const kaze_batch& B, hipStream_t s) {
    KZ_HIP(hipGraphLaunch(B.exec[0], s));
    {
        // the level segment holds every AOS launch of the run; with
        // aos_reduce in the profiling list one event pair brackets it
        ProfScope ps(K_AOS_REDUCE, s);
        KZ_HIP(hipGraphLaunch(B.exec[1], s));
    }
    KZ_HIP(hipGraphLaunch(B.exec[2], s));
    return KAZE_OK;
}

// ============================================================================
// Surrogate scale space: every AOS step may be replaced by the learned
// surrogate, accepted per level by the probe check and otherwise recomputed
// exactly.
// ============================================================================
struct SgLayout {
    size_t scratch, x0, xa, xb, delta, tau, rects, items, total;
    int max_items;
};

// Conv items (chunk * strips + strip) whose output rows/columns meet a probe
// window grown by the receptive-field radius: outside that region stale
// activations can reach at most kProbeHalo - 1 pixels inward.
void sg_probe_items(const sg::Geo& g, const int4* rects, int n, std::vector<int>& out) {
    std::vector<char> mark((size_t)g.strips * g.chunks, 0);
    for (int p = 0; p < n; ++p) {
        const int4 r = rects[p];
        const int xa = std::max(0, r.x - sg::kProbeHalo), xb = std::min(g.W - 1, r.x + r.z - 1 + sg::kProbeHalo);
        const int ya = std::max(0, r.y - sg::kProbeHalo), yb = std::min(g.H - 1, r.y + r.w - 1 + sg::kProbeHalo);
        for (int c = ya / g.R; c <= yb / g.R; ++c)
            for (int st = xa / sg::kStrip; st <= xb / sg::kStrip; ++st) mark[(size_t)c * g.strips + st] = 1;
    }
    out.clear();
    for (size_t i = 0; i < mark.size(); ++i)
        if (mark[i]) out.push_back((int)i);
}

// Probe windows are short: their convolutions run with few rows per wave,
// so that the latency of one wave's row sweep stays small.
constexpr int kProbeRows = 4;
// Images of a surrogate batch (the input-packing grid has one row per image).
constexpr int kSgBatchMaxImages = 4096;

int sg_max_items(const kaze_sg_config* c) {
    // a window of probe_size + 2 halo pixels spans at most this many strips x chunks
    const int span = c->probe_size + 2 * sg::kProbeHalo;
    const int per = (span / sg::kStrip + 2) * (span / kProbeRows + 2);
    return std::max(1, c->probes * per);
}

SgLayout sg_layout(int W, int H, const kaze_params* p, const kaze_sg_config* c, int shape) {
    SgLayout L;
    const int N = p->octaves * p->sublevels;
    const sg::Geo g = sg::make_geo(1, W, H, sg::kConvRows);
    const size_t nhwc = (size_t)g.sx;
    size_t off = 0;
    L.scratch = off;
    off = align256(off + scratch_layout(W, H, hist_bins(p), shape, 0).total);
    L.x0 = off;    off = align256(off + nhwc * 8 * sizeof(sg::bf16));
    L.xa = off;    off = align256(off + nhwc * 32 * sizeof(sg::bf16));
    L.xb = off;    off = align256(off + nhwc * 32 * sizeof(sg::bf16));
    L.delta = off; off = align256(off + (size_t)std::max(1, c->probes) * 2 * kProbeMax * kProbeMax * sizeof(float));
    L.tau = off;   off = align256(off + (size_t)N * sizeof(float));
    L.rects = off; off = align256(off + (size_t)N * std::max(1, c->probes) * sizeof(int4));
    L.max_items = sg_max_items(c);
    L.items = off; off = align256(off + (size_t)N * L.max_items * sizeof(int));
    L.total = off;
    return L;
}

kaze_status check_sg_config(const kaze_sg_config* c) {
    if (!c) return fail(KAZE_ERR_INVALID_ARG, "surrogate config is NULL");
    if (c->probes < 0 || c->probes > 16) return fail(KAZE_ERR_INVALID_ARG, "probes must be in [0, 16]");
    if (c->probe_size < 8 || c->probe_size > kProbeMax)
        return fail(KAZE_ERR_INVALID_ARG, "probe_size must be in [8, %d]", kProbeMax);
    if (isnan(c->bound)) return fail(KAZE_ERR_INVALID_ARG, "bound is NaN");
    if (c->aos_shape < -1 || c->aos_shape >= kAosShapes)
        return fail(KAZE_ERR_INVALID_ARG, "bad AOS tile shape");
    return KAZE_OK;
}

}  // namespace

struct kaze_sg_scale_space {
    int W = 0, H = 0, N = 0, shape = 0, probes = 0;
    float bound = 0.f;
    bool with_det = false, with_nms = false;
    kaze_params p;
    std::vector<Level> lv;
    BatchImage b;
    ImageDesc aos;  // scratch pointers of the AOS step; L, Lnext, gate set per level
    const unsigned char* packed = nullptr;
    sg::Geo geo, geo_probe;
    sg::bf16 *x0 = nullptr, *xa = nullptr, *xb = nullptr;
    float *delta = nullptr, *err = nullptr, *tau = nullptr;
    int4* rects = nullptr;
    int* items = nullptr;
    std::vector<int> item_off, item_cnt;
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
};

namespace {

// The six convolutions of one surrogate step L_i = L_{i-1} + f, over every
// strip of the image or over an item list; gated on *gate <= bound if gate.
kaze_status sg_chain(const kaze_sg_scale_space& S, const sg::Geo& geo, int i, const float* Lp,
                     float* Li, const int* items, int nitems, const float* gate, hipStream_t s) {
    const sg::PackLayout P = sg::pack_layout();
    if (!items) {  // whole image: three fused pairs of layers
        sg::bf16* buf[3] = {S.x0, S.xa, S.xb};
        for (int pr = 0; pr < 3; ++pr) {
            sg::Conv2Args c;
            memset(&c, 0, sizeof(c));
            const int la = 2 * pr, lb = la + 1;
            c.in = buf[pr];
            c.wa = reinterpret_cast<const sg::bf16x8*>(S.packed + P.fwd[la]);
            c.ba = reinterpret_cast<const float*>(S.packed + P.bias[la]);
            c.wb = reinterpret_cast<const sg::bf16x8*>(S.packed + P.fwd[lb]);
            c.bb = reinterpret_cast<const float*>(S.packed + P.bias[lb]);
            c.gate = gate;
            c.bound = S.bound;
            if (pr == 0) {
                c.tauw = reinterpret_cast<const float*>(S.packed + P.tauw);
                c.tau = S.tau + i;
            }
            if (pr < 2) {
                c.out = buf[pr + 1];
            } else {
                c.fout = Li;
                c.base = Lp;
            }
            KZ_LAUNCH(pr == 0 ? K_SG_CONV1 : (pr == 1 ? K_SG_CONV : K_SG_CONV6), s,
                      sg::launch_conv2(pr == 0 ? 8 : 32, pr < 2 ? 2 : 1, c, geo, s));
        }
        return KAZE_OK;
    }
    sg::bf16* buf[sg::kLayers] = {S.x0, S.xa, S.xb, S.xa, S.xb, S.xa};
    for (int l = 0; l < sg::kLayers; ++l) {
        sg::ConvArgs a;
        memset(&a, 0, sizeof(a));
        a.in = buf[l];
        a.wfrag = reinterpret_cast<const sg::bf16x8*>(S.packed + P.fwd[l]);
        a.bias = reinterpret_cast<const float*>(S.packed + P.bias[l]);
        a.items = items;
        a.nitems = nitems;
        a.gate = gate;
        a.bound = S.bound;
        if (l == 0) {
            a.tauw = reinterpret_cast<const float*>(S.packed + P.tauw);
            a.tau = S.tau + i;
        }
        if (l < sg::kLayers - 1) {
            a.out = buf[l + 1];
            KZ_LAUNCH(l == 0 ? K_SG_CONV1 : K_SG_CONV, s,
                      sg::launch_conv(l == 0 ? 8 : 32, 2, sg::EPI_RELU, l == 0, a, geo, s));
        } else {
            a.fout = Li;
            a.base = Lp;
            KZ_LAUNCH(K_SG_CONV6, s, sg::launch_conv(32, 1, sg::EPI_OUT, false, a, geo, s));
        }
    }
    return KAZE_OK;
}

kaze_status sg_segment(const kaze_sg_scale_space& S, int seg, hipStream_t s) {
    const kaze_params* p = &S.p;
    const ImgWork none{nullptr, nullptr, 0};
    if (seg == 0)
        return base_and_k(S.b, none, none, none, kAosShape[0].ty, none,
                          hist_chunk_for((double)S.b.W * S.b.H), p, s);
    if (seg == 2) {
        if (S.with_det)
            KZ_LAUNCH(K_DET, s,
                      launch_det(S.b, none, 0, S.N,
                                 det_levels(S.lv, det_band_for((double)S.b.W * S.b.H)), s));
        if (S.with_nms)
            KZ_LAUNCH(K_NMS, s,
                      launch_nms(S.b, none, S.N, (float)p->det_threshold, nms_radii(p), s));
        return KAZE_OK;
    }
    const Taps tc = gauss_taps(p->sigma_cond);
    const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;
    const size_t plane = (size_t)S.W * S.H;
    const AosWork anone{nullptr, nullptr, 0};
    KZ_LAUNCH(K_FILL, s, launch_fill_u32(reinterpret_cast<unsigned*>(S.err), S.N, 0u, s));
    for (int i = 1; i < S.N; ++i) {
        const float* Lp = S.b.levels + plane * (i - 1);
        float* Li = S.b.levels + plane * i;
        const float tau = (float)S.lv[i].tau;
        // conductivity of L_{i-1}: input of the surrogate and of the probe
        BatchImage bc = S.b;
        bc.levels = const_cast<float*>(Lp);
        KZ_LAUNCH(K_COND, s, launch_cond(bc, none, tc, 1.f, gmode, kAosShape[0].ty, s));
        KZ_LAUNCH(K_SG_PACK, s, sg::launch_pack_input(Lp, S.b.g, S.tau + i, S.x0, nullptr, S.geo, s));
        ImageDesc d = S.aos;
        d.L = Lp;
        d.Lnext = Li;
        if (S.probes > 0) {
            kaze_status st = sg_chain(S, S.geo_probe, i, Lp, Li, S.items + S.item_off[i], S.item_cnt[i],
                                     nullptr, s);
            if (st != KAZE_OK) return st;
            const int4* r = S.rects + (size_t)i * S.probes;
            KZ_LAUNCH(K_SG_PROBE, s, launch_aos_probe(d, r, S.probes, tau, S.delta, s));
            KZ_LAUNCH(K_SG_PROBE, s, launch_probe_err(Lp, Li, S.W, r, S.probes, S.delta,
                                                      reinterpret_cast<unsigned*>(S.err + i), s));
        }
        kaze_status st = sg_chain(S, S.geo, i, Lp, Li, nullptr, 0, S.err + i, s);
        if (st != KAZE_OK) return st;
        d.gate = S.err + i;
        d.bound = S.bound;
        st = aos_step(d, anone, anone, S.shape, tc, tau, true, gmode, 1.f, s);
        if (st != KAZE_OK) return st;
    }
    return KAZE_OK;
}

kaze_status sg_run(const kaze_sg_scale_space& S, bool eager, hipStream_t s) {
    for (int seg = 0; seg < 3; ++seg) {
        // with aos_reduce in the profiling list one event pair brackets the
        // level segment (all steps of the run)
        ProfScope ps(seg == 1 ? K_AOS_REDUCE : K_COUNT, s);
        if (eager) {
            const kaze_status st = sg_segment(S, seg, s);
            if (st != KAZE_OK) return st;
        } else {
            KZ_HIP(hipGraphLaunch(S.exec[seg], s));
        }
    }
    return KAZE_OK;
}

// ============================================================================
// Batched surrogate: the surrogate scale space over many images of uneven
// sizes.  Every phase of a level is one launch over all images (the batch's
// work lists and per-level tables); the probe check, the acceptance and the
// exact fallback are decided per image and level on the device.
// ============================================================================
struct SgBatch {
    float bound = 0.f;
    int probes = 0, np = 0;  // windows per image and level; per level (n x probes)
    const unsigned char* packed = nullptr;
    float* err = nullptr;    // caller's n x N probe errors
    sg::bf16 *x0 = nullptr, *xa = nullptr, *xb = nullptr;  // activations of all images
    float *delta = nullptr, *tau = nullptr;
    BatchImage* cond = nullptr;  // (N-1) x n: conductivity of L_{i-1}
    sg::SgImage* img = nullptr;  // (N-1) x n
    int2* full = nullptr;        // fused-pair items of every image
    int n_full = 0;
    int4* rects = nullptr;       // (N-1) x np probe windows
    int* rect_img = nullptr;     // (N-1) x np: image of each window
    int2* pitems = nullptr;      // conv items meeting the windows, per level
    std::vector<int> pitem_off, pitem_cnt;
};

struct SgBatchLayout {
    size_t x0, xa, xb, delta, tau, cond, img, full, rects, rect_img, pitems, total;
    long long px;  // padded pixels of all images
    int n_full, max_pitems;
};

SgBatchLayout sg_batch_layout(const kaze_image_desc* im, int n, const kaze_params* p,
                              const kaze_sg_config* c) {
    SgBatchLayout L;
    const int N = p->octaves * p->sublevels;
    L.px = 0;
    L.n_full = 0;
    for (int j = 0; j < n; ++j) {
        const sg::Geo g = sg::image_geo(im[j].W, im[j].H, sg::kConvRows);
        L.px += g.sx;
        L.n_full += ((im[j].W + sg::kPairOut - 1) / sg::kPairOut) * g.chunks;
    }
    const size_t np = (size_t)n * std::max(1, c->probes);
    const size_t lv = (size_t)std::max(1, N - 1);
    L.max_pitems = n * sg_max_items(c);
    size_t off = 0;
    L.x0 = off;       off = align256(off + (size_t)L.px * 8 * sizeof(sg::bf16));
    L.xa = off;       off = align256(off + (size_t)L.px * 32 * sizeof(sg::bf16));
    L.xb = off;       off = align256(off + (size_t)L.px * 32 * sizeof(sg::bf16));
    L.delta = off;    off = align256(off + np * 2 * kProbeMax * kProbeMax * sizeof(float));
    L.tau = off;      off = align256(off + (size_t)N * sizeof(float));
    L.cond = off;     off = align256(off + lv * n * sizeof(BatchImage));
    L.img = off;      off = align256(off + lv * n * sizeof(sg::SgImage));
    L.full = off;     off = align256(off + (size_t)L.n_full * sizeof(int2));
    L.rects = off;    off = align256(off + lv * np * sizeof(int4));
    L.rect_img = off; off = align256(off + lv * np * sizeof(int));
    L.pitems = off;   off = align256(off + lv * L.max_pitems * sizeof(int2));
    L.total = off;
    return L;
}

size_t sg_batch_bytes(const kaze_image_desc* im, int n, const kaze_params* p,
                      const kaze_sg_config* c) {
    return sg_batch_layout(im, n, p, c).total;
}

kaze_status sg_batch_check(const kaze_image_desc* im, int n, const kaze_params* p,
                           const SgSpec& sp) {
    kaze_status st = check_sg_config(sp.c);
    if (st != KAZE_OK) return st;
    if (p->substeps != 1)
        return fail(KAZE_ERR_UNSUPPORTED, "the surrogate replaces whole level steps (substeps 1)");
    if (n > kSgBatchMaxImages)
        return fail(KAZE_ERR_UNSUPPORTED, "a surrogate batch holds at most %d images (got %d)",
                    kSgBatchMaxImages, n);
    if (!sp.packed || !aligned(sp.packed, 256))
        return fail(KAZE_ERR_INVALID_ARG, "packed weights must be non-NULL and 256-byte aligned");
    if (!sp.err || !aligned(sp.err, 4)) return fail(KAZE_ERR_INVALID_ARG, "err must be non-NULL");
    const int N = p->octaves * p->sublevels, P = sp.c->probes;
    if (P > 0) {
        if (!sp.probe_xy) return fail(KAZE_ERR_INVALID_ARG, "probe_xy is NULL with probes > 0");
        for (int j = 0; j < n; ++j)
            for (int i = 1; i < N; ++i)
                for (int q = 0; q < P; ++q) {
                    const int* xy = sp.probe_xy + (((size_t)j * N + i) * P + q) * 2;
                    if (xy[0] < 0 || xy[0] >= im[j].W || xy[1] < 0 || xy[1] >= im[j].H)
                        return fail(KAZE_ERR_INVALID_ARG,
                                    "probe (%d, %d) of image %d, level %d outside the image", xy[0],
                                    xy[1], j, i);
                }
    }
    return KAZE_OK;
}

kaze_status sg_batch_build(kaze_batch* B, const kaze_image_desc* im, const SgSpec& sp,
                           char* base, size_t off, const std::vector<size_t>& scratch) {
    const kaze_sg_config* c = sp.c;
    const int n = B->n, N = B->N, P = c->probes;
    const SgBatchLayout L = sg_batch_layout(im, n, &B->p, c);
    if (off % 256) return fail(KAZE_ERR_WORKSPACE, "surrogate tables misaligned");
    SgBatch* G = new SgBatch();
    B->sg = G;  // released with the plan
    char* sb = base + off;
    G->bound = (float)c->bound;
    G->probes = P;
    G->np = n * P;
    G->packed = static_cast<const unsigned char*>(sp.packed);
    G->err = sp.err;
    G->x0 = reinterpret_cast<sg::bf16*>(sb + L.x0);
    G->xa = reinterpret_cast<sg::bf16*>(sb + L.xa);
    G->xb = reinterpret_cast<sg::bf16*>(sb + L.xb);
    G->delta = reinterpret_cast<float*>(sb + L.delta);
    G->tau = reinterpret_cast<float*>(sb + L.tau);
    G->cond = reinterpret_cast<BatchImage*>(sb + L.cond);
    G->img = reinterpret_cast<sg::SgImage*>(sb + L.img);
    G->full = reinterpret_cast<int2*>(sb + L.full);
    G->n_full = L.n_full;
    G->rects = reinterpret_cast<int4*>(sb + L.rects);
    G->rect_img = reinterpret_cast<int*>(sb + L.rect_img);
    G->pitems = reinterpret_cast<int2*>(sb + L.pitems);
    G->pitem_off.assign(N, 0);
    G->pitem_cnt.assign(N, 0);

    // host image of the tables [tau, total)
    const size_t tb = L.tau;
    std::vector<char> host(L.total - tb, 0);
    auto at = [&](size_t o) { return host.data() + (o - tb); };
    float* htau = reinterpret_cast<float*>(at(L.tau));
    BatchImage* hcond = reinterpret_cast<BatchImage*>(at(L.cond));
    sg::SgImage* himg = reinterpret_cast<sg::SgImage*>(at(L.img));
    int2* hfull = reinterpret_cast<int2*>(at(L.full));
    int4* hrect = reinterpret_cast<int4*>(at(L.rects));
    int* hrimg = reinterpret_cast<int*>(at(L.rect_img));
    int2* hpit = reinterpret_cast<int2*>(at(L.pitems));
    std::vector<long long> xoff(n);
    std::vector<float*> gplane(n);
    long long xo = 0;
    int f = 0;
    const int nb = hist_bins(&B->p);
    for (int j = 0; j < n; ++j) {
        xoff[j] = xo;
        const sg::Geo g = sg::image_geo(im[j].W, im[j].H, sg::kConvRows);
        xo += g.sx;
        const int strips = (im[j].W + sg::kPairOut - 1) / sg::kPairOut;
        for (int t = 0; t < strips * g.chunks; ++t) hfull[f++] = make_int2(j, t);
        // the conductivity plane of the image's scratch, as batch_create lays it out
        const Scratch sc = scratch_layout(im[j].W, im[j].H, nb, B->shape, scratch[j], false,
                                          false, B->with_nms ? N : 0);
        gplane[j] = reinterpret_cast<float*>(base + sc.g);
    }
    std::vector<int> tmp;
    std::vector<int4> rj(std::max(1, P));
    for (int i = 1; i < N; ++i) {
        htau[i] = (float)B->lv[i].tau;
        const size_t r0 = (size_t)(i - 1) * n;
        int cnt = 0;
        for (int j = 0; j < n; ++j) {
            const int W = im[j].W, H = im[j].H;
            const size_t plane = (size_t)W * H;
            BatchImage b = batch_image(W, H);
            b.levels = im[j].levels + plane * (i - 1);
            b.g = gplane[j];
            b.k = im[j].k;
            hcond[r0 + j] = b;
            sg::SgImage si;
            si.xoff = xoff[j];
            si.L = im[j].levels + plane * (i - 1);
            si.Lnext = im[j].levels + plane * i;
            si.g = gplane[j];
            si.gate = sp.err + (size_t)j * N + i;
            si.W = W;
            si.H = H;
            himg[r0 + j] = si;
            for (int q = 0; q < P; ++q) {
                const int* xy = sp.probe_xy + (((size_t)j * N + i) * P + q) * 2;
                rj[q] = make_int4(xy[0], xy[1], std::min(c->probe_size, W - xy[0]),
                                  std::min(c->probe_size, H - xy[1]));
                hrect[(size_t)(i - 1) * G->np + (size_t)j * P + q] = rj[q];
                hrimg[(size_t)(i - 1) * G->np + (size_t)j * P + q] = j;
            }
            if (P > 0) {
                sg_probe_items(sg::image_geo(W, H, kProbeRows), rj.data(), P, tmp);
                if (cnt + (int)tmp.size() > L.max_pitems)
                    return fail(KAZE_ERR_UNSUPPORTED, "probe windows need more than %d items",
                                L.max_pitems);
                for (int v : tmp) hpit[(size_t)(i - 1) * L.max_pitems + cnt++] = make_int2(j, v);
            }
        }
        G->pitem_off[i] = (i - 1) * L.max_pitems;
        G->pitem_cnt[i] = cnt;
    }
    hipError_t e = hipMemset(sb + L.x0, 0, L.delta - L.x0);  // zero rings of the activations
    if (e == hipSuccess)
        e = hipMemcpy(sb + tb, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return fail(KAZE_ERR_HIP, "surrogate batch tables: %s", hipGetErrorString(e));
    return KAZE_OK;
}

// The six convolutions of level i over a batched work list: layer by layer
// (probe items, rows of kProbeRows) or as three fused pairs (every image);
// with gate non-NULL each image runs only where its probe error is <= bound.
kaze_status sg_batch_chain(const SgBatch& G, int i, const sg::SgWork& w, bool fused,
                           const float* gate, hipStream_t s) {
    const sg::PackLayout P = sg::pack_layout();
    sg::Geo geo;
    memset(&geo, 0, sizeof(geo));
    if (fused) {
        geo.R = sg::kConvRows;
        sg::bf16* buf[3] = {G.x0, G.xa, G.xb};
        for (int pr = 0; pr < 3; ++pr) {
            sg::Conv2Args c;
            memset(&c, 0, sizeof(c));
            const int la = 2 * pr, lb = la + 1;
            c.in = buf[pr];
            c.wa = reinterpret_cast<const sg::bf16x8*>(G.packed + P.fwd[la]);
            c.ba = reinterpret_cast<const float*>(G.packed + P.bias[la]);
            c.wb = reinterpret_cast<const sg::bf16x8*>(G.packed + P.fwd[lb]);
            c.bb = reinterpret_cast<const float*>(G.packed + P.bias[lb]);
            c.gate = gate;
            c.bound = G.bound;
            c.bw = w;
            if (pr == 0) {
                c.tauw = reinterpret_cast<const float*>(G.packed + P.tauw);
                c.tau = G.tau + i;
            }
            if (pr < 2) c.out = buf[pr + 1];  // fout and base come from the image table
            KZ_LAUNCH(pr == 0 ? K_SG_CONV1 : (pr == 1 ? K_SG_CONV : K_SG_CONV6), s,
                      sg::launch_conv2(pr == 0 ? 8 : 32, pr < 2 ? 2 : 1, c, geo, s));
        }
        return KAZE_OK;
    }
    geo.R = kProbeRows;
    sg::bf16* buf[sg::kLayers] = {G.x0, G.xa, G.xb, G.xa, G.xb, G.xa};
    for (int l = 0; l < sg::kLayers; ++l) {
        sg::ConvArgs a;
        memset(&a, 0, sizeof(a));
        a.in = buf[l];
        a.wfrag = reinterpret_cast<const sg::bf16x8*>(G.packed + P.fwd[l]);
        a.bias = reinterpret_cast<const float*>(G.packed + P.bias[l]);
        a.gate = gate;
        a.bound = G.bound;
        a.bw = w;
        if (l == 0) {
            a.tauw = reinterpret_cast<const float*>(G.packed + P.tauw);
            a.tau = G.tau + i;
        }
        if (l < sg::kLayers - 1) {
            a.out = buf[l + 1];
            KZ_LAUNCH(l == 0 ? K_SG_CONV1 : K_SG_CONV, s,
                      sg::launch_conv(l == 0 ? 8 : 32, 2, sg::EPI_RELU, l == 0, a, geo, s));
        } else {
            KZ_LAUNCH(K_SG_CONV6, s, sg::launch_conv(32, 1, sg::EPI_OUT, false, a, geo, s));
        }
    }
    return KAZE_OK;
}

// The N-1 level steps of a surrogate batch: per level the conductivity, the
// network input, the network on the probe windows and the exact solves
// there, then the network on every accepted image and AOS on every rejected
// one (the per-level descriptors carry the image's error word as gate).
kaze_status sg_batch_levels(const kaze_batch& B, hipStream_t s) {
    const SgBatch& G = *B.sg;
    const kaze_params* p = &B.p;
    const int n = B.n, N = B.N;
    const Taps tc = gauss_taps(p->sigma_cond);
    const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;
    const BatchImage b0 = batch_image(0, 0);
    ImageDesc a0;
    memset(&a0, 0, sizeof(a0));
    KZ_LAUNCH(K_FILL, s, launch_fill_u32(reinterpret_cast<unsigned*>(G.err), n * N, 0u, s));
    for (int i = 1; i < N; ++i) {
        const size_t r0 = (size_t)(i - 1) * n;
        const float tau = (float)B.lv[i].tau;
        const ImgWork ct{G.cond + r0, B.d_aos, B.n_aos};
        KZ_LAUNCH(K_COND, s, launch_cond(b0, ct, tc, 1.f, gmode, kAosShape[B.shape].ty, s));
        const sg::SgImage* si = G.img + r0;
        KZ_LAUNCH(K_SG_PACK, s, sg::launch_pack_input_batch(si, n, G.x0, s));
        const ImageDesc* lvl = B.d_lvl + r0;  // one step per level
        kaze_status st;
        if (G.probes > 0) {
            const sg::SgWork pw{si, G.pitems + G.pitem_off[i], G.pitem_cnt[i]};
            if ((st = sg_batch_chain(G, i, pw, false, nullptr, s)) != KAZE_OK) return st;
            const int4* r = G.rects + (size_t)(i - 1) * G.np;
            const int* ri = G.rect_img + (size_t)(i - 1) * G.np;
            KZ_LAUNCH(K_SG_PROBE, s, launch_aos_probe(a0, r, G.np, tau, G.delta, s, lvl, ri));
            KZ_LAUNCH(K_SG_PROBE, s,
                      launch_probe_err(nullptr, nullptr, 0, r, G.np, G.delta, nullptr, s, lvl, ri));
        }
        const sg::SgWork fw{si, G.full, G.n_full};
        if ((st = sg_batch_chain(G, i, fw, true, G.err, s)) != KAZE_OK) return st;
        const AosWork at{lvl, B.d_aos, B.n_aos};
        const AosWork al{lvl, B.d_lines, B.n_lines};
        // g of L_{i-1} is already in every image's plane: the step reads it
        st = aos_step(a0, at, al, B.shape, tc, tau, false, gmode, 1.f, s);
        if (st != KAZE_OK) return st;
    }
    return KAZE_OK;
}

// Argument checks of the single-image scale space; *need = scratch bytes.
kaze_status check_scale_space_args(const float* img, int W, int H, int ld_img,
                                   const kaze_params* p, const float* levels, const float* k_out,
                                   size_t* need) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if (!img || !levels || !k_out)
        return fail(KAZE_ERR_INVALID_ARG, "img, levels and k_out must be non-NULL");
    if (ld_img < W) return fail(KAZE_ERR_INVALID_ARG, "ld_img (%d) < W (%d)", ld_img, W);
    if (!aligned(img, 4) || !aligned(levels, 4) || !aligned(k_out, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    *need = scratch_layout(W, H, hist_bins(p), default_shape(W, H), 0, p->scheme == KAZE_FED,
                           p->substeps > 1).total;
    return KAZE_OK;
}

// a1-a5 for one image with its scratch at base (scratch_layout, validated).
kaze_status scale_space_launches(const float* img, int W, int H, int ld_img,
                                 const kaze_params* p, float* levels, float* k_out, char* base,
                                 hipStream_t s) {
    const bool fed = p->scheme == KAZE_FED;
    const int m = p->substeps;
    const int shape = default_shape(W, H);
    const Scratch w = scratch_layout(W, H, hist_bins(p), shape, 0, fed, m > 1);
    BatchImage b = batch_image(W, H);
    b.img = img;
    b.ld = ld_img;
    b.levels = levels;
    b.g = reinterpret_cast<float*>(base + w.g);
    b.hist = reinterpret_cast<unsigned*>(base + w.hist);
    b.hmax = reinterpret_cast<unsigned*>(base + w.hmax);
    b.k = k_out;
    const ImgWork none{nullptr, nullptr, 0};
    kaze_status st = base_and_k(b, none, none, none, kAosShape[shape].ty, none,
                                hist_chunk_for((double)W * H), p, s);
    if (st != KAZE_OK) return st;

    std::vector<Level> lv;
    schedule(p, lv);
    const size_t plane = (size_t)W * H;
    const Taps tc = gauss_taps(p->sigma_cond);
    const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;
    ImageDesc d = aos_desc(W, H, shape, base, w, k_out);
    const AosWork anone{nullptr, nullptr, 0};
    float* mid = reinterpret_cast<float*>(base + w.sub);
    for (size_t i = 1; i < lv.size(); ++i) {
        // m sub-steps from level i-1 to level i, alternating between the
        // level's plane and the sub-step plane so that the last one writes
        // the level
        const double tau = lv[i].tau / m;
        const float* src = levels + plane * (i - 1);
        float* out = levels + plane * i;
        for (int q = 0; q < m; ++q) {
            float* dst = ((m - 1 - q) % 2 == 0) ? out : mid;
            d.L = src;
            d.Lnext = dst;
            if (fed) {
                BatchImage bc = b;
                bc.levels = const_cast<float*>(src);  // conductivity of the step's start
                KZ_LAUNCH(K_COND, s, launch_cond(bc, none, tc, 1.f, gmode, kAosShape[shape].ty, s));
                st = fed_cycle(src, b.g, dst, reinterpret_cast<float*>(base + w.tmp), W, H, tau, s);
            } else {
                st = aos_step(d, anone, anone, shape, tc, (float)tau, true, gmode, 1.f, s);
            }
            if (st != KAZE_OK) return st;
            src = dst;
        }
    }
    return KAZE_OK;
}

// ------------------------------------------------- device-resident scratch
// Scratch of kaze_build_scale_space_noalloc: one copy per GPU, allocated
// with the library's code object and held until the process ends.  Host
// code never passes `scratch` itself (on the host it names a stand-in, not
// device memory); it uses the address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kNoAllocScratchBytes = (size_t)KAZE_NOALLOC_SCRATCH_BYTES;
}  // namespace

static __device__ __align__(256) unsigned char scratch[KAZE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch, resolved once per device.
kaze_status noalloc_scratch(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(KAZE_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(KAZE_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(KAZE_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        if (!aligned(ptr, 256))
            return fail(KAZE_ERR_HIP, "device scratch at %p is not 256-byte aligned", ptr);
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
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
    p->k_bins = 300;
    p->k_percentile = 0.7;
    p->k_override = 0.0;
    p->det_threshold = 0.001;
    p->scheme = KAZE_AOS;
    p->extrema_window = KAZE_WINDOW_3X3;
    p->substeps = 1;
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
    return scratch_layout(W, H, hist_bins(p), default_shape(W, H), 0, p->scheme == KAZE_FED,
                          p->substeps > 1)
        .total;
}

kaze_status kaze_build_scale_space(const float* img, int W, int H, int ld_img,
                                   const kaze_params* p, float* levels, float* k_out, void* ws,
                                   size_t ws_bytes, void* stream) {
    size_t need = 0;
    kaze_status st = check_scale_space_args(img, W, H, ld_img, p, levels, k_out, &need);
    if (st != KAZE_OK) return st;
    if (!ws || !aligned(ws, 256) || ws_bytes < need)
        return fail(KAZE_ERR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    need, ws_bytes);
    return scale_space_launches(img, W, H, ld_img, p, levels, k_out, static_cast<char*>(ws),
                                static_cast<hipStream_t>(stream));
}

kaze_status kaze_build_scale_space_noalloc(const float* img, int W, int H, int ld_img,
                                           const kaze_params* p, float* levels, float* k_out,
                                           void* stream) {
    size_t need = 0;
    kaze_status st = check_scale_space_args(img, W, H, ld_img, p, levels, k_out, &need);
    if (st != KAZE_OK) return st;
    if (need > kNoAllocScratchBytes)
        return fail(KAZE_ERR_UNSUPPORTED,
                    "a %dx%d scale space with these parameters needs %zu scratch bytes; the "
                    "device-resident scratch holds %zu",
                    W, H, need, kNoAllocScratchBytes);
    char* base = nullptr;
    if ((st = noalloc_scratch(&base)) != KAZE_OK) return st;
    return scale_space_launches(img, W, H, ld_img, p, levels, k_out, base,
                                static_cast<hipStream_t>(stream));
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
    BatchImage b = batch_image(W, H);
    b.levels = const_cast<float*>(L);  // read only
    b.g = g;
    const int gmode = p->diffusivity == KAZE_G2 ? 0 : 1;
    const ImgWork none{nullptr, nullptr, 0};
    KZ_LAUNCH(K_COND, s,
              launch_cond(b, none, gauss_taps(p->sigma_cond), (float)k, gmode, kAosShape[0].ty, s));
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
    const int shape = default_shape(W, H);
    const Scratch w = scratch_layout(W, H, hist_bins(&p), shape, 0);
    if (!ws || !aligned(ws, 256) || ws_bytes < w.total)
        return fail(KAZE_ERR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    w.total, ws_bytes);
    ImageDesc d = aos_desc(W, H, shape, static_cast<char*>(ws), w, nullptr);
    d.L = L;
    d.Lnext = L_next;
    d.g = const_cast<float*>(g);  // read only when the conductivity is given
    const AosWork anone{nullptr, nullptr, 0};
    return aos_step(d, anone, anone, shape, gauss_taps(p.sigma_cond), (float)tau, false, 0, 1.f,
                    static_cast<hipStream_t>(stream));
}

static_assert(sizeof(kaze_keypoint) == 16 && sizeof(kaze_keypoint_refined) == 24 &&
                  sizeof(RefinedKeypoint) == sizeof(kaze_keypoint_refined),
              "keypoint records as the kernels read and write them");

kaze_status kaze_refine_keypoints(const float* det, int W, int H, const kaze_params* p,
                                  const kaze_keypoint* kps, const int* count, int capacity,
                                  double edge_ratio, kaze_keypoint_refined* out, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if (capacity < 0) return fail(KAZE_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && (!det || !kps || !count || !out))
        return fail(KAZE_ERR_INVALID_ARG, "det, kps, count and out must be non-NULL");
    if (!aligned(det, 4) || !aligned(kps, 4) || !aligned(count, 4) || !aligned(out, 4))
        return fail(KAZE_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
    if (!(edge_ratio > 1.0) || !isfinite(edge_ratio))
        return fail(KAZE_ERR_INVALID_ARG, "edge_ratio must be > 1");
    const float thr = (float)((edge_ratio + 1.0) * (edge_ratio + 1.0) / edge_ratio);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = kaze_num_levels(p);
    KZ_LAUNCH(K_REFINE, s, launch_refine(det, W, H, N, kps, count, capacity, thr, out, s));
    return KAZE_OK;
}

static DescLevels desc_levels(const kaze_params* p) {
    std::vector<Level> lv;
    schedule(p, lv);
    DescLevels dl;
    memset(&dl, 0, sizeof(dl));
    for (size_t i = 0; i < lv.size(); ++i) {
        dl.step[i] = lv[i].step;
        dl.sn[i] = (float)lv[i].sigma_n;
        dl.sigma[i] = (float)lv[i].sigma;
    }
    return dl;
}

kaze_status kaze_derivatives(const float* levels, int W, int H, const kaze_params* p, float* lx,
                             float* ly, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if ((st = check_steps(p)) != KAZE_OK) return st;
    if (!levels || !lx || !ly) return fail(KAZE_ERR_INVALID_ARG, "levels, lx and ly must be non-NULL");
    if (!aligned(levels, 4) || !aligned(lx, 4) || !aligned(ly, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<Level> lv;
    schedule(p, lv);
    const DetLevels dl = det_levels(lv, det_band_for((double)W * H));
    const int N = (int)lv.size();
    bool rows = true;
    for (int i = 0; i < N; ++i) rows = rows && lv[i].step <= 4;
    if (rows) {
        BatchImage b = batch_image(W, H);
        b.levels = const_cast<float*>(levels);  // read only
        KZ_LAUNCH(K_DERIV, s, launch_det_derivs(b, N, dl, lx, ly, s));
    } else {
        KZ_LAUNCH(K_DERIV, s, launch_deriv(levels, W, H, N, desc_levels(p), lx, ly, s));
    }
    return KAZE_OK;
}

kaze_status kaze_describe_keypoints(const float* lx, const float* ly, int W, int H,
                                    const kaze_params* p, const kaze_keypoint_refined* kps,
                                    const int* count, int capacity, float* angles,
                                    float* descriptors, void* stream) {
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    if (capacity < 0) return fail(KAZE_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && (!lx || !ly || !kps || !count || !angles || !descriptors))
        return fail(KAZE_ERR_INVALID_ARG, "lx, ly, kps, count, angles and descriptors must be non-NULL");
    if (!aligned(lx, 4) || !aligned(ly, 4) || !aligned(kps, 4) || !aligned(count, 4) ||
        !aligned(angles, 4) || !aligned(descriptors, 4))
        return fail(KAZE_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KZ_LAUNCH(K_DESCRIBE, s,
              launch_describe(lx, ly, W, H, kaze_num_levels(p), desc_levels(p), kps, count,
                              capacity, angles, descriptors, s));
    return KAZE_OK;
}

int kaze_fed_schedule(double T, double* tau, int capacity) {
    if (!(T > 0.0) || !isfinite(T)) return fail(KAZE_ERR_INVALID_ARG, "T must be > 0 and finite");
    const std::vector<double> t = fed_schedule(T);
    const int n = (int)t.size();
    if (tau && capacity >= n)
        for (int i = 0; i < n; ++i) tau[i] = t[i];
    return n;
}

kaze_status kaze_fed_cycle(const float* L, const float* g, int W, int H, double T, float* L_next,
                           void* ws, size_t ws_bytes, void* stream) {
    kaze_status st = check_size(W, H);
    if (st != KAZE_OK) return st;
    if (!L || !g || !L_next) return fail(KAZE_ERR_INVALID_ARG, "L, g and L_next must be non-NULL");
    if (!aligned(L, 4) || !aligned(g, 4) || !aligned(L_next, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    if (!(T > 0.0) || !isfinite(T)) return fail(KAZE_ERR_INVALID_ARG, "T must be > 0");
    kaze_params p;
    kaze_default_params(&p);
    p.scheme = KAZE_FED;
    const Scratch w = scratch_layout(W, H, hist_bins(&p), 0, 0, true);
    if (!ws || !aligned(ws, 256) || ws_bytes < w.total)
        return fail(KAZE_ERR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    w.total, ws_bytes);
    float* tmp = reinterpret_cast<float*>(static_cast<char*>(ws) + w.tmp);
    return fed_cycle(L, g, L_next, tmp, W, H, T, static_cast<hipStream_t>(stream));
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
    BatchImage b = batch_image(W, H);
    b.levels = const_cast<float*>(levels);  // read only
    b.det = det;
    const ImgWork none{nullptr, nullptr, 0};
    hipStream_t s = static_cast<hipStream_t>(stream);
    KZ_LAUNCH(K_DET, s,
              launch_det(b, none, 0, (int)lv.size(), det_levels(lv, det_band_for((double)W * H)),
                         s));
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
    BatchImage b = batch_image(W, H);
    b.det = const_cast<float*>(det);  // read only
    b.kps = kps;
    b.capacity = capacity;
    b.count = count;
    const ImgWork none{nullptr, nullptr, 0};
    KZ_LAUNCH(K_FILL, s, launch_reset(b, none, 0, 0.f, s));
    KZ_LAUNCH(K_NMS, s, launch_nms(b, none, p->octaves * p->sublevels, (float)p->det_threshold,
                                   nms_radii(p), s));
    return KAZE_OK;
}

// ---------------------------------------------------------------- batches
kaze_status kaze_aos_shape_info(int shape, int* tile_w, int* tile_h, int* row_chunk,
                                int* col_chunk, int* iface_m, int* chunk_lanes_out) {
    if (shape < 0 || shape >= kAosShapes)
        return fail(KAZE_ERR_INVALID_ARG, "AOS shape %d outside [0, %d)", shape, kAosShapes);
    const AosShape& a = kAosShape[shape];
    if (tile_w) *tile_w = kAosTX;
    if (tile_h) *tile_h = a.ty;
    if (row_chunk) *row_chunk = a.rc;
    if (col_chunk) *col_chunk = a.cc;
    if (iface_m) *iface_m = a.m;
    if (chunk_lanes_out) *chunk_lanes_out = chunk_lanes(a.ty, a.rc, a.cc);
    return KAZE_OK;
}

size_t kaze_batch_workspace_bytes(const kaze_image_desc* images, int n, const kaze_params* p,
                                  const kaze_batch_config* cfg) {
    if (check_params(p) != KAZE_OK || p->scheme != KAZE_AOS || !images || n < 1) return 0;
    size_t best = 0;
    for (int sh = 0; sh < kAosShapes; ++sh) {
        if (cfg && cfg->aos_shape >= 0 && cfg->aos_shape != sh) continue;
        bool fits = true;
        for (int j = 0; j < n; ++j)
            fits = fits && check_size(images[j].W, images[j].H) == KAZE_OK &&
                   shape_fits(images[j].W, images[j].H, sh);
        if (fits) best = std::max(best, batch_layout(images, n, p, sh).total);
    }
    return best;
}

kaze_status kaze_batch_create(const kaze_image_desc* images, int n, const kaze_params* p,
                              const kaze_batch_config* cfg, void* ws, size_t ws_bytes,
                              kaze_batch** out) {
    const int shape = cfg && cfg->aos_shape >= 0 ? cfg->aos_shape : default_batch_shape(images, n);
    return batch_create(images, n, p, shape, ws, ws_bytes, out);
}

kaze_status kaze_batch_properties(const kaze_batch* b, int* aos_shape, int* det_levels_in_segment) {
    if (!b) return fail(KAZE_ERR_INVALID_ARG, "batch is NULL");
    if (aos_shape) *aos_shape = b->shape;
    if (det_levels_in_segment)
        *det_levels_in_segment = b->fork_det ? b->N : 0;
    return KAZE_OK;
}

kaze_status kaze_batch_run(kaze_batch* b, int eager, void* stream) {
    if (!b) return fail(KAZE_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (eager) return enqueue_batch(*b, s);
    return run_graphs(*b, s);
}

kaze_status kaze_batch_destroy(kaze_batch* b) {
    if (!b) return KAZE_OK;
    for (hipGraphExec_t& x : b->exec)
        if (x) (void)hipGraphExecDestroy(x);
    for (hipEvent_t ev : b->ev) (void)hipEventDestroy(ev);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b->sg;
    delete b;
    return KAZE_OK;
}

kaze_status kaze_batch_autotune(const kaze_image_desc* images, int n, const kaze_params* p,
                                void* ws, size_t ws_bytes, int reps, void* stream,
                                kaze_batch_config* best, double* ms_per_shape) {
    if (!best) return fail(KAZE_ERR_INVALID_ARG, "best is NULL");
    if (reps < 1) return fail(KAZE_ERR_INVALID_ARG, "reps must be >= 1");
    if (!images || n < 1) return fail(KAZE_ERR_INVALID_ARG, "a batch needs at least one image");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double best_ms = -1.0;
    int best_shape = -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KZ_HIP(hipEventCreate(&e0));
    KZ_HIP(hipEventCreate(&e1));
    kaze_status result = KAZE_OK;
    for (int sh = 0; sh < kAosShapes; ++sh) {
        if (ms_per_shape) ms_per_shape[sh] = -1.0;
        bool fits = true;
        for (int j = 0; j < n; ++j) fits = fits && shape_fits(images[j].W, images[j].H, sh);
        if (!fits) continue;
        kaze_batch* b = nullptr;
        kaze_status st = batch_create(images, n, p, sh, ws, ws_bytes, &b);
        if (st != KAZE_OK) {
            result = st;
            break;
        }
        hipError_t e = run_graphs(*b, s) == KAZE_OK ? hipSuccess : hipErrorUnknown;  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = run_graphs(*b, s) == KAZE_OK ? hipSuccess : hipErrorUnknown;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        kaze_batch_destroy(b);
        if (e != hipSuccess) {
            result = fail(KAZE_ERR_HIP, "autotune timing failed: %s", hipGetErrorString(e));
            break;
        }
        const double per = (double)ms / reps;
        if (ms_per_shape) ms_per_shape[sh] = per;
        if (best_shape < 0 || per < best_ms) {
            best_ms = per;
            best_shape = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != KAZE_OK) return result;
    if (best_shape < 0) return fail(KAZE_ERR_UNSUPPORTED, "no AOS tile shape fits the batch");
    best->aos_shape = best_shape;
    return KAZE_OK;
}

// ------------------------------------------------------ surrogate scale space
kaze_status kaze_sg_default_config(kaze_sg_config* c) {
    if (!c) return fail(KAZE_ERR_INVALID_ARG, "config pointer is NULL");
    c->bound = 6.6e-5;  // 15 steps x 6.6e-5 <= 1e-3
    c->probes = 4;
    c->probe_size = 32;
    c->aos_shape = -1;
    return KAZE_OK;
}

size_t kaze_sg_scale_space_workspace_bytes(int W, int H, const kaze_params* p,
                                           const kaze_sg_config* c) {
    if (check_params(p) != KAZE_OK || p->scheme != KAZE_AOS || p->substeps != 1 ||
        check_sg_config(c) != KAZE_OK || check_size(W, H) != KAZE_OK)
        return 0;
    const int shape = c->aos_shape >= 0 ? c->aos_shape : default_shape(W, H);
    if (!shape_fits(W, H, shape)) return 0;
    return sg_layout(W, H, p, c, shape).total;
}

kaze_status kaze_sg_scale_space_destroy(kaze_sg_scale_space* S) {
    if (!S) return KAZE_OK;
    for (hipGraphExec_t& x : S->exec)
        if (x) (void)hipGraphExecDestroy(x);
    delete S;
    return KAZE_OK;
}

size_t kaze_sg_batch_workspace_bytes(const kaze_image_desc* images, int n, const kaze_params* p,
                                     const kaze_sg_config* c) {
    if (check_sg_config(c) != KAZE_OK) return 0;
    const int shape = c->aos_shape >= 0 ? c->aos_shape : default_batch_shape(images, n);
    if (check_batch(images, n, p, shape) != KAZE_OK) return 0;
    return batch_layout(images, n, p, shape).total + sg_batch_bytes(images, n, p, c);
}

kaze_status kaze_sg_batch_create(const kaze_image_desc* images, int n, const kaze_params* p,
                                 const kaze_sg_config* c, const void* packed, const int* probe_xy,
                                 float* err, void* ws, size_t ws_bytes, kaze_batch** out) {
    if (out) *out = nullptr;
    const kaze_status st = check_sg_config(c);
    if (st != KAZE_OK) return st;
    const SgSpec sp{c, packed, probe_xy, err};
    const int shape = c->aos_shape >= 0 ? c->aos_shape : default_batch_shape(images, n);
    return batch_create(images, n, p, shape, ws, ws_bytes, out, &sp);
}

kaze_status kaze_sg_scale_space_create(const kaze_image_desc* im, const kaze_params* p,
                                       const kaze_sg_config* c, const void* packed,
                                       const int* probe_xy, float* err, void* ws,
                                       size_t ws_bytes, kaze_sg_scale_space** out) {
    if (!out) return fail(KAZE_ERR_INVALID_ARG, "out pointer is NULL");
    *out = nullptr;
    kaze_status st = check_params(p);
    if (st != KAZE_OK) return st;
    if (p->scheme != KAZE_AOS)
        return fail(KAZE_ERR_UNSUPPORTED, "the surrogate falls back to AOS steps only");
    if (p->substeps != 1)
        return fail(KAZE_ERR_UNSUPPORTED, "the surrogate replaces whole level steps (substeps 1)");
    if ((st = check_steps(p)) != KAZE_OK) return st;
    if ((st = check_sg_config(c)) != KAZE_OK) return st;
    if (!im) return fail(KAZE_ERR_INVALID_ARG, "image descriptor is NULL");
    const int W = im->W, H = im->H;
    if ((st = check_size(W, H)) != KAZE_OK) return st;
    const int shape = c->aos_shape >= 0 ? c->aos_shape : default_shape(W, H);
    if (!shape_fits(W, H, shape))
        return fail(KAZE_ERR_UNSUPPORTED, "image does not fit AOS tile shape %d", shape);
    if (!im->img || !im->levels || !im->k)
        return fail(KAZE_ERR_INVALID_ARG, "img, levels and k must be non-NULL");
    if (im->ld_img < W) return fail(KAZE_ERR_INVALID_ARG, "ld_img < W");
    if (im->count && !im->det) return fail(KAZE_ERR_INVALID_ARG, "extrema need det");
    if (im->capacity < 0 || (im->capacity > 0 && !im->kps))
        return fail(KAZE_ERR_INVALID_ARG, "bad keypoint buffer");
    if (!packed || !aligned(packed, 256))
        return fail(KAZE_ERR_INVALID_ARG, "packed weights must be non-NULL and 256-byte aligned");
    if (!err || !aligned(err, 4)) return fail(KAZE_ERR_INVALID_ARG, "err must be non-NULL");
    if (!aligned(im->img, 4) || !aligned(im->levels, 4) || !aligned(im->k, 4))
        return fail(KAZE_ERR_INVALID_ARG, "float buffers must be 4-byte aligned");
    const int N = p->octaves * p->sublevels;
    if (c->probes > 0) {
        if (!probe_xy) return fail(KAZE_ERR_INVALID_ARG, "probe_xy is NULL with probes > 0");
        for (int i = 1; i < N; ++i)
            for (int q = 0; q < c->probes; ++q) {
                const int x0 = probe_xy[((size_t)i * c->probes + q) * 2];
                const int y0 = probe_xy[((size_t)i * c->probes + q) * 2 + 1];
                if (x0 < 0 || x0 >= W || y0 < 0 || y0 >= H)
                    return fail(KAZE_ERR_INVALID_ARG, "probe (%d, %d) of level %d outside the image",
                                x0, y0, i);
            }
    }
    const SgLayout L = sg_layout(W, H, p, c, shape);
    if (!ws || !aligned(ws, 256) || ws_bytes < L.total)
        return fail(KAZE_ERR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    L.total, ws_bytes);

    char* base = static_cast<char*>(ws);
    kaze_sg_scale_space* S = new kaze_sg_scale_space();
    S->W = W;
    S->H = H;
    S->N = N;
    S->shape = shape;
    S->probes = c->probes;
    S->bound = (float)c->bound;
    S->p = *p;
    schedule(p, S->lv);
    S->with_det = im->det != nullptr;
    S->with_nms = im->count != nullptr;
    const Scratch sc = scratch_layout(W, H, hist_bins(p), shape, L.scratch);
    BatchImage b = batch_image(W, H);
    b.img = im->img;
    b.ld = im->ld_img;
    b.levels = im->levels;
    b.det = im->det;
    b.g = reinterpret_cast<float*>(base + sc.g);
    b.hist = reinterpret_cast<unsigned*>(base + sc.hist);
    b.hmax = reinterpret_cast<unsigned*>(base + sc.hmax);
    b.k = im->k;
    b.kps = im->kps;
    b.capacity = im->capacity;
    b.count = im->count;
    S->b = b;
    S->aos = aos_desc(W, H, shape, base, sc, im->k);
    S->packed = static_cast<const unsigned char*>(packed);
    S->geo = sg::make_geo(1, W, H, sg::kConvRows);
    S->geo_probe = sg::make_geo(1, W, H, kProbeRows);
    S->x0 = reinterpret_cast<sg::bf16*>(base + L.x0);
    S->xa = reinterpret_cast<sg::bf16*>(base + L.xa);
    S->xb = reinterpret_cast<sg::bf16*>(base + L.xb);
    S->delta = reinterpret_cast<float*>(base + L.delta);
    S->tau = reinterpret_cast<float*>(base + L.tau);
    S->rects = reinterpret_cast<int4*>(base + L.rects);
    S->items = reinterpret_cast<int*>(base + L.items);
    S->err = err;

    // host tables: tau per level, probe windows and conv items per level
    const int P = std::max(1, c->probes);
    std::vector<float> htau(N, 0.f);
    std::vector<int4> hrect((size_t)N * P, make_int4(0, 0, 0, 0));
    std::vector<int> hitems((size_t)N * L.max_items, 0);
    S->item_off.assign(N, 0);
    S->item_cnt.assign(N, 0);
    std::vector<int> tmp;
    for (int i = 1; i < N; ++i) {
        htau[i] = (float)S->lv[i].tau;
        for (int q = 0; q < c->probes; ++q) {
            const int x0 = probe_xy[((size_t)i * c->probes + q) * 2];
            const int y0 = probe_xy[((size_t)i * c->probes + q) * 2 + 1];
            hrect[(size_t)i * P + q] =
                make_int4(x0, y0, std::min(c->probe_size, W - x0), std::min(c->probe_size, H - y0));
        }
        sg_probe_items(S->geo_probe, hrect.data() + (size_t)i * P, c->probes, tmp);
        if ((int)tmp.size() > L.max_items) {
            kaze_sg_scale_space_destroy(S);
            return fail(KAZE_ERR_UNSUPPORTED, "probe windows need %zu items (max %d)", tmp.size(),
                        L.max_items);
        }
        S->item_off[i] = i * L.max_items;
        S->item_cnt[i] = (int)tmp.size();
        std::copy(tmp.begin(), tmp.end(), hitems.begin() + (size_t)i * L.max_items);
    }
    hipError_t e = hipMemset(base + L.x0, 0, L.delta - L.x0);  // zero rings of the activations
    if (e == hipSuccess) e = hipMemcpy(S->tau, htau.data(), N * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(S->rects, hrect.data(), hrect.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(S->items, hitems.data(), hitems.size() * sizeof(int), hipMemcpyHostToDevice);

    hipStream_t cs = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int seg = 0; seg < 3 && e == hipSuccess && st == KAZE_OK; ++seg) {
        hipGraph_t graph = nullptr;
        g_prof.capturing = true;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = sg_segment(*S, seg, cs);
            const hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (st == KAZE_OK && e2 != hipSuccess) e = e2;
        }
        g_prof.capturing = false;
        if (e == hipSuccess && st == KAZE_OK)
            e = hipGraphInstantiate(&S->exec[seg], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (st != KAZE_OK || e != hipSuccess) {
        kaze_sg_scale_space_destroy(S);
        return st != KAZE_OK ? st : fail(KAZE_ERR_HIP, "surrogate scale-space setup failed: %s",
                                         hipGetErrorString(e));
    }
    *out = S;
    return KAZE_OK;
}

kaze_status kaze_sg_scale_space_run(kaze_sg_scale_space* S, int eager, void* stream) {
    if (!S) return fail(KAZE_ERR_INVALID_ARG, "surrogate scale space is NULL");
    return sg_run(*S, eager != 0, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- utility
const char* kaze_last_error(void) { return g_err; }

kaze_status kaze_profile_begin(const char* kernel_names) {
    if (!kernel_names) return fail(KAZE_ERR_INVALID_ARG, "kernel name list is NULL");
    unsigned mask = 0;
    const char* q = kernel_names;
    while (*q) {
        const char* e = strchr(q, ',');
        const size_t n = e ? (size_t)(e - q) : strlen(q);
        int found = -1;
        for (int i = 0; i < K_COUNT; ++i)
            if (strlen(kKernelNames[i]) == n && strncmp(q, kKernelNames[i], n) == 0) found = i;
        if (found < 0)
            return fail(KAZE_ERR_INVALID_ARG, "unknown kernel name in '%s'", kernel_names);
        mask |= 1u << found;
        q += n;
        if (*q == ',') ++q;
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
    static const std::string names = [] {  // built once, thread-safe initialisation
        std::string s;
        for (int i = 0; i < K_COUNT; ++i) {
            if (i) s += ",";
            s += kKernelNames[i];
        }
        return s;
    }();
    return names.c_str();
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
