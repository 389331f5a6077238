// Internal declarations shared by the HIP translation units of libkaze.
//
// Numerical building blocks used by more than one kernel:
//  * half-sample symmetric index reflection (the border rule of every
//    stencil, consistent with the zero-flux boundary of Eq. 4),
//  * the tridiagonal row of one AOS line system in increment form,
//  * the chunk reduction and the wavefront parallel cyclic reduction (PCR)
//    of the partitioned tridiagonal solver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kaze {

constexpr int kMaxLevels = 64;
constexpr int kMaxSubsteps = 64;  // steps per level
constexpr int kMaxRadius = 16;   // Gaussian radius ceil(3 sigma)
constexpr int kMaxStep = 8;      // Scharr step of the detector
constexpr int kWave = 64;        // CDNA wavefront

// Symmetric filter taps w[0..2r] (w[r] is the centre).
struct Taps {
    int r;
    float w[2 * kMaxRadius + 1];
};

// Per-level constants of the detector response (Eq. 8).
struct DetLevels {
    int step[kMaxLevels];    // Scharr step round(sigma_n)
    float sn2[kMaxLevels];   // sigma_n^2
    float sn[kMaxLevels];    // sigma_n
    int list[kMaxLevels];    // per launch: the levels it covers, in order
    float thr;               // detector threshold of the masks (BatchImage::mask)
    int band;                // rows per detector band (det_band_for)
};

// Rows per band of the detector's strips: short bands give more wavefronts
// for the same work (faster while the levels sit in the 256 MB cache),
// tall ones re-read fewer halo rows (less HBM traffic on large batches).
constexpr int kDetBandShort = 32;
constexpr int kDetBandTall = 64;
constexpr double kTallBandPixels = 32e6;  // pixels per run from which bands are tall
inline int det_band_for(double pixels) {
    return pixels >= kTallBandPixels ? kDetBandTall : kDetBandShort;
}

// Per-level constants of the description stage: Scharr step, sigma_n and
// the level's scale sigma_i (Eq. 6).
struct DescLevels {
    int step[kMaxLevels];
    float sn[kMaxLevels];
    float sigma[kMaxLevels];
};

// The record of kaze_keypoint_refined (24 bytes).
struct RefinedKeypoint {
    float x, y;
    int level;
    float response, edge_ratio;
    int kept;
};

// Global-memory views.  Kernels copy their descriptors into registers
// (resolve), which hides the address space of the pointers inside from the
// compiler: accesses through them become flat loads and stores, which wait
// on both memory counters.  A cast back keeps them global.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) unsigned guint;
typedef __attribute__((address_space(1))) unsigned long long gu64;

// A wave-uniform value in a scalar register (row addresses, loop bounds).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Half-sample symmetric reflection of index i into [0, n):
// -1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2, periodic with period 2n.
__device__ __forceinline__ int reflect_index(int i, int n) {
    if (i >= 0 && i < n) return i;
    const int p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

// One row of a tridiagonal system: a*x[j-1] + b*x[j] + c*x[j+1] = d.
struct Eq {
    float a, b, c, d;
};

__device__ __forceinline__ Eq eq_identity() { return Eq{0.f, 1.f, 0.f, 0.f}; }

// Row j of (I - 2 tau A(g)) delta = 2 tau A(g) L, the AOS line system in
// increment form (delta = u - L).  wl, wr are the coupling weights
// tau*(g[j-1]+g[j]) and tau*(g[j]+g[j+1]) (zero across the line ends) and
// dl = L[j-1]-L[j], dr = L[j+1]-L[j].
__device__ __forceinline__ Eq aos_row(float wl, float wr, float dl, float dr) {
    return Eq{-wl, (1.f + wl) + wr, -wr, __builtin_fmaf(wl, dl, wr * dr)};
}

// Parallel cyclic reduction step: eliminate the couplings of e through the
// neighbouring equations lo (below) and up (above).
__device__ __forceinline__ Eq pcr_reduce(const Eq& e, const Eq& lo, const Eq& up) {
    const float k1 = e.a / lo.b;
    const float k2 = e.c / up.b;
    Eq r;
    r.a = -k1 * lo.a;
    r.b = e.b - k1 * lo.c - k2 * up.a;
    r.c = -k2 * up.c;
    r.d = e.d - k1 * lo.d - k2 * up.d;
    return r;
}

__device__ __forceinline__ float lane_read(float v, int src_lane) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

__device__ __forceinline__ Eq lane_read(const Eq& e, int src_lane) {
    return Eq{lane_read(e.a, src_lane), lane_read(e.b, src_lane),
              lane_read(e.c, src_lane), lane_read(e.d, src_lane)};
}

// Solve the interface system of a partitioned line on one wavefront.
// Lane l owns chunk l and holds the reduced equations of the chunk's first
// unknown (e0, index 2l) and last unknown (e1, index 2l+1); together they
// form a tridiagonal system of 2*64 unknowns (lanes without a chunk hold
// identity rows).  Must be called by all 64 lanes.  Returns the first and
// last unknown of the lane's chunk.
__device__ __forceinline__ void wave_pcr_pairs(Eq e0, Eq e1, int lane, float& z0, float& z1) {
    // stride 1: e0 couples to the previous chunk's last (lane-1, e1) and the
    // own last (e1); e1 couples to the own first (e0) and the next chunk's
    // first (lane+1, e0).
    {
        Eq prev1 = lane_read(e1, lane > 0 ? lane - 1 : 0);
        Eq next0 = lane_read(e0, lane < kWave - 1 ? lane + 1 : kWave - 1);
        if (lane == 0) prev1 = eq_identity();
        if (lane == kWave - 1) next0 = eq_identity();
        const Eq n0 = pcr_reduce(e0, prev1, e1);
        const Eq n1 = pcr_reduce(e1, e0, next0);
        e0 = n0;
        e1 = n1;
    }
    // Now the even and the odd unknowns form two independent tridiagonal
    // systems with one equation per lane; reduce both with lane strides
    // 1, 2, ..., 32.
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const int lo_l = lane - s, up_l = lane + s;
        Eq lo0 = lane_read(e0, lo_l >= 0 ? lo_l : 0);
        Eq up0 = lane_read(e0, up_l < kWave ? up_l : kWave - 1);
        Eq lo1 = lane_read(e1, lo_l >= 0 ? lo_l : 0);
        Eq up1 = lane_read(e1, up_l < kWave ? up_l : kWave - 1);
        if (lo_l < 0) { lo0 = eq_identity(); lo1 = eq_identity(); }
        if (up_l >= kWave) { up0 = eq_identity(); up1 = eq_identity(); }
        const Eq n0 = pcr_reduce(e0, lo0, up0);
        const Eq n1 = pcr_reduce(e1, lo1, up1);
        e0 = n0;
        e1 = n1;
    }
    z0 = e0.d / e0.b;
    z1 = e1.d / e1.b;
}

}  // namespace kaze

// ---------------------------------------------------------------------------
// Descriptors and work lists shared by the kernels and the host code.
// ---------------------------------------------------------------------------
namespace kaze {

constexpr int kTile = 64;          // edge of the stencil tiles
constexpr int kMaxSide = 4096;     // largest image width or height
constexpr int kMaxCondRadius = 4;  // sigma_cond radius that keeps the fused tile within 64 KB of LDS
constexpr int kHistChunk = 8192;   // pixels per block of the histogram kernel
// Runs under kSmallHistPixels take blocks of kHistChunkSmall pixels: four
// times the blocks for the latency of one image (1920x1200: 2059 -> 2072
// images/s), where batches of 18 Mpx and more lost 0.4-2% to the added
// global bin additions.
constexpr int kHistChunkSmall = 2048;
constexpr double kSmallHistPixels = 8e6;
inline int hist_chunk_for(double pixels) {
    return pixels < kSmallHistPixels ? kHistChunkSmall : kHistChunk;
}
constexpr int kHistCopies = 16;   // global copies of the k histogram (atomic contention)
constexpr int kNmsRows = 8;        // rows per thread of the extrema kernel

// Buffers of one image of a (possibly batched) scale-space computation.
struct BatchImage {
    const float* img;   // input, row pitch ld
    int ld;
    float* levels;      // N planes of W x H
    float* det;         // N planes of W x H
    float* g;           // conductivity plane (squared gradient while k is formed)
    unsigned* hist;     // k histogram
    unsigned* hmax;     // max |grad| (float bits) of each gradient tile, one word per tile
    float* k;           // contrast factor (device scalar)
    void* kps;          // keypoints, capacity entries
    int capacity;
    int* count;
    // N planes of H rows x mask_words(W) words: bit b of word (i, y, j) is
    // set iff det_i(x0 + b, y) > DetLevels::thr, x0 the first column of the
    // detector's strip j of level i (words past the level's strips unused).
    // Written by the detector beside det when not null; the extrema kernel
    // then reads only the det values whose bit is set.
    unsigned long long* mask;
    int W, H;
};

// AOS line partition and launch shapes.  Every row line is cut into chunks
// of rc pixels and every column line into chunks of cc pixels; the
// reduction and recovery tiles are kAosTX pixels wide (kAosTX / rc row
// chunks per tile row) and ty high (ty / cc column chunks per tile column);
// the interface solve gives every lane m consecutive chunks of a line.  The
// chunk lengths and m fix the arithmetic (the elimination order), the tile
// height only the launch: shapes that differ in ty alone give bitwise equal
// results, the others agree to FP32 rounding.
struct AosShape {
    int ty, rc, cc, m;
};
constexpr int kAosTX = 60;
constexpr int kAosShapes = 6;
constexpr AosShape kAosShape[kAosShapes] = {
    {32, 30, 32, 4}, {32, 30, 32, 8}, {64, 30, 32, 4},
    {64, 30, 32, 8}, {64, 60, 64, 4}, {64, 60, 64, 8},
};
constexpr int kMaxColChunk = 64;
// Lanes per chunk in the sweeps of a shape: 2 when the tile's row chunks
// fill one wavefront and one column chunk spans the tile height (every
// chunk then goes to a lane pair and all four wavefronts of the tile sweep),
// else 1.
constexpr int chunk_lanes(int ty, int rc, int cc) {
    return (kAosTX / rc) * ty == 64 && cc == ty ? 2 : 1;
}

__host__ __device__ inline int aos_row_chunks(int W, int rc) { return (W + rc - 1) / rc; }
__host__ __device__ inline int aos_col_chunks(int H, int cc) { return (H + cc - 1) / cc; }
__host__ __device__ inline int aos_tiles_of(int W, int H, int ty) {
    return ((W + kAosTX - 1) / kAosTX) * ((H + ty - 1) / ty);
}
// Interface solve: every lane holds M consecutive chunks of a line and a
// line spans iface_lanes(chunks, M) lanes (a power of two), so a wavefront
// serves 64 / iface_lanes lines of one direction of one image.  Work items:
// the row-line groups of the image, then its column-line groups.
// Default shape (aos_shape -1): 60 x 32 tiles, chunks of 30 / 32, and M = 8,
// or M = 4 for launches with few wavefronts, where the shorter lane-local
// elimination and the doubled number of wavefronts win (measured at
// 1920x1200: 9.5 -> 8.4 us per level; on the 64-image batch 8 stays ahead,
// 597 against 607 us per level).
constexpr int kIfaceSmallGroups = 1024;  // wavefronts at M = 8 below which M = 4
__host__ __device__ inline int iface_lanes(int nch, int M) {
    int p = 1;
    while (p * M < nch) p <<= 1;
    return p;
}
__host__ __device__ inline int iface_groups(int lines, int nch, int M) {
    const int per = 64 / iface_lanes(nch, M);
    return (lines + per - 1) / per;
}
inline int aos_line_groups(int W, int H, const AosShape& a) {
    return iface_groups(H, aos_row_chunks(W, a.rc), a.m) +
           iface_groups(W, aos_col_chunks(H, a.cc), a.m);
}
// The default shape for images whose interface launch would have this many
// wavefronts with M = 8: shape 1 (M = 8), or shape 0 (M = 4) below
// kIfaceSmallGroups.
inline int default_shape_for(long long groups_at_m8) {
    return groups_at_m8 < kIfaceSmallGroups ? 0 : 1;
}

// The two reduced equations of a chunk (first and last unknown), each scaled
// to a unit diagonal and stored as (a, c, d): 6 floats per chunk.
constexpr int kEqFloats = 6;

// One image of an AOS step.  Interface equations and solutions are stored
// chunk-major, so that the lanes of one wavefront (consecutive lines) touch
// consecutive addresses.
struct ImageDesc {
    const float* L;   // level i-1, W x H, pitch W
    float* Lnext;     // level i
    float* g;         // conductivity of L (written or read, see the kernel)
    float* rrow;      // reduced equations of the row chunks, [nchr][H][kEqFloats]
    float* rcol;      // ... of the column chunks, [nchc][W][kEqFloats]
    float* zrow;      // first/last unknown of every row chunk, [nchr][H][2]
    float* zcol;      // ... of every column chunk, [nchc][W][2]
    const float* k;   // contrast factor (device scalar); NULL: use the host value
    int W, H, nchr, nchc;
    // optional gate: the step is skipped when *gate <= bound (the level was
    // accepted from the surrogate); NULL: always run
    const float* gate;
    float bound;
};

// Work list of a batched launch: entry t names an image (index into descs)
// and a local tile, line or block index inside it.  With a NULL list the
// launch covers the single image passed by value and entry t is local
// index t.
template <class D>
struct Work {
    const D* descs;
    const int2* items;
    int count;
};

constexpr int kXcds = 8;  // accelerator complex dies; workgroups are dealt round-robin

// Launch-order index t of a one-block-per-item grid of n blocks -> work item,
// such that XCD x (which receives blocks x, x+8, x+16, ...) works through
// one contiguous run of the list: neighbouring tiles, whose rings overlap,
// then share that XCD's L2.
__device__ __forceinline__ int xcd_contiguous(int t, int n) {
    const int x = t % kXcds, j = t / kXcds;
    const int per = n / kXcds, rem = n % kXcds;
    return x * per + (x < rem ? x : rem) + j;
}

// Block (x, y) of a 2-D grid remapped so that XCD x receives a contiguous
// run of the row-major block order (x fastest).
__device__ __forceinline__ void xcd_grid(int& bx, int& by) {
    const int gx = (int)gridDim.x, n = gx * (int)gridDim.y;
    const int t = xcd_contiguous((int)(blockIdx.x + blockIdx.y * gridDim.x), n);
    bx = t % gx;
    by = t / gx;
}

// t must be wave-uniform; the tables are read through the constant address
// space, so descriptor and item land in scalar registers.
template <class D>
__device__ __forceinline__ void resolve(const D& d0, const Work<D>& w, int t, D& d, int& local) {
    if (w.items) {
        typedef __attribute__((address_space(4))) const int cint;
        static_assert(sizeof(D) % sizeof(int) == 0, "descriptors are whole words");
        const cint* it = (const cint*)w.items + 2 * t;
        const cint* src = (const cint*)(w.descs + it[0]);
        int* dst = reinterpret_cast<int*>(&d);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(D) / sizeof(int)); ++i) dst[i] = src[i];
        local = it[1];
    } else {
        d = d0;
        local = t;
    }
}

inline int tiles_of(int W, int H, int tx = kTile, int ty = kTile) {
    return ((W + tx - 1) / tx) * ((H + ty - 1) / ty);
}


enum KernelId {
    K_GAUSS = 0,
    K_GRAD,
    K_HIST,
    K_KSELECT,
    K_COND,
    K_AOS_REDUCE,
    K_AOS_IFACE,
    K_AOS_RECOVER,
    K_DET,
    K_NMS,
    K_FILL,
    K_COPY,
    K_SG_PACK,
    K_SG_CONV1,
    K_SG_CONV,
    K_SG_CONV6,
    K_SG_PROBE,
    K_FED,
    K_REFINE,
    K_DERIV,
    K_DESCRIBE,
    K_COUNT
};

using ImgWork = Work<BatchImage>;
using AosWork = Work<ImageDesc>;

// a1: levels[0] = G_sigma0 * img on 64x64 tiles (items: image, tile).
// also resets each image's counters as launch_reset does (nbins, k_fill)
hipError_t launch_gauss(const BatchImage& d0, const ImgWork& w, const Taps& taps, int nbins,
                        float k_fill, hipStream_t s);
// Conductivity of levels[0] into g with the AOS reduction's band code on
// kAosTX x ty tiles (ty 32 or 64; items: image, tile of that height, or the
// tiles of d0): mode 0 g2, 1 g1 (k from d.k, or k_host if NULL), bitwise the
// g of the fused reduction; mode 2 the squared gradient magnitude and the
// maximum of |grad| of each tile into its hmax word.
hipError_t launch_cond(const BatchImage& d0, const ImgWork& w, const Taps& taps, float k_host,
                       int mode, int ty, hipStream_t s);
// a2: histogram of sqrt(g) (items: image, chunk of `chunk` pixels) and the
// quantile (items: image, 0).
// tile_h: the height of the gradient kernel's tiles, whose per-tile maxima
// of |grad| the two kernels reduce.
hipError_t launch_hist(const BatchImage& d0, const ImgWork& w, int nbins, int tile_h, int chunk,
                       hipStream_t s);
hipError_t launch_kselect(const BatchImage& d0, const ImgWork& w, int nbins,
                          unsigned long long pct_mant, int pct_shift, int tile_h, hipStream_t s);
// Per image (items: image, 0): zero hist, hmax and count; k = k_fill if > 0.
hipError_t launch_reset(const BatchImage& d0, const ImgWork& w, int nbins, float k_fill,
                        hipStream_t s);

// a3-a5: AOS step in three launches on tiles of kAosTX x kAosShape[shape].ty.
// reduce: (conductivity if compute_g, else g is read) + chunk reduction of
// every row and column chunk (items: image, tile); iface: the interface
// system of every line (items: image, group of lines, row groups first, see
// iface_lanes); recover: interior of every chunk and
// L_next = L + (delta_x + delta_y)/2 (items: image, tile).
hipError_t launch_aos_reduce(const ImageDesc& d0, const AosWork& w, int shape, const Taps& tc,
                             float tau, bool compute_g, int gmode, float k_host, hipStream_t s);
hipError_t launch_aos_iface(const ImageDesc& d0, const AosWork& w, int shape, hipStream_t s);
hipError_t launch_aos_recover(const ImageDesc& d0, const AosWork& w, int shape, float tau,
                              hipStream_t s);

// Exact AOS increments on small probe windows: rects[p] = (x0, y0, w, h),
// w, h <= kProbeMax.  Every row and column through a window is solved whole
// (one wavefront per line, chunks of 64 per lane); delta[p] receives the row
// increments [h][w] then the column increments [h][w] (pitch kProbeMax).
// probe_err then compares L + (delta_x + delta_y)/2 with cand on every
// window and raises *err (float bits, atomic max; NaN counts as +inf).
// Batches pass pdesc and rect_img: window p then lies in the image
// pdesc[rect_img[p]], whose L, g, Lnext (the candidate), W, H and gate (the
// error word) replace the single-image arguments.
constexpr int kProbeMax = 32;
hipError_t launch_aos_probe(const ImageDesc& d, const int4* rects, int nprobes, float tau,
                            float* delta, hipStream_t s, const ImageDesc* pdesc = nullptr,
                            const int* rect_img = nullptr);
hipError_t launch_probe_err(const float* L, const float* cand, int W, const int4* rects,
                            int nprobes, const float* delta, unsigned* err, hipStream_t s,
                            const ImageDesc* pdesc = nullptr, const int* rect_img = nullptr);

// a6: det of the levels lev0 .. lev1-1 in strips of 64 - 2S output columns
// (S the level's Scharr step) and bands of rows, four strip-bands per block
// (items: image, block of a level).
hipError_t launch_det(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                      const DetLevels& dl, hipStream_t s);
// Blocks per level of an image for the levels of steps smin..smax.
int det_tiles_of(int W, int H, int smin, int smax, int band);
// a7: extrema of levels 1..N-2 (items: image, block of 64 x 4*kNmsRows pixels).
// Half-side of the cross-level window of each level (1: the 3x3x3 test) and
// the Scharr step of each level (the layout of its detector mask).
struct NmsRadii {
    int h[kMaxLevels];
    int step[kMaxLevels];
};
// masked: the images carry detector masks written with this threshold
// (items: image, block of 256 mask words of a level); else every det value
// is read.
hipError_t launch_nms(const BatchImage& d0, const ImgWork& w, int N, float threshold,
                      const NmsRadii& radii, hipStream_t s, bool masked = false);
int nms_blocks_of(int W, int H, bool masked = false);
// Detector strips of a level with Scharr step S: 64 - 2S output columns
// each, the last one aligned to end at column W.
__host__ __device__ inline int det_strips(int W, int S) {
    const int sw = 64 - 2 * S;
    return W <= sw ? 1 : (W + sw - 1) / sw;
}
// Mask words per row: one per strip at the largest step.
__host__ __device__ inline int mask_words(int W) { return det_strips(W, kMaxStep); }
// Refinement and edge test of capacity-bounded extrema (entries of 16 and 24
// bytes: kaze_keypoint and kaze_keypoint_refined) on N levels of W x H;
// thr = (r+1)^2/r.
hipError_t launch_refine(const float* det, int W, int H, int N, const void* kps,
                         const int* count, int capacity, float thr, void* out, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s);
// Description stage: scale-normalised first derivatives of N levels, and
// orientation + M-SURF descriptor of min(*count, capacity) refined keypoints.
hipError_t launch_deriv(const float* levels, int W, int H, int N, const DescLevels& dl, float* lx,
                        float* ly, hipStream_t s);
// The same derivatives by the detector's row-rolling kernel (levels with a
// Scharr step of at most 4; hipErrorNotSupported otherwise).
hipError_t launch_det_derivs(const BatchImage& b, int N, const DetLevels& dl, float* lx,
                             float* ly, hipStream_t s);
hipError_t launch_describe(const float* lx, const float* ly, int W, int H, int N,
                           const DescLevels& dl, const void* kps, const int* count, int capacity,
                           float* angles, float* desc, hipStream_t s);
hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s);

}  // namespace kaze
