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
};

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
    return Eq{-wl, 1.f + wl + wr, -wr, wl * dl + wr * dr};
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
// Tile-partitioned AOS step: data shared by the kernels of one step.
// ---------------------------------------------------------------------------
namespace kaze {

constexpr int kTile = 64;        // tile edge = chunk length of every line solve
constexpr int kMaxCondRadius = 4;  // sigma_cond radius that keeps the fused tile within 64 KB of LDS

// One image of an AOS step.  Row line y is cut into ncx chunks of kTile
// pixels (tile columns), column line x into ncy chunks (tile rows).
struct ImageDesc {
    const float* L;   // level i-1, W x H, pitch W
    float* Lnext;     // level i
    float* g;         // conductivity of L (written or read, see the kernel)
    float* rrow;      // reduced interface rows of the row lines, [H][ncx][8]
    float* rcol;      // ... of the column lines, [W][ncy][8]
    float* zrow;      // first/last unknown of every row chunk, [H][ncx][2]
    float* zcol;      // ... of every column chunk, [W][ncy][2]
    const float* k;   // contrast factor (device scalar); NULL: use the host value
    int W, H, ncx, ncy;
};

// Work list of a batched launch: entry t names an image and a tile (or a
// line) inside it.  With a NULL list the launch covers image 0 only and
// entry t is tile/line t of the descriptor passed by value.
struct WorkList {
    const ImageDesc* descs;  // device table, one per image (or NULL)
    const int2* items;       // {image, local tile or line index}
    int count;
};

inline int tiles_of(int W, int H) {
    return ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
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
    K_COUNT
};

hipError_t launch_gauss(const float* src, int ld_src, float* dst, int W, int H,
                        const Taps& taps, hipStream_t s);
// Conductivity of L on 64x64 tiles (the same code as the fused AOS kernel).
// mode 0: g2, 1: g1, 2: squared gradient magnitude and the running maximum
// of |grad| into hmax_bits.  k is read from k_dev, or k_host if NULL.
hipError_t launch_cond(const float* L, float* out, int W, int H, const Taps& taps,
                       const float* k_dev, float k_host, int mode, unsigned* hmax_bits,
                       hipStream_t s);
hipError_t launch_hist(const float* m2, int n, const unsigned* hmax_bits, unsigned* hist,
                       int nbins, hipStream_t s);
hipError_t launch_kselect(const unsigned* hist, int nbins, const unsigned* hmax_bits,
                          unsigned long long pct_mant, int pct_shift, float* k_out,
                          hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int n, float v, hipStream_t s);

// AOS step in three launches.  reduce: (conductivity if compute_g, else g
// is read) + chunk reduction of every row and column chunk; iface: the
// interface system of every line by wavefront PCR; recover: interior of
// every chunk and L_next = L + (delta_x + delta_y)/2.
// grid_cap > 0 caps the grid of the line kernel (wavefronts loop over the
// list); the tile kernels run one block per tile.
hipError_t launch_aos_reduce(const ImageDesc& d0, const WorkList& w, const Taps& tc,
                             float tau, bool compute_g, int gmode, float k_host, int grid_cap,
                             hipStream_t s);
hipError_t launch_aos_iface(const ImageDesc& d0, const WorkList& w, int grid_cap,
                            hipStream_t s);
hipError_t launch_aos_recover(const ImageDesc& d0, const WorkList& w, float tau, int grid_cap,
                              hipStream_t s);

hipError_t launch_det(const float* levels, float* det, int W, int H, int N,
                      const DetLevels& dl, hipStream_t s);
hipError_t launch_nms(const float* det, int W, int H, int N, float threshold, void* kps,
                      int capacity, int* count, hipStream_t s);
hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s);

}  // namespace kaze
