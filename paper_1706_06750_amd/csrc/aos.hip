// Semi-implicit step of Eq. 4 by additive operator splitting (AOS):
//   L_i = L_{i-1} + (delta_x + delta_y) / 2,
//   (I - 2 tau A_l(g)) delta_l = 2 tau A_l(g) L_{i-1},   l in {rows, columns},
// where A_l is the 1-D nonlinear diffusion matrix along rows or columns with
// couplings (g_j + g_k)/2 between neighbours and no flux across the image
// border.  Solving for the increment delta = u - L rather than u keeps the
// FP32 error relative to the change of one step, not to the image.
//
// Every row and column system is solved by a partitioned tridiagonal
// method on 64x64 tiles (partitioned / hybrid tridiagonal solvers: Zhang,
// Cohen & Owens, PPoPP 2010; Laszlo, Giles & Appleyard, ACM TOMS 2016):
//
//  1. aos_reduce (one block per tile): the tile of L_{i-1} plus a ring is
//     staged in LDS, the conductivity g is computed there (and written
//     once for step 3), and each tile row and tile column -- a 64-element
//     chunk of its line -- is reduced by one forward sweep to two equations
//     that couple its first and last unknowns to the neighbouring chunks.
//     The sweep also accumulates the back-substitution weights of the
//     chunk's second unknown, so the first unknown's equation needs no
//     backward sweep.
//  2. aos_iface (one wavefront per line): the 2 equations per chunk form a
//     tridiagonal system of 2 x (chunks per line) unknowns, solved by
//     parallel cyclic reduction across the lanes (lane = chunk).
//  3. aos_recover (one block per tile): with both ends of every chunk
//     known, each tile row and column recovers its interior by a Thomas
//     sweep in registers, and L_i = L + (delta_x + delta_y)/2 is stored.
//
// HBM traffic per pixel and step: L read twice, g written once and read
// once, L_i written once, plus 2 x 32 bytes of interface equations per
// 64-pixel chunk.  Tile rows are staged through LDS (the transpose that lets
// one thread walk a row); tile columns are walked by adjacent threads on
// adjacent columns, so every global access is coalesced.
#include "kaze_internal.h"
#include "tile_cond.h"

namespace kaze {
namespace {

constexpr int kBlock = 256;

// v_rcp_f32: <= 1 ulp; the pivots are >= 1 (diagonally dominant rows).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Chunk of kTile unknowns at line positions pos0 .. pos0+kTile-1 of a line of
// n pixels.  Acc::g(k), Acc::L(k) give conductivity and level at chunk
// index k in [-1, kTile] (the ring supplies -1 and kTile).  Positions past
// the line end are identity rows (decoupled, solution 0).
template <class Acc>
__device__ __forceinline__ void chunk_reduce(const Acc& A, int pos0, int n, float tau, Eq& E0,
                                             Eq& E1) {
    float gm = A.g(-1), Lm = A.L(-1), g0 = A.g(0), L0 = A.L(0);
    float gp = A.g(1), Lp = A.L(1);
    float wl = (pos0 > 0 && pos0 < n) ? tau * (gm + g0) : 0.f;
    float wr = (pos0 < n - 1) ? tau * (g0 + gp) : 0.f;
    const Eq first = aos_row(wl, wr, Lm - L0, Lp - L0);
    wl = wr;
    Lm = L0;
    g0 = gp;
    L0 = Lp;
    // x_k + cp x_{k+1} = dp + ep x_0 over the interior, and
    // x_1 = al + be x_0 + P x_{kTile-1} accumulated along the way.
    float cp = 0.f, dp = 0.f, ep = 1.f, P = 1.f, al = 0.f, be = 0.f;
#pragma unroll 8
    for (int k = 1; k <= kTile - 2; ++k) {
        gp = A.g(k + 1);
        Lp = A.L(k + 1);
        wr = (pos0 + k < n - 1) ? tau * (g0 + gp) : 0.f;
        const float d = wl * (Lm - L0) + wr * (Lp - L0);
        const float r = rcp(1.f + wl + wr + wl * cp);
        dp = (d + wl * dp) * r;
        ep = wl * ep * r;
        cp = -wr * r;
        al += P * dp;
        be += P * ep;
        P = -P * cp;
        wl = wr;
        Lm = L0;
        g0 = gp;
        L0 = Lp;
    }
    gp = A.g(kTile);
    Lp = A.L(kTile);
    wr = (pos0 + kTile - 1 < n - 1) ? tau * (g0 + gp) : 0.f;
    const Eq last = aos_row(wl, wr, Lm - L0, Lp - L0);
    E1 = Eq{last.a * ep, last.b - last.a * cp, last.c, last.d - last.a * dp};
    E0 = Eq{first.a, first.b + first.c * be, first.c * P, first.d - first.c * al};
}

// Interior of a chunk by a Thomas sweep with both ends known (z0 at k = 0,
// z1 at k = kTile-1).  On return x[k] holds the increment of every element.
template <class Acc>
__device__ __forceinline__ void chunk_recover(const Acc& A, int pos0, int n, float tau, float z0,
                                              float z1, float (&x)[kTile]) {
    float cpa[kTile];
    float gm = A.g(0), Lm = A.L(0), g0 = A.g(1), L0 = A.L(1);
    float wl = (pos0 + 1 < n) ? tau * (gm + g0) : 0.f;
    float cp = 0.f, dp = 0.f;
#pragma unroll
    for (int k = 1; k <= kTile - 2; ++k) {
        const float gp = A.g(k + 1), Lp = A.L(k + 1);
        const float wr = (pos0 + k < n - 1) ? tau * (g0 + gp) : 0.f;
        float d = wl * (Lm - L0) + wr * (Lp - L0);
        const float b = 1.f + wl + wr;
        float a = -wl, c = -wr;
        if (k == 1) {
            d -= a * z0;
            a = 0.f;
        }
        if (k == kTile - 2) {
            d -= c * z1;
            c = 0.f;
        }
        const float r = rcp(b - a * cp);
        cp = c * r;
        dp = (d - a * dp) * r;
        cpa[k] = cp;
        x[k] = dp;
        wl = wr;
        Lm = L0;
        g0 = gp;
        L0 = Lp;
    }
    x[0] = z0;
    x[kTile - 1] = z1;
#pragma unroll
    for (int k = kTile - 2; k >= 1; --k) x[k] -= cpa[k] * x[k + 1];
}

// LDS accessor of one chunk: element k at offset k * stride (k may be -1).
struct LineAcc {
    const float* gp;  // element 0
    const float* Lp;
    int gs, Ls;       // strides between consecutive chunk elements
    __device__ __forceinline__ float g(int k) const { return gp[k * gs]; }
    __device__ __forceinline__ float L(int k) const { return Lp[k * Ls]; }
};

__device__ __forceinline__ void resolve(const ImageDesc& d0, const WorkList& w, int t,
                                        ImageDesc& d, int& local) {
    if (w.items) {
        const int2 it = w.items[t];
        d = w.descs[it.x];
        local = it.y;
    } else {
        d = d0;
        local = t;
    }
}

__device__ __forceinline__ void store_eqs(float* dst, const Eq& e0, const Eq& e1) {
    float4* o = reinterpret_cast<float4*>(dst);
    o[0] = make_float4(e0.a, e0.b, e0.c, e0.d);
    o[1] = make_float4(e1.a, e1.b, e1.c, e1.d);
}

template <int RG, bool COMPUTE_G>
__global__ __launch_bounds__(kBlock) void aos_reduce_kernel(ImageDesc d0, WorkList w, Taps tc,
                                                            float tau, int gmode, float k_host,
                                                            int count) {
    using G = CondGeom<RG>;
    extern __shared__ float smem[];
    float* sL = smem;
    float* sS = smem + G::offS;
    float* sG = smem + G::offG;
    const int tid = threadIdx.x;

    {
        // one block per work item: a grid-stride loop here was measured to
        // double the register demand (spills) without saving launches
        const int t = blockIdx.x;
        if (t >= count) return;
        ImageDesc d;
        int lt;
        resolve(d0, w, t, d, lt);
        const int W = d.W, H = d.H;
        const int cx = lt % d.ncx, cy = lt / d.ncx;
        const int tx0 = cx * kTile, ty0 = cy * kTile;

        load_L_ring<RG>(d.L, W, H, tx0, ty0, sL);
        if (COMPUTE_G) {
            __syncthreads();
            smooth_tile<RG>(sL, sS, tc);
            __syncthreads();
            const float k = d.k ? d.k[0] : k_host;
            const float inv_k2 = 1.f / (k * k);
            float* gout = d.g;
            scharr_pass<RG>(sS, [&](int gy, int gx, float m2) {
                const float gval = diffusivity(m2, inv_k2, gmode);
                sG[gy * G::pG + gx] = gval;
                const int y = ty0 - 1 + gy, x = tx0 - 1 + gx;
                if (gy >= 1 && gy <= kTile && gx >= 1 && gx <= kTile && y < H && x < W)
                    gout[(size_t)y * W + x] = gval;
            });
        } else {
            stage_region<G::nG, G::nG, G::pG, kBlock>(d.g, W, H, ty0 - 1, tx0 - 1, sG);
        }
        __syncthreads();

        // tile rows (threads 0..63) and tile columns (64..127) share one code
        // path; the choice is uniform per wavefront
        if (tid < 2 * kTile) {
            const bool is_row = tid < kTile;
            const int c = is_row ? tid : tid - kTile;
            const int line = (is_row ? ty0 : tx0) + c;  // image row y or column x
            if (line < (is_row ? H : W)) {
                const LineAcc A = is_row
                    ? LineAcc{sG + (c + 1) * G::pG + 1, sL + (c + G::R) * G::pL + G::R, 1, 1}
                    : LineAcc{sG + G::pG + (c + 1), sL + G::R * G::pL + (c + G::R), G::pG, G::pL};
                Eq e0, e1;
                chunk_reduce(A, is_row ? tx0 : ty0, is_row ? W : H, tau, e0, e1);
                float* dst = is_row ? d.rrow + ((size_t)line * d.ncx + cx) * 8
                                    : d.rcol + ((size_t)line * d.ncy + cy) * 8;
                store_eqs(dst, e0, e1);
            }
        }
        __syncthreads();
    }
}

// One wavefront per line; lane p holds chunk p's two interface equations.
__global__ __launch_bounds__(kBlock) void aos_iface_kernel(ImageDesc d0, WorkList w, int count) {
    const int lane = threadIdx.x % kWave;
    const int waves = kBlock / kWave;
    for (int t = blockIdx.x * waves + threadIdx.x / kWave; t < count; t += gridDim.x * waves) {
        ImageDesc d;
        int line;
        resolve(d0, w, t, d, line);
        const float* R;
        float* Z;
        int nch;
        if (line < d.H) {
            nch = d.ncx;
            R = d.rrow + (size_t)line * nch * 8;
            Z = d.zrow + (size_t)line * nch * 2;
        } else {
            nch = d.ncy;
            R = d.rcol + (size_t)(line - d.H) * nch * 8;
            Z = d.zcol + (size_t)(line - d.H) * nch * 2;
        }
        Eq e0 = eq_identity(), e1 = eq_identity();
        if (lane < nch) {
            const float4* r = reinterpret_cast<const float4*>(R + lane * 8);
            const float4 a = r[0], b = r[1];
            e0 = Eq{a.x, a.y, a.z, a.w};
            e1 = Eq{b.x, b.y, b.z, b.w};
        }
        float z0, z1;
        wave_pcr_pairs(e0, e1, lane, z0, z1);
        if (lane < nch) reinterpret_cast<float2*>(Z + lane * 2)[0] = make_float2(z0, z1);
    }
}

constexpr int kPitchT = kTile + 1;
constexpr int kRecoverThreads = 2 * kTile;  // one thread per tile row and per tile column

__global__ __launch_bounds__(kRecoverThreads) void aos_recover_kernel(ImageDesc d0, WorkList w,
                                                                      float tau, int count) {
    __shared__ float sL[kTile * kPitchT];
    __shared__ float sG[kTile * kPitchT];
    __shared__ float sD[kTile * kPitchT];
    const int tid = threadIdx.x;

    {
        // one block per work item: a grid-stride loop here was measured to
        // double the register demand (spills) without saving launches
        const int t = blockIdx.x;
        if (t >= count) return;
        ImageDesc d;
        int lt;
        resolve(d0, w, t, d, lt);
        const int W = d.W, H = d.H;
        const int cx = lt % d.ncx, cy = lt / d.ncx;
        const int tx0 = cx * kTile, ty0 = cy * kTile;
        const bool full = ty0 + kTile <= H && tx0 + kTile <= W;

        // stage L and g (zero outside the image) in two halves, all loads of
        // a half in flight together
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            constexpr int PER = kTile * kTile / (2 * kRecoverThreads);
            float vl[PER], vg[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int i = tid + (half * PER + j) * kRecoverThreads;
                const int y = ty0 + i / kTile, x = tx0 + i % kTile;
                const bool in = full || (y < H && x < W);
                const size_t o = in ? (size_t)y * W + x : 0;
                vl[j] = in ? d.L[o] : 0.f;
                vg[j] = in ? d.g[o] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int i = tid + (half * PER + j) * kRecoverThreads;
                sL[(i / kTile) * kPitchT + i % kTile] = vl[j];
                sG[(i / kTile) * kPitchT + i % kTile] = vg[j];
            }
        }
        __syncthreads();

        float xs[kTile];
        const bool is_row = tid < kTile;
        const int c = is_row ? tid : tid - kTile;
        const int line = (is_row ? ty0 : tx0) + c;
        const bool active = line < (is_row ? H : W);
        const bool col_thread = !is_row && active;
        if (active) {
            const float2 z = reinterpret_cast<const float2*>(
                is_row ? d.zrow + ((size_t)line * d.ncx + cx) * 2
                       : d.zcol + ((size_t)line * d.ncy + cy) * 2)[0];
            const LineAcc A = is_row ? LineAcc{sG + c * kPitchT, sL + c * kPitchT, 1, 1}
                                     : LineAcc{sG + c, sL + c, kPitchT, kPitchT};
            chunk_recover(A, is_row ? tx0 : ty0, is_row ? W : H, tau, z.x, z.y, xs);
            if (is_row) {
#pragma unroll
                for (int k = 0; k < kTile; ++k) sD[c * kPitchT + k] = xs[k];
            }
        }
        __syncthreads();
        if (col_thread) {
            const int x = tx0 + c;
#pragma unroll
            for (int k = 0; k < kTile; ++k) {
                const int y = ty0 + k;
                if (y < H)
                    d.Lnext[(size_t)y * W + x] =
                        sL[k * kPitchT + c] + 0.5f * (sD[k * kPitchT + c] + xs[k]);
            }
        }
        __syncthreads();
    }
}

int grid_of(int count, int cap) { return cap > 0 && cap < count ? cap : count; }

int work_count(const ImageDesc& d0, const WorkList& w, bool lines) {
    if (w.items) return w.count;
    return lines ? d0.H + d0.W : tiles_of(d0.W, d0.H);
}

}  // namespace

template <int RG>
hipError_t launch_reduce_r(const ImageDesc& d0, const WorkList& w, const Taps& tc, float tau,
                           bool compute_g, int gmode, float k_host, int grid, int count,
                           hipStream_t s) {
    const size_t lds = (size_t)CondGeom<RG>::floats * sizeof(float);
    if (compute_g)
        hipLaunchKernelGGL((aos_reduce_kernel<RG, true>), dim3(grid), dim3(kBlock), lds, s, d0, w,
                           tc, tau, gmode, k_host, count);
    else
        hipLaunchKernelGGL((aos_reduce_kernel<RG, false>), dim3(grid), dim3(kBlock), lds, s, d0,
                           w, tc, tau, gmode, k_host, count);
    return hipGetLastError();
}

hipError_t launch_aos_reduce(const ImageDesc& d0, const WorkList& w, const Taps& tc, float tau,
                             bool compute_g, int gmode, float k_host, int grid_cap,
                             hipStream_t s) {
    const int count = work_count(d0, w, false);
    if (count <= 0) return hipSuccess;
    const int grid = count;
    (void)grid_cap;
    switch (tc.r) {
        case 1: return launch_reduce_r<1>(d0, w, tc, tau, compute_g, gmode, k_host, grid, count, s);
        case 2: return launch_reduce_r<2>(d0, w, tc, tau, compute_g, gmode, k_host, grid, count, s);
        case 3: return launch_reduce_r<3>(d0, w, tc, tau, compute_g, gmode, k_host, grid, count, s);
        case 4: return launch_reduce_r<4>(d0, w, tc, tau, compute_g, gmode, k_host, grid, count, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aos_iface(const ImageDesc& d0, const WorkList& w, int grid_cap, hipStream_t s) {
    const int count = work_count(d0, w, true);
    if (count <= 0) return hipSuccess;
    const int waves = kBlock / kWave;
    hipLaunchKernelGGL(aos_iface_kernel, dim3(grid_of((count + waves - 1) / waves, grid_cap)),
                       dim3(kBlock), 0, s, d0, w, count);
    return hipGetLastError();
}

hipError_t launch_aos_recover(const ImageDesc& d0, const WorkList& w, float tau, int grid_cap,
                              hipStream_t s) {
    const int count = work_count(d0, w, false);
    if (count <= 0) return hipSuccess;
    (void)grid_cap;
    hipLaunchKernelGGL(aos_recover_kernel, dim3(count), dim3(kRecoverThreads), 0, s, d0,
                       w, tau, count);
    return hipGetLastError();
}

}  // namespace kaze
