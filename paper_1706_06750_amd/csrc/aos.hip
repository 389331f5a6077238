// Semi-implicit step of Eq. 4 by additive operator splitting (AOS):
//   L_i = L_{i-1} + (delta_x + delta_y) / 2,
//   (I - 2 tau A_l(g)) delta_l = 2 tau A_l(g) L_{i-1},   l in {rows, columns},
// where A_l is the 1-D nonlinear diffusion matrix along rows or columns with
// couplings (g_j + g_k)/2 between neighbours and no flux across the image
// border.  Solving for the increment delta = u - L rather than u keeps the
// FP32 error relative to the change of one step, not to the image.
//
// Every row and column system is solved by a partitioned tridiagonal
// method on TX x TY tiles (64 or 32 each, chosen per batch by the autotuner;
// partitioned / hybrid tridiagonal solvers: Zhang, Cohen & Owens, PPoPP 2010;
// Laszlo, Giles & Appleyard, ACM TOMS 2016):
//
//  1. aos_reduce (one block per tile): the tile of L_{i-1} plus a ring is
//     staged in LDS, the conductivity g is computed there (and written
//     once for step 3), and each tile row and tile column -- a TX- or
//     TY-element chunk of its line -- is reduced by one forward sweep to two equations
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
// chunk.  Tile rows are staged through LDS (the transpose that lets
// one thread walk a row); tile columns are walked by adjacent threads on
// adjacent columns, so every global access is coalesced.
#include "kaze_internal.h"
#include "tile_cond.h"

namespace kaze {
namespace {

constexpr int kBlock = 256;

// v_rcp_f32: <= 1 ulp; the pivots are >= 1 (diagonally dominant rows).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Chunk of M unknowns at line positions pos0 .. pos0+M-1 of a line of n
// pixels.  Acc::g(k), Acc::L(k) give conductivity and level at chunk index
// k in [-1, M] (the ring supplies -1 and M).  Positions past the line end
// are identity rows (decoupled, solution 0).
template <int M, class Acc>
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
    // x_1 = al + be x_0 + P x_{M-1} accumulated along the way.
    float cp = 0.f, dp = 0.f, ep = 1.f, P = 1.f, al = 0.f, be = 0.f;
#pragma unroll 8
    for (int k = 1; k <= M - 2; ++k) {
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
    gp = A.g(M);
    Lp = A.L(M);
    wr = (pos0 + M - 1 < n - 1) ? tau * (g0 + gp) : 0.f;
    const Eq last = aos_row(wl, wr, Lm - L0, Lp - L0);
    E1 = Eq{last.a * ep, last.b - last.a * cp, last.c, last.d - last.a * dp};
    E0 = Eq{first.a, first.b + first.c * be, first.c * P, first.d - first.c * al};
}

// Interior of a chunk by a Thomas sweep with both ends known (z0 at k = 0,
// z1 at k = M-1).  On return x[k] holds the increment of every element.
template <int M, class Acc>
__device__ __forceinline__ void chunk_recover(const Acc& A, int pos0, int n, float tau, float z0,
                                              float z1, float (&x)[M]) {
    float cpa[M];
    float gm = A.g(0), Lm = A.L(0), g0 = A.g(1), L0 = A.L(1);
    float wl = (pos0 + 1 < n) ? tau * (gm + g0) : 0.f;
    float cp = 0.f, dp = 0.f;
#pragma unroll
    for (int k = 1; k <= M - 2; ++k) {
        const float gp = A.g(k + 1), Lp = A.L(k + 1);
        const float wr = (pos0 + k < n - 1) ? tau * (g0 + gp) : 0.f;
        float d = wl * (Lm - L0) + wr * (Lp - L0);
        const float b = 1.f + wl + wr;
        float a = -wl, c = -wr;
        if (k == 1) {
            d -= a * z0;
            a = 0.f;
        }
        if (k == M - 2) {
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
    x[M - 1] = z1;
#pragma unroll
    for (int k = M - 2; k >= 1; --k) x[k] -= cpa[k] * x[k + 1];
}

// LDS accessor of one chunk: element k at offset k * stride (k may be -1).
struct LineAcc {
    const float* gp;  // element 0
    const float* Lp;
    int gs, Ls;       // strides between consecutive chunk elements
    __device__ __forceinline__ float g(int k) const { return gp[k * gs]; }
    __device__ __forceinline__ float L(int k) const { return Lp[k * Ls]; }
};

__device__ __forceinline__ void store_eqs(float* dst, const Eq& e0, const Eq& e1) {
    float4* o = reinterpret_cast<float4*>(dst);
    o[0] = make_float4(e0.a, e0.b, e0.c, e0.d);
    o[1] = make_float4(e1.a, e1.b, e1.c, e1.d);
}

// Row chunks are walked by threads [0, TY), column chunks by threads
// [128, 128 + TX): rows and columns never share a wavefront.
constexpr int kColThread0 = 128;

template <int RG, int TX, int TY, bool COMPUTE_G>
__global__ __launch_bounds__(kBlock) void aos_reduce_kernel(ImageDesc d0, AosWork w, Taps tc,
                                                            float tau, int gmode, float k_host) {
    using G = CondGeom<RG, TX, TY>;
    extern __shared__ float smem[];
    float* sL = smem;
    float* sS = smem + G::offS;
    float* sG = smem + G::offG;
    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    // one block per work item: a grid-stride loop here was measured to
    // double the register demand (spills) without saving launches
    ImageDesc d;
    int lt;
    resolve(d0, w, xcd_contiguous(t, (int)gridDim.x), d, lt);
    if (d.gate && *d.gate <= d.bound) return;  // whole block
    const int W = d.W, H = d.H;
    const int cx = lt % d.ncx, cy = lt / d.ncx;
    const int tx0 = cx * TX, ty0 = cy * TY;

    load_L_ring<G>(d.L, W, H, tx0, ty0, sL);
    if (COMPUTE_G) {
        __syncthreads();
        smooth_tile<G>(sL, sS, tc);
        __syncthreads();
        const float k = d.k ? d.k[0] : k_host;
        const float inv_k2 = 1.f / (k * k);
        float* gout = d.g;
        scharr_pass<G>(sS, [&](int gy, int gx, float m2) {
            const float gval = diffusivity(m2, inv_k2, gmode);
            sG[gy * G::pG + gx] = gval;
            const int y = ty0 - 1 + gy, x = tx0 - 1 + gx;
            if (gy >= 1 && gy <= TY && gx >= 1 && gx <= TX && y < H && x < W)
                gout[(size_t)y * W + x] = gval;
        });
    } else {
        stage_region<G::nGy, G::nGx, G::pG, kBlock>(d.g, W, H, ty0 - 1, tx0 - 1, sG);
    }
    __syncthreads();

    Eq e0, e1;
    if (tid < TY) {
        const int y = ty0 + tid;
        if (y < H) {
            const LineAcc A{sG + (tid + 1) * G::pG + 1, sL + (tid + G::R) * G::pL + G::R, 1, 1};
            chunk_reduce<TX>(A, tx0, W, tau, e0, e1);
            store_eqs(d.rrow + ((size_t)y * d.ncx + cx) * 8, e0, e1);
        }
    } else if (tid >= kColThread0 && tid < kColThread0 + TX) {
        const int c = tid - kColThread0, x = tx0 + c;
        if (x < W) {
            const LineAcc A{sG + G::pG + (c + 1), sL + G::R * G::pL + (c + G::R), G::pG, G::pL};
            chunk_reduce<TY>(A, ty0, H, tau, e0, e1);
            store_eqs(d.rcol + ((size_t)x * d.ncy + cy) * 8, e0, e1);
        }
    }
}

// One wavefront per line; lane p holds chunk p's two interface equations.
__global__ __launch_bounds__(kBlock) void aos_iface_kernel(ImageDesc d0, AosWork w, int count) {
    const int lane = threadIdx.x % kWave;
    const int waves = kBlock / kWave;
    for (int t = blockIdx.x * waves + threadIdx.x / kWave; t < count; t += gridDim.x * waves) {
        ImageDesc d;
        int line;
        resolve(d0, w, t, d, line);
        if (d.gate && *d.gate <= d.bound) continue;  // whole wavefront
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

// Row chunks: threads [0, TY); column chunks: threads [64, 64 + TX).
constexpr int kRecoverThreads = 128;

template <int TX, int TY>
__global__ __launch_bounds__(kRecoverThreads) void aos_recover_kernel(ImageDesc d0, AosWork w,
                                                                      float tau) {
    constexpr int P = TX + 1;
    __shared__ float sL[TY * P];
    __shared__ float sG[TY * P];
    __shared__ float sD[TY * P];
    const int tid = threadIdx.x;
    ImageDesc d;
    int lt;
    resolve(d0, w, xcd_contiguous((int)blockIdx.x, (int)gridDim.x), d, lt);
    if (d.gate && *d.gate <= d.bound) return;  // whole block
    const int W = d.W, H = d.H;
    const int cx = lt % d.ncx, cy = lt / d.ncx;
    const int tx0 = cx * TX, ty0 = cy * TY;
    const bool full = ty0 + TY <= H && tx0 + TX <= W;

    // stage L and g (zero outside the image) in two halves, all loads of a
    // half in flight together
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        constexpr int PER = TX * TY / (2 * kRecoverThreads);
        float vl[PER], vg[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = tid + (half * PER + j) * kRecoverThreads;
            const int y = ty0 + i / TX, x = tx0 + i % TX;
            const bool in = full || (y < H && x < W);
            const size_t o = in ? (size_t)y * W + x : 0;
            vl[j] = in ? d.L[o] : 0.f;
            vg[j] = in ? d.g[o] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = tid + (half * PER + j) * kRecoverThreads;
            sL[(i / TX) * P + i % TX] = vl[j];
            sG[(i / TX) * P + i % TX] = vg[j];
        }
    }
    __syncthreads();

    float xc[TY];
    const int c = tid - 64;
    const bool col_thread = tid >= 64 && c < TX && tx0 + c < W;
    if (tid < TY && ty0 + tid < H) {
        const int y = ty0 + tid;
        const float2 z = reinterpret_cast<const float2*>(d.zrow + ((size_t)y * d.ncx + cx) * 2)[0];
        float xr[TX];
        const LineAcc A{sG + tid * P, sL + tid * P, 1, 1};
        chunk_recover<TX>(A, tx0, W, tau, z.x, z.y, xr);
#pragma unroll
        for (int k = 0; k < TX; ++k) sD[tid * P + k] = xr[k];
    } else if (col_thread) {
        const int x = tx0 + c;
        const float2 z = reinterpret_cast<const float2*>(d.zcol + ((size_t)x * d.ncy + cy) * 2)[0];
        const LineAcc A{sG + c, sL + c, P, P};
        chunk_recover<TY>(A, ty0, H, tau, z.x, z.y, xc);
    }
    __syncthreads();
    if (col_thread) {
        const int x = tx0 + c;
#pragma unroll
        for (int k = 0; k < TY; ++k) {
            const int y = ty0 + k;
            if (y < H) d.Lnext[(size_t)y * W + x] = sL[k * P + c] + 0.5f * (sD[k * P + c] + xc[k]);
        }
    }
}

// Global-memory accessor of one whole line for the probe solves: element
// k of the chunk at pos0, index clamped into the line (positions outside it
// get zero coupling weights in the chunk routines).
struct GlobalLineAcc {
    const float* gp;  // line element 0
    const float* Lp;
    int stride, pos0, n;
    __device__ __forceinline__ int at(int k) const {
        const int i = pos0 + k;
        return (i < 0 ? 0 : (i >= n ? n - 1 : i)) * stride;
    }
    __device__ __forceinline__ float g(int k) const { return gp[at(k)]; }
    __device__ __forceinline__ float L(int k) const { return Lp[at(k)]; }
};

constexpr int kProbeChunk = 64;  // unknowns per lane: lines of up to 64 x 64

// One wavefront per line through a probe window: lines 0..kProbeMax-1 are
// rows y0 + j, lines kProbeMax.. are columns x0 + j.
__global__ __launch_bounds__(kBlock) void aos_probe_kernel(ImageDesc d, const int4* rects,
                                                           int nprobes, float tau, float* delta) {
    const int lane = threadIdx.x % kWave;
    const int wv = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int probe = wv / (2 * kProbeMax), j = wv % (2 * kProbeMax);
    if (probe >= nprobes) return;
    const int4 r = rects[probe];  // x0, y0, w, h
    const bool row = j < kProbeMax;
    const int off = row ? j : j - kProbeMax;
    if (off >= (row ? r.w : r.z)) return;  // whole wavefront
    const int W = d.W, H = d.H;
    const int n = row ? W : H;
    const int line = row ? r.y + off : r.x + off;
    const int win0 = row ? r.x : r.y, win1 = win0 + (row ? r.z : r.w);
    const size_t base = row ? (size_t)line * W : (size_t)line;
    const int stride = row ? 1 : W;
    const int pos0 = lane * kProbeChunk;
    const GlobalLineAcc A{d.g + base, d.L + base, stride, pos0, n};
    Eq e0 = eq_identity(), e1 = eq_identity();
    if (pos0 < n) chunk_reduce<kProbeChunk>(A, pos0, n, tau, e0, e1);
    float z0, z1;
    wave_pcr_pairs(e0, e1, lane, z0, z1);
    if (pos0 < n && pos0 < win1 && pos0 + kProbeChunk > win0) {
        float x[kProbeChunk];
        chunk_recover<kProbeChunk>(A, pos0, n, tau, z0, z1, x);
        float* out = delta + (size_t)probe * 2 * kProbeMax * kProbeMax;
#pragma unroll
        for (int k = 0; k < kProbeChunk; ++k) {
            const int pos = pos0 + k;
            if (pos >= win0 && pos < win1) {
                if (row)
                    out[off * kProbeMax + (pos - win0)] = x[k];
                else
                    out[kProbeMax * kProbeMax + (pos - win0) * kProbeMax + off] = x[k];
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void probe_err_kernel(const float* L, const float* cand, int W,
                                                           const int4* rects, const float* delta,
                                                           unsigned* err) {
    __shared__ float red[kBlock];
    const int4 r = rects[blockIdx.x];
    const float* dl = delta + (size_t)blockIdx.x * 2 * kProbeMax * kProbeMax;
    float m = 0.f;
    for (int i = threadIdx.x; i < r.z * r.w; i += kBlock) {
        const int py = i / r.z, px = i - py * r.z;
        const size_t o = (size_t)(r.y + py) * W + (r.x + px);
        const float exact =
            L[o] + 0.5f * (dl[py * kProbeMax + px] + dl[kProbeMax * kProbeMax + py * kProbeMax + px]);
        float e = fabsf(cand[o] - exact);
        if (!(e <= 3.402823466e38f)) e = __builtin_inff();  // NaN or inf
        m = e > m ? e : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w2 = kBlock / 2; w2 > 0; w2 >>= 1) {
        if ((int)threadIdx.x < w2) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(err, __float_as_uint(red[0]));
}

int work_count(const ImageDesc& d0, const AosWork& w, int tx, int ty, bool lines) {
    if (w.items) return w.count;
    return lines ? d0.H + d0.W : tiles_of(d0.W, d0.H, tx, ty);
}

template <int RG, int TX, int TY>
hipError_t launch_reduce_t(const ImageDesc& d0, const AosWork& w, const Taps& tc, float tau,
                           bool compute_g, int gmode, float k_host, hipStream_t s) {
    const int count = work_count(d0, w, TX, TY, false);
    if (count <= 0) return hipSuccess;
    const size_t lds = (size_t)CondGeom<RG, TX, TY>::floats * sizeof(float);
    if (compute_g)
        hipLaunchKernelGGL((aos_reduce_kernel<RG, TX, TY, true>), dim3(count), dim3(kBlock), lds,
                           s, d0, w, tc, tau, gmode, k_host);
    else
        hipLaunchKernelGGL((aos_reduce_kernel<RG, TX, TY, false>), dim3(count), dim3(kBlock), lds,
                           s, d0, w, tc, tau, gmode, k_host);
    return hipGetLastError();
}

template <int TX, int TY>
hipError_t launch_reduce_s(const ImageDesc& d0, const AosWork& w, const Taps& tc, float tau,
                           bool compute_g, int gmode, float k_host, hipStream_t s) {
    switch (tc.r) {
        case 1: return launch_reduce_t<1, TX, TY>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case 2: return launch_reduce_t<2, TX, TY>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case 3: return launch_reduce_t<3, TX, TY>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case 4: return launch_reduce_t<4, TX, TY>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        default: return hipErrorInvalidValue;
    }
}

template <int TX, int TY>
hipError_t launch_recover_s(const ImageDesc& d0, const AosWork& w, float tau, hipStream_t s) {
    const int count = work_count(d0, w, TX, TY, false);
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((aos_recover_kernel<TX, TY>), dim3(count), dim3(kRecoverThreads), 0, s, d0,
                       w, tau);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_aos_reduce(const ImageDesc& d0, const AosWork& w, int shape, const Taps& tc,
                             float tau, bool compute_g, int gmode, float k_host, hipStream_t s) {
    switch (shape) {
        case 0: return launch_reduce_s<64, 64>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case 1: return launch_reduce_s<64, 32>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case 2: return launch_reduce_s<32, 64>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case 3: return launch_reduce_s<32, 32>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aos_iface(const ImageDesc& d0, const AosWork& w, hipStream_t s) {
    const int count = work_count(d0, w, 0, 0, true);
    if (count <= 0) return hipSuccess;
    const int waves = kBlock / kWave;
    hipLaunchKernelGGL(aos_iface_kernel, dim3((count + waves - 1) / waves), dim3(kBlock), 0, s, d0,
                       w, count);
    return hipGetLastError();
}

hipError_t launch_aos_recover(const ImageDesc& d0, const AosWork& w, int shape, float tau,
                              hipStream_t s) {
    switch (shape) {
        case 0: return launch_recover_s<64, 64>(d0, w, tau, s);
        case 1: return launch_recover_s<64, 32>(d0, w, tau, s);
        case 2: return launch_recover_s<32, 64>(d0, w, tau, s);
        case 3: return launch_recover_s<32, 32>(d0, w, tau, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aos_probe(const ImageDesc& d, const int4* rects, int nprobes, float tau,
                            float* delta, hipStream_t s) {
    if (nprobes <= 0) return hipSuccess;
    const int waves = nprobes * 2 * kProbeMax, per = kBlock / kWave;
    hipLaunchKernelGGL(aos_probe_kernel, dim3((waves + per - 1) / per), dim3(kBlock), 0, s, d, rects,
                       nprobes, tau, delta);
    return hipGetLastError();
}

hipError_t launch_probe_err(const float* L, const float* cand, int W, const int4* rects,
                            int nprobes, const float* delta, unsigned* err, hipStream_t s) {
    if (nprobes <= 0) return hipSuccess;
    hipLaunchKernelGGL(probe_err_kernel, dim3(nprobes), dim3(kBlock), 0, s, L, cand, W, rects, delta,
                       err);
    return hipGetLastError();
}

}  // namespace kaze
