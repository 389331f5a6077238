// Gaussian pre-smoothing, conductivity and contrast factor (Sec. II-A,
// Eqs. 2-3; Sec. III-A).
//
// All stencils read a 64x16 output tile plus halo into LDS with
// half-sample symmetric reflection at the image border; a symmetric filter
// applied to that extension is itself half-sample symmetric, so halo values
// of an intermediate (smoothed) image equal the reflected interior values.
#include "kaze_internal.h"
#include "tile_cond.h"

namespace kaze {
namespace {

constexpr int TX = 64;
constexpr int TY = 16;
constexpr int BX = 64;
constexpr int BY = 4;

// G_sigma * src for one tile: horizontal then vertical pass through LDS.
__global__ __launch_bounds__(BX* BY) void gauss_kernel(const float* __restrict__ src, int ld,
                                                         float* __restrict__ dst, int W, int H,
                                                         Taps taps) {
    __shared__ float s_in[(TY + 2 * kMaxRadius) * (TX + 2 * kMaxRadius)];
    __shared__ float s_h[(TY + 2 * kMaxRadius) * TX];
    const int r = taps.r;
    const int iw = TX + 2 * r, ih = TY + 2 * r;
    const int tx0 = blockIdx.x * TX, ty0 = blockIdx.y * TY;
    const int tx = threadIdx.x, ty = threadIdx.y;

    for (int ly = ty; ly < ih; ly += BY) {
        const int gy = reflect_index(ty0 + ly - r, H);
        const float* row = src + (size_t)gy * ld;
        for (int lx = tx; lx < iw; lx += BX)
            s_in[ly * iw + lx] = row[reflect_index(tx0 + lx - r, W)];
    }
    __syncthreads();
    for (int ly = ty; ly < ih; ly += BY) {
        float acc = 0.f;
        for (int j = 0; j <= 2 * r; ++j) acc += taps.w[j] * s_in[ly * iw + tx + j];
        s_h[ly * TX + tx] = acc;
    }
    __syncthreads();
    const int gx = tx0 + tx;
    for (int ly = ty; ly < TY; ly += BY) {
        float acc = 0.f;
        for (int j = 0; j <= 2 * r; ++j) acc += taps.w[j] * s_h[(ly + j) * TX + tx];
        const int gy = ty0 + ly;
        if (gx < W && gy < H) dst[(size_t)gy * W + gx] = acc;
    }
}

// Conductivity of L on 64x64 tiles with the same LDS pipeline as the fused
// AOS reduction (tile_cond.h):
// mode 0: g2 = 1/(1 + |grad|^2/k^2)   (Eq. 3)
// mode 1: g1 = exp(-|grad|^2/k^2)     (Eq. 3)
// mode 2: |grad|^2, and the running maximum of |grad| (for the histogram).
__global__ __launch_bounds__(256) void cond_kernel(const float* __restrict__ L,
                                                     float* __restrict__ out, int W, int H,
                                                     Taps taps, const float* __restrict__ k_dev,
                                                     float k_host, int mode,
                                                     unsigned* __restrict__ hmax_bits) {
    extern __shared__ float smem[];
    __shared__ float s_max[256 / kWave];
    const CondTile ct = cond_tile(taps.r);
    float* sL = smem;
    float* sH = smem + ct.offH;
    float* sS = smem + ct.offS;
    const int ncx = (W + kTile - 1) / kTile;
    const int tx0 = (blockIdx.x % ncx) * kTile, ty0 = (blockIdx.x / ncx) * kTile;
    load_L_ring(L, W, H, tx0, ty0, sL, ct);
    __syncthreads();
    smooth_tile(sL, sH, sS, ct, taps);
    __syncthreads();
    const float k = (mode == 2) ? 1.f : (k_dev ? k_dev[0] : k_host);
    const float inv_k2 = 1.f / (k * k);
    float local_max = 0.f;
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
        const int ly = i / kTile, lx = i % kTile;
        const int y = ty0 + ly, x = tx0 + lx;
        if (y >= H || x >= W) continue;
        const float m2 = scharr_m2(sS, ct.pS, ly + 1, lx + 1);
        float v;
        if (mode == 2) {
            v = m2;
            local_max = fmaxf(local_max, sqrtf(m2));
        } else {
            v = diffusivity(m2, inv_k2, mode);
        }
        out[(size_t)y * W + x] = v;
    }
    if (mode == 2) {
        // wavefront max, then one atomic per block (|grad| >= 0, so the
        // float bit pattern orders like an unsigned integer)
        for (int off = kWave / 2; off > 0; off >>= 1)
            local_max = fmaxf(local_max, __shfl_xor(local_max, off, kWave));
        const int t = threadIdx.x;
        if ((t & (kWave - 1)) == 0) s_max[t / kWave] = local_max;
        __syncthreads();
        if (t == 0) {
            float m = s_max[0];
            for (int i = 1; i < 256 / kWave; ++i) m = fmaxf(m, s_max[i]);
            atomicMax(hmax_bits, __float_as_uint(m));
        }
    }
}

// 300-bin (nbins) histogram of |grad| = sqrt(m2) over pixels with m2 > 0:
// bin = min(floor(|grad|/hmax * nbins), nbins-1).  Integer atomics only, so
// the counts are deterministic.
__global__ __launch_bounds__(256) void hist_kernel(const float* __restrict__ m2, int n,
                                                     const unsigned* __restrict__ hmax_bits,
                                                     unsigned* __restrict__ hist, int nbins) {
    extern __shared__ unsigned s_hist[];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) s_hist[i] = 0u;
    __syncthreads();
    const float hmax = __uint_as_float(hmax_bits[0]);
    const float fb = (float)nbins;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float v = m2[i];
        if (v > 0.f) {
            const float m = sqrtf(v);
            int b = (int)floorf(m / hmax * fb);
            b = b < nbins - 1 ? b : nbins - 1;
            b = b > 0 ? b : 0;
            atomicAdd(&s_hist[b], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (s_hist[i]) atomicAdd(&hist[i], s_hist[i]);
}

// Smallest bin b whose cumulative count reaches percentile * npos; k is its
// upper edge hmax*(b+1)/nbins.  No positive gradient: k = 1.  The
// percentile is the exact binary fraction pct_mant * 2^-pct_shift, and the
// test cum >= pct * npos is made exactly in 128-bit integers.
__global__ void kselect_kernel(const unsigned* __restrict__ hist, int nbins,
                               const unsigned* __restrict__ hmax_bits,
                               unsigned long long pct_mant, int pct_shift,
                               float* __restrict__ k_out) {
    if (threadIdx.x != 0) return;
    unsigned long long npos = 0;
    for (int i = 0; i < nbins; ++i) npos += hist[i];
    if (npos == 0) {
        k_out[0] = 1.f;
        return;
    }
    const unsigned __int128 rhs = (unsigned __int128)pct_mant * npos;
    unsigned long long cum = 0;
    int b = nbins - 1;
    for (int i = 0; i < nbins; ++i) {
        cum += hist[i];
        if (((unsigned __int128)cum << pct_shift) >= rhs) {
            b = i;
            break;
        }
    }
    const float hmax = __uint_as_float(hmax_bits[0]);
    k_out[0] = (hmax * (float)(b + 1)) / (float)nbins;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned* p, int n, unsigned v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void fill_f32_kernel(float* p, int n, float v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Streaming copy with 16-byte vector accesses (bandwidth reference).
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                     float4* __restrict__ dst, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void copy_tail_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                 size_t start, size_t n) {
    const size_t i = start + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

int grid_for(size_t n, int block, int cap) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (int)(g < (size_t)cap ? g : (size_t)cap);
}

}  // namespace

hipError_t launch_gauss(const float* src, int ld_src, float* dst, int W, int H,
                        const Taps& taps, hipStream_t s) {
    dim3 grid((W + TX - 1) / TX, (H + TY - 1) / TY), block(BX, BY);
    hipLaunchKernelGGL(gauss_kernel, grid, block, 0, s, src, ld_src, dst, W, H, taps);
    return hipGetLastError();
}

hipError_t launch_cond(const float* L, float* out, int W, int H, const Taps& taps,
                       const float* k_dev, float k_host, int mode, unsigned* hmax_bits,
                       hipStream_t s) {
    const size_t lds = (size_t)cond_tile(taps.r).floats * sizeof(float);
    hipLaunchKernelGGL(cond_kernel, dim3(tiles_of(W, H)), dim3(256), lds, s, L, out, W, H, taps,
                       k_dev, k_host, mode, hmax_bits);
    return hipGetLastError();
}

hipError_t launch_hist(const float* m2, int n, const unsigned* hmax_bits, unsigned* hist,
                       int nbins, hipStream_t s) {
    hipLaunchKernelGGL(hist_kernel, dim3(grid_for(n, 256, 1024)), dim3(256),
                       nbins * sizeof(unsigned), s, m2, n, hmax_bits, hist, nbins);
    return hipGetLastError();
}

hipError_t launch_kselect(const unsigned* hist, int nbins, const unsigned* hmax_bits,
                          unsigned long long pct_mant, int pct_shift, float* k_out,
                          hipStream_t s) {
    hipLaunchKernelGGL(kselect_kernel, dim3(1), dim3(64), 0, s, hist, nbins, hmax_bits,
                       pct_mant, pct_shift, k_out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int n, float v, hipStream_t s) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s) {
    const size_t n4 = n / 4;
    if (n4 > 0) {
        hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n4, 256, 8192)), dim3(256), 0, s,
                           reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n4);
    }
    if (n % 4) {
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(4), 0, s, src, dst, n4 * 4, n);
    }
    return hipGetLastError();
}

}  // namespace kaze
