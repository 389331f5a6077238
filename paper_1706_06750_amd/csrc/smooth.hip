// Gaussian pre-smoothing, conductivity and contrast factor (Sec. II-A,
// Eqs. 2-3; Sec. III-A).
//
// All stencils read a 64x16 output tile plus halo into LDS with
// half-sample symmetric reflection at the image border; a symmetric filter
// applied to that extension is itself half-sample symmetric, so halo values
// of an intermediate (smoothed) image equal the reflected interior values.
#include "kaze_internal.h"

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

// Squared Scharr gradient magnitude of G_sigma_cond * L on one tile, then
// mode 0: g2 = 1/(1 + |grad|^2/k^2)   (Eq. 3)
// mode 1: g1 = exp(-|grad|^2/k^2)     (Eq. 3)
// mode 2: |grad|^2, and the running maximum of |grad| (for the histogram).
__global__ __launch_bounds__(BX* BY) void cond_kernel(const float* __restrict__ L,
                                                        float* __restrict__ out, int W, int H,
                                                        Taps taps, const float* __restrict__ k_dev,
                                                        float k_host, int mode,
                                                        unsigned* __restrict__ hmax_bits) {
    constexpr int RH = kMaxRadius + 1;
    __shared__ float s_in[(TY + 2 * RH) * (TX + 2 * RH)];
    __shared__ float s_h[(TY + 2 * RH) * (TX + 2)];
    __shared__ float s_s[(TY + 2) * (TX + 2)];
    __shared__ float s_max[BX * BY / kWave];
    const int r = taps.r;
    const int rh = r + 1;
    const int iw = TX + 2 * rh, ih = TY + 2 * rh;
    const int tx0 = blockIdx.x * TX, ty0 = blockIdx.y * TY;
    const int tx = threadIdx.x, ty = threadIdx.y;

    for (int ly = ty; ly < ih; ly += BY) {
        const int gy = reflect_index(ty0 + ly - rh, H);
        const float* row = L + (size_t)gy * W;
        for (int lx = tx; lx < iw; lx += BX)
            s_in[ly * iw + lx] = row[reflect_index(tx0 + lx - rh, W)];
    }
    __syncthreads();
    // horizontal pass on columns -1..TX of the tile
    constexpr int HW = TX + 2;
    for (int ly = ty; ly < ih; ly += BY) {
        for (int lx = tx; lx < HW; lx += BX) {
            float acc = 0.f;
            for (int j = 0; j <= 2 * r; ++j) acc += taps.w[j] * s_in[ly * iw + lx + j];
            s_h[ly * HW + lx] = acc;
        }
    }
    __syncthreads();
    // vertical pass on rows -1..TY
    for (int ly = ty; ly < TY + 2; ly += BY) {
        for (int lx = tx; lx < HW; lx += BX) {
            float acc = 0.f;
            for (int j = 0; j <= 2 * r; ++j) acc += taps.w[j] * s_h[(ly + j) * HW + lx];
            s_s[ly * HW + lx] = acc;
        }
    }
    __syncthreads();
    const float k = (mode == 2) ? 1.f : (k_dev ? k_dev[0] : k_host);
    const float inv_k2 = 1.f / (k * k);
    const int gx = tx0 + tx;
    float local_max = 0.f;
    for (int ly = ty; ly < TY; ly += BY) {
        const int cy = ly + 1, cx = tx + 1;
        // Scharr: central difference /2 across, [3 10 3]/16 along
        const float dxm = 0.5f * (s_s[(cy - 1) * HW + cx + 1] - s_s[(cy - 1) * HW + cx - 1]);
        const float dx0 = 0.5f * (s_s[cy * HW + cx + 1] - s_s[cy * HW + cx - 1]);
        const float dxp = 0.5f * (s_s[(cy + 1) * HW + cx + 1] - s_s[(cy + 1) * HW + cx - 1]);
        const float dym = 0.5f * (s_s[(cy + 1) * HW + cx - 1] - s_s[(cy - 1) * HW + cx - 1]);
        const float dy0 = 0.5f * (s_s[(cy + 1) * HW + cx] - s_s[(cy - 1) * HW + cx]);
        const float dyp = 0.5f * (s_s[(cy + 1) * HW + cx + 1] - s_s[(cy - 1) * HW + cx + 1]);
        const float lx = 0.1875f * dxm + 0.625f * dx0 + 0.1875f * dxp;
        const float ly_ = 0.1875f * dym + 0.625f * dy0 + 0.1875f * dyp;
        const float m2 = lx * lx + ly_ * ly_;
        const int gy = ty0 + ly;
        const bool in = gx < W && gy < H;
        float v;
        if (mode == 0)
            v = 1.f / (1.f + m2 * inv_k2);
        else if (mode == 1)
            v = expf(-m2 * inv_k2);
        else {
            v = m2;
            if (in) local_max = fmaxf(local_max, sqrtf(m2));
        }
        if (in) out[(size_t)gy * W + gx] = v;
    }
    if (mode == 2) {
        // wavefront max, then one atomic per block (|grad| >= 0, so the
        // float bit pattern orders like an unsigned integer)
        for (int off = 32; off > 0; off >>= 1)
            local_max = fmaxf(local_max, __shfl_xor(local_max, off, kWave));
        const int t = ty * BX + tx;
        if ((t & (kWave - 1)) == 0) s_max[t / kWave] = local_max;
        __syncthreads();
        if (t == 0) {
            float m = s_max[0];
            for (int i = 1; i < BX * BY / kWave; ++i) m = fmaxf(m, s_max[i]);
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

__global__ __launch_bounds__(256) void g_from_m2_kernel(float* __restrict__ buf, int n,
                                                          const float* __restrict__ k_dev, int mode) {
    const float k = k_dev[0];
    const float inv_k2 = 1.f / (k * k);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float m2 = buf[i];
        buf[i] = (mode == 0) ? 1.f / (1.f + m2 * inv_k2) : expf(-m2 * inv_k2);
    }
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
    dim3 grid((W + TX - 1) / TX, (H + TY - 1) / TY), block(BX, BY);
    hipLaunchKernelGGL(cond_kernel, grid, block, 0, s, L, out, W, H, taps, k_dev, k_host, mode,
                       hmax_bits);
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

hipError_t launch_g_from_m2(float* buf, int n, const float* k_dev, int mode, hipStream_t s) {
    hipLaunchKernelGGL(g_from_m2_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, buf, n,
                       k_dev, mode);
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
