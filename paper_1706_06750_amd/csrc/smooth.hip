// Gaussian pre-smoothing, conductivity and contrast factor (Sec. II-A,
// Eqs. 2-3; Sec. III-A).
//
// Stencils stage a 64x64 output tile plus its ring in LDS with half-sample
// symmetric reflection at the image border; a symmetric filter applied to
// that extension is itself half-sample symmetric, so ring values of an
// intermediate (smoothed) image equal the reflected interior values.
#include "kaze.h"
#include "kaze_internal.h"
#include "tile_stage.h"

namespace kaze {
namespace {

// Per image: zero the histogram copies and the keypoint count; set k when it
// is given rather than formed.  NT threads.
template <int NT>
__device__ __forceinline__ void reset_image(const BatchImage& d, int nbins, float k_fill) {
    if (d.hist)
        for (int i = threadIdx.x; i < nbins * kHistCopies; i += NT) ((guint*)d.hist)[i] = 0u;
    if (threadIdx.x == 0) {
        if (d.count) *(__attribute__((address_space(1))) int*)d.count = 0;
        if (k_fill > 0.f && d.k) *(gfloat*)d.k = k_fill;
    }
}

// ---------------------------------------------------------------- G_sigma0
template <int R>
struct GaussGeom {
    static constexpr int n = kTile + 2 * R;   // staged rows and columns
    static constexpr int pI = n | 1;
    static constexpr int pH = kTile | 1;      // horizontal pass: n rows x kTile cols
    static constexpr int offH = n * pI;
    static constexpr int floats = offH + n * pH;
};

// L_0 = G_sigma0 * img on one 64x64 tile: horizontal then vertical pass.
// The first tile of each image also resets the image's counters (the
// gradient, histogram and extrema kernels that use them run later).
template <int R>
__global__ __launch_bounds__(kTileThreads) void gauss_kernel(BatchImage d0, ImgWork work, Taps taps,
                                                               int nbins, float k_fill) {
    using G = GaussGeom<R>;
    constexpr int T = 2 * R + 1;
    extern __shared__ float smem[];
    float* sI = smem;
    float* sH = smem + G::offH;
    BatchImage d;
    int lt;
    resolve(d0, work, xcd_contiguous((int)blockIdx.x, (int)gridDim.x), d, lt);
    if (lt == 0) reset_image<kTileThreads>(d, nbins, k_fill);
    const gfloat* __restrict__ src = (const gfloat*)d.img;
    gfloat* __restrict__ dst = (gfloat*)d.levels;
    const int W = d.W, H = d.H, ld = d.ld;
    const int ncx = (W + kTile - 1) / kTile;
    const int tx0 = (lt % ncx) * kTile, ty0 = (lt / ncx) * kTile;
    // staged load (the source has row pitch ld)
    {
        constexpr int TOTAL = G::n * G::n, PER = (TOTAL + kTileThreads - 1) / kTileThreads;
        const int gy0 = ty0 - R, gx0 = tx0 - R;
        const bool interior = gy0 >= 0 && gx0 >= 0 && gy0 + G::n <= H && gx0 + G::n <= W;
        float v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * kTileThreads;
            if (i < TOTAL) {
                const int ly = i / G::n, lx = i - ly * G::n;
                const int gy = interior ? gy0 + ly : reflect_index(gy0 + ly, H);
                const int gx = interior ? gx0 + lx : reflect_index(gx0 + lx, W);
                v[j] = src[(size_t)gy * ld + gx];
            }
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * kTileThreads;
            if (i < TOTAL) {
                const int ly = i / G::n, lx = i - ly * G::n;
                sI[ly * G::pI + lx] = v[j];
            }
        }
    }
    float w[T];
#pragma unroll
    for (int t = 0; t < T; ++t) w[t] = taps.w[t];
    __syncthreads();
    {
        constexpr int runs = kTile / kRun, items = runs * G::n;
#pragma unroll
        for (int j = 0; j < (items + kTileThreads - 1) / kTileThreads; ++j) {
            const int i = threadIdx.x + j * kTileThreads;
            if (i < items) {
                const int row = i % G::n, x0 = (i / G::n) * kRun;
                const float* p = sI + row * G::pI + x0;
                float v[kRun + T - 1];
#pragma unroll
                for (int q = 0; q < kRun + T - 1; ++q) v[q] = p[q];
#pragma unroll
                for (int q = 0; q < kRun; ++q) {
                    float acc = 0.f;
#pragma unroll
                    for (int t = 0; t < T; ++t) acc += w[t] * v[q + t];
                    sH[row * G::pH + x0 + q] = acc;
                }
            }
        }
    }
    __syncthreads();
    {
        constexpr int runs = kTile / kRun, items = runs * kTile;
#pragma unroll
        for (int j = 0; j < items / kTileThreads; ++j) {
            const int i = threadIdx.x + j * kTileThreads;
            const int col = i % kTile, y0 = (i / kTile) * kRun;
            const float* p = sH + y0 * G::pH + col;
            float v[kRun + T - 1];
#pragma unroll
            for (int q = 0; q < kRun + T - 1; ++q) v[q] = p[q * G::pH];
            const int x = tx0 + col;
#pragma unroll
            for (int q = 0; q < kRun; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < T; ++t) acc += w[t] * v[q + t];
                const int y = ty0 + y0 + q;
                if (x < W && y < H) dst[(size_t)y * W + x] = acc;
            }
        }
    }
}

// max |grad| of an image: the maximum over the per-tile maxima the gradient
// kernel stored (float bits of values >= 0 order like unsigned integers),
// one slot per tile of the given height.  Called by all 256 threads of a
// block.
__device__ __forceinline__ float hmax_of(const BatchImage& d, int tile_h) {
    __shared__ unsigned s_m[256 / kWave];
    const int n = aos_tiles_of(d.W, d.H, tile_h);
    const guint* part = (const guint*)d.hmax;
    unsigned m = 0u;
    for (int i = threadIdx.x; i < n; i += 256) m = max(m, part[i]);
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) s_m[threadIdx.x / kWave] = m;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 256 / kWave; ++j) m = max(m, s_m[j]);
    return __uint_as_float(m);
}

// --------------------------------------------------------------- contrast k
// 300-bin (nbins) histogram of |grad| = sqrt(m2) over pixels with m2 > 0:
// bin = min(floor(|grad|/hmax * nbins), nbins-1).  Integer atomics only, so
// the counts are deterministic.  Device-scope atomics to one address are
// serialised, so block c adds its counts to global copy c % kHistCopies
// (bin b of copy j at hist[j * nbins + b]), and kselect sums the copies.
// Block c bins pixels [c * chunk_px, (c + 1) * chunk_px).
__global__ __launch_bounds__(256) void hist_kernel(BatchImage d0, ImgWork w, int nbins,
                                                     int tile_h, int chunk_px) {
    extern __shared__ unsigned s_hist[];
    BatchImage d;
    int chunk;
    resolve(d0, w, (int)blockIdx.x, d, chunk);
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) s_hist[i] = 0u;
    __syncthreads();
    const float hmax = hmax_of(d, tile_h);
    const float fb = (float)nbins;
    const int n = d.W * d.H;
    const int i0 = chunk * chunk_px, i1 = min(n, i0 + chunk_px);
    // eight loads in flight per thread before any of them is binned
    constexpr int U = 8;
    const gfloat* __restrict__ src = (const gfloat*)d.g;
    for (int i = i0 + threadIdx.x; i < i1; i += U * blockDim.x) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = i + u * (int)blockDim.x;
            v[u] = j < i1 ? src[j] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v[u] > 0.f) {
                const float m = sqrtf(v[u]);
                int b = (int)floorf(m / hmax * fb);
                b = b < nbins - 1 ? b : nbins - 1;
                b = b > 0 ? b : 0;
                atomicAdd(&s_hist[b], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (s_hist[i]) atomicAdd(&d.hist[(chunk % kHistCopies) * nbins + i], s_hist[i]);
}

// Smallest bin b whose cumulative count reaches percentile * npos; k is its
// upper edge hmax*(b+1)/nbins.  No positive gradient: k = 1.  The
// percentile is the exact binary fraction pct_mant * 2^-pct_shift, and the
// test cum >= pct * npos is made exactly in 128-bit integers.  One block:
// per-thread segment sums, a block scan, then each thread searches its
// segment.
__global__ __launch_bounds__(256) void kselect_kernel(BatchImage d0, ImgWork w, int nbins,
                                                        unsigned long long pct_mant,
                                                        int pct_shift, int tile_h) {
    BatchImage d;
    int unused;
    resolve(d0, w, (int)blockIdx.x, d, unused);
    const guint* __restrict__ hist = (const guint*)d.hist;
    __shared__ unsigned long long s_scan[256];
    __shared__ unsigned s_count[KAZE_MAX_K_BINS];  // bin counts summed over the copies
    __shared__ int s_best;
    const int t = threadIdx.x;
    const int seg = (nbins + 255) / 256;
    const int b0 = t * seg, b1 = min(nbins, b0 + seg);
    unsigned long long part = 0;
    for (int b = b0; b < b1; ++b) {
        unsigned c = 0u;
#pragma unroll
        for (int j = 0; j < kHistCopies; ++j) c += hist[j * nbins + b];
        s_count[b] = c;
        part += c;
    }
    s_scan[t] = part;
    if (t == 0) s_best = nbins - 1;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
        const unsigned long long v = t >= off ? s_scan[t - off] : 0ull;
        __syncthreads();
        s_scan[t] += v;
        __syncthreads();
    }
    const unsigned long long npos = s_scan[255];
    if (npos == 0) {
        if (t == 0) d.k[0] = 1.f;
        return;
    }
    const unsigned __int128 rhs = (unsigned __int128)pct_mant * npos;
    unsigned long long cum = s_scan[t] - part;  // exclusive prefix
    for (int b = b0; b < b1; ++b) {
        cum += s_count[b];  // written by this thread
        if (((unsigned __int128)cum << pct_shift) >= rhs) {
            atomicMin(&s_best, b);
            break;
        }
    }
    __syncthreads();
    const float hmax = hmax_of(d, tile_h);  // every thread of the block
    if (t == 0) d.k[0] = (hmax * (float)(s_best + 1)) / (float)nbins;
}

// ------------------------------------------------------------------ utility
__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned* p, int n, unsigned v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// reset_image() of each image on its own (one block per image)
__global__ __launch_bounds__(256) void reset_kernel(BatchImage d0, ImgWork w, int nbins,
                                                      float k_fill) {
    BatchImage d;
    int unused;
    resolve(d0, w, (int)blockIdx.x, d, unused);
    reset_image<256>(d, nbins, k_fill);
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

int item_count(const ImgWork& w, int single) { return w.items ? w.count : single; }

template <int R>
hipError_t launch_gauss_r(const BatchImage& d0, const ImgWork& w, const Taps& taps, int nbins,
                          float k_fill, hipStream_t s) {
    const int count = item_count(w, tiles_of(d0.W, d0.H));
    if (count <= 0) return hipSuccess;
    const size_t lds = (size_t)GaussGeom<R>::floats * sizeof(float);
    hipLaunchKernelGGL(gauss_kernel<R>, dim3(count), dim3(kTileThreads), lds, s, d0, w, taps,
                       nbins, k_fill);
    return hipGetLastError();
}


}  // namespace

hipError_t launch_gauss(const BatchImage& d0, const ImgWork& w, const Taps& taps, int nbins,
                        float k_fill, hipStream_t s) {
    switch (taps.r) {
#define KZ_G(R) \
    case R: return launch_gauss_r<R>(d0, w, taps, nbins, k_fill, s);
        KZ_G(1) KZ_G(2) KZ_G(3) KZ_G(4) KZ_G(5) KZ_G(6) KZ_G(7) KZ_G(8)
        KZ_G(9) KZ_G(10) KZ_G(11) KZ_G(12) KZ_G(13) KZ_G(14) KZ_G(15) KZ_G(16)
#undef KZ_G
        default: return hipErrorInvalidValue;
    }
}


hipError_t launch_hist(const BatchImage& d0, const ImgWork& w, int nbins, int tile_h, int chunk,
                       hipStream_t s) {
    if (chunk < 256) return hipErrorInvalidValue;
    const int count = item_count(w, (d0.W * d0.H + chunk - 1) / chunk);
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(hist_kernel, dim3(count), dim3(256), nbins * sizeof(unsigned), s, d0, w,
                       nbins, tile_h, chunk);
    return hipGetLastError();
}

hipError_t launch_kselect(const BatchImage& d0, const ImgWork& w, int nbins,
                          unsigned long long pct_mant, int pct_shift, int tile_h, hipStream_t s) {
    const int count = item_count(w, 1);
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(kselect_kernel, dim3(count), dim3(256), 0, s, d0, w, nbins, pct_mant,
                       pct_shift, tile_h);
    return hipGetLastError();
}

hipError_t launch_reset(const BatchImage& d0, const ImgWork& w, int nbins, float k_fill,
                        hipStream_t s) {
    const int count = item_count(w, 1);
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_kernel, dim3(count), dim3(256), 0, s, d0, w, nbins, k_fill);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, p, n, v);
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
