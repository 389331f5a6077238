// Learned surrogate of one AOS step: kernels.
//
// The network is six 3x3 convolutions (cross-correlation, zero padding)
// 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 with ReLU after layers 1..5; its
// output f = (layer 6) / 64 is the residual of the step, L_next ~ L + f.  Inputs are the
// previous level L, its conductivity g and the plane tau / 68.
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation.  Forward and input gradient share one kernel:
//   D[o][p] = sum_{t, c} A_t[o][c] * In[p + t][c],
// A operand = packed weights (16 output channels x 32 K values per
// fragment, kept in VGPRs for the wave's lifetime), B operand = 8 channels
// of one pixel per lane (16 contiguous bytes of an NHWC row), one output
// row of 16 pixels per MFMA column block.  A wave sweeps down a 16-pixel
// strip and keeps the three input rows of the 3x3 window in registers, so
// each input row is loaded once per strip.
//
// Layer 1 uses a three-term BF16 split so that L and g enter with ~16
// significant bits: channels (L_hi, L_lo, L_hi, g_hi, g_lo, g_hi) against
// weights (wL_hi, wL_hi, wL_lo, wg_hi, wg_hi, wg_lo).  The constant tau
// plane is added in the FP32 epilogue from FP32 tap weights (only the taps
// that fall inside the image).
//
// The weight gradient reduces over pixels: K = 32 consecutive pixels of one
// row, read from planar copies (one channel row contiguous) of the layer
// input and of dZ; the tap's column shift is applied in registers with
// byte alignment.  Per-wave partial sums are reduced in a fixed order, so
// every result is deterministic.
#include <algorithm>
#include <atomic>

#include "kaze_internal.h"
#include "sg_internal.h"

namespace kaze {
namespace sg {
namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline bf16x8 zero8() {
    u32x4 z = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(bf16x8, z);
}

__device__ inline bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Workgroup barrier for exchanges through LDS only: waits for the wave's LDS
// accesses, not for its global loads, so rows prefetched into registers stay
// in flight across it (a full __syncthreads also waits for every outstanding
// global load).  The memory clobber keeps the compiler from moving LDS
// accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ------------------------------------------------------------- convolution
template <int CIN>
struct ConvK {
    static constexpr int KS = CIN == 32 ? 9 : 3;  // MFMA K steps per output row
};

// Epilogue for one output row: acc[mb][r] holds output channel 16 mb + 4 q + r
// of pixel x.
template <int MB, int EPI, bool TAU>
__device__ inline void conv_epilogue(const ConvArgs& a, const Geo& g, int s, int y, int x, int q,
                                     const f32x4 (&acc)[MB], const float (&bias)[MB][4],
                                     const float (&tcs)[MB][4][3]) {
    if (x >= g.W) return;
    const size_t pix = (size_t)s * g.sx + (size_t)(y + 1) * g.pw + (x + 1);
    if constexpr (EPI == EPI_OUT) {
        if (q != 0) return;
        const float f = (acc[0][0] + bias[0][0]) * kOutScale;
        const size_t o = ((size_t)s * g.H + y) * g.W + x;
        a.fout[o] = a.base ? a.base[o] + f : f;
        return;
    } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float z = acc[mb][r];
                if constexpr (EPI == EPI_RELU) {
                    z += bias[mb][r];
                    if constexpr (TAU) {  // tau-plane taps inside the image
                        z += tcs[mb][r][1];
                        if (y >= 1) z += tcs[mb][r][0];
                        if (y + 1 < g.H) z += tcs[mb][r][2];
                    }
                    z = z > 0.f ? z : 0.f;
                }
                v[r] = z;
            }
            if constexpr (EPI == EPI_MASK) {
                const bf16x4 m =
                    *reinterpret_cast<const bf16x4*>(a.mask + pix * kCh + 16 * mb + 4 * q);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = (float)m[r] > 0.f ? v[r] : 0.f;
            }
            bf16x4 o = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
            if (a.out) *reinterpret_cast<bf16x4*>(a.out + pix * kCh + 16 * mb + 4 * q) = o;
            if (a.outp) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 16 * mb + 4 * q + r;
                    size_t idx;
                    if constexpr (EPI == EPI_RELU)  // planar X: ring included
                        idx = (((size_t)s * (g.H + 2) + y + 1) * kCh + c) * g.PX + x + 1;
                    else  // planar dZ
                        idx = (((size_t)s * g.H + y) * kCh + c) * g.PZ + x;
                    a.outp[idx] = o[r];
                }
            }
        }
    }
}

template <int CIN, int MB, int EPI, bool TAU>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a, Geo g) {
    constexpr int KS = ConvK<CIN>::KS;
    const int lane = threadIdx.x & 63;
    const int item = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
    int s, rem;
    if (a.bw.imgs) {  // batched inference: this wave's image and its planes
        if (item >= a.bw.count) return;  // whole wave
        const int2 it = a.bw.items[item];
        const SgImage im = a.bw.imgs[it.x];
        if (a.gate && !(*im.gate <= a.bound)) return;  // whole wave
        g = image_geo(im.W, im.H, g.R);
        a.in += im.xoff * CIN;
        if (a.out) a.out += im.xoff * kCh;
        a.fout = im.Lnext;
        a.base = im.L;
        s = 0;
        rem = it.y;
    } else {
        if (a.gate && !(*a.gate <= a.bound)) return;  // whole grid
        const int per = g.strips * g.chunks;
        if (a.items) {
            if (item >= a.nitems) return;  // whole wave
            s = 0;
            rem = a.items[item];
        } else {
            if (item >= g.n * per) return;  // whole wave
            s = item / per;
            rem = item - s * per;
        }
    }
    const int chunk = rem / g.strips;
    const int strip = rem - chunk * g.strips;
    const int y0 = chunk * g.R, y1 = min(g.H, y0 + g.R);
    const int j = lane & 15, q = lane >> 4;
    const int x = strip * kStrip + j;
    const int xl = min(x, g.W - 1);  // ragged lanes read inside the padded row

    bf16x8 wf[MB][KS];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int k = 0; k < KS; ++k) wf[mb][k] = a.wfrag[(mb * KS + k) * 64 + lane];
    float bias[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[mb][r] = (EPI == EPI_MASK) ? 0.f : a.bias[16 * mb + 4 * q + r];
    // layer 1: per output channel and tap row, tau / 68 times the sum of the
    // tau-plane tap weights whose column lies inside the image
    float tcs[MB][4][3];
    if constexpr (TAU) {
        const float taup = a.tau[s] / kTauRef;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int ty = 0; ty < 3; ++ty) {
                    const int co = 16 * mb + 4 * q + r;
                    float t = 0.f;
#pragma unroll
                    for (int tx = 0; tx < 3; ++tx) {
                        const int xx = x + tx - 1;
                        if (xx >= 0 && xx < g.W) t += a.tauw[co * 9 + ty * 3 + tx];
                    }
                    tcs[mb][r][ty] = taup * t;
                }
    }

    // lane's column base: padded pixel (row 0, column xl) of sample s
    const bf16* col = a.in + ((size_t)s * g.sx + xl) * CIN;
    const size_t rowstride = (size_t)g.pw * CIN;

    if constexpr (CIN == 32) {
        const bf16* cq = col + 8 * q;
        // fragments of padded row yp at column offsets 0, 1, 2 (taps dx = -1, 0, +1)
#define KZ_LOADROW(R, yp)                                   \
    {                                                       \
        const bf16* p_ = cq + (size_t)(yp) * rowstride;     \
        R[0] = ld8(p_);                                     \
        R[1] = ld8(p_ + CIN);                               \
        R[2] = ld8(p_ + 2 * CIN);                           \
    }
#define KZ_STEP(yy, RA, RB, RC, RD)                                                   \
    {                                                                                 \
        if ((yy) + 1 < y1) KZ_LOADROW(RD, (yy) + 3)                                   \
        f32x4 acc[MB];                                                                \
        _Pragma("unroll") for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f}; \
        _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                              \
            _Pragma("unroll") for (int mb = 0; mb < MB; ++mb)                         \
                acc[mb] = mfma(wf[mb][dx], RA[dx], acc[mb]);                          \
        _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                              \
            _Pragma("unroll") for (int mb = 0; mb < MB; ++mb)                         \
                acc[mb] = mfma(wf[mb][3 + dx], RB[dx], acc[mb]);                      \
        _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                              \
            _Pragma("unroll") for (int mb = 0; mb < MB; ++mb)                         \
                acc[mb] = mfma(wf[mb][6 + dx], RC[dx], acc[mb]);                      \
        conv_epilogue<MB, EPI, TAU>(a, g, s, (yy), x, q, acc, bias, tcs);             \
    }
        // padded rows y, y+1, y+2 feed output row y; row y+3 is loaded one
        // step ahead
        bf16x8 ra[3], rb[3], rc[3], rd[3];
        KZ_LOADROW(ra, y0)
        KZ_LOADROW(rb, y0 + 1)
        KZ_LOADROW(rc, y0 + 2)
        for (int y = y0; y < y1; y += 4) {
            KZ_STEP(y, ra, rb, rc, rd)
            if (y + 1 < y1) KZ_STEP(y + 1, rb, rc, rd, ra)
            if (y + 2 < y1) KZ_STEP(y + 2, rc, rd, ra, rb)
            if (y + 3 < y1) KZ_STEP(y + 3, rd, ra, rb, rc)
        }
#undef KZ_STEP
#undef KZ_LOADROW
    } else {
        // CIN = 8: K step k covers taps 4k + q (taps >= 9 are zero)
        for (int y = y0; y < y1; ++y) {
            bf16x8 b[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int t = 4 * k + q;
                b[k] = t < 9 ? ld8(col + (size_t)(y + t / 3) * rowstride + (t % 3) * CIN) : zero8();
            }
            f32x4 acc[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < KS; ++k) acc[mb] = mfma(wf[mb][k], b[k], acc[mb]);
            }
            conv_epilogue<MB, EPI, TAU>(a, g, s, y, x, q, acc, bias, tcs);
        }
    }
}

// ------------------------------------------------- two layers in one pass
// Inference: layer a (CINA -> 32, ReLU) and layer b (32 -> 32 with ReLU, or
// 32 -> 1 output) over a strip of kPairOut output columns and R rows, with
// layer a's output kept on chip.  Waves 0-7 ("A") compute layer a on the
// kPairMid columns [x0 - 8, x0 + 120), one 16-column block each, into a ring
// of 4 rows in LDS; positions outside the image are stored as zero, which is
// layer b's zero padding.  Waves 8-11 ("B") compute layer b on 7 blocks of
// 16 columns from that ring.  At step t the A waves produce row y0 - 1 + t
// and the B waves output row y0 + t - 3 from the rows produced at steps
// t-3 .. t-1, so one barrier per step separates writers and readers.  Every
// value is computed by the same MFMA sequence as in conv_kernel, so the
// results are bitwise those of two conv_kernel launches.

constexpr int kPairMid = 128;           // layer-a columns per block (8 blocks)
constexpr int kPairPix = 40;            // LDS pitch of one pixel in BF16 (80 B)
constexpr int kPairThreads = 768;       // 8 A waves + 4 B waves

template <int CINA, int MBB, bool TAU>
__global__ __launch_bounds__(kPairThreads) void conv2_kernel(Conv2Args a, Geo g) {
    constexpr int KSA = CINA == 32 ? 9 : 3;
    __shared__ __align__(16) bf16 ring[4][kPairMid * kPairPix];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, q = lane >> 4;
    int s, strip, chunk;
    if (a.bw.imgs) {  // batched inference: this block's image and its planes
        const int t = blockIdx.x;
        if (t >= a.bw.count) return;  // whole block
        const int2 it = a.bw.items[t];
        const SgImage im = a.bw.imgs[it.x];
        if (a.gate && !(*im.gate <= a.bound)) return;  // whole block
        g = image_geo(im.W, im.H, g.R);
        g.strips = (im.W + kPairOut - 1) / kPairOut;
        a.in += im.xoff * CINA;
        if constexpr (MBB == 2) {
            a.out += im.xoff * kCh;
        } else {
            a.fout = im.Lnext;
            a.base = im.L;
        }
        s = 0;
        strip = it.y % g.strips;
        chunk = it.y / g.strips;
    } else {
        if (a.gate && !(*a.gate <= a.bound)) return;  // whole grid
        s = blockIdx.y;
        strip = (int)blockIdx.x % g.strips;
        chunk = (int)blockIdx.x / g.strips;
    }
    const int x0 = strip * kPairOut, y0 = chunk * g.R, y1 = min(g.H, y0 + g.R);
    const int steps = (y1 - y0) + 3;

    if (wv < 8) {
        // ---------------------------------------------------------- A waves
        const int xm = x0 - 8 + 16 * wv + j;  // this lane's layer-a column
        const bool colok = xm >= 0 && xm < g.W;
        const int xl = min(max(xm, 0), g.W - 1);
        bf16x8 wf[2][KSA];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int k = 0; k < KSA; ++k) wf[mb][k] = a.wa[(mb * KSA + k) * 64 + lane];
        float bias[2][4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) bias[mb][r] = a.ba[16 * mb + 4 * q + r];
        float tcs[2][4][3];
        if constexpr (TAU) {
            const float taup = a.tau[s] / kTauRef;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int ty = 0; ty < 3; ++ty) {
                        const int co = 16 * mb + 4 * q + r;
                        float t = 0.f;
#pragma unroll
                        for (int tx = 0; tx < 3; ++tx) {
                            const int xx = xm + tx - 1;
                            if (xx >= 0 && xx < g.W) t += a.tauw[co * 9 + ty * 3 + tx];
                        }
                        tcs[mb][r][ty] = taup * t;
                    }
        }
        const bf16* col = a.in + ((size_t)s * g.sx + xl) * CINA;
        const size_t rowstride = (size_t)g.pw * CINA;
        bf16* mid = &ring[0][0] + (16 * wv + j) * kPairPix;  // + slot * kPairMid * kPairPix

        // stores layer a's row ya (zero outside the image) into ring slot sl
        auto store_row = [&](int sl, int ya, const f32x4 (&acc)[2]) {
            const bool ok = colok && ya >= 0 && ya < g.H;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float z = acc[mb][r] + bias[mb][r];
                    if constexpr (TAU) {
                        z += tcs[mb][r][1];
                        if (ya >= 1) z += tcs[mb][r][0];
                        if (ya + 1 < g.H) z += tcs[mb][r][2];
                    }
                    z = z > 0.f ? z : 0.f;
                    v[r] = ok ? z : 0.f;
                }
                const bf16x4 o = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
                *reinterpret_cast<bf16x4*>(mid + sl * kPairMid * kPairPix + 16 * mb + 4 * q) = o;
            }
        };

        if constexpr (CINA == 32) {
            const bf16* cq = col + 8 * q;
#define KZ_LOADROW(R, yp)                                                 \
    {                                                                     \
        const int yp_ = (yp);                                             \
        if (yp_ >= 0 && yp_ <= g.H + 1) {                                 \
            const bf16* p_ = cq + (size_t)yp_ * rowstride;                \
            R[0] = ld8(p_);                                               \
            R[1] = ld8(p_ + CINA);                                        \
            R[2] = ld8(p_ + 2 * CINA);                                    \
        }                                                                 \
    }
            // layer-a row ya reads padded rows ya, ya+1, ya+2; the ring of
            // five holds them with rows ya+3 and ya+4 loaded one and two
            // steps ahead
#define KZ_ASTEP(tt, RA, RB, RC, RE)                                                          \
    {                                                                                         \
        const int ya_ = y0 - 1 + (tt);                                                        \
        if ((tt) < steps) {                                                                   \
            if ((tt) <= steps - 4) KZ_LOADROW(RE, ya_ + 4)                                    \
            f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};           \
            if (ya_ >= 0 && ya_ < g.H && (tt) <= steps - 2) {                                 \
                _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                              \
                    _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                          \
                        acc[mb] = mfma(wf[mb][dx], RA[dx], acc[mb]);                          \
                _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                              \
                    _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                          \
                        acc[mb] = mfma(wf[mb][3 + dx], RB[dx], acc[mb]);                      \
                _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                              \
                    _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                          \
                        acc[mb] = mfma(wf[mb][6 + dx], RC[dx], acc[mb]);                      \
            }                                                                                 \
            if ((tt) <= steps - 2) store_row((tt) & 3, ya_, acc);                             \
            lds_barrier();                                                                      \
        }                                                                                     \
    }
            bf16x8 ra[3], rb[3], rc[3], rd[3], re[3];
            KZ_LOADROW(ra, y0 - 1)
            KZ_LOADROW(rb, y0)
            KZ_LOADROW(rc, y0 + 1)
            KZ_LOADROW(rd, y0 + 2)
            for (int t = 0; t < steps; t += 5) {
                KZ_ASTEP(t, ra, rb, rc, re)
                KZ_ASTEP(t + 1, rb, rc, rd, ra)
                KZ_ASTEP(t + 2, rc, rd, re, rb)
                KZ_ASTEP(t + 3, rd, re, ra, rc)
                KZ_ASTEP(t + 4, re, ra, rb, rd)
            }
#undef KZ_ASTEP
#undef KZ_LOADROW
        } else {
            for (int t = 0; t < steps; ++t) {
                const int ya = y0 - 1 + t;
                if (t <= steps - 2) {
                    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
                    if (ya >= 0 && ya < g.H) {
                        bf16x8 b[KSA];
#pragma unroll
                        for (int k = 0; k < KSA; ++k) {
                            const int tp = 4 * k + q;
                            b[k] = tp < 9 ? ld8(col + (size_t)(ya + tp / 3) * rowstride + (tp % 3) * CINA)
                                          : zero8();
                        }
#pragma unroll
                        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                            for (int k = 0; k < KSA; ++k) acc[mb] = mfma(wf[mb][k], b[k], acc[mb]);
                    }
                    store_row(t & 3, ya, acc);
                }
                lds_barrier();    
            }
        }
    } else {
        // ---------------------------------------------------------- B waves
        const int bw = wv - 8;  // output blocks 2 bw, 2 bw + 1 (block 7 does not exist)
        bf16x8 wf[MBB][9];
#pragma unroll
        for (int mb = 0; mb < MBB; ++mb)
#pragma unroll
            for (int k = 0; k < 9; ++k) wf[mb][k] = a.wb[(mb * 9 + k) * 64 + lane];
        float bias[MBB][4];
#pragma unroll
        for (int mb = 0; mb < MBB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) bias[mb][r] = a.bb[16 * mb + 4 * q + r];
        const int nblk = bw < 3 ? 2 : 1;
        for (int t = 0; t < steps; ++t) {
            if (t >= 3) {
                const int yb = y0 + t - 3;
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    if (kb >= nblk) continue;
                    const int k = 2 * bw + kb;
                    const int x = x0 + 16 * k + j;
                    f32x4 acc[MBB];
#pragma unroll
                    for (int mb = 0; mb < MBB; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ty = 0; ty < 3; ++ty) {
                        const bf16* rowp = &ring[(t - 3 + ty) & 3][0] + (16 * k + j + 7) * kPairPix + 8 * q;
                        bf16x8 bv[3];
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx)
                            bv[dx] = *reinterpret_cast<const bf16x8*>(rowp + dx * kPairPix);
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                            for (int mb = 0; mb < MBB; ++mb)
                                acc[mb] = mfma(wf[mb][3 * ty + dx], bv[dx], acc[mb]);
                    }
                    if (x < g.W) {
                        if constexpr (MBB == 1) {
                            if (q == 0) {
                                const float f = (acc[0][0] + bias[0][0]) * kOutScale;
                                const size_t o = ((size_t)s * g.H + yb) * g.W + x;
                                a.fout[o] = a.base ? a.base[o] + f : f;
                            }
                        } else {
                            const size_t pix = (size_t)s * g.sx + (size_t)(yb + 1) * g.pw + (x + 1);
#pragma unroll
                            for (int mb = 0; mb < MBB; ++mb) {
                                float v[4];
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    const float z = acc[mb][r] + bias[mb][r];
                                    v[r] = z > 0.f ? z : 0.f;
                                }
                                const bf16x4 o = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
                                *reinterpret_cast<bf16x4*>(a.out + pix * kCh + 16 * mb + 4 * q) = o;
                            }
                        }
                    }
                }
            }
            lds_barrier();    
        }
    }
}

// ------------------------------------------------------------ input packing
// NHWC8: (L_hi, L_lo, L_hi, g_hi, g_lo, g_hi, 0, 0); planar (weight
// gradient of layer 1): (L_hi, L_lo, g_hi, g_lo, tau_hi, tau_lo, 0, 0).
__device__ inline bf16x8 input_split(float l, float c) {
    const bf16 lh = (bf16)l, ch = (bf16)c;
    const bf16 ll = (bf16)(l - (float)lh), cl = (bf16)(c - (float)ch);
    const bf16 z = (bf16)0.f;
    return bf16x8{lh, ll, lh, ch, cl, ch, z, z};
}

// Batched layer-1 input: blockIdx.y is the image; its pixels are walked with
// a grid stride over blockIdx.x.
__global__ __launch_bounds__(256) void pack_input_batch_kernel(const SgImage* __restrict__ imgs,
                                                               bf16* __restrict__ x0) {
    const SgImage im = imgs[blockIdx.y];
    const size_t per = (size_t)im.W * im.H;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / im.W), x = (int)(i - (size_t)y * im.W);
        const size_t pix = (size_t)im.xoff + (size_t)(y + 1) * (im.W + 2) + (x + 1);
        *reinterpret_cast<bf16x8*>(x0 + pix * 8) = input_split(im.L[i], im.g[i]);
    }
}

__global__ void pack_input_kernel(const float* __restrict__ L, const float* __restrict__ gc,
                                  const float* __restrict__ tau, bf16* __restrict__ x0,
                                  bf16* __restrict__ x0p, Geo g) {
    const size_t per = (size_t)g.W * g.H;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= per * g.n) return;
    const int s = (int)(i / per);
    const size_t r = i - (size_t)s * per;
    const int y = (int)(r / g.W), x = (int)(r - (size_t)y * g.W);
    const float l = L[i], c = gc[i];
    const bf16 lh = (bf16)l, ch = (bf16)c;
    const bf16 ll = (bf16)(l - (float)lh), cl = (bf16)(c - (float)ch);
    const size_t pix = (size_t)s * g.sx + (size_t)(y + 1) * g.pw + (x + 1);
    *reinterpret_cast<bf16x8*>(x0 + pix * 8) = input_split(l, c);
    if (x0p) {
        const float tp = tau[s] / kTauRef;
        const bf16 th = (bf16)tp, tl = (bf16)(tp - (float)th);
        const bf16 pv[6] = {lh, ll, ch, cl, th, tl};
        const size_t rowbase = ((size_t)s * (g.H + 2) + y + 1) * 8;
#pragma unroll
        for (int c2 = 0; c2 < 6; ++c2) x0p[(rowbase + c2) * g.PX + x + 1] = pv[c2];
    }
}

// ---------------------------------------------------------------- the loss
// r = f - (L_next - L); per-block partial sums of w_s r^2; dZ6 =
// (2 w_s r / count) kOutScale in BF16 (NHWC8 channel 0 and planar).
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ f,
                                                   const float* __restrict__ L,
                                                   const float* __restrict__ Ln,
                                                   const float* __restrict__ wts,
                                                   bf16* __restrict__ dz6, bf16* __restrict__ dz6p,
                                                   float* __restrict__ lpart, Geo g, float dscale) {
    __shared__ float red[256];
    const size_t per = (size_t)g.W * g.H;
    const size_t total = per * g.n;
    float acc = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const int s = (int)(i / per);
        const float wr = (f[i] - (Ln[i] - L[i])) * (wts ? wts[s] : 1.f);
        const float r = f[i] - (Ln[i] - L[i]);
        acc += wr * r;
        const size_t rr = i - (size_t)s * per;
        const int y = (int)(rr / g.W), x = (int)(rr - (size_t)y * g.W);
        const bf16 d = (bf16)(wr * dscale);
        dz6[((size_t)s * g.sx + (size_t)(y + 1) * g.pw + (x + 1)) * 8] = d;
        dz6p[((size_t)s * g.H + y) * g.PZ + x] = d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// ------------------------------------------------------- weight gradient
template <int S>
__device__ inline bf16x8 shifted(const bf16x8& lo, const bf16x8& hi) {
    const u32x4 a = __builtin_bit_cast(u32x4, lo);
    const u32x4 b = __builtin_bit_cast(u32x4, hi);
    u32x4 r;
    if constexpr (S == 0) {
        r = a;
    } else if constexpr (S == 2) {
        r = u32x4{a[1], a[2], a[3], b[0]};
    } else {
        r = u32x4{__builtin_amdgcn_alignbyte(a[1], a[0], 2), __builtin_amdgcn_alignbyte(a[2], a[1], 2),
                  __builtin_amdgcn_alignbyte(a[3], a[2], 2), __builtin_amdgcn_alignbyte(b[0], a[3], 2)};
    }
    return __builtin_bit_cast(bf16x8, r);
}

// One wave: 32 pixels of R rows of one sample.  D[co][ci] of tap t
// accumulates sum_p dZ[p][co] X[p + t][ci]; the bias gradient is the same
// product against a ones operand.  Partials: [item][9][32 co][32 ci], then
// [32] bias.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void wgrad_kernel(const bf16* __restrict__ xp,
                                                    const bf16* __restrict__ dzp,
                                                    float* __restrict__ part, Geo g, int R) {
    constexpr int NB = CIN == 32 ? 2 : 1;
    constexpr int MB = COUT == 32 ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int sw = (g.W + kWgStrip - 1) / kWgStrip;
    const int chunks = (g.H + R - 1) / R;
    const int per = sw * chunks;
    if (item >= g.n * per) return;
    const int s = item / per;
    const int rem = item - s * per;
    const int chunk = rem / sw, strip = rem - chunk * sw;
    const int x0 = strip * kWgStrip, y0 = chunk * R, y1 = min(g.H, y0 + R);
    const int i = lane & 15, q = lane >> 4;

    f32x4 acc[9][MB][NB];
    f32x4 accb[MB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[t][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) accb[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (bf16)1.f;

    const bf16* zb = dzp + (size_t)s * g.H * COUT * g.PZ + x0 + 8 * q;
    const bf16* xb = xp + (size_t)s * (g.H + 2) * CIN * g.PX + x0 + 8 * q;

#define KZ_LOADX(X, yp)                                                         \
    _Pragma("unroll") for (int nb = 0; nb < NB; ++nb) {                         \
        const int ci_ = 16 * nb + i;                                            \
        if (ci_ < CIN) {                                                        \
            const bf16* p_ = xb + ((size_t)(yp) * CIN + ci_) * g.PX;            \
            X[nb][0] = ld8(p_);                                                 \
            X[nb][1] = ld8(p_ + 8);                                             \
        } else {                                                                \
            X[nb][0] = zero8();                                                 \
            X[nb][1] = zero8();                                                 \
        }                                                                       \
    }
#define KZ_TAPROW(ty, X)                                                                   \
    _Pragma("unroll") for (int nb = 0; nb < NB; ++nb) {                                    \
        const bf16x8 b0_ = shifted<0>(X[nb][0], X[nb][1]);                                 \
        const bf16x8 b1_ = shifted<1>(X[nb][0], X[nb][1]);                                 \
        const bf16x8 b2_ = shifted<2>(X[nb][0], X[nb][1]);                                 \
        _Pragma("unroll") for (int mb = 0; mb < MB; ++mb) {                                \
            acc[3 * (ty) + 0][mb][nb] = mfma(az[mb], b0_, acc[3 * (ty) + 0][mb][nb]);      \
            acc[3 * (ty) + 1][mb][nb] = mfma(az[mb], b1_, acc[3 * (ty) + 1][mb][nb]);      \
            acc[3 * (ty) + 2][mb][nb] = mfma(az[mb], b2_, acc[3 * (ty) + 2][mb][nb]);      \
        }                                                                                  \
    }
#define KZ_WSTEP(yy, XA, XB, XC)                                                 \
    {                                                                            \
        KZ_LOADX(XC, (yy) + 2)                                                   \
        bf16x8 az[MB];                                                           \
        _Pragma("unroll") for (int mb = 0; mb < MB; ++mb) {                      \
            const int co_ = 16 * mb + i;                                         \
            az[mb] = co_ < COUT ? ld8(zb + ((size_t)(yy) * COUT + co_) * g.PZ) : zero8(); \
        }                                                                        \
        KZ_TAPROW(0, XA)                                                         \
        KZ_TAPROW(1, XB)                                                         \
        KZ_TAPROW(2, XC)                                                         \
        _Pragma("unroll") for (int mb = 0; mb < MB; ++mb) accb[mb] = mfma(az[mb], ones, accb[mb]); \
    }
    bf16x8 xa[NB][2], xb2[NB][2], xc[NB][2];
    KZ_LOADX(xa, y0)
    KZ_LOADX(xb2, y0 + 1)
    for (int y = y0; y < y1; y += 3) {
        KZ_WSTEP(y, xa, xb2, xc)
        if (y + 1 < y1) KZ_WSTEP(y + 1, xb2, xc, xa)
        if (y + 2 < y1) KZ_WSTEP(y + 2, xc, xa, xb2)
    }
#undef KZ_WSTEP
#undef KZ_TAPROW
#undef KZ_LOADX

    float* out = part + (size_t)item * kPartStride;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = 16 * mb + 4 * q + r, ci = 16 * nb + i;
                    out[t * 1024 + co * 32 + ci] = acc[t][mb][nb][r];
                }
    if (i == 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[9 * 1024 + 16 * mb + 4 * q + r] = accb[mb][r];
    }
}

// Sums the per-wave partials of one layer into its slice of the flat
// gradient (weights [co][ci][3][3], then biases).  Block: 64 outputs x 4
// waves; wave w adds items w, w + 4, ...; the four sums are combined in a
// fixed order.
__global__ __launch_bounds__(256) void wreduce_kernel(const float* __restrict__ part, int items,
                                                      int layer, int ci_n, int co_n,
                                                      float* __restrict__ grad) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    const int nw = co_n * ci_n * 9;
    const int nout = nw + co_n;
    int src0 = -1, src1 = -1;
    if (p < nw) {
        const int co = p / (ci_n * 9), rem = p - co * ci_n * 9;
        const int ci = rem / 9, t = rem - ci * 9;
        if (layer == 0) {  // planar input channels (L_hi, L_lo, g_hi, g_lo, tau_hi, tau_lo)
            src0 = t * 1024 + co * 32 + 2 * ci;
            src1 = src0 + 1;
        } else {
            src0 = t * 1024 + co * 32 + ci;
        }
    } else if (p < nout) {
        src0 = 9 * 1024 + (p - nw);
    }
    float s = 0.f;
    if (src0 >= 0)
        for (int it = w; it < items; it += 4) {
            const float* b = part + (size_t)it * kPartStride;
            s += src1 >= 0 ? b[src0] + b[src1] : b[src0];
        }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && p < nout) grad[p] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ __launch_bounds__(256) void sum_kernel(const float* __restrict__ v, int count, float scale,
                                                  float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < count; i += 256) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// --------------------------------------------------------- weight packing
struct PackJob {
    int fwd;     // 1: forward fragments, 0: input-gradient fragments
    int layer;   // 0..5
    int KS;      // K steps per fragment row
    int nfrag;   // MB * KS
    size_t off;  // byte offset in the packed buffer
};
struct PackJobs {
    PackJob j[11];
    int w[kLayers];  // weight offsets in the parameter vector
    int b[kLayers];
    size_t bias_off[kLayers], tauw_off;
};

__device__ inline float hi_of(float w) { return (float)(bf16)w; }

__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ P, unsigned char* packed,
                                                   PackJobs jobs) {
    const PackJob jb = jobs.j[blockIdx.y];
    const int idx = blockIdx.x * 256 + threadIdx.x;  // (fragment, lane)
    if (idx >= jb.nfrag * 64) return;
    const int f = idx / 64, lane = idx - f * 64;
    const int mb = f / jb.KS, ks = f - mb * jb.KS;
    const int i = lane & 15, q = lane >> 4;
    const int l = jb.layer;
    const float* W = P + jobs.w[l];
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (jb.fwd) {
        const int co = 16 * mb + i;
        if (l == 0) {
            const int t = 4 * ks + q;
            if (t < 9) {
                const float wl = W[(co * 3 + 0) * 9 + t], wg = W[(co * 3 + 1) * 9 + t];
                const float lh = hi_of(wl), gh = hi_of(wg);
                v[0] = lh;
                v[1] = lh;
                v[2] = wl - lh;
                v[3] = gh;
                v[4] = gh;
                v[5] = wg - gh;
            }
        } else if (l == kLayers - 1) {
            if (co == 0)
                for (int e = 0; e < 8; ++e) v[e] = W[(8 * q + e) * 9 + ks];
        } else {
            for (int e = 0; e < 8; ++e) v[e] = W[(co * 32 + 8 * q + e) * 9 + ks];
        }
    } else {
        const int ci = 16 * mb + i;  // input channel of the layer = output of dgrad
        if (l == kLayers - 1) {
            const int t = 4 * ks + q;
            if (t < 9) v[0] = W[ci * 9 + 8 - t];
        } else {
            for (int e = 0; e < 8; ++e) v[e] = W[((8 * q + e) * 32 + ci) * 9 + 8 - ks];
        }
    }
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (bf16)v[e];
    *reinterpret_cast<bf16x8*>(packed + jb.off + (size_t)idx * 16) = o;

    if (blockIdx.y == 0 && idx < 32) {  // biases, tau taps
        const int c = idx;
        for (int ll = 0; ll < kLayers; ++ll) {
            const int con = ll == kLayers - 1 ? 1 : 32;
            reinterpret_cast<float*>(packed + jobs.bias_off[ll])[c] = c < con ? P[jobs.b[ll] + c] : 0.f;
        }
        for (int t = 0; t < 9; ++t)
            reinterpret_cast<float*>(packed + jobs.tauw_off)[c * 9 + t] = P[jobs.w[0] + (c * 3 + 2) * 9 + t];
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ gr,
                                                   float* __restrict__ m, float* __restrict__ v, int count,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void zero_kernel(uint4* __restrict__ p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = uint4{0u, 0u, 0u, 0u};
}

}  // namespace

ParamLayout param_layout() {
    ParamLayout L;
    const int ch[kLayers + 1] = {3, 32, 32, 32, 32, 32, 1};
    int o = 0;
    for (int l = 0; l < kLayers; ++l) {
        L.ci[l] = ch[l];
        L.co[l] = ch[l + 1];
        L.w[l] = o;
        o += ch[l] * ch[l + 1] * 9;
        L.b[l] = o;
        o += ch[l + 1];
    }
    return L;
}

namespace {
int fwd_frags(int l) { return l == 0 ? 6 : (l == kLayers - 1 ? 9 : 18); }
int dgr_frags(int l) { return l == 0 ? 0 : (l == kLayers - 1 ? 6 : 18); }
int fwd_ks(int l) { return l == 0 ? 3 : 9; }
int dgr_ks(int l) { return l == kLayers - 1 ? 3 : 9; }
}  // namespace

PackLayout pack_layout() {
    PackLayout P;
    size_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        P.fwd[l] = o;
        o += (size_t)fwd_frags(l) * 64 * 16;
    }
    for (int l = 0; l < kLayers; ++l) {
        P.dgr[l] = o;
        o += (size_t)dgr_frags(l) * 64 * 16;
    }
    for (int l = 0; l < kLayers; ++l) {
        P.bias[l] = o;
        o += 32 * sizeof(float);
    }
    P.tauw = o;
    o += 32 * 9 * sizeof(float);
    P.bytes = (o + 255) & ~(size_t)255;
    return P;
}

Geo make_geo(int n, int W, int H, int R) {
    Geo g;
    g.n = n;
    g.W = W;
    g.H = H;
    g.R = R;
    g.strips = (W + kStrip - 1) / kStrip;
    g.chunks = (H + R - 1) / R;
    g.pw = W + 2;
    g.sx = (long long)(H + 2) * (W + 2);
    g.PZ = kWgStrip * ((W + kWgStrip - 1) / kWgStrip);
    g.PX = g.PZ + 32;
    return g;
}

hipError_t launch_conv(int cin, int mb, int epi, bool tau_term, const ConvArgs& a, const Geo& g,
                       hipStream_t s) {
    const int items = a.bw.imgs ? a.bw.count : (a.items ? a.nitems : g.n * g.strips * g.chunks);
    if (items <= 0) return hipSuccess;
    const dim3 grid((items + 3) / 4), block(256);
    if (cin == 8 && mb == 2 && epi == EPI_RELU && tau_term)
        hipLaunchKernelGGL((conv_kernel<8, 2, EPI_RELU, true>), grid, block, 0, s, a, g);
    else if (cin == 32 && mb == 2 && epi == EPI_RELU && !tau_term)
        hipLaunchKernelGGL((conv_kernel<32, 2, EPI_RELU, false>), grid, block, 0, s, a, g);
    else if (cin == 32 && mb == 1 && epi == EPI_OUT && !tau_term)
        hipLaunchKernelGGL((conv_kernel<32, 1, EPI_OUT, false>), grid, block, 0, s, a, g);
    else if (cin == 32 && mb == 2 && epi == EPI_MASK && !tau_term)
        hipLaunchKernelGGL((conv_kernel<32, 2, EPI_MASK, false>), grid, block, 0, s, a, g);
    else if (cin == 8 && mb == 2 && epi == EPI_MASK && !tau_term)
        hipLaunchKernelGGL((conv_kernel<8, 2, EPI_MASK, false>), grid, block, 0, s, a, g);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Blocks of the fused pair resident on the current device at once (compute
// units x blocks per unit), looked up once per device.
int pair_slots() {
    constexpr int kMaxDevices = 64;
    static std::atomic<int> slots[kMaxDevices];  // 0: not looked up yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    int v = slots[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, conv2_kernel<32, 2, false>,
                                                         kPairThreads, 0) != hipSuccess)
            return 0;
        v = std::max(1, cus * per);
        slots[dev].store(v, std::memory_order_relaxed);  // every thread stores the same value
    }
    return v;
}

// Rows per block of a fused pair over n images of height H in `strips`
// column strips.  A block walks its rows one step each (plus three steps of
// fill), so a launch takes about rounds x (R + 3) steps, rounds being the
// number of times the grid fills the device: the chunk count minimising that
// product.  Every output row is computed by the same instructions whatever
// the block, so the choice does not change a bit of the result.
int pair_rows(int n, int H, int strips) {
    const int slots = pair_slots();
    if (slots <= 0) return kConvRows;
    const long long per = (long long)n * strips;
    long long best = -1;
    int rows = kConvRows;
    for (int chunks = 1; chunks <= H; ++chunks) {
        const int R = (H + chunks - 1) / chunks;
        if ((H + R - 1) / R != chunks) continue;  // same R as fewer chunks
        const long long rounds = (per * chunks + slots - 1) / slots;
        const long long cost = rounds * (R + 3);
        if (best < 0 || cost < best) {
            best = cost;
            rows = R;
        }
    }
    return rows;
}

hipError_t launch_conv2(int cina, int mbb, const Conv2Args& a, const Geo& g, hipStream_t s) {
    const int strips = (g.W + kPairOut - 1) / kPairOut;
    Geo gg = g;
    gg.strips = strips;
    if (!a.bw.imgs) gg.R = pair_rows(g.n, g.H, strips);  // batches: rows fixed by their items
    gg.chunks = (g.H + gg.R - 1) / gg.R;
    if (a.bw.imgs && a.bw.count <= 0) return hipSuccess;
    const dim3 grid = a.bw.imgs ? dim3(a.bw.count) : dim3(strips * gg.chunks, g.n);
    const dim3 block(kPairThreads);
    if (cina == 8 && mbb == 2)
        hipLaunchKernelGGL((conv2_kernel<8, 2, true>), grid, block, 0, s, a, gg);
    else if (cina == 32 && mbb == 2)
        hipLaunchKernelGGL((conv2_kernel<32, 2, false>), grid, block, 0, s, a, gg);
    else if (cina == 32 && mbb == 1)
        hipLaunchKernelGGL((conv2_kernel<32, 1, false>), grid, block, 0, s, a, gg);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pack_input(const float* L, const float* gc, const float* tau, bf16* x0, bf16* x0p,
                             const Geo& g, hipStream_t s) {
    const size_t total = (size_t)g.n * g.W * g.H;
    hipLaunchKernelGGL(pack_input_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, L, gc,
                       tau, x0, x0p, g);
    return hipGetLastError();
}

hipError_t launch_pack_input_batch(const SgImage* imgs, int n, bf16* x0, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_input_batch_kernel, dim3(1024, n), dim3(256), 0, s, imgs, x0);
    return hipGetLastError();
}

int loss_blocks(const Geo& g) {
    const size_t total = (size_t)g.n * g.W * g.H;
    const size_t b = (total + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_loss(const float* f, const float* L, const float* Ln, const float* wts, bf16* dz6,
                       bf16* dz6p, float* lpart, int nblocks, const Geo& g, hipStream_t s) {
    const double count = (double)g.n * g.W * g.H;
    hipLaunchKernelGGL(loss_kernel, dim3(nblocks), dim3(256), 0, s, f, L, Ln, wts, dz6, dz6p, lpart, g,
                       (float)(2.0 * kOutScale / count));
    return hipGetLastError();
}

int wgrad_items(const Geo& g, int R) {
    return g.n * ((g.W + kWgStrip - 1) / kWgStrip) * ((g.H + R - 1) / R);
}

hipError_t launch_wgrad(int cin, int cout, const bf16* xp, const bf16* dzp, float* part, const Geo& g,
                        int R, hipStream_t s) {
    const int items = wgrad_items(g, R);
    const dim3 grid((items + 3) / 4), block(256);
    if (cin == 8 && cout == 32)
        hipLaunchKernelGGL((wgrad_kernel<8, 32>), grid, block, 0, s, xp, dzp, part, g, R);
    else if (cin == 32 && cout == 32)
        hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, block, 0, s, xp, dzp, part, g, R);
    else if (cin == 32 && cout == 1)
        hipLaunchKernelGGL((wgrad_kernel<32, 1>), grid, block, 0, s, xp, dzp, part, g, R);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_wreduce(int layer, const float* part, int items, float* grad, hipStream_t s) {
    const ParamLayout L = param_layout();
    const int nout = L.co[layer] * L.ci[layer] * 9 + L.co[layer];
    hipLaunchKernelGGL(wreduce_kernel, dim3((nout + 63) / 64), dim3(256), 0, s, part, items, layer,
                       L.ci[layer], L.co[layer], grad + L.w[layer]);
    return hipGetLastError();
}

hipError_t launch_sum(const float* v, int count, float scale, float* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, v, count, scale, out);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* params, void* packed, hipStream_t s) {
    const ParamLayout L = param_layout();
    const PackLayout P = pack_layout();
    PackJobs J;
    int n = 0, maxf = 0;
    for (int l = 0; l < kLayers; ++l) {
        J.j[n++] = PackJob{1, l, fwd_ks(l), fwd_frags(l), P.fwd[l]};
        maxf = fwd_frags(l) > maxf ? fwd_frags(l) : maxf;
    }
    for (int l = 1; l < kLayers; ++l) J.j[n++] = PackJob{0, l, dgr_ks(l), dgr_frags(l), P.dgr[l]};
    for (int l = 0; l < kLayers; ++l) {
        J.w[l] = L.w[l];
        J.b[l] = L.b[l];
        J.bias_off[l] = P.bias[l];
    }
    J.tauw_off = P.tauw;
    hipLaunchKernelGGL(pack_kernel, dim3((maxf * 64 + 255) / 256, n), dim3(256), 0, s, params,
                       static_cast<unsigned char*>(packed), J);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* grad, float* m, float* v, int count, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, grad, m, v, count, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint4*>(p), n16);
    return hipGetLastError();
}

}  // namespace sg
}  // namespace kaze
