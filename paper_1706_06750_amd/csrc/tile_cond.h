// Conductivity of one 64x64 tile in LDS (Eqs. 2-3):
//   L (tile + ring R = r + 2, half-sample reflected at the image border)
//   -> horizontal Gaussian pass (r taps each side)
//   -> vertical Gaussian pass: L_s on the tile + 2 ring
//   -> 3x3 Scharr gradient (central difference / 2 across, [3 10 3]/16
//      along): |grad L_s|^2 and g on the tile + 1 ring.
// A symmetric filter applied to a half-sample symmetric extension yields a
// half-sample symmetric result, so ring values past the image border equal
// the reflected in-image values, exactly as if each intermediate image were
// reflected.  Used for the squared gradient behind the contrast factor and
// for the conductivity of batched images; the AOS reduction and the
// conductivity of one image use the band code beside the reduction instead
// (their g are equal bit for bit; this pipeline rounds differently).
//
// Geometry is compile-time (template on the Gaussian radius): every loop is
// unrolled, global loads are staged through registers so that all of a
// thread's loads are in flight together, and each filter pass computes runs
// of 4 outputs per thread to reuse the values it reads from LDS.
#pragma once

#include "kaze_internal.h"

namespace kaze {

// Threads of a smoothing / conductivity tile block: 512 measured faster than
// 256 (Gaussian 15 -> 12.4 us, gradient 21.5 -> 18.4 us per 1920x1200 image):
// with two or three tiles per CU the tiles' latency is what counts.
constexpr int kTileThreads = 512;
constexpr int kRun = 4;  // outputs per thread and work item in the filter passes

// Tile of TX x TY pixels; RG is the Gaussian radius of sigma_cond.
template <int RG, int TX = kTile, int TY = kTile>
struct CondGeom {
    static constexpr int r = RG;                 // Gaussian radius
    static constexpr int R = RG + 2;             // ring of L
    static constexpr int nLy = TY + 2 * R;       // L region
    static constexpr int nLx = TX + 2 * R;
    static constexpr int pL = nLx | 1;           // odd pitches: columns walk distinct banks
    static constexpr int nSy = TY + 4;           // smoothed region (tile + 2 ring)
    static constexpr int nSx = TX + 4;
    static constexpr int pS = nSx | 1;           // horizontal pass: nLy rows x nSx cols; the
                                                 // vertical pass overwrites it in place
    static constexpr int nGy = TY + 2;           // g region (tile + 1 ring)
    static constexpr int nGx = TX + 2;
    static constexpr int pG = nGx | 1;
    static constexpr int offS = nLy * pL;        // smoothing work area
    static constexpr int offG = offS;            // g overwrites the consumed smoothing area
    static constexpr int floats = offS + nLy * pS;
    static_assert(nGy * pG <= nLy * pS, "g must fit in the smoothing area");
    static_assert(nSx % kRun == 0 && nSy % 4 == 0, "runs must tile the passes");
};

// Rectangular region [gy0, gy0+NY) x [gx0, gx0+NX) of a W x H image into LDS
// (pitch P), half-sample reflected outside the image.  All loads of a
// thread are issued before the first LDS store.
template <int NY, int NX, int P, int NT>
__device__ __forceinline__ void stage_region(const float* __restrict__ src, int W, int H, int gy0,
                                             int gx0, float* dst) {
    constexpr int TOTAL = NY * NX;
    constexpr int PER = (TOTAL + NT - 1) / NT;
    const bool interior = gy0 >= 0 && gx0 >= 0 && gy0 + NY <= H && gx0 + NX <= W;
    const gfloat* g = (const gfloat*)src;
    float v[PER];
    if (interior) {
        const gfloat* base = g + (size_t)gy0 * W + gx0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * NT;
            if (i < TOTAL) {
                const int ly = i / NX, lx = i - ly * NX;
                v[j] = base[(size_t)ly * W + lx];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * NT;
            if (i < TOTAL) {
                const int ly = i / NX, lx = i - ly * NX;
                const int gy = reflect_index(gy0 + ly, H), gx = reflect_index(gx0 + lx, W);
                v[j] = g[(size_t)gy * W + gx];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = threadIdx.x + j * NT;
        if (i < TOTAL) {
            const int ly = i / NX, lx = i - ly * NX;
            dst[ly * P + lx] = v[j];
        }
    }
}

// L on the tile + ring R (reflected) into sL.
template <class G>
__device__ __forceinline__ void load_L_ring(const float* __restrict__ L, int W, int H, int tx0,
                                            int ty0, float* sL) {
    stage_region<G::nLy, G::nLx, G::pL, kTileThreads>(L, W, H, ty0 - G::R, tx0 - G::R, sL);
}

// Smoothed image L_s on the tile + 2 ring into sS (nSy x nSx, pitch pS).
template <class G>
__device__ __forceinline__ void smooth_tile(const float* sL, float* sS, const Taps& taps) {
    constexpr int T = 2 * G::r + 1;
    float w[T];
#pragma unroll
    for (int t = 0; t < T; ++t) w[t] = taps.w[t];
    // horizontal: item = (run along x, row); lanes walk rows (odd pitch)
    {
        constexpr int runs = G::nSx / kRun, items = runs * G::nLy;
#pragma unroll 1
        for (int i = threadIdx.x; i < items; i += kTileThreads) {
            const int row = i % G::nLy, x0 = (i / G::nLy) * kRun;
            const float* src = sL + row * G::pL + x0;
            float v[kRun + T - 1];
#pragma unroll
            for (int q = 0; q < kRun + T - 1; ++q) v[q] = src[q];
#pragma unroll
            for (int q = 0; q < kRun; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < T; ++t) acc += w[t] * v[q + t];
                sS[row * G::pS + x0 + q] = acc;
            }
        }
    }
    __syncthreads();
    // vertical, in place: item = (column, quarter of the rows).  Every item
    // reads its inputs into registers before the barrier and writes after.
    {
        constexpr int NQ = 4, QR = G::nSy / NQ, items = NQ * G::nSx;
        constexpr int PER = (items + kTileThreads - 1) / kTileThreads;
        float v[PER][QR + T - 1];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * kTileThreads;
            if (i < items) {
                const int col = i % G::nSx, y0 = (i / G::nSx) * QR;
#pragma unroll
                for (int q = 0; q < QR + T - 1; ++q) v[j][q] = sS[(y0 + q) * G::pS + col];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * kTileThreads;
            if (i < items) {
                const int col = i % G::nSx, y0 = (i / G::nSx) * QR;
#pragma unroll
                for (int q = 0; q < QR; ++q) {
                    float acc = 0.f;
#pragma unroll
                    for (int t = 0; t < T; ++t) acc += w[t] * v[j][q + t];
                    sS[(y0 + q) * G::pS + col] = acc;
                }
            }
        }
    }
}

// Squared Scharr gradient magnitudes of L_s on the g grid (tile + 1 ring),
// computed into registers; after a barrier f(gy, gx, m2) is called once per
// position (gy in [0, TY + 2), gx in [0, TX + 2)), so f may overwrite the
// sS area.
template <class G, class F>
__device__ __forceinline__ void scharr_pass(const float* sS, F&& f) {
    constexpr int runs = (G::nGy + kRun - 1) / kRun, items = runs * G::nGx;
    constexpr int PER = (items + kTileThreads - 1) / kTileThreads;
    float m2[PER][kRun];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = threadIdx.x + j * kTileThreads;
        if (i < items) {
            const int gx = i % G::nGx, gy0 = (i / G::nGx) * kRun;
            // g row gy uses sS rows gy .. gy+2 and columns gx .. gx+2
            float a[kRun + 2], b[kRun + 2], c[kRun + 2];
#pragma unroll
            for (int q = 0; q < kRun + 2; ++q) {
                const int sy = gy0 + q < G::nSy ? gy0 + q : G::nSy - 1;
                const float* p = sS + sy * G::pS + gx;
                a[q] = p[0];
                b[q] = p[1];
                c[q] = p[2];
            }
#pragma unroll
            for (int q = 0; q < kRun; ++q) {
                const float dxm = 0.5f * (c[q] - a[q]);
                const float dx0 = 0.5f * (c[q + 1] - a[q + 1]);
                const float dxp = 0.5f * (c[q + 2] - a[q + 2]);
                const float dym = 0.5f * (a[q + 2] - a[q]);
                const float dy0 = 0.5f * (b[q + 2] - b[q]);
                const float dyp = 0.5f * (c[q + 2] - c[q]);
                const float lx = 0.1875f * dxm + 0.625f * dx0 + 0.1875f * dxp;
                const float ly = 0.1875f * dym + 0.625f * dy0 + 0.1875f * dyp;
                m2[j][q] = lx * lx + ly * ly;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = threadIdx.x + j * kTileThreads;
        if (i < items) {
            const int gx = i % G::nGx, gy0 = (i / G::nGx) * kRun;
#pragma unroll
            for (int q = 0; q < kRun; ++q)
                if (gy0 + q < G::nGy) f(gy0 + q, gx, m2[j][q]);
        }
    }
}

// Perona-Malik conductivity (Eq. 3): mode 0 g2, mode 1 g1.
__device__ __forceinline__ float diffusivity(float m2, float inv_k2, int mode) {
    return mode == 0 ? __builtin_amdgcn_rcpf(1.f + m2 * inv_k2) : expf(-m2 * inv_k2);
}

}  // namespace kaze
