// Conductivity of one 64x64 tile in LDS (Eqs. 2-3):
//   L (tile + ring R = r + 2, half-sample reflected at the image border)
//   -> horizontal Gaussian pass (r taps each side)
//   -> vertical Gaussian pass: L_s on the tile + 2 ring
//   -> 3x3 Scharr gradient (central difference / 2 across, [3 10 3]/16
//      along): |grad L_s|^2 and g on the tile + 1 ring.
// A symmetric filter applied to a half-sample symmetric extension yields a
// half-sample symmetric result, so ring values past the image border equal
// the reflected in-image values, exactly as if each intermediate image were
// reflected.  Used by the standalone conductivity kernel and by the fused
// AOS reduction kernel, so both produce the same g.
#pragma once

#include "kaze_internal.h"

namespace kaze {

// LDS layout (in floats) of the tile pipeline; pitches are odd so that
// threads walking down a column hit distinct banks.
struct CondTile {
    int r, R;       // Gaussian radius, ring of L
    int nL, pL;     // L: nL x nL, pitch pL           (nL = kTile + 2R)
    int pH;         // horizontal pass: nL rows x (kTile + 4) cols
    int nS, pS;     // smoothed: nS x nS              (nS = kTile + 4)
    int nG, pG;     // g: nG x nG, aliases the horizontal pass (nG = kTile + 2)
    int offH, offS, offG;
    int floats;
};

__host__ __device__ inline int odd_pitch(int n) { return n | 1; }

__host__ __device__ inline CondTile cond_tile(int r) {
    CondTile c;
    c.r = r;
    c.R = r + 2;
    c.nL = kTile + 2 * c.R;
    c.pL = odd_pitch(c.nL);
    c.pH = odd_pitch(kTile + 4);
    c.nS = kTile + 4;
    c.pS = odd_pitch(c.nS);
    c.nG = kTile + 2;
    c.pG = odd_pitch(c.nG);
    c.offH = c.nL * c.pL;
    c.offS = c.offH + c.nL * c.pH;
    c.offG = c.offH;  // g overwrites the horizontal pass once it is consumed
    c.floats = c.offS + c.nS * c.pS;
    return c;
}

// L on the tile + ring R (reflected) into sL.
__device__ __forceinline__ void load_L_ring(const float* __restrict__ L, int W, int H, int tx0,
                                            int ty0, float* sL, const CondTile& ct) {
    const int n = ct.nL, total = n * n;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const int ly = i / n, lx = i - ly * n;
        const int gy = reflect_index(ty0 - ct.R + ly, H);
        const int gx = reflect_index(tx0 - ct.R + lx, W);
        sL[ly * ct.pL + lx] = L[(size_t)gy * W + gx];
    }
}

// Smoothed image L_s on the tile + 2 ring into sS (uses the sH region).
__device__ __forceinline__ void smooth_tile(const float* sL, float* sH, float* sS,
                                            const CondTile& ct, const Taps& taps) {
    const int r2 = 2 * ct.r;
    {
        const int cols = kTile + 4, total = ct.nL * cols;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int ly = i / cols, hx = i - ly * cols;
            const float* src = sL + ly * ct.pL + hx;
            float acc = 0.f;
            for (int t = 0; t <= r2; ++t) acc += taps.w[t] * src[t];
            sH[ly * ct.pH + hx] = acc;
        }
    }
    __syncthreads();
    {
        const int n = ct.nS, total = n * n;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const int sy = i / n, sx = i - sy * n;
            const float* src = sH + sy * ct.pH + sx;
            float acc = 0.f;
            for (int t = 0; t <= r2; ++t) acc += taps.w[t] * src[t * ct.pH];
            sS[sy * ct.pS + sx] = acc;
        }
    }
}

// Squared Scharr gradient of L_s at (gy, gx) of the g grid (tile + 1 ring).
__device__ __forceinline__ float scharr_m2(const float* sS, int pS, int gy, int gx) {
    const float* c = sS + (gy + 1) * pS + (gx + 1);
    const float dxm = 0.5f * (c[-pS + 1] - c[-pS - 1]);
    const float dx0 = 0.5f * (c[1] - c[-1]);
    const float dxp = 0.5f * (c[pS + 1] - c[pS - 1]);
    const float dym = 0.5f * (c[pS - 1] - c[-pS - 1]);
    const float dy0 = 0.5f * (c[pS] - c[-pS]);
    const float dyp = 0.5f * (c[pS + 1] - c[-pS + 1]);
    const float lx = 0.1875f * dxm + 0.625f * dx0 + 0.1875f * dxp;
    const float ly = 0.1875f * dym + 0.625f * dy0 + 0.1875f * dyp;
    return lx * lx + ly * ly;
}

// Perona-Malik conductivity (Eq. 3): mode 0 g2, mode 1 g1.
__device__ __forceinline__ float diffusivity(float m2, float inv_k2, int mode) {
    return mode == 0 ? 1.f / (1.f + m2 * inv_k2) : expf(-m2 * inv_k2);
}

}  // namespace kaze
