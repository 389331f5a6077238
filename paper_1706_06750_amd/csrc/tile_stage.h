// Staging of image tiles into LDS for the 64x64-tile kernels (the Gaussian
// pre-smoothing and the detector): the thread count of a smoothing tile and
// a region copy with half-sample reflection at the image border.
#pragma once

#include "kaze_internal.h"

namespace kaze {

// Threads of a smoothing tile block: 512 measured faster than 256 (Gaussian
// 15 -> 12.4 us per 1920x1200 image): with two or three tiles per CU the
// tiles' latency is what counts.
constexpr int kTileThreads = 512;
constexpr int kRun = 4;  // outputs per thread and work item in the filter passes

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

}  // namespace kaze
