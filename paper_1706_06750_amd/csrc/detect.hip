// Detector response (Eq. 8) and 3x3x3 extrema (Sec. II-B).
//
// det_i = sigma_n^2 (L_xx L_yy - L_xy^2) with L_xx = D_x D_x L, L_yy = D_y D_y L,
// L_xy = D_y D_x L, where D_x of step s is the concatenated Scharr filter
//   D_x f(x,y) = sum_{dy in -s,0,s} w_dy (f(x+s, y+dy) - f(x-s, y+dy)) / (2s),
//   w = (3, 10, 3)/16,
// and every derivative image is extended by half-sample reflection before the
// next derivative is taken.  One fused kernel per launch computes the first
// derivatives of a 64x16 tile (plus an s-pixel ring) in LDS and the second
// derivatives and det in registers; L_x, L_y, L_xx, ... never reach memory.
#include "kaze_internal.h"

namespace kaze {
namespace {

constexpr int TX = 64;
constexpr int TY = 16;
constexpr int BX = 64;
constexpr int BY = 4;

__global__ __launch_bounds__(BX* BY) void det_kernel(const float* __restrict__ levels,
                                                       float* __restrict__ det, int W, int H,
                                                       DetLevels dl, int smax) {
    extern __shared__ float smem[];
    const int lev = blockIdx.z;
    const int s = dl.step[lev];
    const float sn2 = dl.sn2[lev];
    const int iw = TX + 4 * smax, ih = TY + 4 * smax;   // input tile + 2s ring
    const int fw = TX + 2 * smax, fh = TY + 2 * smax;   // derivatives + s ring
    float* s_in = smem;
    float* s_lx = s_in + iw * ih;
    float* s_ly = s_lx + fw * fh;
    const size_t plane = (size_t)W * H;
    const float* L = levels + plane * lev;
    const int tx0 = blockIdx.x * TX, ty0 = blockIdx.y * TY;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int ro = 2 * s;  // origin of the input tile inside s_in

    for (int ly = ty; ly < TY + 4 * s; ly += BY) {
        const int gy = reflect_index(ty0 + ly - ro, H);
        const float* row = L + (size_t)gy * W;
        for (int lx = tx; lx < TX + 4 * s; lx += BX)
            s_in[ly * iw + lx] = row[reflect_index(tx0 + lx - ro, W)];
    }
    __syncthreads();

    // First derivatives on the tile plus an s ring.  A ring position outside
    // the image takes the derivative at its reflected in-image position, so
    // the ring holds the reflected derivative image.  Ring positions more
    // than s past the last row/column feed no output pixel and are skipped
    // (their reflected position may lie outside the loaded tile).
    const float inv2s = 1.f / (float)(2 * s);
    for (int py = ty; py < TY + 2 * s; py += BY) {
        const int gy = ty0 + py - s;
        if (gy > H - 1 + s) break;
        const int ry = reflect_index(gy, H) - ty0 + ro;  // row inside s_in
        for (int px = tx; px < TX + 2 * s; px += BX) {
            const int gx = tx0 + px - s;
            if (gx > W - 1 + s) break;
            const int rx = reflect_index(gx, W) - tx0 + ro;
            const float* c = s_in + ry * iw + rx;
            const float ddx_m = c[-s * iw + s] - c[-s * iw - s];
            const float ddx_0 = c[s] - c[-s];
            const float ddx_p = c[s * iw + s] - c[s * iw - s];
            const float ddy_m = c[s * iw - s] - c[-s * iw - s];
            const float ddy_0 = c[s * iw] - c[-s * iw];
            const float ddy_p = c[s * iw + s] - c[-s * iw + s];
            s_lx[py * fw + px] = (0.1875f * ddx_m + 0.625f * ddx_0 + 0.1875f * ddx_p) * inv2s;
            s_ly[py * fw + px] = (0.1875f * ddy_m + 0.625f * ddy_0 + 0.1875f * ddy_p) * inv2s;
        }
    }
    __syncthreads();

    const int gx = tx0 + tx;
    if (gx >= W) return;
    for (int ly = ty; ly < TY; ly += BY) {
        const int gy = ty0 + ly;
        if (gy >= H) break;
        const int cy = ly + s, cx = tx + s;
        const float* lxc = s_lx + cy * fw + cx;
        const float* lyc = s_ly + cy * fw + cx;
        // L_xx = D_x(L_x), L_xy = D_y(L_x), L_yy = D_y(L_y)
        const float xx = 0.1875f * (lxc[-s * fw + s] - lxc[-s * fw - s]) +
                         0.625f * (lxc[s] - lxc[-s]) +
                         0.1875f * (lxc[s * fw + s] - lxc[s * fw - s]);
        const float xy = 0.1875f * (lxc[s * fw - s] - lxc[-s * fw - s]) +
                         0.625f * (lxc[s * fw] - lxc[-s * fw]) +
                         0.1875f * (lxc[s * fw + s] - lxc[-s * fw + s]);
        const float yy = 0.1875f * (lyc[s * fw - s] - lyc[-s * fw - s]) +
                         0.625f * (lyc[s * fw] - lyc[-s * fw]) +
                         0.1875f * (lyc[s * fw + s] - lyc[-s * fw + s]);
        const float Lxx = xx * inv2s, Lxy = xy * inv2s, Lyy = yy * inv2s;
        det[plane * lev + (size_t)gy * W + gx] = sn2 * (Lxx * Lyy - Lxy * Lxy);
    }
}

struct KeypointOut {
    int x, y, level;
    float response;
};

// (x, y, i) is an extremum iff det_i(x,y) > threshold and > all 26
// neighbours in levels i-1..i+1; levels 1..N-2, 1-pixel image border excluded.
__global__ __launch_bounds__(BX* BY) void nms_kernel(const float* __restrict__ det, int W, int H,
                                                       float threshold,
                                                       KeypointOut* __restrict__ kps, int capacity,
                                                       int* __restrict__ count) {
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int lev = blockIdx.z + 1;
    if (x < 1 || y < 1 || x > W - 2 || y > H - 2) return;
    const size_t plane = (size_t)W * H;
    const float* c = det + plane * lev + (size_t)y * W + x;
    const float v = c[0];
    if (!(v > threshold)) return;
    bool is_max = true;
#pragma unroll
    for (int dl = -1; dl <= 1; ++dl) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dl == 0 && dy == 0 && dx == 0) continue;
                const float nb = c[(ptrdiff_t)dl * (ptrdiff_t)plane + dy * W + dx];
                is_max = is_max && (v > nb);
            }
        }
    }
    if (!is_max) return;
    const int idx = atomicAdd(count, 1);
    if (idx < capacity) {
        KeypointOut k;
        k.x = x;
        k.y = y;
        k.level = lev;
        k.response = v;
        kps[idx] = k;
    }
}

}  // namespace

hipError_t launch_det(const float* levels, float* det, int W, int H, int N, const DetLevels& dl,
                      hipStream_t s) {
    int smax = 1;
    for (int i = 0; i < N; ++i) smax = dl.step[i] > smax ? dl.step[i] : smax;
    const size_t lds = sizeof(float) * ((size_t)(TX + 4 * smax) * (TY + 4 * smax) +
                                        2 * (size_t)(TX + 2 * smax) * (TY + 2 * smax));
    dim3 grid((W + TX - 1) / TX, (H + TY - 1) / TY, N), block(BX, BY);
    hipLaunchKernelGGL(det_kernel, grid, block, lds, s, levels, det, W, H, dl, smax);
    return hipGetLastError();
}

hipError_t launch_nms(const float* det, int W, int H, int N, float threshold, void* kps,
                      int capacity, int* count, hipStream_t s) {
    if (N < 3) return hipSuccess;
    dim3 grid((W + BX - 1) / BX, (H + BY - 1) / BY, N - 2), block(BX, BY);
    hipLaunchKernelGGL(nms_kernel, grid, block, 0, s, det, W, H, threshold,
                       static_cast<KeypointOut*>(kps), capacity, count);
    return hipGetLastError();
}

}  // namespace kaze
