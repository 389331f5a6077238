// Detector response (Eq. 8) and 3x3x3 extrema (Sec. II-B).
//
// det_i = sigma_n^2 (L_xx L_yy - L_xy^2) with L_xx = D_x D_x L, L_yy = D_y D_y L,
// L_xy = D_y D_x L, where D_x of step s is the concatenated Scharr filter
//   D_x f(x,y) = sum_{dy in -s,0,s} w_dy (f(x+s, y+dy) - f(x-s, y+dy)) / (2s),
//   w = (3, 10, 3)/16,
// and every derivative image is extended by half-sample reflection before the
// next derivative is taken.  One block per 64x32 tile and level computes the
// first derivatives of the tile plus an s ring in LDS, then the second
// derivatives and det; L_x, L_y, L_xx, ... never reach memory.
#include "kaze_internal.h"
#include "tile_cond.h"

namespace kaze {
namespace {

constexpr int DTX = 64;
constexpr int DTY = 32;

template <int S>
struct DetGeom {
    static constexpr int niy = DTY + 4 * S, nix = DTX + 4 * S;  // staged L
    static constexpr int pI = nix | 1;
    static constexpr int nfy = DTY + 2 * S, nfx = DTX + 2 * S;  // first derivatives
    static constexpr int pF = nfx | 1;
    static constexpr int offX = niy * pI;
    static constexpr int offY = offX + nfy * pF;
    static constexpr int floats = offY + nfy * pF;
};

template <int S>
__global__ __launch_bounds__(kTileThreads) void det_kernel(BatchImage d0, ImgWork w, DetLevels dl,
                                                             int lev0, int lev1) {
    using G = DetGeom<S>;
    extern __shared__ float smem[];
    float* sI = smem;
    float* sX = smem + G::offX;
    float* sY = smem + G::offY;
    // levels of this launch: the ones in [lev0, lev1) with Scharr step S
    int lev = -1;
    for (int i = lev0, seen = 0; i < lev1; ++i)
        if (dl.step[i] == S && seen++ == (int)blockIdx.y) lev = i;
    if (lev < 0) return;  // uniform per block
    BatchImage d;
    int lt;
    resolve(d0, w, (int)blockIdx.x, d, lt);
    const int W = d.W, H = d.H;
    float* __restrict__ det = d.det;
    const float sn2 = dl.sn2[lev];
    const size_t plane = (size_t)W * H;
    const float* L = d.levels + plane * lev;
    const int ncx = (W + DTX - 1) / DTX;
    const int tx0 = (lt % ncx) * DTX, ty0 = (lt / ncx) * DTY;
    stage_region<G::niy, G::nix, G::pI, kTileThreads>(L, W, H, ty0 - 2 * S, tx0 - 2 * S, sI);
    __syncthreads();

    // First derivatives on the tile plus an s ring.  A ring position outside
    // the image takes the derivative at its reflected in-image position, so
    // the ring holds the reflected derivative image.  Ring positions more
    // than s past the last row/column feed no output pixel and are skipped
    // (their reflected position may lie outside the staged region).
    constexpr float inv2s = 1.f / (float)(2 * S);
    constexpr int nf = G::nfy * G::nfx;
    const bool interior = ty0 - S >= 0 && tx0 - S >= 0 && ty0 + DTY + S <= H && tx0 + DTX + S <= W;
#pragma unroll
    for (int j = 0; j < (nf + kTileThreads - 1) / kTileThreads; ++j) {
        const int i = threadIdx.x + j * kTileThreads;
        if (i >= nf) continue;
        const int py = i / G::nfx, px = i - py * G::nfx;
        const int gy = ty0 - S + py, gx = tx0 - S + px;
        int ry = py + S, rx = px + S;  // position inside sI
        if (!interior) {
            if (gy > H - 1 + S || gx > W - 1 + S) continue;
            ry = reflect_index(gy, H) - ty0 + 2 * S;
            rx = reflect_index(gx, W) - tx0 + 2 * S;
        }
        const float* c = sI + ry * G::pI + rx;
        const float a00 = c[-S * G::pI - S], a02 = c[-S * G::pI + S];
        const float a20 = c[S * G::pI - S], a22 = c[S * G::pI + S];
        const float a10 = c[-S], a12 = c[S], a01 = c[-S * G::pI], a21 = c[S * G::pI];
        sX[py * G::pF + px] =
            (0.1875f * (a02 - a00) + 0.625f * (a12 - a10) + 0.1875f * (a22 - a20)) * inv2s;
        sY[py * G::pF + px] =
            (0.1875f * (a20 - a00) + 0.625f * (a21 - a01) + 0.1875f * (a22 - a02)) * inv2s;
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < DTX * DTY / kTileThreads; ++j) {
        const int i = threadIdx.x + j * kTileThreads;
        const int ly = i / DTX, lx = i - ly * DTX;
        const int gy = ty0 + ly, gx = tx0 + lx;
        if (gy >= H || gx >= W) continue;
        const float* x = sX + (ly + S) * G::pF + (lx + S);
        const float* y = sY + (ly + S) * G::pF + (lx + S);
        const float x00 = x[-S * G::pF - S], x02 = x[-S * G::pF + S];
        const float x20 = x[S * G::pF - S], x22 = x[S * G::pF + S];
        const float Lxx = (0.1875f * (x02 - x00) + 0.625f * (x[S] - x[-S]) + 0.1875f * (x22 - x20)) * inv2s;
        const float Lxy = (0.1875f * (x20 - x00) + 0.625f * (x[S * G::pF] - x[-S * G::pF]) +
                           0.1875f * (x22 - x02)) * inv2s;
        const float Lyy = (0.1875f * (y[S * G::pF - S] - y[-S * G::pF - S]) +
                           0.625f * (y[S * G::pF] - y[-S * G::pF]) +
                           0.1875f * (y[S * G::pF + S] - y[-S * G::pF + S])) * inv2s;
        det[plane * lev + (size_t)gy * W + gx] = sn2 * (Lxx * Lyy - Lxy * Lxy);
    }
}

struct KeypointOut {
    int x, y, level;
    float response;
};

// (x, y, i) is an extremum iff det_i(x,y) > threshold and > all 26
// neighbours in levels i-1..i+1; levels 1..N-2, 1-pixel image border
// excluded.  A block covers 64 columns x 4*kNmsRows rows of one level.
__global__ __launch_bounds__(256) void nms_kernel(BatchImage d0, ImgWork w, float threshold) {
    BatchImage d;
    int lb;
    resolve(d0, w, (int)blockIdx.x, d, lb);
    const int W = d.W, H = d.H;
    const int nbx = (W + 63) / 64;
    const int x = (lb % nbx) * 64 + threadIdx.x % 64;
    const int y0 = ((lb / nbx) * 4 + threadIdx.x / 64) * kNmsRows;
    const int lev = blockIdx.y + 1;
    if (x < 1 || x > W - 2) return;
    const size_t plane = (size_t)W * H;
    const float* base = d.det + plane * lev;
    float v[kNmsRows];
#pragma unroll
    for (int q = 0; q < kNmsRows; ++q) {
        const int y = y0 + q;
        v[q] = (y >= 1 && y <= H - 2) ? base[(size_t)y * W + x] : -INFINITY;
    }
    KeypointOut* kps = static_cast<KeypointOut*>(d.kps);
#pragma unroll
    for (int q = 0; q < kNmsRows; ++q) {
        if (!(v[q] > threshold)) continue;
        const int y = y0 + q;
        const float* c = base + (size_t)y * W + x;
        bool is_max = true;
        for (int dl = -1; dl <= 1 && is_max; ++dl)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dl == 0 && dy == 0 && dx == 0) continue;
                    is_max = is_max && (v[q] > c[(ptrdiff_t)dl * (ptrdiff_t)plane + dy * W + dx]);
                }
        if (!is_max) continue;
        const int idx = atomicAdd(d.count, 1);
        if (idx < d.capacity) {
            KeypointOut k;
            k.x = x;
            k.y = y;
            k.level = lev;
            k.response = v[q];
            kps[idx] = k;
        }
    }
}

template <int S>
hipError_t launch_det_s(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                        const DetLevels& dl, hipStream_t s) {
    int n = 0;
    for (int i = lev0; i < lev1; ++i) n += dl.step[i] == S;
    const int count = w.items ? w.count : det_tiles_of(d0.W, d0.H);
    if (n == 0 || count <= 0) return hipSuccess;
    const size_t lds = (size_t)DetGeom<S>::floats * sizeof(float);
    hipLaunchKernelGGL(det_kernel<S>, dim3(count, n), dim3(kTileThreads), lds, s, d0, w, dl, lev0,
                       lev1);
    return hipGetLastError();
}

}  // namespace

int det_tiles_of(int W, int H) { return ((W + DTX - 1) / DTX) * ((H + DTY - 1) / DTY); }

int nms_blocks_of(int W, int H) { return ((W + 63) / 64) * ((H + 4 * kNmsRows - 1) / (4 * kNmsRows)); }

hipError_t launch_det(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                      const DetLevels& dl, hipStream_t s) {
    hipError_t e = hipSuccess;
#define KZ_D(S) \
    if (e == hipSuccess) e = launch_det_s<S>(d0, w, lev0, lev1, dl, s);
    KZ_D(1) KZ_D(2) KZ_D(3) KZ_D(4) KZ_D(5) KZ_D(6) KZ_D(7) KZ_D(8)
#undef KZ_D
    return e;
}

hipError_t launch_nms(const BatchImage& d0, const ImgWork& w, int N, float threshold,
                      hipStream_t s) {
    const int count = w.items ? w.count : nms_blocks_of(d0.W, d0.H);
    if (N < 3 || count <= 0) return hipSuccess;
    hipLaunchKernelGGL(nms_kernel, dim3(count, N - 2), dim3(256), 0, s, d0, w, threshold);
    return hipGetLastError();
}

}  // namespace kaze
