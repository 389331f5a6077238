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
#include <algorithm>
#include <type_traits>

#include "kaze_internal.h"
#include "tile_stage.h"

namespace kaze {
namespace {

constexpr int DTX = 64;
constexpr int DTY = 32;
// Threads of a detector block (512 measured 3% slower than 256 here, where
// the smoothing and conductivity tiles gain from 512).
constexpr int kDetThreads = 256;

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

// det at (ly, lx) of the tile from the first-derivative planes of det_kernel
template <int S, int pF>
__device__ __forceinline__ float det_at(const float* sX, const float* sY, int ly, int lx,
                                        float inv2s, float sn2) {
    const float* x = sX + (ly + S) * pF + (lx + S);
    const float* y = sY + (ly + S) * pF + (lx + S);
    const float x00 = x[-S * pF - S], x02 = x[-S * pF + S];
    const float x20 = x[S * pF - S], x22 = x[S * pF + S];
    const float Lxx = (0.1875f * (x02 - x00) + 0.625f * (x[S] - x[-S]) + 0.1875f * (x22 - x20)) * inv2s;
    const float Lxy = (0.1875f * (x20 - x00) + 0.625f * (x[S * pF] - x[-S * pF]) +
                       0.1875f * (x22 - x02)) * inv2s;
    const float Lyy = (0.1875f * (y[S * pF - S] - y[-S * pF - S]) +
                       0.625f * (y[S * pF] - y[-S * pF]) +
                       0.1875f * (y[S * pF + S] - y[-S * pF + S])) * inv2s;
    return sn2 * (Lxx * Lyy - Lxy * Lxy);
}

template <int S>
__global__ __launch_bounds__(kDetThreads) void det_kernel(BatchImage d0, ImgWork w, DetLevels dl,
                                                             int lev0, int lev1) {
    using G = DetGeom<S>;
    extern __shared__ float smem[];
    float* sI = smem;
    float* sX = smem + G::offX;
    float* sY = smem + G::offY;
    // (tile, level) of this block: the linear block index dealt out so that
    // each XCD works through a contiguous run of tiles of one level, whose
    // rings then share its L2
    int bx, by;
    xcd_grid(bx, by);
    // levels of this launch: the ones in [lev0, lev1) with Scharr step S
    int lev = -1;
    for (int i = lev0, seen = 0; i < lev1; ++i)
        if (dl.step[i] == S && seen++ == by) lev = i;
    if (lev < 0) return;  // uniform per block
    BatchImage d;
    int lt;
    resolve(d0, w, bx, d, lt);
    const int W = d.W, H = d.H;
    gfloat* __restrict__ det = (gfloat*)d.det;
    const float sn2 = dl.sn2[lev];
    const size_t plane = (size_t)W * H;
    const float* L = d.levels + plane * lev;
    const int ncx = (W + DTX - 1) / DTX;
    const int tx0 = (lt % ncx) * DTX, ty0 = (lt / ncx) * DTY;
    stage_region<G::niy, G::nix, G::pI, kDetThreads>(L, W, H, ty0 - 2 * S, tx0 - 2 * S, sI);
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
    for (int j = 0; j < (nf + kDetThreads - 1) / kDetThreads; ++j) {
        const int i = threadIdx.x + j * kDetThreads;
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

    // a wavefront holds one row of the tile (lane = column): its ballot is
    // the row's mask word
    gu64* mrow = d.mask ? (gu64*)d.mask + (size_t)lev * H * mask_words(W) + tx0 / DTX : nullptr;
#pragma unroll
    for (int j = 0; j < DTX * DTY / kDetThreads; ++j) {
        const int i = threadIdx.x + j * kDetThreads;
        const int ly = i / DTX, lx = i - ly * DTX;
        const int gy = ty0 + ly, gx = tx0 + lx;
        const bool in = gy < H && gx < W;
        float v = 0.f;
        if (in) v = det_at<S, G::pF>(sX, sY, ly, lx, inv2s, sn2);
        if (in) det[plane * lev + (size_t)gy * W + gx] = v;
        if (mrow) {
            const unsigned long long bits = __ballot(in && v > dl.thr);
            if (lx == 0 && gy < H) mrow[(size_t)gy * mask_words(W)] = bits;
        }
    }
}


struct KeypointOut {
    int x, y, level;
    float response;
};

__device__ __forceinline__ void push_keypoint(int* count, int capacity, KeypointOut* kps, int x,
                                              int y, int lev, float v) {
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

// (x, y, i) is an extremum iff det_i(x,y) > threshold, > its 8 neighbours
// in level i and > every response of levels i-1 and i+1 within h = radii.h[i]
// pixels in x and y (clipped to the image; h = 1 is the 3x3x3 block);
// levels 1..N-2, 1-pixel image border excluded.  A block covers 64 columns
// x 4*kNmsRows rows of one level.
// WIDE false: every half-side is 1 (the 3x3x3 test, no wavefront-wide part).
template <bool WIDE>
__global__ __launch_bounds__(256) void nms_kernel(BatchImage d0, ImgWork w, float threshold,
                                                  NmsRadii radii) {
    // The descriptor is read with ordinary loads here: the scalar-load form of
    // resolve() measured 53 instead of 34 us per 1920x1200 image in this
    // kernel (and 1234 instead of 786 us on the 64-image batch).
    BatchImage d;
    int bx, by, lb;
    xcd_grid(bx, by);
    if (w.items) {
        const int2 it = w.items[bx];
        d = w.descs[it.x];
        lb = it.y;
    } else {
        d = d0;
        lb = bx;
    }
    const int W = d.W, H = d.H;
    const int nbx = (W + 63) / 64;
    const int x = (lb % nbx) * 64 + threadIdx.x % 64;
    const int y0 = ((lb / nbx) * 4 + threadIdx.x / 64) * kNmsRows;
    const int lev = by + 1;
    const int h = radii.h[lev];
    const size_t plane = (size_t)W * H;
    const gfloat* base = (const gfloat*)d.det + plane * lev;
    KeypointOut* kps = static_cast<KeypointOut*>(d.kps);
    if constexpr (!WIDE)
        if (x < 1 || x > W - 2) return;
    const bool x_in = !WIDE || (x >= 1 && x <= W - 2);
    float v[kNmsRows];
#pragma unroll
    for (int q = 0; q < kNmsRows; ++q) {
        const int y = y0 + q;
        v[q] = (x_in && y >= 1 && y <= H - 2) ? base[(size_t)y * W + x] : -INFINITY;
    }
    if (!WIDE || h == 1) {
        if (!x_in) return;
#pragma unroll
        for (int q = 0; q < kNmsRows; ++q) {
            if (!(v[q] > threshold)) continue;
            const int y = y0 + q;
            const gfloat* c = base + (size_t)y * W + x;
            bool is_max = true;
            for (int dl = -1; dl <= 1 && is_max; ++dl)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dl == 0 && dy == 0 && dx == 0) continue;
                        is_max = is_max && (v[q] > c[(ptrdiff_t)dl * (ptrdiff_t)plane + dy * W + dx]);
                    }
            if (is_max) push_keypoint(d.count, d.capacity, kps, x, y, lev, v[q]);
        }
        return;
    }
    // Wider cross-level window: the own-level 3x3 test per lane, then the
    // wavefront takes its candidates one at a time and all 64 lanes compare
    // the window of levels lev-1 and lev+1 (clipped to the image) together.
    // Every lane of the wavefront runs this part (the row y is uniform).
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int q = 0; q < kNmsRows; ++q) {
        const int y = y0 + q;
        bool cand = v[q] > threshold;  // false outside the image (-inf)
        if (cand) {
            const gfloat* c = base + (size_t)y * W + x;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if (dy != 0 || dx != 0) cand = cand && (v[q] > c[dy * W + dx]);
        }
        unsigned long long m = __ballot(cand);
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int cx = __builtin_amdgcn_readlane(x, l);
            const float cv = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[q]), l));
            const int wy0 = max(y - h, 0), wy1 = min(y + h, H - 1);
            const int wx0 = max(cx - h, 0), wx1 = min(cx + h, W - 1);
            const int ww = wx1 - wx0 + 1, n = ww * (wy1 - wy0 + 1);
            bool ok = true;
            for (int t = lane; t < 2 * n; t += kWave) {
                const int u = t < n ? t : t - n;
                const ptrdiff_t off = t < n ? -(ptrdiff_t)plane : (ptrdiff_t)plane;
                const int yy = wy0 + u / ww, xx = wx0 + u % ww;
                ok = ok && (cv > base[off + (ptrdiff_t)yy * W + xx]);
            }
            if (__ballot(!ok) == 0 && lane == l) push_keypoint(d.count, d.capacity, kps, x, y, lev, v[q]);
        }
    }
}

// The same test with detector masks.  A block takes 256 consecutive 64-bit
// mask words of a level (row segments of 64 pixels, row-major), and only
// the positions whose bit is set (det above the threshold, typically well
// under 1% of them) are read and tested; the rest of the level is never
// loaded.  Set bits come in clusters (blobs of strong response), so they
// are dealt out evenly: a block scan of the words' bit counts numbers the
// block's set bits, and in each round thread t takes bit number
// round * 256 + t.
template <bool WIDE>
__global__ __launch_bounds__(256) void nms_mask_kernel(BatchImage d0, ImgWork w, float threshold,
                                                       NmsRadii radii) {
    __shared__ unsigned long long s_bits[256];
    __shared__ int s_inc[256];  // inclusive prefix sums of the bit counts
    BatchImage d;
    int bx, by, lb;
    xcd_grid(bx, by);
    if (w.items) {
        const int2 it = w.items[bx];
        d = w.descs[it.x];
        lb = it.y;
    } else {
        d = d0;
        lb = bx;
    }
    const int W = d.W, H = d.H, mw = mask_words(W);
    const int lev = by + 1;
    const int h = radii.h[lev];
    const size_t plane = (size_t)W * H;
    const gfloat* base = (const gfloat*)d.det + plane * lev;
    KeypointOut* kps = static_cast<KeypointOut*>(d.kps);
    const int t = threadIdx.x;
    {
        const int g = lb * 256 + t;  // word of the level's mask plane
        const int y = g / mw, xw = g - y * mw;
        unsigned long long bits = 0ull;
        if (y >= 1 && y <= H - 2)  // rows past H fall out here too
            bits = ((const gu64*)d.mask)[(size_t)lev * H * mw + g];
        // columns 1 .. W-2 of the word: bits max(0, 1 - 64 xw) .. W - 2 - 64 xw
        if (xw == 0) bits &= ~1ull;
        const int hi = W - 2 - 64 * xw;
        if (hi < 63) bits &= hi >= 0 ? (2ull << hi) - 1ull : 0ull;
        s_bits[t] = bits;
        s_inc[t] = __popcll(bits);
    }
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
        const int v = t >= off ? s_inc[t - off] : 0;
        __syncthreads();
        s_inc[t] += v;
        __syncthreads();
    }
    const int total = s_inc[255];
    const int lane = t & (kWave - 1);
    for (int r = 0; r < total; r += 256) {  // uniform over the block
        const int q = r + t;
        bool cand = false;
        int x = 0, y = 0;
        float v = 0.f;
        if (q < total) {
            // word o holding bit number q: the first with s_inc[o] > q
            int lo = 0, hi = 255;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_inc[mid] > q) hi = mid;
                else lo = mid + 1;
            }
            unsigned long long bits = s_bits[lo];
            for (int k = q - (s_inc[lo] - __popcll(bits)); k > 0; --k) bits &= bits - 1ull;
            const int g = lb * 256 + lo;
            y = g / mw;
            x = 64 * (g - y * mw) + __ffsll((long long)bits) - 1;
            const gfloat* c = base + (size_t)y * W + x;
            v = c[0];
            cand = v > threshold;
            // own level first (all eight loads issued together), then, for
            // the 3x3x3 test, levels lev-1 and lev+1
            float nb[8];
#pragma unroll
            for (int j = 0, dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    if (dy != 0 || dx != 0) nb[j++] = c[dy * W + dx];
#pragma unroll
            for (int j = 0; j < 8; ++j) cand = cand && v > nb[j];
            if (cand && (!WIDE || h == 1)) {
                float up[9], dn[9];
#pragma unroll
                for (int j = 0, dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx, ++j) {
                        up[j] = c[(ptrdiff_t)plane + dy * W + dx];
                        dn[j] = c[-(ptrdiff_t)plane + dy * W + dx];
                    }
                bool is_max = true;
#pragma unroll
                for (int j = 0; j < 9; ++j) is_max = is_max && v > up[j] && v > dn[j];
                if (is_max) push_keypoint(d.count, d.capacity, kps, x, y, lev, v);
            }
        }
        if constexpr (WIDE) {
            if (h == 1) continue;  // uniform: the level's window is 3x3
            // wider cross-level window: the wavefront checks its candidates
            // one at a time with all 64 lanes over the window of levels
            // lev-1 and lev+1 (clipped to the image)
            unsigned long long m = __ballot(cand);
            while (m) {
                const int l = __ffsll((long long)m) - 1;
                m &= m - 1;
                const int cx = __builtin_amdgcn_readlane(x, l);
                const int cy = __builtin_amdgcn_readlane(y, l);
                const float cv = __builtin_bit_cast(
                    float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
                const int wy0 = max(cy - h, 0), wy1 = min(cy + h, H - 1);
                const int wx0 = max(cx - h, 0), wx1 = min(cx + h, W - 1);
                const int ww = wx1 - wx0 + 1, n = ww * (wy1 - wy0 + 1);
                bool ok = true;
                for (int u2 = lane; u2 < 2 * n; u2 += kWave) {
                    const int u = u2 < n ? u2 : u2 - n;
                    const ptrdiff_t off = u2 < n ? -(ptrdiff_t)plane : (ptrdiff_t)plane;
                    const int yy = wy0 + u / ww, xx = wx0 + u % ww;
                    ok = ok && (cv > base[off + (ptrdiff_t)yy * W + xx]);
                }
                if (__ballot(!ok) == 0 && lane == l)
                    push_keypoint(d.count, d.capacity, kps, x, y, lev, v);
            }
        }
    }
}

// Keypoint refinement (Sec. II-B, Eqs. 9-12): one thread per extremum.  The
// least-squares quadratic on the 3x3 window has orthogonal regressors, so
// each coefficient is a projection of the nine samples.
__global__ __launch_bounds__(256) void refine_kernel(const float* det, int W, int H, int N,
                                                     const KeypointOut* kps, const int* count,
                                                     int capacity, float thr, RefinedKeypoint* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = min(*count, capacity);
    if (i >= n) return;
    const KeypointOut k = kps[i];
    RefinedKeypoint r;
    r.level = k.level;
    if (k.level < 0 || k.level >= N || k.x < 1 || k.x > W - 2 || k.y < 1 || k.y > H - 2) {
        // no full 3x3 window: not a keypoint find_extrema writes
        r.x = (float)k.x;
        r.y = (float)k.y;
        r.response = r.edge_ratio = __builtin_nanf("");
        r.kept = 0;
        out[i] = r;
        return;
    }
    const float* c = det + (size_t)W * H * k.level + (size_t)k.y * W + k.x;
    float p[3][3];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int u = 0; u < 3; ++u) p[v][u] = c[(ptrdiff_t)(v - 1) * W + (u - 1)];
    const float col_l = p[0][0] + p[1][0] + p[2][0], col_m = p[0][1] + p[1][1] + p[2][1];
    const float col_r = p[0][2] + p[1][2] + p[2][2];
    const float row_t = p[0][0] + p[0][1] + p[0][2], row_m = p[1][0] + p[1][1] + p[1][2];
    const float row_b = p[2][0] + p[2][1] + p[2][2];
    const float b = (col_r - col_l) * (1.f / 6.f);
    const float cc = (row_b - row_t) * (1.f / 6.f);
    const float f = ((p[2][2] - p[2][0]) - (p[0][2] - p[0][0])) * 0.25f;
    const float d = ((col_l + col_r) - 2.f * col_m) * (1.f / 6.f);
    const float e = ((row_t + row_b) - 2.f * row_m) * (1.f / 6.f);
    const float a = (col_l + col_m + col_r) * (1.f / 9.f) - (2.f / 3.f) * (d + e);
    const float hxx = 2.f * d, hyy = 2.f * e, hxy = f;
    const float dt = hxx * hyy - hxy * hxy, tr = hxx + hyy;
    r.edge_ratio = dt > 0.f ? tr * tr / dt : __builtin_inff();
    const float du = dt != 0.f ? -(hyy * b - hxy * cc) / dt : __builtin_inff();
    const float dv = dt != 0.f ? -(hxx * cc - hxy * b) / dt : __builtin_inff();
    r.x = k.x + du;
    r.y = k.y + dv;
    r.response = dt != 0.f ? a + b * du + cc * dv + d * du * du + e * dv * dv + f * du * dv
                           : __builtin_nanf("");
    r.kept = dt > 0.f && tr < 0.f && r.edge_ratio < thr && fabsf(du) <= 1.f && fabsf(dv) <= 1.f;
    out[i] = r;
}

// Row-rolling form for steps S <= 4 (the default schedule's are 2 and 3):
// lane = column, so no index needs a division and every row address is
// wave-uniform.  Phase 1 stages L on the tile + 2S ring (row by row, lanes
// over the first 64 columns, the last 4S columns one value per thread);
// phase 2 computes the first derivatives on the tile + S ring, each lane
// walking a band of rows with the three values of its columns c - S, c,
// c + S of every row in registers; phase 3 does the same over the first
// derivatives for L_xx, L_xy, L_yy and stores det row by row.  Ring
// positions outside the image then take the derivative at their reflected
// position (a copy inside LDS, border tiles only).  The arithmetic is the
// 2-D kernel's, term for term.
constexpr int kDetRowsTY = 32;

template <int S>
struct RowDetGeom {
    static constexpr int TY = kDetRowsTY;
    static constexpr int NY = TY + 4 * S, NX = DTX + 4 * S, PI = NX | 1;
    static constexpr int NYF = TY + 2 * S, NXF = DTX + 2 * S, PF = NXF | 1;
    static constexpr int offX = NY * PI, offY = offX + NYF * PF, floats = offY + NYF * PF;
    static constexpr int WAVES = kDetThreads / kWave;
    static constexpr int RPW = (NY + WAVES - 1) / WAVES;     // staged rows per wave
    static constexpr int FB = (NYF + WAVES - 1) / WAVES;     // first-derivative rows per wave
    static constexpr int OB = TY / WAVES;                    // output rows per wave
    static_assert(OB * WAVES == TY, "output bands tile the tile");
};

__device__ __forceinline__ float scharr3(float a0, float a1, float a2) {
    return 0.1875f * a0 + 0.625f * a1 + 0.1875f * a2;
}

// DERIV: write the scale-normalised first derivatives sigma_n L_x and
// sigma_n L_y of the tile to lx and ly instead of det (phases 1-2 only).
// One block: tile bx (of the work list) of level lev, Scharr step S.
template <int S, bool DERIV>
__device__ __forceinline__ void det_rows_tile(float* smem, const BatchImage& d0, const ImgWork& w,
                                              const DetLevels& dl, int lev, int bx, float* lx,
                                              float* ly) {
    using G = RowDetGeom<S>;
    float* sI = smem;
    float* sX = smem + G::offX;
    float* sY = smem + G::offY;
    BatchImage d;
    int lt;
    resolve(d0, w, bx, d, lt);
    const int W = d.W, H = d.H;
    const int tid = threadIdx.x, wave = uniform(tid / kWave), lane = tid % kWave;
    const float sn2 = dl.sn2[lev];
    const size_t plane = (size_t)W * H;
    const gfloat* L = (const gfloat*)(d.levels + plane * lev);
    const int ncx = (W + DTX - 1) / DTX;
    const int tx0 = (lt % ncx) * DTX, ty0 = (lt / ncx) * G::TY;
    constexpr float inv2s = 1.f / (float)(2 * S);

    // phase 1: L on rows ty0-2S.., columns tx0-2S.. (reflected).  Offsets
    // within a plane fit 32 bits (sides <= 4096); a tile whose ring lies in
    // the image skips the reflection.
    {
        const int gy0 = ty0 - 2 * S, gx0 = tx0 - 2 * S;
        const bool inside = gy0 >= 0 && gx0 >= 0 && gy0 + G::NY <= H && gx0 + G::NX <= W;
        constexpr int NE = G::NY * 4 * S;  // the last 4S columns
        constexpr int PE = (NE + kDetThreads - 1) / kDetThreads;
        float v[G::RPW], e[PE];
        if (inside) {
            const gfloat* Lt = L + gy0 * W + gx0;
#pragma unroll
            for (int j = 0; j < G::RPW; ++j) {
                const int r = min(wave + G::WAVES * j, G::NY - 1);
                v[j] = Lt[r * W + lane];
            }
#pragma unroll
            for (int q = 0; q < PE; ++q) {
                const int i = tid + q * kDetThreads;
                const int r = min(i / (4 * S), G::NY - 1), c = DTX + i % (4 * S);
                e[q] = Lt[r * W + c];
            }
        } else {
            const int gxa = reflect_index(gx0 + lane, W);
#pragma unroll
            for (int j = 0; j < G::RPW; ++j) {
                const int r = min(wave + G::WAVES * j, G::NY - 1);
                v[j] = L[uniform(reflect_index(gy0 + r, H)) * W + gxa];
            }
#pragma unroll
            for (int q = 0; q < PE; ++q) {
                const int i = tid + q * kDetThreads;
                const int r = min(i / (4 * S), G::NY - 1), c = DTX + i % (4 * S);
                e[q] = L[reflect_index(gy0 + r, H) * W + reflect_index(gx0 + c, W)];
            }
        }
#pragma unroll
        for (int j = 0; j < G::RPW; ++j) {
            const int r = wave + G::WAVES * j;
            if (r < G::NY) sI[r * G::PI + lane] = v[j];
        }
#pragma unroll
        for (int q = 0; q < PE; ++q) {
            const int i = tid + q * kDetThreads;
            if (i < NE) sI[(i / (4 * S)) * G::PI + DTX + i % (4 * S)] = e[q];
        }
    }
    __syncthreads();

    // phase 2: first derivatives at f-row rf, f-column cf (image row
    // ty0 - S + rf, column tx0 - S + cf), from staged rows rf, rf+S, rf+2S
    // and columns cf, cf+S, cf+2S
    {
        const int f0 = wave * G::FB;
        constexpr int K = G::FB + 2 * S;
        float aL[K], aC[K], aR[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float* row = sI + min(f0 + k, G::NY - 1) * G::PI + lane;
            aL[k] = row[0];
            aC[k] = row[S];
            aR[k] = row[2 * S];
        }
#pragma unroll
        for (int t = 0; t < G::FB; ++t) {
            const int rf = f0 + t;
            if (rf < G::NYF) {
                sX[rf * G::PF + lane] =
                    scharr3(aR[t] - aL[t], aR[t + S] - aL[t + S], aR[t + 2 * S] - aL[t + 2 * S]) * inv2s;
                sY[rf * G::PF + lane] =
                    scharr3(aL[t + 2 * S] - aL[t], aC[t + 2 * S] - aC[t], aR[t + 2 * S] - aR[t]) * inv2s;
            }
        }
        // the last 2S f-columns, one position per thread
        constexpr int NE = G::NYF * 2 * S;
        for (int i = tid; i < NE; i += kDetThreads) {
            const int rf = i / (2 * S), cf = DTX + i % (2 * S);
            const float* c = sI + (rf + S) * G::PI + (cf + S);
            const float a00 = c[-S * G::PI - S], a02 = c[-S * G::PI + S];
            const float a20 = c[S * G::PI - S], a22 = c[S * G::PI + S];
            const float a10 = c[-S], a12 = c[S], a01 = c[-S * G::PI], a21 = c[S * G::PI];
            sX[rf * G::PF + cf] = scharr3(a02 - a00, a12 - a10, a22 - a20) * inv2s;
            sY[rf * G::PF + cf] = scharr3(a20 - a00, a21 - a01, a22 - a02) * inv2s;
        }
    }
    __syncthreads();
    if constexpr (DERIV) {
        // tile pixel (r, c) sits at f-row r + S, f-column c + S
        const float sn = dl.sn[lev];
        const int gx = tx0 + lane;
        gfloat* ox = (gfloat*)lx + plane * lev + (ty0 + wave * G::OB) * W + tx0;
        gfloat* oy = (gfloat*)ly + plane * lev + (ty0 + wave * G::OB) * W + tx0;
#pragma unroll
        for (int t = 0; t < G::OB; ++t) {
            const int rf = wave * G::OB + t + S;
            if (ty0 + wave * G::OB + t < H && gx < W) {
                ox[t * W + lane] = sn * sX[rf * G::PF + lane + S];
                oy[t * W + lane] = sn * sY[rf * G::PF + lane + S];
            }
        }
        return;
    }
    // ring positions outside the image take the derivative at their
    // reflected (in-image, already computed) position
    if (ty0 - S < 0 || tx0 - S < 0 || ty0 + G::TY + S > H || tx0 + DTX + S > W) {
        for (int i = tid; i < G::NYF * G::NXF; i += kDetThreads) {
            const int rf = i / G::NXF, cf = i - rf * G::NXF;
            const int gy = ty0 - S + rf, gx = tx0 - S + cf;
            const bool out = gy < 0 || gx < 0 || gy >= H || gx >= W;
            if (!out || gy > H - 1 + S || gx > W - 1 + S) continue;
            const int sy = reflect_index(gy, H) - ty0 + S, sx = reflect_index(gx, W) - tx0 + S;
            sX[rf * G::PF + cf] = sX[sy * G::PF + sx];
            sY[rf * G::PF + cf] = sY[sy * G::PF + sx];
        }
        __syncthreads();
    }

    // phase 3: output row r (tile) uses f-rows r, r+S, r+2S and f-columns
    // c, c+S, c+2S.  Per f-row k of the wavefront's band: the difference
    // dX = L_x(c+2S) - L_x(c) and the Scharr-weighted sums wX, wY of L_x and
    // L_y over the columns c, c+S, c+2S.  Then, each up to the factor
    // 1/(2S) (the three of them folded into sigma_n^2):
    //   L_xx = scharr3(dX[r], dX[r+S], dX[r+2S]),
    //   L_xy = wX[r+2S] - wX[r],   L_yy = wY[r+2S] - wY[r].
    {
        const int o0 = wave * G::OB;
        constexpr int K = G::OB + 2 * S;
        float dX[K], wX[K], wY[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float* rx = sX + (o0 + k) * G::PF + lane;
            const float* ry = sY + (o0 + k) * G::PF + lane;
            dX[k] = rx[2 * S] - rx[0];
            wX[k] = scharr3(rx[0], rx[S], rx[2 * S]);
            wY[k] = scharr3(ry[0], ry[S], ry[2 * S]);
        }
        const float scale = sn2 * (inv2s * inv2s);
        float v[G::OB];
#pragma unroll
        for (int t = 0; t < G::OB; ++t) {
            const float Lxx = scharr3(dX[t], dX[t + S], dX[t + 2 * S]);
            const float Lxy = wX[t + 2 * S] - wX[t];
            const float Lyy = wY[t + 2 * S] - wY[t];
            v[t] = scale * (Lxx * Lyy - Lxy * Lxy);
        }
        const int gx = tx0 + lane;
        const int rows = uniform(H - (ty0 + o0));  // rows of the band inside the image
        gfloat* out = (gfloat*)(d.det + plane * lev) + (ty0 + o0) * W + tx0;
        // row pointers are wave-uniform (scalar base, the lane as offset)
        if (rows >= G::OB && tx0 + DTX <= W) {
#pragma unroll
            for (int t = 0; t < G::OB; ++t) (out + t * W)[lane] = v[t];
        } else {
#pragma unroll
            for (int t = 0; t < G::OB; ++t)
                if (t < rows && gx < W) (out + t * W)[lane] = v[t];
        }
        if (d.mask) {
            // the mask word of row t is the wavefront's ballot; lane t
            // stores it
            unsigned long long word = 0ull;
#pragma unroll
            for (int t = 0; t < G::OB; ++t) {
                const unsigned long long bits = __ballot(gx < W && v[t] > dl.thr);
                word = lane == t ? bits : word;
            }
            if (lane < G::OB && lane < rows)
                ((gu64*)d.mask)[((size_t)lev * H + ty0 + o0 + lane) * mask_words(W) + tx0 / DTX] =
                    word;
        }
    }
}

template <int S, bool DERIV = false>
__global__ __launch_bounds__(kDetThreads) void det_rows_kernel(BatchImage d0, ImgWork w,
                                                                DetLevels dl, float* lx = nullptr,
                                                                float* ly = nullptr) {
    extern __shared__ float smem[];
    int bx, by;
    xcd_grid(bx, by);
    // the launch's levels (all of Scharr step S) are dl.list[0..gridDim.y)
    det_rows_tile<S, DERIV>(smem, d0, w, dl, dl.list[by], bx, lx, ly);
}

// Levels of two Scharr steps in one launch (one ramp and one tail instead of
// two): each block takes the step of its level.
template <int SA, int SB>
__global__ __launch_bounds__(kDetThreads) void det_rows_pair_kernel(BatchImage d0, ImgWork w,
                                                                     DetLevels dl) {
    extern __shared__ float smem[];
    int bx, by;
    xcd_grid(bx, by);
    const int lev = dl.list[by];
    if (dl.step[lev] == SA)
        det_rows_tile<SA, false>(smem, d0, w, dl, lev, bx, nullptr, nullptr);
    else
        det_rows_tile<SB, false>(smem, d0, w, dl, lev, bx, nullptr, nullptr);
}

template <int S>
hipError_t launch_det_s(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                        const DetLevels& dl, hipStream_t s) {
    DetLevels dls = dl;  // with the list of this launch's levels
    int n = 0;
    for (int i = lev0; i < lev1; ++i)
        if (dl.step[i] == S) dls.list[n++] = i;
    const int count = w.items ? w.count : det_tiles_of(d0.W, d0.H);
    if (n == 0 || count <= 0) return hipSuccess;
    if constexpr (S <= 4) {
        static_assert(kDetRowsTY == DTY, "both forms tile alike");
        const size_t lds = (size_t)RowDetGeom<S>::floats * sizeof(float);
        hipLaunchKernelGGL(det_rows_kernel<S>, dim3(count, n), dim3(kDetThreads), lds, s, d0, w,
                           dls, nullptr, nullptr);
    } else {
        const size_t lds = (size_t)DetGeom<S>::floats * sizeof(float);
        hipLaunchKernelGGL(det_kernel<S>, dim3(count, n), dim3(kDetThreads), lds, s, d0, w, dl,
                           lev0, lev1);
    }
    return hipGetLastError();
}

// Levels of steps SA and SB (and no other) in [lev0, lev1): one launch.
template <int SA, int SB>
hipError_t launch_det_pair(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                           const DetLevels& dl, hipStream_t s) {
    DetLevels dls = dl;
    int n = 0;
    for (int i = lev0; i < lev1; ++i) dls.list[n++] = i;
    const int count = w.items ? w.count : det_tiles_of(d0.W, d0.H);
    if (n == 0 || count <= 0) return hipSuccess;
    const size_t lds =
        (size_t)std::max(RowDetGeom<SA>::floats, RowDetGeom<SB>::floats) * sizeof(float);
    hipLaunchKernelGGL((det_rows_pair_kernel<SA, SB>), dim3(count, n), dim3(kDetThreads), lds, s,
                       d0, w, dls);
    return hipGetLastError();
}

}  // namespace

int det_tiles_of(int W, int H) { return ((W + DTX - 1) / DTX) * ((H + DTY - 1) / DTY); }

int nms_blocks_of(int W, int H, bool masked) {
    if (masked) return (int)(((long long)H * mask_words(W) + 255) / 256);
    return ((W + 63) / 64) * ((H + 4 * kNmsRows - 1) / (4 * kNmsRows));
}

hipError_t launch_det(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                      const DetLevels& dl, hipStream_t s) {
    // two adjacent steps (the default schedule: 2 and 3) share one launch
    int smin = 1 << 30, smax = 0;
    for (int i = lev0; i < lev1; ++i) {
        smin = std::min(smin, dl.step[i]);
        smax = std::max(smax, dl.step[i]);
    }
    if (smax == smin + 1 && smax <= 4) {
        if (smin == 1) return launch_det_pair<1, 2>(d0, w, lev0, lev1, dl, s);
        if (smin == 2) return launch_det_pair<2, 3>(d0, w, lev0, lev1, dl, s);
        return launch_det_pair<3, 4>(d0, w, lev0, lev1, dl, s);
    }
    hipError_t e = hipSuccess;
#define KZ_D(S) \
    if (e == hipSuccess) e = launch_det_s<S>(d0, w, lev0, lev1, dl, s);
    KZ_D(1) KZ_D(2) KZ_D(3) KZ_D(4) KZ_D(5) KZ_D(6) KZ_D(7) KZ_D(8)
#undef KZ_D
    return e;
}

hipError_t launch_det_derivs(const BatchImage& b, int N, const DetLevels& dl, float* lx,
                             float* ly, hipStream_t s) {
    for (int i = 0; i < N; ++i)
        if (dl.step[i] > 4) return hipErrorNotSupported;  // the caller's per-pixel form
    const int count = det_tiles_of(b.W, b.H);
    const ImgWork none{nullptr, nullptr, 0};
    hipError_t e = hipSuccess;
    auto one = [&](auto tag) {
        constexpr int S = decltype(tag)::value;
        DetLevels dls = dl;
        int n = 0;
        for (int i = 0; i < N; ++i)
            if (dl.step[i] == S) dls.list[n++] = i;
        if (n == 0 || e != hipSuccess) return;
        const size_t lds = (size_t)RowDetGeom<S>::floats * sizeof(float);
        hipLaunchKernelGGL((det_rows_kernel<S, true>), dim3(count, n), dim3(kDetThreads), lds, s,
                           b, none, dls, lx, ly);
        e = hipGetLastError();
    };
    one(std::integral_constant<int, 1>{});
    one(std::integral_constant<int, 2>{});
    one(std::integral_constant<int, 3>{});
    one(std::integral_constant<int, 4>{});
    return e;
}

hipError_t launch_refine(const float* det, int W, int H, int N, const void* kps,
                         const int* count, int capacity, float thr, void* out, hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    hipLaunchKernelGGL(refine_kernel, dim3((capacity + 255) / 256), dim3(256), 0, s, det, W, H, N,
                       static_cast<const KeypointOut*>(kps), count, capacity, thr,
                       static_cast<RefinedKeypoint*>(out));
    return hipGetLastError();
}

hipError_t launch_nms(const BatchImage& d0, const ImgWork& w, int N, float threshold,
                      const NmsRadii& radii, hipStream_t s, bool masked) {
    const int count = w.items ? w.count : nms_blocks_of(d0.W, d0.H, masked);
    if (N < 3 || count <= 0) return hipSuccess;
    bool wide = false;
    for (int i = 0; i < N && i < kMaxLevels; ++i) wide = wide || radii.h[i] > 1;
    if (masked && wide)
        hipLaunchKernelGGL(nms_mask_kernel<true>, dim3(count, N - 2), dim3(256), 0, s, d0, w,
                           threshold, radii);
    else if (masked)
        hipLaunchKernelGGL(nms_mask_kernel<false>, dim3(count, N - 2), dim3(256), 0, s, d0, w,
                           threshold, radii);
    else if (wide)
        hipLaunchKernelGGL(nms_kernel<true>, dim3(count, N - 2), dim3(256), 0, s, d0, w, threshold,
                           radii);
    else
        hipLaunchKernelGGL(nms_kernel<false>, dim3(count, N - 2), dim3(256), 0, s, d0, w,
                           threshold, radii);
    return hipGetLastError();
}

}  // namespace kaze
