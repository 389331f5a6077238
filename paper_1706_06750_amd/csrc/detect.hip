// Detector response (Eq. 8) and 3x3x3 extrema (Sec. II-B).
//
// det_i = sigma_n^2 (L_xx L_yy - L_xy^2) with L_xx = D_x D_x L, L_yy = D_y D_y L,
// L_xy = D_y D_x L, where D_x of step s is the concatenated Scharr filter
//   D_x f(x,y) = sum_{dy in -s,0,s} w_dy (f(x+s, y+dy) - f(x-s, y+dy)) / (2s),
//   w = (3, 10, 3)/16,
// and every derivative image is extended by half-sample reflection before the
// next derivative is taken.  L_x, L_y, L_xx, ... never reach memory.
#include <algorithm>
#include <type_traits>

#include "kaze_internal.h"

namespace kaze {
namespace {

// Threads of a detector block: four independent wavefronts.
constexpr int kDetThreads = 256;
constexpr int kDetWaves = kDetThreads / kWave;

// (3 a0 + 10 a1 + 3 a2) / 16 as one multiply and two fused multiply-adds in
// a fixed order, so that every kernel and instantiation rounds alike.
__device__ __forceinline__ float scharr3(float a0, float a1, float a2) {
    return __builtin_fmaf(0.1875f, a2, __builtin_fmaf(0.625f, a1, 0.1875f * a0));
}

// The same weights across rows, rounded alike when the outer rows swap.
__device__ __forceinline__ float scharr3v(float a0, float a1, float a2) {
    return __builtin_fmaf(0.625f, a1, 0.1875f * (a0 + a2));
}

// Raw buffer access to one plane: the resource in scalar registers, the
// row's byte offset in a scalar register, the lane's byte offset in a vector
// register (no 64-bit address arithmetic per lane).  A lane offset at or
// past the plane's bytes reads 0 and writes nothing.
constexpr int kBufWord3 = 0x00020000;  // raw 32-bit buffer (gfx9)
constexpr unsigned kBufOff = 0x80000000u;  // a lane offset past every plane
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_buffer(const float* p, int W, int H) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, W * H * 4, kBufWord3);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// Index i reflected once (half-sample symmetric) into [0, n): |i| <= n and
// i < 2n.
__device__ __forceinline__ int reflect1(int i, int n) {
    return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}

// A wave-uniform 64-bit word into lane t of (lo, hi): two v_writelane_b32
// with the lane in M0 (no other code of this file uses M0).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void place_word(unsigned long long word, int t, unsigned& lo,
                                           unsigned& hi) {
    const unsigned wl = (unsigned)word, wh = (unsigned)(word >> 32);
    asm volatile(
        "s_mov_b32 m0, %4\n\ts_nop 0\n\t"
        "v_writelane_b32 %0, %2, m0\n\tv_writelane_b32 %1, %3, m0"
        : "+v"(lo), "+v"(hi)
        : "s"(wl), "s"(wh), "s"(t)
        : "m0");
}
#pragma clang diagnostic pop

// Exchange between the lanes of one wavefront through LDS: the LDS executes
// a wavefront's instructions in order, and this fence keeps the compiler from
// moving its LDS accesses across the exchange.
__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// ---------------------------------------------------------------------------
// Strip form.  One wavefront computes det for an output strip of
// SW = 64 - 2S columns and a band of B rows of one level.  Lane l holds the
// first derivatives of column fx = x0 - S + l (the strip plus an S ring on
// each side) and the wavefront walks down the rows of the band:
//
//  * per row of L (staged in an LDS row private to the wavefront, the 2S
//    columns past the last lane included):
//      dL = L(fx+S) - L(fx-S),   sL = scharr3(L(fx-S), L(fx), L(fx+S));
//  * per row of first derivatives (rows of L at -S, 0, +S), each 2S times
//    the derivative:
//      Lx' = scharr3(dL[-S], dL[0], dL[+S]),   Ly' = sL[+S] - sL[-S],
//    staged in LDS so that lane l reads lanes l - S and l + S:
//      dX = Lx'(+S) - Lx'(-S),   wX = scharr3(Lx'(-S), Lx', Lx'(+S)),
//      wY = scharr3(Ly'(-S), Ly', Ly'(+S));
//  * per output row (first-derivative rows at -S, 0, +S):
//      Lxx' = scharr3(dX[-S], dX[0], dX[+S]),  Lxy' = wX[+S] - wX[-S],
//      Lyy' = wY[+S] - wY[-S],
//      det = sigma_n^2 / (2S)^4 (Lxx' Lyy' - Lxy'^2).
//
// dL, sL, dX, wX, wY live in register rings over rows.  Reflection: L is
// read at reflected rows and columns; a first derivative outside the image
// is the derivative at the reflected position (the derivative image is
// extended before the second derivative), taken horizontally through the
// lane each output lane reads (reflected lane numbers fixed per wavefront)
// and vertically by reading the reflected row of the rings.  The last strip
// ends at column W and the last band at row H, so the reflected ring rows
// are known at compile time; an output pixel (and its mask bit) is stored by
// the one strip and band that own it.  Vertical differences change sign
// exactly under a vertical mirror and the vertical Scharr sums (scharr3v)
// are symmetric in their outer rows, so det of mirrored levels is the
// mirrored det, bit for bit.
constexpr int kDetBandSmall = 8;   // rows per band of images lower than `band` allows

// Rows per band for images of height H at step S, bands of `band` rows
// (kDetBandShort or kDetBandTall) where they fit: bands of B rows need
// H == B or H >= B + S (only the first band meets the top border, only the
// last the bottom one) and H >= 2S (rows of L one reflection away); lower
// images take the per-pixel form (0).
__host__ __device__ inline int det_band_rows(int H, int S, int band) {
    if (H == band || H >= band + S) return band;
    if ((H == kDetBandSmall || H >= kDetBandSmall + S) && H >= 2 * S) return kDetBandSmall;
    return 0;
}

__host__ __device__ inline int det_units(int W, int H, int S, int band) {
    const int b = det_band_rows(H, S, band);
    return det_strips(W, S) * (b ? (H + b - 1) / b : 1);
}

// Output columns owned by strip j of ns ([c_lo, c_hi)) and its first column
// x0: regular strips at j * SW, the last one aligned to end at W.
__device__ __forceinline__ void strip_span(int W, int SW, int ns, int j, int& x0, int& c_lo,
                                           int& c_hi) {
    if (j == ns - 1) {
        x0 = W > SW ? W - SW : 0;
        c_lo = x0;
        c_hi = W;
    } else {
        x0 = j * SW;
        c_lo = x0;
        c_hi = min(x0 + SW, W - SW);
    }
}

// Lane holding first-derivative column c (reflected into the image) in a
// strip whose lane 0 holds column x0 - S.
__device__ __forceinline__ int deriv_lane(int c, int W, int x0, int S) {
    const int l = reflect_index(c, W) - x0 + S;
    return l < 0 ? 0 : (l > kWave - 1 ? kWave - 1 : l);
}

template <int S, int B>
__device__ __forceinline__ void det_strip_band(const BatchImage& d, int lev, int unit,
                                               const DetLevels& dl, float* wl, int lane) {
#pragma clang fp contract(off)
    constexpr int SW = kWave - 2 * S;
    constexpr int NL = B + 4 * S;  // rows of L
    constexpr int NF = B + 2 * S;  // rows of first derivatives
    static_assert(SW > 0 && B >= S, "strip and band hold the step");
    const int W = d.W, H = d.H;
    const int ns = det_strips(W, S), nb = (H + B - 1) / B;
    const int j = unit % ns, b = unit / ns;
    int x0, c_lo, c_hi;
    strip_span(W, SW, ns, j, x0, c_lo, c_hi);
    const bool last_b = b == nb - 1;
    const int y0 = last_b ? H - B : b * B;
    const int row_hi = last_b ? H : min(y0 + B, H - B);  // owned rows [y0, row_hi)
    const bool top = y0 == 0, bot = last_b;
    const int fx = x0 - S + lane;
    const bool own_lane = lane >= S && lane < kWave - S && fx >= c_lo && fx < c_hi;
    const unsigned ca = 4u * reflect_index(x0 - 2 * S + lane, W);  // byte offsets
    const unsigned cb = 4u * reflect_index(x0 + kWave - 2 * S + min(lane, 2 * S - 1), W);
    const unsigned co = own_lane ? 4u * fx : kBufOff;  // other lanes store nothing
    const unsigned long long own_bits = __builtin_amdgcn_ballot_w64(own_lane);
    const int am = deriv_lane(fx - S, W, x0, S), ap = deriv_lane(fx + S, W, x0, S);
    const size_t plane = (size_t)W * H;
    const __amdgpu_buffer_rsrc_t rL = plane_buffer(d.levels + plane * lev, W, H);
    const __amdgpu_buffer_rsrc_t rD = plane_buffer(d.det + plane * lev, W, H);
    const float scale = dl.sn2[lev] * (1.f / (16.f * S * S * S * S));
    const float thr = dl.thr;
    float* lrow = wl;               // L(x0 - 2S + i), i < 64 + 2S
    float* frx = wl + 2 * kWave;    // Lx' of the lanes
    float* fry = wl + 3 * kWave;    // Ly' of the lanes

    constexpr int D = 6;  // rows of L in flight
    float qa[D], qb[D];
    auto issue = [&](int k) {
        const int y = y0 - 2 * S + k;
        const unsigned ro = 4u * (unsigned)uniform(reflect1(y, H) * W);
        qa[k % D] = buf_load(rL, ca, ro);
        qb[k % D] = buf_load(rL, cb, ro);
    };
#pragma unroll
    for (int k = 0; k < D; ++k) issue(k);

    float dL[NL], sL[NL], dX[NF], wX[NF], wY[NF];
    unsigned mlo = 0u, mhi = 0u;  // mask word of output row t in lane t
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const float A = qa[k % D], E = qb[k % D];
        if (k + D < NL) issue(k + D);
        lrow[lane] = A;
        lrow[kWave + lane] = E;  // lanes >= 2S store copies nobody reads
        wave_lds_sync();
        const float Lc = lrow[lane + S], Lp = lrow[lane + 2 * S];
        wave_lds_sync();
        dL[k] = Lp - A;
        sL[k] = scharr3(A, Lc, Lp);
        if (k < 2 * S) continue;
        const int q = k - 2 * S;  // first-derivative row y0 - S + q
        const float Lx = scharr3v(dL[k - 2 * S], dL[k - S], dL[k]);
        const float Ly = sL[k] - sL[k - 2 * S];
        frx[lane] = Lx;
        fry[lane] = Ly;
        wave_lds_sync();
        const float xm = frx[am], xp = frx[ap], ym = fry[am], yp = fry[ap];
        wave_lds_sync();
        dX[q] = xp - xm;
        wX[q] = scharr3(xm, Lx, xp);
        wY[q] = scharr3(ym, Ly, yp);
        if (q < 2 * S) continue;
        const int t = q - 2 * S;  // output row y0 + t: derivative rows t, t + S, t + 2S
        float dxa = dX[t], wxa = wX[t], wya = wY[t];
        float dxc = dX[t + 2 * S], wxc = wX[t + 2 * S], wyc = wY[t + 2 * S];
        if (t < S && top) {  // row y0 + t - S < 0: row S - 1 - t
            dxa = dX[2 * S - 1 - t];
            wxa = wX[2 * S - 1 - t];
            wya = wY[2 * S - 1 - t];
        }
        if (t >= B - S && bot) {  // row y0 + t + S >= H: row 2H - 1 - (y0 + t + S)
            dxc = dX[2 * B - 1 - t];
            wxc = wX[2 * B - 1 - t];
            wyc = wY[2 * B - 1 - t];
        }
        const float Lxx = scharr3v(dxa, dX[t + S], dxc);
        const float Lxy = wxc - wxa;
        const float Lyy = wyc - wya;
        const float v = scale * __builtin_fmaf(Lxx, Lyy, -(Lxy * Lxy));
        const int yo = y0 + t;
        if (yo < row_hi) {  // uniform
            buf_store(v, rD, co, 4u * (unsigned)(yo * W));
            if (d.mask)
                place_word((__builtin_amdgcn_ballot_w64(v > thr) & own_bits) >> S, t, mlo, mhi);
        }
    }
    if (d.mask && lane < B && y0 + lane < row_hi) {
        const int mw = mask_words(W);
        ((gu64*)d.mask)[((size_t)lev * H + y0 + lane) * mw + j] =
            ((unsigned long long)mhi << 32) | mlo;
    }
}

// Per-pixel form for images too low for a band (det_band_rows 0): one
// wavefront per strip and all rows, every first derivative formed at its
// reflected position from nine loads of L.  The same formulas as the strip
// form.
template <int S>
__device__ __forceinline__ void det_strip_pixels(const BatchImage& d, int lev, int j,
                                                 const DetLevels& dl, int lane) {
#pragma clang fp contract(off)
    constexpr int SW = kWave - 2 * S;
    const int W = d.W, H = d.H;
    const int ns = det_strips(W, S);
    int x0, c_lo, c_hi;
    strip_span(W, SW, ns, j, x0, c_lo, c_hi);
    const int fx = x0 - S + lane;
    const bool own_lane = lane >= S && lane < kWave - S && fx >= c_lo && fx < c_hi;
    const int ox = own_lane ? fx : c_lo;  // in-image column for every lane
    const size_t plane = (size_t)W * H;
    const gfloat* L = (const gfloat*)d.levels + plane * lev;
    gfloat* det = (gfloat*)d.det + plane * lev;
    const float scale = dl.sn2[lev] * (1.f / (16.f * S * S * S * S));
    // (Lx', Ly') at (xf, yf), extended by reflection
    auto deriv = [&](int xf, int yf, float& lx, float& ly) {
        const int xr = reflect_index(xf, W), yr = reflect_index(yf, H);
        const int xa = reflect_index(xr - S, W), xb = reflect_index(xr + S, W);
        float dd[3], ss[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const gfloat* r = L + (ptrdiff_t)reflect_index(yr + (i - 1) * S, H) * W;
            const float a = r[xa], c = r[xr], e = r[xb];
            dd[i] = e - a;
            ss[i] = scharr3(a, c, e);
        }
        lx = scharr3v(dd[0], dd[1], dd[2]);
        ly = ss[2] - ss[0];
    };
    for (int yo = 0; yo < H; ++yo) {
        float dXr[3], wXr[3], wYr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int yf = yo + (i - 1) * S;
            float xm, ym, xc, yc, xp, yp;
            deriv(ox - S, yf, xm, ym);
            deriv(ox, yf, xc, yc);
            deriv(ox + S, yf, xp, yp);
            dXr[i] = xp - xm;
            wXr[i] = scharr3(xm, xc, xp);
            wYr[i] = scharr3(ym, yc, yp);
        }
        const float Lxx = scharr3v(dXr[0], dXr[1], dXr[2]);
        const float Lxy = wXr[2] - wXr[0];
        const float Lyy = wYr[2] - wYr[0];
        const float v = scale * __builtin_fmaf(Lxx, Lyy, -(Lxy * Lxy));
        if (own_lane) (det + (ptrdiff_t)yo * W)[fx] = v;
        if (d.mask) {
            const unsigned long long bits = __ballot(own_lane && v > dl.thr) >> S;
            if (lane == 0)
                ((gu64*)d.mask)[((size_t)lev * H + yo) * mask_words(W) + j] = bits;
        }
    }
}

template <int S>
__device__ __forceinline__ void det_strip_unit(const BatchImage& d, int lev, int unit,
                                               const DetLevels& dl, float* wl, int lane) {
    if (unit >= det_units(d.W, d.H, S, dl.band)) return;  // uniform per wavefront
    const int B = det_band_rows(d.H, S, dl.band);
    if (B == kDetBandTall)
        det_strip_band<S, kDetBandTall>(d, lev, unit, dl, wl, lane);
    else if (B == kDetBandShort)
        det_strip_band<S, kDetBandShort>(d, lev, unit, dl, wl, lane);
    else if (B == kDetBandSmall)
        det_strip_band<S, kDetBandSmall>(d, lev, unit, dl, wl, lane);
    else
        det_strip_pixels<S>(d, lev, unit, dl, lane);
}

// Levels of Scharr step S (dl.list[0 .. gridDim.y)), or (SB > 0) of steps SA
// and SB in one launch, each block taking the step of its level.  Block bx
// of a level holds units 4 bx .. 4 bx + 3 of its image (one per wavefront,
// strips fastest); blocks run XCD by XCD so that neighbouring strips and
// bands share an L2.
template <int SA, int SB>
__global__ __launch_bounds__(kDetThreads) void det_strip_kernel(BatchImage d0, ImgWork w,
                                                                 DetLevels dl) {
    __shared__ float s_rows[kDetWaves][4 * kWave];
    int bx, by;
    xcd_grid(bx, by);
    const int lev = dl.list[by];
    BatchImage d;
    int lb;
    resolve(d0, w, bx, d, lb);
    const int wave = uniform((int)threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
    const int unit = lb * kDetWaves + wave;
    if (SB == 0 || dl.step[lev] == SA)
        det_strip_unit<SA>(d, lev, unit, dl, s_rows[wave], lane);
    else
        det_strip_unit<SB == 0 ? SA : SB>(d, lev, unit, dl, s_rows[wave], lane);
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
// mask words of a level (the row segments of the detector's strips,
// row-major), and only
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
    // the level's detector strips: word (y, j) holds bit b for column x0_j + b
    const int sw = kWave - 2 * radii.step[lev], ns = det_strips(W, radii.step[lev]);
    const size_t plane = (size_t)W * H;
    const gfloat* base = (const gfloat*)d.det + plane * lev;
    KeypointOut* kps = static_cast<KeypointOut*>(d.kps);
    const int t = threadIdx.x;
    {
        const int g = lb * 256 + t;  // word of the level's mask plane
        const int y = g / mw, xw = g - y * mw;
        unsigned long long bits = 0ull;
        if (y >= 1 && y <= H - 2 && xw < ns)  // rows past H fall out here too
            bits = ((const gu64*)d.mask)[(size_t)lev * H * mw + g];
        // columns 1 .. W-2 of the word: bits 1 - x0 .. W - 2 - x0
        const int x0 = xw == ns - 1 ? max(W - sw, 0) : xw * sw;
        if (x0 == 0) bits &= ~1ull;
        const int hi = W - 2 - x0;
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
            const int xw = g - y * mw;
            x = (xw == ns - 1 ? max(W - sw, 0) : xw * sw) + __ffsll((long long)bits) - 1;
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


// First derivatives for the description stage (steps S <= 4): the
// scale-normalised sigma_n L_x and sigma_n L_y of every pixel, on 64 x 32
// tiles, lane = column.  Phase 1 stages L on the tile + 2S ring (row by row,
// lanes over the first 64 columns, the last 4S columns one value per
// thread); phase 2 computes the first derivatives on the tile + S ring, each
// lane walking a band of rows with the three values of its columns c - S,
// c, c + S of every row in registers.
constexpr int DTX = 64;
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

// One block: tile bx of level lev, Scharr step S; sigma_n L_x and
// sigma_n L_y of the tile to lx and ly.
template <int S>
__device__ __forceinline__ void deriv_rows_tile(float* smem, const BatchImage& d0, const ImgWork& w,
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
}

template <int S>
__global__ __launch_bounds__(kDetThreads) void deriv_rows_kernel(BatchImage d0, ImgWork w,
                                                                  DetLevels dl, float* lx,
                                                                  float* ly) {
    extern __shared__ float smem[];
    int bx, by;
    xcd_grid(bx, by);
    // the launch's levels (all of Scharr step S) are dl.list[0..gridDim.y)
    deriv_rows_tile<S>(smem, d0, w, dl, dl.list[by], bx, lx, ly);
}

// Strip launch of the levels in [lev0, lev1) with Scharr step S (SB = 0) or
// steps SA and SB.
template <int SA, int SB>
hipError_t launch_det_strips(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                             const DetLevels& dl, hipStream_t s) {
    DetLevels dls = dl;  // with the list of this launch's levels
    int n = 0;
    for (int i = lev0; i < lev1; ++i)
        if (dl.step[i] == SA || (SB > 0 && dl.step[i] == SB)) dls.list[n++] = i;
    const int count = w.items ? w.count : det_tiles_of(d0.W, d0.H, SA, SB > 0 ? SB : SA, dl.band);
    if (n == 0 || count <= 0) return hipSuccess;
    hipLaunchKernelGGL((det_strip_kernel<SA, SB>), dim3(count, n), dim3(kDetThreads), 0, s, d0,
                       w, dls);
    return hipGetLastError();
}

}  // namespace

int det_tiles_of(int W, int H, int smin, int smax, int band) {
    int n = 0;
    for (int S = smin; S <= smax; ++S)
        n = std::max(n, (det_units(W, H, S, band) + kDetWaves - 1) / kDetWaves);
    return n;
}

int nms_blocks_of(int W, int H, bool masked) {
    if (masked) return (int)(((long long)H * mask_words(W) + 255) / 256);
    return ((W + 63) / 64) * ((H + 4 * kNmsRows - 1) / (4 * kNmsRows));
}

hipError_t launch_det(const BatchImage& d0, const ImgWork& w, int lev0, int lev1,
                      const DetLevels& dl, hipStream_t s) {
    if (dl.band != kDetBandShort && dl.band != kDetBandTall) return hipErrorInvalidValue;
    // two adjacent steps (the default schedule: 2 and 3) share one launch
    int smin = 1 << 30, smax = 0;
    for (int i = lev0; i < lev1; ++i) {
        smin = std::min(smin, dl.step[i]);
        smax = std::max(smax, dl.step[i]);
    }
    if (smax == 0) return hipSuccess;
    if (smax < 1 || smax > kMaxStep || smin < 1) return hipErrorInvalidValue;
    if (smax == smin + 1) {
        switch (smin) {
            case 1: return launch_det_strips<1, 2>(d0, w, lev0, lev1, dl, s);
            case 2: return launch_det_strips<2, 3>(d0, w, lev0, lev1, dl, s);
            case 3: return launch_det_strips<3, 4>(d0, w, lev0, lev1, dl, s);
            case 4: return launch_det_strips<4, 5>(d0, w, lev0, lev1, dl, s);
            case 5: return launch_det_strips<5, 6>(d0, w, lev0, lev1, dl, s);
            case 6: return launch_det_strips<6, 7>(d0, w, lev0, lev1, dl, s);
            default: return launch_det_strips<7, 8>(d0, w, lev0, lev1, dl, s);
        }
    }
    hipError_t e = hipSuccess;
#define KZ_D(S) \
    if (e == hipSuccess) e = launch_det_strips<S, 0>(d0, w, lev0, lev1, dl, s);
    KZ_D(1) KZ_D(2) KZ_D(3) KZ_D(4) KZ_D(5) KZ_D(6) KZ_D(7) KZ_D(8)
#undef KZ_D
    return e;
}

hipError_t launch_det_derivs(const BatchImage& b, int N, const DetLevels& dl, float* lx,
                             float* ly, hipStream_t s) {
    for (int i = 0; i < N; ++i)
        if (dl.step[i] > 4) return hipErrorNotSupported;  // the caller's per-pixel form
    const int count = ((b.W + DTX - 1) / DTX) * ((b.H + kDetRowsTY - 1) / kDetRowsTY);
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
        hipLaunchKernelGGL((deriv_rows_kernel<S>), dim3(count, n), dim3(kDetThreads), lds, s, b,
                           none, dls, lx, ly);
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
