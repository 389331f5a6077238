// Description stage (Sec. II-C, Sec. III-C): scale-normalised first
// derivatives of every level, the dominant orientation of each keypoint and
// its 64-D M-SURF descriptor.
//
// Derivatives: Lx = sigma_n D_x L, Ly = sigma_n D_y L with the detector's
// concatenated Scharr filter of step round(sigma_n) (Eq. 8), one thread per
// pixel reading its 3x3 neighbourhood of step s (reflected at the border).
//
// Orientation and descriptor: one block of 256 threads per keypoint, scale
// unit s = sigma_i of its level.  Samples at real positions are bilinear in
// Lx and Ly with the image reflected (period 2n) outside.
//  * Orientation: the 113 integer offsets (u, v) with u^2 + v^2 <= 36, one
//    per thread, each a Gaussian-weighted (2.5 s) response with its angle,
//    kept in LDS; the sum of a pi/3 sector changes only where an edge
//    crosses a response, so the 226 half-open sectors that start just after
//    or end at a response's angle hold every sum it takes; one thread per
//    sector, and the block takes the longest (ties: the lowest sector index).
//  * Descriptor: 4 x 4 subregions of 9 x 9 samples (step s, centres at
//    -7.5, -2.5, 2.5, 7.5 s along and across the orientation), 16 threads
//    per subregion with 5-6 samples each, gathered before they are summed;
//    Gaussian weights 2.5 s at the subregion centre and 1.5 subregions over
//    the 4 x 4 mask; sums of the derivatives along and across the
//    orientation and of their magnitudes; unit length over the 64 values.
#include "kaze_internal.h"

namespace kaze {
namespace {

constexpr int kDerivTX = 64, kDerivTY = 4;
constexpr int kOriSamples = 113;     // integer (u, v), u^2 + v^2 <= 36
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kSector = 1.04719755119659774615f;  // pi / 3

struct OriTable {
    signed char u[kOriSamples], v[kOriSamples];
};

constexpr OriTable make_ori_table() {
    OriTable t{};
    int n = 0;
    for (int v = -6; v <= 6; ++v)
        for (int u = -6; u <= 6; ++u)
            if (u * u + v * v <= 36) {
                t.u[n] = (signed char)u;
                t.v[n] = (signed char)v;
                ++n;
            }
    return t;
}

__constant__ OriTable kOri = make_ori_table();

__global__ __launch_bounds__(kDerivTX * kDerivTY) void deriv_kernel(const float* levels, int W,
                                                                      int H, DescLevels dl,
                                                                      float* lx, float* ly) {
    const int x = blockIdx.x * kDerivTX + (int)(threadIdx.x % kDerivTX);
    const int y = blockIdx.y * kDerivTY + (int)(threadIdx.x / kDerivTX);
    const int lev = blockIdx.z;
    if (x >= W || y >= H) return;
    const int S = dl.step[lev];
    const size_t plane = (size_t)W * H;
    const float* L = levels + plane * lev;
    const bool in = x >= S && x < W - S && y >= S && y < H - S;
    const int xm = in ? x - S : reflect_index(x - S, W), xp = in ? x + S : reflect_index(x + S, W);
    const int ym = in ? y - S : reflect_index(y - S, H), yp = in ? y + S : reflect_index(y + S, H);
    const float* rm = L + (size_t)ym * W;
    const float* r0 = L + (size_t)y * W;
    const float* rp = L + (size_t)yp * W;
    const float a00 = rm[xm], a01 = rm[x], a02 = rm[xp];
    const float a10 = r0[xm], a12 = r0[xp];
    const float a20 = rp[xm], a21 = rp[x], a22 = rp[xp];
    const float k = dl.sn[lev] / (float)(2 * S);
    const size_t o = plane * lev + (size_t)y * W + x;
    lx[o] = k * (0.1875f * (a02 - a00) + 0.625f * (a12 - a10) + 0.1875f * (a22 - a20));
    ly[o] = k * (0.1875f * (a20 - a00) + 0.625f * (a21 - a01) + 0.1875f * (a22 - a02));
}

__device__ __forceinline__ void bilinear2(const float* gx, const float* gy, int W, int H, float x,
                                          float y, float& vx, float& vy) {
    const float fx0 = floorf(x), fy0 = floorf(y);
    const float fx = x - fx0, fy = y - fy0;
    const int x0 = (int)fx0, y0 = (int)fy0;
    const int xa = reflect_index(x0, W), xb = reflect_index(x0 + 1, W);
    const size_t ya = (size_t)reflect_index(y0, H) * W, yb = (size_t)reflect_index(y0 + 1, H) * W;
    const float tx = (1.f - fx) * gx[ya + xa] + fx * gx[ya + xb];
    const float bx = (1.f - fx) * gx[yb + xa] + fx * gx[yb + xb];
    const float ty = (1.f - fx) * gy[ya + xa] + fx * gy[ya + xb];
    const float by = (1.f - fx) * gy[yb + xa] + fx * gy[yb + xb];
    vx = (1.f - fy) * tx + fy * bx;
    vy = (1.f - fy) * ty + fy * by;
}

struct Best {
    float len2;
    int idx;
    float sx, sy;
};

// by value, field by field: a select between a shared and a private
// record would take their addresses
__device__ __forceinline__ Best better(Best a, Best b) {
    const bool t = b.len2 > a.len2 || (b.len2 == a.len2 && b.idx < a.idx);
    return Best{t ? b.len2 : a.len2, t ? b.idx : a.idx, t ? b.sx : a.sx, t ? b.sy : a.sy};
}

__device__ __forceinline__ Best shfl_best(const Best& b, int mask) {
    Best o;
    o.len2 = __shfl_xor(b.len2, mask);
    o.idx = __shfl_xor(b.idx, mask);
    o.sx = __shfl_xor(b.sx, mask);
    o.sy = __shfl_xor(b.sy, mask);
    return o;
}

constexpr int kDescThreads = 256;
constexpr int kDescWaves = kDescThreads / kWave;

// One block per keypoint: thread t < 113 takes orientation sample t; thread
// t < 226 evaluates sector t (sample t / 2, "after" for even t, "before"
// for odd t, the order of the tie rule); for the descriptor thread t takes
// subregion t / 16 and every 16th of its 81 samples from t % 16.
__global__ __launch_bounds__(kDescThreads) void describe_kernel(
    const float* lx, const float* ly, int W, int H, int N, DescLevels dl, const RefinedKeypoint* kps,
    const int* count, int capacity, float* angles, float* desc) {
    __shared__ float sRx[kOriSamples + 3], sRy[kOriSamples + 3], sPhi[kOriSamples + 3];
    __shared__ Best sBest[kDescWaves];
    __shared__ float sSq[kDescWaves];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int i = blockIdx.x;
    if (i >= min(*count, capacity)) return;  // whole block
    const RefinedKeypoint k = kps[i];
    const bool ok = k.level >= 0 && k.level < N && isfinite(k.x) && isfinite(k.y);
    const float s = ok ? dl.sigma[k.level] : 0.f;
    const size_t plane = (size_t)W * H;
    const float* gx = lx + plane * (ok ? k.level : 0);
    const float* gy = ly + plane * (ok ? k.level : 0);

    if (tid < kOriSamples) {
        float rx = 0.f, ry = 0.f;
        if (ok) {
            const float u = kOri.u[tid], v = kOri.v[tid];
            const float w = expf(-(u * u + v * v) * (1.f / 12.5f));
            float vx, vy;
            bilinear2(gx, gy, W, H, k.x + s * u, k.y + s * v, vx, vy);
            rx = w * vx;
            ry = w * vy;
        }
        sRx[tid] = rx;
        sRy[tid] = ry;
        sPhi[tid] = atan2f(ry, rx);
    }
    __syncthreads();
    Best best{-1.f, 1 << 30, 0.f, 0.f};
    if (tid < 2 * kOriSamples) {
        const float pk = sPhi[tid >> 1];
        const bool after = (tid & 1) == 0;
        float ax = 0.f, ay = 0.f;
#pragma unroll 8
        for (int j = 0; j < kOriSamples; ++j) {
            const float pj = sPhi[j];
            float d = after ? pj - pk : pk - pj;
            if (d < 0.f) d += kTwoPi;
            const bool in = after ? (d > 0.f && d <= kSector) : d < kSector;
            ax += in ? sRx[j] : 0.f;
            ay += in ? sRy[j] : 0.f;
        }
        best = Best{ax * ax + ay * ay, tid, ax, ay};
    }
    for (int m = kWave / 2; m >= 1; m >>= 1) best = better(best, shfl_best(best, m));
    if (lane == 0) sBest[wave] = best;
    __syncthreads();
    best = sBest[0];
    for (int w = 1; w < kDescWaves; ++w) best = better(best, sBest[w]);
    const float theta = atan2f(best.sy, best.sx);
    // cos and sin of theta = atan2(sy, sx) are the unit sum itself
    const float slen = sqrtf(best.sx * best.sx + best.sy * best.sy);
    const float c = slen > 0.f ? best.sx / slen : 1.f, sn = slen > 0.f ? best.sy / slen : 0.f;

    const int sr = tid >> 4, part = tid & 15;
    const int a = sr & 3, b = sr >> 2;
    const float cu = -7.5f + 5.f * a, cv = -7.5f + 5.f * b;
    float su = 0.f, sv = 0.f, mu = 0.f, mv = 0.f;
    if (ok) {
        float vx[6], vy[6], w[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {  // gather all samples first
            const int q = part + 16 * m;
            const int tv = q / 9, tu = q - 9 * (q / 9);
            const float u = cu - 4.f + tu, v = cv - 4.f + tv;
            w[m] = q < 81 ? expf(-(float)((tu - 4) * (tu - 4) + (tv - 4) * (tv - 4)) * (1.f / 12.5f))
                          : 0.f;
            vx[m] = vy[m] = 0.f;
            if (q < 81)
                bilinear2(gx, gy, W, H, k.x + s * (u * c - v * sn), k.y + s * (u * sn + v * c),
                          vx[m], vy[m]);
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const float du = vx[m] * c + vy[m] * sn, dv = -vx[m] * sn + vy[m] * c;
            su += w[m] * du;
            sv += w[m] * dv;
            mu += w[m] * fabsf(du);
            mv += w[m] * fabsf(dv);
        }
    }
    for (int m = 1; m <= 8; m <<= 1) {
        su += __shfl_xor(su, m);
        sv += __shfl_xor(sv, m);
        mu += __shfl_xor(mu, m);
        mv += __shfl_xor(mv, m);
    }
    const float w2 = expf(-((a - 1.5f) * (a - 1.5f) + (b - 1.5f) * (b - 1.5f)) * (1.f / 4.5f));
    su *= w2;
    sv *= w2;
    mu *= w2;
    mv *= w2;
    float sq = part == 0 ? su * su + sv * sv + mu * mu + mv * mv : 0.f;
    for (int m = kWave / 2; m >= 1; m >>= 1) sq += __shfl_xor(sq, m);
    if (lane == 0) sSq[wave] = sq;
    __syncthreads();
    float tot = 0.f;
    for (int w = 0; w < kDescWaves; ++w) tot += sSq[w];
    const float len = sqrtf(tot);
    const float inv = len > 0.f ? 1.f / len : 0.f;
    if (part == 0) {
        float* o = desc + (size_t)i * 64 + sr * 4;
        o[0] = su * inv;
        o[1] = sv * inv;
        o[2] = mu * inv;
        o[3] = mv * inv;
    }
    if (tid == 0) angles[i] = ok ? theta : __builtin_nanf("");
}

}  // namespace

hipError_t launch_deriv(const float* levels, int W, int H, int N, const DescLevels& dl, float* lx,
                        float* ly, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const dim3 grid((W + kDerivTX - 1) / kDerivTX, (H + kDerivTY - 1) / kDerivTY, N);
    hipLaunchKernelGGL(deriv_kernel, grid, dim3(kDerivTX * kDerivTY), 0, s, levels, W, H, dl, lx,
                       ly);
    return hipGetLastError();
}

hipError_t launch_describe(const float* lx, const float* ly, int W, int H, int N,
                           const DescLevels& dl, const void* kps, const int* count, int capacity,
                           float* angles, float* desc, hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    hipLaunchKernelGGL(describe_kernel, dim3(capacity), dim3(kDescThreads), 0, s, lx, ly, W, H,
                       N, dl, static_cast<const RefinedKeypoint*>(kps), count, capacity, angles,
                       desc);
    return hipGetLastError();
}

}  // namespace kaze
