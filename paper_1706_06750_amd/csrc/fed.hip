// Fast explicit diffusion (Eq. 5): one cycle of n explicit steps
//   L <- L + tau_j sum_q (g_p + g_q)/2 (L_q - L_p)
// over the 4-neighbours q of every pixel, with the conductivity g of the
// level before held fixed and the step sizes tau_j of the cycle applied in
// an order that keeps the intermediate growth of rounding errors small.
//
// GPU form: kFedS steps per launch, temporally blocked in LDS.  A block
// holds a 64 x 64 region (the output tile plus a ring of kFedS pixels,
// half-sample reflected at the image border, which makes the flux across
// the border vanish and stays mirrored under every step).  Each lane owns
// one column of the region and each wavefront a band of 16 rows: the lane
// keeps its 16 values and their four flux weights in registers; the values
// go through one of two LDS planes per step so that the neighbouring
// columns and bands can read them.  Every step recomputes the whole region;
// values within kFedS - s pixels of the region edge are wrong after step s
// (their outer neighbours are missing), which never reaches the tile.
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>

#include "fed_internal.h"

namespace kaze {

// ------------------------------------------------------------------ host
namespace {

// max over mu of |prod (1 + tau mu)| for the prefix / suffix products of an
// order, on the grid mu = -8 + 8 i / 2000 (the spectrum of the explicit
// operator with g <= 1 lies in [-8, 0]).
double order_bound(const std::vector<double>& tau, const std::vector<int>& order) {
#pragma clang fp contract(off)
    constexpr int M = 2001;
    const int n = (int)tau.size();
    std::vector<double> mu(M);
    const double step = 8.0 / (M - 1);
    for (int i = 0; i < M; ++i) mu[i] = i * step + -8.0;
    mu[M - 1] = 0.0;
    std::vector<double> prefix(n + 1), suffix(n + 1);
    std::vector<double> pr(M, 1.0);
    prefix[0] = 1.0;
    for (int k = 0; k < n; ++k) {
        double m = 0.0;
        for (int i = 0; i < M; ++i) {
            pr[i] = pr[i] * (1.0 + tau[order[k]] * mu[i]);
            m = std::max(m, std::fabs(pr[i]));
        }
        prefix[k + 1] = m;
    }
    std::fill(pr.begin(), pr.end(), 1.0);
    suffix[n] = 1.0;
    for (int k = n - 1; k >= 0; --k) {
        double m = 0.0;
        for (int i = 0; i < M; ++i) {
            pr[i] = pr[i] * (1.0 + tau[order[k]] * mu[i]);
            m = std::max(m, std::fabs(pr[i]));
        }
        suffix[k] = m;
    }
    double b = 0.0;
    for (int k = 0; k <= n; ++k) b = std::max(b, prefix[k] * suffix[k]);
    return b;
}

std::vector<double> compute_schedule(double T) {
#pragma clang fp contract(off)
    int n = 1;
    while (kFedTauMax * (n * n + n) / 3.0 < T) ++n;
    std::vector<double> tau(n);
    double sum = 0.0;
    for (int j = 0; j < n; ++j) {
        const double c = std::cos(M_PI * (2.0 * j + 1.0) / (4.0 * n + 2.0));
        tau[j] = kFedTauMax / (2.0 * c * c);
        sum += tau[j];
    }
    for (double& t : tau) t *= T / sum;
    // order j = kappa * i mod n with the kappa (coprime to n, smallest on
    // ties) of least bound
    double best = -1.0;
    int best_k = 1;
    for (int kappa = 1; kappa < std::max(n, 2); ++kappa) {
        if (std::gcd(kappa, n) != 1) continue;
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = (int)(((long long)kappa * i) % n);
        const double b = order_bound(tau, order);
        if (best < 0.0 || b < best * (1.0 - 1e-12)) {
            best = b;
            best_k = kappa;
        }
    }
    std::vector<double> out(n);
    for (int i = 0; i < n; ++i) out[i] = tau[(int)(((long long)best_k * i) % n)];
    return out;
}

}  // namespace

std::vector<double> fed_schedule(double T) {
    if (!(T > 0.0) || !std::isfinite(T)) return {};
    static std::mutex mu;
    static std::map<double, std::vector<double>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(T);
    if (it != cache.end()) return it->second;
    std::vector<double> s = compute_schedule(T);
    cache.emplace(T, s);
    return s;
}

// ---------------------------------------------------------------- device
namespace {

__device__ __forceinline__ int reflect_clamp(int i, int n) {
    i = i < 0 ? -1 - i : i;
    i = i >= n ? 2 * n - 1 - i : i;
    return i < 0 ? 0 : i;
}

constexpr int kFedThreads = 256;
constexpr int kFedRows = kFedRegion / (kFedThreads / kWave);  // rows per lane
constexpr int kFedPitch = kFedRegion + 1;

// The step's multiply-adds are spelled out (contraction off), so that a
// cycle gives the same bits whatever the number of steps per launch.
__global__ __launch_bounds__(kFedThreads) void fed_kernel(const float* src, const float* g,
                                                          float* dst, int W, int H,
                                                          FedSteps st) {
#pragma clang fp contract(off)
    __shared__ float sA[kFedRegion * kFedPitch];
    __shared__ float sB[kFedRegion * kFedPitch];
    const int wave = uniform(threadIdx.x >> 6), c = threadIdx.x & (kWave - 1);
    const int ntx = (W + kFedTile - 1) / kFedTile;
    const int t = blockIdx.x;
    const int tx0 = (t % ntx) * kFedTile, ty0 = (t / ntx) * kFedTile;
    const int r0 = wave * kFedRows;  // first region row of this lane
    const int gx = reflect_clamp(tx0 - kFedS + c, W);

    // conductivity of the region into plane A, values into registers
    float v[kFedRows];
    {
        float gv[kFedRows];
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) {
            const ptrdiff_t row = (ptrdiff_t)uniform(reflect_clamp(ty0 - kFedS + r0 + k, H)) * W;
            gv[k] = ((const gfloat*)g)[row + gx];
            v[k] = ((const gfloat*)src)[row + gx];
        }
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) sA[(r0 + k) * kFedPitch + c] = gv[k];
    }
    __syncthreads();
    // flux weights g_p + g_q towards the four neighbours (a missing
    // neighbour at the region edge takes g_p, its flux is zero anyway)
    float wl[kFedRows], wr[kFedRows], wu[kFedRows], wd[kFedRows];
    {
        const float* a = sA + r0 * kFedPitch + c;
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) {
            const float gp = a[k * kFedPitch];
            const float gl = c > 0 ? a[k * kFedPitch - 1] : gp;
            const float gr = c < kFedRegion - 1 ? a[k * kFedPitch + 1] : gp;
            const float gu = (r0 + k > 0) ? a[(k - 1) * kFedPitch] : gp;
            const float gd = (r0 + k < kFedRegion - 1) ? a[(k + 1) * kFedPitch] : gp;
            wl[k] = gp + gl;
            wr[k] = gp + gr;
            wu[k] = gp + gu;
            wd[k] = gp + gd;
        }
    }
    __syncthreads();  // plane A is free for values from here on

#pragma unroll
    for (int j = 0; j < kFedS; ++j) {
        if (j >= st.n) break;  // uniform
        float* P = (j & 1) ? sB : sA;
        float* p = P + r0 * kFedPitch + c;
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) p[k * kFedPitch] = v[k];
        __syncthreads();
        const float h = st.half_tau[j];
        float up = r0 > 0 ? p[-kFedPitch] : v[0];
        const float below = r0 + kFedRows < kFedRegion ? p[kFedRows * kFedPitch] : v[kFedRows - 1];
        float nv[kFedRows];
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) {
            const float x = v[k];
            const float l = c > 0 ? p[k * kFedPitch - 1] : x;
            const float r = c < kFedRegion - 1 ? p[k * kFedPitch + 1] : x;
            const float d = k + 1 < kFedRows ? v[k + 1] : below;
            float f = wl[k] * (l - x);
            f = __builtin_fmaf(wr[k], r - x, f);
            f = __builtin_fmaf(wu[k], up - x, f);
            f = __builtin_fmaf(wd[k], d - x, f);
            nv[k] = __builtin_fmaf(h, f, x);
            up = x;
        }
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) v[k] = nv[k];
    }

    // the tile: region rows / columns [kFedS, kFedRegion - kFedS)
    const int x = tx0 - kFedS + c;
    if (c >= kFedS && c < kFedRegion - kFedS && x < W) {
#pragma unroll
        for (int k = 0; k < kFedRows; ++k) {
            const int r = r0 + k, y = ty0 - kFedS + r;
            if (r >= kFedS && r < kFedRegion - kFedS && y < H)
                ((gfloat*)dst)[(ptrdiff_t)y * W + x] = v[k];
        }
    }
}

}  // namespace

hipError_t launch_fed(const float* src, const float* g, float* dst, int W, int H,
                      const FedSteps& st, hipStream_t s) {
    if (st.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fed_kernel, dim3(fed_tiles_of(W, H)), dim3(kFedThreads), 0, s, src, g, dst,
                       W, H, st);
    return hipGetLastError();
}

}  // namespace kaze
