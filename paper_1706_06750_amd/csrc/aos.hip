// Semi-implicit step of Eq. 4 by additive operator splitting (AOS):
//   L_i = L_{i-1} + (delta_x + delta_y) / 2,
//   (I - 2 tau A_l(g)) delta_l = 2 tau A_l(g) L_{i-1},   l in {x, y},
// where A_l is the 1-D nonlinear diffusion matrix along rows (l = x) or
// columns (l = y) with couplings (g_j + g_k)/2 between neighbours and no flux
// across the image border.  Solving for the increment delta = u - L instead
// of u keeps the FP32 error relative to the (small) change of a step rather
// than to the image itself.
//
// Every line system is solved with a partitioned tridiagonal method: the
// line is cut into chunks; each chunk eliminates its interior unknowns with
// one top-down and one bottom-up sweep, leaving two equations that couple
// its first and last unknowns to the neighbouring chunks; that interface
// system (2 unknowns per chunk) is solved by parallel cyclic reduction on
// one wavefront; each chunk then recovers its interior by a Thomas sweep
// with both ends known.  (Partitioned and hybrid tridiagonal solvers:
// Zhang, Cohen & Owens, PPoPP 2010; Laszlo, Giles & Appleyard, ACM TOMS
// 2016.)
//
// Rows (contiguous in memory): one wavefront per row.  The row is loaded
// coalesced into LDS, lane l owns the contiguous chunk [l*m, (l+1)*m), the
// interface system is reduced with cross-lane permutes, and the increment
// is written back coalesced.
// Columns (stride W): one thread per column segment of MC rows, adjacent
// lanes on adjacent columns so every load and store is coalesced; three
// kernels (chunk reduction, interface solve, interior recovery + average).
#include "kaze_internal.h"

namespace kaze {

int col_chunk_rows(int H) {
    if (H <= 16 * kWave) return 16;
    if (H <= 32 * kWave) return 32;
    return 64;
}

void row_partition(int W, int* lanes, int* per_lane) {
    int m = (W + kWave - 1) / kWave;
    if (m < 2) m = 2;
    *per_lane = m;
    *lanes = (W + m - 1) / m;
}

namespace {

// --------------------------------------------------------------------------
// Rows
// --------------------------------------------------------------------------
// Row j of the system along a row held in LDS (identity beyond the row end).
__device__ __forceinline__ Eq row_eq_lds(const float* sL, const float* sg, int X, int W,
                                         float tau) {
    if (X >= W) return eq_identity();
    const float g0 = sg[X], L0 = sL[X];
    float wl = 0.f, wr = 0.f, dl = 0.f, dr = 0.f;
    if (X > 0) {
        wl = tau * (sg[X - 1] + g0);
        dl = sL[X - 1] - L0;
    }
    if (X < W - 1) {
        wr = tau * (g0 + sg[X + 1]);
        dr = sL[X + 1] - L0;
    }
    return aos_row(wl, wr, dl, dr);
}

template <int RPB>
__global__ __launch_bounds__(kWave* RPB) void aos_rows_kernel(const float* __restrict__ L,
                                                                const float* __restrict__ g,
                                                                float* __restrict__ dx, int W,
                                                                int H, int m, float tau) {
    extern __shared__ float smem[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int y = blockIdx.x * RPB + wave;
    const int Wp = kWave * m;
    float* sL = smem + (size_t)wave * 2 * Wp;
    float* sg = sL + Wp;
    const bool row_ok = y < H;

    if (row_ok) {
        const float* Lr = L + (size_t)y * W;
        const float* gr = g + (size_t)y * W;
        for (int x = lane; x < Wp; x += kWave) {
            const bool in = x < W;
            sL[x] = in ? Lr[x] : 0.f;
            sg[x] = in ? gr[x] : 0.f;
        }
    }
    __syncthreads();

    const int x0 = lane * m;
    const bool mine = row_ok && x0 < W;
    Eq e0 = eq_identity(), e1 = eq_identity();
    if (mine) {
        // top-down over the interior: x_k + cp x_{k+1} = dp + ep x_0
        float cp = 0.f, dp = 0.f, ep = 1.f;
        for (int k = 1; k <= m - 2; ++k) {
            const Eq e = row_eq_lds(sL, sg, x0 + k, W, tau);
            const float r = 1.f / (e.b - e.a * cp);
            dp = (e.d - e.a * dp) * r;
            ep = -e.a * ep * r;
            cp = e.c * r;
        }
        {
            const Eq e = row_eq_lds(sL, sg, x0 + m - 1, W, tau);
            e1 = Eq{e.a * ep, e.b - e.a * cp, e.c, e.d - e.a * dp};
        }
        // bottom-up over the interior: x_k + ap x_{k-1} = dq + eq x_{m-1}
        float ap = 0.f, dq = 0.f, eq = 1.f;
        for (int k = m - 2; k >= 1; --k) {
            const Eq e = row_eq_lds(sL, sg, x0 + k, W, tau);
            const float r = 1.f / (e.b - e.c * ap);
            dq = (e.d - e.c * dq) * r;
            eq = -e.c * eq * r;
            ap = e.a * r;
        }
        {
            const Eq e = row_eq_lds(sL, sg, x0, W, tau);
            e0 = Eq{e.a, e.b - e.c * ap, e.c * eq, e.d - e.c * dq};
        }
    }
    float z0, z1;
    wave_pcr_pairs(e0, e1, lane, z0, z1);
    __syncthreads();  // every lane is done reading its neighbours' data

    if (mine) {
        // interior Thomas with x_0 = z0 and x_{m-1} = z1; (cp, dp) overwrite
        // the (g, L) slots already consumed, so neighbours roll in registers
        float gm = sg[x0], Lm = sL[x0];
        float g0 = sg[x0 + 1], L0 = sL[x0 + 1];
        float cp = 0.f, dp = 0.f;
        for (int k = 1; k <= m - 2; ++k) {
            const int X = x0 + k;
            const float gp = sg[X + 1], Lp = sL[X + 1];
            Eq e = eq_identity();
            if (X < W) {
                const bool has_r = X < W - 1;
                e = aos_row(tau * (gm + g0), has_r ? tau * (g0 + gp) : 0.f, Lm - L0,
                            has_r ? Lp - L0 : 0.f);
            }
            if (k == 1) {
                e.d -= e.a * z0;
                e.a = 0.f;
            }
            if (k == m - 2) {
                e.d -= e.c * z1;
                e.c = 0.f;
            }
            const float r = 1.f / (e.b - e.a * cp);
            cp = e.c * r;
            dp = (e.d - e.a * dp) * r;
            sg[X] = cp;
            sL[X] = dp;
            gm = g0;
            Lm = L0;
            g0 = gp;
            L0 = Lp;
        }
        float xn = z1;
        for (int k = m - 2; k >= 1; --k) {
            const int X = x0 + k;
            const float xk = sL[X] - sg[X] * xn;
            sL[X] = xk;
            xn = xk;
        }
        sL[x0] = z0;
        sL[x0 + m - 1] = z1;
    }
    __syncthreads();
    if (row_ok) {
        float* out = dx + (size_t)y * W;
        for (int x = lane; x < W; x += kWave) out[x] = sL[x];
    }
}

// --------------------------------------------------------------------------
// Columns
// --------------------------------------------------------------------------
constexpr int CB_X = 64;  // columns per block (one wavefront)
constexpr int CB_Y = 4;   // column segments per block

// Load rows y0-1 .. y0+MC of column x (zero outside the image) and form the
// coupling weights w[j] between rows y0-1+j and y0+j (zero across the
// image border and into the padding below row H-1).
template <int MC>
__device__ __forceinline__ void load_col_segment(const float* __restrict__ L,
                                                 const float* __restrict__ g, int x, int y0,
                                                 int W, int H, float tau, float (&Lr)[MC + 2],
                                                 float (&w)[MC + 1]) {
    float gr[MC + 2];
#pragma unroll
    for (int j = 0; j < MC + 2; ++j) {
        const int yy = y0 - 1 + j;
        const bool ok = yy >= 0 && yy < H;
        Lr[j] = ok ? L[(size_t)yy * W + x] : 0.f;
        gr[j] = ok ? g[(size_t)yy * W + x] : 0.f;
    }
#pragma unroll
    for (int j = 0; j <= MC; ++j) {
        const int ya = y0 - 1 + j;
        w[j] = (ya >= 0 && ya + 1 < H) ? tau * (gr[j] + gr[j + 1]) : 0.f;
    }
}

template <int MC>
__device__ __forceinline__ Eq col_eq(const float (&Lr)[MC + 2], const float (&w)[MC + 1], int k) {
    return aos_row(w[k], w[k + 1], Lr[k] - Lr[k + 1], Lr[k + 2] - Lr[k + 1]);
}

template <int MC>
__global__ __launch_bounds__(CB_X* CB_Y) void aos_col_reduce_kernel(
    const float* __restrict__ L, const float* __restrict__ g, float* __restrict__ red, int W,
    int H, int Pc, float tau) {
    const int x = blockIdx.x * CB_X + threadIdx.x;
    const int p = blockIdx.y * CB_Y + threadIdx.y;
    if (x >= W || p >= Pc) return;
    float Lr[MC + 2], w[MC + 1];
    load_col_segment<MC>(L, g, x, p * MC, W, H, tau, Lr, w);

    float cp = 0.f, dp = 0.f, ep = 1.f;
#pragma unroll
    for (int k = 1; k <= MC - 2; ++k) {
        const Eq e = col_eq<MC>(Lr, w, k);
        const float r = 1.f / (e.b - e.a * cp);
        dp = (e.d - e.a * dp) * r;
        ep = -e.a * ep * r;
        cp = e.c * r;
    }
    const Eq el = col_eq<MC>(Lr, w, MC - 1);
    const Eq e1{el.a * ep, el.b - el.a * cp, el.c, el.d - el.a * dp};

    float ap = 0.f, dq = 0.f, eq = 1.f;
#pragma unroll
    for (int k = MC - 2; k >= 1; --k) {
        const Eq e = col_eq<MC>(Lr, w, k);
        const float r = 1.f / (e.b - e.c * ap);
        dq = (e.d - e.c * dq) * r;
        eq = -e.c * eq * r;
        ap = e.a * r;
    }
    const Eq ef = col_eq<MC>(Lr, w, 0);
    const Eq e0{ef.a, ef.b - ef.c * ap, ef.c * eq, ef.d - ef.c * dq};

    float4* o = reinterpret_cast<float4*>(red + ((size_t)x * Pc + p) * 8);
    o[0] = make_float4(e0.a, e0.b, e0.c, e0.d);
    o[1] = make_float4(e1.a, e1.b, e1.c, e1.d);
}

// One wavefront per column: lane p holds segment p's two interface rows.
__global__ __launch_bounds__(256) void aos_col_iface_kernel(const float* __restrict__ red,
                                                              float* __restrict__ z, int W,
                                                              int Pc) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int x = blockIdx.x * (256 / kWave) + wave;
    Eq e0 = eq_identity(), e1 = eq_identity();
    const bool mine = x < W && lane < Pc;
    if (mine) {
        const float4* r = reinterpret_cast<const float4*>(red + ((size_t)x * Pc + lane) * 8);
        const float4 a = r[0], b = r[1];
        e0 = Eq{a.x, a.y, a.z, a.w};
        e1 = Eq{b.x, b.y, b.z, b.w};
    }
    float z0, z1;
    wave_pcr_pairs(e0, e1, lane, z0, z1);
    if (mine) reinterpret_cast<float2*>(z + ((size_t)x * Pc + lane) * 2)[0] = make_float2(z0, z1);
}

template <int MC>
__global__ __launch_bounds__(CB_X* CB_Y) void aos_col_final_kernel(
    const float* __restrict__ L, const float* __restrict__ g, const float* __restrict__ z,
    const float* __restrict__ dx, float* __restrict__ Lnext, int W, int H, int Pc, float tau) {
    const int x = blockIdx.x * CB_X + threadIdx.x;
    const int p = blockIdx.y * CB_Y + threadIdx.y;
    if (x >= W || p >= Pc) return;
    const int y0 = p * MC;
    float Lr[MC + 2], w[MC + 1];
    load_col_segment<MC>(L, g, x, y0, W, H, tau, Lr, w);
    const float2 zz = reinterpret_cast<const float2*>(z + ((size_t)x * Pc + p) * 2)[0];

    float cp[MC], dp[MC];
    float cprev = 0.f, dprev = 0.f;
#pragma unroll
    for (int k = 1; k <= MC - 2; ++k) {
        Eq e = col_eq<MC>(Lr, w, k);
        if (k == 1) {
            e.d -= e.a * zz.x;
            e.a = 0.f;
        }
        if (k == MC - 2) {
            e.d -= e.c * zz.y;
            e.c = 0.f;
        }
        const float r = 1.f / (e.b - e.a * cprev);
        cprev = e.c * r;
        dprev = (e.d - e.a * dprev) * r;
        cp[k] = cprev;
        dp[k] = dprev;
    }
    float xs[MC];
    xs[0] = zz.x;
    xs[MC - 1] = zz.y;
#pragma unroll
    for (int k = MC - 2; k >= 1; --k) xs[k] = dp[k] - cp[k] * xs[k + 1];

#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const int y = y0 + k;
        if (y < H) {
            const size_t i = (size_t)y * W + x;
            Lnext[i] = Lr[k + 1] + 0.5f * (dx[i] + xs[k]);
        }
    }
}

}  // namespace

hipError_t launch_aos_rows(const float* L, const float* g, float* dx, int W, int H, float tau,
                           hipStream_t s) {
    int lanes, m;
    row_partition(W, &lanes, &m);
    const size_t row_bytes = (size_t)2 * kWave * m * sizeof(float);
    int rpb = (int)(65536 / row_bytes);
    if (rpb >= 4) {
        hipLaunchKernelGGL(aos_rows_kernel<4>, dim3((H + 3) / 4), dim3(4 * kWave), 4 * row_bytes,
                           s, L, g, dx, W, H, m, tau);
    } else if (rpb >= 2) {
        hipLaunchKernelGGL(aos_rows_kernel<2>, dim3((H + 1) / 2), dim3(2 * kWave), 2 * row_bytes,
                           s, L, g, dx, W, H, m, tau);
    } else {
        hipLaunchKernelGGL(aos_rows_kernel<1>, dim3(H), dim3(kWave), row_bytes, s, L, g, dx, W,
                           H, m, tau);
    }
    return hipGetLastError();
}

hipError_t launch_aos_col_reduce(const float* L, const float* g, float* red, int W, int H,
                                 float tau, hipStream_t s) {
    const int MC = col_chunk_rows(H);
    const int Pc = (H + MC - 1) / MC;
    dim3 grid((W + CB_X - 1) / CB_X, (Pc + CB_Y - 1) / CB_Y), block(CB_X, CB_Y);
    if (MC == 16)
        hipLaunchKernelGGL(aos_col_reduce_kernel<16>, grid, block, 0, s, L, g, red, W, H, Pc, tau);
    else if (MC == 32)
        hipLaunchKernelGGL(aos_col_reduce_kernel<32>, grid, block, 0, s, L, g, red, W, H, Pc, tau);
    else
        hipLaunchKernelGGL(aos_col_reduce_kernel<64>, grid, block, 0, s, L, g, red, W, H, Pc, tau);
    return hipGetLastError();
}

hipError_t launch_aos_col_iface(const float* red, float* z, int W, int H, hipStream_t s) {
    const int MC = col_chunk_rows(H);
    const int Pc = (H + MC - 1) / MC;
    const int cols_per_block = 256 / kWave;
    hipLaunchKernelGGL(aos_col_iface_kernel, dim3((W + cols_per_block - 1) / cols_per_block),
                       dim3(256), 0, s, red, z, W, Pc);
    return hipGetLastError();
}

hipError_t launch_aos_col_final(const float* L, const float* g, const float* z, const float* dx,
                                float* Lnext, int W, int H, float tau, hipStream_t s) {
    const int MC = col_chunk_rows(H);
    const int Pc = (H + MC - 1) / MC;
    dim3 grid((W + CB_X - 1) / CB_X, (Pc + CB_Y - 1) / CB_Y), block(CB_X, CB_Y);
    if (MC == 16)
        hipLaunchKernelGGL(aos_col_final_kernel<16>, grid, block, 0, s, L, g, z, dx, Lnext, W, H,
                           Pc, tau);
    else if (MC == 32)
        hipLaunchKernelGGL(aos_col_final_kernel<32>, grid, block, 0, s, L, g, z, dx, Lnext, W, H,
                           Pc, tau);
    else
        hipLaunchKernelGGL(aos_col_final_kernel<64>, grid, block, 0, s, L, g, z, dx, Lnext, W, H,
                           Pc, tau);
    return hipGetLastError();
}

}  // namespace kaze
