// Semi-implicit step of Eq. 4 by additive operator splitting (AOS):
//   L_i = L_{i-1} + (delta_x + delta_y) / 2,
//   (I - 2 tau A_l(g)) delta_l = 2 tau A_l(g) L_{i-1},   l in {rows, columns},
// where A_l is the 1-D nonlinear diffusion matrix along rows or columns with
// couplings (g_j + g_k)/2 between neighbours and no flux across the image
// border.  Solving for the increment delta = u - L rather than u keeps the
// FP32 error relative to the change of one step, not to the image.
//
// Every row and column system is solved by a partitioned tridiagonal
// method on TX x TY tiles (64 or 32 each, chosen per batch by the autotuner;
// partitioned / hybrid tridiagonal solvers: Zhang, Cohen & Owens, PPoPP 2010;
// Laszlo, Giles & Appleyard, ACM TOMS 2016):
//
//  1. aos_reduce (one block per tile): the tile of L_{i-1} plus a ring is
//     staged in LDS, the conductivity g is computed there (and written
//     once for step 3), and each tile row and tile column -- a TX- or
//     TY-element chunk of its line -- is reduced by one forward sweep to two equations
//     that couple its first and last unknowns to the neighbouring chunks.
//     The sweep also accumulates the back-substitution weights of the
//     chunk's second unknown, so the first unknown's equation needs no
//     backward sweep.
//  2. aos_iface (one wavefront per line): the 2 equations per chunk form a
//     tridiagonal system of 2 x (chunks per line) unknowns, solved by
//     parallel cyclic reduction across the lanes (lane = chunk).
//  3. aos_recover (one block per tile): with both ends of every chunk
//     known, each tile row and column recovers its interior by a Thomas
//     sweep in registers, and L_i = L + (delta_x + delta_y)/2 is stored.
//
// HBM traffic per pixel and step: L read twice, g written once and read
// once, L_i written once, plus 24 bytes of interface equations per chunk
// (two equations scaled to a unit diagonal) and 8 bytes of solved ends.  Tile rows are staged through LDS (the transpose that lets
// one thread walk a row); tile columns are walked by adjacent threads on
// adjacent columns, so every global access is coalesced.
#include "kaze_internal.h"

namespace kaze {
namespace {

constexpr int kBlock = 256;

// v_rcp_f32: <= 1 ulp; the pivots are >= 1 (diagonally dominant rows).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Coupling weight tau*(g_a + g_b) between neighbours a, b of a line, zero
// across the line end when `inside` is false.  PRE: the accessor returns g
// already multiplied by tau.  CHECK = false: the caller guarantees the whole
// chunk and its right neighbour lie inside the line, so no test is made.
template <bool CHECK, bool PRE>
__device__ __forceinline__ float coupling(bool inside, float tau, float ga, float gb) {
    const float w = PRE ? ga + gb : tau * (ga + gb);
    return CHECK ? (inside ? w : 0.f) : w;
}

// Chunk of M unknowns at line positions pos0 .. pos0+M-1 of a line of n
// pixels.  Acc::g(k), Acc::L(k) give conductivity and level at chunk index
// k in [-1, M] (the ring supplies -1 and M).  Positions past the line end
// are identity rows (decoupled, solution 0).  The right-hand side of row k
// is the flux difference f_k - f_{k-1}, f_k = w_{k,k+1} (L_{k+1} - L_k):
// each flux is formed once and used by both rows it joins.
template <int M, bool CHECK = true, bool PRE = false, class Acc>
__device__ __forceinline__ void chunk_reduce(const Acc& A, int pos0, int n, float tau, Eq& E0,
                                             Eq& E1) {
#pragma clang fp contract(off)
    const float gm = A.g(-1), Lm = A.L(-1);
    float g0 = A.g(0), L0 = A.L(0);
    float gp = A.g(1), Lp = A.L(1);
    float wl = coupling<true, PRE>(pos0 > 0 && pos0 < n, tau, gm, g0);
    float fl = wl * (L0 - Lm);  // flux into the chunk across its left end
    float wr = coupling<CHECK, PRE>(pos0 < n - 1, tau, g0, gp);
    float fr = wr * (Lp - L0);
    const Eq first{-wl, (1.f + wl) + wr, -wr, fr - fl};
    wl = wr;
    fl = fr;
    g0 = gp;
    L0 = Lp;
    // x_k + cp x_{k+1} = dp + ep x_0 over the interior, and
    // x_1 = al + be x_0 + P x_{M-1} accumulated along the way.
    float cp = 0.f, dp = 0.f, ep = 1.f, P = 1.f, al = 0.f, be = 0.f;
#pragma unroll
    for (int k = 1; k <= M - 2; ++k) {
        gp = A.g(k + 1);
        Lp = A.L(k + 1);
        wr = coupling<CHECK, PRE>(pos0 + k < n - 1, tau, g0, gp);
        fr = wr * (Lp - L0);
        const float d = fr - fl;
        const float r = rcp(__builtin_fmaf(wl, cp, (1.f + wl) + wr));
        dp = __builtin_fmaf(wl, dp, d) * r;
        ep = (wl * ep) * r;
        cp = -wr * r;
        al = __builtin_fmaf(P, dp, al);
        be = __builtin_fmaf(P, ep, be);
        P = -P * cp;
        wl = wr;
        fl = fr;
        g0 = gp;
        L0 = Lp;
    }
    gp = A.g(M);
    Lp = A.L(M);
    wr = coupling<CHECK, PRE>(pos0 + M - 1 < n - 1, tau, g0, gp);
    fr = wr * (Lp - L0);
    const Eq last{-wl, (1.f + wl) + wr, -wr, fr - fl};
    E1 = Eq{last.a * ep, last.b - last.a * cp, last.c, last.d - last.a * dp};
    E0 = Eq{first.a, first.b + first.c * be, first.c * P, first.d - first.c * al};
}

// Interior of a chunk by a Thomas sweep with both ends known (z0 at k = 0,
// z1 at k = M-1).  On return x[k] holds the increment of every element.
template <int M, bool CHECK = true, bool PRE = false, class Acc>
__device__ __forceinline__ void chunk_recover(const Acc& A, int pos0, int n, float tau, float z0,
                                              float z1, float (&x)[M]) {
#pragma clang fp contract(off)
    float cpa[M];
    const float gm = A.g(0), Lm = A.L(0);
    float g0 = A.g(1), L0 = A.L(1);
    float wl = coupling<CHECK, PRE>(pos0 + 1 < n, tau, gm, g0);
    float fl = wl * (L0 - Lm);
    float cp = 0.f, dp = 0.f;
#pragma unroll
    for (int k = 1; k <= M - 2; ++k) {
        const float gp = A.g(k + 1), Lp = A.L(k + 1);
        const float wr = coupling<CHECK, PRE>(pos0 + k < n - 1, tau, g0, gp);
        const float fr = wr * (Lp - L0);
        float d = fr - fl;
        const float b = (1.f + wl) + wr;
        float a = -wl, c = -wr;
        if (k == 1) {
            d = __builtin_fmaf(-a, z0, d);
            a = 0.f;
        }
        if (k == M - 2) {
            d = __builtin_fmaf(-c, z1, d);
            c = 0.f;
        }
        const float r = rcp(__builtin_fmaf(-a, cp, b));
        cp = c * r;
        dp = __builtin_fmaf(-a, dp, d) * r;
        cpa[k] = cp;
        x[k] = dp;
        wl = wr;
        fl = fr;
        g0 = gp;
        L0 = Lp;
    }
    x[0] = z0;
    x[M - 1] = z1;
#pragma unroll
    for (int k = M - 2; k >= 1; --k) x[k] = __builtin_fmaf(-cpa[k], x[k + 1], x[k]);
}

// The interior of a chunk (both ends known, as in chunk_recover) in two
// halves on two lanes: the lower lane eliminates rows 1 .. MH forward from
// x_0, the upper lane rows M-2 .. MH+1 backward from x_{M-1}; then
//   x_MH = dp - cp x_{MH+1},  x_{MH+1} = dq - aq x_MH
// gives the two middle values (split_middle), and each lane substitutes
// back through its own half.  Every coefficient of the lower half is formed
// as in chunk_recover, and the upper half mirrors it.
template <int M>
struct SplitChunk {
    static constexpr int MH = (M - 2) / 2;  // last interior row of the lower half
    static constexpr int NU = M - 1 - MH;   // elements MH+1 .. M-1 of the upper half
    static_assert(MH >= 1 && NU >= 2, "both halves hold interior rows");
};

// Lower lane: x[k] for k = 0 .. MH holds dp_k (x_0 = z0), cpa[k] cp_k.
template <int M, bool CHECK, class Acc>
__device__ __forceinline__ void split_lower(const Acc& A, int pos0, int n, float z0,
                                            float (&x)[SplitChunk<M>::MH + 1],
                                            float (&cpa)[SplitChunk<M>::MH + 1]) {
#pragma clang fp contract(off)
    constexpr int MH = SplitChunk<M>::MH;
    const float gm = A.g(0), Lm = A.L(0);
    float g0 = A.g(1), L0 = A.L(1);
    float wl = coupling<CHECK, true>(pos0 + 1 < n, 1.f, gm, g0);
    float fl = wl * (L0 - Lm);
    float cp = 0.f, dp = 0.f;
#pragma unroll
    for (int k = 1; k <= MH; ++k) {
        const float gp = A.g(k + 1), Lp = A.L(k + 1);
        const float wr = coupling<CHECK, true>(pos0 + k < n - 1, 1.f, g0, gp);
        const float fr = wr * (Lp - L0);
        float d = fr - fl;
        const float b = (1.f + wl) + wr;
        float a = -wl;
        const float c = -wr;
        if (k == 1) {
            d = __builtin_fmaf(-a, z0, d);
            a = 0.f;
        }
        const float r = rcp(__builtin_fmaf(-a, cp, b));
        cp = c * r;
        dp = __builtin_fmaf(-a, dp, d) * r;
        cpa[k] = cp;
        x[k] = dp;
        wl = wr;
        fl = fr;
        g0 = gp;
        L0 = Lp;
    }
    x[0] = z0;
}

// Upper lane: x[i] for element MH+1+i (i = 0 .. NU-1) holds dq (the last,
// element M-1, holds z1), aqa[i] aq.
template <int M, bool CHECK, class Acc>
__device__ __forceinline__ void split_upper(const Acc& A, int pos0, int n, float z1,
                                            float (&x)[SplitChunk<M>::NU],
                                            float (&aqa)[SplitChunk<M>::NU]) {
#pragma clang fp contract(off)
    constexpr int MH = SplitChunk<M>::MH;
    const float gq = A.g(M - 1), Lq = A.L(M - 1);
    float g0 = A.g(M - 2), L0 = A.L(M - 2);
    float wr = coupling<CHECK, true>(pos0 + M - 2 < n - 1, 1.f, g0, gq);
    float fr = wr * (Lq - L0);
    float aq = 0.f, dq = 0.f;
#pragma unroll
    for (int k = M - 2; k >= MH + 1; --k) {
        const float gm = A.g(k - 1), Lm = A.L(k - 1);
        const float wl = coupling<CHECK, true>(pos0 + k - 1 < n - 1, 1.f, gm, g0);
        const float fl = wl * (L0 - Lm);
        float d = fr - fl;
        const float b = (1.f + wl) + wr;
        const float a = -wl;
        float c = -wr;
        if (k == M - 2) {
            d = __builtin_fmaf(-c, z1, d);
            c = 0.f;
        }
        const float r = rcp(__builtin_fmaf(-c, aq, b));
        aq = a * r;
        dq = __builtin_fmaf(-c, dq, d) * r;
        aqa[k - MH - 1] = aq;
        x[k - MH - 1] = dq;
        wr = wl;
        fr = fl;
        g0 = gm;
        L0 = Lm;
    }
    x[SplitChunk<M>::NU - 1] = z1;
}

// The two middle values from the lower lane's (cp, dp) at MH and the upper
// lane's (aq, dq) at MH+1; both lanes evaluate it alike.
__device__ __forceinline__ void split_middle(float cp, float dp, float aq, float dq, float& xm,
                                             float& xm1) {
#pragma clang fp contract(off)
    xm = __builtin_fmaf(-cp, dq, dp) * rcp(__builtin_fmaf(-cp, aq, 1.f));
    xm1 = __builtin_fmaf(-aq, xm, dq);
}

// Value of the neighbouring lane of the pair (lanes 2i, 2i+1).
__device__ __forceinline__ float pair_swap(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}

// A chunk reduced in two halves on a lane pair (even lane: lower half, odd:
// upper half, each by chunk_reduce): the lower half's last row and the upper
// half's first row couple the two middle unknowns x_h, x_{h+1}; solving that
// 2x2 in terms of x_0 and x_{M-1} and substituting into the lower half's
// first row and the upper half's last row gives the chunk's own two
// equations, which the even lane returns in (e0, e1).
__device__ __forceinline__ void merge_halves(Eq& e0, Eq& e1) {
#pragma clang fp contract(off)
    const Eq u0{pair_swap(e0.a), pair_swap(e0.b), pair_swap(e0.c), pair_swap(e0.d)};
    const Eq u1{pair_swap(e1.a), pair_swap(e1.b), pair_swap(e1.c), pair_swap(e1.d)};
    // e1: e1.a x_0 + e1.b x_h + e1.c x_{h+1} = e1.d
    // u0: u0.a x_h + u0.b x_{h+1} + u0.c x_{M-1} = u0.d
    const float inv = rcp(e1.b * u0.b - e1.c * u0.a);
    const float a0 = (e1.d * u0.b - e1.c * u0.d) * inv;  // x_h = a0 + a1 x_0 + a2 x_{M-1}
    const float a1 = -(e1.a * u0.b) * inv;
    const float a2 = (e1.c * u0.c) * inv;
    const float b0 = (e1.b * u0.d - u0.a * e1.d) * inv;  // x_{h+1} = b0 + b1 x_0 + b2 x_{M-1}
    const float b1 = (e1.a * u0.a) * inv;
    const float b2 = -(e1.b * u0.c) * inv;
    const Eq m0{e0.a, e0.b + e0.c * a1, e0.c * a2, e0.d - e0.c * a0};
    const Eq m1{u1.a * b1, u1.b + u1.a * b2, u1.c, u1.d - u1.a * b0};
    e0 = m0;
    e1 = m1;
}

// LDS accessor of one chunk with compile-time strides: element k (which may
// be -1) at gp[k * GS] and Lp[k * LS], so every access is an immediate
// offset from the thread's base address.
template <int GS, int LS>
struct LdsLine {
    const float* gp;  // element 0
    const float* Lp;
    __device__ __forceinline__ float g(int k) const { return gp[k * GS]; }
    __device__ __forceinline__ float L(int k) const { return Lp[k * LS]; }
};

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) vf4 gvf4;
typedef __attribute__((address_space(1))) vf2 gvf2;

// The chunk's two equations scaled to a unit diagonal (the pivots are >= 1:
// diagonally dominant rows), as (a0, c0, d0, a1, c1, d1) in three 8-byte
// stores.
__device__ __forceinline__ void store_eqs(float* dst, const Eq& e0, const Eq& e1) {
    const float r0 = rcp(e0.b), r1 = rcp(e1.b);
    gvf2* o = (gvf2*)dst;
    o[0] = vf2{e0.a * r0, e0.c * r0};
    o[1] = vf2{e0.d * r0, e1.a * r1};
    o[2] = vf2{e1.c * r1, e1.d * r1};
}

// Index i of a line of n pixels reflected half-sample symmetrically into
// [0, n) (one reflection covers every ring used here, n >= 8), clamped for
// positions of partial tiles far past the image, which feed no output.
__device__ __forceinline__ int reflect_clamp(int i, int n) {
    i = i < 0 ? -1 - i : i;
    i = i >= n ? 2 * n - 1 - i : i;
    return i < 0 ? 0 : i;
}

// Image planes are read and written through gfloat with wave-uniform row
// offsets: a row access is one load or store with a scalar base and the
// lane's byte offset.

// LDS geometry of the reduction tile: kAosTX x TY pixels.  With the
// conductivity computed here (CG) the tile holds L on a ring of RG + 2 (the
// Gaussian of radius RG plus Scharr plus the chunk ends), the smoothed image
// S on the tile + 2 ring (exactly one wavefront wide: kAosTX + 4 = 64) and g
// on the tile + 1 ring; otherwise L and g on the tile + 1 ring.  The S area
// has rows beyond the tile + 2 ring so that every wavefront's band of g rows
// reads whole rows; they are never written and feed no stored value.  S is
// dead once g is formed, so g takes S's place (a barrier between the last
// read of S and the first write of g): less LDS per tile, more tiles per CU.
template <int RG, int TY, bool CG>
struct RedGeom {
    static constexpr int WAVES = 4;
    static constexpr int R = CG ? RG + 2 : 1;
    static constexpr int NLY = TY + 2 * R, NLX = kAosTX + 2 * R, PL = NLX | 1;
    static constexpr int NSY = TY + 4, PS = kWave + 1;
    static constexpr int NGY = TY + 2, NGX = kAosTX + 2, PG = NGX | 1;
    static constexpr int SPW = (NSY + WAVES - 1) / WAVES;  // S rows per wavefront
    static constexpr int QPW = (NGY + WAVES - 1) / WAVES;  // g rows per wavefront
    static constexpr int NSA = WAVES * QPW + 2;             // S rows allocated
    static constexpr int offS = NLY * PL;
    static constexpr int offG = offS;  // g over S (CG) or right after L
    static constexpr int floats = offS + (CG && NSA * PS > NGY * PG ? NSA * PS : NGY * PG);
    static constexpr int floatsLS = offS + NSA * PS;  // L and S (the conductivity kernel)
    static_assert(kAosTX + 4 == kWave, "the smoothed band is one wavefront wide");
    static_assert(NLX <= 2 * kWave, "two loads per L row");
    static_assert(SPW * WAVES == NSY, "S bands tile the region");
    static_assert(NSA >= NSY, "S area holds the region");
};

constexpr int kRedThreads = 256;

// Rows [0, NY) x columns [0, NX) of src, with image origin (gy0, gx0),
// half-sample reflected at the image border, into LDS at pitch P, each value
// times `scale`; wavefront w loads rows w, w+4, ...; lane l loads columns l
// and 64 + l (those below NX).  All loads of a lane are issued before its
// first LDS store.
template <int NY, int NX, int P, int NT = kRedThreads>
__device__ __forceinline__ void load_region(const float* src, int W, int H, int gy0, int gx0,
                                            float scale, float* dst, int wave, int lane) {
    constexpr int WAVES = NT / kWave;
    constexpr int PER = (NY + WAVES - 1) / WAVES;
    const gfloat* gs = (const gfloat*)src;
    const bool has_a = lane < NX;
    const bool has_b = lane < NX - kWave;
    const int xa = reflect_clamp(gx0 + lane, W);
    const int xb = reflect_clamp(gx0 + kWave + lane, W);
    float va[PER], vb[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int r = wave + WAVES * i;
        if (r < NY) {
            const gfloat* row = gs + (ptrdiff_t)uniform(reflect_clamp(gy0 + r, H)) * W;
            va[i] = has_a ? row[xa] : 0.f;
            vb[i] = has_b ? row[xb] : 0.f;
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int r = wave + WAVES * i;
        if (r < NY) {
            if (has_a) dst[r * P + lane] = scale * va[i];
            if (has_b) dst[r * P + kWave + lane] = scale * vb[i];
        }
    }
}

// Perona-Malik conductivity (Eq. 3) as a compile-time choice: GM 0 g2,
// GM 1 g1; m2 is the squared gradient magnitude times 1/k^2.  GM 2 passes
// it through (with k = 1: the squared gradient itself).
template <int GM>
__device__ __forceinline__ float diffusivity_of(float m2k) {
    if constexpr (GM == 2) return m2k;
    return GM == 0 ? __builtin_amdgcn_rcpf(1.f + m2k) : expf(-m2k);
}

// The Gaussian-smoothed image S on rows [s0, s0 + SPW) of a grid of 64
// columns (one lane per column) whose element (s, j) is the Gaussian of the
// L region around (s + r, j + r): the horizontal pass is recomputed along
// the band in registers, the vertical pass rolls over it.
template <int r, int SPW, int PL, int PS>
__device__ __forceinline__ void smooth_band(const float* sL, float* sS, int s0, int lane,
                                            const float (&w)[2 * r + 1]) {
#pragma clang fp contract(off)
    float h[SPW + 2 * r];
    const float* lp = sL + s0 * PL + lane;
#pragma unroll
    for (int k = 0; k < SPW + 2 * r; ++k) {
        const float* q = lp + k * PL;
        float acc = w[r] * q[r];
#pragma unroll
        for (int t = 0; t < r; ++t) acc = __builtin_fmaf(w[t], q[t] + q[2 * r - t], acc);
        h[k] = acc;
    }
    float* sp = sS + s0 * PS + lane;
#pragma unroll
    for (int k = 0; k < SPW; ++k) {
        float acc = w[r] * h[k + r];
#pragma unroll
        for (int t = 0; t < r; ++t) acc = __builtin_fmaf(w[t], h[k + t] + h[k + 2 * r - t], acc);
        sp[k * PS] = acc;
    }
}

// Conductivity on rows [q0, q0 + QPW) of a grid whose element (q, i) is
// centred on S(q + 1, i + 1): the 3x3 Scharr gradient of S with weights
// (1, 10/3, 1) instead of (3, 10, 3) and unscaled (Lx' = 32 Lx / 3,
// Ly' = 32 Ly / 3, so |grad|^2 = 9 m2' / 1024, folded into c2 =
// 9/(1024 k^2)) and g of Eq. 3 for column ic, into gv.
constexpr float kTenThirds = 10.f / 3.f;

template <int QPW, int PS, int GM>
__device__ __forceinline__ void conductivity_band(const float* sS, int q0, int ic, float c2,
                                                  float (&gv)[QPW]) {
#pragma clang fp contract(off)
    const float* sp = sS + q0 * PS + ic;
    float D[QPW + 2], Tt[QPW + 2];
#pragma unroll
    for (int k = 0; k < QPW + 2; ++k) {
        const float a = sp[k * PS], b = sp[k * PS + 1], c = sp[k * PS + 2];
        D[k] = c - a;
        Tt[k] = __builtin_fmaf(kTenThirds, b, a + c);
    }
#pragma unroll
    for (int k = 0; k < QPW; ++k) {
        const float lx = __builtin_fmaf(kTenThirds, D[k + 1], D[k] + D[k + 2]);
        const float ly = Tt[k + 2] - Tt[k];
        gv[k] = diffusivity_of<GM>(__builtin_fmaf(lx, lx, ly * ly) * c2);
    }
}

// Phases 2-3 of the reduction with the conductivity: S on the tile + 2 ring
// (each wavefront a band of rows), then g on the tile + 1 ring: tau * g into
// LDS for the sweeps and g of the tile to gout for the recovery.
template <int RG, int TY, int GM>
__device__ __forceinline__ void tile_conductivity(const float* sL, float* sS, float* sG,
                                                  const Taps& tc, float inv_k2, float tau,
                                                  float* gout, int W, int H, int tx0, int ty0,
                                                  int wave, int lane) {
    using G = RedGeom<RG, TY, true>;
    constexpr int T = 2 * RG + 1;
    float w[T];
#pragma unroll
    for (int t = 0; t < T; ++t) w[t] = tc.w[t];
    smooth_band<RG, G::SPW, G::PL, G::PS>(sL, sS, wave * G::SPW, lane, w);
    __syncthreads();
    const int q0 = wave * G::QPW;
    float gv[G::QPW];
    conductivity_band<G::QPW, G::PS, GM>(sS, q0, lane < G::NGX ? lane : G::NGX - 1,
                                         inv_k2 * (9.f / 1024.f), gv);
    __syncthreads();  // every wavefront has read S: g overwrites it
    const bool lane_g = lane < G::NGX;
    const bool col_in = lane >= 1 && lane <= kAosTX && tx0 - 1 + lane < W;
    float* gl = sG + q0 * G::PG + lane;
    gfloat* grow = (gfloat*)gout + (ptrdiff_t)uniform(ty0 - 1 + q0) * W + (tx0 - 1);
#pragma unroll
    for (int k = 0; k < G::QPW; ++k) {
        const int q = q0 + k;
        if (q < G::NGY) {
            if (lane_g) gl[k * G::PG] = tau * gv[k];
            if (q >= 1 && q <= TY && ty0 - 1 + q < H && col_in)
                grow[(ptrdiff_t)k * W + lane] = gv[k];
        }
    }
}

// Chunks of one tile: kAosTX / RC row chunks per tile row, walked by the
// lanes of TY / RPW wavefronts (lane = RPW * chunk + row), and TY / CC
// column chunks per tile column, one wavefront each (lane = column), so
// every sweep runs on full wavefronts.
template <int TY, int RC, int CC>
struct TileChunks {
    static constexpr int HALVES = kAosTX / RC;  // row chunks per tile row
    static constexpr int RPW = kWave / HALVES;  // tile rows per row wavefront
    static constexpr int SWR = TY / RPW;        // row wavefronts
    static constexpr int SWC = TY / CC;         // column wavefronts
    static_assert(HALVES * RC == kAosTX && SWR * RPW == TY && SWC * CC == TY, "tiles hold whole chunks");
    static_assert(SWR + SWC <= 4 && RC <= CC && CC <= kMaxColChunk, "four wavefronts per tile");
};

// Reduction: one block of 256 threads per tile of kAosTX x TY pixels; each
// tile row and tile column chunk (TileChunks) is reduced by one forward
// sweep to two equations.  The LDS copy of g is pre-multiplied by tau.
template <int RG, int TY, int RC, int CC, bool CG, int GM>
__global__ __launch_bounds__(kRedThreads) void aos_reduce_kernel(ImageDesc d0, AosWork w, Taps tc,
                                                                 float tau, float k_host) {
    using G = RedGeom<RG, TY, CG>;
    using T = TileChunks<TY, RC, CC>;
    extern __shared__ float smem[];
    float* sL = smem;
    float* sS = smem + G::offS;
    float* sG = smem + G::offG;
    const int tid = threadIdx.x, wave = uniform(tid >> 6), lane = tid & (kWave - 1);
    ImageDesc d;
    int lt;
    resolve(d0, w, xcd_contiguous((int)blockIdx.x, (int)gridDim.x), d, lt);
    if (d.gate && *d.gate <= d.bound) return;  // whole block
    const int W = d.W, H = d.H;
    const int ntx = (W + kAosTX - 1) / kAosTX;
    const int cx = lt % ntx, cy = lt / ntx;
    const int tx0 = cx * kAosTX, ty0 = cy * TY;

    const float k = CG && d.k ? d.k[0] : k_host;  // issued with the staging loads
    load_region<G::NLY, G::NLX, G::PL>(d.L, W, H, ty0 - G::R, tx0 - G::R, 1.f, sL, wave, lane);
    if constexpr (!CG)
        load_region<G::NGY, G::NGX, G::PG>(d.g, W, H, ty0 - 1, tx0 - 1, tau, sG, wave, lane);
    __syncthreads();
    if constexpr (CG) {
        tile_conductivity<RG, TY, GM>(sL, sS, sG, tc, 1.f / (k * k), tau, d.g, W, H, tx0, ty0,
                                      wave, lane);
        __syncthreads();
    }

    Eq e0, e1;
    if constexpr (chunk_lanes(TY, RC, CC) == 2) {
        // one wavefront of row chunks and one column chunk per tile column:
        // two lanes per chunk, rows in wavefronts 0-1, columns in 2-3
        // (merge_halves)
        constexpr int MR = RC / 2, MC = CC / 2;
        static_assert(2 * MR == RC && 2 * MC == CC, "chunks of even length");
        const int half = lane & 1, line = 32 * (wave & 1) + (lane >> 1);
        if (wave < 2) {
            const int r = line % TY, h = line / TY;  // row chunk h of tile row r
            const int y = ty0 + r, pos0 = tx0 + h * RC;
            if (y < H && pos0 < W) {
                const LdsLine<1, 1> A{sG + (r + 1) * G::PG + 1 + h * RC + half * MR,
                                      sL + (r + G::R) * G::PL + G::R + h * RC + half * MR};
                if (tx0 + kAosTX < W)
                    chunk_reduce<MR, false, true>(A, pos0 + half * MR, W, 1.f, e0, e1);
                else
                    chunk_reduce<MR, true, true>(A, pos0 + half * MR, W, 1.f, e0, e1);
                merge_halves(e0, e1);
                if (!half)
                    store_eqs(d.rrow + ((size_t)(T::HALVES * cx + h) * H + y) * kEqFloats, e0, e1);
            }
        } else {
            const int x = tx0 + line;
            if (line < kAosTX && x < W) {
                const LdsLine<G::PG, G::PL> A{sG + (half * MC + 1) * G::PG + 1 + line,
                                              sL + (half * MC + G::R) * G::PL + G::R + line};
                if (ty0 + CC < H)
                    chunk_reduce<MC, false, true>(A, ty0 + half * MC, H, 1.f, e0, e1);
                else
                    chunk_reduce<MC, true, true>(A, ty0 + half * MC, H, 1.f, e0, e1);
                merge_halves(e0, e1);
                if (!half) store_eqs(d.rcol + ((size_t)(ty0 / CC) * W + x) * kEqFloats, e0, e1);
            }
        }
    } else if (wave < T::SWR) {
        const int r = wave * T::RPW + (lane % T::RPW), h = lane / T::RPW;
        const int y = ty0 + r, pos0 = tx0 + h * RC;
        if (y < H && pos0 < W) {
            const LdsLine<1, 1> A{sG + (r + 1) * G::PG + 1 + h * RC,
                                  sL + (r + G::R) * G::PL + G::R + h * RC};
            if (tx0 + kAosTX < W)  // the tile row's chunks and their right neighbours inside
                chunk_reduce<RC, false, true>(A, pos0, W, 1.f, e0, e1);
            else
                chunk_reduce<RC, true, true>(A, pos0, W, 1.f, e0, e1);
            store_eqs(d.rrow + ((size_t)(T::HALVES * cx + h) * H + y) * kEqFloats, e0, e1);
        }
    } else if (wave < T::SWR + T::SWC) {
        const int v = wave - T::SWR, c = lane;
        const int x = tx0 + c, pos0 = ty0 + v * CC;
        if (c < kAosTX && x < W && pos0 < H) {
            const LdsLine<G::PG, G::PL> A{sG + (v * CC + 1) * G::PG + 1 + c,
                                          sL + (v * CC + G::R) * G::PL + G::R + c};
            if (pos0 + CC < H)
                chunk_reduce<CC, false, true>(A, pos0, H, 1.f, e0, e1);
            else
                chunk_reduce<CC, true, true>(A, pos0, H, 1.f, e0, e1);
            store_eqs(d.rcol + ((size_t)(pos0 / CC) * W + x) * kEqFloats, e0, e1);
        }
    }
}

// Conductivity on kAosTX x TY tiles with the reduction's own band code: L
// on the tile + (RG + 2) ring, the smoothed band, the Scharr gradient, and
// per position of the tile (GM 0) g2 or (GM 1) g1 -- the g the fused
// reduction computes, bit for bit -- or (GM 2) the squared gradient
// magnitude |grad L_s|^2, with the tile's maximum of |grad| stored in the
// tile's word of the image's maxima (no atomics: the histogram and the
// quantile kernels reduce the words).  Items: (image, tile)
// as the reduction's, or tiles of d0 without a work list.
template <int RG, int GM, int TY>
__global__ __launch_bounds__(kRedThreads) void cond_band_kernel(BatchImage d0, ImgWork w, Taps tc,
                                                                float k_host) {
    using G = RedGeom<RG, TY, true>;
    extern __shared__ float smem[];
    __shared__ float s_max[kRedThreads / kWave];
    float* sL = smem;
    float* sS = smem + G::offS;
    const int tid = threadIdx.x, wave = uniform(tid >> 6), lane = tid & (kWave - 1);
    BatchImage d;
    int lt;
    resolve(d0, w, xcd_contiguous((int)blockIdx.x, (int)gridDim.x), d, lt);
    const int W = d.W, H = d.H;
    const int ntx = (W + kAosTX - 1) / kAosTX;
    const int tx0 = (lt % ntx) * kAosTX, ty0 = (lt / ntx) * TY;
    load_region<G::NLY, G::NLX, G::PL>(d.levels, W, H, ty0 - G::R, tx0 - G::R, 1.f, sL, wave,
                                       lane);
    __syncthreads();
    constexpr int T = 2 * RG + 1;
    float wt[T];
#pragma unroll
    for (int t = 0; t < T; ++t) wt[t] = tc.w[t];
    smooth_band<RG, G::SPW, G::PL, G::PS>(sL, sS, wave * G::SPW, lane, wt);
    __syncthreads();
    const float k = GM == 2 ? 1.f : (d.k ? *(const gfloat*)d.k : k_host);
    const float inv_k2 = 1.f / (k * k);  // as the reduction forms it
    const int q0 = wave * G::QPW;
    float gv[G::QPW];
    conductivity_band<G::QPW, G::PS, GM>(sS, q0, lane < G::NGX ? lane : G::NGX - 1,
                                         inv_k2 * (9.f / 1024.f), gv);
    const bool col_in = lane >= 1 && lane <= kAosTX && tx0 - 1 + lane < W;
    gfloat* grow = (gfloat*)d.g + (ptrdiff_t)uniform(ty0 - 1 + q0) * W + (tx0 - 1);
    float m2max = 0.f;
#pragma unroll
    for (int j = 0; j < G::QPW; ++j) {
        const int q = q0 + j;
        if (q >= 1 && q <= TY && ty0 - 1 + q < H && col_in) {
            grow[(ptrdiff_t)j * W + lane] = gv[j];
            if constexpr (GM == 2) m2max = fmaxf(m2max, gv[j]);
        }
    }
    if constexpr (GM == 2) {
        // the square root is monotone, so the maximum is taken on |grad|^2
        for (int off = kWave / 2; off > 0; off >>= 1)
            m2max = fmaxf(m2max, __shfl_xor(m2max, off, kWave));
        if (lane == 0) s_max[wave] = m2max;
        __syncthreads();
        if (tid == 0) {
            float m = s_max[0];
            for (int i = 1; i < kRedThreads / kWave; ++i) m = fmaxf(m, s_max[i]);
            ((guint*)d.hmax)[lt] = __float_as_uint(sqrtf(m));
        }
    }
}

template <int RG, int TY>
hipError_t launch_cond_band_t(const BatchImage& d0, const ImgWork& w, const Taps& tc,
                              float k_host, int gmode, hipStream_t s) {
    const int count = w.items ? w.count : aos_tiles_of(d0.W, d0.H, TY);
    if (count <= 0) return hipSuccess;
    const size_t lds = (size_t)RedGeom<RG, TY, true>::floatsLS * sizeof(float);
#define KZ_CB(GM)                                                                            \
    hipLaunchKernelGGL((cond_band_kernel<RG, GM, TY>), dim3(count), dim3(kRedThreads), lds, s, \
                       d0, w, tc, k_host)
    if (gmode == 0) KZ_CB(0);
    else if (gmode == 1) KZ_CB(1);
    else KZ_CB(2);
#undef KZ_CB
    return hipGetLastError();
}

template <int RG>
hipError_t launch_cond_band_r(const BatchImage& d0, const ImgWork& w, const Taps& tc,
                              float k_host, int gmode, int ty, hipStream_t s) {
    if (ty == 32) return launch_cond_band_t<RG, 32>(d0, w, tc, k_host, gmode, s);
    if (ty == 64) return launch_cond_band_t<RG, 64>(d0, w, tc, k_host, gmode, s);
    return hipErrorInvalidValue;
}

// PCR step with reciprocal pivots (the pivots of these diagonally
// dominant systems are >= their off-diagonal sums).
__device__ __forceinline__ Eq pcr_reduce_rcp(const Eq& e, const Eq& lo, const Eq& up) {
    const float k1 = e.a * rcp(lo.b);
    const float k2 = e.c * rcp(up.b);
    return Eq{-k1 * lo.a, e.b - k1 * lo.c - k2 * up.a, -k2 * up.c, e.d - k1 * lo.d - k2 * up.d};
}

// Equations of lane l - S (below) and l + S (above) within the lane's row of
// 16 (DPP row shifts, S < 16); a source outside the row reads zeros, which
// the callers replace by identity rows (segments of at most 16 lanes never
// reach across a row).
template <int S>
__device__ __forceinline__ float dpp_below(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x110 + S, 0xF, 0xF, true));
}
template <int S>
__device__ __forceinline__ float dpp_above(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x100 + S, 0xF, 0xF, true));
}
template <int S>
__device__ __forceinline__ Eq eq_below(const Eq& e) {
    return Eq{dpp_below<S>(e.a), dpp_below<S>(e.b), dpp_below<S>(e.c), dpp_below<S>(e.d)};
}
template <int S>
__device__ __forceinline__ Eq eq_above(const Eq& e) {
    return Eq{dpp_above<S>(e.a), dpp_above<S>(e.b), dpp_above<S>(e.c), dpp_above<S>(e.d)};
}

// One PCR round at stride S with DPP exchanges (segments of P <= 16 lanes).
template <int S>
__device__ __forceinline__ void pcr_round_dpp(Eq& e0, Eq& e1, int pos, int P) {
    const bool has_lo = pos >= S, has_up = pos + S < P;
    Eq lo0 = eq_below<S>(e0), up0 = eq_above<S>(e0);
    Eq lo1 = eq_below<S>(e1), up1 = eq_above<S>(e1);
    if (!has_lo) { lo0 = eq_identity(); lo1 = eq_identity(); }
    if (!has_up) { up0 = eq_identity(); up1 = eq_identity(); }
    const Eq n0 = pcr_reduce_rcp(e0, lo0, up0);
    const Eq n1 = pcr_reduce_rcp(e1, lo1, up1);
    e0 = n0;
    e1 = n1;
}

// PCR over segments of P lanes (P a power of two, segments aligned): lane
// `pos` of a segment holds the two reduced equations of its part of the
// line (e0 for its first unknown, e1 for its last); neighbours outside the
// segment are identity rows.  Every lane of the wavefront must take part.
__device__ __forceinline__ void seg_pcr_pairs(Eq e0, Eq e1, int lane, int pos, int P, float& z0,
                                              float& z1) {
    if (P <= 16) {  // wave-uniform: every exchange inside a DPP row, same values
        {
            Eq prev1 = eq_below<1>(e1);
            Eq next0 = eq_above<1>(e0);
            if (pos == 0) prev1 = eq_identity();
            if (pos == P - 1) next0 = eq_identity();
            const Eq n0 = pcr_reduce_rcp(e0, prev1, e1);
            const Eq n1 = pcr_reduce_rcp(e1, e0, next0);
            e0 = n0;
            e1 = n1;
        }
        if (P > 1) pcr_round_dpp<1>(e0, e1, pos, P);
        if (P > 2) pcr_round_dpp<2>(e0, e1, pos, P);
        if (P > 4) pcr_round_dpp<4>(e0, e1, pos, P);
        if (P > 8) pcr_round_dpp<8>(e0, e1, pos, P);
        z0 = e0.d * rcp(e0.b);
        z1 = e1.d * rcp(e1.b);
        return;
    }
    {
        Eq prev1 = lane_read(e1, lane > 0 ? lane - 1 : 0);
        Eq next0 = lane_read(e0, lane < kWave - 1 ? lane + 1 : kWave - 1);
        if (pos == 0) prev1 = eq_identity();
        if (pos == P - 1) next0 = eq_identity();
        const Eq n0 = pcr_reduce_rcp(e0, prev1, e1);
        const Eq n1 = pcr_reduce_rcp(e1, e0, next0);
        e0 = n0;
        e1 = n1;
    }
    for (int st = 1; st < P; st <<= 1) {
        const bool has_lo = pos >= st, has_up = pos + st < P;
        Eq lo0 = lane_read(e0, has_lo ? lane - st : lane);
        Eq up0 = lane_read(e0, has_up ? lane + st : lane);
        Eq lo1 = lane_read(e1, has_lo ? lane - st : lane);
        Eq up1 = lane_read(e1, has_up ? lane + st : lane);
        if (!has_lo) { lo0 = eq_identity(); lo1 = eq_identity(); }
        if (!has_up) { up0 = eq_identity(); up1 = eq_identity(); }
        const Eq n0 = pcr_reduce_rcp(e0, lo0, up0);
        const Eq n1 = pcr_reduce_rcp(e1, lo1, up1);
        e0 = n0;
        e1 = n1;
    }
    z0 = e0.d * rcp(e0.b);
    z1 = e1.d * rcp(e1.b);
}

// Interface systems.  A line of nch chunks has 2 nch unknowns (first and
// last of every chunk) coupled by the chunks' reduced equations into one
// tridiagonal system.  Lane `pos` of the line's P = iface_lanes(nch) lanes
// holds chunks pos*kIfaceM .. pos*kIfaceM + kIfaceM - 1 (identity rows past
// the line end): it reduces its 2 kIfaceM rows to two equations in its first
// and last unknown (the same elimination as the chunk reduction), the lanes
// of the line solve those by PCR, and each lane substitutes back through its
// own rows, kept in registers.  All loads of a lane are issued at once.
constexpr int kIfaceThreads = 256;

template <int kIfaceM>
__global__ __launch_bounds__(kIfaceThreads) void aos_iface_kernel(ImageDesc d0, AosWork w,
                                                                   int count) {
    constexpr int NR = 2 * kIfaceM;  // rows per lane
    const int t = uniform(blockIdx.x * (kIfaceThreads / kWave) + (int)(threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    if (t >= count) return;  // whole wavefront
    ImageDesc d;
    int grp;
    resolve(d0, w, t, d, grp);
    if (d.gate && *d.gate <= d.bound) return;  // whole wavefront
    const int rgroups = iface_groups(d.H, d.nchr, kIfaceM);
    const bool row = grp < rgroups;
    const int nch = row ? d.nchr : d.nchc;
    const int nl = row ? d.H : d.W;
    const int P = iface_lanes(nch, kIfaceM);
    const int pos = lane & (P - 1);
    const int line = (row ? grp : grp - rgroups) * (kWave / P) + lane / P;
    const bool live = line < nl;
    const int lc = live ? line : nl - 1;  // clamped: every lane loads in bounds
    gfloat* R = (gfloat*)(row ? d.rrow : d.rcol) + (size_t)lc * kEqFloats;
    gfloat* Z = (gfloat*)(row ? d.zrow : d.zcol) + (size_t)lc * 2;
    const size_t rs = (size_t)nl * kEqFloats, zs = (size_t)nl * 2;  // chunk strides
    const int c0 = pos * kIfaceM;

    Eq e[NR];
    {
        vf2 va[kIfaceM], vb[kIfaceM], vc[kIfaceM];
#pragma unroll
        for (int j = 0; j < kIfaceM; ++j) {
            const int c = c0 + j < nch ? c0 + j : nch - 1;
            const gvf2* q = (const gvf2*)(R + c * rs);
            va[j] = q[0];
            vb[j] = q[1];
            vc[j] = q[2];
        }
#pragma unroll
        for (int j = 0; j < kIfaceM; ++j) {
            const bool ok = c0 + j < nch;
            e[2 * j] = ok ? Eq{va[j].x, 1.f, va[j].y, vb[j].x} : eq_identity();
            e[2 * j + 1] = ok ? Eq{vb[j].y, 1.f, vc[j].x, vc[j].y} : eq_identity();
        }
    }
    // x_k = dp_k + ep_k x_0 - cp_k x_{k+1} for the interior rows k, and
    // x_1 = al + be x_0 + pp x_{NR-1}
    float CP[NR], DP[NR], EP[NR];
    float cp = 0.f, dp = 0.f, ep = 1.f, pp = 1.f, al = 0.f, be = 0.f;
#pragma unroll
    for (int k = 1; k <= NR - 2; ++k) {
        const Eq& q = e[k];
        const float r = rcp(q.b - q.a * cp);
        dp = (q.d - q.a * dp) * r;
        ep = -q.a * ep * r;
        cp = q.c * r;
        al += pp * dp;
        be += pp * ep;
        pp = -pp * cp;
        CP[k] = cp;
        DP[k] = dp;
        EP[k] = ep;
    }
    const Eq& f = e[0];
    const Eq& l = e[NR - 1];
    const Eq E0{f.a, f.b + f.c * be, f.c * pp, f.d - f.c * al};
    const Eq E1{l.a * ep, l.b - l.a * cp, l.c, l.d - l.a * dp};
    float x[NR];
    seg_pcr_pairs(E0, E1, lane, pos, P, x[0], x[NR - 1]);
#pragma unroll
    for (int k = NR - 2; k >= 1; --k) x[k] = DP[k] + EP[k] * x[0] - CP[k] * x[k + 1];
#pragma unroll
    for (int j = 0; j < kIfaceM; ++j)
        if (live && c0 + j < nch) *(gvf2*)(Z + (c0 + j) * zs) = vf2{x[2 * j], x[2 * j + 1]};
}

// Recovery: the row and column wavefronts of TileChunks; L and tau * g of
// the tile staged in LDS.  Both sweeps keep their increments in registers;
// after a barrier the row lanes fold theirs into the LDS copy of L
// (L + delta_x / 2), and after a second one the column lanes store
// L_i = L + (delta_x + delta_y)/2 one row at a time (coalesced).
template <int TY, int RC, int CC>
__global__ __launch_bounds__(TY * 4) void aos_recover_kernel(ImageDesc d0, AosWork w, float tau) {
    constexpr int NT = TY * 4, WAVES = NT / kWave;
    using T = TileChunks<TY, RC, CC>;
    // LDS layout: (row, column) of the tile at sL[row * PL + column], tau * g
    // at sG[row * PG + column]
    constexpr int PL = kAosTX + 1, PG = kAosTX + 1;
    extern __shared__ float smem[];
    float* sL = smem;
    float* sG = smem + TY * PL;
    const int tid = threadIdx.x, wave = uniform(tid >> 6), lane = tid & (kWave - 1);
    ImageDesc d;
    int lt;
    resolve(d0, w, xcd_contiguous((int)blockIdx.x, (int)gridDim.x), d, lt);
    if (d.gate && *d.gate <= d.bound) return;  // whole block
    const int W = d.W, H = d.H;
    const int ntx = (W + kAosTX - 1) / kAosTX;
    const int cx = lt % ntx, cy = lt / ntx;
    const int tx0 = cx * kAosTX, ty0 = cy * TY;
    {
        constexpr int PER = TY / WAVES;
        const bool in_x = lane < kAosTX && tx0 + lane < W;
        const gfloat* Lb = (const gfloat*)d.L + (ptrdiff_t)uniform(ty0 + wave) * W + tx0;
        const gfloat* gb = (const gfloat*)d.g + (ptrdiff_t)uniform(ty0 + wave) * W + tx0;
        float vl[PER], vg[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const bool in = in_x && ty0 + wave + WAVES * i < H;
            vl[i] = in ? Lb[(ptrdiff_t)(WAVES * i) * W + lane] : 0.f;
            vg[i] = in ? gb[(ptrdiff_t)(WAVES * i) * W + lane] : 0.f;
        }
        if (lane < kAosTX) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int r = wave + WAVES * i;
                sL[r * PL + lane] = vl[i];
                sG[r * PG + lane] = tau * vg[i];
            }
        }
    }
    __syncthreads();
    float xs[CC];  // row lanes: delta_x of the chunk; column lanes: delta_y
    const int v = wave - T::SWR, c = lane;
    const int xcol = tx0 + c, pos0c = ty0 + v * CC;
    const bool col_lane =
        wave >= T::SWR && wave < T::SWR + T::SWC && c < kAosTX && xcol < W && pos0c < H;
    const int r = wave * T::RPW + (lane % T::RPW), h = lane / T::RPW;
    const bool row_lane = wave < T::SWR && ty0 + r < H && tx0 + h * RC < W;
    if (row_lane) {
        const int y = ty0 + r, pos0 = tx0 + h * RC;
        const vf2 z =
            *(const gvf2*)((const gfloat*)d.zrow + ((size_t)(T::HALVES * cx + h) * H + y) * 2);
        const LdsLine<1, 1> A{sG + r * PG + h * RC, sL + r * PL + h * RC};
        float (&xr)[RC] = *reinterpret_cast<float (*)[RC]>(xs);
        if (tx0 + kAosTX < W)
            chunk_recover<RC, false, true>(A, pos0, W, 1.f, z.x, z.y, xr);
        else
            chunk_recover<RC, true, true>(A, pos0, W, 1.f, z.x, z.y, xr);
    } else if (col_lane) {
        const vf2 z = *(const gvf2*)((const gfloat*)d.zcol + ((size_t)(pos0c / CC) * W + xcol) * 2);
        const LdsLine<PG, PL> A{sG + v * CC * PG + c, sL + v * CC * PL + c};
        if (pos0c + CC < H)
            chunk_recover<CC, false, true>(A, pos0c, H, 1.f, z.x, z.y, xs);
        else
            chunk_recover<CC, true, true>(A, pos0c, H, 1.f, z.x, z.y, xs);
    }
    __syncthreads();
    if (row_lane) {
        float* lp = sL + r * PL + h * RC;
#pragma unroll
        for (int k = 0; k < RC; ++k) lp[k] = __builtin_fmaf(0.5f, xs[k], lp[k]);
    }
    __syncthreads();
    if (col_lane) {
        gfloat* ob = (gfloat*)d.Lnext + (ptrdiff_t)uniform(pos0c) * W + tx0;
        const int rows = uniform(H - pos0c);
#pragma unroll
        for (int k = 0; k < CC; ++k) {
            const int rr = v * CC + k;
            if (k < rows)
                ob[(ptrdiff_t)k * W + c] = __builtin_fmaf(0.5f, xs[k], sL[rr * PL + c]);
        }
    }
}

// Recovery of tiles with one wavefront of row chunks and one column chunk
// per tile column (60 x 64 tiles with chunks of 60 and 64, 60 x 32 tiles
// with chunks of 30 and 32): each chunk is solved by two lanes (split_lower
// / split_upper) in two wavefronts, rows in wavefronts 0 (lower halves) and
// 1 (upper halves), columns in 2 and 3, so the serial walk is half a chunk
// long and four wavefronts sweep.  The middle values pass through LDS;
// otherwise as aos_recover_kernel.
template <int TY, int RC, int CC>
__global__ __launch_bounds__(256) void aos_recover_split_kernel(ImageDesc d0, AosWork w,
                                                                float tau) {
    using T = TileChunks<TY, RC, CC>;
    static_assert(chunk_lanes(TY, RC, CC) == 2 && T::HALVES * TY == kWave,
                  "one wavefront of row chunks and one column chunk per tile column");
    using SR = SplitChunk<RC>;
    using SC = SplitChunk<CC>;
    constexpr int WAVES = 4;
    constexpr int PL = kAosTX + 1, PG = kAosTX + 1;
    extern __shared__ float smem[];
    float* sL = smem;
    float* sG = smem + TY * PL;
    float* sX = sG + TY * PG;  // [direction][half][lane][2]
    const int tid = threadIdx.x, wave = uniform(tid >> 6), lane = tid & (kWave - 1);
    ImageDesc d;
    int lt;
    resolve(d0, w, xcd_contiguous((int)blockIdx.x, (int)gridDim.x), d, lt);
    if (d.gate && *d.gate <= d.bound) return;  // whole block
    const int W = d.W, H = d.H;
    const int ntx = (W + kAosTX - 1) / kAosTX;
    const int cx = lt % ntx, cy = lt / ntx;
    const int tx0 = cx * kAosTX, ty0 = cy * TY;
    const bool rows = wave < 2, upper = (wave & 1) != 0;  // wave-uniform
    // row lanes: chunk h of tile row r (lane = h TY + r); column lanes: tile column `lane`
    const int r = lane % TY, h = lane / TY;
    const int y = ty0 + r, xcol = tx0 + lane, px0 = tx0 + h * RC;
    const bool live = rows ? (y < H && px0 < W) : (lane < kAosTX && xcol < W);
    vf2 z = {0.f, 0.f};  // the chunk's end values, loaded with the tile
    if (live)
        z = rows ? *(const gvf2*)((const gfloat*)d.zrow + ((size_t)(T::HALVES * cx + h) * H + y) * 2)
                 : *(const gvf2*)((const gfloat*)d.zcol + ((size_t)(ty0 / CC) * W + xcol) * 2);
    {
        constexpr int PER = TY / WAVES;
        const bool in_x = lane < kAosTX && tx0 + lane < W;
        const gfloat* Lb = (const gfloat*)d.L + (ptrdiff_t)uniform(ty0 + wave) * W + tx0;
        const gfloat* gb = (const gfloat*)d.g + (ptrdiff_t)uniform(ty0 + wave) * W + tx0;
        float vl[PER], vg[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const bool in = in_x && ty0 + wave + WAVES * i < H;
            vl[i] = in ? Lb[(ptrdiff_t)(WAVES * i) * W + lane] : 0.f;
            vg[i] = in ? gb[(ptrdiff_t)(WAVES * i) * W + lane] : 0.f;
        }
        if (lane < kAosTX) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int rr = wave + WAVES * i;
                sL[rr * PL + lane] = vl[i];
                sG[rr * PG + lane] = tau * vg[i];
            }
        }
    }
    __syncthreads();
    // one half of a chunk per lane: the lower half's dp (x_0 = z0) and cp,
    // or the upper half's dq (its last element z1) and aq
    constexpr int NX = SC::NU > SR::MH + 1 ? SC::NU : SR::MH + 1;
    static_assert(SC::MH + 1 <= NX && SR::NU <= NX, "halves fit");
    float x[NX], c[NX];
    float* ex = sX + ((rows ? 0 : 2) + (upper ? 1 : 0)) * 2 * kWave + 2 * lane;
    const float* partner = sX + ((rows ? 0 : 2) + (upper ? 0 : 1)) * 2 * kWave + 2 * lane;
    if (live) {
        if (rows) {
            const LdsLine<1, 1> A{sG + r * PG + h * RC, sL + r * PL + h * RC};
            const bool chk = !(tx0 + kAosTX < W);
            if (!upper) {
                auto& xl = *reinterpret_cast<float (*)[SR::MH + 1]>(x);
                auto& cl = *reinterpret_cast<float (*)[SR::MH + 1]>(c);
                if (chk)
                    split_lower<RC, true>(A, px0, W, z.x, xl, cl);
                else
                    split_lower<RC, false>(A, px0, W, z.x, xl, cl);
                ex[0] = c[SR::MH];
                ex[1] = x[SR::MH];
            } else {
                auto& xu = *reinterpret_cast<float (*)[SR::NU]>(x);
                auto& cu = *reinterpret_cast<float (*)[SR::NU]>(c);
                if (chk)
                    split_upper<RC, true>(A, px0, W, z.y, xu, cu);
                else
                    split_upper<RC, false>(A, px0, W, z.y, xu, cu);
                ex[0] = c[0];
                ex[1] = x[0];
            }
        } else {
            const LdsLine<PG, PL> A{sG + lane, sL + lane};
            const bool chk = !(ty0 + CC < H);
            if (!upper) {
                auto& xl = *reinterpret_cast<float (*)[SC::MH + 1]>(x);
                auto& cl = *reinterpret_cast<float (*)[SC::MH + 1]>(c);
                if (chk)
                    split_lower<CC, true>(A, ty0, H, z.x, xl, cl);
                else
                    split_lower<CC, false>(A, ty0, H, z.x, xl, cl);
                ex[0] = c[SC::MH];
                ex[1] = x[SC::MH];
            } else {
                auto& xu = *reinterpret_cast<float (*)[SC::NU]>(x);
                auto& cu = *reinterpret_cast<float (*)[SC::NU]>(c);
                if (chk)
                    split_upper<CC, true>(A, ty0, H, z.y, xu, cu);
                else
                    split_upper<CC, false>(A, ty0, H, z.y, xu, cu);
                ex[0] = c[0];
                ex[1] = x[0];
            }
        }
    }
    __syncthreads();  // the middle coefficients of every chunk are in LDS
    if (live) {
        float xm, xm1;
        if (!upper) {
            split_middle(ex[0], ex[1], partner[0], partner[1], xm, xm1);
            if (rows) {
                x[SR::MH] = xm;
#pragma unroll
                for (int k = SR::MH - 1; k >= 1; --k) x[k] = __builtin_fmaf(-c[k], x[k + 1], x[k]);
            } else {
                x[SC::MH] = xm;
#pragma unroll
                for (int k = SC::MH - 1; k >= 1; --k) x[k] = __builtin_fmaf(-c[k], x[k + 1], x[k]);
            }
        } else {
            split_middle(partner[0], partner[1], ex[0], ex[1], xm, xm1);
            x[0] = xm1;
            if (rows) {
#pragma unroll
                for (int i = 1; i <= SR::NU - 2; ++i) x[i] = __builtin_fmaf(-c[i], x[i - 1], x[i]);
            } else {
#pragma unroll
                for (int i = 1; i <= SC::NU - 2; ++i) x[i] = __builtin_fmaf(-c[i], x[i - 1], x[i]);
            }
        }
    }
    if (rows && live) {  // L + delta_x / 2 into the LDS copy of L (rows own their elements)
        float* lp = sL + r * PL + h * RC;
        if (!upper) {
#pragma unroll
            for (int k = 0; k <= SR::MH; ++k) lp[k] = __builtin_fmaf(0.5f, x[k], lp[k]);
        } else {
#pragma unroll
            for (int i = 0; i < SR::NU; ++i)
                lp[SR::MH + 1 + i] = __builtin_fmaf(0.5f, x[i], lp[SR::MH + 1 + i]);
        }
    }
    __syncthreads();
    if (!rows && live) {  // L_i = L + (delta_x + delta_y)/2, one row at a time
        gfloat* ob = (gfloat*)d.Lnext + (ptrdiff_t)uniform(ty0) * W + tx0;
        const int nrows = uniform(H - ty0);
        if (!upper) {
#pragma unroll
            for (int k = 0; k <= SC::MH; ++k)
                if (k < nrows)
                    ob[(ptrdiff_t)k * W + lane] = __builtin_fmaf(0.5f, x[k], sL[k * PL + lane]);
        } else {
#pragma unroll
            for (int i = 0; i < SC::NU; ++i) {
                const int k = SC::MH + 1 + i;
                if (k < nrows)
                    ob[(ptrdiff_t)k * W + lane] = __builtin_fmaf(0.5f, x[i], sL[k * PL + lane]);
            }
        }
    }
}

// Global-memory accessor of one whole line for the probe solves: element
// k of the chunk at pos0, index clamped into the line (positions outside it
// get zero coupling weights in the chunk routines).
struct GlobalLineAcc {
    const float* gp;  // line element 0
    const float* Lp;
    int stride, pos0, n;
    __device__ __forceinline__ int at(int k) const {
        const int i = pos0 + k;
        return (i < 0 ? 0 : (i >= n ? n - 1 : i)) * stride;
    }
    __device__ __forceinline__ float g(int k) const { return gp[at(k)]; }
    __device__ __forceinline__ float L(int k) const { return Lp[at(k)]; }
};

constexpr int kProbeChunk = 64;  // unknowns per lane: lines of up to 64 x 64

// One wavefront per line through a probe window: lines 0..kProbeMax-1 are
// rows y0 + j, lines kProbeMax.. are columns x0 + j.  With pdesc (batches)
// probe p belongs to the image pdesc[rect_img[p]], else to d.
__global__ __launch_bounds__(kBlock) void aos_probe_kernel(ImageDesc d, const int4* rects,
                                                           int nprobes, float tau, float* delta,
                                                           const ImageDesc* pdesc,
                                                           const int* rect_img) {
    const int lane = threadIdx.x % kWave;
    const int wv = uniform(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);
    const int probe = wv / (2 * kProbeMax), j = wv % (2 * kProbeMax);
    if (probe >= nprobes) return;
    if (pdesc) d = pdesc[rect_img[probe]];
    const int4 r = rects[probe];  // x0, y0, w, h
    const bool row = j < kProbeMax;
    const int off = row ? j : j - kProbeMax;
    if (off >= (row ? r.w : r.z)) return;  // whole wavefront
    const int W = d.W, H = d.H;
    const int n = row ? W : H;
    const int line = row ? r.y + off : r.x + off;
    const int win0 = row ? r.x : r.y, win1 = win0 + (row ? r.z : r.w);
    const size_t base = row ? (size_t)line * W : (size_t)line;
    const int stride = row ? 1 : W;
    const int pos0 = lane * kProbeChunk;
    const GlobalLineAcc A{d.g + base, d.L + base, stride, pos0, n};
    Eq e0 = eq_identity(), e1 = eq_identity();
    if (pos0 < n) chunk_reduce<kProbeChunk>(A, pos0, n, tau, e0, e1);
    float z0, z1;
    wave_pcr_pairs(e0, e1, lane, z0, z1);
    if (pos0 < n && pos0 < win1 && pos0 + kProbeChunk > win0) {
        float x[kProbeChunk];
        chunk_recover<kProbeChunk>(A, pos0, n, tau, z0, z1, x);
        float* out = delta + (size_t)probe * 2 * kProbeMax * kProbeMax;
#pragma unroll
        for (int k = 0; k < kProbeChunk; ++k) {
            const int pos = pos0 + k;
            if (pos >= win0 && pos < win1) {
                if (row)
                    out[off * kProbeMax + (pos - win0)] = x[k];
                else
                    out[kProbeMax * kProbeMax + (pos - win0) * kProbeMax + off] = x[k];
            }
        }
    }
}

// Largest |cand - exact| over probe window blockIdx.x into *err (atomic max
// of the float bits).  With pdesc the window's image supplies L (d.L), the
// candidate (d.Lnext), the width and the error word (d.gate).
__global__ __launch_bounds__(kBlock) void probe_err_kernel(const float* L, const float* cand, int W,
                                                           const int4* rects, const float* delta,
                                                           unsigned* err, const ImageDesc* pdesc,
                                                           const int* rect_img) {
    __shared__ float red[kBlock];
    if (pdesc) {
        const ImageDesc& d = pdesc[rect_img[blockIdx.x]];
        L = d.L;
        cand = d.Lnext;
        W = d.W;
        err = reinterpret_cast<unsigned*>(const_cast<float*>(d.gate));
    }
    const int4 r = rects[blockIdx.x];
    const float* dl = delta + (size_t)blockIdx.x * 2 * kProbeMax * kProbeMax;
    float m = 0.f;
    for (int i = threadIdx.x; i < r.z * r.w; i += kBlock) {
        const int py = i / r.z, px = i - py * r.z;
        const size_t o = (size_t)(r.y + py) * W + (r.x + px);
        const float exact =
            L[o] + 0.5f * (dl[py * kProbeMax + px] + dl[kProbeMax * kProbeMax + py * kProbeMax + px]);
        float e = fabsf(cand[o] - exact);
        if (!(e <= 3.402823466e38f)) e = __builtin_inff();  // NaN or inf
        m = e > m ? e : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w2 = kBlock / 2; w2 > 0; w2 >>= 1) {
        if ((int)threadIdx.x < w2) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(err, __float_as_uint(red[0]));
}

int work_count(const ImageDesc& d0, const AosWork& w, int ty, int lines_m) {
    if (w.items) return w.count;
    return lines_m ? iface_groups(d0.H, d0.nchr, lines_m) + iface_groups(d0.W, d0.nchc, lines_m)
                   : aos_tiles_of(d0.W, d0.H, ty);
}

template <int RG, int TY, int RC, int CC, bool CG, int GM>
hipError_t launch_reduce_t(const ImageDesc& d0, const AosWork& w, const Taps& tc, float tau,
                           float k_host, hipStream_t s) {
    const int count = work_count(d0, w, TY, 0);
    if (count <= 0) return hipSuccess;
    const size_t lds = (size_t)RedGeom<RG, TY, CG>::floats * sizeof(float);
    hipLaunchKernelGGL((aos_reduce_kernel<RG, TY, RC, CC, CG, GM>), dim3(count),
                       dim3(kRedThreads), lds, s, d0, w, tc, tau, k_host);
    return hipGetLastError();
}

template <int RG, int TY, int RC, int CC>
hipError_t launch_reduce_g(const ImageDesc& d0, const AosWork& w, const Taps& tc, float tau,
                           int gmode, float k_host, hipStream_t s) {
    if (gmode == 0) return launch_reduce_t<RG, TY, RC, CC, true, 0>(d0, w, tc, tau, k_host, s);
    if (gmode == 1) return launch_reduce_t<RG, TY, RC, CC, true, 1>(d0, w, tc, tau, k_host, s);
    return hipErrorInvalidValue;
}

template <int TY, int RC, int CC>
hipError_t launch_reduce_s(const ImageDesc& d0, const AosWork& w, const Taps& tc, float tau,
                           bool compute_g, int gmode, float k_host, hipStream_t s) {
    if (!compute_g) return launch_reduce_t<1, TY, RC, CC, false, 0>(d0, w, tc, tau, k_host, s);
    switch (tc.r) {
        case 1: return launch_reduce_g<1, TY, RC, CC>(d0, w, tc, tau, gmode, k_host, s);
        case 2: return launch_reduce_g<2, TY, RC, CC>(d0, w, tc, tau, gmode, k_host, s);
        case 3: return launch_reduce_g<3, TY, RC, CC>(d0, w, tc, tau, gmode, k_host, s);
        case 4: return launch_reduce_g<4, TY, RC, CC>(d0, w, tc, tau, gmode, k_host, s);
        default: return hipErrorInvalidValue;
    }
}

template <int TY, int RC, int CC>
hipError_t launch_recover_t(const ImageDesc& d0, const AosWork& w, float tau, hipStream_t s) {
    const int count = work_count(d0, w, TY, 0);
    if (count <= 0) return hipSuccess;
    const size_t lds = (size_t)2 * TY * (kAosTX + 1) * sizeof(float);
    hipLaunchKernelGGL((aos_recover_kernel<TY, RC, CC>), dim3(count), dim3(TY * 4), lds, s, d0, w,
                       tau);
    return hipGetLastError();
}

// Long chunks (a row chunk across the tile, a column chunk down it): two
// lanes per chunk (aos_recover_split_kernel).
template <int TY, int RC, int CC>
hipError_t launch_recover_split_t(const ImageDesc& d0, const AosWork& w, float tau,
                                  hipStream_t s) {
    const int count = work_count(d0, w, TY, 0);
    if (count <= 0) return hipSuccess;
    const size_t lds = ((size_t)2 * TY * (kAosTX + 1) + 4 * 2 * kWave) * sizeof(float);
    hipLaunchKernelGGL((aos_recover_split_kernel<TY, RC, CC>), dim3(count), dim3(256), lds, s, d0,
                       w, tau);
    return hipGetLastError();
}

// Tile height and chunk lengths of a shape, as compiled kernel variants.
enum AosVariant { AV_32_SHORT = 0, AV_64_SHORT = 1, AV_64_LONG = 2, AV_NONE = -1 };
AosVariant aos_variant(int shape) {
    if (shape < 0 || shape >= kAosShapes) return AV_NONE;
    const AosShape& a = kAosShape[shape];
    if (a.ty == 32 && a.rc == 30 && a.cc == 32) return AV_32_SHORT;
    if (a.ty == 64 && a.rc == 30 && a.cc == 32) return AV_64_SHORT;
    if (a.ty == 64 && a.rc == 60 && a.cc == 64) return AV_64_LONG;
    return AV_NONE;
}

}  // namespace

hipError_t launch_cond(const BatchImage& d0, const ImgWork& w, const Taps& tc, float k_host,
                       int mode, int ty, hipStream_t s) {
    if (mode < 0 || mode > 2) return hipErrorInvalidValue;
    switch (tc.r) {
        case 1: return launch_cond_band_r<1>(d0, w, tc, k_host, mode, ty, s);
        case 2: return launch_cond_band_r<2>(d0, w, tc, k_host, mode, ty, s);
        case 3: return launch_cond_band_r<3>(d0, w, tc, k_host, mode, ty, s);
        case 4: return launch_cond_band_r<4>(d0, w, tc, k_host, mode, ty, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aos_reduce(const ImageDesc& d0, const AosWork& w, int shape, const Taps& tc,
                             float tau, bool compute_g, int gmode, float k_host, hipStream_t s) {
    switch (aos_variant(shape)) {
        case AV_32_SHORT:
            return launch_reduce_s<32, 30, 32>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case AV_64_SHORT:
            return launch_reduce_s<64, 30, 32>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        case AV_64_LONG:
            return launch_reduce_s<64, 60, 64>(d0, w, tc, tau, compute_g, gmode, k_host, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aos_iface(const ImageDesc& d0, const AosWork& w, int shape, hipStream_t s) {
    if (shape < 0 || shape >= kAosShapes) return hipErrorInvalidValue;
    const int M = kAosShape[shape].m;
    const int count = work_count(d0, w, 0, M);
    if (count <= 0) return hipSuccess;
    const int waves = kIfaceThreads / kWave;
    if (M == 4)
        hipLaunchKernelGGL(aos_iface_kernel<4>, dim3((count + waves - 1) / waves),
                           dim3(kIfaceThreads), 0, s, d0, w, count);
    else if (M == 8)
        hipLaunchKernelGGL(aos_iface_kernel<8>, dim3((count + waves - 1) / waves),
                           dim3(kIfaceThreads), 0, s, d0, w, count);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

static_assert(chunk_lanes(32, 30, 32) == 2 && chunk_lanes(64, 30, 32) == 1 &&
                  chunk_lanes(64, 60, 64) == 2,
              "the recovery variants below match the lanes per chunk of each shape");

hipError_t launch_aos_recover(const ImageDesc& d0, const AosWork& w, int shape, float tau,
                              hipStream_t s) {
    switch (aos_variant(shape)) {
        case AV_32_SHORT: return launch_recover_split_t<32, 30, 32>(d0, w, tau, s);
        case AV_64_SHORT: return launch_recover_t<64, 30, 32>(d0, w, tau, s);
        case AV_64_LONG: return launch_recover_split_t<64, 60, 64>(d0, w, tau, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aos_probe(const ImageDesc& d, const int4* rects, int nprobes, float tau,
                            float* delta, hipStream_t s, const ImageDesc* pdesc,
                            const int* rect_img) {
    if (nprobes <= 0) return hipSuccess;
    const int waves = nprobes * 2 * kProbeMax, per = kBlock / kWave;
    hipLaunchKernelGGL(aos_probe_kernel, dim3((waves + per - 1) / per), dim3(kBlock), 0, s, d, rects,
                       nprobes, tau, delta, pdesc, rect_img);
    return hipGetLastError();
}

hipError_t launch_probe_err(const float* L, const float* cand, int W, const int4* rects,
                            int nprobes, const float* delta, unsigned* err, hipStream_t s,
                            const ImageDesc* pdesc, const int* rect_img) {
    if (nprobes <= 0) return hipSuccess;
    hipLaunchKernelGGL(probe_err_kernel, dim3(nprobes), dim3(kBlock), 0, s, L, cand, W, rects, delta,
                       err, pdesc, rect_img);
    return hipGetLastError();
}

}  // namespace kaze
