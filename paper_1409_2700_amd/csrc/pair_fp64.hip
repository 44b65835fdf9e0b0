// Pair phase of the MCPT(2) sweep in FP64 on CDNA4 matrix cores.
//
// For a stored pair (X, Y) with V = V_XY (nX x nY, rows (i,a) of X, columns
// (j,b) of Y) and the spin-adapted monomer combinations M = 2T - S(T):
//
//   Tau  = D_XY * (V + M_X V + V M_Y^T)       Eq. 59: source + T_X and T_Y couplings
//   E_D2 = 4 <V, Tau>                          Eq. 55
//   G_X += Tau V^T,   G_Y += Tau^T V           Eq. 58: the pair term seen from X and from Y
//
// (the Eq. 58 pair term of monomer X is G_X + G_X^T; the monomer kernel adds
// the transpose).  The four products are dense n x n x n contractions on
// v_mfma_f64_16x16x4_f64.
//
// Structure.  Persistent workgroups walk the pair list; workgroup b runs on
// XCD b % 8 and each XCD takes a contiguous range of the monomer-sorted pairs,
// so the M and G blocks it touches stay in its L2.  Two variants:
//  * LDS-resident V (pairs with nX (npY + 2) doubles <= 157,696 B): eight
//    wavefronts (two per SIMD, so one wave's memory waits are covered by the
//    other's MFMAs), one workgroup per CU.  V is staged once per pair into LDS
//    (row stride npY + 2 doubles so column-chunk reads of 16 rows fall on
//    distinct banks) and every product reads it from there: V is streamed from
//    HBM once per pass, and the L2 is asked for the next pair's V while the
//    current pair's second phase runs.
//  * V from L2 (larger pairs): four wavefronts, two workgroups per CU.
// M_X, M_Y and Tau (a per-workgroup scratch slot, needed transposed for G_X and
// untransposed for G_Y) come from L2 with the next k-chunk prefetched into
// registers.  Output tiles of 16 x 16 are grouped into 3 x 3 super-blocks
// (accumulators in registers, each operand fragment reused three times); whole
// super-blocks go round-robin to the wavefronts and the super-blocks left over
// as 1 x 3 row strips, so the SIMDs get (nearly) equal work between barriers.
// Task shapes are compile-time (3 x 3, 1 x 3 or a single tile) so each MFMA
// block is straight-line code.  A wave raises its issue priority while it runs
// an MFMA block, so the two waves of a SIMD tend to alternate whole blocks (one
// computes while the other's operand loads are in flight) instead of
// interleaving single instructions.
//
// Operand layout of the instruction (measured): A lane l = (row l%16, k l/16),
// B lane l = (k l/16, column l%16), accumulator element t of lane l = (row
// l/16 + 4t, column l%16).  A 16-deep k chunk is loaded as 4 contiguous values
// per lane, so lane l covers k = k0 + 4*(l/16) + s at step s for both operands.
#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kThreadsL = 512;   // LDS-resident V: eight wavefronts, one workgroup per CU
constexpr int kThreadsG = 256;   // V from L2: four wavefronts, two workgroups per CU
constexpr int kSB = 3;           // super-block edge in tiles
constexpr int kXcds = 8;
constexpr int kLdsV = 19712;     // LDS doubles for V (157,696 B): nX * (npY + 2) must fit
constexpr int kLdsD = 640;       // LDS doubles for the energy differences of X and Y: npX + npY must fit

template <int R, int C>
struct Shape {
    static constexpr int NR = R, NC = C;
};

__device__ inline d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline d4 load4(const double* p) { return *reinterpret_cast<const d4*>(p); }

// 4 consecutive doubles from LDS at a 16-byte aligned address
__device__ inline d4 lds4(const double* p) {
    const d2 lo = *reinterpret_cast<const d2*>(p);
    const d2 hi = *reinterpret_cast<const d2*>(p + 2);
    d4 r;
    r.x = lo.x;
    r.y = lo.y;
    r.z = hi.x;
    r.w = hi.y;
    return r;
}

__device__ inline void split(const d4& v, double (&o)[4]) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
}

__device__ inline int acc_row(int lane, int t) { return (lane >> 4) + 4 * t; }
__device__ inline int acc_col(int lane) { return lane & 15; }

template <int NR, int NC>
__device__ inline void zero(d4 (&acc)[NR][NC]) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[i][j] = d4(0.0);
}

template <int NR, int NC>
__device__ inline void mma_block(d4 (&acc)[NR][NC], const double (&a)[NR][4], const double (&b)[NC][4]) {
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
    __builtin_amdgcn_s_setprio(0);
}

struct PairView {
    const double* V;      // nX x nY, row-major, global
    const double* MX;     // npX x npX
    const double* MY;     // npY x npY
    const double* dX;     // e_i - e_a over rows (i,a) of X
    const double* dY;     // e_j - e_b over columns (j,b) of Y
    double* GX;
    double* GY;
    int nX, npX;
    int nY, npY;
    int ldv;              // LDS row stride of V (npY + 2) when staged
};

// ---------------------------------------------------------------------------
// V staged in LDS (sV: nX rows, row stride ldv, columns >= nY zero)
// ---------------------------------------------------------------------------

// acc += M_X V + V M_Y^T on tiles (r0.., c0..) of the npX x npY output
template <int NR, int NC>
__device__ void tau_sb_lds(const PairView& p, const double* sV, int r0, int c0, int lane, d4 (&acc)[NR][NC]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    d4 an[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) an[i] = load4(p.MX + (int64_t)((r0 + i) * 16 + lr) * p.npX + lk);
    for (int k0 = 0; k0 < p.npX; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i) split(an[i], a[i]);
        if (k0 + 16 < p.npX) {
#pragma unroll
            for (int i = 0; i < NR; ++i)
                an[i] = load4(p.MX + (int64_t)((r0 + i) * 16 + lr) * p.npX + k0 + 16 + lk);
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int c = (c0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (kk < p.nX) ? sV[kk * p.ldv + c] : 0.0;
            }
        }
        mma_block(acc, a, b);
    }
    d4 bn[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) bn[j] = load4(p.MY + (int64_t)((c0 + j) * 16 + lr) * p.npY + lk);
    for (int k0 = 0; k0 < p.npY; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int j = 0; j < NC; ++j) split(bn[j], b[j]);
        if (k0 + 16 < p.npY) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
                bn[j] = load4(p.MY + (int64_t)((c0 + j) * 16 + lr) * p.npY + k0 + 16 + lk);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int r = (r0 + i) * 16 + lr;
            split((r < p.nX) ? lds4(sV + r * p.ldv + k0 + lk) : d4(0.0), a[i]);
        }
        mma_block(acc, a, b);
    }
}

// acc = sum_c Tau[r][c] V[q][c]   (G_X tiles)
template <int NR, int NC>
__device__ void gx_sb_lds(const PairView& p, const double* sV, const double* tau, int r0, int q0, int lane,
                          d4 (&acc)[NR][NC]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    d4 an[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) an[i] = load4(tau + (int64_t)((r0 + i) * 16 + lr) * p.npY + lk);
    for (int k0 = 0; k0 < p.npY; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i) split(an[i], a[i]);
        if (k0 + 16 < p.npY) {
#pragma unroll
            for (int i = 0; i < NR; ++i)
                an[i] = load4(tau + (int64_t)((r0 + i) * 16 + lr) * p.npY + k0 + 16 + lk);
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int q = (q0 + j) * 16 + lr;
            split((q < p.nX) ? lds4(sV + q * p.ldv + k0 + lk) : d4(0.0), b[j]);
        }
        mma_block(acc, a, b);
    }
}

// acc = sum_r Tau[r][c] V[r][q]   (G_Y tiles)
template <int NR, int NC>
__device__ void gy_sb_lds(const PairView& p, const double* sV, const double* tau, int c0, int q0, int lane,
                          d4 (&acc)[NR][NC]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    double an[NR][4];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int s = 0; s < 4; ++s) an[i][s] = tau[(int64_t)(lk + s) * p.npY + (c0 + i) * 16 + lr];
    for (int k0 = 0; k0 < p.npX; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) a[i][s] = an[i][s];
        if (k0 + 16 < p.npX) {
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    an[i][s] = tau[(int64_t)(k0 + 16 + lk + s) * p.npY + (c0 + i) * 16 + lr];
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int q = (q0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (kk < p.nX) ? sV[kk * p.ldv + q] : 0.0;
            }
        }
        mma_block(acc, a, b);
    }
}

// ---------------------------------------------------------------------------
// V read from global memory (pairs too large for LDS)
// ---------------------------------------------------------------------------
template <int NR, int NC>
__device__ void tau_sb_glb(const PairView& p, int r0, int c0, int lane, d4 (&acc)[NR][NC]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int k0 = 0; k0 < p.npX; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i) split(load4(p.MX + (int64_t)((r0 + i) * 16 + lr) * p.npX + k0 + lk), a[i]);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int c = (c0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (kk < p.nX && c < p.nY) ? p.V[(int64_t)kk * p.nY + c] : 0.0;
            }
        }
        mma_block(acc, a, b);
    }
    for (int k0 = 0; k0 < p.npY; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int r = (r0 + i) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                a[i][s] = (r < p.nX && kk < p.nY) ? p.V[(int64_t)r * p.nY + kk] : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) split(load4(p.MY + (int64_t)((c0 + j) * 16 + lr) * p.npY + k0 + lk), b[j]);
        mma_block(acc, a, b);
    }
}

template <int NR, int NC>
__device__ void gx_sb_glb(const PairView& p, const double* tau, int r0, int q0, int lane, d4 (&acc)[NR][NC]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int k0 = 0; k0 < p.npY; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i) split(load4(tau + (int64_t)((r0 + i) * 16 + lr) * p.npY + k0 + lk), a[i]);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int q = (q0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (q < p.nX && kk < p.nY) ? p.V[(int64_t)q * p.nY + kk] : 0.0;
            }
        }
        mma_block(acc, a, b);
    }
}

template <int NR, int NC>
__device__ void gy_sb_glb(const PairView& p, const double* tau, int c0, int q0, int lane, d4 (&acc)[NR][NC]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int k0 = 0; k0 < p.npX; k0 += 16) {
        double a[NR][4], b[NC][4];
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) a[i][s] = tau[(int64_t)(k0 + lk + s) * p.npY + (c0 + i) * 16 + lr];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int q = (q0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (kk < p.nX && q < p.nY) ? p.V[(int64_t)kk * p.nY + q] : 0.0;
            }
        }
        mma_block(acc, a, b);
    }
}

// ---------------------------------------------------------------------------
// task lists: full super-blocks round-robin over the waves (partial edge
// super-blocks as single tiles of the same wave), the remainder tile by tile
// ---------------------------------------------------------------------------
struct Grid {
    int RT, CT, SR, SC, n;    // tiles, super-blocks per dimension, super-block count
};

__device__ inline Grid make_grid(int RT, int CT) {
    Grid g;
    g.RT = RT;
    g.CT = CT;
    g.SR = (RT + kSB - 1) / kSB;
    g.SC = (CT + kSB - 1) / kSB;
    g.n = g.SR * g.SC;
    return g;
}

// Visit the tasks of `wave` over the concatenation of grids g0 and g1 (g1 may be
// empty): f(which, r0, c0, shape) in tile coordinates, shape Shape<3,3>,
// Shape<1,3> or Shape<1,1>.  Full super-blocks go round-robin to the waves; the
// super-blocks left over after the last full round are cut into 1 x 3 row
// strips (three independent accumulators keep the MFMA pipe busy, where single
// tiles would wait on each k chunk) and dealt out one by one.  Edge super-blocks
// narrower than three tiles run as single tiles.
template <class F>
__device__ inline void for_tasks(const Grid& g0, const Grid& g1, int wave, int nwaves, F&& f) {
    const int total = g0.n + g1.n;
    const int full = total - total % nwaves;
    for (int sb = wave; sb < full; sb += nwaves) {
        const int which = sb >= g0.n ? 1 : 0;
        const Grid& g = which ? g1 : g0;
        const int s = which ? sb - g0.n : sb;
        const int r0 = (s / g.SC) * kSB, c0 = (s % g.SC) * kSB;
        const int nr = min(kSB, g.RT - r0), nc = min(kSB, g.CT - c0);
        if (nr == kSB && nc == kSB) {
            f(which, r0, c0, Shape<kSB, kSB>{});
        } else {
            for (int i = 0; i < nr; ++i) {
                if (nc == kSB) f(which, r0 + i, c0, Shape<1, kSB>{});
                else
                    for (int j = 0; j < nc; ++j) f(which, r0 + i, c0 + j, Shape<1, 1>{});
            }
        }
    }
    int idx = 0;
    for (int sb = full; sb < total; ++sb) {
        const int which = sb >= g0.n ? 1 : 0;
        const Grid& g = which ? g1 : g0;
        const int s = which ? sb - g0.n : sb;
        const int r0 = (s / g.SC) * kSB, c0 = (s % g.SC) * kSB;
        const int nr = min(kSB, g.RT - r0), nc = min(kSB, g.CT - c0);
        for (int i = 0; i < nr; ++i) {
            if (nc == kSB) {
                if (idx++ % nwaves == wave) f(which, r0 + i, c0, Shape<1, kSB>{});
            } else {
                for (int j = 0; j < nc; ++j, ++idx)
                    if (idx % nwaves == wave) f(which, r0 + i, c0 + j, Shape<1, 1>{});
            }
        }
    }
}

// G block contributions: FP64 atomics into G, or (deterministic mode) plain
// stores of the whole padded block into the pair's partial slot
template <int NR, int NC>
__device__ inline void atomic_flush(double* G, double* part, int ld, int n, int r0, int q0, int lane,
                                    const d4 (&acc)[NR][NC]) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int c = (q0 + j) * 16 + acc_col(lane);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = (r0 + i) * 16 + acc_row(lane, t);
                if (part) part[(int64_t)r * ld + c] = acc[i][j][t];
                else if (r < n && c < n) unsafeAtomicAdd(G + (int64_t)r * ld + c, acc[i][j][t]);
            }
        }
}

__device__ inline double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ inline int64_t pair_for(int64_t it, int64_t n_pair) {
    const int g = gridDim.x;
    if (g % kXcds != 0) return (int64_t)blockIdx.x + it * g;
    const int xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds, per = g / kXcds;
    const int64_t begin = n_pair * xcd / kXcds, end = n_pair * (xcd + 1) / kXcds;
    const int64_t p = begin + local + it * per;
    return p < end ? p : INT64_MAX;
}

__device__ inline PairView make_view(const PairDesc& pd, const MonoDesc* monos, const double* dif,
                                     const double* V, const double* M, double* G) {
    const MonoDesc dx = monos[pd.x], dy = monos[pd.y];
    PairView p;
    p.V = V + pd.v_off;
    p.MX = M + dx.mat_off;
    p.MY = M + dy.mat_off;
    p.dX = dif + dx.dif_off;
    p.dY = dif + dy.dif_off;
    p.GX = G + dx.mat_off;
    p.GY = G + dy.mat_off;
    p.nX = dx.n;
    p.npX = dx.np;
    p.nY = dy.n;
    p.npY = dy.np;
    p.ldv = dy.np + 2;
    return p;
}

// One body for both variants: IN_LDS stages V in LDS (the pair list given to
// it holds only pairs that fit); otherwise V is read from L2.  DIMER (1: every
// monomer of one size, 2: any sizes, from the pair's descriptor) adds the
// dimer-internal source of po to the numerator of Tau and keeps Tau.
template <bool IN_LDS, int NT, int DIMER>
__device__ inline void pair_body(const PairDesc* __restrict__ pairs, int64_t n_pair,
                                 const MonoDesc* __restrict__ monos, const double* __restrict__ dif,
                                 const double* __restrict__ V, const double* __restrict__ M,
                                 double* __restrict__ G, double* __restrict__ scratch, int64_t slot_elems,
                                 double* __restrict__ ed2, int couple, const ClState* __restrict__ cl,
                                 PartOut po, double* sV, double* sD, double* red) {
    constexpr int NW = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* tau = scratch + (int64_t)blockIdx.x * slot_elems;
    double sink = 0.0;
    for (int64_t it = 0;; ++it) {
        const int64_t pi = pair_for(it, n_pair);
        if (pi >= n_pair) break;
        const PairDesc pd = pairs[pi];
        if (cl && cl[pd.cluster].done) continue;   // cluster stopped: uniform over the workgroup
        const PairView p = make_view(pd, monos, dif, V, M, G);
        const int RB = p.npX / 16, CB = p.npY / 16;

        if (IN_LDS) {   // stage V: rows of X, columns of Y zero-padded to ldv; loads batched
            constexpr int kRows = 4, kCols = 3;
            for (int rb = wave; rb < p.nX; rb += NW * kRows)
                for (int cb = 0; cb < p.ldv; cb += 64 * kCols) {
                    double tmp[kRows][kCols];
#pragma unroll
                    for (int k = 0; k < kRows; ++k)
#pragma unroll
                        for (int m = 0; m < kCols; ++m) {
                            const int r = rb + NW * k, c = cb + lane + 64 * m;
                            tmp[k][m] = (r < p.nX && c < p.nY) ? p.V[(int64_t)r * p.nY + c] : 0.0;
                        }
#pragma unroll
                    for (int k = 0; k < kRows; ++k)
#pragma unroll
                        for (int m = 0; m < kCols; ++m) {
                            const int r = rb + NW * k, c = cb + lane + 64 * m;
                            if (r < p.nX && c < p.ldv) sV[r * p.ldv + c] = tmp[k][m];
                        }
                }
            // the energy differences of X's rows and Y's columns (zero in the padding) for the epilogue
            for (int k = threadIdx.x; k < p.npX + p.npY; k += NT) sD[k] = k < p.npX ? p.dX[k] : p.dY[k - p.npX];
            __syncthreads();
        }

        // ---- Tau = D_XY * (V + M_X V + V M_Y^T), E_D2 = 4 <V, Tau> ----
        double epart = 0.0;
        // the pair's dimer-internal source and Tau (sizes and offsets from its descriptor)
        int dvx = 1, dvy = 1, dm1 = 0, dm2 = 0;
        const double *Sp = nullptr, *Y1p = nullptr, *Y2p = nullptr;
        double* Tp = nullptr;
        if (DIMER == 1) {   // one size: every pair's matrices np x np at orig * mat_stride
            dvx = dvy = po.v;
            dm1 = dm2 = p.npY;
            Sp = po.S + pd.orig * po.mat_stride;
            Y1p = po.Y1 + pd.orig * po.mat_stride;
            Y2p = po.Y2 + pd.orig * po.mat_stride;
            Tp = po.tau_out + pd.orig * po.mat_stride;
        } else if (DIMER == 2) {
            const DimerDesc& e = po.dd[pd.orig];
            dvx = e.vx;
            dvy = e.vy;
            dm1 = e.m1;
            dm2 = e.m2;
            Sp = po.S + e.tau_off;
            Y1p = po.Y1 + e.y1_off;
            Y2p = po.Y2 + e.y2_off;
            Tp = po.tau_out + e.tau_off;
        }
        for_tasks(make_grid(RB, CB), make_grid(0, 0), wave, NW, [&](int, int r0, int c0, auto shape) {
            constexpr int NR = decltype(shape)::NR, NC = decltype(shape)::NC;
            d4 acc[NR][NC];
            zero(acc);
            if (IN_LDS) tau_sb_lds(p, sV, r0, c0, lane, acc);
            else tau_sb_glb(p, r0, c0, lane, acc);
            // Epilogue, one tile column at a time: its inputs are gathered before its stores to
            // the Tau slot (a global store orders later global loads behind it), indices are
            // clamped into the valid block and the padding is masked by selects, so the loads
            // issue back to back with one wait instead of a branch and a round trip per element.
            // dX and dY are read at the padded indices directly (zero beyond n; masked).
            const double* dXs = IN_LDS ? sD : p.dX;
            const double* dYs = IN_LDS ? sD + p.npX : p.dY;
            double dxr[NR][4];
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) dxr[i][t] = dXs[(r0 + i) * 16 + acc_row(lane, t)];
            if constexpr (DIMER == 0) {
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const int c = (c0 + j) * 16 + acc_col(lane);
                    const int cc = min(c, p.nY - 1);
                    const double dyc = dYs[c];
                    double vv[NR][4];
#pragma unroll
                    for (int i = 0; i < NR; ++i)
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int rr = min((r0 + i) * 16 + acc_row(lane, t), p.nX - 1);
                            vv[i][t] = IN_LDS ? sV[rr * p.ldv + c] : p.V[(int64_t)rr * p.nY + cc];
                        }
#pragma unroll
                    for (int i = 0; i < NR; ++i)
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int r = (r0 + i) * 16 + acc_row(lane, t);
                            const bool ok = r < p.nX && c < p.nY;
                            const double dinv = recip(dxr[i][t] + dyc);
                            const double tv = ok ? dinv * (vv[i][t] + acc[i][j][t]) : 0.0;
                            epart += ok ? vv[i][t] * tv : 0.0;
                            if (couple) tau[(int64_t)r * p.npY + c] = tv;
                        }
                }
            } else {
                // with the dimer source, four reads per element (V, S and the two cross-ring
                // products at the clamped element rr = (ii,a), cc = (jj,b)): one tile at a time,
                // or the gathered values of a whole tile column spill
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const int c = (c0 + j) * 16 + acc_col(lane);
                    const int cc = min(c, p.nY - 1);
                    const double dyc = dYs[c];
#pragma unroll
                    for (int i = 0; i < NR; ++i) {
                        double vv[4], dsrc[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int rr = min((r0 + i) * 16 + acc_row(lane, t), p.nX - 1);
                            const int r = (r0 + i) * 16 + acc_row(lane, t);
                            vv[t] = IN_LDS ? sV[rr * p.ldv + c] : p.V[(int64_t)rr * p.nY + cc];
                            if (DIMER == 1) {
                                const int ii = rr / dvx, a = rr - ii * dvx, jj = cc / dvx, b = cc - jj * dvx;
                                dsrc[t] = Sp[(int64_t)r * p.npY + c] -
                                          Y1p[(int64_t)(ii * dvx + b) * dm1 + jj * dvx + a] -
                                          Y2p[(int64_t)(jj * dvx + a) * dm1 + ii * dvx + b];
                            } else {
                                const int ii = rr / dvx, a = rr - ii * dvx, jj = cc / dvy, b = cc - jj * dvy;
                                dsrc[t] = Sp[(int64_t)r * p.npY + c] -
                                          Y1p[(int64_t)(ii * dvy + b) * dm2 + jj * dvx + a] -
                                          Y2p[(int64_t)(jj * dvx + a) * dm1 + ii * dvy + b];
                            }
                        }
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int r = (r0 + i) * 16 + acc_row(lane, t);
                            const bool ok = r < p.nX && c < p.nY;
                            const double dinv = recip(dxr[i][t] + dyc);
                            const double tv = ok ? dinv * (vv[t] + dsrc[t] + acc[i][j][t]) : 0.0;
                            epart += ok ? vv[t] * tv : 0.0;
                            if (couple) tau[(int64_t)r * p.npY + c] = tv;
                            Tp[(int64_t)r * p.npY + c] = tv;
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        });
        epart = wave_sum(epart);
        if (lane == 0) red[wave] = epart;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += red[w];
            ed2[pd.orig] = 4.0 * s;
        }
        if (IN_LDS) {   // ask the L2 for the next pair's V while this pair finishes
            const int64_t pn = pair_for(it + 1, n_pair);
            if (pn < n_pair) {
                const PairDesc nd = pairs[pn];
                const int64_t nv = (int64_t)monos[nd.x].n * monos[nd.y].n;
                const double* vn = V + nd.v_off;
                for (int64_t e = (int64_t)threadIdx.x * 16; e < nv; e += (int64_t)NT * 16) sink += vn[e];
            }
        }
        if (couple) {
            // ---- G_X += Tau V^T (RB x RB tiles), G_Y += Tau^T V (CB x CB tiles) ----
            for_tasks(make_grid(RB, RB), make_grid(CB, CB), wave, NW, [&](int which, int r0, int c0, auto shape) {
                constexpr int NR = decltype(shape)::NR, NC = decltype(shape)::NC;
                d4 acc[NR][NC];
                zero(acc);
                if (which == 0) {
                    if (IN_LDS) gx_sb_lds(p, sV, tau, r0, c0, lane, acc);
                    else gx_sb_glb(p, tau, r0, c0, lane, acc);
                    atomic_flush(p.GX, po.part ? po.part + po.off[pi] : nullptr, p.npX, p.nX, r0, c0, lane, acc);
                } else {
                    if (IN_LDS) gy_sb_lds(p, sV, tau, r0, c0, lane, acc);
                    else gy_sb_glb(p, tau, r0, c0, lane, acc);
                    atomic_flush(p.GY, po.part ? po.part + po.off[pi] + (int64_t)p.npX * p.npX : nullptr, p.npY,
                                 p.nY, r0, c0, lane, acc);
                }
            });
        }
        __syncthreads();
    }
    if (sink == 1.2345e300) ed2[0] = sink;   // keeps the prefetch loads; never true for finite inputs
}

template <int DIMER>
__global__ __launch_bounds__(kThreadsL) void pair_fp64_lds_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ dif, const double* __restrict__ V, const double* __restrict__ M,
    double* __restrict__ G, double* __restrict__ scratch, int64_t slot_elems,
    double* __restrict__ ed2, int couple, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl, PartOut po) {
    if (ctrl && ctrl->done) return;
    __shared__ __align__(16) double sV[kLdsV];
    __shared__ double sD[kLdsD];
    __shared__ double red[kThreadsL / 64];
    pair_body<true, kThreadsL, DIMER>(pairs, n_pair, monos, dif, V, M, G, scratch, slot_elems, ed2, couple, cl, po, sV,
                                      sD, red);
}

template <int DIMER>
__global__ __launch_bounds__(kThreadsG, 2) void pair_fp64_glb_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ dif, const double* __restrict__ V, const double* __restrict__ M,
    double* __restrict__ G, double* __restrict__ scratch, int64_t slot_elems,
    double* __restrict__ ed2, int couple, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl, PartOut po) {
    if (ctrl && ctrl->done) return;
    __shared__ double red[kThreadsG / 64];
    pair_body<false, kThreadsG, DIMER>(pairs, n_pair, monos, dif, V, M, G, scratch, slot_elems, ed2, couple, cl, po,
                                       nullptr, nullptr, red);
}

// ---------------------------------------------------------------------------
// pairs from L2, split: Tau tasks, then G tasks, each a 3 x 3 block of tiles
// of one pair (edge blocks tile by tile), taken by the waves of the XCD the
// pair belongs to in pair order
// ---------------------------------------------------------------------------
__device__ inline int sb_count(int tiles) { return (tiles + kSB - 1) / kSB; }

// the pair j of XCD group [b, e) that task t falls in (pre: exclusive prefix of task counts)
__device__ inline int task_pair(const int32_t* __restrict__ pre, int b, int e, int t) {
    int lo = b, hi = e - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// wave-level task loop shared by the two kernels: f(j, local task) for every task of this wave
template <class F>
__device__ inline void for_glb_tasks(const GlbTasks& T, int wave, F&& f) {
    constexpr int NW = kThreadsG / 64;
    const int x = blockIdx.x % kXcds, local = blockIdx.x / kXcds, per = gridDim.x / kXcds;
    const int b = T.xbeg[x], e = T.xbeg[x + 1];
    if (b >= e) return;
    const int t1 = T.pre[e], gw = local * NW + wave, nw = per * NW;
    for (int t = T.pre[b] + gw; t < t1; t += nw) {
        const int j = task_pair(T.pre, b, e, t);
        f(j, t - T.pre[j]);
    }
}

// Tau = D_XY * (V + M_X V + V M_Y^T) on tiles (r0.., c0..) into the pair's Tau slot; returns the
// lane's part of <V, Tau>
template <int NR, int NC>
__device__ inline double tau_block_glb(const PairView& p, double* tau, int r0, int c0, int lane, int couple) {
    d4 acc[NR][NC];
    zero(acc);
    tau_sb_glb(p, r0, c0, lane, acc);
    double dxr[NR][4];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) dxr[i][t] = p.dX[(r0 + i) * 16 + acc_row(lane, t)];
    double epart = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const int c = (c0 + j) * 16 + acc_col(lane);
        const int cc = min(c, p.nY - 1);
        const double dyc = p.dY[c];
        double vv[NR][4];
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int rr = min((r0 + i) * 16 + acc_row(lane, t), p.nX - 1);
                vv[i][t] = p.V[(int64_t)rr * p.nY + cc];
            }
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = (r0 + i) * 16 + acc_row(lane, t);
                const bool ok = r < p.nX && c < p.nY;
                const double tv = ok ? recip(dxr[i][t] + dyc) * (vv[i][t] + acc[i][j][t]) : 0.0;
                epart += ok ? vv[i][t] * tv : 0.0;
                if (couple) tau[(int64_t)r * p.npY + c] = tv;
            }
    }
    return epart;
}

// E_D2 of the chunk's pairs of live clusters set to zero before their Tau tasks add to it
__global__ __launch_bounds__(256) void glb_zero_ed2_kernel(const PairDesc* __restrict__ pairs,
                                                            const int32_t* __restrict__ xpair, int n,
                                                            double* __restrict__ ed2, const Ctrl* __restrict__ ctrl,
                                                            const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const PairDesc pd = pairs[xpair[k]];
    if (cl && cl[pd.cluster].done) return;
    ed2[pd.orig] = 0.0;
}

__global__ __launch_bounds__(kThreadsG, 2) void pair_glb_tau_kernel(
    GlbTasks T, const PairDesc* __restrict__ pairs, const MonoDesc* __restrict__ monos,
    const double* __restrict__ dif, const double* __restrict__ V, const double* __restrict__ M,
    double* __restrict__ scratch, double* __restrict__ ed2, int couple, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for_glb_tasks(T, wave, [&](int j, int lt) {
        const PairDesc pd = pairs[T.xpair[j]];
        if (cl && cl[pd.cluster].done) return;   // uniform over the wave
        const PairView p = make_view(pd, monos, dif, V, M, nullptr);
        double* tau = scratch + T.tau_off[j];
        const int RB = p.npX / 16, CB = p.npY / 16, SC = sb_count(CB);
        const int r0 = (lt / SC) * kSB, c0 = (lt % SC) * kSB;
        const int nr = min(kSB, RB - r0), nc = min(kSB, CB - c0);
        double epart = 0.0;
        if (nr == kSB && nc == kSB) {
            epart = tau_block_glb<kSB, kSB>(p, tau, r0, c0, lane, couple);
        } else {
            for (int i = 0; i < nr; ++i)
                for (int k = 0; k < nc; ++k) epart += tau_block_glb<1, 1>(p, tau, r0 + i, c0 + k, lane, couple);
        }
        epart = wave_sum(epart);
        if (lane == 0) unsafeAtomicAdd(ed2 + pd.orig, 4.0 * epart);
    });
}

template <int NR, int NC>
__device__ inline void g_block_glb(const PairView& p, const double* tau, int which, int r0, int c0, int lane) {
    d4 acc[NR][NC];
    zero(acc);
    if (which == 0) {
        gx_sb_glb(p, tau, r0, c0, lane, acc);
        atomic_flush(p.GX, nullptr, p.npX, p.nX, r0, c0, lane, acc);
    } else {
        gy_sb_glb(p, tau, r0, c0, lane, acc);
        atomic_flush(p.GY, nullptr, p.npY, p.nY, r0, c0, lane, acc);
    }
}

__global__ __launch_bounds__(kThreadsG, 2) void pair_glb_g_kernel(
    GlbTasks T, const PairDesc* __restrict__ pairs, const MonoDesc* __restrict__ monos,
    const double* __restrict__ dif, const double* __restrict__ V, const double* __restrict__ M,
    double* __restrict__ G, const double* __restrict__ scratch, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for_glb_tasks(T, wave, [&](int j, int lt) {
        const PairDesc pd = pairs[T.xpair[j]];
        if (cl && cl[pd.cluster].done) return;
        const PairView p = make_view(pd, monos, dif, V, M, G);
        const double* tau = scratch + T.tau_off[j];
        const int RB = p.npX / 16, CB = p.npY / 16, SR = sb_count(RB), SC = sb_count(CB);
        const int which = lt < SR * SR ? 0 : 1;
        const int S = which ? SC : SR, n = which ? CB : RB, u = which ? lt - SR * SR : lt;
        const int r0 = (u / S) * kSB, c0 = (u % S) * kSB;
        const int nr = min(kSB, n - r0), nc = min(kSB, n - c0);
        if (nr == kSB && nc == kSB) {
            g_block_glb<kSB, kSB>(p, tau, which, r0, c0, lane);
        } else {
            for (int i = 0; i < nr; ++i)
                for (int k = 0; k < nc; ++k) g_block_glb<1, 1>(p, tau, which, r0 + i, c0 + k, lane);
        }
    });
}

}  // namespace

int glb_tau_tasks(int npX, int npY) {
    const int sr = (npX / 16 + kSB - 1) / kSB, sc = (npY / 16 + kSB - 1) / kSB;
    return sr * sc;
}

int glb_g_tasks(int npX, int npY) {
    const int sr = (npX / 16 + kSB - 1) / kSB, sc = (npY / 16 + kSB - 1) / kSB;
    return sr * sr + sc * sc;
}

void launch_pair_fp64_split(const GlbTasks& tau_tasks, const GlbTasks& g_tasks, int n_chunk_pairs,
                            const PairDesc* pairs, const MonoDesc* monos, const double* dif, const double* V,
                            const double* M, double* G, double* scratch, int grid, double* ed2, int couple,
                            const Ctrl* ctrl, const ClState* cl, hipStream_t s) {
    if (n_chunk_pairs <= 0) return;
    hipLaunchKernelGGL(glb_zero_ed2_kernel, dim3((n_chunk_pairs + 255) / 256), dim3(256), 0, s, pairs,
                       tau_tasks.xpair, n_chunk_pairs, ed2, ctrl, cl);
    hipLaunchKernelGGL(pair_glb_tau_kernel, dim3(grid), dim3(kThreadsG), 0, s, tau_tasks, pairs, monos, dif, V, M,
                       scratch, ed2, couple, ctrl, cl);
    if (couple)
        hipLaunchKernelGGL(pair_glb_g_kernel, dim3(grid), dim3(kThreadsG), 0, s, g_tasks, pairs, monos, dif, V, M,
                           G, scratch, ctrl, cl);
}

int pair_fp64_blocks_per_cu(int lds_variant) {
    int n = 0;
    hipError_t e = lds_variant
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_fp64_lds_kernel<0>, kThreadsL, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_fp64_glb_kernel<0>, kThreadsG, 0);
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

bool pair_fits_lds(int nX, int npX, int npY) { return (int64_t)nX * (npY + 2) <= kLdsV && npX + npY <= kLdsD; }

void launch_pair_fp64(int lds_variant, PartOut po, const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos,
                      const double* dif, const double* V, const double* M, double* G, double* scratch,
                      int64_t slot_elems, int grid, double* ed2, int couple, const Ctrl* ctrl, const ClState* cl,
                      hipStream_t s) {
    if (n_pair <= 0) return;
    const int dimer = po.S == nullptr ? 0 : po.dd ? 2 : 1;
    if (lds_variant) {
        if (dimer == 2)
            hipLaunchKernelGGL(pair_fp64_lds_kernel<2>, dim3(grid), dim3(kThreadsL), 0, s, pairs, n_pair, monos,
                               dif, V, M, G, scratch, slot_elems, ed2, couple, ctrl, cl, po);
        else if (dimer == 1)
            hipLaunchKernelGGL(pair_fp64_lds_kernel<1>, dim3(grid), dim3(kThreadsL), 0, s, pairs, n_pair, monos,
                               dif, V, M, G, scratch, slot_elems, ed2, couple, ctrl, cl, po);
        else
            hipLaunchKernelGGL(pair_fp64_lds_kernel<0>, dim3(grid), dim3(kThreadsL), 0, s, pairs, n_pair, monos,
                               dif, V, M, G, scratch, slot_elems, ed2, couple, ctrl, cl, po);
    } else {
        if (dimer == 2)
            hipLaunchKernelGGL(pair_fp64_glb_kernel<2>, dim3(grid), dim3(kThreadsG), 0, s, pairs, n_pair, monos,
                               dif, V, M, G, scratch, slot_elems, ed2, couple, ctrl, cl, po);
        else if (dimer == 1)
            hipLaunchKernelGGL(pair_fp64_glb_kernel<1>, dim3(grid), dim3(kThreadsG), 0, s, pairs, n_pair, monos,
                               dif, V, M, G, scratch, slot_elems, ed2, couple, ctrl, cl, po);
        else
            hipLaunchKernelGGL(pair_fp64_glb_kernel<0>, dim3(grid), dim3(kThreadsG), 0, s, pairs, n_pair, monos,
                               dif, V, M, G, scratch, slot_elems, ed2, couple, ctrl, cl, po);
    }
}

}  // namespace mcpt
