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
// the transpose).  All four products are dense n x n x n contractions, run on
// v_mfma_f64_16x16x4_f64.  Each wavefront owns a super-block of SB x SB output
// tiles of 16 x 16 and keeps their accumulators in registers; the 4-deep K
// step of the instruction is fed from a 16-deep chunk that every lane loads as
// one contiguous run of 4 values, so lane l covers k = k0 + 4*(l/16) + s at
// step s for both operands.  Tau lives in a per-workgroup scratch slot (it is
// needed transposed for G_X and untransposed for G_Y), which the workgroup
// reuses for every pair it processes.  Workgroups are persistent; workgroup b
// runs on XCD b % 8, and each XCD is given a contiguous range of the pair list
// (sorted by monomer), so the monomer matrices it touches stay in its L2.
#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSB = 3;          // 3 x 3 tiles of 16 x 16 per wavefront
constexpr int kXcds = 8;

__device__ inline d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline d4 load4(const double* p) { return *reinterpret_cast<const d4*>(p); }

// Position of accumulator element t (0..3) of lane `lane` inside its 16 x 16 tile
// for v_mfma_f64_16x16x4_f64: rows lane/16, lane/16 + 4, + 8, + 12 of column lane%16
// (operands: A lane l = (row l%16, k l/16), B lane l = (k l/16, column l%16)).
__device__ inline int acc_row(int lane, int t) { return (lane >> 4) + 4 * t; }
__device__ inline int acc_col(int lane, int t) { return lane & 15; }

struct PairView {
    const double* V;      // nX x nY, row-major
    const double* MX;     // npX x npX
    const double* MY;     // npY x npY
    const double* eX;     // oX occupied then vX virtual energies
    const double* eY;
    double* GX;
    double* GY;
    int oX, vX, nX, npX;
    int oY, vY, nY, npY;
};

// acc[i][j] += sum_k MX[r][k] V[k][c] + sum_k V[r][k] MY[c][k] over the tiles
// (rb0 + i, cb0 + j) of the npX x npY output.
__device__ void tau_tiles(const PairView& p, int rb0, int cb0, int RB, int CB, int lane,
                          d4 (&acc)[kSB][kSB]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int k0 = 0; k0 < p.npX; k0 += 16) {
        d4 a[kSB];
#pragma unroll
        for (int i = 0; i < kSB; ++i)
            a[i] = (rb0 + i < RB) ? load4(p.MX + (int64_t)((rb0 + i) * 16 + lr) * p.npX + k0 + lk) : d4(0.0);
        double b[kSB][4];
#pragma unroll
        for (int j = 0; j < kSB; ++j) {
            const int c = (cb0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (kk < p.nX && c < p.nY) ? p.V[(int64_t)kk * p.nY + c] : 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < kSB; ++i)
#pragma unroll
                for (int j = 0; j < kSB; ++j)
                    if (rb0 + i < RB && cb0 + j < CB) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
    }
    for (int k0 = 0; k0 < p.npY; k0 += 16) {
        double a[kSB][4];
#pragma unroll
        for (int i = 0; i < kSB; ++i) {
            const int r = (rb0 + i) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                a[i][s] = (r < p.nX && kk < p.nY) ? p.V[(int64_t)r * p.nY + kk] : 0.0;
            }
        }
        d4 b[kSB];
#pragma unroll
        for (int j = 0; j < kSB; ++j)
            b[j] = (cb0 + j < CB) ? load4(p.MY + (int64_t)((cb0 + j) * 16 + lr) * p.npY + k0 + lk) : d4(0.0);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < kSB; ++i)
#pragma unroll
                for (int j = 0; j < kSB; ++j)
                    if (rb0 + i < RB && cb0 + j < CB) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
    }
}

// acc[i][j] = sum_c Tau[r][c] V[r'][c]   (G_X tiles (rb0+i, rb'0+j), npX x npX)
__device__ void gx_tiles(const PairView& p, const double* tau, int rb0, int qb0, int RB, int lane,
                         d4 (&acc)[kSB][kSB]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int k0 = 0; k0 < p.npY; k0 += 16) {
        d4 a[kSB];
#pragma unroll
        for (int i = 0; i < kSB; ++i)
            a[i] = (rb0 + i < RB) ? load4(tau + (int64_t)((rb0 + i) * 16 + lr) * p.npY + k0 + lk) : d4(0.0);
        double b[kSB][4];
#pragma unroll
        for (int j = 0; j < kSB; ++j) {
            const int q = (qb0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (q < p.nX && kk < p.nY) ? p.V[(int64_t)q * p.nY + kk] : 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < kSB; ++i)
#pragma unroll
                for (int j = 0; j < kSB; ++j)
                    if (rb0 + i < RB && qb0 + j < RB) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
    }
}

// acc[i][j] = sum_r Tau[r][c] V[r][c']   (G_Y tiles (cb0+i, qb0+j), npY x npY)
__device__ void gy_tiles(const PairView& p, const double* tau, int cb0, int qb0, int CB, int lane,
                         d4 (&acc)[kSB][kSB]) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int k0 = 0; k0 < p.npX; k0 += 16) {
        double a[kSB][4];
#pragma unroll
        for (int i = 0; i < kSB; ++i) {
            const int c = (cb0 + i) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                a[i][s] = (cb0 + i < CB) ? tau[(int64_t)(k0 + lk + s) * p.npY + c] : 0.0;
        }
        double b[kSB][4];
#pragma unroll
        for (int j = 0; j < kSB; ++j) {
            const int q = (qb0 + j) * 16 + lr;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + lk + s;
                b[j][s] = (kk < p.nX && q < p.nY) ? p.V[(int64_t)kk * p.nY + q] : 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < kSB; ++i)
#pragma unroll
                for (int j = 0; j < kSB; ++j)
                    if (cb0 + i < CB && qb0 + j < CB) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
    }
}

__device__ inline void atomic_flush(double* G, int ld, int n, int rb0, int qb0, int lane,
                                    const d4 (&acc)[kSB][kSB]) {
#pragma unroll
    for (int i = 0; i < kSB; ++i)
#pragma unroll
        for (int j = 0; j < kSB; ++j) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = (qb0 + j) * 16 + acc_col(lane, t);
                const int r = (rb0 + i) * 16 + acc_row(lane, t);
                if (r < n && c < n) unsafeAtomicAdd(G + (int64_t)r * ld + c, acc[i][j][t]);
            }
        }
}

__device__ inline double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ inline int64_t pair_for(int64_t it, int64_t n_pair) {
    // XCD-contiguous order: workgroup b runs on XCD b % 8
    const int g = gridDim.x;
    if (g % kXcds != 0) return (int64_t)blockIdx.x + it * g;
    const int xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds, per = g / kXcds;
    const int64_t begin = n_pair * xcd / kXcds, end = n_pair * (xcd + 1) / kXcds;
    const int64_t p = begin + local + it * per;
    return p < end ? p : INT64_MAX;
}

__global__ __launch_bounds__(kThreads) void pair_fp64_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ eps, const double* __restrict__ V, const double* __restrict__ M,
    double* __restrict__ G, double* __restrict__ scratch, int64_t slot_elems,
    double* __restrict__ ed2, int couple, const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    __shared__ double red[kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* tau = scratch + (int64_t)blockIdx.x * slot_elems;
    for (int64_t it = 0;; ++it) {
        const int64_t pi = pair_for(it, n_pair);
        if (pi >= n_pair) break;
        const PairDesc pd = pairs[pi];
        const MonoDesc dx = monos[pd.x], dy = monos[pd.y];
        PairView p;
        p.V = V + pd.v_off;
        p.MX = M + dx.mat_off;
        p.MY = M + dy.mat_off;
        p.eX = eps + dx.eps_off;
        p.eY = eps + dy.eps_off;
        p.GX = G + dx.mat_off;
        p.GY = G + dy.mat_off;
        p.oX = dx.o; p.vX = dx.v; p.nX = dx.n; p.npX = dx.np;
        p.oY = dy.o; p.vY = dy.v; p.nY = dy.n; p.npY = dy.np;
        const int RB = p.npX / 16, CB = p.npY / 16;
        const int SR = (RB + kSB - 1) / kSB, SC = (CB + kSB - 1) / kSB;
        const int rot = (int)(pi % kWaves);

        // ---- Tau = D_XY * (V + M_X V + V M_Y^T), E_D2 = 4 <V, Tau> ----
        double epart = 0.0;
        for (int sb = (wave + rot) % kWaves; sb < SR * SC; sb += kWaves) {
            const int rb0 = (sb / SC) * kSB, cb0 = (sb % SC) * kSB;
            d4 acc[kSB][kSB];
#pragma unroll
            for (int i = 0; i < kSB; ++i)
#pragma unroll
                for (int j = 0; j < kSB; ++j) acc[i][j] = d4(0.0);
            tau_tiles(p, rb0, cb0, RB, CB, lane, acc);
#pragma unroll
            for (int i = 0; i < kSB; ++i)
#pragma unroll
                for (int j = 0; j < kSB; ++j) {
                    if (rb0 + i >= RB || cb0 + j >= CB) continue;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int c = (cb0 + j) * 16 + acc_col(lane, t);
                        const int jo = c / p.vY, b = c - jo * p.vY;
                        const int r = (rb0 + i) * 16 + acc_row(lane, t);
                        double tv = 0.0;
                        if (r < p.nX && c < p.nY) {
                            const int io = r / p.vX, a = r - io * p.vX;
                            const double dinv =
                                1.0 / (((p.eX[io] + p.eY[jo]) - p.eX[p.oX + a]) - p.eY[p.oY + b]);
                            const double v = p.V[(int64_t)r * p.nY + c];
                            tv = dinv * (v + acc[i][j][t]);
                            epart += v * tv;
                        }
                        if (couple) tau[(int64_t)r * p.npY + c] = tv;
                    }
                }
        }
        epart = wave_sum(epart);
        if (lane == 0) red[wave] = epart;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[w];
            ed2[pd.orig] = 4.0 * s;
        }
        if (couple) {
            // ---- G_X += Tau V^T (npX x npX),  G_Y += Tau^T V (npY x npY) ----
            const int SX = SR * SR, SY = SC * SC;
            for (int sb = (wave + rot) % kWaves; sb < SX + SY; sb += kWaves) {
                d4 acc[kSB][kSB];
#pragma unroll
                for (int i = 0; i < kSB; ++i)
#pragma unroll
                    for (int j = 0; j < kSB; ++j) acc[i][j] = d4(0.0);
                if (sb < SX) {
                    const int rb0 = (sb / SR) * kSB, qb0 = (sb % SR) * kSB;
                    gx_tiles(p, tau, rb0, qb0, RB, lane, acc);
                    atomic_flush(p.GX, p.npX, p.nX, rb0, qb0, lane, acc);
                } else {
                    const int s2 = sb - SX;
                    const int cb0 = (s2 / SC) * kSB, qb0 = (s2 % SC) * kSB;
                    gy_tiles(p, tau, cb0, qb0, CB, lane, acc);
                    atomic_flush(p.GY, p.npY, p.nY, cb0, qb0, lane, acc);
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

int pair_fp64_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_fp64_kernel, kThreads, 0) != hipSuccess ||
        n < 1)
        n = 1;
    return n;
}

void launch_pair_fp64(const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos, const double* eps,
                      const double* V, const double* M, double* G, double* scratch, int64_t slot_elems,
                      int grid, double* ed2, int couple, const Ctrl* ctrl, hipStream_t s) {
    if (n_pair <= 0) return;
    hipLaunchKernelGGL(pair_fp64_kernel, dim3(grid), dim3(kThreads), 0, s, pairs, n_pair, monos, eps,
                       V, M, G, scratch, slot_elems, ed2, couple, ctrl);
}

}  // namespace mcpt
