// Intramonomer terms of the monomer doubles equation (Eq. 58) on CDNA4 matrix
// cores, FP64.
//
// With T-hat[(i,a),(j,b)] = T^{ab}_{ij} and M-hat = 2T - S(T) (S swaps the
// occupied indices), the terms of Eq. 58 that stay on monomer X are
//
//   L = P + H + R + R^T
//   P[(i,a),(j,b)] = sum_{c,d} <ab|cd> T[(i,c),(j,d)]          particle-particle ladder
//   H[(i,a),(j,b)] = sum_{k,l} <kl|ij> T[(k,a),(l,b)]          hole-hole ladder
//   R = K M - J T - Vs(J Vs(T))                                 the four ring combinations
//
// where K[(i,a),(j,b)] = <ab|ij> (the intra block, also the exchange-type ring
// integral for real orbitals), J[(i,a),(j,b)] = <aj|bi> = (ab|ji) and Vs swaps
// the virtual indices, Vs(A)[(i,a),(j,b)] = A[(i,b),(j,a)].  The printed ring
// terms come in pairs related by (i,a) <-> (i1,a1), which is R and R^T.
//
// Kernels (per sweep, after the pair phase, before the monomer update):
//  * lccd_ring_kernel: R12 = K M - J T and Y = J Vs(T), dense np x np x np
//    products on v_mfma_f64_16x16x4_f64 in 3 x 3 super-blocks of 16 x 16 tiles,
//    operands from L2 (a monomer's matrices are 166 KB at o = 5, v = 27).
//  * lccd_ladder_kernel: P as the product W[(a,b),(c,d)] x T[(i,c),(j,d)] of
//    the v^2 x v^2 integral matrix (streamed from HBM once per sweep, rows
//    padded to 16) with the o^2 amplitude columns gathered from T through an LDS
//    offset table; its epilogue adds H, R12 and Y at the (r, c) and (c, r)
//    positions and writes L.  This is the HBM-bound part: v^4 integrals per
//    monomer, each used o^2 times.
#include "lccd.hpp"

namespace mcpt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kLccdThreads = 256;   // four wavefronts
constexpr int kRingSB = 3;          // ring super-block edge in tiles
constexpr int kLadRT = 2;           // ladder row tiles per wave task
constexpr int kLadCT = 4;           // ladder column tiles per pass (o^2 <= 64 in one pass)

__device__ inline d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline d4 load4(const double* p) { return *reinterpret_cast<const d4*>(p); }

// accumulator element t of lane l sits at row l/16 + 4t, column l%16;
// operand lane l carries row (A) or column (B) l%16 and k = 4 (l/16) + s at step s
__device__ inline int acc_row(int lane, int t) { return (lane >> 4) + 4 * t; }

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
// W_X (v^2 x v^2, caller layout) -> rows of ldw doubles, rows and columns
// zero-padded to multiples of 16; J_X[i][j][a][b] = <ia|jb> -> J-hat[(i,a),(j,b)]
// = J_X[j][i][a][b] in the np x np monomer layout.  A null source skips its part.
__global__ void lccd_pack_kernel(const MonoDesc* __restrict__ monos, const LccdDesc* __restrict__ ld,
                                 const double* __restrict__ w_raw, const double* __restrict__ j_raw,
                                 double* __restrict__ W, double* __restrict__ J) {
    const int x = blockIdx.y;
    const MonoDesc d = monos[x];
    const LccdDesc l = ld[x];
    const int v2 = d.v * d.v;
    const int64_t nw = w_raw ? (int64_t)l.w_rows * l.ldw : 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / l.ldw), k = (int)(e - (int64_t)r * l.ldw);
        W[l.w_off + e] = (r < v2 && k < v2) ? w_raw[l.w_raw_off + (int64_t)r * v2 + k] : 0.0;
    }
    const int np = d.np, n = d.n, o = d.o, v = d.v;
    const int64_t nn = j_raw ? (int64_t)np * np : 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / np), c = (int)(e - (int64_t)r * np);
        double val = 0.0;
        if (r < n && c < n) {
            const int i = r / v, a = r - i * v, j = c / v, b = c - j * v;
            val = j_raw[d.raw_off + (((int64_t)j * o + i) * v + a) * v + b];
        }
        J[d.mat_off + e] = val;
    }
}

// ---------------------------------------------------------------------------
// ring products
// ---------------------------------------------------------------------------
// One wave task: a super-block of up to 3 x 3 output tiles of either
// R12 = K M - J T (kind 0) or Y = J Vs(T) (kind 1).  Rows or columns past the
// padded edge are clamped for the loads and skipped for the stores.
__global__ __launch_bounds__(kLccdThreads) void lccd_ring_kernel(
    const MonoDesc* __restrict__ monos, int blocks_per_mono, const double* __restrict__ K,
    const double* __restrict__ J, const double* __restrict__ T, const double* __restrict__ M,
    double* __restrict__ R12, double* __restrict__ Y, const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int x = blockIdx.x / blocks_per_mono;
    const int part = blockIdx.x - x * blocks_per_mono;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;
    __shared__ int kofs[kLccdMaxNp];   // Vs(T) row k = (i2, a2) -> i2 v np + a2 (0 past n)
    const int np = d.np, n = d.n, v = d.v;
    for (int k = threadIdx.x; k < np; k += kLccdThreads) {
        const int i2 = k / v, a2 = k - i2 * v;
        kofs[k] = k < n ? i2 * v * np + a2 : 0;
    }
    __syncthreads();
    const double* Kx = K + d.mat_off;
    const double* Jx = J + d.mat_off;
    const double* Tx = T + d.mat_off;
    const double* Mx = M + d.mat_off;
    const int nt = np / 16;
    const int nsb = (nt + kRingSB - 1) / kRingSB;
    const int tasks = 2 * nsb * nsb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int task = part * (kLccdThreads / 64) + wave; task < tasks; task += blocks_per_mono * (kLccdThreads / 64)) {
        const int kind = task / (nsb * nsb);
        const int sb = task - kind * nsb * nsb;
        const int tr0 = (sb / nsb) * kRingSB, tc0 = (sb % nsb) * kRingSB;
        int arow[kRingSB], bcol[kRingSB], ycol[kRingSB];
#pragma unroll
        for (int u = 0; u < kRingSB; ++u) {
            const int r = (tr0 + u) * 16 + lr, c = (tc0 + u) * 16 + lr;
            arow[u] = r < np ? r : 0;
            bcol[u] = c < np ? c : 0;
            const int i1 = c / v, a = c - i1 * v;
            ycol[u] = c < n ? a * np + i1 * v : 0;   // Vs(T) column c = (i1, a)
        }
        d4 acc[kRingSB][kRingSB];
#pragma unroll
        for (int u = 0; u < kRingSB; ++u)
#pragma unroll
            for (int w = 0; w < kRingSB; ++w) acc[u][w] = d4(0.0);
        // kind 0: two products into one accumulator, the second with -J
        const int nprod = kind == 0 ? 2 : 1;
        for (int pr = 0; pr < nprod; ++pr) {
            const double* A = (kind == 0 && pr == 0) ? Kx : Jx;
            const double sgn = (kind == 0 && pr == 1) ? -1.0 : 1.0;
            const double* B = (kind == 0 && pr == 0) ? Mx : Tx;
            for (int k0 = 0; k0 < np; k0 += 16) {
                double a[kRingSB][4], b[kRingSB][4];
#pragma unroll
                for (int u = 0; u < kRingSB; ++u) {
                    const d4 av = load4(A + (int64_t)arow[u] * np + k0 + lk);
                    a[u][0] = sgn * av.x;
                    a[u][1] = sgn * av.y;
                    a[u][2] = sgn * av.z;
                    a[u][3] = sgn * av.w;
                }
                if (kind == 0) {
#pragma unroll
                    for (int w = 0; w < kRingSB; ++w)
#pragma unroll
                        for (int s = 0; s < 4; ++s) b[w][s] = B[(int64_t)(k0 + lk + s) * np + bcol[w]];
                } else {
#pragma unroll
                    for (int w = 0; w < kRingSB; ++w)
#pragma unroll
                        for (int s = 0; s < 4; ++s) b[w][s] = Tx[kofs[k0 + lk + s] + ycol[w]];
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int u = 0; u < kRingSB; ++u)
#pragma unroll
                        for (int w = 0; w < kRingSB; ++w) acc[u][w] = mfma(a[u][s], b[w][s], acc[u][w]);
            }
        }
        double* out = (kind == 0 ? R12 : Y) + d.mat_off;
#pragma unroll
        for (int u = 0; u < kRingSB; ++u)
#pragma unroll
            for (int w = 0; w < kRingSB; ++w) {
                const int c = (tc0 + w) * 16 + lr;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int r = (tr0 + u) * 16 + acc_row(lane, t);
                    if (r < n && c < n) out[(int64_t)r * np + c] = acc[u][w][t];
                }
            }
    }
}

// ---------------------------------------------------------------------------
// ladders and assembly of L
// ---------------------------------------------------------------------------
// Wave task: kLadRT row tiles of W (rows (a,b)) against up to kLadCT column
// tiles of the gathered amplitudes (columns (i,j)); passes over column groups
// when o^2 > 64.  The epilogue writes L[(i,a),(j,b)].
__global__ __launch_bounds__(kLccdThreads) void lccd_ladder_kernel(
    const MonoDesc* __restrict__ monos, const LccdDesc* __restrict__ ld, int blocks_per_mono,
    const double* __restrict__ W, const double* __restrict__ Q, const double* __restrict__ T,
    const double* __restrict__ R12, const double* __restrict__ Y, double* __restrict__ L,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int x = blockIdx.x / blocks_per_mono;
    const int part = blockIdx.x - x * blocks_per_mono;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;
    const LccdDesc l = ld[x];
    __shared__ int kofs[kLccdMaxLdw];   // W column k = (c, d) -> T offset c np + d (0 past v^2)
    const int np = d.np, n = d.n, o = d.o, v = d.v, v2 = v * v, o2 = o * o;
    for (int k = threadIdx.x; k < l.ldw; k += kLccdThreads) {
        const int c = k / v, dd = k - c * v;
        kofs[k] = k < v2 ? c * np + dd : 0;
    }
    __syncthreads();
    const double* Wx = W + l.w_off;
    const double* Qx = Q + l.q_off;
    const double* Tx = T + d.mat_off;
    const double* Rx = R12 + d.mat_off;
    const double* Yx = Y + d.mat_off;
    double* Lx = L + d.mat_off;
    const int nrt = l.w_rows / 16;
    const int ntask_r = (nrt + kLadRT - 1) / kLadRT;
    const int nct = (o2 + 15) / 16;
    const int ngroups = (nct + kLadCT - 1) / kLadCT;
    const int tasks = ntask_r * ngroups;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int task = part * (kLccdThreads / 64) + wave; task < tasks; task += blocks_per_mono * (kLccdThreads / 64)) {
        const int tr0 = (task / ngroups) * kLadRT;
        const int tc0 = (task % ngroups) * kLadCT;
        int arow[kLadRT], bbase[kLadCT];
#pragma unroll
        for (int u = 0; u < kLadRT; ++u) {
            const int r = (tr0 + u) * 16 + lr;
            arow[u] = r < l.w_rows ? r : 0;
        }
#pragma unroll
        for (int w = 0; w < kLadCT; ++w) {
            const int col = (tc0 + w) * 16 + lr;   // (i, j)
            const int i = col / o, j = col - i * o;
            bbase[w] = col < o2 ? i * v * np + j * v : 0;
        }
        d4 acc[kLadRT][kLadCT];
#pragma unroll
        for (int u = 0; u < kLadRT; ++u)
#pragma unroll
            for (int w = 0; w < kLadCT; ++w) acc[u][w] = d4(0.0);
        d4 an[kLadRT];
#pragma unroll
        for (int u = 0; u < kLadRT; ++u) an[u] = load4(Wx + (int64_t)arow[u] * l.ldw + lk);
        for (int k0 = 0; k0 < l.ldw; k0 += 16) {
            double a[kLadRT][4], b[kLadCT][4];
#pragma unroll
            for (int u = 0; u < kLadRT; ++u) {
                a[u][0] = an[u].x;
                a[u][1] = an[u].y;
                a[u][2] = an[u].z;
                a[u][3] = an[u].w;
            }
            if (k0 + 16 < l.ldw) {
#pragma unroll
                for (int u = 0; u < kLadRT; ++u) an[u] = load4(Wx + (int64_t)arow[u] * l.ldw + k0 + 16 + lk);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int ko = kofs[k0 + lk + s];
#pragma unroll
                for (int w = 0; w < kLadCT; ++w) b[w][s] = Tx[ko + bbase[w]];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int u = 0; u < kLadRT; ++u)
#pragma unroll
                    for (int w = 0; w < kLadCT; ++w) acc[u][w] = mfma(a[u][s], b[w][s], acc[u][w]);
        }
        // epilogue: element (m = (a,b), col = (i,j)) -> L[(i,a),(j,b)]
#pragma unroll
        for (int w = 0; w < kLadCT; ++w) {
            const int col = (tc0 + w) * 16 + lr;
            if (col >= o2) continue;
            const int i = col / o, j = col - i * o;
#pragma unroll
            for (int u = 0; u < kLadRT; ++u)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int m = (tr0 + u) * 16 + acc_row(lane, t);
                    if (m >= v2) continue;
                    const int a = m / v, b = m - a * v;
                    const int r = i * v + a, c = j * v + b;
                    double h = 0.0;   // sum_{k,l} <kl|ij> T[(k,a),(l,b)]
                    for (int k = 0; k < o; ++k)
                        for (int q = 0; q < o; ++q)
                            h += Qx[((k * o + q) * o + i) * o + j] * Tx[(int64_t)(k * v + a) * np + q * v + b];
                    const double rr = Rx[(int64_t)r * np + c] - Yx[(int64_t)(i * v + b) * np + j * v + a];
                    const double rt = Rx[(int64_t)c * np + r] - Yx[(int64_t)(j * v + a) * np + i * v + b];
                    Lx[(int64_t)r * np + c] = ((acc[u][w][t] + h) + rr) + rt;
                }
        }
    }
    (void)n;
}

}  // namespace

void launch_lccd_pack(const MonoDesc* monos, const LccdDesc* ld, int n_mono, const double* w_raw,
                      const double* j_raw, double* W, double* J, hipStream_t s) {
    if (n_mono <= 0) return;
    hipLaunchKernelGGL(lccd_pack_kernel, dim3(64, n_mono), dim3(256), 0, s, monos, ld, w_raw, j_raw, W, J);
}

int lccd_ring_blocks(int max_np) {
    const int nt = max_np / 16, nsb = (nt + kRingSB - 1) / kRingSB;
    const int tasks = 2 * nsb * nsb, per_block = kLccdThreads / 64;
    const int b = (tasks + per_block - 1) / per_block;
    return b < 8 ? b : 8;
}

int lccd_ladder_blocks(int max_w_rows, int max_o) {
    const int nrt = max_w_rows / 16, ntr = (nrt + kLadRT - 1) / kLadRT;
    const int nct = (max_o * max_o + 15) / 16, ng = (nct + kLadCT - 1) / kLadCT;
    const int tasks = ntr * ng, per_block = kLccdThreads / 64;
    const int b = (tasks + per_block - 1) / per_block;
    return b < 64 ? b : 64;
}

void launch_lccd_ring(const MonoDesc* monos, int n_mono, int ring_blocks, const double* K, const double* J,
                      const double* T, const double* M, double* R12, double* Y, const Ctrl* ctrl, const ClState* cl,
                      hipStream_t s) {
    if (n_mono <= 0 || ring_blocks <= 0) return;
    hipLaunchKernelGGL(lccd_ring_kernel, dim3(n_mono * ring_blocks), dim3(kLccdThreads), 0, s, monos, ring_blocks, K,
                       J, T, M, R12, Y, ctrl, cl);
}

void launch_lccd_ladder(const MonoDesc* monos, const LccdDesc* ld, int n_mono, int ladder_blocks, const double* W,
                        const double* Q, const double* T, const double* R12, const double* Y, double* L,
                        const Ctrl* ctrl, const ClState* cl, hipStream_t s) {
    if (n_mono <= 0 || ladder_blocks <= 0) return;
    hipLaunchKernelGGL(lccd_ladder_kernel, dim3(n_mono * ladder_blocks), dim3(kLccdThreads), 0, s, monos, ld,
                       ladder_blocks, W, Q, T, R12, Y, L, ctrl, cl);
}

}  // namespace mcpt
