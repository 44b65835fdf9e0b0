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
//    offset table, then H on the same accumulators (k over the o^2 hole pairs,
//    A = T gathered, B = <kl|ij>); its epilogue adds R12 and Y at the (r, c)
//    and (c, r) positions and writes L.  This is the HBM-bound part: v^4
//    integrals per monomer, each used o^2 times.
//  Both kernels place every workgroup of a monomer on one XCD.
#include "lccd.hpp"

namespace mcpt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kLccdThreads = 256;   // four wavefronts
constexpr int kRingSB = 3;          // ring super-block edge in tiles
constexpr int kLadRT = 4;           // ladder row tiles per wave task
constexpr int kLadCT = 4;           // ladder column tiles per task at most (the launch takes ceil(o^2 / 16))
constexpr int kXcds = 8;            // XCDs of the chip; workgroup b runs on XCD b % 8
constexpr int kLadLdsThreads = 768; // LDS-staged ladder: twelve wavefronts (three per SIMD), one workgroup per CU

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
// W_X (v^2 x v^2, caller layout) -> w_rows rows of ldw doubles, zero-padded
// (rows to a multiple of 16, columns to a multiple of 32); J_X[i][j][a][b] = <ia|jb> -> J-hat[(i,a),(j,b)]
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
__global__ __launch_bounds__(kLccdThreads, 2) void lccd_ring_kernel(
    const MonoDesc* __restrict__ monos, int n_mono, int blocks_per_mono, const double* __restrict__ K,
    const double* __restrict__ J, const double* __restrict__ T, const double* __restrict__ M,
    double* __restrict__ R12, double* __restrict__ Y, const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    // all blocks of one monomer on one XCD (block b runs on XCD b % 8): its matrices are fetched once
    const int q = blockIdx.x / kXcds;
    const int part = q % blocks_per_mono;
    const int x = (q / blocks_per_mono) * kXcds + (int)(blockIdx.x % kXcds);
    if (x >= n_mono) return;
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
        // kind 0: two products into one accumulator, the second with -J.  The k
        // chunks of the products run as one sequence with the next chunk's
        // operands in flight (the load past the last chunk repeats the last one
        // instead of being branched around, so waits stay in issue order).
        const int nk = np / 16;
        const int nchunk = (kind == 0 ? 2 : 1) * nk;
        d4 an[kRingSB];
        double bn[kRingSB][4];
        auto load_chunk = [&](int ch) {
            const int pr = ch / nk, k0 = (ch - pr * nk) * 16;
            const double* A = (kind == 0 && pr == 0) ? Kx : Jx;
#pragma unroll
            for (int u = 0; u < kRingSB; ++u) an[u] = load4(A + (int64_t)arow[u] * np + k0 + lk);
            if (kind == 0) {
                const double* B = pr == 0 ? Mx : Tx;
#pragma unroll
                for (int w = 0; w < kRingSB; ++w)
#pragma unroll
                    for (int s = 0; s < 4; ++s) bn[w][s] = B[(int64_t)(k0 + lk + s) * np + bcol[w]];
            } else {
#pragma unroll
                for (int w = 0; w < kRingSB; ++w)
#pragma unroll
                    for (int s = 0; s < 4; ++s) bn[w][s] = Tx[kofs[k0 + lk + s] + ycol[w]];
            }
        };
        load_chunk(0);
        for (int ch = 0; ch < nchunk; ++ch) {
            const double sgn = (kind == 0 && ch >= nk) ? -1.0 : 1.0;
            double a[kRingSB][4], b[kRingSB][4];
#pragma unroll
            for (int u = 0; u < kRingSB; ++u) {
                a[u][0] = sgn * an[u].x;
                a[u][1] = sgn * an[u].y;
                a[u][2] = sgn * an[u].z;
                a[u][3] = sgn * an[u].w;
            }
#pragma unroll
            for (int w = 0; w < kRingSB; ++w)
#pragma unroll
                for (int s = 0; s < 4; ++s) b[w][s] = bn[w][s];
            load_chunk(ch + 1 < nchunk ? ch + 1 : ch);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int u = 0; u < kRingSB; ++u)
#pragma unroll
                    for (int w = 0; w < kRingSB; ++w) acc[u][w] = mfma(a[u][s], b[w][s], acc[u][w]);
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
struct LadderView {
    const double* W;     // packed integral matrix of the monomer (w_rows x ldw)
    const double* Q;     // <kl|ij> as an o^2 x o^2 matrix, rows (k,l), columns (i,j)
    const double* T;
    const double* R12;
    const double* Y;
    double* L;
    const int* kofs;     // W column k = (c,d) -> T offset c ldt + d
    const int* hofs;     // hole pair kk = (k,l) -> T offset k vx ldt + l vy
    int ldw, w_rows, np, o, v, o2, v2;
    int ldt;             // row stride of T: np in global memory, n when staged in LDS
    // the two sides of the amplitudes (rows (i,a): i < o, a < vx; columns (j,b): j < oy, b < vy):
    // a monomer's, o = oy and v = vx = vy; a pair's, X and Y; ldl is the row stride of L
    int oy, vx, vy, ldl;
};

// One wave task: kLadRT row tiles (rows m = (a,b) of W) x CT column tiles
// (columns n = (i,j)).  acc = sum_{(c,d)} W[m][(c,d)] T[(i,c),(j,d)]
//                           + sum_{(k,l)} T[(k,a),(l,b)] <kl|ij>      (P + H)
// then L[(i,a),(j,b)] = acc + R[(i,a),(j,b)] + R[(j,b),(i,a)].
template <int RT, int CT, int PD, bool WITH_R>
__device__ void ladder_task(const LadderView& g, int tr0, int tc0, int lane) {
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    int arow[RT], hrow[RT], bbase[CT], ncol[CT];
#pragma unroll
    for (int u = 0; u < RT; ++u) {
        const int m = (tr0 + u) * 16 + lr;
        arow[u] = m < g.w_rows ? m : 0;
        const int a = m / g.vy, b = m - a * g.vy;
        hrow[u] = m < g.v2 ? a * g.ldt + b : 0;
    }
#pragma unroll
    for (int w = 0; w < CT; ++w) {
        const int n = (tc0 + w) * 16 + lr;
        const int i = n / g.oy, j = n - i * g.oy;
        bbase[w] = n < g.o2 ? i * g.vx * g.ldt + j * g.vy : 0;
        ncol[w] = n;
    }
    d4 acc[RT][CT];
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int w = 0; w < CT; ++w) acc[u][w] = d4(0.0);
    // particle-particle ladder: W streamed once with PD k chunks in flight
    // (pf[q] holds chunk q modulo PD), the gathered amplitude columns of the
    // next chunk in flight.  Loads past the last chunk are redirected to chunk 0
    // (in bounds) and their products multiplied by zero instead of branched
    // around, so the memory counters are waited on in issue order: the gathers
    // of a chunk are issued before the W rows PD chunks ahead, and waiting for
    // them leaves those W loads in flight.  Scheduling barriers keep that order.
    d4 pf[PD][RT];
    double bn[CT][4], b[CT][4];
    const double* wrow[RT];
#pragma unroll
    for (int u = 0; u < RT; ++u) wrow[u] = g.W + (int64_t)arow[u] * g.ldw + lk;
#pragma unroll
    for (int q = 0; q < PD; ++q)
#pragma unroll
        for (int u = 0; u < RT; ++u) pf[q][u] = load4(wrow[u] + (16 * q < g.ldw ? 16 * q : 0));
    auto gather = [&](int k0) {
        const int kb = k0 < g.ldw ? k0 : 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int ko = g.kofs[kb + lk + s];
#pragma unroll
            for (int w = 0; w < CT; ++w) bn[w][s] = g.T[ko + bbase[w]];
        }
    };
    gather(0);
    for (int k0 = 0; k0 < g.ldw; k0 += 16 * PD) {
#pragma unroll
        for (int q = 0; q < PD; ++q) {
            const int kc = k0 + 16 * q;
            const double live = kc < g.ldw ? 1.0 : 0.0;
#pragma unroll
            for (int w = 0; w < CT; ++w)
#pragma unroll
                for (int s = 0; s < 4; ++s) b[w][s] = live * bn[w][s];
            gather(kc + 16);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int u = 0; u < RT; ++u)
#pragma unroll
                    for (int w = 0; w < CT; ++w) acc[u][w] = mfma(pf[q][u][s], b[w][s], acc[u][w]);
            __builtin_amdgcn_sched_barrier(0);
            const int nx = kc + 16 * PD < g.ldw ? kc + 16 * PD : 0;
#pragma unroll
            for (int u = 0; u < RT; ++u) pf[q][u] = load4(wrow[u] + nx);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // hole-hole ladder on the same accumulators: k runs over the o^2 hole pairs (k,l)
    for (int k0 = 0; k0 < g.o2; k0 += 16) {
        double a[RT][4], b[CT][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = k0 + lk + s;
            const bool ok = kk < g.o2;
            const int ho = g.hofs[kk];
#pragma unroll
            for (int u = 0; u < RT; ++u) a[u][s] = g.T[ho + hrow[u]];
#pragma unroll
            for (int w = 0; w < CT; ++w) b[w][s] = (ok && ncol[w] < g.o2) ? g.Q[kk * g.o2 + ncol[w]] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int u = 0; u < RT; ++u)
#pragma unroll
                for (int w = 0; w < CT; ++w) acc[u][w] = mfma(a[u][s], b[w][s], acc[u][w]);
    }
    // epilogue: element (m = (a,b), n = (i,j)) -> L[(i,a),(j,b)]
#pragma unroll
    for (int w = 0; w < CT; ++w) {
        const int n = ncol[w];
        if (n >= g.o2) continue;
        const int i = n / g.oy, j = n - i * g.oy;
#pragma unroll
        for (int u = 0; u < RT; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int m = (tr0 + u) * 16 + acc_row(lane, t);
                if (m >= g.v2) continue;
                const int a = m / g.vy, b = m - a * g.vy;
                const int r = i * g.vx + a, c = j * g.vy + b;
                if (WITH_R) {
                    const double rr = g.R12[(int64_t)r * g.np + c] - g.Y[(int64_t)(i * g.v + b) * g.np + j * g.v + a];
                    const double rt = g.R12[(int64_t)c * g.np + r] - g.Y[(int64_t)(j * g.v + a) * g.np + i * g.v + b];
                    g.L[(int64_t)r * g.np + c] = (acc[u][w][t] + rr) + rt;
                } else {
                    g.L[(int64_t)r * g.ldl + c] = acc[u][w][t];
                }
            }
    }
}

// L += R + R^T with R = R12 - Vs(Y), by v x v block pairs {(i,j), (j,i)}, i <= j:
// the four blocks of R12 and Y of a block pair are read once, row-contiguous,
// and the transposed elements come from LDS (4 v (v + 1) doubles per block
// pair); as many block pairs as fit in lds_doubles go per round, so the loads
// of a round are all in flight together.
__device__ inline void block_pair(int p, int o, int* i, int* j) {
    int r = 0;
    while (p >= o - r) {   // row r of the upper triangle holds o - r pairs
        p -= o - r;
        ++r;
    }
    *i = r;
    *j = r + p;
}

__device__ void add_rings(const LadderView& g, double* sbuf, int lds_doubles) {
    const int o = g.o, v = g.v, np = g.np, vs = v + 1, vv = v * v;
    const int per = 4 * v * vs;
    const int npairs = o * (o + 1) / 2;
    const int cap = lds_doubles / per > 0 ? lds_doubles / per : 1;
    for (int p0 = 0; p0 < npairs; p0 += cap) {
        const int cnt = npairs - p0 < cap ? npairs - p0 : cap;
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * vv; e += blockDim.x) {
            const int q = e / vv, ab = e - q * vv, a = ab / v, b = ab - a * v;
            int i, j;
            block_pair(p0 + q, o, &i, &j);
            double* r0 = sbuf + (int64_t)q * per;   // R12 block (i,j), R12 block (j,i), Y (i,j), Y (j,i)
            const int64_t ij = (int64_t)(i * v + a) * np + j * v + b, ji = (int64_t)(j * v + a) * np + i * v + b;
            r0[a * vs + b] = g.R12[ij];
            r0[v * vs + a * vs + b] = g.R12[ji];
            r0[2 * v * vs + a * vs + b] = g.Y[ij];
            r0[3 * v * vs + a * vs + b] = g.Y[ji];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * vv; e += blockDim.x) {
            const int q = e / vv, ab = e - q * vv, a = ab / v, b = ab - a * v;
            int i, j;
            block_pair(p0 + q, o, &i, &j);
            const double* r0 = sbuf + (int64_t)q * per;
            const double* r1 = r0 + v * vs;
            const double* y0 = r1 + v * vs;
            const double* y1 = y0 + v * vs;
            const int64_t e1 = (int64_t)(i * v + a) * np + j * v + b;
            // (i,a),(j,b): R12[(i,a),(j,b)] - Y[(i,b),(j,a)] + R12[(j,b),(i,a)] - Y[(j,a),(i,b)]
            g.L[e1] += (r0[a * vs + b] - y0[b * vs + a]) + (r1[b * vs + a] - y1[a * vs + b]);
            if (i != j) {
                const int64_t e2 = (int64_t)(j * v + a) * np + i * v + b;
                // (j,a),(i,b): R12[(j,a),(i,b)] - Y[(j,b),(i,a)] + R12[(i,b),(j,a)] - Y[(i,a),(j,b)]
                g.L[e2] += (r1[a * vs + b] - y1[b * vs + a]) + (r0[b * vs + a] - y0[a * vs + b]);
            }
        }
    }
}

// All blocks of one monomer run on one XCD (block b -> XCD b % 8), so the
// monomer's T, R12 and Y are fetched into one L2 once per sweep while its W
// streams through.  Grid: n_mono rounded up to 8, times blocks_per_mono.
template <int CT>
__global__ __launch_bounds__(kLccdThreads, 2) void lccd_ladder_kernel(
    const MonoDesc* __restrict__ monos, const LccdDesc* __restrict__ ld, int n_mono, int blocks_per_mono,
    const double* __restrict__ W, const double* __restrict__ Q, const double* __restrict__ T,
    const double* __restrict__ R12, const double* __restrict__ Y, double* __restrict__ L, int rings,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int q = blockIdx.x / kXcds;
    const int part = q % blocks_per_mono;
    const int x = (q / blocks_per_mono) * kXcds + (int)(blockIdx.x % kXcds);
    if (x >= n_mono) return;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;
    const LccdDesc l = ld[x];
    __shared__ int kofs[kLccdMaxLdw];
    __shared__ int hofs[64];
    const int np = d.np, o = d.o, v = d.v, v2 = v * v, o2 = o * o;
    for (int k = threadIdx.x; k < l.ldw; k += kLccdThreads) {
        const int c = k / v, dd = k - c * v;
        kofs[k] = k < v2 ? c * np + dd : 0;
    }
    for (int k = threadIdx.x; k < 64; k += kLccdThreads) {
        const int kk = k / o, ll = k - kk * o;
        hofs[k] = k < o2 ? kk * v * np + ll * v : 0;
    }
    __syncthreads();
    LadderView g{W + l.w_off, Q + l.q_off, T + d.mat_off, rings ? R12 + d.mat_off : nullptr,
                 rings ? Y + d.mat_off : nullptr, L + d.mat_off, kofs, hofs, l.ldw, l.w_rows, np, o, v, o2, v2, np,
                 o, v, v, np};
    const int nrt = l.w_rows / 16;
    const int ntask_r = (nrt + kLadRT - 1) / kLadRT;
    const int nct = (o2 + 15) / 16;
    const int ngroups = (nct + CT - 1) / CT;
    const int tasks = ntask_r * ngroups;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int task = part * (kLccdThreads / 64) + wave; task < tasks; task += blocks_per_mono * (kLccdThreads / 64)) {
        if (rings) ladder_task<kLadRT, CT, 2, true>(g, (task / ngroups) * kLadRT, (task % ngroups) * CT, lane);
        else ladder_task<kLadRT, CT, 2, false>(g, (task / ngroups) * kLadRT, (task % ngroups) * CT, lane);
    }
}

// The same with the monomer's amplitudes staged in LDS (n x n doubles, row
// stride n; 146 KB at o = 5, v = 27): one workgroup of eight waves per monomer,
// so the B operand gathers and the hole-ladder operands read LDS.  The tasks
// write L = P + H; a final pass over block pairs adds the ring terms with
// row-contiguous reads of R12 and Y (their scattered reads in the task
// epilogues fetched a 128-byte line for every 8 bytes used).
template <int CT>
__global__ __launch_bounds__(kLadLdsThreads) void lccd_ladder_lds_kernel(
    const MonoDesc* __restrict__ monos, const LccdDesc* __restrict__ ld, int lds_doubles,
    const double* __restrict__ W, const double* __restrict__ Q, const double* __restrict__ T,
    const double* __restrict__ R12, const double* __restrict__ Y, double* __restrict__ L, int rings,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int x = blockIdx.x;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;
    const LccdDesc l = ld[x];
    extern __shared__ double lds[];
    const int np = d.np, n = d.n, o = d.o, v = d.v, v2 = v * v, o2 = o * o;
    double* sT = lds;
    int* kofs = reinterpret_cast<int*>(lds + n * n);
    int* hofs = kofs + l.ldw;
    const double* Tx = T + d.mat_off;
    // staging: eight independent loads in flight per thread before the LDS stores
    constexpr int U = 8;
    const int nn = n * n;
    for (int e0 = threadIdx.x; e0 < nn; e0 += U * kLadLdsThreads) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * kLadLdsThreads;
            const int r = e / n, c = e - r * n;
            t[u] = e < nn ? Tx[(int64_t)r * np + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * kLadLdsThreads;
            if (e < nn) sT[e] = t[u];
        }
    }
    for (int k = threadIdx.x; k < l.ldw; k += kLadLdsThreads) {
        const int c = k / v, dd = k - c * v;
        kofs[k] = k < v2 ? c * n + dd : 0;
    }
    for (int k = threadIdx.x; k < 64; k += kLadLdsThreads) {
        const int kk = k / o, ll = k - kk * o;
        hofs[k] = k < o2 ? kk * v * n + ll * v : 0;
    }
    __syncthreads();
    LadderView g{W + l.w_off, Q + l.q_off, sT, rings ? R12 + d.mat_off : nullptr, rings ? Y + d.mat_off : nullptr,
                 L + d.mat_off, kofs, hofs, l.ldw, l.w_rows, np, o, v, o2, v2, n, o, v, v, np};
    constexpr int RT = 2;
    const int nrt = l.w_rows / 16;
    const int ntask_r = (nrt + RT - 1) / RT;
    const int nct = (o2 + 15) / 16;
    const int ngroups = (nct + CT - 1) / CT;
    const int tasks = ntask_r * ngroups;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int task = wave; task < tasks; task += kLadLdsThreads / 64)
        ladder_task<RT, CT, 2, false>(g, (task / ngroups) * RT, (task % ngroups) * CT, lane);
    if (!rings) return;
    // every wave is done with the staged amplitudes and its L stores are visible to the workgroup
    __syncthreads();
    add_rings(g, lds, lds_doubles);
}

// ---------------------------------------------------------------------------
// ring terms of the dimer equation (Eq. 59)
// ---------------------------------------------------------------------------
// One product of a ring task into acc: A rows (k-contiguous, 32-byte loads, row stride lda) times B
// over k < K (a multiple of 16), where BM selects B[k][c] = B[k ldb + c] (0), B[c ldb + k] (1,
// k-contiguous), or the Vs gather B[kofs[k] + ycol[c]] (2).  The next k chunk's operands are in
// flight while the current one is multiplied; the load past the last chunk repeats it instead of
// being branched around.
template <int BM>
__device__ inline void ring_product(d4 (&acc)[kRingSB][kRingSB], const double* A, const double* B, const int* kofs,
                                    const int (&arow)[kRingSB], const int (&bcol)[kRingSB],
                                    const int (&ycol)[kRingSB], int lda, int ldb, int K, int lk) {
    d4 an[kRingSB];
    double bn[kRingSB][4];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kRingSB; ++u) an[u] = load4(A + (int64_t)arow[u] * lda + k0 + lk);
#pragma unroll
        for (int w = 0; w < kRingSB; ++w) {
            if (BM == 1) {
                const d4 t = load4(B + (int64_t)bcol[w] * ldb + k0 + lk);
                bn[w][0] = t.x;
                bn[w][1] = t.y;
                bn[w][2] = t.z;
                bn[w][3] = t.w;
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = k0 + lk + s;
                    bn[w][s] = BM == 0 ? B[(int64_t)k * ldb + bcol[w]] : B[kofs[k] + ycol[w]];
                }
            }
        }
    };
    load_chunk(0);
    for (int k0 = 0; k0 < K; k0 += 16) {
        double a[kRingSB][4], b[kRingSB][4];
#pragma unroll
        for (int u = 0; u < kRingSB; ++u) {
            a[u][0] = an[u].x;
            a[u][1] = an[u].y;
            a[u][2] = an[u].z;
            a[u][3] = an[u].w;
        }
#pragma unroll
        for (int w = 0; w < kRingSB; ++w)
#pragma unroll
            for (int s = 0; s < 4; ++s) b[w][s] = bn[w][s];
        load_chunk(k0 + 16 < K ? k0 + 16 : k0);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int u = 0; u < kRingSB; ++u)
#pragma unroll
                for (int w = 0; w < kRingSB; ++w) acc[u][w] = mfma(a[u][s], b[w][s], acc[u][w]);
    }
}

// For a pair with amplitudes Tau (npx x npy, rows (i,a) of X, columns (j,b) of Y) the
// monomer rings are (2 K_X - J_X) Tau + Tau (2 K_Y - J_Y)^T, two products into one
// accumulator added in place into the pair's source S (which holds the two ladders, stored
// before this launch; every element of S has one owner task); the cross rings are
// Y1 = C_X-hat Vs(Tau) (rows (i,b), columns (j,a)) and Y2 = C_Y-hat Vs(Tau^T) (rows (j,a),
// columns (i,b)), stored as they come out, and the pair kernel subtracts Y1[(i,b),(j,a)] and
// Y2[(j,a),(i,b)] when it forms Tau.  K-hat[(i,a),(i1,a1)] = K[i,i1,a,a1] and
// J-hat[(i,a),(i1,a1)] = J[i1,i,a,a1] of the monomer (2 K-hat - J-hat formed once per monomer
// at attach), C_X-hat[(i,b),(i1,b1)] = C_X[i1][i][b][b1], C_Y-hat[(j,a),(j1,a1)] =
// C_Y[j1][j][a][a1], Vs the swap of the two virtual indices.  Tasks are 3 x 3 super-blocks of
// 16 x 16 tiles of the three outputs; all blocks of a pair run on one XCD.
__host__ __device__ inline int ring_nsb(int rows) { return (rows / 16 + kRingSB - 1) / kRingSB; }

__global__ __launch_bounds__(kLccdThreads, 2) void dimer_ring_kernel(
    const DimerDesc* __restrict__ dd, const MonoDesc* __restrict__ monos, int n_pair, int blocks_per_pair,
    const double* __restrict__ RM, const double* __restrict__ CX, const double* __restrict__ CY,
    const double* __restrict__ Tau, double* __restrict__ S, double* __restrict__ Y1, double* __restrict__ Y2,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int q = blockIdx.x / kXcds;
    const int part = q % blocks_per_pair;
    const int p = (q / blocks_per_pair) * kXcds + (int)(blockIdx.x % kXcds);
    if (p >= n_pair) return;
    const DimerDesc e = dd[p];
    if (cl && cl[e.cluster].done) return;
    __shared__ int kofs[2][kLccdMaxNp];   // Vs gathers: row k of Vs(Tau) / Vs(Tau^T)
    const int npx = e.npx, npy = e.npy, vx = e.vx, vy = e.vy;
    const int n1 = e.ox * vy, n2 = e.oy * vx;   // rows (i,b) of Y1, rows (j,a) of Y2
    for (int k = threadIdx.x; k < e.m1; k += kLccdThreads) {   // Vs(Tau) row (i1,b1)
        const int i1 = k / vy, b1 = k - i1 * vy;
        kofs[0][k] = k < n1 ? i1 * vx * npy + b1 : 0;
    }
    for (int k = threadIdx.x; k < e.m2; k += kLccdThreads) {   // Vs(Tau^T) row (j1,a1)
        const int j1 = k / vx, a1 = k - j1 * vx;
        kofs[1][k] = k < n2 ? a1 * npy + j1 * vy : 0;
    }
    __syncthreads();
    const double* Tp = Tau + e.tau_off;
    const double* RX = RM + monos[e.x].mat_off;
    const double* RY = RM + monos[e.y].mat_off;
    const int s0c = ring_nsb(npy), s1c = ring_nsb(e.m2), s2c = ring_nsb(e.m1);
    const int t0 = ring_nsb(npx) * s0c, t1 = ring_nsb(e.m1) * s1c, t2 = ring_nsb(e.m2) * s2c;
    const int tasks = t0 + t1 + t2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    for (int task = part * (kLccdThreads / 64) + wave; task < tasks; task += blocks_per_pair * (kLccdThreads / 64)) {
        // kind 0: monomer rings into S; 1: C_X-hat Vs(Tau) into Y1; 2: C_Y-hat Vs(Tau^T) into Y2
        const int kind = task < t0 ? 0 : task < t0 + t1 ? 1 : 2;
        const int sb = task - (kind == 0 ? 0 : kind == 1 ? t0 : t0 + t1);
        const int nsc = kind == 0 ? s0c : kind == 1 ? s1c : s2c;
        const int tr0 = (sb / nsc) * kRingSB, tc0 = (sb % nsc) * kRingSB;
        const int rows = kind == 0 ? npx : kind == 1 ? e.m1 : e.m2;     // padded extents of the output
        const int cols = kind == 0 ? npy : kind == 1 ? e.m2 : e.m1;
        const int nr = kind == 0 ? e.nx : kind == 1 ? n1 : n2;           // valid extents
        const int nc = kind == 0 ? e.ny : kind == 1 ? n2 : n1;
        int arow[kRingSB], bcol[kRingSB], ycol[kRingSB];
#pragma unroll
        for (int u = 0; u < kRingSB; ++u) {
            const int r = (tr0 + u) * 16 + lr, c = (tc0 + u) * 16 + lr;
            arow[u] = r < rows ? r : 0;
            bcol[u] = c < cols ? c : 0;
            if (kind == 1) {   // Vs(Tau) column (j,a)
                const int j = c / vx, a = c - j * vx;
                ycol[u] = c < n2 ? a * npy + j * vy : 0;
            } else {           // Vs(Tau^T) column (i,b)
                const int i = c / vy, b = c - i * vy;
                ycol[u] = c < n1 ? i * vx * npy + b : 0;
            }
        }
        d4 acc[kRingSB][kRingSB];
#pragma unroll
        for (int u = 0; u < kRingSB; ++u)
#pragma unroll
            for (int w = 0; w < kRingSB; ++w) acc[u][w] = d4(0.0);
        if (kind == 0) {   // (2K - J)_X Tau + Tau (2K - J)_Y^T on one accumulator
            ring_product<0>(acc, RX, Tp, nullptr, arow, bcol, ycol, npx, npy, npx, lk);
            ring_product<1>(acc, Tp, RY, nullptr, arow, bcol, ycol, npy, npy, npy, lk);
        } else if (kind == 1) {
            ring_product<2>(acc, CX + e.cx_off, Tp, kofs[0], arow, bcol, ycol, e.m1, 0, e.m1, lk);
        } else {
            ring_product<2>(acc, CY + e.cy_off, Tp, kofs[1], arow, bcol, ycol, e.m2, 0, e.m2, lk);
        }
        double* out = kind == 0 ? S + e.tau_off : kind == 1 ? Y1 + e.y1_off : Y2 + e.y2_off;
#pragma unroll
        for (int u = 0; u < kRingSB; ++u)
#pragma unroll
            for (int w = 0; w < kRingSB; ++w) {
                const int c = (tc0 + w) * 16 + lr;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int r = (tr0 + u) * 16 + acc_row(lane, t);
                    if (r >= nr || c >= nc) continue;
                    if (kind == 0) out[(int64_t)r * cols + c] += acc[u][w][t];
                    else out[(int64_t)r * cols + c] = acc[u][w][t];
                }
            }
    }
}

// The pair ladders from global memory for pairs of any two monomer sizes: the monomer
// ladder task on a pair's Tau (rows (i,a) of X, columns (j,b) of Y, row stride npy) with
// its W_XY (rows (a,b), columns (a1,b1)) and Q_XY (rows (i1,j1), columns (i,j)); S = P + H.
template <int CT>
__global__ __launch_bounds__(kLccdThreads, 2) void dimer_ladder_kernel(
    const DimerDesc* __restrict__ dd, int n_pair, int blocks_per_pair, const double* __restrict__ W,
    const double* __restrict__ Q, const double* __restrict__ Tau, double* __restrict__ S,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    const int q = blockIdx.x / kXcds;
    const int part = q % blocks_per_pair;
    const int p = (q / blocks_per_pair) * kXcds + (int)(blockIdx.x % kXcds);
    if (p >= n_pair) return;
    const DimerDesc e = dd[p];
    if (cl && cl[e.cluster].done) return;
    __shared__ int kofs[kLccdMaxLdw];
    __shared__ int hofs[64];
    const int vx = e.vx, vy = e.vy, oy = e.oy, v2 = vx * vy, o2 = e.ox * oy, ldt = e.npy;
    for (int k = threadIdx.x; k < e.ldw; k += kLccdThreads) {   // W column (a1,b1)
        const int c = k / vy, d = k - c * vy;
        kofs[k] = k < v2 ? c * ldt + d : 0;
    }
    for (int k = threadIdx.x; k < 64; k += kLccdThreads) {       // hole pair (k,l)
        const int kk = k / oy, ll = k - kk * oy;
        hofs[k] = k < o2 ? kk * vx * ldt + ll * vy : 0;
    }
    __syncthreads();
    LadderView g{W + e.w_off, Q + e.q_off, Tau + e.tau_off, nullptr, nullptr, S + e.tau_off, kofs, hofs, e.ldw,
                 e.w_rows, e.npx, e.ox, vx, o2, v2, ldt, oy, vx, vy, ldt};
    const int nrt = e.w_rows / 16;
    const int ntask_r = (nrt + kLadRT - 1) / kLadRT;
    const int nct = (o2 + 15) / 16;
    const int ngroups = (nct + CT - 1) / CT;
    const int tasks = ntask_r * ngroups;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int task = part * (kLccdThreads / 64) + wave; task < tasks; task += blocks_per_pair * (kLccdThreads / 64))
        ladder_task<kLadRT, CT, 2, false>(g, (task / ngroups) * kLadRT, (task % ngroups) * CT, lane);
}

// W_XY, C_X-hat and C_Y-hat of every pair from the caller's concatenated classes
__global__ void dimer_pack_kernel(const DimerDesc* __restrict__ dd, const double* __restrict__ w_raw,
                                  const double* __restrict__ cx_raw, const double* __restrict__ cy_raw,
                                  double* __restrict__ W, double* __restrict__ CX, double* __restrict__ CY) {
    const DimerDesc e = dd[blockIdx.y];
    const int64_t step = (int64_t)gridDim.x * blockDim.x, first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v2 = e.vx * e.vy;
    if (w_raw)
        for (int64_t k = first; k < (int64_t)e.w_rows * e.ldw; k += step) {
            const int r = (int)(k / e.ldw), c = (int)(k - (int64_t)r * e.ldw);
            W[e.w_off + k] = (r < v2 && c < v2) ? w_raw[e.w_raw_off + (int64_t)r * v2 + c] : 0.0;
        }
    if (cx_raw) {   // C_X-hat[(i,b),(i1,b1)] = C_X[i1][i][b][b1], rows and columns over (ox, vy)
        const int n1 = e.ox * e.vy;
        for (int64_t k = first; k < (int64_t)e.m1 * e.m1; k += step) {
            const int r = (int)(k / e.m1), c = (int)(k - (int64_t)r * e.m1);
            double val = 0.0;
            if (r < n1 && c < n1) {
                const int i = r / e.vy, b = r - i * e.vy, i1 = c / e.vy, b1 = c - i1 * e.vy;
                val = cx_raw[e.cx_raw_off + (((int64_t)i1 * e.ox + i) * e.vy + b) * e.vy + b1];
            }
            CX[e.cx_off + k] = val;
        }
    }
    if (cy_raw) {   // C_Y-hat[(j,a),(j1,a1)] = C_Y[j1][j][a][a1], rows and columns over (oy, vx)
        const int n2 = e.oy * e.vx;
        for (int64_t k = first; k < (int64_t)e.m2 * e.m2; k += step) {
            const int r = (int)(k / e.m2), c = (int)(k - (int64_t)r * e.m2);
            double val = 0.0;
            if (r < n2 && c < n2) {
                const int j = r / e.vx, a = r - j * e.vx, j1 = c / e.vx, a1 = c - j1 * e.vx;
                val = cy_raw[e.cy_raw_off + (((int64_t)j1 * e.oy + j) * e.vx + a) * e.vx + a1];
            }
            CY[e.cy_off + k] = val;
        }
    }
}

// RM = 2 K - J over a buffer of monomer matrices (the ring matrix of the monomer rings of Eq. 59)
__global__ void ring_matrix_kernel(const double* __restrict__ K, const double* __restrict__ J, double* __restrict__ RM,
                                   int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        RM[e] = 2.0 * K[e] - J[e];
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

int lccd_ladder_ct(int max_o) {
    const int nct = (max_o * max_o + 15) / 16;
    return nct < kLadCT ? nct : kLadCT;
}

int lccd_ladder_blocks(int max_w_rows, int max_o) {
    const int nrt = max_w_rows / 16, ntr = (nrt + kLadRT - 1) / kLadRT;
    const int nct = (max_o * max_o + 15) / 16, ct = lccd_ladder_ct(max_o), ng = (nct + ct - 1) / ct;
    const int tasks = ntr * ng, per_block = kLccdThreads / 64;
    const int b = (tasks + per_block - 1) / per_block;
    return b < 64 ? b : 64;
}

void launch_lccd_ring(const MonoDesc* monos, int n_mono, int ring_blocks, const double* K, const double* J,
                      const double* T, const double* M, double* R12, double* Y, const Ctrl* ctrl, const ClState* cl,
                      hipStream_t s) {
    if (n_mono <= 0 || ring_blocks <= 0) return;
    const int groups = (n_mono + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(lccd_ring_kernel, dim3(groups * kXcds * ring_blocks), dim3(kLccdThreads), 0, s, monos, n_mono,
                       ring_blocks, K, J, T, M, R12, Y, ctrl, cl);
}

int64_t lccd_ladder_lds_bytes(int n, int v, int ldw) {
    const int64_t stage = (int64_t)n * n * 8 + (int64_t)(ldw + 64) * 4;
    const int64_t rings = (int64_t)4 * v * (v + 1) * 8;
    return stage > rings ? stage : rings;
}

int64_t lccd_lds_limit() { return 160 * 1024; }

void launch_lccd_ladder(const MonoDesc* monos, const LccdDesc* ld, int n_mono, int ladder_blocks, int ct,
                        int64_t lds_bytes, const double* W, const double* Q, const double* T, const double* R12,
                        const double* Y, double* L, const Ctrl* ctrl, const ClState* cl, hipStream_t s, int rings) {
    if (n_mono <= 0 || ladder_blocks <= 0) return;
    if (lds_bytes > 0) {
        const dim3 grid(n_mono), block(kLadLdsThreads);
        switch (ct) {
#define LDS_CASE(C)                                                                                              \
    case C: {                                                                                                    \
        static bool attr = false;                                                                                \
        if (!attr) {                                                                                             \
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lccd_ladder_lds_kernel<C>),                 \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lccd_lds_limit());         \
            attr = true;                                                                                         \
        }                                                                                                        \
        hipLaunchKernelGGL(lccd_ladder_lds_kernel<C>, grid, block, (size_t)lds_bytes, s, monos, ld,            \
                           (int)(lds_bytes / 8), W, Q, T, R12, Y, L, rings, ctrl, cl);                           \
        return;                                                                                                  \
    }
            LDS_CASE(1)
            LDS_CASE(2)
            LDS_CASE(3)
            default:
                break;
#undef LDS_CASE
        }
    }
    const dim3 grid(((n_mono + kXcds - 1) / kXcds) * kXcds * ladder_blocks), block(kLccdThreads);
    switch (ct) {
        case 1:
            hipLaunchKernelGGL(lccd_ladder_kernel<1>, grid, block, 0, s, monos, ld, n_mono, ladder_blocks, W, Q, T,
                               R12, Y, L, rings, ctrl, cl);
            break;
        case 2:
            hipLaunchKernelGGL(lccd_ladder_kernel<2>, grid, block, 0, s, monos, ld, n_mono, ladder_blocks, W, Q, T,
                               R12, Y, L, rings, ctrl, cl);
            break;
        case 3:
            hipLaunchKernelGGL(lccd_ladder_kernel<3>, grid, block, 0, s, monos, ld, n_mono, ladder_blocks, W, Q, T,
                               R12, Y, L, rings, ctrl, cl);
            break;
        default:
            hipLaunchKernelGGL(lccd_ladder_kernel<4>, grid, block, 0, s, monos, ld, n_mono, ladder_blocks, W, Q, T,
                               R12, Y, L, rings, ctrl, cl);
            break;
    }
}

int dimer_ring_tasks(const DimerDesc& d) {
    return ring_nsb(d.npx) * ring_nsb(d.npy) + ring_nsb(d.m1) * ring_nsb(d.m2) + ring_nsb(d.m2) * ring_nsb(d.m1);
}

int dimer_ring_blocks(int max_tasks) {
    const int per_block = kLccdThreads / 64;
    const int b = (max_tasks + per_block - 1) / per_block;
    return b < 64 ? (b > 0 ? b : 1) : 64;
}

void launch_dimer_ring(const DimerDesc* dd, const MonoDesc* monos, int n_pair, int blocks, const double* RM,
                       const double* CX, const double* CY, const double* Tau, double* S, double* Y1, double* Y2,
                       const Ctrl* ctrl, const ClState* cl, hipStream_t s) {
    if (n_pair <= 0 || blocks <= 0) return;
    const dim3 grid(((n_pair + kXcds - 1) / kXcds) * kXcds * blocks), block(kLccdThreads);
    hipLaunchKernelGGL(dimer_ring_kernel, grid, block, 0, s, dd, monos, n_pair, blocks, RM, CX, CY, Tau, S, Y1, Y2,
                       ctrl, cl);
}

void launch_dimer_pack(const DimerDesc* dd, int n_pair, const double* w_raw, const double* cx_raw,
                       const double* cy_raw, double* W, double* CX, double* CY, hipStream_t s) {
    if (n_pair <= 0) return;
    hipLaunchKernelGGL(dimer_pack_kernel, dim3(64, n_pair), dim3(256), 0, s, dd, w_raw, cx_raw, cy_raw, W, CX, CY);
}

int dimer_ladder_ct(int max_o2) {
    const int nct = (max_o2 + 15) / 16;
    return nct < kLadCT ? nct : kLadCT;
}

int dimer_ladder_blocks(int max_w_rows, int max_o2) {
    const int nrt = max_w_rows / 16, ntr = (nrt + kLadRT - 1) / kLadRT;
    const int nct = (max_o2 + 15) / 16, ct = dimer_ladder_ct(max_o2), ng = (nct + ct - 1) / ct;
    const int tasks = ntr * ng, per_block = kLccdThreads / 64;
    const int b = (tasks + per_block - 1) / per_block;
    return b < 64 ? (b > 0 ? b : 1) : 64;
}

void launch_dimer_ladder(const DimerDesc* dd, int n_pair, int blocks_per_pair, int ct, const double* W,
                         const double* Q, const double* Tau, double* S, const Ctrl* ctrl, const ClState* cl,
                         hipStream_t s) {
    if (n_pair <= 0 || blocks_per_pair <= 0) return;
    const dim3 grid(((n_pair + kXcds - 1) / kXcds) * kXcds * blocks_per_pair), block(kLccdThreads);
    switch (ct) {
        case 1:
            hipLaunchKernelGGL(dimer_ladder_kernel<1>, grid, block, 0, s, dd, n_pair, blocks_per_pair, W, Q, Tau, S,
                               ctrl, cl);
            break;
        case 2:
            hipLaunchKernelGGL(dimer_ladder_kernel<2>, grid, block, 0, s, dd, n_pair, blocks_per_pair, W, Q, Tau, S,
                               ctrl, cl);
            break;
        case 3:
            hipLaunchKernelGGL(dimer_ladder_kernel<3>, grid, block, 0, s, dd, n_pair, blocks_per_pair, W, Q, Tau, S,
                               ctrl, cl);
            break;
        default:
            hipLaunchKernelGGL(dimer_ladder_kernel<4>, grid, block, 0, s, dd, n_pair, blocks_per_pair, W, Q, Tau, S,
                               ctrl, cl);
            break;
    }
}

void launch_ring_matrix(const double* K, const double* J, double* RM, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(ring_matrix_kernel, dim3(1024), dim3(256), 0, s, K, J, RM, n);
}

}  // namespace mcpt
