// Singles sweep of MCPT(2) (Eq. 57, program-flow step 4) on the resident dimer
// blocks.
//
// With the terms the inputs can form, one Jacobi sweep is
//
//   u_X = sum over neighbours Y of v^{ak}_{ic} t^c_k = sum_Y V_XY t_Y
//   t_X <- (w_X + u_X) / (e_i - e_a)                      (eps^i_a of Eq. 57)
//   E_M1(X) = 2 w^i_a t^a_i                               (Eq. 53)
//
// where v^{ak}_{ic} = (ai|ck) = V_XY[(i,a),(k,c)] is the Coulomb block the
// doubles use; each stored pair feeds both of its monomers, u_X += V_XY t_Y and
// u_Y += V_XY^T t_X.  The pair phase is two matrix-vector products per block:
// 4 flops per 8-byte element, so it is bound by streaming V from HBM once per
// sweep (6.1 GB at 1000 monomers) and the kernel is built for that: every V
// element is read exactly once, by coalesced 8-byte loads (a wave reads 64
// consecutive elements of one row), with four rows times up to four 64-column
// chunks in flight per wave and several workgroups per CU.  A wave owns rows
// r = wave (mod 4): its lanes sum V[r][c] t_Y[c] over their columns and a wave
// reduction gives the row's share of u_X; the same loads add V[r][c] t_X[r]
// into per-lane column sums, combined over the waves in LDS, for u_Y.  Partial
// sums reach u by FP64 atomics, one per row and column per pair.
//
// Vectors t, u and w use the padded per-monomer layout of the energy
// differences (dif_off, element (i,a) = i v + a), so the denominator of element
// e is 1 / dif[e].
#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

constexpr int kSThreads = 256;               // four waves
constexpr int kSWaves = kSThreads / 64;
constexpr int kColChunks = 4;                // 64-column chunks per lane per pass: 256 columns
constexpr int kRowUnroll = 4;                // rows of one wave in flight together
constexpr int kMonoThreadsS = 256;
static_assert(kColChunks * 64 == kSThreads, "one column-sum slot per thread");

__device__ inline double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ inline double max_nan(double a, double b) { return (a != a || b != b) ? NAN : (a > b ? a : b); }

template <int NT>
__device__ double block_reduce(double x, double* sh, bool is_max) {
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            sh[threadIdx.x] = is_max ? max_nan(sh[threadIdx.x], sh[threadIdx.x + s]) : sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// u_X += V_XY t_Y and u_Y += V_XY^T t_X for every stored pair of a live cluster.
// Dynamic LDS: max_n doubles for the row sums of the current pair.
__global__ __launch_bounds__(kSThreads) void singles_pair_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ V, const double* __restrict__ t, double* __restrict__ u,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    extern __shared__ double s_rows[];
    __shared__ double s_cols[kColChunks * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t pi = blockIdx.x; pi < n_pair; pi += gridDim.x) {
        const PairDesc pd = pairs[pi];
        if (cl && cl[pd.cluster].done) continue;   // uniform over the workgroup
        const MonoDesc dx = monos[pd.x], dy = monos[pd.y];
        const int nX = dx.n, nY = dy.n;
        const double* v = V + pd.v_off;
        const double* tX = t + dx.dif_off;
        const double* tY = t + dy.dif_off;
        for (int r = threadIdx.x; r < nX; r += kSThreads) s_rows[r] = 0.0;
        s_cols[threadIdx.x] = 0.0;   // kColChunks * 64 == kSThreads
        __syncthreads();
        for (int c0 = 0; c0 < nY; c0 += 64 * kColChunks) {
            double ty[kColChunks], cy[kColChunks];
#pragma unroll
            for (int k = 0; k < kColChunks; ++k) {
                const int c = c0 + 64 * k + lane;
                ty[k] = c < nY ? tY[c] : 0.0;
                cy[k] = 0.0;
            }
            for (int r0 = wave; r0 < nX; r0 += kSWaves * kRowUnroll) {
                double vv[kRowUnroll][kColChunks], tx[kRowUnroll];
#pragma unroll
                for (int j = 0; j < kRowUnroll; ++j) {
                    const int r = r0 + j * kSWaves;
                    tx[j] = r < nX ? tX[r] : 0.0;
#pragma unroll
                    for (int k = 0; k < kColChunks; ++k) {
                        const int c = c0 + 64 * k + lane;
                        vv[j][k] = (r < nX && c < nY) ? v[(int64_t)r * nY + c] : 0.0;
                    }
                }
#pragma unroll
                for (int j = 0; j < kRowUnroll; ++j) {
                    double p = 0.0;
#pragma unroll
                    for (int k = 0; k < kColChunks; ++k) {
                        p = fma(vv[j][k], ty[k], p);
                        cy[k] = fma(vv[j][k], tx[j], cy[k]);
                    }
                    p = wave_sum(p);
                    const int r = r0 + j * kSWaves;
                    if (lane == 0 && r < nX) s_rows[r] += p;   // row r belongs to this wave only
                }
            }
#pragma unroll
            for (int k = 0; k < kColChunks; ++k)
                if (c0 + 64 * k + lane < nY) atomicAdd(&s_cols[64 * k + lane], cy[k]);
            __syncthreads();
            {
                const int c = c0 + threadIdx.x;
                if (c < nY) unsafeAtomicAdd(u + dy.dif_off + c, s_cols[threadIdx.x]);
                s_cols[threadIdx.x] = 0.0;
            }
            __syncthreads();
        }
        for (int r = threadIdx.x; r < nX; r += kSThreads) unsafeAtomicAdd(u + dx.dif_off + r, s_rows[r]);
        __syncthreads();   // s_rows is reset for the next pair
    }
}

// init: t = w / d (first order), E_M1 into em1 and em1_0.
// update: t' = (w + u) / d, residual max|t' - t|, E_M1(t'), u cleared for the next sweep.
__global__ __launch_bounds__(kMonoThreadsS) void singles_mono_kernel(
    int init, const MonoDesc* __restrict__ monos, const double* __restrict__ dif, const double* __restrict__ w,
    double* __restrict__ u, double* __restrict__ t, double* __restrict__ em1, double* __restrict__ em1_0,
    double* __restrict__ res, const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    __shared__ double sh[kMonoThreadsS];
    const int x = blockIdx.x;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;
    const double* dx = dif + d.dif_off;
    const double* wx = w + d.dif_off;
    double* ux = u + d.dif_off;
    double* tx = t + d.dif_off;
    double e = 0.0, rmax = 0.0;
    for (int k = threadIdx.x; k < d.n; k += kMonoThreadsS) {
        const double di = recip(dx[k]);
        if (init) {
            const double tn = di * wx[k];
            tx[k] = tn;
            e += wx[k] * tn;
        } else {
            const double tn = di * (wx[k] + ux[k]);
            rmax = max_nan(rmax, fabs(tn - tx[k]));
            tx[k] = tn;
            ux[k] = 0.0;
            e += wx[k] * tn;
        }
    }
    e = block_reduce<kMonoThreadsS>(e, sh, false);
    rmax = block_reduce<kMonoThreadsS>(rmax, sh, true);
    if (threadIdx.x == 0) {
        em1[x] = 2.0 * e;
        if (init) em1_0[x] = 2.0 * e;
        else res[x] = rmax;
    }
}

// Per-cluster sums of E_M1 and of its first-order value (into e_mono, e_mono0).
__global__ __launch_bounds__(kMonoThreadsS) void singles_cluster_kernel(const int64_t* __restrict__ cl_mono,
                                                                        const double* __restrict__ em1,
                                                                        const double* __restrict__ em1_0,
                                                                        ClState* __restrict__ cl) {
    __shared__ double sh[kMonoThreadsS];
    const int q = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = cl_mono[q] + threadIdx.x; i < cl_mono[q + 1]; i += kMonoThreadsS) {
        a += em1[i];
        b += em1_0[i];
    }
    a = block_reduce<kMonoThreadsS>(a, sh, false);
    b = block_reduce<kMonoThreadsS>(b, sh, false);
    if (threadIdx.x == 0) {
        cl[q].e_mono = a;
        cl[q].e_mono0 = b;
    }
}

// compact w (monomers concatenated, n values each, starting at woff[x]) into the padded layout
__global__ __launch_bounds__(kMonoThreadsS) void singles_scatter_kernel(const MonoDesc* __restrict__ monos,
                                                                        const int64_t* __restrict__ woff,
                                                                        const double* __restrict__ compact,
                                                                        double* __restrict__ padded) {
    const MonoDesc d = monos[blockIdx.x];
    const double* src = compact + woff[blockIdx.x];
    double* dst = padded + d.dif_off;
    for (int k = threadIdx.x; k < d.np; k += kMonoThreadsS) dst[k] = k < d.n ? src[k] : 0.0;
}

}  // namespace

int64_t singles_lds_bytes(int max_n) { return (int64_t)max_n * (int64_t)sizeof(double); }

int singles_pair_grid(int n_cu, int max_n) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, singles_pair_kernel, kSThreads,
                                                     (size_t)singles_lds_bytes(max_n)) != hipSuccess ||
        per < 1)
        per = 1;
    per = per > 8 ? 8 : per;
    return n_cu * per;
}

void launch_singles_pair(const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos, const double* V,
                         const double* t, double* u, int max_n, int grid, const Ctrl* ctrl, const ClState* cl,
                         hipStream_t s) {
    if (n_pair <= 0) return;
    hipLaunchKernelGGL(singles_pair_kernel, dim3(grid), dim3(kSThreads), (size_t)singles_lds_bytes(max_n), s, pairs,
                       n_pair, monos, V, t, u, ctrl, cl);
}

void launch_singles_mono(int init, const MonoDesc* monos, int n_mono, const double* dif, const double* w, double* u,
                         double* t, double* em1, double* em1_0, double* res, const Ctrl* ctrl, const ClState* cl,
                         hipStream_t s) {
    if (n_mono <= 0) return;
    hipLaunchKernelGGL(singles_mono_kernel, dim3(n_mono), dim3(kMonoThreadsS), 0, s, init, monos, dif, w, u, t, em1,
                       em1_0, res, ctrl, cl);
}

void launch_singles_clusters(int n_cl, const int64_t* cl_mono, const double* em1, const double* em1_0, ClState* cl,
                             hipStream_t s) {
    hipLaunchKernelGGL(singles_cluster_kernel, dim3(n_cl), dim3(kMonoThreadsS), 0, s, cl_mono, em1, em1_0, cl);
}

void launch_singles_scatter(const MonoDesc* monos, int n_mono, const int64_t* woff, const double* compact,
                            double* padded, hipStream_t s) {
    if (n_mono <= 0) return;
    hipLaunchKernelGGL(singles_scatter_kernel, dim3(n_mono), dim3(kMonoThreadsS), 0, s, monos, woff, compact, padded);
}

}  // namespace mcpt
