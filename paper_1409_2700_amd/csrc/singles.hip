// Singles sweep of MCPT(2) (Eq. 57, program-flow step 4) on the resident dimer
// blocks.
//
// With the terms the inputs can form, one Jacobi sweep is
//
//   u_X = sum over neighbours Y of v^{ak}_{ic} t^c_k = sum_Y V_XY t_Y
//   t_X <- (w_X + 2 u_X) / (e_i - e_a)                    (eps^i_a of Eq. 57)
//
// (the 2 sums k, c of Y over both spins)
//   E_M1(X) = 2 w^i_a t^a_i                               (Eq. 53)
//
// where v^{ak}_{ic} = (ai|ck) = V_XY[(i,a),(k,c)] is the Coulomb block the
// doubles use; each stored pair feeds both of its monomers, u_X += V_XY t_Y and
// u_Y += V_XY^T t_X.  The pair phase is two matrix-vector products per block:
// 4 flops per 8-byte element, so it is bound by streaming V from HBM once per
// sweep (6.1 GB at 1000 monomers) and the kernel is built for that.  Each wave
// owns a pair (no barriers, no LDS): its four 16-lane groups read four rows at
// a time, a lane taking columns l, l + 16, ... (each group reads 128
// consecutive bytes of its row per load: four row segments per load
// instruction), with four such row quadruples - thirty-six loads of a 144-column
// pass - in flight per wave.  A row's sum V[r][:] t_Y is finished by a
// 16-lane shuffle reduction (four steps for four rows at once); the same loads
// add V[r][c] t_X[r] into per-lane column sums, combined over the four groups
// once per pair.  Sums reach u by FP64 atomics: one per row and column per pair
// (and per 144-column pass for wider monomers).
//
// Vectors t, u and w use the padded per-monomer layout of the energy
// differences (dif_off, element (i,a) = i v + a), so the denominator of element
// e is 1 / dif[e].
#include "singles.hpp"

namespace mcpt {

namespace {

constexpr int kSThreads = 256;               // four waves, each on its own pair
constexpr int kSWaves = kSThreads / 64;
constexpr int kSlots = 9;                    // 16-column chunks per lane per pass: 144 columns
constexpr int kRowIters = 4;                 // four-row groups of one wave in flight together
constexpr int kMonoThreadsS = 256;

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

// u_X += V_XY t_Y and u_Y += V_XY^T t_X for every stored pair of a live cluster,
// one pair per wave.
__global__ __launch_bounds__(kSThreads) void singles_pair_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ V, const double* __restrict__ t, double* __restrict__ u,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    // the wave index is uniform over the wave: with it in a scalar register the pair and
    // monomer descriptors are scalar loads and every V address is a scalar base + lane offset
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, l = lane & 15;
    const int64_t stride = (int64_t)gridDim.x * kSWaves;
    for (int64_t pi = (int64_t)blockIdx.x * kSWaves + wave; pi < n_pair; pi += stride) {
        const PairDesc pd = pairs[pi];
        if (cl && cl[pd.cluster].done) continue;   // uniform over the wave
        const MonoDesc dx = monos[pd.x], dy = monos[pd.y];
        const int nX = dx.n, nY = dy.n;
        const double* v = V + pd.v_off;
        const double* tX = t + dx.dif_off;
        const double* tY = t + dy.dif_off;
        double* uX = u + dx.dif_off;
        double* uY = u + dy.dif_off;
        for (int c0 = 0; c0 < nY; c0 += 16 * kSlots) {
            double ty[kSlots], cy[kSlots];
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                const int c = c0 + 16 * k + l;
                ty[k] = c < nY ? tY[c] : 0.0;
                cy[k] = 0.0;
            }
            for (int r0 = 0; r0 < nX; r0 += 4 * kRowIters) {
                double vv[kRowIters][kSlots], tx[kRowIters];
#pragma unroll
                for (int i = 0; i < kRowIters; ++i) {
                    const int r = r0 + 4 * i + g;
                    tx[i] = r < nX ? tX[r] : 0.0;
#pragma unroll
                    for (int k = 0; k < kSlots; ++k) {
                        const int c = c0 + 16 * k + l;
                        // 32-bit element offset (a block holds far fewer than 2^29 values): scalar base + lane offset
                        vv[i][k] = (r < nX && c < nY) ? __builtin_nontemporal_load(v + (unsigned)(r * nY + c)) : 0.0;
                    }
                }
#pragma unroll
                for (int i = 0; i < kRowIters; ++i) {
                    double p = 0.0;
#pragma unroll
                    for (int k = 0; k < kSlots; ++k) {
                        p = fma(vv[i][k], ty[k], p);
                        cy[k] = fma(vv[i][k], tx[i], cy[k]);
                    }
                    // sum over the 16 lanes of the group (xor masks below 16 stay inside it)
                    p += __shfl_xor(p, 8, 64);
                    p += __shfl_xor(p, 4, 64);
                    p += __shfl_xor(p, 2, 64);
                    p += __shfl_xor(p, 1, 64);
                    const int r = r0 + 4 * i + g;
                    if (l == 0 && r < nX) unsafeAtomicAdd(uX + r, p);
                }
            }
            // column sums over the four row groups
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                cy[k] += __shfl_xor(cy[k], 16, 64);
                cy[k] += __shfl_xor(cy[k], 32, 64);
            }
            if (g == 0) {
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    const int c = c0 + 16 * k + l;
                    if (c < nY) unsafeAtomicAdd(uY + c, cy[k]);
                }
            }
        }
    }
}

// Intramonomer term of Eq. 57, formed when the full monomer equation's integral
// classes are attached: ui_X[(i,a)] = sum over (i1,a1) of
// (2 v^{a i1}_{i a1} - v^{a i}_{a1 i1}) t^{a1}_{i1}, with v^{a i1}_{i a1} =
// (ai|a1 i1) = K-hat[(i,a),(i1,a1)] and v^{a i}_{a1 i1} = (a a1|i i1) =
// J[i][i1][a][a1], which the packed J-hat[(r,c)] = J[c_occ][r_occ][r_vir][c_vir]
// holds at [(i1,a),(i,a1)].  One workgroup per monomer, t staged in LDS, a wave
// per output row with the lanes over its columns (both matrices are read once per
// sweep: 2 n^2 doubles per monomer, HBM-bound and small beside the pair phase).
constexpr int kMaxN = 4096;
__global__ __launch_bounds__(kMonoThreadsS) void singles_intra_kernel(
    const MonoDesc* __restrict__ monos, const double* __restrict__ K, const double* __restrict__ Jh,
    const double* __restrict__ t, double* __restrict__ ui, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl) {
    if (ctrl && ctrl->done) return;
    __shared__ double st[kMaxN];
    const int x = blockIdx.x;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;
    const int v = d.v, n = d.n, np = d.np;
    const double* Kx = K + d.mat_off;
    const double* Jx = Jh + d.mat_off;
    for (int k = threadIdx.x; k < n; k += kMonoThreadsS) st[k] = t[d.dif_off + k];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int r = wave; r < n; r += kMonoThreadsS / 64) {
        const int i = r / v, a = r - i * v;
        double acc = 0.0;
        for (int c = lane; c < n; c += 64) {
            const int i1 = c / v, a1 = c - i1 * v;
            acc += (2.0 * Kx[(int64_t)r * np + c] - Jx[(int64_t)(i1 * v + a) * np + i * v + a1]) * st[c];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) ui[d.dif_off + r] = acc;
    }
}

// init: t = w / d (first order), E_M1 into em1 and em1_0.
// update: t' = (w + (2 u + ui)) / d (ui: the intramonomer term, or none), residual
// max|t' - t|, E_M1(t'), u cleared for the next sweep.
__global__ __launch_bounds__(kMonoThreadsS) void singles_mono_kernel(
    int init, const MonoDesc* __restrict__ monos, const double* __restrict__ dif, const double* __restrict__ w,
    double* __restrict__ u, const double* __restrict__ ui, double* __restrict__ t, double* __restrict__ em1,
    double* __restrict__ em1_0, double* __restrict__ res, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl) {
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
            const double cpl = ui ? kSpinSum * ux[k] + ui[d.dif_off + k] : kSpinSum * ux[k];
            const double tn = di * (wx[k] + cpl);
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

int singles_pair_grid(int n_cu) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, singles_pair_kernel, kSThreads, 0) != hipSuccess || per < 1)
        per = 1;
    return n_cu * per;
}

void launch_singles_pair(const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos, const double* V,
                         const double* t, double* u, int grid, const Ctrl* ctrl, const ClState* cl, hipStream_t s) {
    if (n_pair <= 0) return;
    hipLaunchKernelGGL(singles_pair_kernel, dim3(grid), dim3(kSThreads), 0, s, pairs, n_pair, monos, V, t, u, ctrl,
                       cl);
}

void launch_singles_mono(int init, const MonoDesc* monos, int n_mono, const double* dif, const double* w, double* u,
                         const double* ui, double* t, double* em1, double* em1_0, double* res, const Ctrl* ctrl,
                         const ClState* cl, hipStream_t s) {
    if (n_mono <= 0) return;
    hipLaunchKernelGGL(singles_mono_kernel, dim3(n_mono), dim3(kMonoThreadsS), 0, s, init, monos, dif, w, u, ui, t,
                       em1, em1_0, res, ctrl, cl);
}

void launch_singles_intra(const MonoDesc* monos, int n_mono, const double* K, const double* Jh, const double* t,
                          double* ui, const Ctrl* ctrl, const ClState* cl, hipStream_t s) {
    if (n_mono <= 0) return;
    hipLaunchKernelGGL(singles_intra_kernel, dim3(n_mono), dim3(kMonoThreadsS), 0, s, monos, K, Jh, t, ui, ctrl, cl);
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
