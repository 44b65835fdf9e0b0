// Elementwise and reduction kernels of the MCPT(2) path: layout packing, the
// monomer phase (Eq. 58 divided by its denominators, Eq. 54 energy) and the
// per-sweep residual / stopping rule.
#include <cfloat>
#include <cmath>

#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

constexpr int kMonoThreads = 256;
constexpr int kReduceThreads = 1024;

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// caller layout K[i][j][a][b] (o,o,v,v)  <->  packed np x np, row (i,a), column (j,b)
__global__ void pack_kernel(const MonoDesc* __restrict__ monos, const double* __restrict__ raw,
                            double* __restrict__ packed, int to_packed) {
    const MonoDesc d = monos[blockIdx.x];
    const int o = d.o, v = d.v, n = d.n, np = d.np;
    const int nn = n * n;
    for (int idx = blockIdx.y * blockDim.x + threadIdx.x; idx < nn; idx += gridDim.y * blockDim.x) {
        const int r = idx / n, c = idx - r * n;
        const int i = r / v, a = r - i * v;
        const int j = c / v, b = c - j * v;
        const int64_t ri = d.raw_off + ((int64_t)(i * o + j) * v + a) * v + b;
        const int64_t pi = d.mat_off + (int64_t)r * np + c;
        if (to_packed)
            packed[pi] = raw[ri];
        else
            packed[ri] = raw[pi];   // here `raw` is the packed source and `packed` the caller layout
    }
}

__global__ void nonfinite_kernel(const double* __restrict__ p, int64_t n, int32_t* flag) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (bad) *flag = 1;
}

// V blocks of listed pairs multiplied by their factors (finite-displacement
// geometries: couplings rescaled by (R0 / R)^3); block b covers pair b.
__global__ void scale_blocks_kernel(const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                                    const double* __restrict__ f, double* __restrict__ V) {
    const int64_t o = off[blockIdx.x], n = len[blockIdx.x];
    const double s = f[blockIdx.x];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) V[o + i] *= s;
}

template <int NT>
__device__ double block_sum(double x, double* sh) {
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// max that propagates NaN (so a non-finite residual is seen by the stopping rule)
__device__ inline double max_nan(double a, double b) { return (a != a || b != b) ? NAN : (a > b ? a : b); }

template <int NT>
__device__ double block_max(double x, double* sh) {
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = max_nan(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Monomer phase, one workgroup per monomer.  For element (r, c) = ((i,a),(j,b))
// the occupied-swapped partner S(r, c) = ((j,a),(i,b)) has the same denominator
// e_i + e_j - e_a - e_b (Eqs. 60-61), formed as (e_i - e_a) + (e_j - e_b) from the
// per-monomer differences; both values are formed by the same thread so the
// spin-adapted combination 2X - S(X) of Eq. 59 needs no second pass (values at
// S(r, c) are recomputed from inputs, never read from an output).
// E_M2 = <2K - S(K), T> = <K, M> (Eq. 54).  Modes:
//   init      T = D K, M, E_M2 -> em2 and em2_0
//   update    T' = D (K + 2 (G + G^T)), residual |T' - T|, M', E_M2(T')  (2: spin sum)
//   from_t    M and E_M2 of the stored T
//   e0        E_M2 of D K into em2_0 only
//   update_r  as update, and R = T' - T kept, low-precision copy of 2R - S(R)
//   corr      delta = R + 2 D (G + G^T) (homogeneous equation), low-precision 2 delta - S(delta)
//   apply     T += delta - R (elementwise)
// Mlo (optional) receives the low-precision copy of the combination written.
// G is read, and Gz cleared, in GT: double, or float for the FP32 accumulation
// buffers of BF16 sweeps.
template <class E, class GT>
__global__ __launch_bounds__(kMonoThreads) void monomer_kernel(
    int mode, const MonoDesc* __restrict__ monos, const double* __restrict__ dif,
    const double* __restrict__ K, const GT* __restrict__ G, GT* __restrict__ Gz,
    double* __restrict__ T, double* __restrict__ M, double* __restrict__ R, double* __restrict__ Dl,
    E* __restrict__ Mlo, const int64_t* __restrict__ mlo_off, int lo_chunk, double* __restrict__ em2,
    double* __restrict__ em2_0, double* __restrict__ res, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl, const double* __restrict__ Lt) {
    if (ctrl && ctrl->done) return;
    __shared__ double sh[kMonoThreads];
    const int x = blockIdx.x;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;   // this monomer's cluster has stopped
    const int v = d.v, n = d.n, np = d.np;
    const double* dx = dif + d.dif_off;
    const double* Kx = K + d.mat_off;
    const GT* Gx = G ? G + d.mat_off : nullptr;
    double* Tx = T + d.mat_off;
    double* Mx = M + d.mat_off;
    double* Rx = R ? R + d.mat_off : nullptr;
    double* Dx = Dl ? Dl + d.mat_off : nullptr;
    E* Ml = Mlo ? Mlo + mlo_off[x] : nullptr;
    const int ldl = (n + lo_chunk - 1) / lo_chunk * lo_chunk;
    double rmax = 0.0, esum = 0.0;
    const int nn = n * n;
    for (int idx = threadIdx.x; idx < nn; idx += kMonoThreads) {
        const int r = idx / n, c = idx - r * n;
        const int i = r / v, a = r - i * v;
        const int j = c / v, b = c - j * v;
        const int rs = j * v + a, cs = i * v + b;
        const int64_t e_rc = (int64_t)r * np + c, e_s = (int64_t)rs * np + cs;
        const int64_t e_t = (int64_t)c * np + r, e_st = (int64_t)cs * np + rs;
        if (mode == kMonoApply) {
            Tx[e_rc] += Dx[e_rc] - Rx[e_rc];
            continue;
        }
        const double dinv = recip(dx[r] + dx[c]);
        double tn, ts, lo = 0.0;
        bool has_lo = false;
        if (mode == kMonoUpdate || mode == kMonoUpdateR) {
            if (Lt) {   // intramonomer terms of the full monomer equation
                const double* Lx = Lt + d.mat_off;
                tn = dinv * (((Kx[e_rc] + kSpinSum * (double)Gx[e_rc]) + kSpinSum * (double)Gx[e_t]) + Lx[e_rc]);
                ts = dinv * (((Kx[e_s] + kSpinSum * (double)Gx[e_s]) + kSpinSum * (double)Gx[e_st]) + Lx[e_s]);
            } else {
                tn = dinv * ((Kx[e_rc] + kSpinSum * (double)Gx[e_rc]) + kSpinSum * (double)Gx[e_t]);
                ts = dinv * ((Kx[e_s] + kSpinSum * (double)Gx[e_s]) + kSpinSum * (double)Gx[e_st]);
            }
            const double told = Tx[e_rc];
            rmax = max_nan(rmax, fabs(tn - told));
            if (mode == kMonoUpdateR) {
                // R at S(r,c) would need the old T there, which its own thread overwrites;
                // the combination 2R - S(R) is formed by a following rlo launch instead.
                Rx[e_rc] = tn - told;
            } else {
                lo = 2.0 * tn - ts;
                has_lo = true;
            }
        } else if (mode == kMonoCorr) {
            if (Lt) {   // intramonomer terms of the correction (full monomer equation)
                const double* Lx = Lt + d.mat_off;
                tn = Rx[e_rc] + dinv * ((kSpinSum * (double)Gx[e_rc] + kSpinSum * (double)Gx[e_t]) + Lx[e_rc]);
                ts = Rx[e_s] + dinv * ((kSpinSum * (double)Gx[e_s] + kSpinSum * (double)Gx[e_st]) + Lx[e_s]);
            } else {
                tn = Rx[e_rc] + dinv * (kSpinSum * (double)Gx[e_rc] + kSpinSum * (double)Gx[e_t]);
                ts = Rx[e_s] + dinv * (kSpinSum * (double)Gx[e_s] + kSpinSum * (double)Gx[e_st]);
            }
            Dx[e_rc] = tn;
            lo = 2.0 * tn - ts;
            has_lo = true;
            if (Lt) Mx[e_rc] = lo;   // FP64 2 delta - S(delta) for the next intramonomer terms
        } else if (mode == kMonoRlo) {
            tn = Rx[e_rc];
            ts = Rx[e_s];
            lo = 2.0 * tn - ts;
            has_lo = true;
            if (Lt) Mx[e_rc] = lo;
        } else if (mode == kMonoFromT) {
            tn = Tx[e_rc];
            ts = Tx[e_s];
        } else {
            tn = dinv * Kx[e_rc];
            ts = dinv * Kx[e_s];
        }
        if (mode != kMonoCorr && mode != kMonoRlo) {
            const double m = 2.0 * tn - ts;
            esum += Kx[e_rc] * m;
            if (mode == kMonoInit || mode == kMonoUpdate || mode == kMonoUpdateR) Tx[e_rc] = tn;
            if (mode != kMonoE0) Mx[e_rc] = m;
            if (!has_lo) {
                lo = m;
                has_lo = true;
            }
        }
        if (Ml && has_lo) Ml[(int64_t)r * ldl + c] = (E)(float)lo;
    }
    if (Gz) {
        GT* gz = Gz + d.mat_off;
        const int npp = np * np;
        for (int idx = threadIdx.x; idx < npp; idx += kMonoThreads) gz[idx] = GT(0);
    }
    if (mode == kMonoApply || mode == kMonoRlo || mode == kMonoCorr) return;
    const double etot = block_sum<kMonoThreads>(esum, sh);
    const double rtot = block_max<kMonoThreads>(rmax, sh);
    if (threadIdx.x == 0) {
        if (mode == kMonoE0) {
            em2_0[x] = etot;
        } else {
            em2[x] = etot;
            if (mode == kMonoInit) em2_0[x] = etot;
            if (mode == kMonoUpdate || mode == kMonoUpdateR) res[x] = rtot;
        }
    }
}

// Stopping rule, same as the oracle's, per cluster: converged when r < tol;
// diverged when r is not finite, r > 1e6 r_1, or r rose in each of the last
// three sweeps and exceeds r_1; not converged when max_sweeps sweeps ran.
// The same monomer phase organised by v x v blocks.  In the (i,a),(j,b) layout
// the occupied swap S maps block (i,j) onto block (j,i) element for element
// ((a,b) -> (a,b)), and G^T at (i,a),(j,b) is element (b,a) of block (j,i).  One
// pass over the block pair {(i,j), (j,i)} therefore reads every element once:
// K, T and R along contiguous block rows, G through LDS for the transposed
// read.  Results are bitwise those of monomer_kernel (same operations in the
// same order per element).
template <class E, int VMAX, class GT>
__global__ __launch_bounds__(kMonoThreads) void monomer_blocks_kernel(
    int mode, const MonoDesc* __restrict__ monos, const double* __restrict__ dif,
    const double* __restrict__ K, const GT* __restrict__ G, GT* __restrict__ Gz,
    double* __restrict__ T, double* __restrict__ M, double* __restrict__ R, double* __restrict__ Dl,
    E* __restrict__ Mlo, const int64_t* __restrict__ mlo_off, int lo_chunk, double* __restrict__ em2,
    double* __restrict__ em2_0, double* __restrict__ res, const Ctrl* __restrict__ ctrl,
    const ClState* __restrict__ cl, const double* __restrict__ Lt) {
    if (ctrl && ctrl->done) return;
    __shared__ double sh[kMonoThreads];
    __shared__ double sg[2][VMAX][VMAX + 1];
    const int x = blockIdx.x;
    const MonoDesc d = monos[x];
    if (cl && cl[d.cluster].done) return;   // this monomer's cluster has stopped
    const int o = d.o, v = d.v, n = d.n, np = d.np;
    const double* dx = dif + d.dif_off;
    const double* Kx = K + d.mat_off;
    const GT* Gx = G ? G + d.mat_off : nullptr;
    double* Tx = T + d.mat_off;
    double* Mx = M + d.mat_off;
    double* Rx = R ? R + d.mat_off : nullptr;
    double* Dx = Dl ? Dl + d.mat_off : nullptr;
    E* Ml = Mlo ? Mlo + mlo_off[x] : nullptr;
    const int ldl = (n + lo_chunk - 1) / lo_chunk * lo_chunk;
    const bool need_g = mode == kMonoUpdate || mode == kMonoUpdateR || mode == kMonoCorr;
    double rmax = 0.0, esum = 0.0;
    for (int i = 0; i < o; ++i)
        for (int j = i; j < o; ++j) {
            const bool diag = i == j;
            if (need_g) {
                __syncthreads();   // the previous block pair is done with sg
                for (int idx = threadIdx.x; idx < v * v; idx += kMonoThreads) {
                    const int a = idx / v, b = idx - a * v;
                    sg[0][a][b] = kSpinSum * (double)Gx[(int64_t)(i * v + a) * np + j * v + b];
                    sg[1][a][b] = kSpinSum * (double)Gx[(int64_t)(j * v + a) * np + i * v + b];
                }
                __syncthreads();
            }
            for (int idx = threadIdx.x; idx < v * v; idx += kMonoThreads) {
                const int a = idx / v, b = idx - a * v;
                const int r1 = i * v + a, c1 = j * v + b, r2 = j * v + a, c2 = i * v + b;
                const int64_t e1 = (int64_t)r1 * np + c1, e2 = (int64_t)r2 * np + c2;
                if (mode == kMonoApply) {
                    Tx[e1] += Dx[e1] - Rx[e1];
                    if (!diag) Tx[e2] += Dx[e2] - Rx[e2];
                    continue;
                }
                const double d1 = recip(dx[r1] + dx[c1]), d2 = recip(dx[r2] + dx[c2]);
                double t1, t2, lo1 = 0.0, lo2 = 0.0;
                bool has_lo = false;
                if (mode == kMonoUpdate || mode == kMonoUpdateR) {
                    if (Lt) {   // intramonomer terms of the full monomer equation
                        const double* Lx = Lt + d.mat_off;
                        t1 = d1 * (((Kx[e1] + sg[0][a][b]) + sg[1][b][a]) + Lx[e1]);
                        t2 = d2 * (((Kx[e2] + sg[1][a][b]) + sg[0][b][a]) + Lx[e2]);
                    } else {
                        t1 = d1 * ((Kx[e1] + sg[0][a][b]) + sg[1][b][a]);
                        t2 = d2 * ((Kx[e2] + sg[1][a][b]) + sg[0][b][a]);
                    }
                    const double o1 = Tx[e1], o2 = Tx[e2];
                    rmax = max_nan(rmax, fabs(t1 - o1));
                    if (!diag) rmax = max_nan(rmax, fabs(t2 - o2));
                    if (mode == kMonoUpdateR) {
                        Rx[e1] = t1 - o1;
                        if (!diag) Rx[e2] = t2 - o2;
                    } else {
                        lo1 = 2.0 * t1 - t2;
                        lo2 = 2.0 * t2 - t1;
                        has_lo = true;
                    }
                } else if (mode == kMonoCorr) {
                    if (Lt) {   // intramonomer terms of the correction (full monomer equation)
                        const double* Lx = Lt + d.mat_off;
                        t1 = Rx[e1] + d1 * ((sg[0][a][b] + sg[1][b][a]) + Lx[e1]);
                        t2 = Rx[e2] + d2 * ((sg[1][a][b] + sg[0][b][a]) + Lx[e2]);
                    } else {
                        t1 = Rx[e1] + d1 * (sg[0][a][b] + sg[1][b][a]);
                        t2 = Rx[e2] + d2 * (sg[1][a][b] + sg[0][b][a]);
                    }
                    Dx[e1] = t1;
                    if (!diag) Dx[e2] = t2;
                    lo1 = 2.0 * t1 - t2;
                    lo2 = 2.0 * t2 - t1;
                    has_lo = true;
                    if (Lt) {   // FP64 2 delta - S(delta) for the next intramonomer terms
                        Mx[e1] = lo1;
                        if (!diag) Mx[e2] = lo2;
                    }
                } else if (mode == kMonoRlo) {
                    t1 = Rx[e1];
                    t2 = Rx[e2];
                    lo1 = 2.0 * t1 - t2;
                    lo2 = 2.0 * t2 - t1;
                    has_lo = true;
                    if (Lt) {
                        Mx[e1] = lo1;
                        if (!diag) Mx[e2] = lo2;
                    }
                } else if (mode == kMonoFromT) {
                    t1 = Tx[e1];
                    t2 = Tx[e2];
                } else {
                    t1 = d1 * Kx[e1];
                    t2 = d2 * Kx[e2];
                }
                if (mode != kMonoCorr && mode != kMonoRlo) {
                    const double m1 = 2.0 * t1 - t2, m2 = 2.0 * t2 - t1;
                    esum += Kx[e1] * m1;
                    if (!diag) esum += Kx[e2] * m2;
                    if (mode == kMonoInit || mode == kMonoUpdate || mode == kMonoUpdateR) {
                        Tx[e1] = t1;
                        if (!diag) Tx[e2] = t2;
                    }
                    if (mode != kMonoE0) {
                        Mx[e1] = m1;
                        if (!diag) Mx[e2] = m2;
                    }
                    if (!has_lo) {
                        lo1 = m1;
                        lo2 = m2;
                        has_lo = true;
                    }
                }
                if (Ml && has_lo) {
                    Ml[(int64_t)r1 * ldl + c1] = (E)(float)lo1;
                    if (!diag) Ml[(int64_t)r2 * ldl + c2] = (E)(float)lo2;
                }
            }
        }
    if (Gz) {
        GT* gz = Gz + d.mat_off;
        const int npp = np * np;
        for (int idx = threadIdx.x; idx < npp; idx += kMonoThreads) gz[idx] = GT(0);
    }
    if (mode == kMonoApply || mode == kMonoRlo || mode == kMonoCorr) return;
    const double etot = block_sum<kMonoThreads>(esum, sh);
    const double rtot = block_max<kMonoThreads>(rmax, sh);
    if (threadIdx.x == 0) {
        if (mode == kMonoE0) {
            em2_0[x] = etot;
        } else {
            em2[x] = etot;
            if (mode == kMonoInit) em2_0[x] = etot;
            if (mode == kMonoUpdate || mode == kMonoUpdateR) res[x] = rtot;
        }
    }
}

// Convergence test of one sweep, one workgroup per cluster: max|dT| over the
// cluster's monomers, its residual history and the stopping rules (tolerance,
// divergence, sweep limit).  Clusters that have stopped are left untouched.
__global__ __launch_bounds__(kReduceThreads) void reduce_sweep_kernel(
    const int64_t* __restrict__ cl_mono, const double* __restrict__ res, ClState* __restrict__ cl,
    double* __restrict__ hist_all, const Ctrl* __restrict__ ctrl) {
    const int q = blockIdx.x;
    if (ctrl->done || cl[q].done) return;
    __shared__ double sh[kReduceThreads];
    double m = 0.0;
    for (int64_t i = cl_mono[q] + threadIdx.x; i < cl_mono[q + 1]; i += kReduceThreads) m = max_nan(m, res[i]);
    const double r = block_max<kReduceThreads>(m, sh);
    if (threadIdx.x != 0) return;
    double* h = hist_all + (int64_t)q * kMaxSweeps;
    const int s = cl[q].sweeps;
    h[s] = r;
    int status = 0, done = 0;
    if (!(r <= DBL_MAX)) {
        status = -5;
        done = 1;
    } else if (!ctrl->fixed) {
        if (r < ctrl->tol) {
            done = 1;
        } else if (r > 1e6 * h[0] ||
                   (s >= 3 && h[s] > h[s - 1] && h[s - 1] > h[s - 2] && h[s - 2] > h[s - 3] && r > h[0])) {
            status = -5;
            done = 1;
        } else if (s + 1 >= ctrl->max_sweeps) {
            status = -4;
            done = 1;
        }
    } else if (s + 1 >= ctrl->max_sweeps) {
        done = 1;
    }
    cl[q].sweeps = s + 1;
    cl[q].residual = r;
    cl[q].status = status;
    cl[q].done = done;
}

// Batch-wide view of the per-cluster states: done when every cluster is, the
// worst status (diverged before not converged), the largest sweep count and residual.
__global__ __launch_bounds__(kReduceThreads) void reduce_ctrl_kernel(int n_cl, const ClState* __restrict__ cl,
                                                                     Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double sh[kReduceThreads];
    double notdone = 0.0, nstat = 0.0, sw = 0.0, rmax = 0.0;
    for (int q = threadIdx.x; q < n_cl; q += kReduceThreads) {
        notdone = fmax(notdone, cl[q].done ? 0.0 : 1.0);
        nstat = fmax(nstat, (double)-cl[q].status);
        sw = fmax(sw, (double)cl[q].sweeps);
        rmax = max_nan(rmax, cl[q].residual);
    }
    notdone = block_max<kReduceThreads>(notdone, sh);
    nstat = block_max<kReduceThreads>(nstat, sh);
    sw = block_max<kReduceThreads>(sw, sh);
    rmax = block_max<kReduceThreads>(rmax, sh);
    if (threadIdx.x == 0) {
        ctrl->sweeps = (int)sw;
        ctrl->residual = rmax;
        ctrl->status = -(int)nstat;
        ctrl->done = notdone == 0.0;
    }
}

// Per-cluster energy sums (Eqs. 54-56), one workgroup per cluster.
__global__ __launch_bounds__(kReduceThreads) void reduce_final_kernel(
    const int64_t* __restrict__ cl_mono, const int64_t* __restrict__ cl_pair, const double* __restrict__ em2,
    const double* __restrict__ em2_0, const double* __restrict__ ed2, ClState* __restrict__ cl) {
    const int q = blockIdx.x;
    __shared__ double sh[kReduceThreads];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = cl_mono[q] + threadIdx.x; i < cl_mono[q + 1]; i += kReduceThreads) {
        a += em2[i];
        c += em2_0[i];
    }
    for (int64_t i = cl_pair[q] + threadIdx.x; i < cl_pair[q + 1]; i += kReduceThreads) b += ed2[i];
    a = block_sum<kReduceThreads>(a, sh);
    b = block_sum<kReduceThreads>(b, sh);
    c = block_sum<kReduceThreads>(c, sh);
    if (threadIdx.x == 0) {
        cl[q].e_mono = a;
        cl[q].e_dimer = b;
        cl[q].e_mono0 = c;
    }
}

// Batch totals of the per-cluster energies, summed in cluster order.
__global__ void reduce_total_kernel(int n_cl, const ClState* __restrict__ cl, Ctrl* __restrict__ ctrl) {
    if (threadIdx.x != 0) return;
    double ta = 0.0, tb = 0.0, tc = 0.0;
    for (int q = 0; q < n_cl; ++q) {
        ta += cl[q].e_mono;
        tb += cl[q].e_dimer;
        tc += cl[q].e_mono0;
    }
    ctrl->e_mono = ta;
    ctrl->e_dimer = tb;
    ctrl->e_mono0 = tc;
}

// Deterministic G: G_X[e] = sum over the monomer's stored partial blocks, in
// pair order (one workgroup per monomer, threads over the np^2 elements).
__global__ __launch_bounds__(256) void reduce_parts_kernel(const MonoDesc* __restrict__ monos,
                                                           const int64_t* __restrict__ csr_off,
                                                           const int64_t* __restrict__ csr,
                                                           const double* __restrict__ part, double* __restrict__ G,
                                                           const ClState* __restrict__ cl,
                                                           const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    const MonoDesc d = monos[blockIdx.x];
    if (cl && cl[d.cluster].done) return;
    const int64_t e0 = csr_off[blockIdx.x], e1 = csr_off[blockIdx.x + 1];
    const int64_t nn = (int64_t)d.np * d.np;
    double* g = G + d.mat_off;
    for (int64_t k = threadIdx.x; k < nn; k += 256) {
        double sum = 0.0;
        for (int64_t e = e0; e < e1; ++e) sum += part[csr[e] + k];
        g[k] = sum;
    }
}

int grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

void launch_fill(double* p, int64_t n, double value, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, value);
}

void launch_pack(const MonoDesc* monos, int n_mono, const double* raw, double* packed, int max_n,
                 hipStream_t s) {
    const int gy = (max_n * max_n + 255) / 256 > 64 ? 64 : (max_n * max_n + 255) / 256;
    hipLaunchKernelGGL(pack_kernel, dim3(n_mono, gy), dim3(256), 0, s, monos, raw, packed, 1);
}

void launch_unpack(const MonoDesc* monos, int n_mono, const double* packed, double* raw, int max_n,
                   hipStream_t s) {
    const int gy = (max_n * max_n + 255) / 256 > 64 ? 64 : (max_n * max_n + 255) / 256;
    hipLaunchKernelGGL(pack_kernel, dim3(n_mono, gy), dim3(256), 0, s, monos, packed, raw, 0);
}

void launch_scale_blocks(const int64_t* off, const int64_t* len, const double* f, int64_t n, double* V,
                         hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_blocks_kernel, dim3((unsigned)n), dim3(256), 0, s, off, len, f, V);
}

void launch_nonfinite(const double* p, int64_t n, int32_t* flag, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256)),
                       dim3(256), 0, s, p, n, flag);
}

// Blocked kernel when every monomer's v fits its LDS tiles, the element-wise one otherwise.
template <class E, class GT>
void monomer_dispatch(int max_v, int mode, const MonoDesc* monos, int n_mono, const double* dif, const double* K,
                      const GT* G, GT* G_zero, double* T, double* M, double* R, double* Dl, E* Mlo,
                      const int64_t* mlo_off, int chunk, double* em2, double* em2_0, double* res, const Ctrl* ctrl,
                      const ClState* cl, hipStream_t s, const double* Lt = nullptr) {
    if (n_mono <= 0) return;
    if (max_v <= 32)
        hipLaunchKernelGGL((monomer_blocks_kernel<E, 32, GT>), dim3(n_mono), dim3(kMonoThreads), 0, s, mode, monos,
                           dif, K, G, G_zero, T, M, R, Dl, Mlo, mlo_off, chunk, em2, em2_0, res, ctrl, cl, Lt);
    else if (max_v <= 64)
        hipLaunchKernelGGL((monomer_blocks_kernel<E, 64, GT>), dim3(n_mono), dim3(kMonoThreads), 0, s, mode, monos,
                           dif, K, G, G_zero, T, M, R, Dl, Mlo, mlo_off, chunk, em2, em2_0, res, ctrl, cl, Lt);
    else
        hipLaunchKernelGGL((monomer_kernel<E, GT>), dim3(n_mono), dim3(kMonoThreads), 0, s, mode, monos, dif, K, G,
                           G_zero, T, M, R, Dl, Mlo, mlo_off, chunk, em2, em2_0, res, ctrl, cl, Lt);
}

void launch_monomer(int mode, const MonoDesc* monos, int n_mono, int max_v, const double* dif, const double* K,
                    const double* G, double* G_zero, double* T, double* M, double* em2,
                    double* em2_0, double* res, const Ctrl* ctrl, const ClState* cl, hipStream_t s,
                    const double* L) {
    monomer_dispatch<float, double>(max_v, mode, monos, n_mono, dif, K, G, G_zero, T, M, nullptr, nullptr, nullptr,
                                    nullptr, 16, em2, em2_0, res, ctrl, cl, s, L);
}

void launch_monomer_mixed(int mode, int precision, const MonoDesc* monos, int n_mono, int max_v, const double* dif,
                          const double* K, const double* G, double* G_zero, double* T, double* M, double* R,
                          double* Dl, void* Mlo, const int64_t* mlo_off, double* em2, double* em2_0,
                          double* res, const Ctrl* ctrl, const ClState* cl, hipStream_t s, const float* Gf,
                          float* Gf_zero, const double* L) {
    if (precision == 2 && (Gf || Gf_zero))
        monomer_dispatch<__bf16, float>(max_v, mode, monos, n_mono, dif, K, Gf, Gf_zero, T, M, R, Dl,
                                        static_cast<__bf16*>(Mlo), mlo_off, 32, em2, em2_0, res, ctrl, cl, s, L);
    else if (precision == 2)
        monomer_dispatch<__bf16, double>(max_v, mode, monos, n_mono, dif, K, G, G_zero, T, M, R, Dl,
                                         static_cast<__bf16*>(Mlo), mlo_off, 32, em2, em2_0, res, ctrl, cl, s, L);
    else
        monomer_dispatch<float, double>(max_v, mode, monos, n_mono, dif, K, G, G_zero, T, M, R, Dl,
                                        static_cast<float*>(Mlo), mlo_off, 16, em2, em2_0, res, ctrl, cl, s, L);
}

void launch_reduce_sweep(int n_cl, const int64_t* cl_mono, const double* res, ClState* cl, double* hist,
                         Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(reduce_sweep_kernel, dim3(n_cl), dim3(kReduceThreads), 0, s, cl_mono, res, cl, hist, ctrl);
    hipLaunchKernelGGL(reduce_ctrl_kernel, dim3(1), dim3(kReduceThreads), 0, s, n_cl, cl, ctrl);
}

void launch_reduce_parts(const MonoDesc* monos, int n_mono, const int64_t* csr_off, const int64_t* csr,
                         const double* part, double* G, const ClState* cl, const Ctrl* ctrl, hipStream_t s) {
    if (n_mono <= 0) return;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(n_mono), dim3(256), 0, s, monos, csr_off, csr, part, G, cl, ctrl);
}

void launch_reduce_final(int n_cl, const int64_t* cl_mono, const int64_t* cl_pair, const double* em2,
                         const double* em2_0, const double* ed2, ClState* cl, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(reduce_final_kernel, dim3(n_cl), dim3(kReduceThreads), 0, s, cl_mono, cl_pair, em2, em2_0,
                       ed2, cl);
    hipLaunchKernelGGL(reduce_total_kernel, dim3(1), dim3(64), 0, s, n_cl, cl, ctrl);
}

}  // namespace mcpt
