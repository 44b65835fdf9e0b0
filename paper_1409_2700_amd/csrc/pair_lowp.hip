// Pair phase in reduced precision (FP32 or BF16 matrix-core inputs, FP32
// accumulation) for the mixed-precision form of the MCPT(2) sweep.
//
// Same products as the FP64 pair phase (Eq. 59 Tau, Eq. 55 E_D2, the Eq. 58
// contractions G_X += Tau V^T, G_Y += Tau^T V), with:
//   * operands stored so the contraction index k is contiguous in every one of
//     them: V and V^T (per pair, converted once per problem), M (per monomer,
//     written by the monomer kernel each sweep), Tau and Tau^T (per-workgroup
//     scratch), each row padded to a multiple of the k chunk and zero there;
//     every operand fragment is then one 16-byte load per lane;
//   * the epilogue in FP64: denominators 1 / (d_X + d_Y) (Eqs. 60-61), the
//     source term, Tau and 4 <V, Tau> (Eq. 55); G accumulated in FP64;
//   * `source` = 0 drops the integral term V from Tau (the homogeneous
//     correction equation of the FP64 polish).
// FP32 runs v_mfma_f32_16x16x4_f32 four times per 16-deep chunk; BF16 runs one
// v_mfma_f32_16x16x32_bf16 per 32-deep chunk.  Both accumulate 16 x 16 tiles
// with lane l holding rows 4*(l/16) + t of column l%16 (measured), and lane l
// supplies k = k0 + KL*(l/16) + e of both operands (KL = 4 or 8 contiguous
// values).
#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSB = 3;
constexpr int kXcds = 8;

template <class E>
struct Lowp;

template <>
struct Lowp<float> {
    static constexpr int KL = 4;    // contiguous k per lane
    static constexpr int KC = 16;   // k per chunk
    typedef f4 Frag;
    __device__ static inline f4 mma(const Frag& a, const Frag& b, f4 c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, c, 0, 0, 0);
    }
    __device__ static inline float from(double x) { return (float)x; }
    __device__ static inline double to_d(float x) { return (double)x; }
};

template <>
struct Lowp<__bf16> {
    static constexpr int KL = 8;
    static constexpr int KC = 32;
    typedef bf8 Frag;
    __device__ static inline f4 mma(const Frag& a, const Frag& b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static inline __bf16 from(double x) { return (__bf16)(float)x; }
    __device__ static inline double to_d(__bf16 x) { return (double)(float)x; }
};

template <int R, int C>
struct Shape {
    static constexpr int NR = R, NC = C;
};

template <class E>
__device__ inline typename Lowp<E>::Frag frag(const E* p) {
    return *reinterpret_cast<const typename Lowp<E>::Frag*>(p);
}

// acc[i][j] += sum_k A[(m0 + i) * 16 + row][k] * Bt[(n0 + j) * 16 + col][k], k < K,
// with A and Bt row-major (row strides lda, ldb), k contiguous.
template <class E, int NR, int NC>
__device__ inline void gemm_tiles(const E* A, int lda, const E* Bt, int ldb, int K, int m0, int n0, int lane,
                                  f4 (&acc)[NR][NC]) {
    typedef Lowp<E> L;
    const int lr = lane & 15, lk = (lane >> 4) * L::KL;
    const E* ap[NR];
    const E* bp[NC];
#pragma unroll
    for (int i = 0; i < NR; ++i) ap[i] = A + (int64_t)((m0 + i) * 16 + lr) * lda + lk;
#pragma unroll
    for (int j = 0; j < NC; ++j) bp[j] = Bt + (int64_t)((n0 + j) * 16 + lr) * ldb + lk;
    typename L::Frag an[NR], bn[NC];
#pragma unroll
    for (int i = 0; i < NR; ++i) an[i] = frag(ap[i]);
#pragma unroll
    for (int j = 0; j < NC; ++j) bn[j] = frag(bp[j]);
    for (int k0 = 0; k0 < K; k0 += L::KC) {
        typename L::Frag a[NR], b[NC];
#pragma unroll
        for (int i = 0; i < NR; ++i) a[i] = an[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) b[j] = bn[j];
        if (k0 + L::KC < K) {
#pragma unroll
            for (int i = 0; i < NR; ++i) an[i] = frag(ap[i] + k0 + L::KC);
#pragma unroll
            for (int j = 0; j < NC; ++j) bn[j] = frag(bp[j] + k0 + L::KC);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[i][j] = L::mma(a[i], b[j], acc[i][j]);
    }
}

template <int NR, int NC>
__device__ inline void zero(f4 (&acc)[NR][NC]) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[i][j] = f4(0.f);
}

struct Grid {
    int RT, CT, SR, SC, n;
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

template <class F>
__device__ inline void for_tasks(const Grid& g0, const Grid& g1, int wave, F&& f) {
    const int total = g0.n + g1.n;
    const int full = total - total % kWaves;
    for (int sb = wave; sb < full; sb += kWaves) {
        const int which = sb >= g0.n ? 1 : 0;
        const Grid& g = which ? g1 : g0;
        const int s = which ? sb - g0.n : sb;
        const int r0 = (s / g.SC) * kSB, c0 = (s % g.SC) * kSB;
        const int nr = min(kSB, g.RT - r0), nc = min(kSB, g.CT - c0);
        if (nr == kSB && nc == kSB) {
            f(which, r0, c0, Shape<kSB, kSB>{});
        } else {
            for (int i = 0; i < nr; ++i)
                for (int j = 0; j < nc; ++j) f(which, r0 + i, c0 + j, Shape<1, 1>{});
        }
    }
    int idx = 0;
    for (int sb = full; sb < total; ++sb) {
        const int which = sb >= g0.n ? 1 : 0;
        const Grid& g = which ? g1 : g0;
        const int s = which ? sb - g0.n : sb;
        const int r0 = (s / g.SC) * kSB, c0 = (s % g.SC) * kSB;
        const int nr = min(kSB, g.RT - r0), nc = min(kSB, g.CT - c0);
        for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nc; ++j, ++idx)
                if (idx % kWaves == wave) f(which, r0 + i, c0 + j, Shape<1, 1>{});
    }
}

__device__ inline int acc_row(int lane, int t) { return ((lane >> 4) << 2) + t; }
__device__ inline int acc_col(int lane) { return lane & 15; }

template <int NR, int NC>
__device__ inline void atomic_flush(double* G, int ld, int n, int r0, int q0, int lane, const f4 (&acc)[NR][NC]) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int c = (q0 + j) * 16 + acc_col(lane);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = (r0 + i) * 16 + acc_row(lane, t);
                if (r < n && c < n) unsafeAtomicAdd(G + (int64_t)r * ld + c, (double)acc[i][j][t]);
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

// Layout of the reduced-precision copies of a pair (offset lo_off of the pair):
//   V   npX rows x ldY  (ldY = nY rounded up to the k chunk), then
//   V^T npY rows x ldX.
template <class E>
__global__ __launch_bounds__(kThreads) void convert_v_kernel(const PairDesc* __restrict__ pairs,
                                                              const MonoDesc* __restrict__ monos,
                                                              const double* __restrict__ V, E* __restrict__ Vlo,
                                                              const int64_t* __restrict__ lo_off) {
    typedef Lowp<E> L;
    const PairDesc pd = pairs[blockIdx.x];
    const MonoDesc dx = monos[pd.x], dy = monos[pd.y];
    const int ldX = (dx.n + L::KC - 1) / L::KC * L::KC, ldY = (dy.n + L::KC - 1) / L::KC * L::KC;
    const double* v = V + pd.v_off;
    E* vl = Vlo + lo_off[blockIdx.x];
    E* vt = vl + (int64_t)dx.np * ldY;
    for (int idx = threadIdx.x; idx < dx.np * ldY; idx += kThreads) {
        const int r = idx / ldY, c = idx - r * ldY;
        vl[idx] = L::from((r < dx.n && c < dy.n) ? v[(int64_t)r * dy.n + c] : 0.0);
    }
    for (int idx = threadIdx.x; idx < dy.np * ldX; idx += kThreads) {
        const int c = idx / ldX, r = idx - c * ldX;
        vt[idx] = L::from((r < dx.n && c < dy.n) ? v[(int64_t)r * dy.n + c] : 0.0);
    }
}

template <class E>
__global__ __launch_bounds__(kThreads) void pair_lowp_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ dif, const E* __restrict__ Vlo, const int64_t* __restrict__ lo_off,
    const E* __restrict__ Mlo, const int64_t* __restrict__ mlo_off, double* __restrict__ G,
    E* __restrict__ scratch, int64_t slot_elems, double* __restrict__ ed2, int source, int couple,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl) {
    typedef Lowp<E> L;
    if (ctrl && ctrl->done) return;
    __shared__ double red[kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    E* tau = scratch + (int64_t)blockIdx.x * slot_elems;
    for (int64_t it = 0;; ++it) {
        const int64_t pi = pair_for(it, n_pair);
        if (pi >= n_pair) break;
        const PairDesc pd = pairs[pi];
        if (cl && cl[pd.cluster].done) continue;   // cluster stopped: uniform over the workgroup
        const MonoDesc dx = monos[pd.x], dy = monos[pd.y];
        const int nX = dx.n, nY = dy.n, npX = dx.np, npY = dy.np;
        const int ldX = (nX + L::KC - 1) / L::KC * L::KC, ldY = (nY + L::KC - 1) / L::KC * L::KC;
        const E* V = Vlo + lo_off[pi];
        const E* Vt = V + (int64_t)npX * ldY;
        const E* MX = Mlo + mlo_off[pd.x];
        const E* MY = Mlo + mlo_off[pd.y];
        const double* dX = dif + dx.dif_off;
        const double* dY = dif + dy.dif_off;
        E* tauT = tau + (int64_t)npX * ldY;   // Tau: npX x ldY; Tau^T: npY x ldX
        const int RB = npX / 16, CB = npY / 16;

        // ---- Tau = D_XY * (source V + M_X V + V M_Y^T), E_D2 = 4 <V, Tau> ----
        double epart = 0.0;
        for_tasks(make_grid(RB, CB), make_grid(0, 0), wave, [&](int, int r0, int c0, auto shape) {
            constexpr int NR = decltype(shape)::NR, NC = decltype(shape)::NC;
            f4 acc[NR][NC];
            zero(acc);
            gemm_tiles<E, NR, NC>(MX, ldX, Vt, ldX, ldX, r0, c0, lane, acc);   // M_X V
            gemm_tiles<E, NR, NC>(V, ldY, MY, ldY, ldY, r0, c0, lane, acc);    // V M_Y^T
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int c = (c0 + j) * 16 + acc_col(lane);
                const double dc = c < nY ? dY[c] : 0.0;
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    E tv4[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int r = (r0 + i) * 16 + acc_row(lane, t);
                        double tv = 0.0;
                        if (r < nX && c < nY) {
                            const double dinv = 1.0 / (dX[r] + dc);
                            const double v = L::to_d(V[(int64_t)r * ldY + c]);
                            tv = dinv * ((source ? v : 0.0) + (double)acc[i][j][t]);
                            epart += v * tv;
                        }
                        tv4[t] = L::from(tv);
                        if (couple) tau[(int64_t)r * ldY + c] = tv4[t];
                    }
                    if (couple) {   // Tau^T row c, 4 consecutive columns
                        E* q = tauT + (int64_t)c * ldX + (r0 + i) * 16 + acc_row(lane, 0);
#pragma unroll
                        for (int t = 0; t < 4; ++t) q[t] = tv4[t];
                    }
                }
            }
        });
        if (couple) {   // zero the k padding of Tau (columns npY..ldY) and Tau^T (columns npX..ldX)
            for (int idx = threadIdx.x; idx < npX * (ldY - npY); idx += kThreads) {
                const int r = idx / (ldY - npY), c = npY + idx % (ldY - npY);
                tau[(int64_t)r * ldY + c] = L::from(0.0);
            }
            for (int idx = threadIdx.x; idx < npY * (ldX - npX); idx += kThreads) {
                const int r = idx / (ldX - npX), c = npX + idx % (ldX - npX);
                tauT[(int64_t)r * ldX + c] = L::from(0.0);
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
            double* GX = G + dx.mat_off;
            double* GY = G + dy.mat_off;
            // ---- G_X += Tau V^T (contract over Y index), G_Y += Tau^T V (contract over X index) ----
            for_tasks(make_grid(RB, RB), make_grid(CB, CB), wave, [&](int which, int r0, int c0, auto shape) {
                constexpr int NR = decltype(shape)::NR, NC = decltype(shape)::NC;
                f4 acc[NR][NC];
                zero(acc);
                if (which == 0) {
                    gemm_tiles<E, NR, NC>(tau, ldY, V, ldY, ldY, r0, c0, lane, acc);
                    atomic_flush(GX, npX, nX, r0, c0, lane, acc);
                } else {
                    gemm_tiles<E, NR, NC>(tauT, ldX, Vt, ldX, ldX, r0, c0, lane, acc);
                    atomic_flush(GY, npY, nY, r0, c0, lane, acc);
                }
            });
        }
        __syncthreads();
    }
}

}  // namespace

int lowp_chunk(int precision) { return precision == 2 ? Lowp<__bf16>::KC : Lowp<float>::KC; }

void launch_convert_v(int precision, const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos,
                      const double* V, void* Vlo, const int64_t* lo_off, hipStream_t s) {
    if (n_pair <= 0) return;
    if (precision == 2)
        hipLaunchKernelGGL(convert_v_kernel<__bf16>, dim3(n_pair), dim3(kThreads), 0, s, pairs, monos, V,
                           static_cast<__bf16*>(Vlo), lo_off);
    else
        hipLaunchKernelGGL(convert_v_kernel<float>, dim3(n_pair), dim3(kThreads), 0, s, pairs, monos, V,
                           static_cast<float*>(Vlo), lo_off);
}

int pair_lowp_blocks_per_cu(int precision) {
    int n = 0;
    hipError_t e = precision == 2
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_lowp_kernel<__bf16>, kThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_lowp_kernel<float>, kThreads, 0);
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

void launch_pair_lowp(int precision, const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos,
                      const double* dif, const void* Vlo, const int64_t* lo_off, const void* Mlo,
                      const int64_t* mlo_off, double* G, void* scratch, int64_t slot_elems, int grid, double* ed2,
                      int source, int couple, const Ctrl* ctrl, const ClState* cl, hipStream_t s) {
    if (n_pair <= 0) return;
    if (precision == 2)
        hipLaunchKernelGGL(pair_lowp_kernel<__bf16>, dim3(grid), dim3(kThreads), 0, s, pairs, n_pair, monos, dif,
                           static_cast<const __bf16*>(Vlo), lo_off, static_cast<const __bf16*>(Mlo), mlo_off, G,
                           static_cast<__bf16*>(scratch), slot_elems, ed2, source, couple, ctrl, cl);
    else
        hipLaunchKernelGGL(pair_lowp_kernel<float>, dim3(grid), dim3(kThreads), 0, s, pairs, n_pair, monos, dif,
                           static_cast<const float*>(Vlo), lo_off, static_cast<const float*>(Mlo), mlo_off, G,
                           static_cast<float*>(scratch), slot_elems, ed2, source, couple, ctrl, cl);
}

}  // namespace mcpt
