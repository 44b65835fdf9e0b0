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
//     source term, Tau and 4 <V, Tau> (Eq. 55); G accumulated in FP64, or
//     in FP32 when the caller passes an FP32 buffer (BF16 sweeps);
//   * `source` = 0 drops the integral term V from Tau (the homogeneous
//     correction equation of the FP64 polish).
// FP32 runs v_mfma_f32_16x16x4_f32 four times per 16-deep chunk; BF16 runs one
// v_mfma_f32_16x16x32_bf16 per 32-deep chunk.  Both accumulate 16 x 16 tiles
// with lane l holding rows 4*(l/16) + t of column l%16 (measured), and lane l
// supplies k = k0 + KL*(l/16) + e of both operands (KL = 4 or 8 contiguous
// values).
#include <utility>

#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s4 lds_s4;

constexpr int kThreads = 256;   // conversion kernel
constexpr int kXcds = 8;

// Tunable shapes of the pair kernel: super-block edge SB (a wave computes SB x SB
// output tiles of 16 x 16 per task), waves per workgroup NW, and how many k
// chunks of operand fragments are in flight ahead of the MFMAs (PD).
struct Variant {
    int sb, nw, pd;
};
constexpr Variant kVariants[] = {{3, 8, 1}, {3, 8, 2}, {3, 8, 3}, {2, 8, 2}, {2, 8, 3}, {4, 8, 1},
                                 {3, 4, 2}, {2, 16, 1}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

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

// Operand sources of a 16 x KC fragment (lane l: row 16*tile + l%16, KL
// contiguous k from k0 + KL*(l/16)):
//   Rows: a row-major matrix with k contiguous (global memory or LDS);
//   Cols: the transpose of a row-major LDS matrix (element (row, k) at
//         p[k * ld + row]), read as KL scalars per lane; every row k of the
//         chunk must be readable, and rows at or past the matrix's last are
//         zero (padding rows), so the reads need no condition.
template <class E>
struct Rows {
    const E* p;
    int ld;
    __device__ typename Lowp<E>::Frag operator()(int tile, int k0, int lane) const {
        return frag(p + (int64_t)(tile * 16 + (lane & 15)) * ld + k0 + (lane >> 4) * Lowp<E>::KL);
    }
};

template <class E>
struct Cols {
    const E* p;
    int ld;
    __device__ typename Lowp<E>::Frag operator()(int tile, int k0, int lane) const {
        typename Lowp<E>::Frag f;
        const int k = k0 + (lane >> 4) * Lowp<E>::KL;
        const E* q = p + (int64_t)k * ld + tile * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < Lowp<E>::KL; ++e) f[e] = q[(int64_t)e * ld];
        return f;
    }
};

// BF16 fragment of the transpose of a row-major LDS matrix (element (row, k) at
// p[k * ld + row]) by two LDS transpose reads (ds_read_b64_tr_b16).  Within each
// group of 16 lanes that instruction hands lane i, as its element j, element
// i % 4 of the 4 consecutive 16-bit values at the address of lane 4 j + i / 4
// of the group (measured).  So lane s of group g reads the 8 bytes at row
// k0 + 8 g + 4 h + s / 4 (h = 0, 1 for the two halves of the fragment), columns
// 16 tile + 4 (s % 4) .. + 3, and lane i receives column 16 tile + i of rows
// k0 + 8 g + 4 h + j: the fragment the MFMA expects, k contiguous per lane.
// Rows up to the last k of the chunk must be staged (zero past the matrix).
struct ColsTr {
    const __bf16* p;
    int ld;
    __device__ bf8 operator()(int tile, int k0, int lane) const {
        const int g = lane >> 4, s = lane & 15;
        __bf16* q = const_cast<__bf16*>(p) + (k0 + 8 * g + (s >> 2)) * ld + tile * 16 + 4 * (s & 3);
        const s4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)q);
        const s4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(q + 4 * ld));
        const bf4 a = __builtin_bit_cast(bf4, lo), b = __builtin_bit_cast(bf4, hi);
        return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
    }
};

// acc[i][j] += sum_k A(m0 + i)[row][k] * B(n0 + j)[col][k] for k < K, with the
// fragments of the PD chunks after the current one in flight (a ring of PD
// register slots, the loop unrolled by PD so every slot index is static).
template <class E, int NR, int NC, int PD, class SA, class SB_>
__device__ inline void gemm(const SA& A, const SB_& B, int K, int m0, int n0, int lane, f4 (&acc)[NR][NC]) {
    typedef Lowp<E> L;
    typename L::Frag ra[PD][NR], rb[PD][NC];
#pragma unroll
    for (int d = 0; d < PD; ++d)
        if (d * L::KC < K) {
#pragma unroll
            for (int i = 0; i < NR; ++i) ra[d][i] = A(m0 + i, d * L::KC, lane);
#pragma unroll
            for (int j = 0; j < NC; ++j) rb[d][j] = B(n0 + j, d * L::KC, lane);
        }
    for (int k0 = 0; k0 < K; k0 += PD * L::KC) {
#pragma unroll
        for (int d = 0; d < PD; ++d) {
            const int kc = k0 + d * L::KC;
            if (kc < K) {
                typename L::Frag a[NR], b[NC];
#pragma unroll
                for (int i = 0; i < NR; ++i) a[i] = ra[d][i];
#pragma unroll
                for (int j = 0; j < NC; ++j) b[j] = rb[d][j];
                const int kn = kc + PD * L::KC;
                if (kn < K) {
#pragma unroll
                    for (int i = 0; i < NR; ++i) ra[d][i] = A(m0 + i, kn, lane);
#pragma unroll
                    for (int j = 0; j < NC; ++j) rb[d][j] = B(n0 + j, kn, lane);
                }
#pragma unroll
                for (int i = 0; i < NR; ++i)
#pragma unroll
                    for (int j = 0; j < NC; ++j) acc[i][j] = L::mma(a[i], b[j], acc[i][j]);
            }
        }
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

template <int SB>
__device__ inline Grid make_grid(int RT, int CT) {
    Grid g;
    g.RT = RT;
    g.CT = CT;
    g.SR = (RT + SB - 1) / SB;
    g.SC = (CT + SB - 1) / SB;
    g.n = g.SR * g.SC;
    return g;
}

// Wave tasks over one or two tile grids: full SB x SB super-blocks are dealt
// round-robin; the super-blocks left over after the last full round, and edge
// super-blocks, are cut into 1 x SB row strips where they are SB tiles wide
// (several accumulators in flight instead of one) and into single tiles
// otherwise, dealt one by one.  Shapes with 16 waves (128 registers per lane)
// use single tiles only: the strip code paths would spill there.
template <int SB, int NW, class F>
__device__ inline void for_tasks(const Grid& g0, const Grid& g1, int wave, F&& f) {
    constexpr int kSB = SB, kWaves = NW;
    constexpr bool kStrips = NW <= 8;
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
            for (int i = 0; i < nr; ++i) {
                if (kStrips && nc == kSB) f(which, r0 + i, c0, Shape<1, kStrips ? kSB : 1>{});
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
            if (kStrips && nc == kSB) {
                if (idx++ % kWaves == wave) f(which, r0 + i, c0, Shape<1, kStrips ? kSB : 1>{});
            } else {
                for (int j = 0; j < nc; ++j, ++idx)
                    if (idx % kWaves == wave) f(which, r0 + i, c0 + j, Shape<1, 1>{});
            }
        }
    }
}

__device__ inline int acc_row(int lane, int t) { return ((lane >> 4) << 2) + t; }
__device__ inline int acc_col(int lane) { return lane & 15; }

// G block contributions: stored partials (deterministic mode), FP32 atomics
// into the FP32 accumulation buffer (BF16 sweeps), or FP64 atomics into G
template <int NR, int NC>
__device__ inline void atomic_flush(double* G, float* Gf, double* part, int ld, int n, int r0, int q0, int lane,
                                    const f4 (&acc)[NR][NC]) {
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int c = (q0 + j) * 16 + acc_col(lane);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = (r0 + i) * 16 + acc_row(lane, t);
                if (part) part[(int64_t)r * ld + c] = (double)acc[i][j][t];
                else if (r < n && c < n) {
                    if (Gf) unsafeAtomicAdd(Gf + (int64_t)r * ld + c, acc[i][j][t]);
                    else unsafeAtomicAdd(G + (int64_t)r * ld + c, (double)acc[i][j][t]);
                }
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

// Bytes of LDS the LDS-resident variant needs for a pair: FP32 keeps V (npX
// rows); BF16 keeps V and Tau, each with ldX rows (npX, then zero rows up to the
// k range of the transposed fragments read from them), each row padded by 16
// bytes so that the 16-byte fragment reads of 8 consecutive rows fall on
// distinct bank groups.
template <class E>
__host__ __device__ inline int lds_row(int ld) { return ld + 16 / (int)sizeof(E); }

template <class E>
__host__ __device__ inline int64_t lds_bytes(int npX, int npY, int ldX, int ldY) {
    (void)npY;
    if (sizeof(E) == 2) return 2 * (int64_t)ldX * lds_row<E>(ldY) * sizeof(E);
    return (int64_t)npX * lds_row<E>(ldY) * sizeof(E);
}

// One pair per workgroup iteration.  IN_LDS: V is staged in LDS once per pair
// (BF16 also keeps Tau in LDS and reads the transposed operands, V^T and Tau^T,
// from them with LDS transpose reads; FP32 reads V^T fragments as columns of the
// staged V) and every product takes one operand from LDS and the other (M_X,
// M_Y, and Tau and Tau^T for FP32) from L2 (BF16 G_X and G_Y: both from LDS);
// otherwise both operands come from L2.
template <class E, int SB, int NW, int PD, bool IN_LDS>
__global__ __launch_bounds__(NW * 64) void pair_lowp_kernel(
    const PairDesc* __restrict__ pairs, int64_t n_pair, const MonoDesc* __restrict__ monos,
    const double* __restrict__ dif, const E* __restrict__ Vlo, const int64_t* __restrict__ lo_off,
    const E* __restrict__ Mlo, const int64_t* __restrict__ mlo_off, double* __restrict__ G, float* __restrict__ Gf,
    E* __restrict__ scratch, int64_t slot_elems, double* __restrict__ ed2, int source, int couple,
    const Ctrl* __restrict__ ctrl, const ClState* __restrict__ cl, PartOut po) {
    typedef Lowp<E> L;
    constexpr int kThreadsK = NW * 64;
    constexpr bool kTrLds = IN_LDS && sizeof(E) == 2;
    if (ctrl && ctrl->done) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double red[NW];
    E* sV = reinterpret_cast<E*>(lds_raw);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    E* tau = scratch + (int64_t)blockIdx.x * slot_elems;
    float sink = 0.f;
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
        const int sldY = lds_row<E>(ldY);
        E* sTau = sV + (int64_t)ldX * sldY;   // BF16 only

        if (IN_LDS) {   // stage V with 16-byte copies; padding rows and columns come zero
            constexpr int VE = 16 / sizeof(E);
            typedef uint4 Chunk;
            const int cy = ldY / VE;
            for (int idx = threadIdx.x; idx < npX * cy; idx += kThreadsK) {
                const int r = idx / cy, c = idx - r * cy;
                *reinterpret_cast<Chunk*>(sV + r * sldY + c * VE) =
                    *reinterpret_cast<const Chunk*>(V + (int64_t)r * ldY + c * VE);
            }
            if (kTrLds) {
                // V and Tau rows npX..ldX-1: zero, read as the k padding of the transposed fragments
                for (int idx = threadIdx.x; idx < (ldX - npX) * sldY; idx += kThreadsK) {
                    sV[(int64_t)npX * sldY + idx] = L::from(0.0);
                    sTau[(int64_t)npX * sldY + idx] = L::from(0.0);
                }
            }
            __syncthreads();
        }
        auto v_at = [&](int r, int c) -> double {
            return L::to_d(IN_LDS ? sV[r * sldY + c] : V[(int64_t)r * ldY + c]);
        };
        // the four operand roles of V: rows of V (k over Y), rows of V^T (k over X)
        auto vrows = [&]() { return Rows<E>{IN_LDS ? sV : V, IN_LDS ? sldY : ldY}; };

        // ---- Tau = D_XY * (source V + M_X V + V M_Y^T), E_D2 = 4 <V, Tau> ----
        double epart = 0.0;
        for_tasks<SB, NW>(make_grid<SB>(RB, CB), make_grid<SB>(0, 0), wave, [&](int, int r0, int c0, auto shape) {
            constexpr int NR = decltype(shape)::NR, NC = decltype(shape)::NC;
            f4 acc[NR][NC];
            zero(acc);
            if constexpr (kTrLds) gemm<E, NR, NC, PD>(Rows<E>{MX, ldX}, ColsTr{sV, sldY}, ldX, r0, c0, lane, acc);   // M_X V
            else if (IN_LDS) gemm<E, NR, NC, PD>(Rows<E>{MX, ldX}, Cols<E>{sV, sldY}, ldX, r0, c0, lane, acc);
            else gemm<E, NR, NC, PD>(Rows<E>{MX, ldX}, Rows<E>{Vt, ldX}, ldX, r0, c0, lane, acc);
            gemm<E, NR, NC, PD>(vrows(), Rows<E>{MY, ldY}, ldY, r0, c0, lane, acc);                        // V M_Y^T
            // Epilogue, tile by tile: a tile's energy differences and V values are read
            // before its stores, at the padded indices (V, its copies and the differences
            // are zero-padded, so every read is in bounds), and the padding is masked by
            // selects: the loads issue back to back instead of one branch and one L2 round
            // trip per element.
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int c = (c0 + j) * 16 + acc_col(lane);
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const double dc = dY[c];
                    double dr[4], vv[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int r = (r0 + i) * 16 + acc_row(lane, t);
                        dr[t] = dX[r];
                        vv[t] = v_at(r, c);
                    }
                    E tv4[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int r = (r0 + i) * 16 + acc_row(lane, t);
                        const bool ok = r < nX && c < nY;
                        const double dinv = recip(dr[t] + dc);
                        const double v = vv[t];
                        const double tv = ok ? dinv * ((source ? v : 0.0) + (double)acc[i][j][t]) : 0.0;
                        epart += ok ? v * tv : 0.0;
                        tv4[t] = L::from(tv);
                        if (couple) {
                            if (kTrLds) sTau[r * sldY + c] = tv4[t];
                            else tau[(int64_t)r * ldY + c] = tv4[t];
                        }
                    }
                    if (couple && !kTrLds) {   // Tau^T row c, 4 consecutive columns (BF16 reads Tau from LDS)
                        E* q = tauT + (int64_t)c * ldX + (r0 + i) * 16 + acc_row(lane, 0);
#pragma unroll
                        for (int t = 0; t < 4; ++t) q[t] = tv4[t];
                    }
                    // keep the next tile's loads after this tile's work (hoisting every tile's
                    // loads would hold all their inputs in registers at once)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        });
        if (couple) {   // zero the k padding of Tau (columns npY..ldY) and Tau^T (columns npX..ldX)
            for (int idx = threadIdx.x; idx < npX * (ldY - npY); idx += kThreadsK) {
                const int r = idx / (ldY - npY), c = npY + idx % (ldY - npY);
                if (kTrLds) sTau[r * sldY + c] = L::from(0.0);
                else tau[(int64_t)r * ldY + c] = L::from(0.0);
            }
            for (int idx = threadIdx.x; !kTrLds && idx < npY * (ldX - npX); idx += kThreadsK) {
                const int r = idx / (ldX - npX), c = npX + idx % (ldX - npX);
                tauT[(int64_t)r * ldX + c] = L::from(0.0);
            }
        }
        epart = wave_sum(epart);
        if (lane == 0) red[wave] = epart;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int w = 0; w < NW; ++w) sum += red[w];
            ed2[pd.orig] = 4.0 * sum;
        }
        if (IN_LDS) {   // ask the L2 for the next pair's V while this pair finishes
            const int64_t pn = pair_for(it + 1, n_pair);
            if (pn < n_pair) {
                const PairDesc nd = pairs[pn];
                const MonoDesc nx = monos[nd.x], ny = monos[nd.y];
                const int64_t ne = (int64_t)nx.np * ((ny.n + L::KC - 1) / L::KC * L::KC);   // V, not V^T
                const E* vn = Vlo + lo_off[pn];
                for (int64_t e = (int64_t)threadIdx.x * (64 / sizeof(E)); e < ne; e += (int64_t)kThreadsK * (64 / sizeof(E)))
                    sink += (float)vn[e];
            }
        }
        if (couple) {
            double* GX = G ? G + dx.mat_off : nullptr;
            double* GY = G ? G + dy.mat_off : nullptr;
            float* GfX = Gf ? Gf + dx.mat_off : nullptr;
            float* GfY = Gf ? Gf + dy.mat_off : nullptr;
            // ---- G_X += Tau V^T (contract over Y index), G_Y += Tau^T V (contract over X index) ----
            for_tasks<SB, NW>(make_grid<SB>(RB, RB), make_grid<SB>(CB, CB), wave,
                              [&](int which, int r0, int c0, auto shape) {
                constexpr int NR = decltype(shape)::NR, NC = decltype(shape)::NC;
                f4 acc[NR][NC];
                zero(acc);
                if (which == 0) {
                    if (kTrLds) gemm<E, NR, NC, PD>(Rows<E>{sTau, sldY}, vrows(), ldY, r0, c0, lane, acc);
                    else gemm<E, NR, NC, PD>(Rows<E>{tau, ldY}, vrows(), ldY, r0, c0, lane, acc);
                    atomic_flush(GX, GfX, po.part ? po.part + po.off[pi] : nullptr, npX, nX, r0, c0, lane, acc);
                } else {
                    if constexpr (kTrLds)   // Tau^T and V, both transposed from the row-major LDS copies
                        gemm<E, NR, NC, PD>(ColsTr{sTau, sldY}, ColsTr{sV, sldY}, ldX, r0, c0, lane, acc);
                    else if (IN_LDS)
                        gemm<E, NR, NC, PD>(Rows<E>{tauT, ldX}, Cols<E>{sV, sldY}, ldX, r0, c0, lane, acc);
                    else gemm<E, NR, NC, PD>(Rows<E>{tauT, ldX}, Rows<E>{Vt, ldX}, ldX, r0, c0, lane, acc);
                    atomic_flush(GY, GfY, po.part ? po.part + po.off[pi] + (int64_t)npX * npX : nullptr, npY, nY, r0,
                                 c0, lane, acc);
                }
            });
        }
        __syncthreads();
    }
    if (sink == 1.2345e30f) ed2[0] = sink;   // keeps the prefetch loads; never true for finite inputs
}

template <class E, int V, bool IN_LDS>
const void* kernel_of() {
    return reinterpret_cast<const void*>(
        pair_lowp_kernel<E, kVariants[V].sb, kVariants[V].nw, kVariants[V].pd, IN_LDS>);
}

template <class E, bool IN_LDS, int... V>
const void* pick(int v, std::integer_sequence<int, V...>) {
    const void* k = nullptr;
    ((k = (v == V ? kernel_of<E, V, IN_LDS>() : k)), ...);
    return k;
}

const void* lowp_kernel(int precision, int variant, bool in_lds) {
    const auto seq = std::make_integer_sequence<int, kNumVariants>{};
    if (precision == 2) return in_lds ? pick<__bf16, true>(variant, seq) : pick<__bf16, false>(variant, seq);
    return in_lds ? pick<float, true>(variant, seq) : pick<float, false>(variant, seq);
}

int lowp_variant_threads(int variant) { return kVariants[variant].nw * 64; }

}  // namespace

int lowp_chunk(int precision) { return precision == 2 ? Lowp<__bf16>::KC : Lowp<float>::KC; }

int lowp_variants() { return kNumVariants; }

void lowp_variant_shape(int variant, int* sb, int* nw, int* pd) {
    *sb = kVariants[variant].sb;
    *nw = kVariants[variant].nw;
    *pd = kVariants[variant].pd;
}

int64_t lowp_lds_bytes(int precision, int nX, int nY) {
    const int kc = lowp_chunk(precision);
    const int npX = (nX + 15) / 16 * 16, npY = (nY + 15) / 16 * 16;
    const int ldX = (nX + kc - 1) / kc * kc, ldY = (nY + kc - 1) / kc * kc;
    return precision == 2 ? lds_bytes<__bf16>(npX, npY, ldX, ldY) : lds_bytes<float>(npX, npY, ldX, ldY);
}

int64_t lowp_lds_limit() { return 160 * 1024 - 1024; }

int pair_lowp_blocks_per_cu(int precision, int variant, int64_t lds_bytes) {
    int n = 0;
    const bool in_lds = lds_bytes > 0;
    if (in_lds) (void)hipFuncSetAttribute(lowp_kernel(precision, variant, true),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lowp_lds_limit());
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lowp_kernel(precision, variant, in_lds),
                                                                lowp_variant_threads(variant),
                                                                in_lds ? (size_t)lds_bytes : 0);
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

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

void launch_pair_lowp(int precision, int variant, int64_t lds_bytes, PartOut po, const PairDesc* pairs, int64_t n_pair,
                      const MonoDesc* monos, const double* dif, const void* Vlo, const int64_t* lo_off,
                      const void* Mlo, const int64_t* mlo_off, double* G, float* Gf, void* scratch, int64_t slot_elems,
                      int grid, double* ed2, int source, int couple, const Ctrl* ctrl, const ClState* cl,
                      hipStream_t s) {
    if (n_pair <= 0) return;
    void* args[] = {(void*)&pairs, (void*)&n_pair, (void*)&monos, (void*)&dif, (void*)&Vlo, (void*)&lo_off,
                    (void*)&Mlo, (void*)&mlo_off, (void*)&G, (void*)&Gf, (void*)&scratch, (void*)&slot_elems, (void*)&ed2,
                    (void*)&source, (void*)&couple, (void*)&ctrl, (void*)&cl, (void*)&po};
    (void)hipLaunchKernel(lowp_kernel(precision, variant, lds_bytes > 0), dim3(grid),
                          dim3(lowp_variant_threads(variant)), args, (size_t)std::max<int64_t>(lds_bytes, 0), s);
}

}  // namespace mcpt
