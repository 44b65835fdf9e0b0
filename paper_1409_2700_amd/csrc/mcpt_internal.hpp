// Internal declarations of the MCPT(2) HIP path (not part of the C ABI).
//
// Device layout of a resident problem:
//   monomer X: o, v, n = o*v, np = n rounded up to 16; every per-monomer
//   matrix (K, T, M, G) is np x np, row-major, row (i,a) = i*v + a, column
//   (j,b) = j*v + b, zero in the padding; matrices of all monomers are
//   concatenated at mat_off.
//   pair p = (X, Y): V_XY stored as given, nX x nY row-major (unpadded), at v_off.
//   dif: per monomer np values d[(i,a)] = e_i - e_a (zero in the padding), so
//   every denominator of Eqs. 60-61 is 1 / (d_X[(i,a)] + d_Y[(j,b)]).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mcpt {

constexpr int kTile = 16;              // MFMA tile edge; matrices are padded to a multiple
constexpr int kMaxSweeps = 4096;       // length of the device residual history
// The pair terms of Eqs. 57 and 58 sum k, c of the neighbour Y over both spins
// (a closed-shell Coulomb loop; with it the equations are restricted LCCD,
// Sec. II.A): the accumulated pair sums G and u enter the monomer updates twice.
constexpr double kSpinSum = 2.0;

// 1 / d for the denominators of Eqs. 60-61 (negative, |d| well above zero):
// the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r + r (1 - d r), each of which squares the relative error, so the
// result is within an ulp or so of the quotient at a fraction of the cost of
// an IEEE division.
__device__ inline double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Deterministic accumulation: instead of adding its G_X and G_Y blocks to G
// with atomics, pair p stores them at part + off[p] (np_X^2 values, then
// np_Y^2), and a per-monomer kernel sums the stored blocks in pair order.
// A stored pair of the dimer-internal terms of Eq. 59 (X = its first monomer): sizes and where
// its matrices sit.  Tau and the source S are npx x npy (rows (i,a) = i vx + a, columns
// (j,b) = j vy + b); the cross-ring classes C_X-hat (rows (i,b) = i vy + b) and C_Y-hat (rows
// (j,a) = j vx + a) are m1 x m1 and m2 x m2, and their products Y1 = C_X-hat Vs(Tau) and
// Y2 = C_Y-hat Vs(Tau^T) m1 x m2 and m2 x m1 (m1, m2 = ox vy and oy vx rounded up to 16);
// W_XY is packed as w_rows x ldw (rows (a,b) = a vy + b padded to 16, columns to 32).
struct DimerDesc {
    int32_t x, y;
    int32_t ox, vx, oy, vy;
    int32_t nx, ny, npx, npy;
    int32_t m1, m2;
    int32_t w_rows, ldw;
    int32_t cluster, pad;
    int64_t tau_off;       // Tau and S
    int64_t y1_off, y2_off;
    int64_t cx_off, cy_off;
    int64_t w_off, q_off;  // packed W_XY; Q_XY ((ox oy) x (ox oy), caller layout)
    int64_t w_raw_off, cx_raw_off, cy_raw_off;   // the pair's classes in the caller's concatenation
};

struct PartOut {
    double* part;            // nullptr: FP64 atomics into G
    const int64_t* off;      // per pair of the launch
    // dimer-internal terms (FP64 kernel only): S - Y1[(i,b),(j,a)] - Y2[(j,a),(i,b)] adds into
    // the numerator of Tau[(i,a),(j,b)] and Tau is kept in tau_out (S nullptr: none of it).  Every
    // monomer of one size (dd nullptr): all np x np at orig * mat_stride, v virtuals; otherwise at
    // the offsets of the pair's DimerDesc (dd, indexed by the caller's pair index)
    const double* S = nullptr;
    const double* Y1 = nullptr;
    const double* Y2 = nullptr;
    double* tau_out = nullptr;
    const DimerDesc* dd = nullptr;
    int64_t mat_stride = 0;
    int v = 0;
};

struct MonoDesc {
    int32_t o, v, n, np;
    int64_t eps_off;                   // first energy of X in eps
    int64_t mat_off;                   // first element of X's np x np matrices
    int64_t raw_off;                   // first element of X's o*o*v*v block in caller layout
    int64_t dif_off;                   // first element of X's np orbital-energy differences
    int32_t cluster;                   // cluster (request) the monomer belongs to
    int32_t pad;
};

struct PairDesc {
    int32_t x, y;                      // x is the row side (i,a) of V, y the column side (j,b)
    int64_t v_off;                     // first element of V_XY
    int64_t orig;                      // index of the pair in the caller's list
    int32_t cluster;
    int32_t pad;
};

// Per-cluster iteration state: a batch holds several independent clusters,
// each stopping on its own residual exactly as it would alone.
struct ClState {
    int32_t done;                      // 1: converged / diverged / out of sweeps; its work is skipped
    int32_t status;                    // 0, -4 (not converged) or -5 (diverged)
    int32_t sweeps;
    int32_t pad;
    double residual;
    double e_mono, e_dimer, e_mono0;
};

// Device-side iteration state.  The reduction kernel of every sweep appends
// each live cluster's residual to its history, applies the stopping rules and
// sets the cluster's `done`; `done` here is set when every cluster is done.
// Sweep kernels launched after that return at once (or skip the done
// clusters), so sweeps issued ahead of a host check end exactly at the sweep
// that met the rule.
struct Ctrl {
    int32_t done;
    int32_t status;                    // worst cluster status
    int32_t sweeps;                    // most sweeps of any cluster
    int32_t fixed;                     // 1: run exactly max_sweeps, no convergence test
    int32_t max_sweeps;
    int32_t pad;
    double tol;
    double residual;                   // largest last residual over clusters
    double e_mono, e_dimer, e_mono0;   // sums written by the final reduction
};

enum MonoMode : int {
    kMonoInit = 0,      // T = D*K, M, E_M2 -> em2 and em2_0
    kMonoUpdate = 1,    // T' = D*(K + G + G^T), residual, M', E_M2(T')
    kMonoFromT = 2,     // M and E_M2 from the T already stored
    kMonoE0 = 3,        // E_M2 of D*K into em2_0 only (warm starts)
    kMonoUpdateR = 4,   // update, keeping R = T' - T (FP64 polish sweep)
    kMonoCorr = 5,      // delta = R + D*(G + G^T), low-precision 2 delta - S(delta)
    kMonoApply = 6,     // T += delta - R
    kMonoRlo = 7        // low-precision 2R - S(R)
};

// ---- launchers (kernels_common.hip) ----
void launch_fill(double* p, int64_t n, double value, hipStream_t s);
void launch_pack(const MonoDesc* monos, int n_mono, const double* raw, double* packed,
                 int max_n, hipStream_t s);
void launch_unpack(const MonoDesc* monos, int n_mono, const double* packed, double* raw,
                   int max_n, hipStream_t s);
void launch_nonfinite(const double* p, int64_t n, int32_t* flag, hipStream_t s);
// V[off[b] .. off[b] + len[b]) *= f[b] for b < n
void launch_scale_blocks(const int64_t* off, const int64_t* len, const double* f, int64_t n, double* V,
                         hipStream_t s);
void launch_monomer(int mode, const MonoDesc* monos, int n_mono, int max_v, const double* dif,
                    const double* K, const double* G, double* G_zero, double* T, double* M,
                    double* em2, double* em2_0, double* res, const Ctrl* ctrl, const ClState* cl,
                    hipStream_t s, const double* L = nullptr);   // L: extra term of the update (full monomer equation)
// Gf / Gf_zero: the FP32 accumulation buffers of BF16 sweeps, read and cleared instead of G / G_zero
void launch_monomer_mixed(int mode, int precision, const MonoDesc* monos, int n_mono, int max_v, const double* dif,
                          const double* K, const double* G, double* G_zero, double* T, double* M, double* R,
                          double* Dl, void* Mlo, const int64_t* mlo_off, double* em2, double* em2_0,
                          double* res, const Ctrl* ctrl, const ClState* cl, hipStream_t s,
                          const float* Gf = nullptr, float* Gf_zero = nullptr, const double* L = nullptr);
// (L: the intramonomer terms of the full monomer equation, added by the update and correction modes;
//  with L, the rlo and corr modes also store the FP64 2 delta - S(delta) in M)
void launch_reduce_sweep(int n_cl, const int64_t* cl_mono, const double* res, ClState* cl, double* hist,
                         Ctrl* ctrl, hipStream_t s);
// G_X = sum of the stored partial blocks of monomer X (csr[csr_off[X] .. csr_off[X+1]):
// offsets into part, in pair order); skips stopped clusters
void launch_reduce_parts(const MonoDesc* monos, int n_mono, const int64_t* csr_off, const int64_t* csr,
                         const double* part, double* G, const ClState* cl, const Ctrl* ctrl, hipStream_t s);
void launch_reduce_final(int n_cl, const int64_t* cl_mono, const int64_t* cl_pair, const double* em2,
                         const double* em2_0, const double* ed2, ClState* cl, Ctrl* ctrl, hipStream_t s);

// ---- FP64 MFMA pair phase (pair_fp64.hip) ----
// Eq. 59 (Tau from V, M_X, M_Y) and, if couple != 0, the Eq. 58 contractions
// G_X += Tau V^T, G_Y += Tau^T V for every pair; E_D2 of every pair.  Two
// variants: lds_variant = 1 stages V in LDS (pairs with pair_fits_lds), 0 reads
// V from L2 (any size).
void launch_pair_fp64(int lds_variant, PartOut po, const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos,
                      const double* dif, const double* V, const double* M, double* G,
                      double* scratch, int64_t slot_elems, int grid, double* ed2, int couple,
                      const Ctrl* ctrl, const ClState* cl, hipStream_t s);
int pair_fp64_blocks_per_cu(int lds_variant);
bool pair_fits_lds(int nX, int npX, int npY);
// Pairs read from L2 in two launches per chunk of at most one pair per persistent workgroup:
// Tau of every pair (into the chunk's slots of the Tau scratch), then, if couple != 0, G.  Pair k
// of a chunk belongs to XCD k % 8, whose workgroups take its pairs' tasks (3 x 3 tile blocks) in
// pair order: a few pairs per XCD at a time, dealt out in even rounds of blocks rather than whole
// pairs per workgroup.  Plain FP64 form only (no dimer source, no stored partials).
struct GlbTasks {
    const int32_t* xpair;   // processing index of each pair of the chunk, grouped by XCD
    const int64_t* tau_off; // element offset of its Tau in the scratch (row stride npY)
    const int32_t* pre;     // exclusive prefix of the pairs' task counts (n + 1 entries)
    int xbeg[9];            // XCD x's pairs: xpair[xbeg[x] .. xbeg[x + 1])
};
// tasks of a pair: Tau blocks SR x SC, G blocks SR^2 + SC^2 (SR = ceil(npX / 48), SC = ceil(npY / 48))
int glb_tau_tasks(int npX, int npY);
int glb_g_tasks(int npX, int npY);
void launch_pair_fp64_split(const GlbTasks& tau_tasks, const GlbTasks& g_tasks, int n_chunk_pairs,
                            const PairDesc* pairs, const MonoDesc* monos, const double* dif, const double* V,
                            const double* M, double* G, double* scratch, int grid, double* ed2, int couple,
                            const Ctrl* ctrl, const ClState* cl, hipStream_t s);

// ---- reduced-precision pair phase (pair_lowp.hip); precision 1 = FP32, 2 = BF16 ----
int lowp_chunk(int precision);   // k chunk: rows of low-precision operands are padded to it
void launch_convert_v(int precision, const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos,
                      const double* V, void* Vlo, const int64_t* lo_off, hipStream_t s);
// reduced-precision pair kernel: `variant` selects one of lowp_variants() tile shapes;
// lds_bytes > 0 selects the LDS-resident-V kernel with that much dynamic LDS
// (every pair of the launch must need at most that much: lowp_lds_bytes)
int lowp_variants();
void lowp_variant_shape(int variant, int* sb, int* nw, int* pd);
int64_t lowp_lds_bytes(int precision, int nX, int nY);
int64_t lowp_lds_limit();
int pair_lowp_blocks_per_cu(int precision, int variant, int64_t lds_bytes);
void launch_pair_lowp(int precision, int variant, int64_t lds_bytes, PartOut po, const PairDesc* pairs, int64_t n_pair,
                      const MonoDesc* monos, const double* dif, const void* Vlo, const int64_t* lo_off,
                      const void* Mlo, const int64_t* mlo_off, double* G, float* Gf, void* scratch, int64_t slot_elems,
                      int grid, double* ed2, int source, int couple, const Ctrl* ctrl, const ClState* cl,
                      hipStream_t s);   // Gf non-null: G contributions in FP32 (G unused)

}  // namespace mcpt
