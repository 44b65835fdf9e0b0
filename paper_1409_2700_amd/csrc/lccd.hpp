// Intramonomer terms of Eq. 58 (full monomer equation): device layout and
// launchers (not part of the C ABI).
#pragma once

#include "mcpt_internal.hpp"

namespace mcpt {

constexpr int kLccdMaxNp = 1024;     // padded o v of a monomer the ring kernel's offset table holds
constexpr int kLccdMaxLdw = 4096;    // padded v^2 the ladder kernel's offset table holds (v <= 64)

// Per monomer: where its packed integral matrix W (w_rows x ldw, rows (a,b)
// zero-padded to 16, columns (c,d) to 32) and its raw <kl|ij> block sit.
struct LccdDesc {
    int64_t w_off;       // first element of the packed W in the device buffer
    int64_t w_raw_off;   // first element of W_X in the caller's concatenated layout
    int64_t q_off;       // first element of Q_X (o^4, caller layout) in the device buffer
    int32_t w_rows;      // v^2 rounded up to 16
    int32_t ldw;         // v^2 rounded up to 32
};

void launch_lccd_pack(const MonoDesc* monos, const LccdDesc* ld, int n_mono, const double* w_raw,
                      const double* j_raw, double* W, double* J, hipStream_t s);
int lccd_ring_blocks(int max_np);
int lccd_ladder_blocks(int max_w_rows, int max_o);
int lccd_ladder_ct(int max_o);   // column tiles per ladder task: ceil(max_o^2 / 16), at most 4
// R12 = K M - J T and Y = J Vs(T) for every live monomer
void launch_lccd_ring(const MonoDesc* monos, int n_mono, int ring_blocks, const double* K, const double* J,
                      const double* T, const double* M, double* R12, double* Y, const Ctrl* ctrl, const ClState* cl,
                      hipStream_t s);
// LDS bytes of the LDS-staged ladder kernel for a monomer (its n x n amplitudes
// and offset tables, later four v x (v + 1) ring blocks), and the per-workgroup limit
int64_t lccd_ladder_lds_bytes(int n, int v, int ldw);
int64_t lccd_lds_limit();
// L = P + H + R + R^T (R = R12 - Vs(Y)) for every live monomer; lds_bytes > 0
// selects the LDS-staged kernel (every monomer must need at most that much)
void launch_lccd_ladder(const MonoDesc* monos, const LccdDesc* ld, int n_mono, int ladder_blocks, int ct,
                        int64_t lds_bytes, const double* W, const double* Q, const double* T, const double* R12,
                        const double* Y, double* L, const Ctrl* ctrl, const ClState* cl, hipStream_t s,
                        int rings = 1);

// The ring terms of the dimer equation: the monomer rings added into S (which must hold the
// ladders), the cross rings stored in Y1 and Y2 for the pair kernel.  dimer_ring_blocks: the
// workgroups per pair for the pair of the most ring tasks.
int dimer_ring_tasks(const DimerDesc& d);
int dimer_ring_blocks(int max_tasks);
// RM = 2 K - J of the monomers (n elements of the monomer matrix buffers)
void launch_ring_matrix(const double* K, const double* J, double* RM, int64_t n, hipStream_t s);
void launch_dimer_ring(const DimerDesc* dd, const MonoDesc* monos, int n_pair, int blocks, const double* RM,
                       const double* CX, const double* CY, const double* Tau, double* S, double* Y1, double* Y2,
                       const Ctrl* ctrl, const ClState* cl, hipStream_t s);
// Pack the caller's dimer classes of every pair into the layouts of its DimerDesc: W_XY, C_X-hat
// [(i,b),(i1,b1)] = C_X[i1][i][b][b1] and C_Y-hat[(j,a),(j1,a1)] = C_Y[j1][j][a][a1] (a null source
// skips its part)
void launch_dimer_pack(const DimerDesc* dd, int n_pair, const double* w_raw, const double* cx_raw,
                       const double* cy_raw, double* W, double* CX, double* CY, hipStream_t s);
// The pair ladders of every live pair from global memory: S = P + H (stored), for pairs of any
// two monomer sizes; blocks_per_pair and ct as lccd_ladder_blocks / lccd_ladder_ct of the
// largest w_rows and ox oy
void launch_dimer_ladder(const DimerDesc* dd, int n_pair, int blocks_per_pair, int ct, const double* W,
                         const double* Q, const double* Tau, double* S, const Ctrl* ctrl, const ClState* cl,
                         hipStream_t s);
int dimer_ladder_blocks(int max_w_rows, int max_o2);
int dimer_ladder_ct(int max_o2);

}  // namespace mcpt
