// Launchers of the singles sweep (singles.hip); internal, not part of the C ABI.
#pragma once

#include "mcpt_internal.hpp"

namespace mcpt {

int singles_pair_grid(int n_cu);
// u_X += V_XY t_Y and u_Y += V_XY^T t_X over the stored pairs of the live clusters
void launch_singles_pair(const PairDesc* pairs, int64_t n_pair, const MonoDesc* monos, const double* V,
                         const double* t, double* u, int grid, const Ctrl* ctrl, const ClState* cl, hipStream_t s);
// init = 1: t = w / d; 0: t = (w + 2 u + ui) / d with the residual, u cleared (ui may be null)
void launch_singles_mono(int init, const MonoDesc* monos, int n_mono, const double* dif, const double* w, double* u,
                         const double* ui, double* t, double* em1, double* em1_0, double* res, const Ctrl* ctrl,
                         const ClState* cl, hipStream_t s);
// ui_X = (2 K-hat - J) t_X, the intramonomer term of Eq. 57 (packed K-hat and J-hat of the
// full monomer equation)
void launch_singles_intra(const MonoDesc* monos, int n_mono, const double* K, const double* Jh, const double* t,
                          double* ui, const Ctrl* ctrl, const ClState* cl, hipStream_t s);
// per-cluster sums of E_M1 and its first-order value into ClState e_mono / e_mono0
void launch_singles_clusters(int n_cl, const int64_t* cl_mono, const double* em1, const double* em1_0, ClState* cl,
                             hipStream_t s);
// compact per-monomer vectors (offsets woff) into the padded dif layout
void launch_singles_scatter(const MonoDesc* monos, int n_mono, const int64_t* woff, const double* compact,
                            double* padded, hipStream_t s);

}  // namespace mcpt
