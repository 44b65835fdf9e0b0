/*
 * mcpt.h - C ABI of the MCPT(2) doubles hot path on one AMD Instinct MI355X.
 *
 * Method: Byrd et al., "Molecular Cluster Perturbation Theory. I. Formalism",
 * Sec. II.C.  The library solves, for every monomer X of a cluster, the monomer
 * doubles amplitudes T_X (Eq. 58, tm2) and, for every pair (X, Y) inside the
 * cutoff, the dimer doubles amplitudes Tau_XY (Eq. 59, td2), iterated to
 * self-consistency as in step 6 of the program flow, and evaluates the monomer
 * energies E_M2(X) (Eq. 54), their shift dE_M2(X) (Eq. 56) and the dimer
 * energies E_D2(XY) (Eq. 55).
 *
 * Terms kept: the source integrals, the pair coupling of Eq. 58 and the
 * monomer-amplitude coupling of Eq. 59 - the terms that the two integral
 * classes taken as input can form.  Each amplitude equation is solved as
 * eps * amplitude = integral + coupling terms, with eps^{ij}_{ab} =
 * e_i + e_j - e_a - e_b < 0 (Eqs. 60-61).  Every dimer integral of Eqs. 55,
 * 58, 59 is the one Coulomb block (ai|bj) of real orbitals (Eq. 29); the
 * reversed pair uses its transpose.  The isolated-monomer reference of Eq. 56
 * is the energy at zero coupling, E_M2 at T = D * K.
 *
 * Conventions for every call:
 *  - Every function returns an mcpt_status; no C++ exception crosses the ABI.
 *  - On error no output is written and mcpt_last_error() describes the cause
 *    (message stored per calling thread, valid until its next call).
 *  - Input arrays are owned by the caller and are copied before the call
 *    returns; output arrays are allocated by the caller.
 *  - Device memory and resident problems belong to the context until
 *    mcpt_release() or mcpt_destroy().
 *  - A context is used by one host thread at a time; the serving calls
 *    (mcpt_submit ...) run the solves on the context's own worker threads.
 */
#ifndef MCPT_H
#define MCPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCPT_OK = 0,
    MCPT_PENDING = 1,            /* mcpt_poll: the request has not finished yet */
    MCPT_ERR_INVALID = -1,       /* bad sizes, pair list, options or denominator >= 0 */
    MCPT_ERR_NOMEM = -2,         /* device allocation failed */
    MCPT_ERR_DEVICE = -3,        /* HIP runtime error (message in mcpt_last_error) */
    MCPT_ERR_NOT_CONVERGED = -4, /* max_sweeps reached with residual >= tol */
    MCPT_ERR_DIVERGED = -5,      /* residual non-finite, > 1e6 x first, or 3 rises above first */
    MCPT_ERR_NONFINITE = -6,     /* NaN or Inf in the inputs */
    MCPT_ERR_ADMISSION = -7,     /* problem larger than the free part of the context's HBM budget */
    MCPT_ERR_UNKNOWN_ID = -8     /* no resident problem / ticket with that id */
} mcpt_status;

/* Arithmetic of the pair contractions (Eqs. 58-59).  Denominators, residual,
 * energies and the monomer update are FP64 in every mode.  Reduced precision
 * with polish = 1 is defect correction: each FP64 sweep gives the FP64 residual
 * r = F(T) - T (the convergence test), then inner_sweeps reduced-precision sweeps
 * of the homogeneous equation delta = r + L(delta) (no integral source terms)
 * give the correction T += delta; the final energies come from an FP64 pass.
 * With polish = 0 the reduced-precision sweeps iterate Eqs. 58-59 directly. */
typedef enum {
    MCPT_FP64 = 0,               /* FP64 MFMA */
    MCPT_FP32 = 1,               /* FP32 MFMA, FP32 accumulation */
    MCPT_BF16 = 2                /* BF16 MFMA inputs, FP32 accumulation */
} mcpt_precision;

typedef enum {
    MCPT_HOST = 0,               /* eps, k_intra, v_dimer are host pointers */
    MCPT_DEVICE = 1              /* eps, k_intra, v_dimer are device pointers on the context's GPU */
} mcpt_memory;

typedef struct mcpt_ctx mcpt_ctx;   /* opaque: device, stream, resident problems */

/* One cluster: monomer orbital energies and intra-monomer integrals from
 * step 1-2 of the program flow, the cutoff pair list and the dimer blocks of
 * step 2 (Eq. 29).  All offsets are implied by n_occ, n_vir and pair. */
typedef struct {
    int32_t        n_mono;   /* N >= 1 */
    const int32_t *n_occ;    /* [N] o_X >= 1 (host) */
    const int32_t *n_vir;    /* [N] v_X >= 1 (host) */
    const double  *eps;      /* sum_X (o_X + v_X): per monomer o_X occupied then v_X virtual energies, Eh */
    const double  *k_intra;  /* sum_X o_X^2 v_X^2: K_X[i][j][a][b] = <ab|ij>, row-major, monomers concatenated */
    int64_t        n_pair;   /* P >= 0 */
    const int32_t *pair;     /* [P][2] (X, Y), X != Y, each unordered pair at most once (host) */
    const double  *v_dimer;  /* sum_p o_X v_X o_Y v_Y: V_XY[i][a][j][b] = (ai|bj), i,a on X, j,b on Y, row-major, pairs concatenated */
    int32_t        memory;   /* mcpt_memory of eps, k_intra, v_dimer */
} mcpt_problem;

typedef struct {
    double         tol;          /* > 0: stop at the first sweep with max|T_new - T| < tol;
                                    == 0: run exactly max_sweeps sweeps (no convergence test) */
    int32_t        max_sweeps;   /* >= 0 */
    int32_t        precision;    /* mcpt_precision of the pair contractions */
    int32_t        polish;       /* reduced precision: 1 = FP64 defect-correction sweeps until the
                                    FP64 residual < tol; 0 = stop at the reduced-precision residual */
    int32_t        deterministic;/* 0: the pair contributions to G (Eq. 58) are added with FP64 atomics,
                                    results repeat to rounding; 1: each pair stores its blocks and a
                                    per-monomer pass sums them in pair order, results repeat bitwise
                                    (extra HBM: sum over pairs of (npX^2 + npY^2) doubles) */
    int32_t        check_every;  /* sweeps issued between host checks of the device residual (>= 1) */
    int32_t        inner_sweeps; /* reduced precision + polish: correction sweeps per FP64 sweep
                                    (0 = default: 4 for BF16, 6 for FP32) */
    const double  *warm_t;       /* NULL, or host T (layout of t_amp in mcpt_energy) to start from */
    int32_t        graph;        /* 1: capture the sweeps issued between host checks in a HIP graph and
                                    replay it (per-launch timing is not recorded then) */
    int32_t        autotune;     /* reduced precision: 1 = if the context has no tile choice for this
                                    problem's pair-shape mix, run mcpt_autotune first; 0 = use the
                                    context's choice or the default tile shape */
} mcpt_options;

typedef struct {
    double  e_total;        /* e_mono + e_dimer, Eh */
    double  e_mono;         /* sum_X E_M2(X) (Eq. 54) */
    double  e_dimer;        /* sum over unordered pairs of E_D2(XY) (Eq. 55) */
    double  e_mono0;        /* sum_X E_M2 at zero coupling (reference of Eq. 56) */
    double  residual;       /* max|T_new - T| of the last sweep */
    double  seconds;        /* wall time of the solve on the host */
    int32_t sweeps;         /* sweeps run (reduced-precision + FP64 polish) */
    int32_t polish_sweeps;  /* of which FP64 residual sweeps in polish mode */
    int32_t status;         /* mcpt_status of this solve */
    int32_t iso_sweeps;     /* full monomer equation (mcpt_lccd_attach): sweeps of the isolated-monomer
                               LCCD of step 5; 0 otherwise */
} mcpt_summary;

/* Per-launch kernel timing, recorded with HIP events on the context's stream
 * while enabled (mcpt_set_timing). */
typedef struct {
    double  pair_ms;        /* summed duration of pair-phase launches (Eqs. 58-59 contractions) */
    double  mono_ms;        /* summed duration of monomer-phase launches */
    int64_t pair_launches;
    int64_t mono_launches;
    double  pair_flops;     /* algorithmic flops of the timed pair launches: 4 nX nY (nX + nY) per pair
                               with coupling, 2 nX nY (nX + nY) for energy-only passes */
    double  pair_v_bytes;   /* dimer-block bytes those launches streamed (sizeof element x nX nY per pair) */
    double  lowp_ms;        /* summed duration of reduced-precision pair-phase launches */
    int64_t lowp_launches;
    double  lowp_flops;     /* algorithmic flops of those launches (4 nX nY (nX + nY) per pair) */
    double  lowp_v_bytes;   /* bytes of the reduced-precision dimer blocks (V and V^T) they read */
    double  singles_ms;     /* summed duration of singles pair-phase launches (mcpt_singles) */
    int64_t singles_launches;
    double  singles_v_bytes;/* dimer-block bytes those launches streamed (8 nX nY per pair) */
    double  lccd_ring_ms;   /* full monomer equation: summed duration of the ring-product launches */
    double  lccd_ladder_ms; /* summed duration of the ladder launches (particle-particle ladder, hole-hole
                               ladder and assembly of the intramonomer terms) */
    int64_t lccd_launches;  /* ladder launches */
    double  lccd_w_bytes;   /* <ab|cd> integral bytes those launches streamed (8 v^4 per monomer, rows
                               padded to 16) */
    double  lccd_ladder_flops; /* algorithmic flops of their particle-particle ladders (2 o^2 v^4 per monomer) */
    double  dimer_ladder_ms;/* dimer-internal terms (mcpt_dimer_attach): summed duration of the pair ladder
                               launches (X-vv|Y-vv and oo|oo ladders of Eq. 59) */
    double  dimer_ring_ms;  /* summed duration of the dimer ring launches (monomer and cross rings of Eq. 59) */
    int64_t dimer_launches; /* pair ladder launches */
    double  dimer_w_bytes;  /* <a b|a1 b1> integral bytes those launches streamed (8 vX vY vX vY per pair,
                               rows padded to 16) */
    double  dimer_ladder_flops; /* algorithmic flops of their X-vv|Y-vv ladders (2 oX oY vX^2 vY^2 per pair) */
} mcpt_timing;

/* Create a context on HIP device `device`; at most hbm_budget_bytes of device
 * memory are used for resident problems (0 = 90% of free memory).
 * Errors: MCPT_ERR_INVALID (no such device), MCPT_ERR_DEVICE. */
mcpt_status mcpt_create(int device, size_t hbm_budget_bytes, mcpt_ctx **out);

/* Free every resident problem, the stream and the context.  NULL is a no-op. */
void mcpt_destroy(mcpt_ctx *ctx);

/* Message of the last error on this thread ("" if none). */
const char *mcpt_last_error(void);

/* Use an existing HIP stream (hipStream_t, e.g. a PyTorch stream) for all
 * later work of this context; NULL restores the context's own stream. */
mcpt_status mcpt_set_stream(mcpt_ctx *ctx, void *hip_stream);

/* Validate a problem and copy it to the device (program-flow step 2 output:
 * energies, integrals, pair list).  Builds the packed monomer layout and the
 * pair table; the result stays resident under *id.
 * Errors: MCPT_ERR_INVALID (sizes, pairs out of range, X == Y, duplicate
 * pair, max occupied energy >= min virtual energy of a monomer),
 * MCPT_ERR_NONFINITE, MCPT_ERR_ADMISSION, MCPT_ERR_NOMEM, MCPT_ERR_DEVICE. */
mcpt_status mcpt_upload(mcpt_ctx *ctx, const mcpt_problem *prob, uint64_t *id);

/* Solve a resident problem (step 6: macro iterations of Eqs. 58-59 until
 * converged, then Eqs. 54-56).  Writes *out (may be NULL).  Returns the
 * solve's status: MCPT_OK, MCPT_ERR_NOT_CONVERGED (results are those of the
 * last sweep), MCPT_ERR_DIVERGED (no results), MCPT_ERR_INVALID (options),
 * MCPT_ERR_UNKNOWN_ID, MCPT_ERR_DEVICE. */
mcpt_status mcpt_run(mcpt_ctx *ctx, uint64_t id, const mcpt_options *opts, mcpt_summary *out);

/* For callers that cannot allocate device memory (code running under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mcpt_run of
 * a resident problem in FP64 (eager sweeps; precision MCPT_FP64, deterministic
 * 0 and graph 0, else MCPT_ERR_INVALID) that allocates nothing.  The Tau
 * scratch of the pair kernels - one slot of the largest pair's padded
 * np_X x np_Y doubles per persistent workgroup - comes from a fixed
 * library-owned device array of MCPT_STATIC_SCRATCH_BYTES instead of the
 * context's allocated scratch; the grid is limited to the slots that fit.  A
 * problem whose largest slot alone exceeds it is rejected (MCPT_ERR_INVALID).
 * Each GPU keeps its own copy of the array until the process ends; every call
 * on one GPU uses that copy, so calls that overlap on a GPU (several contexts
 * or threads) race.  Results, outputs and errors otherwise as mcpt_run (FP64
 * atomics in the pair kernels: equal to mcpt_run to rounding, not bitwise). */
#define MCPT_STATIC_SCRATCH_BYTES (64ull << 20)
mcpt_status mcpt_run_static(mcpt_ctx *ctx, uint64_t id, const mcpt_options *opts, mcpt_summary *out);

/* Batching form: upload n independent clusters (probs[0..n-1], e.g. clusters
 * of different sizes and orbital counts) as one resident problem.  A run then
 * sweeps all of them together - every pair phase is one persistent launch over
 * the pairs of every live cluster (FP64: one launch for the pairs whose V
 * block fits in LDS and one for the rest) - while each cluster keeps its own
 * convergence test, so it stops at the same sweep as it would alone and its
 * results equal its solo solve.  mcpt_energy returns the clusters' arrays
 * concatenated in input order; mcpt_cluster_results gives per-cluster
 * summaries.  Errors as mcpt_upload (the message names the cluster). */
mcpt_status mcpt_upload_batch(mcpt_ctx *ctx, const mcpt_problem *probs, int32_t n, uint64_t *id);

/* mcpt_upload_batch followed by mcpt_run; per_cluster[n] (may be NULL) receives
 * each cluster's summary.  Returns the worst cluster status. */
mcpt_status mcpt_solve_batch(mcpt_ctx *ctx, const mcpt_problem *probs, int32_t n, const mcpt_options *opts,
                             uint64_t *id, mcpt_summary *per_cluster);

/* Per-cluster summaries of the last run of a resident batch (n = its cluster
 * count; a single upload is a batch of one).
 * Errors: MCPT_ERR_UNKNOWN_ID, MCPT_ERR_INVALID (wrong n, never run). */
mcpt_status mcpt_cluster_results(mcpt_ctx *ctx, uint64_t id, int32_t n, mcpt_summary *out);

/* mcpt_upload followed by mcpt_run; the problem stays resident under *id. */
mcpt_status mcpt_solve(mcpt_ctx *ctx, const mcpt_problem *prob, const mcpt_options *opts,
                       uint64_t *id, mcpt_summary *out);

/* Per-monomer and per-pair results of the last run of a resident problem.
 * e_m2[N]: E_M2(X) (Eq. 54); de_m2[N]: E_M2(X) minus its zero-coupling value
 * (Eq. 56); e_d2[P]: E_D2 of each stored pair (Eq. 55); t_amp[sum_X o^2 v^2]:
 * T_X[i][j][a][b] = T^{ab}_{ij}, monomers concatenated.  Any may be NULL.
 * Errors: MCPT_ERR_UNKNOWN_ID, MCPT_ERR_INVALID (never run), MCPT_ERR_DEVICE. */
mcpt_status mcpt_energy(mcpt_ctx *ctx, uint64_t id, double *e_m2, double *de_m2, double *e_d2,
                        double *t_amp);

/* Free a resident problem. Errors: MCPT_ERR_UNKNOWN_ID. */
mcpt_status mcpt_release(mcpt_ctx *ctx, uint64_t id);

/* ---- Singles amplitudes (Eq. 57, program-flow step 4) ----
 * With the terms the inputs can form - the embedding source w and the pair sum
 * over neighbours Y of v^{ak}_{ic} t^c_k, where v^{ak}_{ic} = (ai|ck) =
 * V_XY[i][a][k][c] is the resident dimer block (the reversed pair uses V_XY^T),
 * summed over both spins of k, c (a factor 2); and, when the intramonomer
 * classes are attached (mcpt_lccd_attach), the intramonomer term
 * (2 v^{a i1}_{i a1} - v^{a i}_{a1 i1}) t^{a1}_{i1} with v^{a i1}_{i a1} =
 * K[i][i1][a][a1] and v^{a i}_{a1 i1} = (a a1|i i1) = J[i][i1][a][a1] - a sweep
 * is t_X = (w_X + 2 sum_Y V_XY t_Y [+ (2K - J) t_X]) / (e_i - e_a) for every
 * monomer from the previous t (Jacobi), from the first-order start
 * t = w / (e_i - e_a).  Each cluster of a batch stops on its own
 * max|t_new - t| < tol (tol == 0: exactly max_sweeps sweeps) under the divergence
 * rule of mcpt_run; then E_M1(X) = 2 w.t_X (Eq. 53).  Singles and doubles are
 * independent equations: mcpt_singles neither reads nor changes the doubles
 * amplitudes or results of the problem. */
typedef struct {
    double  e_m1;        /* sum over monomers of E_M1(X) */
    double  e_m1_0;      /* the same at the first-order amplitudes (zero coupling) */
    double  residual;    /* largest last residual over clusters */
    double  seconds;     /* wall time of the call */
    int32_t sweeps;      /* most sweeps of any cluster */
    int32_t status;      /* mcpt_status of the solve (worst cluster) */
} mcpt_singles_summary;

/* Solve the singles of a resident problem.  w: sum_X o_X v_X values
 * w_X[i][a] = w^a_i (the occupied-virtual block of the embedding operator of
 * Eq. 26), monomers concatenated in upload order, on the host or (memory =
 * MCPT_DEVICE) on the context's GPU; read before the call returns.  opts: tol,
 * max_sweeps and check_every are used; precision must be MCPT_FP64 and
 * deterministic 0; the other fields are ignored.  Writes *out (may be NULL).
 * Returns the solve status as mcpt_run does; also MCPT_ERR_NONFINITE (w not
 * finite), MCPT_ERR_ADMISSION (the singles buffers - three vectors of
 * sum_X n_X doubles padded as the monomer matrices' rows, three of N doubles
 * and a 32 KiB residual history per cluster, made on the first call and kept
 * with the problem - exceed the budget), MCPT_ERR_INVALID (options),
 * MCPT_ERR_UNKNOWN_ID, MCPT_ERR_DEVICE. */
mcpt_status mcpt_singles(mcpt_ctx *ctx, uint64_t id, const double *w, int32_t memory, const mcpt_options *opts,
                         mcpt_singles_summary *out);

/* Results of the last mcpt_singles of a resident problem: e_m1[N] = E_M1(X)
 * and t1[sum_X o_X v_X] = t_X[i][a] = t^a_i, monomers concatenated; either may
 * be NULL.  Errors: MCPT_ERR_UNKNOWN_ID, MCPT_ERR_INVALID (no singles result:
 * never solved, or diverged), MCPT_ERR_DEVICE. */
mcpt_status mcpt_singles_result(mcpt_ctx *ctx, uint64_t id, double *e_m1, double *t1);

/* ---- Full monomer equation (Eq. 58 with its intramonomer terms; step 5) ----
 * With these integral classes attached, mcpt_run solves the monomer doubles of
 * Eq. 58 with every printed term: besides the source and the pair term, the
 * particle-particle ladder v^{a a1}_{a2 a3} T^{a2 a3}_{i i1}, the hole-hole
 * ladder v^{i2 i3}_{i i1} T^{a a1}_{i2 i3} and the four ring combinations,
 * whose exchange-type integrals v^{a i2}_{i a2} = v^{i2 a}_{a2 i} are read from
 * K (real orbitals: (ai|kc) = (ai|ck)) and whose Coulomb-type integrals
 * v^{a i2}_{a2 i} = (a a2|i2 i) from J.  Each run first iterates every
 * monomer's equation without the pair term (step 5, the isolated-monomer LCCD,
 * same tol, max_sweeps and stopping rule), keeps E_LCCD(X) = E_M2 of that
 * solution as the reference of Eq. 56 (mcpt_energy's de_m2 and the summary's
 * e_mono0), then runs the coupled sweeps (step 6) from the first-order
 * amplitudes: pair phase (Eq. 59), intramonomer terms from the current T,
 * monomer update.  Reduced precision (with or without polish), HIP-graph
 * capture and batches work as for mcpt_run; the intramonomer terms are formed
 * in FP64 in every sweep, and in polish mode also for each correction (of the
 * correction's own amplitudes); step 5 runs in FP64.  No deterministic mode.  Dimer amplitudes keep the terms of Eq. 59
 * listed at the top (its dimer-internal terms need dimer integral classes that
 * are not inputs).  Sizes per monomer: o <= 8, v <= 64 and o v <= 1024. */
typedef struct {
    const double *w_vvvv;   /* sum_X v_X^4: W_X[a][b][c][d] = <ab|cd>, row-major, monomers in upload order */
    const double *q_oooo;   /* sum_X o_X^4: Q_X[i][j][k][l] = <ij|kl> */
    const double *j_oovv;   /* sum_X o_X^2 v_X^2: J_X[i][j][a][b] = <ia|jb> = (ij|ab) */
    int32_t       memory;   /* mcpt_memory of the three arrays */
} mcpt_lccd_integrals;

/* Attach (ints != NULL) or detach (NULL) the intramonomer integral classes of
 * a resident problem.  The arrays are read before the call returns; the packed
 * copies (W as v^2 x v^2 rows padded to 16: ~8 v^4 bytes per monomer), Q, the
 * packed J and three np x np term buffers per monomer stay with the problem
 * and count against the budget.  The problem's last results are dropped.
 * Errors: MCPT_ERR_INVALID (NULL array, memory, monomer sizes),
 * MCPT_ERR_NONFINITE, MCPT_ERR_ADMISSION, MCPT_ERR_NOMEM, MCPT_ERR_UNKNOWN_ID,
 * MCPT_ERR_DEVICE.  mcpt_run of an attached problem returns MCPT_ERR_INVALID
 * for deterministic = 1, and MCPT_ERR_DIVERGED (no results) when step 5
 * diverges for any cluster. */
mcpt_status mcpt_lccd_attach(mcpt_ctx *ctx, uint64_t id, const mcpt_lccd_integrals *ints);

/* ---- Dimer-internal terms of the dimer equation (Eq. 59) ----
 * The terms of Eq. 59 that act on the dimer amplitudes themselves: the
 * X-vv|Y-vv ladder v^{ab}_{a1 b1} Tau^{a1 b1}_{ij}, the oo|oo ladder
 * v^{i1 j1}_{ij} Tau^{ab}_{i1 j1}, the cross rings -v^{b i1}_{b1 i} Tau^{a b1}_{i1 j}
 * and -v^{a j1}_{a1 j} Tau^{a1 b}_{i j1}, and the monomer rings
 * (2 v^{i1 a}_{a1 i} - v^{a i1}_{a1 i}) Tau^{a1 b}_{i1 j} and their Y mirror (K and
 * the J of mcpt_lccd_attach).  With them Tau is an unknown of its own: each
 * coupled sweep forms Eq. 59 from the current T and the previous sweep's Tau
 * (zero before the first), then Eq. 58 from the new Tau; the final energies use
 * one more Eq. 59 step.  Per stored pair (X its first monomer), all row-major
 * FP64, concatenated over the pairs in the caller's pair order: */
typedef struct {
    const double *w_vvvv;   /* vX vY vX vY: W_XY[a][b][a1][b1] = <a b|a1 b1> = (a a1|b b1) */
    const double *q_oooo;   /* oX oY oX oY: Q_XY[i1][j1][i][j] = <i1 j1|i j> = (i1 i|j1 j) */
    const double *c_x;      /* oX oX vY vY: C_X[i1][i][b][b1] = (i1 i|b b1) */
    const double *c_y;      /* oY oY vX vX: C_Y[j1][j][a][a1] = (j1 j|a a1) */
    int32_t       memory;   /* mcpt_memory of the four arrays */
} mcpt_dimer_integrals;

/* Attach (ints != NULL) or detach (NULL) the dimer classes of a resident
 * problem whose intramonomer integrals are attached (mcpt_lccd_attach; detaching
 * those, or attaching them again, detaches these too).  Every monomer must have
 * o <= 8 and v <= 64 (the two monomers of a pair may differ in size), and the
 * problem at most 65,535 pairs.  When every monomer has one size whose n x n
 * Tau fits 160 KiB of LDS (o = 5, v = 27 is 146 KB) with o^2 <= 48, the pair
 * ladder stages each pair's Tau in LDS; otherwise it reads Tau from global
 * memory.  The classes of the pairs are concatenated in the caller's pair
 * order, each with its own pair's sizes.  The arrays are read
 * before the call returns; the packed copies (W_XY as vX vY rows padded to 16,
 * columns to 32: ~8 (vX vY)^2 bytes per pair), Q_XY, the packed C_X and C_Y
 * (oX vY and oY vX square, padded to 16), per pair Tau and the
 * ladder-plus-monomer-ring source S (npX x npY each) and the two cross-ring
 * products Y1, Y2 (oX vY x oY vX and its transpose shape, padded), and one
 * np x np matrix per monomer (2K - J of the monomer rings) stay with the
 * problem and count against the budget.  The
 * problem's last results are dropped.  mcpt_run of an attached problem accepts
 * only the FP64 form (precision MCPT_FP64) and has no deterministic mode: its
 * results are reproducible to rounding only (the pair kernel adds the G_X and
 * G_Y contributions with FP64 atomics; the dimer terms themselves use none).
 * Errors: MCPT_ERR_INVALID (NULL array, memory, no intramonomer integrals,
 * sizes), MCPT_ERR_NONFINITE, MCPT_ERR_ADMISSION, MCPT_ERR_NOMEM,
 * MCPT_ERR_UNKNOWN_ID, MCPT_ERR_DEVICE. */
mcpt_status mcpt_dimer_attach(mcpt_ctx *ctx, uint64_t id, const mcpt_dimer_integrals *ints);

/* Dimer amplitudes of the last run of a problem with the dimer terms attached:
 * the Tau of the final Eq. 59 step, from which E_D2 is formed (Eq. 55).
 * tau[sum over pairs of oX vX oY vY] (caller-allocated) receives
 * Tau_XY[i][a][j][b] = Tau^{ab}_{ij} (i, a on the pair's first monomer),
 * row-major, pairs concatenated in the caller's pair order.
 * Errors: MCPT_ERR_INVALID (NULL, no dimer terms attached, never run),
 * MCPT_ERR_UNKNOWN_ID, MCPT_ERR_DEVICE. */
mcpt_status mcpt_dimer_tau(mcpt_ctx *ctx, uint64_t id, double *tau);

/* ---- Finite-displacement geometries (Sec. IV.A: harmonic frequencies from
 * single points on a five-point grid, step 0.01 A in the paper) ----
 * A displaced geometry keeps every monomer's energies and intra block and the
 * undisplaced pair list; only the dimer couplings of the moved monomers
 * change, V_XY -> (R0 / R)^3 V_XY for the caller's coupling model.  Both calls
 * build displaced problems on the device from a resident base problem, with
 * no host upload. */

/* New resident problem *id: the resident problem `base` with the blocks of the
 * listed pairs (indices into base's pair list, each at most once) multiplied
 * by scale[k] (finite).  Arrays are read before the call returns.  The copy
 * holds its own device memory (as much as the base's plain upload) until
 * mcpt_release; it carries the base's inputs only (not its results, singles
 * source or attached intramonomer integrals).  Errors: MCPT_ERR_INVALID (NULL array, index out of range or
 * repeated), MCPT_ERR_NONFINITE, MCPT_ERR_ADMISSION, MCPT_ERR_NOMEM,
 * MCPT_ERR_UNKNOWN_ID, MCPT_ERR_DEVICE. */
mcpt_status mcpt_upload_scaled(mcpt_ctx *ctx, uint64_t base, int64_t n, const int64_t *pair, const double *scale,
                               uint64_t *id);

typedef struct {
    int64_t        n_pair;   /* pairs whose blocks the displacement rescales */
    const int64_t *pair;     /* [n_pair] indices into the base problem's pair list */
    const double  *scale;    /* [4][n_pair] factors at the displacements -2h, -h, +h, +2h */
} mcpt_fd_mode;

typedef struct {
    double  e[5];            /* unit energy at -2h, -h, 0, +h, +2h, Eh */
    double  d2e;             /* (-e[4] + 16 e[3] - 30 e[2] + 16 e[1] - e[0]) / (12 step^2) */
    int32_t sweeps[5];       /* doubles sweeps of each point */
    int32_t status;          /* mcpt_status of the mode */
    int32_t reserved;
} mcpt_fd_result;

/* Five-point second derivatives of the unit energy of Eq. 66 along
 * displacement modes.  The unit energy of a geometry is the sum over the n_cell
 * listed monomers of E_M2(X) (Eq. 54) and, when w is not NULL (host, the
 * singles source of mcpt_singles), of E_M1(X) (Eq. 53); the E_SCF(X) of Eq. 66
 * does not change with these displacements (monomer integrals are fixed) and
 * is left out.  The base problem is solved first (opts; its results stay, as
 * after mcpt_run); each displaced point is a scaled copy (mcpt_upload_scaled)
 * solved from the base's converged amplitudes (warm start), then released.
 * opts->warm_t must be NULL.  step is the displacement h (any length unit; d2e
 * is per unit squared).  out[n_modes] receives the results.  Returns the first
 * failing status (the message names mode and point); a base problem with
 * intramonomer integrals attached is rejected (MCPT_ERR_INVALID). */
mcpt_status mcpt_fd_stencil(mcpt_ctx *ctx, uint64_t base, int32_t n_modes, const mcpt_fd_mode *modes,
                            int32_t n_cell, const int32_t *cell, double step, const double *w,
                            const mcpt_options *opts, mcpt_fd_result *out);

/* ---- Device characterization (roofline reporting; not part of the method) ----
 * Sustained FP64 rates of the device, measured with register-only streams of
 * independent operations at two waves per SIMD (the FP64 pair kernel's
 * occupancy): v_mfma_f64_16x16x4 alone, and v_fma_f64 alone, in algorithmic
 * TFLOP/s; the shader clock from the core clock counter against the 100 MHz
 * real-time counter (of the last stream).  Allocates and frees its own small
 * buffers on the device; takes ~0.1 s.
 * Errors: MCPT_ERR_INVALID (no such device, NULL), MCPT_ERR_NOMEM, MCPT_ERR_DEVICE. */
typedef struct {
    double  mfma_f64_tflops;
    double  valu_f64_tflops;
    double  clock_ghz;
    int32_t compute_units;
} mcpt_rates;
mcpt_status mcpt_device_rates(int device, mcpt_rates *out);

/* ---- Tile autotuner of the reduced-precision pair kernel ----
 * The kernel exists in several tile shapes: each wave computes sb x sb output
 * tiles of 16 x 16 per task, nw waves per workgroup, pd k chunks loaded ahead.  mcpt_autotune times one
 * coupled pair phase of the resident problem per shape and keeps the fastest,
 * for this problem and, under its pair-shape key (block shapes and their share
 * of the flops, pair count to a power of two), for every later problem of the
 * context with the same key.  It overwrites the problem's last results (run it
 * again afterwards).  The table can be saved and restored as text lines
 * "key sb nw pd". */
typedef struct {
    int32_t n_variants;     /* shapes timed */
    int32_t best;           /* index of the fastest */
    int32_t sb[16], nw[16]; /* tiles per task edge and waves per workgroup of each */
    int32_t pd[16];         /* k chunks of operand fragments loaded ahead of the MFMAs */
    int32_t reserved;
    double  ms[16];         /* one coupled pair phase, milliseconds */
} mcpt_tune_result;

/* Errors: MCPT_ERR_INVALID (precision not FP32 / BF16), MCPT_ERR_UNKNOWN_ID, MCPT_ERR_DEVICE. */
mcpt_status mcpt_autotune(mcpt_ctx *ctx, uint64_t id, int32_t precision, mcpt_tune_result *out);

/* Write the tuning table as text into buf (capacity cap, may be NULL); *len = bytes needed
 * including the terminating NUL.  Errors: MCPT_ERR_INVALID (buffer too small). */
mcpt_status mcpt_tune_export(mcpt_ctx *ctx, char *buf, size_t cap, size_t *len);

/* Add the lines of an exported table.  Errors: MCPT_ERR_INVALID (malformed line, unknown shape). */
mcpt_status mcpt_tune_import(mcpt_ctx *ctx, const char *text);

/* Enable (1) or disable (0) per-launch kernel timing; enabling resets the totals. */
mcpt_status mcpt_set_timing(mcpt_ctx *ctx, int enable);

/* Read the timing totals since timing was enabled. */
mcpt_status mcpt_timing_read(mcpt_ctx *ctx, mcpt_timing *out);

/* ---- Serving form: continuous batching of arriving solves ----
 *
 * Requests (clusters of any size, e.g. finite-displacement geometries of the
 * workflow that sums MCPT(2) energies over displaced structures) are queued
 * by mcpt_submit and solved by the context's worker threads, each on its own
 * HIP stream.  A free worker admits the oldest queued request once its device
 * footprint (the bytes mcpt_upload and, for reduced precision, the
 * reduced-precision copies would allocate) fits in the HBM budget beside the
 * resident problems and the reservations of the other workers, and fuses into
 * the same batch later queued requests with the same options and a pair-phase
 * cost within a factor of four of it, while they fit.  The batch runs as an
 * mcpt_upload_batch problem, so each request's result is the one its own
 * solve gives.  Requests that arrive while batches run are taken by the next
 * free worker, and the workers' batches run concurrently on the device.  FP64
 * batches retire each request at the sweep tick where its solve stops and can
 * also admit queued requests there (mcpt_serve_tick_mode).
 * Results stay resident until mcpt_release(ticket); they count against the
 * budget, so admission waits while released memory is needed.
 */
typedef struct {
    uint64_t completed;         /* requests finished since the scheduler started */
    uint64_t batches;           /* batches run */
    uint64_t budget;            /* HBM budget of the context, bytes */
    uint64_t bytes_in_use;      /* device bytes of resident problems and results */
    uint64_t bytes_reserved;    /* bytes reserved by workers for uploads in progress */
    int32_t  queued;            /* requests waiting for admission */
    int32_t  running_batches;   /* batches on the device now */
    int32_t  workers;           /* worker threads (0 before the first submission) */
    int32_t  tickets;           /* live tickets (queued, running or holding results) */
    uint64_t staging_pinned_bytes;  /* pinned host staging held for request copies */
    uint64_t staged_pageable;   /* request arrays copied to pageable memory (staging full) */
    uint64_t joined_at_ticks;   /* requests admitted into running batches at sweep ticks */
} mcpt_serve_counters;

/* Scheduler parameters; only before the first mcpt_submit of the context.
 * workers: concurrent batches (streams), 1..16 (default 4); max_batch:
 * requests per batch, 1..4096 (default 32); max_batch_pairs: pairs per batch
 * (default 2^20).  Errors: MCPT_ERR_INVALID (range, scheduler running). */
mcpt_status mcpt_serve_config(mcpt_ctx *ctx, int32_t workers, int32_t max_batch, int64_t max_batch_pairs);

/* What a served batch of FP64 plain sweeps (no graph, deterministic mode or warm
 * start) does at its sweep ticks, the host checks after every check_every sweeps;
 * only before the first mcpt_submit of the context.
 *   MCPT_SERVE_BATCH_END: nothing; every request of the batch is reported when the
 *     last one stops, as for other options.
 *   MCPT_SERVE_RETIRE_AT_TICKS (default): a request whose solve has stopped retires
 *     at that tick: its energies are computed (the energy pass over its pairs only)
 *     and it is reported while the batch's other requests go on; its results stay
 *     in the batch's memory until its ticket is released.
 *   MCPT_SERVE_JOIN_AT_TICKS: as RETIRE, and while every worker is busy and at most
 *     as many requests are queued as there are workers, requests at the head of the
 *     queue with the same options and a pair-phase cost within a factor of four of
 *     the batch's first request join it, in queue order, within max_batch,
 *     max_batch_pairs and the budget (each priced at twice its footprint while it
 *     comes in), if together they are at least as large as the batch's unfinished
 *     requests: they are uploaded on a second stream of the worker while the batch
 *     keeps sweeping, then copied with the unfinished clusters, whose iteration state
 *     is kept, into one batch that the next sweeps run as one launch per kernel.
 *     Measured on a served stream of mixed sizes, this shortens the median latency
 *     at moderate load and costs capacity and tail latency.
 * In every mode a request's sweeps and result are those of its own solve (to the
 * rounding of the G atomics).  Errors: MCPT_ERR_INVALID (unknown mode, scheduler
 * running). */
enum { MCPT_SERVE_BATCH_END = 0, MCPT_SERVE_RETIRE_AT_TICKS = 1, MCPT_SERVE_JOIN_AT_TICKS = 2 };
mcpt_status mcpt_serve_tick_mode(mcpt_ctx *ctx, int32_t mode);

/* Host staging of submitted requests; only before the first mcpt_submit of the
 * context.  mcpt_submit copies a request's integral arrays into pinned host
 * blocks (power-of-two sizes from 1 MiB, made with hipHostMalloc on first need
 * and reused by later requests), so the copy lands in pages that exist and the
 * worker's upload is a DMA transfer; bytes caps the pinned memory held (default
 * 16 GiB; 0: every request is copied to ordinary pageable memory, as it is when
 * the cap is reached).  The blocks are freed with the context.
 * Errors: MCPT_ERR_INVALID (scheduler running). */
mcpt_status mcpt_serve_staging(mcpt_ctx *ctx, uint64_t bytes);

/* Queue one solve.  The problem (host memory only) and options are checked and
 * copied before the call returns; *ticket names the request in mcpt_poll,
 * mcpt_wait, and, once done, mcpt_energy and mcpt_release.
 * Errors: MCPT_ERR_INVALID, MCPT_ERR_NONFINITE (as mcpt_upload, plus device
 * memory), MCPT_ERR_ADMISSION (footprint larger than the whole budget). */
mcpt_status mcpt_submit(mcpt_ctx *ctx, const mcpt_problem *prob, const mcpt_options *opts, uint64_t *ticket);

/* MCPT_PENDING while the request is queued or running; MCPT_OK once done, with
 * *out (may be NULL) its summary: status is the solve's status (OK,
 * NOT_CONVERGED, DIVERGED, or the error that stopped its batch, described by
 * mcpt_last_error after this call) and seconds is the latency from submission
 * to result.  Errors: MCPT_ERR_UNKNOWN_ID. */
mcpt_status mcpt_poll(mcpt_ctx *ctx, uint64_t ticket, mcpt_summary *out);

/* As mcpt_poll, blocking up to timeout_ms milliseconds (< 0: no limit). */
mcpt_status mcpt_wait(mcpt_ctx *ctx, uint64_t ticket, int32_t timeout_ms, mcpt_summary *out);

/* Scheduler counters and memory accounting. */
mcpt_status mcpt_serve_stats(mcpt_ctx *ctx, mcpt_serve_counters *out);

#ifdef __cplusplus
}
#endif

#endif /* MCPT_H */
