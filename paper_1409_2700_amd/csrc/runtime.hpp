// Host runtime of libmcpt (not part of the C ABI): resident problems, the
// per-stream execution resources, the context, and the serving scheduler's
// request table.
//
// Threading: every field of mcpt_ctx marked "mu" is read and written under
// ctx->mu.  A resident problem is used by one thread at a time: the client
// thread for problems it uploaded, one serving worker for a served batch.
#pragma once

#include <array>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mcpt.h"
#include "host.hpp"
#include "lccd.hpp"
#include "mcpt_internal.hpp"

namespace mcpt {

struct Resident {
    uint64_t id = 0;
    int n_mono = 0;
    int64_t n_pair = 0;
    int max_n = 0, max_np = 0, max_v = 0;   // largest n, padded n and virtual count over monomers
    int64_t eps_elems = 0, dif_elems = 0, raw_elems = 0, mat_elems = 0, v_elems = 0, max_slot = 0;
    std::vector<MonoDesc> monos;
    std::vector<PairDesc> pairs;      // LDS-variant pairs, then the others; each range sorted by
                                      // monomer for locality; .orig is the caller's index
    int64_t n_lds = 0;                // pairs served by the LDS-resident-V kernel
    // device
    MonoDesc* d_monos = nullptr;
    PairDesc* d_pairs = nullptr;
    double *d_dif = nullptr, *d_raw = nullptr, *d_K = nullptr, *d_T = nullptr, *d_M = nullptr;
    double *d_G[2] = {nullptr, nullptr};
    double* d_V = nullptr;
    double *d_em2 = nullptr, *d_em2_0 = nullptr, *d_ed2 = nullptr, *d_res = nullptr;
    // clusters of a batch: monomer and pair ranges (caller order), per-cluster state and history
    int n_cl = 1;
    std::vector<int64_t> cl_mono, cl_pair;
    int64_t *d_cl_mono = nullptr, *d_cl_pair = nullptr;
    std::vector<int64_t> cl_v;        // first V element of each cluster (n_cl + 1)
    ClState* d_cl = nullptr;
    double* d_hist = nullptr;
    std::vector<mcpt_summary> cl_last;
    std::vector<int32_t> cl_bad;      // cluster has a non-finite input (served batches only)
    std::vector<void*> allocations;
    size_t bytes = 0;
    bool has_result = false;
    mcpt_summary last{};
    // reduced-precision copies (mixed-precision form), made on first use of a precision
    int lo_prec = 0;
    int lo_variant = 0;           // tile shape of the reduced-precision pair kernel
    int64_t lo_n_lds = 0;         // leading pairs served by the LDS-resident reduced-precision kernel
    int64_t lo_lds_bytes = 0;     // dynamic LDS of that kernel (largest pair of the range)
    std::string shape_key;        // pair-shape signature used by the tile autotuner
    void *d_Vlo = nullptr, *d_Mlo = nullptr;
    int64_t *d_lo_off = nullptr, *d_mlo_off = nullptr;
    double *d_R = nullptr, *d_Dl = nullptr;
    float* d_G32[2] = {nullptr, nullptr};   // BF16 sweeps: G accumulated in FP32 (double-buffered like d_G)
    int64_t lo_slot = 0;          // elements of one low-precision Tau + Tau^T scratch slot
    double lo_v_bytes = 0.0;      // bytes of the low-precision V and V^T
    std::vector<void*> lo_allocations;
    size_t lo_bytes = 0;
    // singles (made on the first mcpt_singles; freed with the problem): vectors in the padded
    // dif layout, per-monomer energies and residuals, per-cluster state and history
    double *d_w1 = nullptr, *d_t1 = nullptr, *d_u1 = nullptr;
    double* d_ui1 = nullptr;          // intramonomer term of Eq. 57 (with the full monomer equation attached)
    double *d_em1 = nullptr, *d_em1_0 = nullptr, *d_res1 = nullptr, *d_hist1 = nullptr;
    ClState* d_cl1 = nullptr;
    int64_t* d_woff = nullptr;        // compact offsets of w per monomer (N + 1)
    bool has_singles = false;
    mcpt_singles_summary singles_last{};
    // full monomer equation (mcpt_lccd_attach): packed intramonomer integrals, the per-sweep
    // term buffers and E_LCCD of step 5; freed by a detach or with the problem
    bool lccd = false;
    std::vector<LccdDesc> lccd_desc;
    LccdDesc* d_lccd = nullptr;
    double *d_W = nullptr, *d_Q = nullptr, *d_J = nullptr;
    double *d_L = nullptr, *d_R12 = nullptr, *d_Y = nullptr, *d_elccd = nullptr;
    int lccd_ring_blocks = 0, lccd_ladder_blocks = 0, lccd_ct = 1;
    int64_t lccd_lds_bytes = 0;       // > 0: the LDS-staged ladder kernel with this much dynamic LDS
    double lccd_w_bytes = 0.0;        // packed-integral bytes the ladder kernel streams per sweep
    double lccd_w_flops = 0.0;        // algorithmic flops of the particle-particle ladder per sweep
    std::vector<void*> lccd_allocations;
    size_t lccd_bytes = 0;
    // dimer-internal terms of Eq. 59 (mcpt_dimer_attach): per pair a MonoDesc / LccdDesc
    // placing its n x n matrices and packed W_XY, Q_XY, so the monomer ladder kernel runs on pairs
    bool dimer = false;
    DimerDesc* d_dd = nullptr;
    MonoDesc* d_pmono = nullptr;
    LccdDesc* d_plccd = nullptr;
    double *d_DW = nullptr, *d_DQ = nullptr, *d_DCX = nullptr, *d_DCY = nullptr, *d_Tau = nullptr, *d_S = nullptr;
    double* d_DRM = nullptr;          // 2 K - J per monomer (the monomer rings of Eq. 59)
    double *d_DY1 = nullptr, *d_DY2 = nullptr;   // the cross-ring products of each pair
    std::vector<DimerDesc> dimer_desc;   // per pair (caller order): sizes and offsets
    int64_t dimer_tau_elems = 0;         // elements of the Tau (and S) buffer
    bool dimer_one_size = false;         // every monomer of one size: Tau, S, Y1, Y2 np x np per pair
    int dimer_ring_blocks = 0, dimer_ct = 1, dimer_ladder_blocks = 1;
    int64_t dimer_lds_bytes = 0;
    double dimer_w_bytes = 0.0, dimer_w_flops = 0.0;
    std::vector<void*> dimer_allocations;
    size_t dimer_bytes = 0;
    // captured sweep graph: valid for one form, one execution resource set and one body count
    hipGraphExec_t graph = nullptr;
    int graph_prec = -1, graph_sweeps = 0, graph_parity = 0;
    std::array<int64_t, 6> graph_key{};   // buffers and grids baked into the captured launches
    // deterministic mode: per-pair partial G blocks and their per-monomer summation lists
    bool det_on = false;
    double* d_part = nullptr;
    int64_t *d_part_off = nullptr, *d_csr_off = nullptr, *d_csr = nullptr;
    std::vector<void*> det_allocations;
    size_t det_bytes = 0;
    // served batches: owned by the scheduler, never visible to the caller under this id
    bool internal = false;
    int refs = 0;                 // tickets still holding this batch's results, + 1 while a worker runs it
    // pairs read from L2 in the split form (launch_pair_fp64_split): per chunk of at most one pair
    // per persistent workgroup, the XCD-grouped pair lists, Tau offsets and task prefixes
    bool glb_plan = false;
    std::vector<GlbTasks> glb_tau, glb_g;
    std::vector<int> glb_n;
    // served batches with admission at sweep ticks: the G buffer the next sweep accumulates
    // into, and the cluster selection of the energy pass of clusters that finished
    int g_cur = 0;
    ClState* d_cl_sel = nullptr;
};

struct Timing {
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
        int kind;   // 0 FP64 pair phase, 1 monomer phase, 2 reduced-precision pair phase, 3 singles pair phase,
                    // 4 intramonomer ring products, 5 intramonomer ladders and assembly
        double flops, vbytes;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    mcpt_timing tot{};
};

// What one stream needs to run solves independently of other streams: the
// control word (device + pinned host copy), the flag used by input checks, and
// the per-workgroup Tau scratch of the pair kernels.
struct Exec {
    hipStream_t stream = nullptr;
    hipStream_t own = nullptr;
    Ctrl* d_ctrl = nullptr;
    Ctrl* h_ctrl = nullptr;             // pinned
    int32_t* d_flag = nullptr;
    int32_t* h_flag = nullptr;          // pinned
    double* d_scratch = nullptr;        // FP64 Tau, one slot per workgroup
    int64_t scratch_slot = 0;
    int scratch_slots = 0;
    bool fixed_scratch = false;         // d_scratch is the library's static array: never reallocated
    int grid_cap = 0;                   // > 0: FP64 pair-kernel grids limited to the slots that fit
    void* d_scratch_lo = nullptr;       // reduced-precision Tau and Tau^T
    size_t scratch_lo_bytes = 0;
    int grid_lo = 0, grid_lo_lds = 0;   // persistent grids of the reduced-precision kernels
    Timing timing;
    size_t reserved = 0;                // HBM reserved by admission for the upload in progress (mu)
};

// One served request: inputs copied at submission, then its place in a batch.
// Pinned host staging of served requests: blocks of power-of-two sizes made with
// hipHostMalloc on first need, up to a cap, and reused for later requests, so a
// submission copies into memory whose pages already exist and the worker's
// upload is a DMA transfer.  take() returns nullptr when the cap is reached.
class PinnedPool {
public:
    ~PinnedPool();
    void set_cap(size_t bytes);
    double* take(size_t bytes);
    void give(double* p);
    size_t held() const;
    uint64_t pageable() const;
    void count_pageable();
private:
    mutable std::mutex mu_;
    size_t cap_ = size_t(16) << 30;
    size_t held_ = 0;
    uint64_t pageable_ = 0;
    std::map<int, std::vector<double*>> free_;   // log2 block size -> free blocks
    std::map<double*, int> cls_;                  // every block -> log2 size
};

// A request's copy of a caller array: a pinned pool block, or ordinary memory
// when the pool is full.
class HostBuf {
public:
    HostBuf() = default;
    HostBuf(double* p, PinnedPool* pool) : p_(p), pool_(pool) {}
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    HostBuf(HostBuf&& o) noexcept : p_(o.p_), pool_(o.pool_) { o.p_ = nullptr; }
    HostBuf& operator=(HostBuf&& o) noexcept {
        if (this != &o) {
            reset();
            p_ = o.p_;
            pool_ = o.pool_;
            o.p_ = nullptr;
        }
        return *this;
    }
    ~HostBuf() { reset(); }
    double* get() const { return p_; }
    void reset() {
        if (!p_) return;
        if (pool_) pool_->give(p_);
        else delete[] p_;
        p_ = nullptr;
    }
private:
    double* p_ = nullptr;
    PinnedPool* pool_ = nullptr;
};

struct Request {
    uint64_t ticket = 0;
    int state = 0;                      // 0 queued, 1 running, 2 done
    std::vector<int32_t> n_occ, n_vir, pair;
    std::vector<double> eps, warm_t;
    HostBuf k_intra, v_dimer;
    mcpt_problem prob{};                // points into the vectors above
    mcpt_options opts{};
    size_t footprint = 0;               // device bytes of the request alone
    int size_class = 0;                 // log2 of its pair-phase flops per sweep (batch fusing)
    double t_submit = 0.0;              // steady-clock seconds
    mcpt_summary sum{};
    uint64_t batch = 0;                 // internal resident id of the batch once run
    int cluster = 0;                    // index of the request in that batch
    std::string error;                  // message of a failed request
};

struct ServeParams {
    int workers = 4;                    // concurrent streams, each running one batch at a time
    int max_batch = 32;                 // requests fused into one batch
    int64_t max_batch_pairs = 1 << 20;  // pair budget of one batch
    int tick_mode = MCPT_SERVE_RETIRE_AT_TICKS;   // mcpt_serve_tick_mode: what FP64 batches do at sweep ticks
};

struct Server {
    PinnedPool pool;                    // first member: outlives the requests' buffers
    ServeParams params;
    std::deque<uint64_t> queue;         // queued tickets in arrival order (mu)
    std::map<uint64_t, std::unique_ptr<Request>> reqs;   // every live ticket (mu)
    std::vector<std::thread> workers;
    std::vector<std::unique_ptr<Exec>> execs;
    std::vector<std::unique_ptr<Exec>> uploads;   // per worker: the stream joiners are uploaded on
    std::condition_variable cv;         // queue, memory or stop changed
    std::condition_variable done_cv;    // a request finished
    bool stop = false;
    int busy = 0;                       // workers running a batch (mu)
    uint64_t batches = 0, served = 0;   // counters (mu)
    uint64_t joined = 0;                // requests admitted into running batches at sweep ticks (mu)
};

}  // namespace mcpt

struct mcpt_ctx {
    int device = 0;
    int n_cu = 0;
    std::mutex mu;
    size_t budget = 0, in_use = 0;      // mu
    size_t reserved = 0;                // sum of Exec::reserved (mu)
    uint64_t next_id = 1;               // mu
    std::map<uint64_t, std::unique_ptr<mcpt::Resident>> res;   // mu
    int grid_lds = 0, grid_glb = 0;     // persistent grids of the two FP64 pair-kernel variants
    mcpt::Exec main;                    // the caller's stream (mcpt_run, mcpt_energy, ...)
    std::map<std::string, int> tune;    // autotuned lowp variant per "precision/shape key" (mu)
    double* static_scratch = nullptr;   // this device's copy of the static Tau scratch (mcpt_run_static)
    std::unique_ptr<mcpt::Server> server;
};

namespace mcpt {

// shared between the solver runtime and the serving scheduler (the host-only
// helpers - errors, validation, batch formation - are in host.hpp)
mcpt_status exec_init(mcpt_ctx* c, Exec& x);
void exec_free(mcpt_ctx* c, Exec& x);
mcpt_status validate_options(const mcpt_options* o);
size_t footprint(const mcpt_problem* pbs, int n, int precision);
mcpt_status upload_batch(mcpt_ctx* c, Exec& x, const mcpt_problem* pbs, int n_cl, bool internal, uint64_t* id);
mcpt_status run(mcpt_ctx* c, Exec& x, Resident* R, const mcpt_options* o, mcpt_summary* out);
void release_resident(mcpt_ctx* c, uint64_t id);   // takes mu itself
mcpt_status slice_results(mcpt_ctx* c, Exec& x, Resident* R, int q, double* e_m2, double* de_m2, double* e_d2,
                          double* t_amp);
// Served FP64 batches with admission at sweep ticks (the plain Jacobi form only):
// join_init starts the iteration of a freshly uploaded batch (T = D K, every cluster
// at sweep 0, clusters with non-finite inputs stopped); join_sweeps runs `every`
// sweeps and returns every cluster's state; join_finish computes the energies of
// finished clusters, whose results then stay readable in the batch (slice_results)
// while its other clusters go on (*has: a result exists - converged or out of
// sweeps; *sums the summaries); join_concat builds one batch from clusters of
// several batches, keeping each cluster's iteration state, so its sweeps continue
// exactly where they stopped.
mcpt_status join_init(mcpt_ctx* c, Exec& x, Resident* R);
mcpt_status join_sweeps(mcpt_ctx* c, Exec& x, Resident* R, const mcpt_options* o, std::vector<ClState>* cs);
mcpt_status join_finish(mcpt_ctx* c, Exec& x, Resident* R, const std::vector<int>& qs, const mcpt_options* o,
                        std::vector<char>* has, std::vector<mcpt_summary>* sums);
mcpt_status join_concat(mcpt_ctx* c, Exec& x, const std::vector<std::pair<Resident*, int>>& parts, uint64_t* id);
void serve_stop(mcpt_ctx* c);
bool serve_owns(mcpt_ctx* c, uint64_t ticket);
mcpt_status serve_energy(mcpt_ctx* c, uint64_t ticket, double* e_m2, double* de_m2, double* e_d2, double* t_amp);
mcpt_status serve_release(mcpt_ctx* c, uint64_t ticket);

}  // namespace mcpt
