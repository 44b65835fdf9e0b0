// C ABI and host runtime of the MCPT(2) hot path: validation and upload of a
// problem (program flow step 2 output), the sweep driver of step 6, and the
// energy read-back (Eqs. 54-56).  See include/mcpt.h for the contract.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <unordered_set>
#include <array>
#include <vector>

#include "../../include/mcpt.h"
#include "mcpt_internal.hpp"
#include "host.hpp"
#include "runtime.hpp"
#include "singles.hpp"

namespace mcpt {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(MCPT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

int round_up(int x, int m) { return (x + m - 1) / m * m; }

#ifndef MCPT_PAIR_BLOCK
#define MCPT_PAIR_BLOCK 8
#endif
constexpr int kPairBlock = MCPT_PAIR_BLOCK;   // monomer block edge of the pair order (1: plain (min, max) order)

mcpt_status ensure_device(mcpt_ctx* c) {
    HIP_TRY(hipSetDevice(c->device));
    return MCPT_OK;
}

void free_lowp(mcpt_ctx* c, Resident* r) {
    for (void* p : r->lo_allocations) (void)hipFree(p);
    r->lo_allocations.clear();
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use -= std::min(c->in_use, r->lo_bytes);
    }
    r->lo_bytes = 0;
    r->lo_prec = 0;
    r->d_Vlo = r->d_Mlo = nullptr;
    r->d_lo_off = r->d_mlo_off = nullptr;
    r->d_R = r->d_Dl = nullptr;
    r->d_G32[0] = r->d_G32[1] = nullptr;
}

void free_det(mcpt_ctx* c, Resident* r) {
    for (void* p : r->det_allocations) (void)hipFree(p);
    r->det_allocations.clear();
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use -= std::min(c->in_use, r->det_bytes);
    }
    r->det_bytes = 0;
    r->d_part = nullptr;
    r->d_part_off = r->d_csr_off = r->d_csr = nullptr;
}

void drop_graph(Resident* r) {
    if (r->graph) (void)hipGraphExecDestroy(r->graph);
    r->graph = nullptr;
    r->graph_prec = -1;
}

void free_dimer(mcpt_ctx* c, Resident* r) {
    for (void* p : r->dimer_allocations) (void)hipFree(p);
    r->dimer_allocations.clear();
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use -= std::min(c->in_use, r->dimer_bytes);
    }
    r->dimer_bytes = 0;
    r->dimer_desc.clear();
    r->dimer_tau_elems = 0;
    r->dimer = false;
    r->d_dd = nullptr;
    r->d_pmono = nullptr;
    r->d_plccd = nullptr;
    r->d_DW = r->d_DQ = r->d_DCX = r->d_DCY = r->d_Tau = r->d_S = r->d_DRM = r->d_DY1 = r->d_DY2 = nullptr;
}

void free_lccd(mcpt_ctx* c, Resident* r) {
    free_dimer(c, r);
    for (void* p : r->lccd_allocations) (void)hipFree(p);
    r->lccd_allocations.clear();
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use -= std::min(c->in_use, r->lccd_bytes);
    }
    r->lccd_bytes = 0;
    r->lccd = false;
    r->lccd_desc.clear();
    r->d_lccd = nullptr;
    r->d_W = r->d_Q = r->d_J = r->d_L = r->d_R12 = r->d_Y = r->d_elccd = nullptr;
}

void free_resident(mcpt_ctx* c, Resident* r) {
    drop_graph(r);
    free_lccd(c, r);
    free_det(c, r);
    free_lowp(c, r);
    for (void* p : r->allocations) (void)hipFree(p);
    r->allocations.clear();
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use -= std::min(c->in_use, r->bytes);
    }
    r->bytes = 0;
}

mcpt_status lo_alloc(mcpt_ctx* c, Exec& x, Resident* r, void** out, size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (c->in_use + (c->reserved - x.reserved) + bytes > c->budget)
            return fail(MCPT_ERR_ADMISSION, "reduced-precision copies exceed the budget");
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MCPT_ERR_NOMEM, "hipMalloc of reduced-precision copies failed");
    }
    r->lo_allocations.push_back(p);
    r->lo_bytes += bytes;
    std::lock_guard<std::mutex> g(c->mu);
    c->in_use += bytes;
    *out = p;
    return MCPT_OK;
}

template <class T>
mcpt_status dev_alloc(mcpt_ctx* c, Resident* r, T** out, int64_t count) {
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    bytes = (bytes + 255) / 256 * 256;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MCPT_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                        hipGetErrorString(e));
    }
    r->allocations.push_back(p);
    r->bytes += bytes;
    std::lock_guard<std::mutex> g(c->mu);
    c->in_use += bytes;
    *out = static_cast<T*>(p);
    return MCPT_OK;
}

hipEvent_t take_event(Timing& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void drain_timing(Timing& t) {
    for (auto& r : t.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            if (r.kind == 0) {
                t.tot.pair_ms += ms;
                t.tot.pair_launches += 1;
                t.tot.pair_flops += r.flops;
                t.tot.pair_v_bytes += r.vbytes;
            } else if (r.kind == 2) {
                t.tot.lowp_ms += ms;
                t.tot.lowp_launches += 1;
                t.tot.lowp_flops += r.flops;
                t.tot.lowp_v_bytes += r.vbytes;
            } else if (r.kind == 3) {
                t.tot.singles_ms += ms;
                t.tot.singles_launches += 1;
                t.tot.singles_v_bytes += r.vbytes;
            } else if (r.kind == 4) {
                t.tot.lccd_ring_ms += ms;
            } else if (r.kind == 5) {
                t.tot.lccd_ladder_ms += ms;
                t.tot.lccd_launches += 1;
                t.tot.lccd_w_bytes += r.vbytes;
                t.tot.lccd_ladder_flops += r.flops;
            } else if (r.kind == 6) {
                t.tot.dimer_ladder_ms += ms;
                t.tot.dimer_launches += 1;
                t.tot.dimer_w_bytes += r.vbytes;
                t.tot.dimer_ladder_flops += r.flops;
            } else if (r.kind == 7) {
                t.tot.dimer_ring_ms += ms;
            } else {
                t.tot.mono_ms += ms;
                t.tot.mono_launches += 1;
            }
        }
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.pending.clear();
}

mcpt_status ensure_scratch(mcpt_ctx* c, Exec& x, int64_t slot_elems) {
    if (x.fixed_scratch)   // the caller sized the static scratch; nothing may be allocated here
        return slot_elems <= x.scratch_slot ? MCPT_OK : fail(MCPT_ERR_INVALID, "Tau slot exceeds the static scratch");
    const int grid = std::max(c->grid_lds, c->grid_glb);
    if (x.d_scratch && x.scratch_slot >= slot_elems && x.scratch_slots >= grid) return MCPT_OK;
    if (x.d_scratch) {
        HIP_TRY(hipStreamSynchronize(x.stream));
        (void)hipFree(x.d_scratch);
        x.d_scratch = nullptr;
    }
    const int64_t slot = std::max<int64_t>(slot_elems, x.scratch_slot);
    hipError_t e = hipMalloc(&x.d_scratch, (size_t)slot * grid * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        x.d_scratch = nullptr;
        return fail(MCPT_ERR_NOMEM, "scratch allocation failed");
    }
    x.scratch_slot = slot;
    x.scratch_slots = grid;
    return MCPT_OK;
}

double pair_flops(const Resident& r, bool couple) {
    double f = 0.0;
    for (const auto& p : r.pairs) {
        const double nx = r.monos[p.x].n, ny = r.monos[p.y].n;
        f += (couple ? 4.0 : 2.0) * nx * ny * (nx + ny);
    }
    return f;
}

// Upload one or more independent clusters as one resident problem: monomers
// and pairs are concatenated cluster after cluster (pair indices shifted by the
// cluster's first monomer), each monomer and pair carries its cluster id, and
// every cluster keeps its own stopping state during a run.
// Processing order of the pairs: LDS-variant pairs first; within each range, blocks of
// kPairBlock x kPairBlock monomers (lower, upper index), so that the pairs an XCD works on
// at a time share few monomers' M and G blocks.
void order_pairs(Resident* r) {
    const std::vector<MonoDesc>& m = r->monos;
    auto lds = [&m](const PairDesc& d) { return pair_fits_lds(m[d.x].n, m[d.x].np, m[d.y].np); };
    const int B = kPairBlock;
    std::stable_sort(r->pairs.begin(), r->pairs.end(), [&](const PairDesc& a, const PairDesc& b) {
        const bool la = lds(a), lb = lds(b);
        if (la != lb) return la;
        const int a0 = std::min(a.x, a.y), b0 = std::min(b.x, b.y);
        const int a1 = std::max(a.x, a.y), b1 = std::max(b.x, b.y);
        if (a0 / B != b0 / B) return a0 / B < b0 / B;
        if (a1 / B != b1 / B) return a1 / B < b1 / B;
        if (a0 != b0) return a0 < b0;
        return a1 < b1;
    });
    r->n_lds = std::count_if(r->pairs.begin(), r->pairs.end(), lds);
}

mcpt_status upload_batch(mcpt_ctx* c, Exec& x, const mcpt_problem* pbs, int n_cl, bool internal, uint64_t* id_out) {
    if (!pbs || n_cl < 1) return fail(MCPT_ERR_INVALID, "need at least one problem");
    if (!id_out) return fail(MCPT_ERR_INVALID, "id is NULL");
    mcpt_status st;
    for (int q = 0; q < n_cl; ++q) {
        if ((st = validate_problem(&pbs[q])) != MCPT_OK) {
            if (n_cl > 1) prefix_error("cluster " + std::to_string(q) + ": ");
            return st;
        }
    }
    if ((st = ensure_device(c)) != MCPT_OK) return st;
    auto r = std::make_unique<Resident>();
    r->n_cl = n_cl;
    r->cl_mono.assign(n_cl + 1, 0);
    r->cl_pair.assign(n_cl + 1, 0);
    for (int q = 0; q < n_cl; ++q) {
        r->cl_mono[q + 1] = r->cl_mono[q] + pbs[q].n_mono;
        r->cl_pair[q + 1] = r->cl_pair[q] + pbs[q].n_pair;
    }
    if (r->cl_mono[n_cl] > INT32_MAX) return fail(MCPT_ERR_INVALID, "too many monomers");
    r->n_mono = (int)r->cl_mono[n_cl];
    r->n_pair = r->cl_pair[n_cl];
    r->monos.resize(r->n_mono);
    int64_t eoff = 0, roff = 0, moff = 0, doff = 0;
    std::vector<int64_t> eps_cl(n_cl + 1, 0), raw_cl(n_cl + 1, 0), v_cl(n_cl + 1, 0);
    for (int q = 0; q < n_cl; ++q) {
        const mcpt_problem* pb = &pbs[q];
        eps_cl[q] = eoff;
        raw_cl[q] = roff;
        for (int lx = 0; lx < pb->n_mono; ++lx) {
            MonoDesc& d = r->monos[r->cl_mono[q] + lx];
            d.o = pb->n_occ[lx];
            d.v = pb->n_vir[lx];
            d.n = d.o * d.v;
            d.np = round_up(d.n, kTile);
            d.eps_off = eoff;
            d.raw_off = roff;
            d.mat_off = moff;
            d.dif_off = doff;
            d.cluster = q;
            d.pad = 0;
            doff += d.np;
            eoff += d.o + d.v;
            roff += (int64_t)d.n * d.n;
            moff += (int64_t)d.np * d.np;
            r->max_n = std::max(r->max_n, d.n);
            r->max_v = std::max(r->max_v, d.v);
            r->max_np = std::max(r->max_np, d.np);
        }
    }
    eps_cl[n_cl] = eoff;
    raw_cl[n_cl] = roff;
    r->eps_elems = eoff;
    r->dif_elems = doff;
    r->raw_elems = roff;
    r->mat_elems = moff;
    // pairs: caller order gives V offsets; processing order is sorted by (min, max) monomer
    r->pairs.resize(r->n_pair);
    int64_t vo = 0;
    for (int q = 0; q < n_cl; ++q) {
        const mcpt_problem* pb = &pbs[q];
        v_cl[q] = vo;
        const int base = (int)r->cl_mono[q];
        for (int64_t lp = 0; lp < pb->n_pair; ++lp) {
            const int64_t p = r->cl_pair[q] + lp;
            PairDesc& d = r->pairs[p];
            d.x = base + pb->pair[2 * lp];
            d.y = base + pb->pair[2 * lp + 1];
            d.v_off = vo;
            d.orig = p;
            d.cluster = q;
            d.pad = 0;
            vo += (int64_t)r->monos[d.x].n * r->monos[d.y].n;
            r->max_slot = std::max<int64_t>(r->max_slot, (int64_t)r->monos[d.x].np * r->monos[d.y].np);
        }
    }
    v_cl[n_cl] = vo;
    r->v_elems = vo;
    r->cl_v = v_cl;
    order_pairs(r.get());
    // energies: validated on the host (small)
    std::vector<double> eps(eoff);
    for (int q = 0; q < n_cl; ++q) {
        const size_t bytes = (eps_cl[q + 1] - eps_cl[q]) * sizeof(double);
        if (pbs[q].memory == MCPT_HOST) std::memcpy(eps.data() + eps_cl[q], pbs[q].eps, bytes);
        else HIP_TRY(hipMemcpy(eps.data() + eps_cl[q], pbs[q].eps, bytes, hipMemcpyDeviceToHost));
        std::vector<double> one(eps.begin() + eps_cl[q], eps.begin() + eps_cl[q + 1]);
        if ((st = check_energies(one.data(), &pbs[q])) != MCPT_OK) {
            if (n_cl > 1) prefix_error("cluster " + std::to_string(q) + ": ");
            return st;
        }
    }
    // orbital-energy differences d[(i,a)] = e_i - e_a (Eqs. 60-61 as d_X + d_Y)
    std::vector<double> dif(doff, 0.0);
    for (int x = 0; x < r->n_mono; ++x) {
        const MonoDesc& d = r->monos[x];
        const double* e = eps.data() + d.eps_off;
        for (int i = 0; i < d.o; ++i)
            for (int a = 0; a < d.v; ++a) dif[d.dif_off + i * d.v + a] = e[i] - e[d.o + a];
    }
    // footprint and admission
    const size_t need = footprint(pbs, n_cl, MCPT_FP64);
    {
        std::lock_guard<std::mutex> g(c->mu);
        const size_t others = c->reserved - x.reserved;
        if (c->in_use + others + need > c->budget)
            return fail(MCPT_ERR_ADMISSION, "problem needs " + std::to_string(need) + " bytes; budget " +
                                                std::to_string(c->budget) + ", in use " +
                                                std::to_string(c->in_use + others));
    }
    Resident* R = r.get();
#define ALLOC(ptr, n)                                          \
    do {                                                       \
        if ((st = dev_alloc(c, R, &(ptr), (n))) != MCPT_OK) { \
            free_resident(c, R);                               \
            return st;                                         \
        }                                                      \
    } while (0)
    ALLOC(R->d_monos, R->n_mono);
    ALLOC(R->d_pairs, std::max<int64_t>(R->n_pair, 1));
    ALLOC(R->d_dif, doff);
    ALLOC(R->d_raw, R->raw_elems);
    ALLOC(R->d_K, R->mat_elems);
    ALLOC(R->d_T, R->mat_elems);
    ALLOC(R->d_M, R->mat_elems);
    ALLOC(R->d_G[0], R->mat_elems);
    ALLOC(R->d_G[1], R->mat_elems);
    ALLOC(R->d_V, std::max<int64_t>(R->v_elems, 1));
    ALLOC(R->d_em2, R->n_mono);
    ALLOC(R->d_em2_0, R->n_mono);
    ALLOC(R->d_res, R->n_mono);
    ALLOC(R->d_ed2, std::max<int64_t>(R->n_pair, 1));
    ALLOC(R->d_cl, n_cl);
    ALLOC(R->d_hist, (int64_t)n_cl * kMaxSweeps);
    ALLOC(R->d_cl_mono, n_cl + 1);
    ALLOC(R->d_cl_pair, n_cl + 1);
#undef ALLOC
    hipStream_t s = x.stream;
#define DTRY(expr)                   \
    do {                             \
        hipError_t e_ = (expr);      \
        if (e_ != hipSuccess) {      \
            free_resident(c, R);     \
            return fail(MCPT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                            \
    } while (0)
    DTRY(hipMemcpyAsync(R->d_monos, R->monos.data(), R->monos.size() * sizeof(MonoDesc), hipMemcpyHostToDevice, s));
    if (R->n_pair)
        DTRY(hipMemcpyAsync(R->d_pairs, R->pairs.data(), R->pairs.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s));
    DTRY(hipMemcpyAsync(R->d_dif, dif.data(), doff * sizeof(double), hipMemcpyHostToDevice, s));
    DTRY(hipMemcpyAsync(R->d_cl_mono, R->cl_mono.data(), (n_cl + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DTRY(hipMemcpyAsync(R->d_cl_pair, R->cl_pair.data(), (n_cl + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    for (int q = 0; q < n_cl; ++q) {
        const hipMemcpyKind kind = pbs[q].memory == MCPT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (raw_cl[q + 1] > raw_cl[q])
            DTRY(hipMemcpyAsync(R->d_raw + raw_cl[q], pbs[q].k_intra, (raw_cl[q + 1] - raw_cl[q]) * sizeof(double),
                                kind, s));
        if (v_cl[q + 1] > v_cl[q])
            DTRY(hipMemcpyAsync(R->d_V + v_cl[q], pbs[q].v_dimer, (v_cl[q + 1] - v_cl[q]) * sizeof(double), kind, s));
    }
    // non-finite inputs, flagged per cluster
    int32_t* d_bad = nullptr;
    if ((st = dev_alloc(c, R, &d_bad, n_cl)) != MCPT_OK) {
        free_resident(c, R);
        return st;
    }
    DTRY(hipMemsetAsync(d_bad, 0, n_cl * sizeof(int32_t), s));
    DTRY(hipMemsetAsync(R->d_cl, 0, n_cl * sizeof(ClState), s));
    for (int q = 0; q < n_cl; ++q) {
        launch_nonfinite(R->d_raw + raw_cl[q], raw_cl[q + 1] - raw_cl[q], d_bad + q, s);
        launch_nonfinite(R->d_V + v_cl[q], v_cl[q + 1] - v_cl[q], d_bad + q, s);
    }
    launch_fill(R->d_K, R->mat_elems, 0.0, s);
    launch_fill(R->d_T, R->mat_elems, 0.0, s);
    launch_fill(R->d_M, R->mat_elems, 0.0, s);
    launch_fill(R->d_G[0], R->mat_elems, 0.0, s);
    launch_fill(R->d_G[1], R->mat_elems, 0.0, s);
    launch_pack(R->d_monos, R->n_mono, R->d_raw, R->d_K, R->max_n, s);
    DTRY(hipGetLastError());
    R->cl_bad.assign(n_cl, 0);
    DTRY(hipMemcpyAsync(R->cl_bad.data(), d_bad, n_cl * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DTRY(hipStreamSynchronize(s));
#undef DTRY
    for (int q = 0; q < n_cl; ++q) {
        // a caller's upload fails as a whole; a served batch keeps the other clusters
        if (R->cl_bad[q] && !internal) {
            free_resident(c, R);
            return fail(MCPT_ERR_NONFINITE, (n_cl > 1 ? "cluster " + std::to_string(q) + ": " : std::string()) +
                                                "non-finite value in k_intra or v_dimer");
        }
    }
    r->cl_last.assign(n_cl, mcpt_summary{});
    r->internal = internal;
    std::lock_guard<std::mutex> g(c->mu);
    r->id = c->next_id++;
    *id_out = r->id;
    c->res[r->id] = std::move(r);
    return MCPT_OK;
}

// Device bytes that upload_batch (and, for a reduced precision, ensure_lowp)
// allocates for these clusters; sizes only, so admission can price a request
// before anything is allocated.  Every buffer is rounded up to 256 bytes.
size_t footprint(const mcpt_problem* pbs, int n, int precision) {
    const LayoutSizes ls{(int64_t)sizeof(MonoDesc), (int64_t)sizeof(PairDesc), (int64_t)sizeof(ClState), kTile,
                         kMaxSweeps, lowp_chunk(MCPT_FP32), lowp_chunk(MCPT_BF16)};
    return footprint(pbs, n, precision, ls);
}

mcpt_status exec_init(mcpt_ctx* c, Exec& x) {
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipStreamCreateWithFlags(&x.own, hipStreamNonBlocking));
    x.stream = x.own;
    HIP_TRY(hipMalloc(&x.d_ctrl, sizeof(Ctrl)));
    HIP_TRY(hipHostMalloc(&x.h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
    HIP_TRY(hipMalloc(&x.d_flag, sizeof(int32_t)));
    HIP_TRY(hipHostMalloc(&x.h_flag, sizeof(int32_t), hipHostMallocDefault));
    return MCPT_OK;
}

void exec_free(mcpt_ctx* c, Exec& x) {
    (void)hipSetDevice(c->device);
    if (x.stream) (void)hipStreamSynchronize(x.stream);
    if (x.timing.on) drain_timing(x.timing);
    for (hipEvent_t e : x.timing.pool) (void)hipEventDestroy(e);
    x.timing.pool.clear();
    if (x.d_scratch) (void)hipFree(x.d_scratch);
    if (x.d_scratch_lo) (void)hipFree(x.d_scratch_lo);
    if (x.d_ctrl) (void)hipFree(x.d_ctrl);
    if (x.d_flag) (void)hipFree(x.d_flag);
    if (x.h_ctrl) (void)hipHostFree(x.h_ctrl);
    if (x.h_flag) (void)hipHostFree(x.h_flag);
    if (x.own) (void)hipStreamDestroy(x.own);
    x = Exec{};
}

void release_resident(mcpt_ctx* c, uint64_t id) {
    std::unique_ptr<Resident> r;
    {
        std::lock_guard<std::mutex> g(c->mu);
        auto it = c->res.find(id);
        if (it == c->res.end()) return;
        r = std::move(it->second);
        c->res.erase(it);
    }
    free_resident(c, r.get());
}

// Results of cluster q of a resident problem (q < 0: every cluster, concatenated).
mcpt_status slice_results(mcpt_ctx* c, Exec& x, Resident* R, int q, double* e_m2, double* de_m2, double* e_d2,
                          double* t_amp) {
    if (!R->has_result) return fail(MCPT_ERR_INVALID, "problem has no result (not run, or diverged)");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = x.stream;
    const int64_t m0 = q < 0 ? 0 : R->cl_mono[q], m1 = q < 0 ? R->n_mono : R->cl_mono[q + 1];
    const int64_t p0 = q < 0 ? 0 : R->cl_pair[q], p1 = q < 0 ? R->n_pair : R->cl_pair[q + 1];
    std::vector<double> a(m1 - m0), b(m1 - m0);
    if (m1 > m0) {
        HIP_TRY(hipMemcpyAsync(a.data(), R->d_em2 + m0, (m1 - m0) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(b.data(), R->d_em2_0 + m0, (m1 - m0) * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (e_d2 && p1 > p0)
        HIP_TRY(hipMemcpyAsync(e_d2, R->d_ed2 + p0, (p1 - p0) * sizeof(double), hipMemcpyDeviceToHost, s));
    if (t_amp && m1 > m0) {
        // only these monomers' T (a served batch may still be sweeping its other clusters)
        launch_unpack(R->d_monos + m0, (int)(m1 - m0), R->d_T, R->d_raw, R->max_n, s);
        HIP_TRY(hipGetLastError());
        const int64_t r0 = R->monos[m0].raw_off;
        const int64_t r1 = m1 < R->n_mono ? R->monos[m1].raw_off : R->raw_elems;
        HIP_TRY(hipMemcpyAsync(t_amp, R->d_raw + r0, (r1 - r0) * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t k = 0; k < m1 - m0; ++k) {
        if (e_m2) e_m2[k] = a[k];
        if (de_m2) de_m2[k] = a[k] - b[k];
    }
    return MCPT_OK;
}

mcpt_status validate_options(const mcpt_options* o) {
    if (!o) return fail(MCPT_ERR_INVALID, "options are NULL");
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(MCPT_ERR_INVALID, "tol must be finite and >= 0");
    if (o->max_sweeps < 0 || o->max_sweeps >= kMaxSweeps)
        return fail(MCPT_ERR_INVALID, "max_sweeps must be in [0, " + std::to_string(kMaxSweeps - 1) + "]");
    if (o->precision < MCPT_FP64 || o->precision > MCPT_BF16)
        return fail(MCPT_ERR_INVALID, "precision must be MCPT_FP64, MCPT_FP32 or MCPT_BF16");
    if (o->check_every < 0) return fail(MCPT_ERR_INVALID, "check_every must be >= 0");
    if (o->inner_sweeps < 0 || o->inner_sweeps > 64) return fail(MCPT_ERR_INVALID, "inner_sweeps must be in [0, 64]");
    if (o->deterministic != 0 && o->deterministic != 1) return fail(MCPT_ERR_INVALID, "deterministic must be 0 or 1");
    if (o->graph != 0 && o->graph != 1) return fail(MCPT_ERR_INVALID, "graph must be 0 or 1");
    if (o->autotune != 0 && o->autotune != 1) return fail(MCPT_ERR_INVALID, "autotune must be 0 or 1");
    return MCPT_OK;
}

void record_begin(Exec& x, hipEvent_t* a) {
    if (!x.timing.on) return;
    *a = take_event(x.timing);
    (void)hipEventRecord(*a, x.stream);
}

void record_end(Exec& x, hipEvent_t a, int kind, double flops, double vbytes) {
    if (!x.timing.on) return;
    hipEvent_t b = take_event(x.timing);
    (void)hipEventRecord(b, x.stream);
    x.timing.pending.push_back({a, b, kind, flops, vbytes});
}

// Pair phase over all pairs: the LDS-resident-V kernel for the pairs that fit,
// then the L2 variant for the rest (same stream, so G accumulates in order).
#ifndef MCPT_GLB_SPLIT
#define MCPT_GLB_SPLIT 1
#endif

// Task layout of the split form for the pairs read from L2 (processing indices n_lds..n_pair):
// chunks of at most grid_glb pairs, so that each chunk's Tau fits the Tau scratch (one slot of the
// largest pair per persistent workgroup); pair k of a chunk goes to XCD k % 8.
mcpt_status ensure_glb_plan(mcpt_ctx* c, Resident* R) {
    if (R->glb_plan) return MCPT_OK;
    const int64_t first = R->n_lds, n = R->n_pair - R->n_lds;
    const int chunk = std::max(c->grid_glb, 1);
    std::vector<int32_t> xpair, pre_tau, pre_g;
    std::vector<int64_t> off;
    struct Bases {
        size_t x, p;
        int m;
        std::array<int, 9> xbeg;
    };
    std::vector<Bases> bases;
    for (int64_t k0 = 0; k0 < n; k0 += chunk) {
        const int m = (int)std::min<int64_t>(chunk, n - k0);
        Bases b{xpair.size(), pre_tau.size(), m, {}};
        int64_t o = 0;
        int32_t tt = 0, tg = 0;
        for (int xc = 0; xc < 8; ++xc) {
            b.xbeg[xc] = (int)(xpair.size() - b.x);
            for (int k = xc; k < m; k += 8) {
                const PairDesc& d = R->pairs[first + k0 + k];
                const int npX = R->monos[d.x].np, npY = R->monos[d.y].np;
                xpair.push_back((int32_t)(first + k0 + k));
                off.push_back(o);
                pre_tau.push_back(tt);
                pre_g.push_back(tg);
                o += (int64_t)npX * npY;
                tt += glb_tau_tasks(npX, npY);
                tg += glb_g_tasks(npX, npY);
            }
        }
        b.xbeg[8] = m;
        pre_tau.push_back(tt);
        pre_g.push_back(tg);
        bases.push_back(b);
    }
    R->glb_tau.clear();
    R->glb_g.clear();
    R->glb_n.clear();
    if (n > 0) {
        int32_t *d_xpair = nullptr, *d_pt = nullptr, *d_pg = nullptr;
        int64_t* d_off = nullptr;
        mcpt_status st;
        if ((st = dev_alloc(c, R, &d_xpair, (int64_t)xpair.size())) != MCPT_OK ||
            (st = dev_alloc(c, R, &d_off, (int64_t)off.size())) != MCPT_OK ||
            (st = dev_alloc(c, R, &d_pt, (int64_t)pre_tau.size())) != MCPT_OK ||
            (st = dev_alloc(c, R, &d_pg, (int64_t)pre_g.size())) != MCPT_OK)
            return st;
        HIP_TRY(hipMemcpy(d_xpair, xpair.data(), xpair.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_off, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_pt, pre_tau.data(), pre_tau.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_pg, pre_g.data(), pre_g.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        for (const Bases& b : bases) {
            GlbTasks t{d_xpair + b.x, d_off + b.x, d_pt + b.p, {}};
            for (int i = 0; i < 9; ++i) t.xbeg[i] = b.xbeg[i];
            GlbTasks g = t;
            g.pre = d_pg + b.p;
            R->glb_tau.push_back(t);
            R->glb_g.push_back(g);
            R->glb_n.push_back(b.m);
        }
    }
    R->glb_plan = true;
    return MCPT_OK;
}

void pair_phase(mcpt_ctx* c, Exec& x, Resident* R, double* G, int couple, const Ctrl* ctrl,
                const ClState* cl_sel = nullptr) {
    // the final energy pass covers every cluster, or those cl_sel does not mark done
    const ClState* cl = cl_sel ? cl_sel : ctrl ? R->d_cl : nullptr;
    const bool det = R->det_on && couple;
    PartOut p0{det ? R->d_part : nullptr, R->d_part_off};
    PartOut p1{det ? R->d_part : nullptr, R->d_part_off ? R->d_part_off + R->n_lds : nullptr};
    if (R->dimer) {
        // dimer-internal terms of Eq. 59 from the previous Tau into S: the two ladders (stored), then the
        // rings (added); the pair kernels add S into the numerator of Tau and keep the new Tau
        hipEvent_t a = nullptr;
        record_begin(x, &a);
        if (R->dimer_lds_bytes > 0)
            launch_lccd_ladder(R->d_pmono, R->d_plccd, (int)R->n_pair, 1, R->dimer_ct, R->dimer_lds_bytes, R->d_DW,
                               R->d_DQ, R->d_Tau, nullptr, nullptr, R->d_S, ctrl, cl, x.stream, 0);
        else
            launch_dimer_ladder(R->d_dd, (int)R->n_pair, R->dimer_ladder_blocks, R->dimer_ct, R->d_DW, R->d_DQ,
                                R->d_Tau, R->d_S, ctrl, cl, x.stream);
        record_end(x, a, 6, R->dimer_w_flops, R->dimer_w_bytes);
        record_begin(x, &a);
        launch_dimer_ring(R->d_dd, R->d_monos, (int)R->n_pair, R->dimer_ring_blocks, R->d_DRM, R->d_DCX, R->d_DCY,
                          R->d_Tau, R->d_S, R->d_DY1, R->d_DY2, ctrl, cl, x.stream);
        record_end(x, a, 7, 0.0, 0.0);
        p0.S = p1.S = R->d_S;
        p0.Y1 = p1.Y1 = R->d_DY1;
        p0.Y2 = p1.Y2 = R->d_DY2;
        p0.tau_out = p1.tau_out = R->d_Tau;
        if (R->dimer_one_size) {   // np x np per pair at orig * np^2 (the one-size source form)
            p0.mat_stride = p1.mat_stride = (int64_t)R->monos[0].np * R->monos[0].np;
            p0.v = p1.v = R->monos[0].v;
        } else {
            p0.dd = p1.dd = R->d_dd;
        }
    }
    const int g_lds = x.grid_cap > 0 ? std::min(c->grid_lds, x.grid_cap) : c->grid_lds;
    const int g_glb = x.grid_cap > 0 ? std::min(c->grid_glb, x.grid_cap) : c->grid_glb;
    launch_pair_fp64(1, p0, R->d_pairs, R->n_lds, R->d_monos, R->d_dif, R->d_V, R->d_M, G, x.d_scratch,
                     x.scratch_slot, g_lds, R->d_ed2, couple, ctrl, cl, x.stream);
    // pairs from L2: split into Tau and G launches per chunk (XCD-local tasks) in the plain form
    // (not in deterministic mode, energy pass included: the split form adds E_D2 with atomics)
    const bool split = MCPT_GLB_SPLIT && R->n_pair > R->n_lds && !R->dimer && !R->det_on && !x.fixed_scratch &&
                       x.grid_cap == 0 && x.scratch_slots >= c->grid_glb && x.scratch_slot >= R->max_slot &&
                       ensure_glb_plan(c, R) == MCPT_OK;
    if (split) {
        for (size_t k = 0; k < R->glb_n.size(); ++k)
            launch_pair_fp64_split(R->glb_tau[k], R->glb_g[k], R->glb_n[k], R->d_pairs, R->d_monos, R->d_dif,
                                   R->d_V, R->d_M, G, x.d_scratch, g_glb, R->d_ed2, couple, ctrl, cl, x.stream);
    } else {
        launch_pair_fp64(0, p1, R->d_pairs + R->n_lds, R->n_pair - R->n_lds, R->d_monos, R->d_dif, R->d_V, R->d_M,
                         G, x.d_scratch, x.scratch_slot, g_glb, R->d_ed2, couple, ctrl, cl, x.stream);
    }
    if (det) launch_reduce_parts(R->d_monos, R->n_mono, R->d_csr_off, R->d_csr, R->d_part, G, R->d_cl, ctrl, x.stream);
}

// Buffers of the deterministic mode: a partial G_X and G_Y block per pair and,
// per monomer, the offsets of its blocks in pair order (the summation order).
mcpt_status ensure_det(mcpt_ctx* c, Exec& x, Resident* R) {
    if (R->d_part) return MCPT_OK;
    std::vector<int64_t> off(std::max<int64_t>(R->n_pair, 1), 0);
    std::vector<std::vector<std::pair<int64_t, int64_t>>> per(R->n_mono);   // (caller pair index, offset)
    int64_t tot = 0;
    for (int64_t p = 0; p < R->n_pair; ++p) {
        const PairDesc& d = R->pairs[p];
        const int64_t nx = R->monos[d.x].np, ny = R->monos[d.y].np;
        off[p] = tot;
        per[d.x].push_back({d.orig, tot});
        per[d.y].push_back({d.orig, tot + nx * nx});
        tot += nx * nx + ny * ny;
    }
    std::vector<int64_t> csr_off(R->n_mono + 1, 0), csr;
    csr.reserve(2 * R->n_pair);
    for (int m = 0; m < R->n_mono; ++m) {
        std::sort(per[m].begin(), per[m].end());
        for (const auto& e : per[m]) csr.push_back(e.second);
        csr_off[m + 1] = (int64_t)csr.size();
    }
    if (csr.empty()) csr.push_back(0);
    void *part = nullptr, *o = nullptr, *co = nullptr, *cs = nullptr;
    mcpt_status st;
    auto alloc = [&](void** out, size_t bytes) -> mcpt_status {
        bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        {
            std::lock_guard<std::mutex> g(c->mu);
            if (c->in_use + (c->reserved - x.reserved) + bytes > c->budget)
                return fail(MCPT_ERR_ADMISSION, "deterministic-mode partials (" + std::to_string(bytes) +
                                                    " bytes) exceed the HBM budget");
        }
        hipError_t e = hipMalloc(out, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MCPT_ERR_NOMEM, "hipMalloc of deterministic-mode partials failed");
        }
        R->det_allocations.push_back(*out);
        R->det_bytes += bytes;
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use += bytes;
        return MCPT_OK;
    };
    if ((st = alloc(&part, (size_t)std::max<int64_t>(tot, 1) * 8)) != MCPT_OK ||
        (st = alloc(&o, off.size() * 8)) != MCPT_OK || (st = alloc(&co, csr_off.size() * 8)) != MCPT_OK ||
        (st = alloc(&cs, csr.size() * 8)) != MCPT_OK) {
        free_det(c, R);
        return st;
    }
    HIP_TRY(hipMemcpyAsync(o, off.data(), off.size() * 8, hipMemcpyHostToDevice, x.stream));
    HIP_TRY(hipMemcpyAsync(co, csr_off.data(), csr_off.size() * 8, hipMemcpyHostToDevice, x.stream));
    HIP_TRY(hipMemcpyAsync(cs, csr.data(), csr.size() * 8, hipMemcpyHostToDevice, x.stream));
    HIP_TRY(hipStreamSynchronize(x.stream));
    R->d_part = static_cast<double*>(part);
    R->d_part_off = static_cast<int64_t*>(o);
    R->d_csr_off = static_cast<int64_t*>(co);
    R->d_csr = static_cast<int64_t*>(cs);
    return MCPT_OK;
}

// Reduced-precision copies of a resident problem for `prec` (1 FP32, 2 BF16):
// V and V^T per pair (rows padded to 16, k padded to the chunk), M per monomer,
// and FP64 buffers for the polish residual R and correction delta.
mcpt_status ensure_lowp(mcpt_ctx* c, Exec& x, Resident* R, int prec) {
    if (R->lo_prec == prec) return MCPT_OK;
    drop_graph(R);
    free_lowp(c, R);
    const int kc = lowp_chunk(prec);
    const size_t es = prec == MCPT_BF16 ? 2 : 4;
    auto ld = [kc](int n) { return (int64_t)((n + kc - 1) / kc * kc); };
    std::vector<int64_t> lo_off(std::max<int64_t>(R->n_pair, 1), 0), mlo_off(R->n_mono);
    int64_t vo = 0, slot = 0;
    for (int64_t p = 0; p < R->n_pair; ++p) {
        const MonoDesc &dx = R->monos[R->pairs[p].x], &dy = R->monos[R->pairs[p].y];
        lo_off[p] = vo;
        const int64_t sz = dx.np * ld(dy.n) + dy.np * ld(dx.n);
        vo += sz;
        slot = std::max(slot, sz);   // scratch slot: Tau and Tau^T
    }
    int64_t mo = 0;
    for (int x = 0; x < R->n_mono; ++x) {
        mlo_off[x] = mo;
        mo += R->monos[x].np * ld(R->monos[x].n);
    }
    mcpt_status st;
    void *vlo = nullptr, *mlo = nullptr, *lo_o = nullptr, *mlo_o = nullptr, *rr = nullptr, *dd = nullptr,
         *g32 = nullptr;
    if ((st = lo_alloc(c, x, R, &vlo, vo * es)) != MCPT_OK || (st = lo_alloc(c, x, R, &mlo, mo * es)) != MCPT_OK ||
        (st = lo_alloc(c, x, R, &lo_o, lo_off.size() * 8)) != MCPT_OK ||
        (st = lo_alloc(c, x, R, &mlo_o, mlo_off.size() * 8)) != MCPT_OK ||
        (st = lo_alloc(c, x, R, &rr, R->mat_elems * 8)) != MCPT_OK ||
        (st = lo_alloc(c, x, R, &dd, R->mat_elems * 8)) != MCPT_OK ||
        (prec == MCPT_BF16 && (st = lo_alloc(c, x, R, &g32, R->mat_elems * 8)) != MCPT_OK)) {
        free_lowp(c, R);
        return st;
    }
    hipStream_t s = x.stream;
    HIP_TRY(hipMemcpyAsync(lo_o, lo_off.data(), lo_off.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(mlo_o, mlo_off.data(), mlo_off.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(mlo, 0, mo * es, s));   // padding of M stays zero
    launch_fill(static_cast<double*>(rr), R->mat_elems, 0.0, s);
    launch_fill(static_cast<double*>(dd), R->mat_elems, 0.0, s);
    launch_convert_v(prec, R->d_pairs, R->n_pair, R->d_monos, R->d_V, vlo, static_cast<int64_t*>(lo_o), s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    R->d_Vlo = vlo;
    R->d_Mlo = mlo;
    R->d_lo_off = static_cast<int64_t*>(lo_o);
    R->d_mlo_off = static_cast<int64_t*>(mlo_o);
    R->d_R = static_cast<double*>(rr);
    R->d_Dl = static_cast<double*>(dd);
    if (g32) {
        launch_fill(static_cast<double*>(g32), R->mat_elems, 0.0, s);   // 2 x mat_elems floats
        R->d_G32[0] = static_cast<float*>(g32);
        R->d_G32[1] = R->d_G32[0] + R->mat_elems;
    }
    R->lo_slot = (slot + 63) / 64 * 64;   // keeps every slot 16-byte aligned
    R->lo_v_bytes = (double)vo * es;
    R->lo_prec = prec;
    // leading pairs whose V (and, for BF16, Tau) fit in LDS run in the LDS-resident kernel
    R->lo_n_lds = 0;
    R->lo_lds_bytes = 0;
    while (R->lo_n_lds < R->n_pair) {
        const PairDesc& d = R->pairs[R->lo_n_lds];
        const int64_t b = lowp_lds_bytes(prec, R->monos[d.x].n, R->monos[d.y].n);
        if (b > lowp_lds_limit()) break;
        R->lo_lds_bytes = std::max(R->lo_lds_bytes, b);
        ++R->lo_n_lds;
    }
    return MCPT_OK;
}

// Per-stream scratch of the reduced-precision pair kernel (Tau and Tau^T per workgroup).
mcpt_status ensure_scratch_lo(mcpt_ctx* c, Exec& x, const Resident* R, int prec) {
    const size_t es = prec == MCPT_BF16 ? 2 : 4;
    x.grid_lo = std::max(8, c->n_cu * pair_lowp_blocks_per_cu(prec, R->lo_variant, 0) / 8 * 8);
    x.grid_lo_lds = R->lo_n_lds ? std::max(8, c->n_cu * pair_lowp_blocks_per_cu(prec, R->lo_variant, R->lo_lds_bytes) / 8 * 8)
                                : 0;
    const size_t need = (size_t)R->lo_slot * es * std::max(x.grid_lo, x.grid_lo_lds);
    if (need > x.scratch_lo_bytes) {
        HIP_TRY(hipStreamSynchronize(x.stream));
        if (x.d_scratch_lo) (void)hipFree(x.d_scratch_lo);
        x.d_scratch_lo = nullptr;
        x.scratch_lo_bytes = 0;
        hipError_t e = hipMalloc(&x.d_scratch_lo, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            x.d_scratch_lo = nullptr;
            return fail(MCPT_ERR_NOMEM, "reduced-precision scratch allocation failed");
        }
        x.scratch_lo_bytes = need;
    }
    return MCPT_OK;
}

// `every`: cover the pairs of every cluster (the autotuner), not only those still iterating
// Reduced-precision pair phase: the LDS-resident-V kernel for the leading pairs
// that fit, then the L2 variant for the rest (same stream, so G accumulates in order).
// Gf non-null: G contributions go to that FP32 buffer (not in deterministic mode).
void lowp_phase(mcpt_ctx* c, Exec& x, Resident* R, double* G, float* Gf, int source, bool every = false) {
    const ClState* cl = every ? nullptr : R->d_cl;
    const int64_t nl = R->lo_n_lds;
    const bool det = R->det_on && !every;
    const PartOut p0{det ? R->d_part : nullptr, R->d_part_off};
    const PartOut p1{det ? R->d_part : nullptr, R->d_part_off ? R->d_part_off + nl : nullptr};
    launch_pair_lowp(R->lo_prec, R->lo_variant, R->lo_lds_bytes, p0, R->d_pairs, nl, R->d_monos, R->d_dif, R->d_Vlo,
                     R->d_lo_off, R->d_Mlo, R->d_mlo_off, G, Gf, x.d_scratch_lo, R->lo_slot, x.grid_lo_lds, R->d_ed2,
                     source, 1, nullptr, cl, x.stream);
    launch_pair_lowp(R->lo_prec, R->lo_variant, 0, p1, R->d_pairs + nl, R->n_pair - nl, R->d_monos, R->d_dif, R->d_Vlo,
                     R->d_lo_off + nl, R->d_Mlo, R->d_mlo_off, G, Gf, x.d_scratch_lo, R->lo_slot, x.grid_lo, R->d_ed2,
                     source, 1, nullptr, cl, x.stream);
    if (det) launch_reduce_parts(R->d_monos, R->n_mono, R->d_csr_off, R->d_csr, R->d_part, G, R->d_cl, nullptr, x.stream);
}

void mixed_mono(mcpt_ctx* c, Exec& x, Resident* R, int mode, const double* G, double* Gz, bool lo_out, const Ctrl* ctrl,
                const float* Gf = nullptr, float* Gfz = nullptr) {
    // full monomer equation: the update and correction modes add the intramonomer terms held in L
    const bool with_l = R->lccd && (mode == kMonoUpdate || mode == kMonoUpdateR || mode == kMonoCorr || mode == kMonoRlo);
    launch_monomer_mixed(mode, R->lo_prec, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, G, Gz, R->d_T, R->d_M, R->d_R,
                         R->d_Dl, lo_out ? R->d_Mlo : nullptr, R->d_mlo_off, R->d_em2, R->d_em2_0, R->d_res, ctrl,
                         R->d_cl, x.stream, Gf, Gfz, with_l ? R->d_L : nullptr);
}

mcpt_status sync_ctrl(Exec& x) {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(x.h_ctrl, x.d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, x.stream));
    HIP_TRY(hipStreamSynchronize(x.stream));
    return MCPT_OK;
}

// Signature of a problem's pair phase for the tile autotuner: the distinct
// padded block shapes (npX x npY, smaller first) with their share of the
// pair-phase flops in tenths, and the pair count to a power of two.
std::string shape_key(const Resident* R, int prec) {
    std::map<std::pair<int, int>, double> w;
    double tot = 0.0;
    for (const PairDesc& p : R->pairs) {
        int a = R->monos[p.x].np, b = R->monos[p.y].np;
        if (a > b) std::swap(a, b);
        const double f = (double)a * b * (a + b);
        w[{a, b}] += f;
        tot += f;
    }
    std::string k = std::string(prec == MCPT_BF16 ? "bf16" : "fp32");
    for (const auto& kv : w)
        k += "/" + std::to_string(kv.first.first) + "x" + std::to_string(kv.first.second) + ":" +
             std::to_string((int)std::lround(10.0 * kv.second / std::max(tot, 1.0)));
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= R->n_pair) ++lg;
    return k + "/p2^" + std::to_string(lg);
}

// Time one coupled reduced-precision pair phase per tile-shape variant on the
// resident problem and keep the fastest (for this problem and, under its shape
// key, for later problems of the context).  Clobbers G and E_D2: the problem's
// previous results are invalidated.
mcpt_status autotune(mcpt_ctx* c, Exec& x, Resident* R, int prec, mcpt_tune_result* out) {
    mcpt_status st;
    if ((st = ensure_device(c)) != MCPT_OK || (st = ensure_lowp(c, x, R, prec)) != MCPT_OK) return st;
    R->has_result = false;
    const int nv = std::min(lowp_variants(), 16);
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    std::vector<double> ms(nv, 0.0);
    int best = 0;
    for (int v = 0; v < nv; ++v) {
        R->lo_variant = v;
        if ((st = ensure_scratch_lo(c, x, R, prec)) != MCPT_OK) break;
        lowp_phase(c, x, R, R->d_G[0], R->d_G32[0], 1, true);   // warm-up
        HIP_TRY(hipEventRecord(a, x.stream));
        constexpr int reps = 3;
        for (int k = 0; k < reps; ++k) lowp_phase(c, x, R, R->d_G[0], R->d_G32[0], 1, true);
        HIP_TRY(hipEventRecord(b, x.stream));
        HIP_TRY(hipEventSynchronize(b));
        HIP_TRY(hipGetLastError());
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, a, b));
        ms[v] = t / reps;
        if (ms[v] < ms[best]) best = v;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != MCPT_OK) return st;
    R->lo_variant = best;
    {
        std::lock_guard<std::mutex> g(c->mu);
        c->tune[shape_key(R, prec)] = best;
    }
    if (out) {
        *out = mcpt_tune_result{};
        out->n_variants = nv;
        out->best = best;
        for (int v = 0; v < nv; ++v) {
            lowp_variant_shape(v, &out->sb[v], &out->nw[v], &out->pd[v]);
            out->ms[v] = ms[v];
        }
    }
    return ensure_scratch_lo(c, x, R, prec);
}

// Singles buffers of a resident problem, made once and kept with it.
mcpt_status ensure_singles(mcpt_ctx* c, Exec& x, Resident* R) {
    if (R->d_w1) return MCPT_OK;
    auto rnd = [](int64_t bytes) { return (size_t)((std::max<int64_t>(bytes, 1) + 255) / 256 * 256); };
    const size_t need = 3 * rnd(8 * R->dif_elems) + 3 * rnd(8 * (int64_t)R->n_mono) +
                        rnd(8 * (int64_t)R->n_cl * kMaxSweeps) + rnd((int64_t)R->n_cl * (int64_t)sizeof(ClState)) +
                        rnd(8 * (int64_t)(R->n_mono + 1));
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (c->in_use + (c->reserved - x.reserved) + need > c->budget)
            return fail(MCPT_ERR_ADMISSION, "singles buffers exceed the budget");
    }
    mcpt_status st;
    if ((st = dev_alloc(c, R, &R->d_w1, R->dif_elems)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_t1, R->dif_elems)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_u1, R->dif_elems)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_em1, R->n_mono)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_em1_0, R->n_mono)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_res1, R->n_mono)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_hist1, (int64_t)R->n_cl * kMaxSweeps)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_cl1, R->n_cl)) != MCPT_OK ||
        (st = dev_alloc(c, R, &R->d_woff, (int64_t)R->n_mono + 1)) != MCPT_OK) {
        R->d_w1 = nullptr;   // the pieces already made stay with the problem and are freed with it
        return st;
    }
    std::vector<int64_t> woff(R->n_mono + 1, 0);
    for (int m = 0; m < R->n_mono; ++m) woff[m + 1] = woff[m] + R->monos[m].n;
    HIP_TRY(hipMemcpyAsync(R->d_woff, woff.data(), woff.size() * sizeof(int64_t), hipMemcpyHostToDevice, x.stream));
    HIP_TRY(hipStreamSynchronize(x.stream));
    return MCPT_OK;
}

// Singles solve of a resident problem (Eq. 57 pair coupling, Eq. 53 energies).
mcpt_status singles(mcpt_ctx* c, Exec& x, Resident* R, const double* w, int32_t memory, const mcpt_options* o,
                    mcpt_singles_summary* out) {
    mcpt_status st = validate_options(o);
    if (st != MCPT_OK) return st;
    if (o->precision != MCPT_FP64) return fail(MCPT_ERR_INVALID, "singles run in FP64 only");
    if (o->deterministic) return fail(MCPT_ERR_INVALID, "singles have no deterministic mode");
    if (memory != MCPT_HOST && memory != MCPT_DEVICE) return fail(MCPT_ERR_INVALID, "memory must be MCPT_HOST or MCPT_DEVICE");
    int64_t nw = 0;
    for (const MonoDesc& m : R->monos) nw += m.n;
    if (!w && nw > 0) return fail(MCPT_ERR_INVALID, "w is NULL");
    if ((st = ensure_device(c)) != MCPT_OK || (st = ensure_singles(c, x, R)) != MCPT_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = x.stream;
    R->has_singles = false;
    // w: checked, then scattered into the padded layout (d_u1 stages the compact copy)
    if (nw > 0) {
        if (memory == MCPT_HOST) {
            for (int64_t k = 0; k < nw; ++k)
                if (!std::isfinite(w[k])) return fail(MCPT_ERR_NONFINITE, "w has a non-finite value");
            HIP_TRY(hipMemcpyAsync(R->d_u1, w, nw * sizeof(double), hipMemcpyHostToDevice, s));
        } else {
            HIP_TRY(hipMemcpyAsync(R->d_u1, w, nw * sizeof(double), hipMemcpyDeviceToDevice, s));
            *x.h_flag = 0;
            HIP_TRY(hipMemcpyAsync(x.d_flag, x.h_flag, sizeof(int32_t), hipMemcpyHostToDevice, s));
            launch_nonfinite(R->d_u1, nw, x.d_flag, s);
            HIP_TRY(hipMemcpyAsync(x.h_flag, x.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (*x.h_flag) return fail(MCPT_ERR_NONFINITE, "w has a non-finite value");
        }
        launch_singles_scatter(R->d_monos, R->n_mono, R->d_woff, R->d_u1, R->d_w1, s);
    }
    launch_fill(R->d_u1, R->dif_elems, 0.0, s);
    Ctrl& h = *x.h_ctrl;
    std::memset(&h, 0, sizeof(Ctrl));
    h.fixed = o->tol == 0.0;
    h.max_sweeps = o->max_sweeps;
    h.tol = o->tol;
    HIP_TRY(hipMemcpyAsync(x.d_ctrl, &h, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    {
        std::vector<ClState> zero(R->n_cl, ClState{});
        for (int q = 0; q < R->n_cl; ++q)
            if (!R->cl_bad.empty() && R->cl_bad[q]) {
                zero[q].done = 1;
                zero[q].status = MCPT_ERR_NONFINITE;
            }
        HIP_TRY(hipMemcpyAsync(R->d_cl1, zero.data(), R->n_cl * sizeof(ClState), hipMemcpyHostToDevice, s));
    }
    // with the intramonomer classes attached, Eq. 57's intramonomer term joins the pair sum
    const bool intra = R->lccd;
    if (intra && !R->d_ui1 && (st = dev_alloc(c, R, &R->d_ui1, R->dif_elems)) != MCPT_OK) return st;
    launch_singles_mono(1, R->d_monos, R->n_mono, R->d_dif, R->d_w1, R->d_u1, nullptr, R->d_t1, R->d_em1,
                        R->d_em1_0, R->d_res1, nullptr, R->d_cl1, s);
    HIP_TRY(hipGetLastError());
    const int grid = singles_pair_grid(c->n_cu);
    const double vb = (double)R->v_elems * sizeof(double);
    const int every = o->check_every > 0 ? o->check_every : 1;
    int issued = 0;
    while (issued < o->max_sweeps) {
        const int batch = std::min(every, o->max_sweeps - issued);
        for (int k = 0; k < batch; ++k) {
            hipEvent_t a = nullptr;
            record_begin(x, &a);
            launch_singles_pair(R->d_pairs, R->n_pair, R->d_monos, R->d_V, R->d_t1, R->d_u1, grid, x.d_ctrl, R->d_cl1,
                                s);
            record_end(x, a, 3, 0.0, vb);
            if (intra)
                launch_singles_intra(R->d_monos, R->n_mono, R->d_K, R->d_J, R->d_t1, R->d_ui1, x.d_ctrl, R->d_cl1, s);
            launch_singles_mono(0, R->d_monos, R->n_mono, R->d_dif, R->d_w1, R->d_u1, intra ? R->d_ui1 : nullptr,
                                R->d_t1, R->d_em1, R->d_em1_0, R->d_res1, x.d_ctrl, R->d_cl1, s);
            launch_reduce_sweep(R->n_cl, R->d_cl_mono, R->d_res1, R->d_cl1, R->d_hist1, x.d_ctrl, s);
            ++issued;
        }
        if ((st = sync_ctrl(x)) != MCPT_OK) return st;
        if (h.done) break;
    }
    launch_singles_clusters(R->n_cl, R->d_cl_mono, R->d_em1, R->d_em1_0, R->d_cl1, s);
    std::vector<ClState> cs(R->n_cl);
    HIP_TRY(hipMemcpyAsync(cs.data(), R->d_cl1, R->n_cl * sizeof(ClState), hipMemcpyDeviceToHost, s));
    if ((st = sync_ctrl(x)) != MCPT_OK) return st;
    if (x.timing.on) drain_timing(x.timing);
    mcpt_singles_summary sm{};
    for (const ClState& q : cs) {
        sm.e_m1 += q.e_mono;
        sm.e_m1_0 += q.e_mono0;
    }
    sm.residual = h.residual;
    sm.sweeps = h.sweeps;
    sm.status = h.status;
    sm.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    R->singles_last = sm;
    if (out) *out = sm;
    if (sm.status == MCPT_ERR_DIVERGED && R->n_cl == 1)
        return fail(MCPT_ERR_DIVERGED, "singles iteration diverged after " + std::to_string(sm.sweeps) + " sweeps");
    R->has_singles = true;
    if (sm.status == MCPT_ERR_NOT_CONVERGED)
        return fail(MCPT_ERR_NOT_CONVERGED, "singles not converged in " + std::to_string(o->max_sweeps) + " sweeps");
    return (mcpt_status)sm.status;
}

// Intramonomer integral classes of the full monomer equation (Eq. 58):
// validated, copied, packed and kept with the problem; in == nullptr detaches.
mcpt_status lccd_attach(mcpt_ctx* c, Exec& x, Resident* R, const mcpt_lccd_integrals* in) {
    mcpt_status st;
    if ((st = ensure_device(c)) != MCPT_OK) return st;
    hipStream_t s = x.stream;
    HIP_TRY(hipStreamSynchronize(s));
    drop_graph(R);
    free_lccd(c, R);
    if (!in) return MCPT_OK;
    if (in->memory != MCPT_HOST && in->memory != MCPT_DEVICE)
        return fail(MCPT_ERR_INVALID, "memory must be MCPT_HOST or MCPT_DEVICE");
    std::vector<LccdDesc> ld(R->n_mono);
    int64_t nw = 0, nq = 0, w_pack = 0;
    int max_rows = 16, max_o = 1, max_np = 16;
    for (int m = 0; m < R->n_mono; ++m) {
        const MonoDesc& d = R->monos[m];
        if (d.o > 8 || d.v > 64 || d.np > kLccdMaxNp)
            return fail(MCPT_ERR_INVALID, "monomer " + std::to_string(m) +
                                              ": the full monomer equation supports o <= 8, v <= 64, o v <= 1024");
        const int v2 = d.v * d.v, rows = round_up(v2, 16), cols = round_up(v2, 32);
        ld[m] = LccdDesc{w_pack, nw, nq, rows, cols};
        w_pack += (int64_t)rows * cols;
        nw += (int64_t)v2 * v2;
        nq += (int64_t)d.o * d.o * d.o * d.o;
        max_rows = std::max(max_rows, rows);
        max_o = std::max(max_o, d.o);
        max_np = std::max(max_np, d.np);
    }
    const int64_t nj = R->raw_elems;
    if ((nw > 0 && !in->w_vvvv) || (nq > 0 && !in->q_oooo) || (nj > 0 && !in->j_oovv))
        return fail(MCPT_ERR_INVALID, "an integral array is NULL");
    const bool host = in->memory == MCPT_HOST;
    if (host) {
        auto finite = [](const double* p, int64_t n) {
            for (int64_t k = 0; k < n; ++k)
                if (!std::isfinite(p[k])) return false;
            return true;
        };
        if (!finite(in->w_vvvv, nw) || !finite(in->q_oooo, nq) || !finite(in->j_oovv, nj))
            return fail(MCPT_ERR_NONFINITE, "intramonomer integrals have a non-finite value");
    } else {
        *x.h_flag = 0;
        HIP_TRY(hipMemcpyAsync(x.d_flag, x.h_flag, sizeof(int32_t), hipMemcpyHostToDevice, s));
        launch_nonfinite(in->w_vvvv, nw, x.d_flag, s);
        launch_nonfinite(in->q_oooo, nq, x.d_flag, s);
        launch_nonfinite(in->j_oovv, nj, x.d_flag, s);
        HIP_TRY(hipMemcpyAsync(x.h_flag, x.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*x.h_flag) return fail(MCPT_ERR_NONFINITE, "intramonomer integrals have a non-finite value");
    }
    auto rnd = [](int64_t bytes) { return (size_t)((std::max<int64_t>(bytes, 1) + 255) / 256 * 256); };
    const size_t keep = rnd(8 * w_pack) + rnd(8 * nq) + 4 * rnd(8 * R->mat_elems) + rnd(8 * (int64_t)R->n_mono) +
                        rnd((int64_t)sizeof(LccdDesc) * R->n_mono);
    const size_t staging = host ? rnd(8 * std::max(nw, nj)) : 0;
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (c->in_use + (c->reserved - x.reserved) + keep + staging > c->budget)
            return fail(MCPT_ERR_ADMISSION, "intramonomer integrals exceed the budget");
    }
    auto alloc = [&](void** out, size_t bytes) -> mcpt_status {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MCPT_ERR_NOMEM, "hipMalloc of intramonomer buffers failed");
        }
        R->lccd_allocations.push_back(p);
        R->lccd_bytes += bytes;
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use += bytes;
        *out = p;
        return MCPT_OK;
    };
    void* pv[8] = {};
    if ((st = alloc(&pv[0], rnd(8 * w_pack))) != MCPT_OK || (st = alloc(&pv[1], rnd(8 * nq))) != MCPT_OK ||
        (st = alloc(&pv[2], rnd(8 * R->mat_elems))) != MCPT_OK ||
        (st = alloc(&pv[3], rnd(8 * R->mat_elems))) != MCPT_OK ||
        (st = alloc(&pv[4], rnd(8 * R->mat_elems))) != MCPT_OK ||
        (st = alloc(&pv[5], rnd(8 * R->mat_elems))) != MCPT_OK ||
        (st = alloc(&pv[6], rnd(8 * (int64_t)R->n_mono))) != MCPT_OK ||
        (st = alloc(&pv[7], rnd((int64_t)sizeof(LccdDesc) * R->n_mono))) != MCPT_OK) {
        free_lccd(c, R);
        return st;
    }
    R->d_W = static_cast<double*>(pv[0]);
    R->d_Q = static_cast<double*>(pv[1]);
    R->d_J = static_cast<double*>(pv[2]);
    R->d_L = static_cast<double*>(pv[3]);
    R->d_R12 = static_cast<double*>(pv[4]);
    R->d_Y = static_cast<double*>(pv[5]);
    R->d_elccd = static_cast<double*>(pv[6]);
    R->d_lccd = static_cast<LccdDesc*>(pv[7]);
    R->lccd_desc = ld;
    auto fail_free = [&](mcpt_status e) {
        free_lccd(c, R);
        return e;
    };
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(R->d_lccd, ld.data(), ld.size() * sizeof(LccdDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
        (nq > 0 && hipMemcpyAsync(R->d_Q, in->q_oooo, nq * sizeof(double), kind, s) != hipSuccess))
        return fail_free(fail(MCPT_ERR_DEVICE, "copy of intramonomer integrals failed"));
    launch_fill(R->d_L, R->mat_elems, 0.0, s);
    launch_fill(R->d_R12, R->mat_elems, 0.0, s);
    launch_fill(R->d_Y, R->mat_elems, 0.0, s);
    if (host) {
        // host arrays go through one temporary device buffer, W and then J
        void* stage = nullptr;
        if (hipMalloc(&stage, staging) != hipSuccess) {
            (void)hipGetLastError();
            return fail_free(fail(MCPT_ERR_NOMEM, "hipMalloc of the integral staging buffer failed"));
        }
        hipError_t e = hipMemcpyAsync(stage, in->w_vvvv, nw * sizeof(double), hipMemcpyHostToDevice, s);
        launch_lccd_pack(R->d_monos, R->d_lccd, R->n_mono, static_cast<double*>(stage), nullptr, R->d_W, nullptr, s);
        if (e == hipSuccess) e = hipMemcpyAsync(stage, in->j_oovv, nj * sizeof(double), hipMemcpyHostToDevice, s);
        launch_lccd_pack(R->d_monos, R->d_lccd, R->n_mono, nullptr, static_cast<double*>(stage), nullptr, R->d_J, s);
        const hipError_t e2 = hipStreamSynchronize(s);
        (void)hipFree(stage);
        if (e != hipSuccess || e2 != hipSuccess)
            return fail_free(fail(MCPT_ERR_DEVICE, "upload of intramonomer integrals failed"));
    } else {
        launch_lccd_pack(R->d_monos, R->d_lccd, R->n_mono, in->w_vvvv, in->j_oovv, R->d_W, R->d_J, s);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail_free(fail(MCPT_ERR_DEVICE, "packing of intramonomer integrals failed"));
    R->lccd_ring_blocks = lccd_ring_blocks(max_np);
    R->lccd_ladder_blocks = lccd_ladder_blocks(max_rows, max_o);
    R->lccd_ct = lccd_ladder_ct(max_o);
    // the LDS-staged ladder when every monomer's amplitudes fit one workgroup's LDS
    R->lccd_lds_bytes = 0;
    for (int m = 0; m < R->n_mono; ++m)
        R->lccd_lds_bytes =
            std::max(R->lccd_lds_bytes, lccd_ladder_lds_bytes(R->monos[m].n, R->monos[m].v, ld[m].ldw));
    if (R->lccd_lds_bytes > lccd_lds_limit() || R->lccd_ct > 3) R->lccd_lds_bytes = 0;
    R->lccd_w_bytes = 8.0 * (double)w_pack;
    double fl = 0.0;
    for (const MonoDesc& d : R->monos) fl += 2.0 * (double)d.o * d.o * (double)d.v * d.v * (double)d.v * d.v;
    R->lccd_w_flops = fl;
    R->lccd = true;
    R->has_result = false;
    return MCPT_OK;
}

// Dimer classes of the dimer-internal terms of Eq. 59: validated, copied, packed
// and kept with the problem; in == nullptr detaches.  Each pair gets a DimerDesc
// (sizes of its two monomers, offsets of its matrices).  When every monomer has
// one size and a pair's n x n Tau fits one workgroup's LDS, the pair ladders run
// on the LDS-staged monomer ladder kernel, each pair described to it as a
// monomer would be (n = o v, its matrices at its Tau offset, its W_XY packed like
// a monomer's W); otherwise on the global-memory pair ladder kernel.
mcpt_status dimer_attach(mcpt_ctx* c, Exec& x, Resident* R, const mcpt_dimer_integrals* in) {
    mcpt_status st;
    if ((st = ensure_device(c)) != MCPT_OK) return st;
    hipStream_t s = x.stream;
    HIP_TRY(hipStreamSynchronize(s));
    drop_graph(R);
    free_dimer(c, R);
    R->has_result = false;
    if (!in) return MCPT_OK;
    if (!R->lccd) return fail(MCPT_ERR_INVALID, "the dimer-internal terms need the intramonomer integrals attached");
    if (in->memory != MCPT_HOST && in->memory != MCPT_DEVICE)
        return fail(MCPT_ERR_INVALID, "memory must be MCPT_HOST or MCPT_DEVICE");
    if (R->n_mono <= 0 || R->n_pair <= 0) return fail(MCPT_ERR_INVALID, "the problem has no pairs");
    if (R->n_pair > 65535) return fail(MCPT_ERR_INVALID, "the dimer-internal terms support at most 65,535 pairs");
    for (const MonoDesc& m : R->monos)
        if (m.o > 8 || m.v > 64) return fail(MCPT_ERR_INVALID, "the dimer-internal terms support o <= 8 and v <= 64");
    const MonoDesc m0 = R->monos[0];
    bool one_size = true;
    for (const MonoDesc& m : R->monos) one_size = one_size && m.o == m0.o && m.v == m0.v;
    const int64_t P = R->n_pair;
    // per pair (caller order): sizes, offsets in the packed buffers and in the caller's concatenation
    std::vector<DimerDesc> dd(P);
    for (const PairDesc& pd : R->pairs) {
        DimerDesc d{};
        d.x = pd.x;
        d.y = pd.y;
        d.cluster = pd.cluster;
        dd[pd.orig] = d;
    }
    int64_t nw = 0, nq = 0, ncx = 0, ncy = 0, w_pack = 0, tau_el = 0, y_el = 0, cx_el = 0, cy_el = 0;
    int max_rows = 16, max_o2 = 1, max_ring = 1;
    double w_flops = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        DimerDesc& d = dd[p];
        const MonoDesc &mx = R->monos[d.x], &my = R->monos[d.y];
        d.ox = mx.o;
        d.vx = mx.v;
        d.oy = my.o;
        d.vy = my.v;
        d.nx = mx.n;
        d.ny = my.n;
        d.npx = mx.np;
        d.npy = my.np;
        d.m1 = round_up(d.ox * d.vy, 16);
        d.m2 = round_up(d.oy * d.vx, 16);
        const int v2 = d.vx * d.vy, o2 = d.ox * d.oy;
        d.w_rows = round_up(v2, 16);
        d.ldw = round_up(v2, 32);
        d.w_raw_off = nw;
        d.q_off = nq;
        d.cx_raw_off = ncx;
        d.cy_raw_off = ncy;
        d.w_off = w_pack;
        d.tau_off = tau_el;
        d.y1_off = d.y2_off = y_el;   // Y1 and Y2 sit in two buffers of the same layout size
        d.cx_off = cx_el;
        d.cy_off = cy_el;
        nw += (int64_t)v2 * v2;
        nq += (int64_t)o2 * o2;
        ncx += (int64_t)d.ox * d.ox * d.vy * d.vy;
        ncy += (int64_t)d.oy * d.oy * d.vx * d.vx;
        w_pack += (int64_t)d.w_rows * d.ldw;
        tau_el += (int64_t)d.npx * d.npy;
        y_el += (int64_t)d.m1 * d.m2;
        cx_el += (int64_t)d.m1 * d.m1;
        cy_el += (int64_t)d.m2 * d.m2;
        max_rows = std::max(max_rows, d.w_rows);
        max_o2 = std::max(max_o2, o2);
        max_ring = std::max(max_ring, dimer_ring_tasks(d));
        w_flops += 2.0 * o2 * (double)v2 * v2;
    }
    // the LDS-staged ladder for one-size problems whose pairs fit it (the pair is its own "monomer")
    const int np = m0.np, n = m0.n;
    int64_t lds = 0;
    if (one_size) {
        lds = lccd_ladder_lds_bytes(n, m0.v, round_up(m0.v * m0.v, 32));
        if (lds > lccd_lds_limit() || lccd_ladder_ct(m0.o) > 3) lds = 0;
    }
    if (!in->w_vvvv || !in->q_oooo || !in->c_x || !in->c_y) return fail(MCPT_ERR_INVALID, "an integral array is NULL");
    const bool host = in->memory == MCPT_HOST;
    if (host) {
        auto finite = [](const double* p, int64_t k) {
            for (int64_t e = 0; e < k; ++e)
                if (!std::isfinite(p[e])) return false;
            return true;
        };
        if (!finite(in->w_vvvv, nw) || !finite(in->q_oooo, nq) || !finite(in->c_x, ncx) || !finite(in->c_y, ncy))
            return fail(MCPT_ERR_NONFINITE, "dimer integrals have a non-finite value");
    } else {
        *x.h_flag = 0;
        HIP_TRY(hipMemcpyAsync(x.d_flag, x.h_flag, sizeof(int32_t), hipMemcpyHostToDevice, s));
        launch_nonfinite(in->w_vvvv, nw, x.d_flag, s);
        launch_nonfinite(in->q_oooo, nq, x.d_flag, s);
        launch_nonfinite(in->c_x, ncx, x.d_flag, s);
        launch_nonfinite(in->c_y, ncy, x.d_flag, s);
        HIP_TRY(hipMemcpyAsync(x.h_flag, x.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*x.h_flag) return fail(MCPT_ERR_NONFINITE, "dimer integrals have a non-finite value");
    }
    // the LDS-staged ladder takes monomer-like descriptors of the pairs
    std::vector<MonoDesc> pm(lds > 0 ? P : 0);
    std::vector<LccdDesc> pl(lds > 0 ? P : 0);
    for (int64_t p = 0; lds > 0 && p < P; ++p) {
        MonoDesc d{};
        d.o = m0.o;
        d.v = m0.v;
        d.n = n;
        d.np = np;
        d.mat_off = dd[p].tau_off;
        d.cluster = dd[p].cluster;
        pm[p] = d;
        pl[p] = LccdDesc{dd[p].w_off, dd[p].w_raw_off, dd[p].q_off, dd[p].w_rows, dd[p].ldw};
    }
    auto rnd = [](int64_t bytes) { return (size_t)((std::max<int64_t>(bytes, 1) + 255) / 256 * 256); };
    const size_t sizes[12] = {rnd(8 * w_pack), rnd(8 * nq), rnd(8 * cx_el), rnd(8 * cy_el), rnd(8 * tau_el),
                              rnd(8 * tau_el), rnd(sizeof(DimerDesc) * P), rnd(sizeof(MonoDesc) * pm.size()),
                              rnd(sizeof(LccdDesc) * pl.size()), rnd(8 * R->mat_elems), rnd(8 * y_el),
                              rnd(8 * y_el)};
    size_t keep = 0;
    for (size_t b : sizes) keep += b;
    const size_t staging = host ? rnd(8 * std::max(nw, std::max(ncx, ncy))) : 0;
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (c->in_use + (c->reserved - x.reserved) + keep + staging > c->budget)
            return fail(MCPT_ERR_ADMISSION, "dimer integrals exceed the budget");
    }
    auto alloc = [&](void** out, size_t bytes) -> mcpt_status {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MCPT_ERR_NOMEM, "hipMalloc of dimer buffers failed");
        }
        R->dimer_allocations.push_back(p);
        R->dimer_bytes += bytes;
        std::lock_guard<std::mutex> g(c->mu);
        c->in_use += bytes;
        *out = p;
        return MCPT_OK;
    };
    void* pv[12] = {};
    for (int k = 0; k < 12; ++k)
        if ((st = alloc(&pv[k], sizes[k])) != MCPT_OK) {
            free_dimer(c, R);
            return st;
        }
    R->d_DW = static_cast<double*>(pv[0]);
    R->d_DQ = static_cast<double*>(pv[1]);
    R->d_DCX = static_cast<double*>(pv[2]);
    R->d_DCY = static_cast<double*>(pv[3]);
    R->d_Tau = static_cast<double*>(pv[4]);
    R->d_S = static_cast<double*>(pv[5]);
    R->d_dd = static_cast<DimerDesc*>(pv[6]);
    R->d_pmono = static_cast<MonoDesc*>(pv[7]);
    R->d_plccd = static_cast<LccdDesc*>(pv[8]);
    R->d_DRM = static_cast<double*>(pv[9]);
    R->d_DY1 = static_cast<double*>(pv[10]);
    R->d_DY2 = static_cast<double*>(pv[11]);
    auto fail_free = [&](mcpt_status e) {
        free_dimer(c, R);
        return e;
    };
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(R->d_dd, dd.data(), P * sizeof(DimerDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
        (lds > 0 && hipMemcpyAsync(R->d_pmono, pm.data(), P * sizeof(MonoDesc), hipMemcpyHostToDevice, s) != hipSuccess) ||
        (lds > 0 && hipMemcpyAsync(R->d_plccd, pl.data(), P * sizeof(LccdDesc), hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(R->d_DQ, in->q_oooo, nq * sizeof(double), kind, s) != hipSuccess)
        return fail_free(fail(MCPT_ERR_DEVICE, "copy of dimer integrals failed"));
    launch_fill(R->d_Tau, tau_el, 0.0, s);
    launch_fill(R->d_S, tau_el, 0.0, s);
    launch_fill(R->d_DY1, y_el, 0.0, s);
    launch_fill(R->d_DY2, y_el, 0.0, s);
    launch_ring_matrix(R->d_K, R->d_J, R->d_DRM, R->mat_elems, s);
    const int pn = (int)P;
    if (host) {
        // host arrays go through one temporary device buffer: W, then C_X, then C_Y
        void* stage = nullptr;
        if (hipMalloc(&stage, staging) != hipSuccess) {
            (void)hipGetLastError();
            return fail_free(fail(MCPT_ERR_NOMEM, "hipMalloc of the integral staging buffer failed"));
        }
        double* sd = static_cast<double*>(stage);
        hipError_t e = hipMemcpyAsync(stage, in->w_vvvv, nw * sizeof(double), hipMemcpyHostToDevice, s);
        launch_dimer_pack(R->d_dd, pn, sd, nullptr, nullptr, R->d_DW, nullptr, nullptr, s);
        if (e == hipSuccess) e = hipMemcpyAsync(stage, in->c_x, ncx * sizeof(double), hipMemcpyHostToDevice, s);
        launch_dimer_pack(R->d_dd, pn, nullptr, sd, nullptr, nullptr, R->d_DCX, nullptr, s);
        if (e == hipSuccess) e = hipMemcpyAsync(stage, in->c_y, ncy * sizeof(double), hipMemcpyHostToDevice, s);
        launch_dimer_pack(R->d_dd, pn, nullptr, nullptr, sd, nullptr, nullptr, R->d_DCY, s);
        const hipError_t e2 = hipStreamSynchronize(s);
        (void)hipFree(stage);
        if (e != hipSuccess || e2 != hipSuccess) return fail_free(fail(MCPT_ERR_DEVICE, "upload of dimer integrals failed"));
    } else {
        launch_dimer_pack(R->d_dd, pn, in->w_vvvv, in->c_x, in->c_y, R->d_DW, R->d_DCX, R->d_DCY, s);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail_free(fail(MCPT_ERR_DEVICE, "packing of dimer integrals failed"));
    R->dimer_desc = std::move(dd);
    R->dimer_one_size = one_size;
    R->dimer_tau_elems = tau_el;
    R->dimer_lds_bytes = lds;
    R->dimer_ct = lds > 0 ? lccd_ladder_ct(m0.o) : dimer_ladder_ct(max_o2);
    R->dimer_ladder_blocks = lds > 0 ? 1 : dimer_ladder_blocks(max_rows, max_o2);
    R->dimer_ring_blocks = dimer_ring_blocks(max_ring);
    R->dimer_w_bytes = 8.0 * (double)w_pack;
    R->dimer_w_flops = w_flops;
    R->dimer = true;
    return MCPT_OK;
}

// A new resident problem that is the resident problem B with the blocks of the
// listed pairs (caller indices) multiplied by their factors: a displaced
// geometry whose couplings are rescaled (Sec. IV.A), made on the device from
// B's packed inputs without a host upload.
mcpt_status clone_scaled(mcpt_ctx* c, Exec& x, Resident* B, int64_t n, const int64_t* pair, const double* scale,
                         uint64_t* id_out) {
    if (!id_out) return fail(MCPT_ERR_INVALID, "id is NULL");
    if (n < 0 || (n > 0 && (!pair || !scale))) return fail(MCPT_ERR_INVALID, "pair or scale is NULL");
    mcpt_status st;
    if ((st = ensure_device(c)) != MCPT_OK) return st;
    std::vector<int64_t> where(B->n_pair, -1);
    for (int64_t q = 0; q < B->n_pair; ++q) where[B->pairs[q].orig] = q;
    std::vector<int64_t> off(n), len(n);
    std::unordered_set<int64_t> seen;
    for (int64_t k = 0; k < n; ++k) {
        if (pair[k] < 0 || pair[k] >= B->n_pair)
            return fail(MCPT_ERR_INVALID, "pair index " + std::to_string(pair[k]) + " out of range");
        if (!seen.insert(pair[k]).second)
            return fail(MCPT_ERR_INVALID, "pair " + std::to_string(pair[k]) + " listed twice");
        if (!std::isfinite(scale[k])) return fail(MCPT_ERR_NONFINITE, "non-finite scale factor");
        const PairDesc& d = B->pairs[where[pair[k]]];
        off[k] = d.v_off;
        len[k] = (int64_t)B->monos[d.x].n * B->monos[d.y].n;
    }
    auto rnd = [](int64_t bytes) { return (size_t)((std::max<int64_t>(bytes, 1) + 255) / 256 * 256); };
    const size_t need = rnd(sizeof(MonoDesc) * (int64_t)B->n_mono) + rnd(sizeof(PairDesc) * B->n_pair) +
                        rnd(8 * B->dif_elems) + rnd(8 * B->raw_elems) + 5 * rnd(8 * B->mat_elems) +
                        rnd(8 * B->v_elems) + 3 * rnd(8 * (int64_t)B->n_mono) + rnd(8 * B->n_pair) +
                        rnd((int64_t)sizeof(ClState) * B->n_cl) + rnd(8 * (int64_t)B->n_cl * kMaxSweeps) +
                        2 * rnd(8 * (int64_t)(B->n_cl + 1)) + 3 * rnd(8 * n);
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (c->in_use + (c->reserved - x.reserved) + need > c->budget)
            return fail(MCPT_ERR_ADMISSION, "displaced copy needs " + std::to_string(need) + " bytes beyond the budget");
    }
    auto r = std::make_unique<Resident>();
    Resident* R = r.get();
    R->n_mono = B->n_mono;
    R->n_pair = B->n_pair;
    R->max_n = B->max_n;
    R->max_np = B->max_np;
    R->max_v = B->max_v;
    R->eps_elems = B->eps_elems;
    R->dif_elems = B->dif_elems;
    R->raw_elems = B->raw_elems;
    R->mat_elems = B->mat_elems;
    R->v_elems = B->v_elems;
    R->max_slot = B->max_slot;
    R->monos = B->monos;
    R->pairs = B->pairs;
    R->n_lds = B->n_lds;
    R->n_cl = B->n_cl;
    R->cl_mono = B->cl_mono;
    R->cl_pair = B->cl_pair;
    R->cl_bad = B->cl_bad;
    R->cl_last.assign(R->n_cl, mcpt_summary{});
#define ALLOC(ptr, cnt)                                          \
    do {                                                         \
        if ((st = dev_alloc(c, R, &(ptr), (cnt))) != MCPT_OK) { \
            free_resident(c, R);                                 \
            return st;                                           \
        }                                                        \
    } while (0)
    int64_t *d_off = nullptr, *d_len = nullptr;
    double* d_f = nullptr;
    ALLOC(R->d_monos, R->n_mono);
    ALLOC(R->d_pairs, std::max<int64_t>(R->n_pair, 1));
    ALLOC(R->d_dif, R->dif_elems);
    ALLOC(R->d_raw, R->raw_elems);
    ALLOC(R->d_K, R->mat_elems);
    ALLOC(R->d_T, R->mat_elems);
    ALLOC(R->d_M, R->mat_elems);
    ALLOC(R->d_G[0], R->mat_elems);
    ALLOC(R->d_G[1], R->mat_elems);
    ALLOC(R->d_V, std::max<int64_t>(R->v_elems, 1));
    ALLOC(R->d_em2, R->n_mono);
    ALLOC(R->d_em2_0, R->n_mono);
    ALLOC(R->d_res, R->n_mono);
    ALLOC(R->d_ed2, std::max<int64_t>(R->n_pair, 1));
    ALLOC(R->d_cl, R->n_cl);
    ALLOC(R->d_hist, (int64_t)R->n_cl * kMaxSweeps);
    ALLOC(R->d_cl_mono, R->n_cl + 1);
    ALLOC(R->d_cl_pair, R->n_cl + 1);
    ALLOC(d_off, std::max<int64_t>(n, 1));
    ALLOC(d_len, std::max<int64_t>(n, 1));
    ALLOC(d_f, std::max<int64_t>(n, 1));
#undef ALLOC
    hipStream_t s = x.stream;
    const hipMemcpyKind dd = hipMemcpyDeviceToDevice;
    auto copy = [&](void* dst, const void* src, int64_t bytes) {
        return bytes > 0 ? hipMemcpyAsync(dst, src, bytes, dd, s) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = copy(R->d_monos, B->d_monos, sizeof(MonoDesc) * (int64_t)R->n_mono);
    if (e == hipSuccess) e = copy(R->d_pairs, B->d_pairs, sizeof(PairDesc) * R->n_pair);
    if (e == hipSuccess) e = copy(R->d_dif, B->d_dif, 8 * R->dif_elems);
    if (e == hipSuccess) e = copy(R->d_K, B->d_K, 8 * R->mat_elems);
    if (e == hipSuccess) e = copy(R->d_V, B->d_V, 8 * R->v_elems);
    if (e == hipSuccess) e = copy(R->d_cl_mono, B->d_cl_mono, 8 * (int64_t)(R->n_cl + 1));
    if (e == hipSuccess) e = copy(R->d_cl_pair, B->d_cl_pair, 8 * (int64_t)(R->n_cl + 1));
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(d_off, off.data(), 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(d_len, len.data(), 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(d_f, scale, 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        launch_scale_blocks(d_off, d_len, d_f, n, R->d_V, s);
        launch_fill(R->d_T, R->mat_elems, 0.0, s);
        launch_fill(R->d_M, R->mat_elems, 0.0, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_resident(c, R);
        return fail(MCPT_ERR_DEVICE, std::string("displaced copy: ") + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> g(c->mu);
    r->id = c->next_id++;
    *id_out = r->id;
    c->res[r->id] = std::move(r);
    return MCPT_OK;
}

// Unit energy of Eq. 66 over the listed monomers from the last results of R:
// E_M2 (Eq. 54) and, after a singles solve, E_M1 (Eq. 53).
mcpt_status unit_energy(Exec& x, Resident* R, int32_t n_cell, const int32_t* cell, bool with_singles, double* e) {
    std::vector<double> a(R->n_mono), b;
    HIP_TRY(hipMemcpyAsync(a.data(), R->d_em2, 8 * (int64_t)R->n_mono, hipMemcpyDeviceToHost, x.stream));
    if (with_singles) {
        b.resize(R->n_mono);
        HIP_TRY(hipMemcpyAsync(b.data(), R->d_em1, 8 * (int64_t)R->n_mono, hipMemcpyDeviceToHost, x.stream));
    }
    HIP_TRY(hipStreamSynchronize(x.stream));
    double sum = 0.0;
    for (int32_t k = 0; k < n_cell; ++k) {
        sum += a[cell[k]];
        if (with_singles) sum += b[cell[k]];
    }
    *e = sum;
    return MCPT_OK;
}

// Five-point finite-difference second derivatives of the unit energy along
// displacement modes (Sec. IV.A): the base geometry and, per mode, the four
// displaced geometries -2h, -h, +h, +2h as rescaled copies of the base, each
// solved from the base's converged amplitudes.
mcpt_status fd_stencil(mcpt_ctx* c, Exec& x, Resident* B, int32_t n_modes, const mcpt_fd_mode* modes, int32_t n_cell,
                       const int32_t* cell, double step, const double* w, const mcpt_options* o,
                       mcpt_fd_result* out) {
    if (n_modes < 1 || !modes || !out) return fail(MCPT_ERR_INVALID, "need at least one mode and an output array");
    if (n_cell < 1 || !cell) return fail(MCPT_ERR_INVALID, "need at least one unit-cell monomer");
    if (!(step > 0.0) || !std::isfinite(step)) return fail(MCPT_ERR_INVALID, "step must be positive");
    for (int32_t k = 0; k < n_cell; ++k)
        if (cell[k] < 0 || cell[k] >= B->n_mono) return fail(MCPT_ERR_INVALID, "unit-cell monomer out of range");
    if (B->lccd) return fail(MCPT_ERR_INVALID, "finite differences run on problems without intramonomer integrals");
    mcpt_status st = validate_options(o);
    if (st != MCPT_OK) return st;
    if (o->warm_t) return fail(MCPT_ERR_INVALID, "warm_t is set by the finite-difference driver");
    const bool sg = w != nullptr;
    const auto point = [&](Resident* R, const mcpt_options* oo, double* e, int32_t* sweeps) -> mcpt_status {
        mcpt_summary sm{};
        mcpt_status r = run(c, x, R, oo, &sm);
        if (r != MCPT_OK) return r;
        *sweeps = sm.sweeps;
        if (sg) {
            mcpt_options os = *oo;
            os.warm_t = nullptr;
            os.precision = MCPT_FP64;
            os.deterministic = 0;
            mcpt_singles_summary ss{};
            if ((r = singles(c, x, R, w, MCPT_HOST, &os, &ss)) != MCPT_OK) return r;
        }
        return unit_energy(x, R, n_cell, cell, sg, e);
    };
    double e0 = 0.0;
    int32_t sw0 = 0;
    if ((st = point(B, o, &e0, &sw0)) != MCPT_OK) return st;
    std::vector<double> t0(B->raw_elems);
    if ((st = slice_results(c, x, B, -1, nullptr, nullptr, nullptr, t0.data())) != MCPT_OK) return st;
    mcpt_options ow = *o;
    ow.warm_t = t0.data();
    for (int32_t m = 0; m < n_modes; ++m) {
        mcpt_fd_result& r = out[m];
        r = mcpt_fd_result{};
        r.e[2] = e0;
        r.sweeps[2] = sw0;
        static const int slot[4] = {0, 1, 3, 4};   // -2h, -h, +h, +2h
        for (int k = 0; k < 4; ++k) {
            uint64_t id = 0;
            if ((st = clone_scaled(c, x, B, modes[m].n_pair, modes[m].pair,
                                   modes[m].scale ? modes[m].scale + (int64_t)k * modes[m].n_pair : nullptr, &id)) !=
                MCPT_OK)
                return st;
            Resident* R = nullptr;
            {
                std::lock_guard<std::mutex> g(c->mu);
                R = c->res[id].get();
            }
            st = point(R, &ow, &r.e[slot[k]], &r.sweeps[slot[k]]);
            const std::string msg = last_error_text();
            (void)hipStreamSynchronize(x.stream);
            release_resident(c, id);
            if (st != MCPT_OK) {
                r.status = st;
                return fail(st, "mode " + std::to_string(m) + ", point " + std::to_string(k) + ": " + msg);
            }
        }
        r.d2e = (-r.e[4] + 16.0 * r.e[3] - 30.0 * r.e[2] + 16.0 * r.e[1] - r.e[0]) / (12.0 * step * step);
        r.status = MCPT_OK;
    }
    clear_error();
    return MCPT_OK;
}

mcpt_status run(mcpt_ctx* c, Exec& x, Resident* R, const mcpt_options* o, mcpt_summary* out) {
    mcpt_status st = validate_options(o);
    if (st != MCPT_OK) return st;
    if ((st = ensure_device(c)) != MCPT_OK) return st;
    if ((st = ensure_scratch(c, x, R->max_slot)) != MCPT_OK) return st;
    // the split form's task layout, built here because its copies may not run under graph capture
    // (the solve that allocates nothing keeps the one-launch kernel)
    if (!x.fixed_scratch && (st = ensure_glb_plan(c, R)) != MCPT_OK) return st;
    if (R->dimer && o->precision != MCPT_FP64)
        return fail(MCPT_ERR_INVALID, "a problem with dimer-internal terms runs in FP64 only");
    if (R->lccd && o->deterministic)
        return fail(MCPT_ERR_INVALID, "the full monomer equation has no deterministic mode");
    R->det_on = o->deterministic != 0;
    if (R->det_on && (st = ensure_det(c, x, R)) != MCPT_OK) return st;
    const int prec = o->precision;
    if (prec != MCPT_FP64) {
        if ((st = ensure_lowp(c, x, R, prec)) != MCPT_OK) return st;
        const std::string key = shape_key(R, prec);
        int tuned = -1;
        {
            std::lock_guard<std::mutex> g(c->mu);
            auto it = c->tune.find(key);
            if (it != c->tune.end()) tuned = it->second;
        }
        if (tuned >= 0 && tuned < lowp_variants()) R->lo_variant = tuned;
        else if (o->autotune && (st = autotune(c, x, R, prec, nullptr)) != MCPT_OK) return st;
        if ((st = ensure_scratch_lo(c, x, R, prec)) != MCPT_OK) return st;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = x.stream;
    R->has_result = false;
    Ctrl& h = *x.h_ctrl;
    auto reset_state = [&]() -> mcpt_status {
        std::memset(&h, 0, sizeof(Ctrl));
        h.fixed = o->tol == 0.0;
        h.max_sweeps = o->max_sweeps;
        h.tol = o->tol;
        HIP_TRY(hipMemcpyAsync(x.d_ctrl, &h, sizeof(Ctrl), hipMemcpyHostToDevice, s));
        std::vector<ClState> zero(R->n_cl, ClState{});
        for (int q = 0; q < R->n_cl; ++q)
            if (!R->cl_bad.empty() && R->cl_bad[q]) {   // never swept; reported as non-finite input
                zero[q].done = 1;
                zero[q].status = MCPT_ERR_NONFINITE;
            }
        HIP_TRY(hipMemcpyAsync(R->d_cl, zero.data(), R->n_cl * sizeof(ClState), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return MCPT_OK;
    };
    if ((st = reset_state()) != MCPT_OK) return st;
    if (R->dimer) launch_fill(R->d_Tau, R->dimer_tau_elems, 0.0, s);   // Tau before the first sweep
    launch_fill(R->d_G[0], R->mat_elems, 0.0, s);
    launch_fill(R->d_G[1], R->mat_elems, 0.0, s);
    // intramonomer terms of the full monomer equation, L = P + H + R + R^T from the current T and M
    // (of amplitudes Tin with Min = 2 Tin - S(Tin): T itself, or a defect correction in the polish form)
    auto lccd_terms = [&](const Ctrl* ctrl, const double* Tin = nullptr) {
        if (!Tin) Tin = R->d_T;
        hipEvent_t a = nullptr;
        record_begin(x, &a);
        launch_lccd_ring(R->d_monos, R->n_mono, R->lccd_ring_blocks, R->d_K, R->d_J, Tin, R->d_M, R->d_R12, R->d_Y,
                         ctrl, R->d_cl, s);
        record_end(x, a, 4, 0.0, 0.0);
        record_begin(x, &a);
        launch_lccd_ladder(R->d_monos, R->d_lccd, R->n_mono, R->lccd_ladder_blocks, R->lccd_ct, R->lccd_lds_bytes,
                           R->d_W, R->d_Q, Tin, R->d_R12, R->d_Y, R->d_L, ctrl, R->d_cl, s);
        record_end(x, a, 5, R->lccd_w_flops, R->lccd_w_bytes);
    };
    std::vector<int32_t> iso_sweeps(R->n_cl, 0);
    int iso_max = 0;
    if (R->lccd) {
        // step 5: every monomer's LCCD without its environment (no pair phase, G stays zero),
        // same stopping rule; E_LCCD(X) is kept as the reference of Eq. 56
        launch_monomer(kMonoInit, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, nullptr, nullptr, R->d_T, R->d_M,
                       R->d_em2, R->d_em2_0, R->d_res, nullptr, nullptr, s);
        const int every5 = o->check_every > 0 ? o->check_every : 1;
        int issued = 0;
        while (issued < o->max_sweeps) {
            const int batch = std::min(every5, o->max_sweeps - issued);
            for (int k = 0; k < batch; ++k) {
                lccd_terms(x.d_ctrl);
                launch_monomer(kMonoUpdate, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, R->d_G[0], R->d_G[1],
                               R->d_T, R->d_M, R->d_em2, R->d_em2_0, R->d_res, x.d_ctrl, R->d_cl, s, R->d_L);
                launch_reduce_sweep(R->n_cl, R->d_cl_mono, R->d_res, R->d_cl, R->d_hist, x.d_ctrl, s);
                ++issued;
            }
            if ((st = sync_ctrl(x)) != MCPT_OK) return st;
            if (h.done) break;
        }
        std::vector<ClState> cs(R->n_cl);
        HIP_TRY(hipMemcpyAsync(cs.data(), R->d_cl, R->n_cl * sizeof(ClState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(R->d_elccd, R->d_em2, R->n_mono * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int q = 0; q < R->n_cl; ++q) {
            iso_sweeps[q] = cs[q].sweeps;
            if (cs[q].status == MCPT_ERR_DIVERGED) {
                if (x.timing.on) drain_timing(x.timing);
                return fail(MCPT_ERR_DIVERGED, "isolated-monomer LCCD (step 5) of cluster " + std::to_string(q) +
                                                   " diverged after " + std::to_string(cs[q].sweeps) + " sweeps");
            }
        }
        iso_max = h.sweeps;
        if ((st = reset_state()) != MCPT_OK) return st;
    }
    // BF16 sweeps accumulate G in FP32 (its rounding is far below the BF16 products');
    // deterministic mode keeps the FP64 partial-block path
    const bool g32 = prec == MCPT_BF16 && !R->det_on && R->d_G32[0];
    if (g32) launch_fill(reinterpret_cast<double*>(R->d_G32[0]), R->mat_elems, 0.0, s);   // both FP32 buffers
    if (o->warm_t) {
        HIP_TRY(hipMemcpyAsync(R->d_raw, o->warm_t, R->raw_elems * sizeof(double), hipMemcpyHostToDevice, s));
        launch_fill(R->d_T, R->mat_elems, 0.0, s);
        launch_pack(R->d_monos, R->n_mono, R->d_raw, R->d_T, R->max_n, s);
        launch_monomer(kMonoE0, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, nullptr, nullptr, R->d_T, R->d_M,
                       R->d_em2, R->d_em2_0, R->d_res, nullptr, nullptr, s);
        launch_monomer(kMonoFromT, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, nullptr, nullptr, R->d_T,
                       R->d_M, R->d_em2, R->d_em2_0, R->d_res, nullptr, nullptr, s);
    } else {
        launch_monomer(kMonoInit, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, nullptr, nullptr, R->d_T, R->d_M,
                       R->d_em2, R->d_em2_0, R->d_res, nullptr, nullptr, s);
    }
    if (prec != MCPT_FP64) mixed_mono(c, x, R, kMonoFromT, nullptr, nullptr, true, nullptr);   // M in low precision
    HIP_TRY(hipGetLastError());
    const double fl_sweep = pair_flops(*R, true), fl_final = pair_flops(*R, false);
    const double vb = (double)R->v_elems * sizeof(double);
    const int every = o->check_every > 0 ? o->check_every : 1;
    int cur = 0, cur32 = 0, n_lo = 0, n_hi = 0;
    // one reduced-precision sweep: pair products into G (FP64 or FP32 buffer of the current
    // parity), then the monomer pass that reads it and clears the other buffer of the pair
    auto lo_pair = [&](int source) {
        if (g32) lowp_phase(c, x, R, nullptr, R->d_G32[cur32], source);
        else lowp_phase(c, x, R, R->d_G[cur], nullptr, source);
    };
    const double* corr_src = nullptr;   // amplitudes of the current correction (R, then delta)
    auto lo_mono = [&](int mode, const Ctrl* ctrl) {
        if (R->lccd && mode == kMonoUpdate) lccd_terms(ctrl);
        if (R->lccd && mode == kMonoCorr) lccd_terms(ctrl, corr_src);
        if (g32) {
            mixed_mono(c, x, R, mode, nullptr, nullptr, true, ctrl, R->d_G32[cur32], R->d_G32[cur32 ^ 1]);
            cur32 ^= 1;
        } else {
            mixed_mono(c, x, R, mode, R->d_G[cur], R->d_G[cur ^ 1], true, ctrl);
            cur ^= 1;
        }
    };
    const bool timing_on = x.timing.on && !o->graph;
    const int inner = o->inner_sweeps > 0 ? o->inner_sweeps : (prec == MCPT_BF16 ? 4 : 6);   // measured best at 1000 monomers
    const int n_pre = std::min(inner + 1, o->max_sweeps);
    const bool saved_timing = x.timing.on;
    x.timing.on = timing_on;

    if (prec == MCPT_FP64 || !o->polish) {
        // plain Jacobi sweeps: FP64, or reduced precision with the integral source terms
        auto issue_sweep = [&]() {
            if (prec == MCPT_FP64) {
                pair_phase(c, x, R, R->d_G[cur], 1, x.d_ctrl);
                if (R->lccd) lccd_terms(x.d_ctrl);
                launch_monomer(kMonoUpdate, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, R->d_G[cur], R->d_G[cur ^ 1],
                               R->d_T, R->d_M, R->d_em2, R->d_em2_0, R->d_res, x.d_ctrl, R->d_cl, s,
                               R->lccd ? R->d_L : nullptr);
                cur ^= 1;
            } else {
                lo_pair(1);
                lo_mono(kMonoUpdate, x.d_ctrl);
            }
            launch_reduce_sweep(R->n_cl, R->d_cl_mono, R->d_res, R->d_cl, R->d_hist, x.d_ctrl, s);
        };
        int issued = 0;
        if (o->graph && o->max_sweeps > 0) {
            // an even number of sweeps per graph keeps the G double-buffer parity of every replay
            const int gk = (every % 2) ? 2 * every : every;
            const std::array<int64_t, 6> key{(int64_t)(uintptr_t)x.d_scratch, (int64_t)(uintptr_t)x.d_scratch_lo,
                                             (int64_t)(uintptr_t)x.d_ctrl, x.scratch_slot,
                                             (int64_t)c->grid_lds * 1000000 + c->grid_glb,
                                             ((int64_t)x.grid_lo * 10000 + x.grid_lo_lds) * 1000 + R->lo_variant};
            const int gprec = prec + (R->det_on ? 8 : 0) + (R->lccd ? 32 : 0);
            if (!R->graph || R->graph_prec != gprec || R->graph_sweeps != gk || R->graph_key != key) {
                drop_graph(R);
                hipGraph_t g = nullptr;
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < gk; ++k) issue_sweep();
                const hipError_t ec = hipStreamEndCapture(s, &g);
                if (ec != hipSuccess) return fail(MCPT_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
                const hipError_t ei = hipGraphInstantiate(&R->graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ei != hipSuccess) {
                    R->graph = nullptr;
                    return fail(MCPT_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
                }
                R->graph_prec = gprec;
                R->graph_sweeps = gk;
                R->graph_key = key;
            }
            cur = cur32 = 0;
            while (issued < o->max_sweeps) {
                HIP_TRY(hipGraphLaunch(R->graph, s));
                issued += gk;
                if ((st = sync_ctrl(x)) != MCPT_OK) return st;
                if (h.done) break;
            }
        }
        while (!o->graph && issued < o->max_sweeps) {
            const int batch = std::min(every, o->max_sweeps - issued);
            for (int k = 0; k < batch; ++k) {
                hipEvent_t a = nullptr;
                record_begin(x, &a);
                if (prec == MCPT_FP64) {
                    pair_phase(c, x, R, R->d_G[cur], 1, x.d_ctrl);
                    record_end(x, a, 0, fl_sweep, vb);
                    if (R->lccd) lccd_terms(x.d_ctrl);
                } else {
                    lo_pair(1);
                    record_end(x, a, 2, fl_sweep, R->lo_v_bytes);
                }
                record_begin(x, &a);
                if (prec == MCPT_FP64) {
                    launch_monomer(kMonoUpdate, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, R->d_G[cur],
                                   R->d_G[cur ^ 1], R->d_T, R->d_M, R->d_em2, R->d_em2_0, R->d_res, x.d_ctrl,
                                   R->d_cl, s, R->lccd ? R->d_L : nullptr);
                    cur ^= 1;
                } else {
                    lo_mono(kMonoUpdate, x.d_ctrl);
                }
                record_end(x, a, 1, 0.0, 0.0);
                launch_reduce_sweep(R->n_cl, R->d_cl_mono, R->d_res, R->d_cl, R->d_hist, x.d_ctrl, s);
                ++issued;
            }
            if ((st = sync_ctrl(x)) != MCPT_OK) return st;
            if (h.done) break;
        }
        if (prec == MCPT_FP64) n_hi = h.sweeps;
        else n_lo = h.sweeps;
    } else {
        // FP64 defect correction: each FP64 sweep gives r = F(T) - T and the convergence test;
        // `inner` reduced-precision sweeps solve delta = r + L(delta); then T += delta.
        auto fp64_sweep = [&]() {
            hipEvent_t a = nullptr;
            record_begin(x, &a);
            pair_phase(c, x, R, R->d_G[cur], 1, x.d_ctrl);
            record_end(x, a, 0, fl_sweep, vb);
            if (R->lccd) lccd_terms(x.d_ctrl);
            mixed_mono(c, x, R, kMonoUpdateR, R->d_G[cur], R->d_G[cur ^ 1], false, x.d_ctrl);
            launch_reduce_sweep(R->n_cl, R->d_cl_mono, R->d_res, R->d_cl, R->d_hist, x.d_ctrl, s);
            cur ^= 1;
        };
        auto correction = [&]() {
            mixed_mono(c, x, R, kMonoRlo, nullptr, nullptr, true, nullptr);
            for (int k = 0; k < inner; ++k) {
                hipEvent_t a = nullptr;
                record_begin(x, &a);
                lo_pair(0);
                record_end(x, a, 2, fl_sweep, R->lo_v_bytes);
                corr_src = k == 0 ? R->d_R : R->d_Dl;   // delta_0 = R, then the last correction
                lo_mono(kMonoCorr, nullptr);
            }
            mixed_mono(c, x, R, kMonoApply, nullptr, nullptr, false, nullptr);
            mixed_mono(c, x, R, kMonoFromT, nullptr, nullptr, false, nullptr);
        };
        for (int k = 0; k < n_pre; ++k) {   // a few plain reduced-precision sweeps first
            hipEvent_t a = nullptr;
            record_begin(x, &a);
            lo_pair(1);
            record_end(x, a, 2, fl_sweep, R->lo_v_bytes);
            lo_mono(kMonoUpdate, nullptr);
        }
        fp64_sweep();
        if ((st = sync_ctrl(x)) != MCPT_OK) return st;
        if (o->graph && !h.done) {
            // one body = correction + FP64 sweep; bodies per graph chosen so that a replay
            // returns the G double buffers to the parities they started from
            int gb = every;
            if (g32 ? gb % 2 : (gb * (inner + 1)) % 2) gb *= 2;
            const std::array<int64_t, 6> key{(int64_t)(uintptr_t)x.d_scratch, (int64_t)(uintptr_t)x.d_scratch_lo,
                                             (int64_t)(uintptr_t)x.d_ctrl, x.scratch_slot,
                                             (int64_t)c->grid_lds * 1000000 + c->grid_glb,
                                             (((int64_t)x.grid_lo * 10000 + x.grid_lo_lds) * 1000 + R->lo_variant) * 1000 +
                                                 inner};
            const int gprec = 16 + prec + (R->det_on ? 8 : 0) + (R->lccd ? 32 : 0);
            const int parity = cur + 2 * cur32;
            if (!R->graph || R->graph_prec != gprec || R->graph_sweeps != gb || R->graph_key != key ||
                R->graph_parity != parity) {
                drop_graph(R);
                const int cur0 = cur, cur32_0 = cur32;
                hipGraph_t g = nullptr;
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < gb; ++k) {
                    correction();
                    fp64_sweep();
                }
                const hipError_t ec = hipStreamEndCapture(s, &g);
                if (ec != hipSuccess) return fail(MCPT_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
                const hipError_t ei = hipGraphInstantiate(&R->graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ei != hipSuccess) {
                    R->graph = nullptr;
                    return fail(MCPT_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
                }
                R->graph_prec = gprec;
                R->graph_sweeps = gb;
                R->graph_key = key;
                R->graph_parity = parity;
                cur = cur0;
                cur32 = cur32_0;
            }
            while (!h.done) {
                HIP_TRY(hipGraphLaunch(R->graph, s));
                if ((st = sync_ctrl(x)) != MCPT_OK) return st;
            }
        }
        while (!h.done) {
            correction();
            fp64_sweep();
            if ((st = sync_ctrl(x)) != MCPT_OK) return st;
        }
        n_hi = h.sweeps;
        n_lo = n_pre + inner * (n_hi - 1);
    }
    if (h.status == MCPT_ERR_DIVERGED && R->n_cl == 1) {
        if (x.timing.on) drain_timing(x.timing);
        x.timing.on = saved_timing;
        mcpt_summary sm{};
        sm.residual = h.residual;
        sm.sweeps = n_lo + n_hi;
        sm.polish_sweeps = (prec != MCPT_FP64 && o->polish) ? n_hi : 0;
        sm.status = MCPT_ERR_DIVERGED;
        sm.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        R->last = sm;
        if (out) *out = sm;
        return fail(MCPT_ERR_DIVERGED, "iteration diverged after " + std::to_string(sm.sweeps) + " sweeps");
    }
    // energies of the returned amplitudes: FP64 Tau recomputed from the final T
    {
        hipEvent_t a = nullptr;
        record_begin(x, &a);
        pair_phase(c, x, R, R->d_G[cur], 0, nullptr);
        record_end(x, a, 0, fl_final, vb);
    }
    if (R->lccd)   // the reference of Eq. 56 is the isolated-monomer LCCD energy of step 5
        HIP_TRY(hipMemcpyAsync(R->d_em2_0, R->d_elccd, R->n_mono * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_reduce_final(R->n_cl, R->d_cl_mono, R->d_cl_pair, R->d_em2, R->d_em2_0, R->d_ed2, R->d_cl, x.d_ctrl, s);
    if ((st = sync_ctrl(x)) != MCPT_OK) return st;
    if (x.timing.on) drain_timing(x.timing);
    x.timing.on = saved_timing;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    {
        std::vector<ClState> cs(R->n_cl);
        HIP_TRY(hipMemcpy(cs.data(), R->d_cl, R->n_cl * sizeof(ClState), hipMemcpyDeviceToHost));
        for (int q = 0; q < R->n_cl; ++q) {
            mcpt_summary& cq = R->cl_last[q];
            cq = mcpt_summary{};
            cq.e_mono = cs[q].e_mono;
            cq.e_dimer = cs[q].e_dimer;
            cq.e_total = cs[q].e_mono + cs[q].e_dimer;
            cq.e_mono0 = cs[q].e_mono0;
            cq.residual = cs[q].residual;
            cq.sweeps = cs[q].sweeps;
            cq.iso_sweeps = iso_sweeps[q];
            cq.seconds = secs;
            if (cs[q].status == MCPT_ERR_NONFINITE) cq.status = MCPT_ERR_NONFINITE;
            else if (h.fixed) cq.status = cs[q].status == MCPT_ERR_DIVERGED ? MCPT_ERR_DIVERGED : MCPT_OK;
            else if (cs[q].status == MCPT_ERR_DIVERGED) cq.status = MCPT_ERR_DIVERGED;
            else if (cs[q].sweeps > 0 && cs[q].residual < o->tol) cq.status = MCPT_OK;
            else cq.status = MCPT_ERR_NOT_CONVERGED;
            if (prec != MCPT_FP64 && o->polish) {   // reduced-precision sweeps are shared by the batch
                cq.polish_sweeps = cs[q].sweeps;
                cq.sweeps = n_pre + inner * std::max(cs[q].sweeps - 1, 0) + cs[q].sweeps;
            } else if (prec != MCPT_FP64) {
                cq.sweeps = cs[q].sweeps;
            }
        }
    }
    mcpt_summary sm{};
    sm.e_mono = h.e_mono;
    sm.e_dimer = h.e_dimer;
    sm.e_total = h.e_mono + h.e_dimer;
    sm.e_mono0 = h.e_mono0;
    sm.residual = h.residual;
    sm.sweeps = n_lo + n_hi;
    sm.polish_sweeps = (prec != MCPT_FP64 && o->polish) ? n_hi : 0;
    sm.iso_sweeps = iso_max;
    sm.status = MCPT_OK;
    for (int q = 0; q < R->n_cl; ++q)
        if (R->cl_last[q].status == MCPT_ERR_DIVERGED || (R->cl_last[q].status != MCPT_OK && sm.status == MCPT_OK))
            sm.status = R->cl_last[q].status;
    sm.seconds = secs;
    R->has_result = true;
    R->last = sm;
    if (out) *out = sm;
    if (sm.status != MCPT_OK)
        return fail((mcpt_status)sm.status, "not converged after " + std::to_string(sm.sweeps) + " sweeps");
    clear_error();
    return MCPT_OK;
}

// ---- served FP64 batches with admission at sweep ticks ----

mcpt_status join_init(mcpt_ctx* c, Exec& x, Resident* R) {
    mcpt_status st;
    if ((st = ensure_device(c)) != MCPT_OK) return st;
    hipStream_t s = x.stream;   // no Tau scratch needed here: join_sweeps sizes the sweeping stream's
    std::vector<ClState> cs(R->n_cl, ClState{});
    for (int q = 0; q < R->n_cl; ++q)
        if (!R->cl_bad.empty() && R->cl_bad[q]) {   // never swept; reported as non-finite input
            cs[q].done = 1;
            cs[q].status = MCPT_ERR_NONFINITE;
        }
    HIP_TRY(hipMemcpyAsync(R->d_cl, cs.data(), R->n_cl * sizeof(ClState), hipMemcpyHostToDevice, s));
    launch_monomer(kMonoInit, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, nullptr, nullptr, R->d_T, R->d_M,
                   R->d_em2, R->d_em2_0, R->d_res, nullptr, nullptr, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    R->g_cur = 0;   // upload left both G buffers zero
    R->has_result = false;
    return MCPT_OK;
}

mcpt_status join_sweeps(mcpt_ctx* c, Exec& x, Resident* R, const mcpt_options* o, std::vector<ClState>* cs) {
    mcpt_status st;
    if ((st = ensure_scratch(c, x, R->max_slot)) != MCPT_OK) return st;
    hipStream_t s = x.stream;
    Ctrl& h = *x.h_ctrl;   // the stream is idle: the last tick synchronised it
    std::memset(&h, 0, sizeof(Ctrl));
    h.fixed = o->tol == 0.0;
    h.max_sweeps = o->max_sweeps;
    h.tol = o->tol;
    HIP_TRY(hipMemcpyAsync(x.d_ctrl, &h, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    const int every = o->check_every > 0 ? o->check_every : 1;
    for (int k = 0; k < every; ++k) {
        int& cur = R->g_cur;
        pair_phase(c, x, R, R->d_G[cur], 1, x.d_ctrl);
        launch_monomer(kMonoUpdate, R->d_monos, R->n_mono, R->max_v, R->d_dif, R->d_K, R->d_G[cur], R->d_G[cur ^ 1],
                       R->d_T, R->d_M, R->d_em2, R->d_em2_0, R->d_res, x.d_ctrl, R->d_cl, s);
        cur ^= 1;
        launch_reduce_sweep(R->n_cl, R->d_cl_mono, R->d_res, R->d_cl, R->d_hist, x.d_ctrl, s);
    }
    if ((st = sync_ctrl(x)) != MCPT_OK) return st;
    cs->assign(R->n_cl, ClState{});
    HIP_TRY(hipMemcpyAsync(cs->data(), R->d_cl, R->n_cl * sizeof(ClState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MCPT_OK;
}

mcpt_status join_finish(mcpt_ctx* c, Exec& x, Resident* R, const std::vector<int>& qs, const mcpt_options* o,
                        std::vector<char>* has, std::vector<mcpt_summary>* sums) {
    mcpt_status st;
    hipStream_t s = x.stream;
    has->assign(qs.size(), 0);
    sums->assign(qs.size(), mcpt_summary{});
    std::vector<ClState> cs(R->n_cl);
    HIP_TRY(hipMemcpyAsync(cs.data(), R->d_cl, R->n_cl * sizeof(ClState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // results exist for converged clusters and for those out of sweeps, as in a solve
    std::vector<char> keep(R->n_cl, 0);
    bool any = false;
    for (int q : qs)
        if (cs[q].status != MCPT_ERR_DIVERGED && cs[q].status != MCPT_ERR_NONFINITE) keep[q] = any = true;
    if (any) {
        // energies of the finished clusters' final amplitudes: the energy pass over their pairs only
        // (a selection that marks every other cluster done), then the per-cluster sums
        if (!R->d_cl_sel && (st = dev_alloc(c, R, &R->d_cl_sel, R->n_cl)) != MCPT_OK) return st;
        std::vector<ClState> sel(R->n_cl, ClState{});
        for (int q = 0; q < R->n_cl; ++q) sel[q].done = keep[q] ? 0 : 1;
        HIP_TRY(hipMemcpyAsync(R->d_cl_sel, sel.data(), R->n_cl * sizeof(ClState), hipMemcpyHostToDevice, s));
        pair_phase(c, x, R, R->d_G[R->g_cur], 0, nullptr, R->d_cl_sel);
        launch_reduce_final(R->n_cl, R->d_cl_mono, R->d_cl_pair, R->d_em2, R->d_em2_0, R->d_ed2, R->d_cl, x.d_ctrl, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(cs.data(), R->d_cl, R->n_cl * sizeof(ClState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        R->has_result = true;   // the finished clusters' results can be read (slice_results)
    }
    for (size_t i = 0; i < qs.size(); ++i) {
        const int q = qs[i];
        mcpt_summary& sm = (*sums)[i];
        sm.residual = cs[q].residual;
        sm.sweeps = cs[q].sweeps;
        if (cs[q].status == MCPT_ERR_NONFINITE) sm.status = MCPT_ERR_NONFINITE;
        else if (cs[q].status == MCPT_ERR_DIVERGED) sm.status = MCPT_ERR_DIVERGED;
        else if (o->tol == 0.0 || (cs[q].sweeps > 0 && cs[q].residual < o->tol)) sm.status = MCPT_OK;
        else sm.status = MCPT_ERR_NOT_CONVERGED;
        if (!keep[q]) continue;
        (*has)[i] = 1;
        sm.e_mono = cs[q].e_mono;
        sm.e_dimer = cs[q].e_dimer;
        sm.e_total = cs[q].e_mono + cs[q].e_dimer;
        sm.e_mono0 = cs[q].e_mono0;
    }
    return MCPT_OK;
}

mcpt_status join_concat(mcpt_ctx* c, Exec& x, const std::vector<std::pair<Resident*, int>>& parts, uint64_t* id_out) {
    if (parts.empty()) return fail(MCPT_ERR_INVALID, "nothing to join");
    mcpt_status st;
    auto m = std::make_unique<Resident>();
    Resident* M = m.get();
    const int n_cl = (int)parts.size();
    M->n_cl = n_cl;
    M->cl_mono.assign(n_cl + 1, 0);
    M->cl_pair.assign(n_cl + 1, 0);
    M->cl_v.assign(n_cl + 1, 0);
    M->cl_bad.assign(n_cl, 0);
    // the element ranges of cluster q of R in each array (clusters are contiguous, in order)
    struct Span {
        int64_t m0, m1, p0, p1, v0, v1, mat0, mat1, dif0, dif1, raw0, raw1, eps0, eps1;
    };
    auto span_of = [](const Resident* R, int q) {
        Span r{};
        r.m0 = R->cl_mono[q];
        r.m1 = R->cl_mono[q + 1];
        r.p0 = R->cl_pair[q];
        r.p1 = R->cl_pair[q + 1];
        r.v0 = R->cl_v[q];
        r.v1 = R->cl_v[q + 1];
        const bool last = r.m1 >= R->n_mono;
        const MonoDesc& a = R->monos[r.m0];
        r.mat0 = a.mat_off;
        r.dif0 = a.dif_off;
        r.raw0 = a.raw_off;
        r.eps0 = a.eps_off;
        r.mat1 = last ? R->mat_elems : R->monos[r.m1].mat_off;
        r.dif1 = last ? R->dif_elems : R->monos[r.m1].dif_off;
        r.raw1 = last ? R->raw_elems : R->monos[r.m1].raw_off;
        r.eps1 = last ? R->eps_elems : R->monos[r.m1].eps_off;
        return r;
    };
    std::vector<Span> sp(n_cl);
    std::vector<Span> dst(n_cl);
    int64_t mat = 0, dif = 0, raw = 0, eps = 0;
    for (int k = 0; k < n_cl; ++k) {
        const Resident* R = parts[k].first;
        const int q = parts[k].second;
        const Span a = sp[k] = span_of(R, q);
        Span& b = dst[k];
        b.m0 = M->cl_mono[k];
        b.p0 = M->cl_pair[k];
        b.v0 = M->cl_v[k];
        b.mat0 = mat;
        b.dif0 = dif;
        b.raw0 = raw;
        b.eps0 = eps;
        for (int64_t i = a.m0; i < a.m1; ++i) {
            MonoDesc d = R->monos[i];
            d.mat_off += b.mat0 - a.mat0;
            d.dif_off += b.dif0 - a.dif0;
            d.raw_off += b.raw0 - a.raw0;
            d.eps_off += b.eps0 - a.eps0;
            d.cluster = k;
            M->monos.push_back(d);
            M->max_n = std::max(M->max_n, d.n);
            M->max_v = std::max(M->max_v, d.v);
            M->max_np = std::max(M->max_np, d.np);
        }
        for (const PairDesc& pd : R->pairs) {
            if (pd.cluster != q) continue;
            PairDesc e = pd;
            e.x = (int)(e.x + b.m0 - a.m0);
            e.y = (int)(e.y + b.m0 - a.m0);
            e.v_off += b.v0 - a.v0;
            e.orig += b.p0 - a.p0;
            e.cluster = k;
            M->pairs.push_back(e);
        }
        M->cl_mono[k + 1] = b.m0 + (a.m1 - a.m0);
        M->cl_pair[k + 1] = b.p0 + (a.p1 - a.p0);
        M->cl_v[k + 1] = b.v0 + (a.v1 - a.v0);
        mat += a.mat1 - a.mat0;
        dif += a.dif1 - a.dif0;
        raw += a.raw1 - a.raw0;
        eps += a.eps1 - a.eps0;
        if (!R->cl_bad.empty()) M->cl_bad[k] = R->cl_bad[q];
    }
    if (M->cl_mono[n_cl] > INT32_MAX) return fail(MCPT_ERR_INVALID, "too many monomers");
    M->n_mono = (int)M->cl_mono[n_cl];
    M->n_pair = M->cl_pair[n_cl];
    M->v_elems = M->cl_v[n_cl];
    M->mat_elems = mat;
    M->dif_elems = dif;
    M->raw_elems = raw;
    M->eps_elems = eps;
    for (const PairDesc& d : M->pairs)
        M->max_slot = std::max<int64_t>(M->max_slot, (int64_t)M->monos[d.x].np * M->monos[d.y].np);
    order_pairs(M);
#define ALLOC(ptr, n)                                          \
    do {                                                       \
        if ((st = dev_alloc(c, M, &(ptr), (n))) != MCPT_OK) { \
            free_resident(c, M);                               \
            return st;                                         \
        }                                                      \
    } while (0)
    ALLOC(M->d_monos, M->n_mono);
    ALLOC(M->d_pairs, std::max<int64_t>(M->n_pair, 1));
    ALLOC(M->d_dif, M->dif_elems);
    ALLOC(M->d_raw, M->raw_elems);
    ALLOC(M->d_K, M->mat_elems);
    ALLOC(M->d_T, M->mat_elems);
    ALLOC(M->d_M, M->mat_elems);
    ALLOC(M->d_G[0], M->mat_elems);
    ALLOC(M->d_G[1], M->mat_elems);
    ALLOC(M->d_V, std::max<int64_t>(M->v_elems, 1));
    ALLOC(M->d_em2, M->n_mono);
    ALLOC(M->d_em2_0, M->n_mono);
    ALLOC(M->d_res, M->n_mono);
    ALLOC(M->d_ed2, std::max<int64_t>(M->n_pair, 1));
    ALLOC(M->d_cl, n_cl);
    ALLOC(M->d_hist, (int64_t)n_cl * kMaxSweeps);
    ALLOC(M->d_cl_mono, n_cl + 1);
    ALLOC(M->d_cl_pair, n_cl + 1);
#undef ALLOC
    hipStream_t s = x.stream;
    struct Copy {
        void* dst;
        const void* src;
        size_t bytes;
    };
    std::vector<Copy> copies;   // device to device
    auto dd = [&](void* d, const void* src, int64_t bytes) {
        if (bytes > 0) copies.push_back({d, src, (size_t)bytes});
    };
    for (int k = 0; k < n_cl; ++k) {
        const Resident* R = parts[k].first;
        const int q = parts[k].second;
        const Span& a = sp[k];
        const Span& b = dst[k];
        const int64_t D = sizeof(double);
        dd(M->d_dif + b.dif0, R->d_dif + a.dif0, (a.dif1 - a.dif0) * D);
        dd(M->d_K + b.mat0, R->d_K + a.mat0, (a.mat1 - a.mat0) * D);
        dd(M->d_T + b.mat0, R->d_T + a.mat0, (a.mat1 - a.mat0) * D);
        dd(M->d_M + b.mat0, R->d_M + a.mat0, (a.mat1 - a.mat0) * D);
        dd(M->d_V + b.v0, R->d_V + a.v0, (a.v1 - a.v0) * D);
        dd(M->d_em2 + b.m0, R->d_em2 + a.m0, (a.m1 - a.m0) * D);
        dd(M->d_em2_0 + b.m0, R->d_em2_0 + a.m0, (a.m1 - a.m0) * D);
        dd(M->d_res + b.m0, R->d_res + a.m0, (a.m1 - a.m0) * D);
        dd(M->d_ed2 + b.p0, R->d_ed2 + a.p0, (a.p1 - a.p0) * D);
        dd(M->d_cl + k, R->d_cl + q, (int64_t)sizeof(ClState));
        dd(M->d_hist + (int64_t)k * kMaxSweeps, R->d_hist + (int64_t)q * kMaxSweeps, kMaxSweeps * D);
    }
    hipError_t e = hipSuccess;
    for (const Copy& cp : copies) {
        e = hipMemcpyAsync(cp.dst, cp.src, cp.bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(M->d_monos, M->monos.data(), M->monos.size() * sizeof(MonoDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && M->n_pair)
        e = hipMemcpyAsync(M->d_pairs, M->pairs.data(), M->pairs.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(M->d_cl_mono, M->cl_mono.data(), (n_cl + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(M->d_cl_pair, M->cl_pair.data(), (n_cl + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        // both G buffers zero: the next sweep accumulates into one and its update clears the other
        launch_fill(M->d_G[0], M->mat_elems, 0.0, s);
        launch_fill(M->d_G[1], M->mat_elems, 0.0, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_resident(c, M);
        return fail(MCPT_ERR_DEVICE, std::string("joining batches: ") + hipGetErrorString(e));
    }
    M->g_cur = 0;
    M->internal = true;
    M->cl_last.assign(n_cl, mcpt_summary{});
    std::lock_guard<std::mutex> g(c->mu);
    M->id = c->next_id++;
    *id_out = M->id;
    c->res[M->id] = std::move(m);
    return MCPT_OK;
}

}  // namespace mcpt

using namespace mcpt;

// Tau scratch of mcpt_run_static, for callers that cannot allocate device memory:
// one slot of the largest pair's padded npX x npY Tau per persistent workgroup of
// the FP64 pair kernels.  Each GPU the library runs on holds its own copy for the
// life of the process.  In host code `scratch` names a host-side stand-in, never
// the device array: kernels receive the address hipGetSymbolAddress returns for
// the current device (static_scratch_of).  Every mcpt_run_static on one GPU uses
// that GPU's copy, so calls that overlap on a GPU race; the pair kernels write
// each Tau slot in full before reading it, so no clearing is needed.
static __device__ __align__(256) double scratch[MCPT_STATIC_SCRATCH_BYTES / sizeof(double)];

namespace {

std::mutex g_static_mu;
std::map<int, double*> g_static_ptr;   // device -> address of its copy of scratch (g_static_mu)

// The device address of this device's scratch array; the device must be current.
mcpt_status static_scratch_of(int device, double** out) {
    std::lock_guard<std::mutex> g(g_static_mu);
    auto it = g_static_ptr.find(device);
    if (it == g_static_ptr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MCPT_ERR_DEVICE, std::string("hipGetSymbolAddress of the static scratch: ") +
                                             hipGetErrorString(e));
        it = g_static_ptr.emplace(device, static_cast<double*>(ptr)).first;
    }
    *out = it->second;
    return MCPT_OK;
}

// A caller-visible resident problem (served batches are reached through their tickets).
Resident* find_resident(mcpt_ctx* c, uint64_t id) {
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->res.find(id);
    if (it == c->res.end() || it->second->internal) return nullptr;
    return it->second.get();
}

mcpt_status unknown(uint64_t id) { return fail(MCPT_ERR_UNKNOWN_ID, "unknown problem id " + std::to_string(id)); }

}  // namespace

extern "C" {

mcpt_status mcpt_create(int device, size_t hbm_budget_bytes, mcpt_ctx** out) {
    if (!out) return fail(MCPT_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(MCPT_ERR_INVALID, "no HIP device " + std::to_string(device));
    auto c = std::make_unique<mcpt_ctx>();
    c->device = device;
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    c->n_cu = prop.multiProcessorCount;
    c->grid_lds = std::max(8, c->n_cu * pair_fp64_blocks_per_cu(1) / 8 * 8);
    c->grid_glb = std::max(8, c->n_cu * pair_fp64_blocks_per_cu(0) / 8 * 8);
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    mcpt_status st = exec_init(c.get(), c->main);
    if (st != MCPT_OK) {
        exec_free(c.get(), c->main);
        return st;
    }
    if ((st = static_scratch_of(device, &c->static_scratch)) != MCPT_OK) {
        exec_free(c.get(), c->main);
        return st;
    }
    clear_error();
    *out = c.release();
    return MCPT_OK;
}

void mcpt_destroy(mcpt_ctx* c) {
    if (!c) return;
    serve_stop(c);
    (void)hipSetDevice(c->device);
    if (c->main.stream) (void)hipStreamSynchronize(c->main.stream);
    for (auto& kv : c->res) free_resident(c, kv.second.get());
    c->res.clear();
    exec_free(c, c->main);
    delete c;
}

const char* mcpt_last_error(void) { return last_error_text().c_str(); }

mcpt_status mcpt_set_stream(mcpt_ctx* c, void* hip_stream) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->main.stream));
    c->main.stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->main.own;
    return MCPT_OK;
}

mcpt_status mcpt_upload(mcpt_ctx* c, const mcpt_problem* prob, uint64_t* id) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    try {
        return upload_batch(c, c->main, prob, 1, false, id);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_upload_batch(mcpt_ctx* c, const mcpt_problem* probs, int32_t n, uint64_t* id) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    try {
        return upload_batch(c, c->main, probs, n, false, id);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_cluster_results(mcpt_ctx* c, uint64_t id, int32_t n, mcpt_summary* out) {
    if (!c || !out) return fail(MCPT_ERR_INVALID, "ctx or out is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    if (n != R->n_cl) return fail(MCPT_ERR_INVALID, "problem holds " + std::to_string(R->n_cl) + " clusters");
    if (!R->has_result) return fail(MCPT_ERR_INVALID, "problem has no result (not run, or diverged)");
    for (int q = 0; q < n; ++q) out[q] = R->cl_last[q];
    return MCPT_OK;
}

mcpt_status mcpt_solve_batch(mcpt_ctx* c, const mcpt_problem* probs, int32_t n, const mcpt_options* opts,
                             uint64_t* id, mcpt_summary* per_cluster) {
    mcpt_status st = validate_options(opts);
    if (st != MCPT_OK) return st;
    uint64_t local = 0;
    st = mcpt_upload_batch(c, probs, n, &local);
    if (st != MCPT_OK) return st;
    if (id) *id = local;
    st = mcpt_run(c, local, opts, nullptr);
    if (per_cluster) {
        Resident* R = find_resident(c, local);
        if (R && R->has_result)
            for (int q = 0; q < n; ++q) per_cluster[q] = R->cl_last[q];
    }
    return st;
}

mcpt_status mcpt_run(mcpt_ctx* c, uint64_t id, const mcpt_options* opts, mcpt_summary* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    try {
        return run(c, c->main, R, opts, out);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_run_static(mcpt_ctx* c, uint64_t id, const mcpt_options* opts, mcpt_summary* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    mcpt_status st = validate_options(opts);
    if (st != MCPT_OK) return st;
    if (opts->precision != MCPT_FP64 || opts->deterministic || opts->graph)
        return fail(MCPT_ERR_INVALID, "mcpt_run_static runs the FP64 eager solve only (precision FP64, "
                                      "deterministic 0, graph 0)");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    const int64_t slot_bytes = R->max_slot * (int64_t)sizeof(double);
    const int64_t slots = (int64_t)MCPT_STATIC_SCRATCH_BYTES / std::max<int64_t>(slot_bytes, 1);
    if (slots < 1)
        return fail(MCPT_ERR_INVALID, "the largest pair's Tau slot (" + std::to_string(slot_bytes) +
                                          " bytes) exceeds the static scratch of " +
                                          std::to_string((long long)MCPT_STATIC_SCRATCH_BYTES) + " bytes");
    // the context's stream and control word, with the static array as the Tau scratch
    Exec y;
    y.stream = c->main.stream;
    y.d_ctrl = c->main.d_ctrl;
    y.h_ctrl = c->main.h_ctrl;
    y.d_flag = c->main.d_flag;
    y.h_flag = c->main.h_flag;
    y.d_scratch = c->static_scratch;
    y.scratch_slot = R->max_slot;
    y.scratch_slots = (int)std::min<int64_t>(slots, std::max(c->grid_lds, c->grid_glb));
    y.fixed_scratch = true;
    y.grid_cap = y.scratch_slots;
    try {
        return run(c, y, R, opts, out);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_solve(mcpt_ctx* c, const mcpt_problem* prob, const mcpt_options* opts, uint64_t* id,
                       mcpt_summary* out) {
    mcpt_status st = validate_options(opts);
    if (st != MCPT_OK) return st;
    uint64_t local = 0;
    st = mcpt_upload(c, prob, &local);
    if (st != MCPT_OK) return st;
    if (id) *id = local;
    return mcpt_run(c, local, opts, out);
}

mcpt_status mcpt_energy(mcpt_ctx* c, uint64_t id, double* e_m2, double* de_m2, double* e_d2, double* t_amp) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    if (serve_owns(c, id)) return serve_energy(c, id, e_m2, de_m2, e_d2, t_amp);
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    return slice_results(c, c->main, R, -1, e_m2, de_m2, e_d2, t_amp);
}

mcpt_status mcpt_release(mcpt_ctx* c, uint64_t id) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    if (serve_owns(c, id)) return serve_release(c, id);
    if (!find_resident(c, id)) return unknown(id);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->main.stream);
    release_resident(c, id);
    return MCPT_OK;
}

mcpt_status mcpt_upload_scaled(mcpt_ctx* c, uint64_t base, int64_t n, const int64_t* pair, const double* scale,
                               uint64_t* id) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* B = find_resident(c, base);
    if (!B) return unknown(base);
    try {
        return clone_scaled(c, c->main, B, n, pair, scale, id);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_fd_stencil(mcpt_ctx* c, uint64_t base, int32_t n_modes, const mcpt_fd_mode* modes, int32_t n_cell,
                            const int32_t* cell, double step, const double* w, const mcpt_options* opts,
                            mcpt_fd_result* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* B = find_resident(c, base);
    if (!B) return unknown(base);
    try {
        return fd_stencil(c, c->main, B, n_modes, modes, n_cell, cell, step, w, opts, out);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_lccd_attach(mcpt_ctx* c, uint64_t id, const mcpt_lccd_integrals* ints) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    try {
        return lccd_attach(c, c->main, R, ints);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_dimer_attach(mcpt_ctx* c, uint64_t id, const mcpt_dimer_integrals* ints) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    try {
        return dimer_attach(c, c->main, R, ints);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_dimer_tau(mcpt_ctx* c, uint64_t id, double* tau) {
    if (!c || !tau) return fail(MCPT_ERR_INVALID, "ctx or tau is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    if (!R->dimer) return fail(MCPT_ERR_INVALID, "problem has no dimer-internal terms attached");
    if (!R->has_result) return fail(MCPT_ERR_INVALID, "problem has no result (not run, or diverged)");
    HIP_TRY(hipSetDevice(c->device));
    std::vector<double> h((size_t)R->dimer_tau_elems);
    if (R->dimer_tau_elems > 0)
        HIP_TRY(hipMemcpyAsync(h.data(), R->d_Tau, R->dimer_tau_elems * sizeof(double), hipMemcpyDeviceToHost,
                               c->main.stream));
    HIP_TRY(hipStreamSynchronize(c->main.stream));
    // pair p (caller order) is stored npx x npy at its tau_off, row (i,a) = i vx + a, column (j,b) = j vy + b
    int64_t out = 0;
    for (const DimerDesc& d : R->dimer_desc) {
        for (int r = 0; r < d.nx; ++r)
            std::memcpy(tau + out + (int64_t)r * d.ny, h.data() + d.tau_off + (int64_t)r * d.npy, d.ny * sizeof(double));
        out += (int64_t)d.nx * d.ny;
    }
    return MCPT_OK;
}

mcpt_status mcpt_singles(mcpt_ctx* c, uint64_t id, const double* w, int32_t memory, const mcpt_options* opts,
                         mcpt_singles_summary* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    try {
        return singles(c, c->main, R, w, memory, opts, out);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_singles_result(mcpt_ctx* c, uint64_t id, double* e_m1, double* t1) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    if (!R->has_singles) return fail(MCPT_ERR_INVALID, "problem has no singles result (not solved, or diverged)");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = c->main.stream;
    if (e_m1 && R->n_mono > 0)
        HIP_TRY(hipMemcpyAsync(e_m1, R->d_em1, R->n_mono * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<double> tp;
    if (t1 && R->dif_elems > 0) {
        tp.resize(R->dif_elems);
        HIP_TRY(hipMemcpyAsync(tp.data(), R->d_t1, R->dif_elems * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (t1) {
        int64_t k = 0;
        for (const MonoDesc& m : R->monos)
            for (int e = 0; e < m.n; ++e) t1[k++] = tp[m.dif_off + e];
    }
    return MCPT_OK;
}

mcpt_status mcpt_autotune(mcpt_ctx* c, uint64_t id, int32_t precision, mcpt_tune_result* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    if (precision != MCPT_FP32 && precision != MCPT_BF16)
        return fail(MCPT_ERR_INVALID, "tile variants exist for MCPT_FP32 and MCPT_BF16 only");
    Resident* R = find_resident(c, id);
    if (!R) return unknown(id);
    try {
        return autotune(c, c->main, R, precision, out);
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_tune_export(mcpt_ctx* c, char* buf, size_t cap, size_t* len) {
    if (!c || !len) return fail(MCPT_ERR_INVALID, "ctx or len is NULL");
    std::string text;
    {
        std::lock_guard<std::mutex> g(c->mu);
        for (const auto& kv : c->tune) {
            int sb = 0, nw = 0, pd = 0;
            lowp_variant_shape(kv.second, &sb, &nw, &pd);
            text += kv.first + " " + std::to_string(sb) + " " + std::to_string(nw) + " " + std::to_string(pd) + "\n";
        }
    }
    *len = text.size() + 1;
    if (buf && cap >= text.size() + 1) std::memcpy(buf, text.c_str(), text.size() + 1);
    else if (buf) return fail(MCPT_ERR_INVALID, "buffer too small: " + std::to_string(text.size() + 1) + " bytes");
    return MCPT_OK;
}

mcpt_status mcpt_tune_import(mcpt_ctx* c, const char* text) {
    if (!c || !text) return fail(MCPT_ERR_INVALID, "ctx or text is NULL");
    std::vector<int> shapes(3 * lowp_variants());
    for (int k = 0; k < lowp_variants(); ++k)
        lowp_variant_shape(k, &shapes[3 * k], &shapes[3 * k + 1], &shapes[3 * k + 2]);
    std::map<std::string, int> add;
    const mcpt_status st = parse_tune_table(text, shapes.data(), lowp_variants(), &add);
    if (st != MCPT_OK) return st;
    std::lock_guard<std::mutex> g(c->mu);
    for (const auto& kv : add) c->tune[kv.first] = kv.second;
    return MCPT_OK;
}

mcpt_status mcpt_set_timing(mcpt_ctx* c, int enable) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->main.stream));
    drain_timing(c->main.timing);
    c->main.timing.on = enable != 0;
    c->main.timing.tot = mcpt_timing{};
    return MCPT_OK;
}

mcpt_status mcpt_timing_read(mcpt_ctx* c, mcpt_timing* out) {
    if (!c || !out) return fail(MCPT_ERR_INVALID, "ctx or out is NULL");
    HIP_TRY(hipStreamSynchronize(c->main.stream));
    drain_timing(c->main.timing);
    *out = c->main.timing.tot;
    return MCPT_OK;
}

}  // extern "C"
