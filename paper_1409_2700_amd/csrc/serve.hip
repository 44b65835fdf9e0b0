// Serving: MCPT(2) solves submitted as independent requests (clusters of
// different sizes, displaced geometries) and run by a pool of worker streams.
//
// Scheduling.  A worker that is free takes the request at the head of the
// queue if its device footprint fits next to what is resident and reserved,
// then fuses into the same batch the later queued requests that share its
// options and size class and still fit (at most max_batch requests and
// max_batch_pairs pairs).  The batch is uploaded as one resident problem with
// one cluster per request and solved with per-cluster stopping, so each
// request's result is the one its own solve gives.  Requests that arrive while
// batches run are taken by the next free worker: the workers' streams run
// concurrently, so batches overlap on the device, and a request never waits
// for the whole queue to drain.  FP64 batches of plain sweeps work at sweep
// ticks (run_joined): at each host check their finished requests retire, and,
// in the join mode, compatible queued requests join the running clusters in one
// batch.  Results stay resident on the device until the ticket is released; the
// memory they hold counts against the admission budget.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mcpt {

PinnedPool::~PinnedPool() {
    for (auto& kv : cls_) (void)hipHostFree(kv.first);
}

void PinnedPool::set_cap(size_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    cap_ = bytes;
}

double* PinnedPool::take(size_t bytes) {
    int k = 20;                                   // blocks of 1 MiB and up
    while ((size_t(1) << k) < bytes) ++k;
    std::lock_guard<std::mutex> g(mu_);
    auto it = free_.find(k);
    if (it != free_.end() && !it->second.empty()) {
        double* p = it->second.back();
        it->second.pop_back();
        return p;
    }
    const size_t sz = size_t(1) << k;
    if (held_ + sz > cap_) return nullptr;
    void* p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess || !p) {
        (void)hipGetLastError();
        return nullptr;
    }
    held_ += sz;
    cls_[static_cast<double*>(p)] = k;
    return static_cast<double*>(p);
}

void PinnedPool::give(double* p) {
    std::lock_guard<std::mutex> g(mu_);
    free_[cls_.at(p)].push_back(p);
}

size_t PinnedPool::held() const {
    std::lock_guard<std::mutex> g(mu_);
    return held_;
}

uint64_t PinnedPool::pageable() const {
    std::lock_guard<std::mutex> g(mu_);
    return pageable_;
}

void PinnedPool::count_pageable() {
    std::lock_guard<std::mutex> g(mu_);
    ++pageable_;
}

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool head_fits(mcpt_ctx* c, Server& S) {
    if (S.queue.empty()) return false;
    const Request* h = S.reqs[S.queue.front()].get();
    return c->in_use + c->reserved + h->footprint <= c->budget;
}

// A served FP64 batch with admission at sweep ticks; request mem[q] is cluster q of the
// running batch.  At every host check the clusters that finished are reported; their results
// stay readable in the batch (its other clusters' sweeps skip them) until their tickets are
// released.  In the join mode, compatible requests at the head of the queue are uploaded on the
// worker's second stream (xu, from a helper thread) while the batch keeps sweeping, and at the
// first tick after the upload they are joined with the unfinished clusters into a new batch that
// continues each cluster's iteration where it stopped, so a request's sweeps and result are
// those of its own solve.  A batch is freed once neither a worker runs it nor a ticket holds
// results in it (Resident::refs).  Called and returns without mu; the caller's reservation
// x.reserved is kept equal to the unfinished requests' footprint (plus twice the joiners' until
// they are merged).
void run_joined(mcpt_ctx* c, Server& S, Exec& x, Exec& xu, std::vector<Request*> mem) {
    const mcpt_options o = mem.front()->opts;
    const int cls = mem.front()->size_class;
    auto report = [&](Request* r, const mcpt_summary& sm, uint64_t res, int q, const std::string& err, double t) {
        r->sum = sm;
        r->batch = res;
        r->cluster = q;
        if (sm.status != MCPT_OK) r->error = err.empty() ? "request did not converge" : err;
        r->sum.seconds = t - r->t_submit;   // latency: submission to result
        r->state = 2;
        ++S.served;
    };
    auto fail_group = [&](const std::vector<Request*>& g, mcpt_status st, const std::string& err) {
        const double t = now_s();
        std::lock_guard<std::mutex> lg(c->mu);
        for (Request* r : g) {
            mcpt_summary sm{};
            sm.status = st == MCPT_OK ? MCPT_ERR_DEVICE : st;
            report(r, sm, 0, 0, err, t);
        }
        S.done_cv.notify_all();
        S.cv.notify_all();
    };
    auto reserve = [&](size_t bytes) {   // under mu; an upload on xu leaves this worker's reservation out too
        c->reserved -= std::min(c->reserved, x.reserved);
        x.reserved = xu.reserved = bytes;
        c->reserved += bytes;
    };
    auto leave = [&](uint64_t id) {   // the worker's hold on a batch ends; freed if no ticket holds results
        bool drop = false;
        {
            std::lock_guard<std::mutex> lg(c->mu);
            drop = --c->res[id]->refs == 0;
        }
        if (drop) release_resident(c, id);
    };
    // upload a group as a new batch on stream ex and start its iteration (T = D K)
    auto start = [&](Exec& ex, std::vector<Request*>& g, uint64_t* id, std::string* err) -> mcpt_status {
        std::vector<mcpt_problem> probs;
        probs.reserve(g.size());
        for (Request* r : g) probs.push_back(r->prob);
        mcpt_status st;
        try {
            st = upload_batch(c, ex, probs.data(), (int)probs.size(), true, id);
        } catch (const std::exception& e) {
            st = fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
        }
        for (Request* r : g) {   // the device holds the inputs now (or the upload failed)
            r->k_intra.reset();
            r->v_dimer.reset();
            r->prob.k_intra = r->prob.v_dimer = nullptr;
        }
        if (st == MCPT_OK) {
            Resident* B = nullptr;
            {
                std::lock_guard<std::mutex> lg(c->mu);
                B = c->res[*id].get();
                B->refs = 1;
            }
            if ((st = join_init(c, ex, B)) != MCPT_OK) release_resident(c, *id);
        }
        if (st != MCPT_OK) *err = last_error_text();   // the error text is per thread
        return st;
    };
    // joiners on their way to the device
    struct Pending {
        std::vector<Request*> g;
        size_t bytes = 0;          // their reservation: twice their footprint
        uint64_t bid = 0;
        mcpt_status st = MCPT_OK;
        std::string err;
        std::atomic<bool> finished{false};
        std::thread th;
    };
    std::unique_ptr<Pending> pend;
    auto finish_upload = [&]() {   // wait for the helper thread; on failure the joiners fail
        pend->th.join();
        if (pend->st != MCPT_OK) {
            fail_group(pend->g, pend->st, pend->err);
            pend.reset();
        }
    };

    uint64_t rid = 0;
    std::string err0;
    mcpt_status st = start(x, mem, &rid, &err0);
    if (st != MCPT_OK) {
        fail_group(mem, st, err0);
        return;
    }
    Resident* R = nullptr;
    {
        std::lock_guard<std::mutex> lg(c->mu);
        R = c->res[rid].get();
    }
    std::vector<char> done(mem.size(), 0);
    for (;;) {
        std::vector<ClState> cs;
        st = join_sweeps(c, x, R, &o, &cs);
        std::vector<int> fin, live;
        std::vector<char> has;
        std::vector<mcpt_summary> sums;
        if (st == MCPT_OK) {
            for (size_t q = 0; q < mem.size(); ++q) {
                if (cs[q].done && !done[q]) fin.push_back((int)q);
                if (!cs[q].done) live.push_back((int)q);
            }
            if (!fin.empty()) st = join_finish(c, x, R, fin, &o, &has, &sums);
        }
        if (st != MCPT_OK) {
            const std::string err = last_error_text();
            std::vector<Request*> rest;
            for (size_t q = 0; q < mem.size(); ++q)
                if (!done[q]) rest.push_back(mem[q]);
            if (pend) {   // the joiners fail with the batch they were to join
                finish_upload();
                if (pend) {
                    leave(pend->bid);
                    rest.insert(rest.end(), pend->g.begin(), pend->g.end());
                }
            }
            fail_group(rest, st, err);
            leave(rid);
            return;
        }
        std::vector<Request*> joiners;
        {
            std::lock_guard<std::mutex> lg(c->mu);
            const double t = now_s();
            for (size_t i = 0; i < fin.size(); ++i) {
                report(mem[fin[i]], sums[i], has[i] ? rid : 0, fin[i], std::string(), t);
                if (has[i]) ++R->refs;
                done[fin[i]] = 1;
            }
            size_t fp_live = 0;
            int64_t live_pairs = 0;
            for (int q : live) {
                fp_live += mem[q]->footprint;
                live_pairs += mem[q]->prob.n_pair;
            }
            const size_t pending = pend ? pend->bytes : 0;
            reserve(fp_live + pending);
            const size_t used = c->in_use + (c->reserved - x.reserved) + fp_live + pending;
            // joins below saturation only: with more requests queued than workers, batches formed at
            // their start keep the device as busy; one group of joiners at a time
            if (S.params.tick_mode == MCPT_SERVE_JOIN_AT_TICKS && !pend && !live.empty() && !S.stop &&
                !S.queue.empty() && S.busy >= (int)S.workers.size() && S.queue.size() <= S.workers.size() &&
                used < c->budget) {
                std::vector<QueuedRequest> view;
                view.reserve(S.queue.size());
                for (uint64_t tk : S.queue) {
                    const Request* r = S.reqs[tk].get();
                    view.push_back({r->footprint, r->prob.n_pair, r->size_class, &r->opts});
                }
                const std::vector<size_t> take =
                    join_batch(view, c->budget - used, o, cls, (int)live.size(), live_pairs, fp_live,
                               S.params.max_batch, S.params.max_batch_pairs);
                size_t add = 0;
                for (size_t i : take) {
                    Request* r = S.reqs[S.queue[i]].get();
                    r->state = 1;
                    joiners.push_back(r);
                    add += 2 * r->footprint;
                }
                for (size_t k = take.size(); k-- > 0;) S.queue.erase(S.queue.begin() + (std::ptrdiff_t)take[k]);
                if (!joiners.empty()) {
                    reserve(fp_live + add);
                    S.joined += joiners.size();
                }
            }
            if (!fin.empty()) {
                S.done_cv.notify_all();
                S.cv.notify_all();
            }
        }
        if (!joiners.empty()) {   // upload them while the batch goes on sweeping
            pend = std::make_unique<Pending>();
            pend->g = joiners;
            for (Request* r : joiners) pend->bytes += 2 * r->footprint;
            Pending* pp = pend.get();
            pp->th = std::thread([&start, &xu, pp] {
                pp->st = start(xu, pp->g, &pp->bid, &pp->err);
                pp->finished.store(true, std::memory_order_release);
            });
        }
        // merge a finished upload (or wait for it when nothing else is left to sweep)
        bool ready = false;
        if (pend && (live.empty() || pend->finished.load(std::memory_order_acquire))) {
            finish_upload();
            ready = pend != nullptr;
        }
        if (ready) {
            const uint64_t bid = pend->bid;
            std::vector<Request*> jg = pend->g;
            pend.reset();
            bool replaced = false;
            if (live.empty()) {   // nothing to carry over: the joiners' batch runs as it is
                leave(rid);
                rid = bid;
                mem = jg;
                replaced = true;
            } else {
                Resident* B = nullptr;
                {
                    std::lock_guard<std::mutex> lg(c->mu);
                    B = c->res[bid].get();
                }
                std::vector<std::pair<Resident*, int>> parts;
                for (int q : live) parts.push_back({R, q});
                for (int k = 0; k < (int)jg.size(); ++k) parts.push_back({B, k});
                uint64_t mid = 0;
                st = join_concat(c, x, parts, &mid);
                if (st != MCPT_OK) {
                    fail_group(jg, st, last_error_text());
                } else {
                    {
                        std::lock_guard<std::mutex> lg(c->mu);
                        c->res[mid]->refs = 1;
                    }
                    leave(rid);
                    rid = mid;
                    std::vector<Request*> next;
                    for (int q : live) next.push_back(mem[q]);
                    next.insert(next.end(), jg.begin(), jg.end());
                    mem = next;
                    replaced = true;
                }
                leave(bid);
            }
            if (replaced) done.assign(mem.size(), 0);
            std::lock_guard<std::mutex> lg(c->mu);
            R = c->res[rid].get();
            size_t fp = 0;
            for (size_t q = 0; q < mem.size(); ++q)
                if (!done[q]) fp += mem[q]->footprint;
            reserve(fp);
            continue;
        }
        if (live.empty() && !pend) {
            leave(rid);
            return;
        }
    }
}

void worker_loop(mcpt_ctx* c, int w) {
    Server& S = *c->server;
    Exec& x = *S.execs[w];
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        S.cv.wait(lk, [&] { return S.stop || head_fits(c, S); });
        if (S.stop) break;
        // ---- form a batch: the head, then compatible queued requests that fit ----
        std::vector<QueuedRequest> view;
        view.reserve(S.queue.size());
        for (uint64_t t : S.queue) {
            const Request* r = S.reqs[t].get();
            view.push_back({r->footprint, r->prob.n_pair, r->size_class, &r->opts});
        }
        const std::vector<size_t> take =
            form_batch(view, c->budget - c->in_use - c->reserved, S.params.max_batch, S.params.max_batch_pairs);
        std::vector<Request*> group;
        size_t reserve = 0;
        for (size_t i : take) {
            Request* r = S.reqs[S.queue[i]].get();
            group.push_back(r);
            reserve += r->footprint;
            r->state = 1;
        }
        for (size_t k = take.size(); k-- > 0;) S.queue.erase(S.queue.begin() + (std::ptrdiff_t)take[k]);
        Request* head = group.front();
        x.reserved = reserve;
        c->reserved += reserve;
        ++S.busy;
        lk.unlock();
        if (S.params.tick_mode != MCPT_SERVE_BATCH_END && joinable(head->opts)) {
            run_joined(c, S, x, *S.uploads[w], group);
            lk.lock();
            c->reserved -= std::min(c->reserved, x.reserved);
            x.reserved = S.uploads[w]->reserved = 0;
            --S.busy;
            ++S.batches;
            S.done_cv.notify_all();
            S.cv.notify_all();
            continue;
        }

        // ---- upload and solve the batch on this worker's stream ----
        std::vector<mcpt_problem> probs;
        probs.reserve(group.size());
        for (Request* r : group) probs.push_back(r->prob);
        mcpt_options opts = head->opts;
        uint64_t bid = 0;
        mcpt_summary sm{};
        mcpt_status st = MCPT_OK;
        Resident* R = nullptr;
        std::string err;
        try {
            st = upload_batch(c, x, probs.data(), (int)probs.size(), true, &bid);
            for (Request* r : group) {   // the device holds the inputs now
                r->k_intra.reset();
                r->v_dimer.reset();
                r->prob.k_intra = r->prob.v_dimer = nullptr;
            }
            if (st == MCPT_OK) {
                {
                    std::lock_guard<std::mutex> g(c->mu);
                    R = c->res[bid].get();
                }
                st = run(c, x, R, &opts, &sm);
            }
        } catch (const std::exception& e) {
            st = fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
        }
        if (st != MCPT_OK) err = last_error_text();
        const bool results = R && R->has_result;
        const double t_done = now_s();

        lk.lock();
        c->reserved -= std::min(c->reserved, x.reserved);
        x.reserved = 0;
        int holders = 0;
        for (size_t q = 0; q < group.size(); ++q) {
            Request* r = group[q];
            if (results) {
                r->sum = R->cl_last[q];
                r->batch = bid;
                r->cluster = (int)q;
                if (r->sum.status == MCPT_ERR_DIVERGED || r->sum.status == MCPT_ERR_NONFINITE) r->batch = 0;
                else ++holders;
            } else {
                r->sum = sm;
                r->sum.status = st == MCPT_OK ? MCPT_ERR_DEVICE : st;
                r->batch = 0;
            }
            if (r->sum.status != MCPT_OK) r->error = err.empty() ? "request did not converge" : err;
            r->sum.seconds = t_done - r->t_submit;   // latency: submission to result
            r->state = 2;
        }
        if (R) R->refs = holders;
        --S.busy;
        ++S.batches;
        S.served += group.size();
        const bool drop = R && holders == 0;
        if (drop) {   // nothing to keep: free the batch now
            lk.unlock();
            release_resident(c, bid);
            lk.lock();
        }
        S.done_cv.notify_all();
        S.cv.notify_all();
    }
}

// Host-side checks of a submitted problem: sizes, pairs and orbital energies
// (everything upload checks on the host), so that a bad request fails at
// submission and never inside a shared batch.  Non-finite integrals are found
// on the device per request: that request alone fails, with MCPT_ERR_NONFINITE.
mcpt_status check_request(const mcpt_problem* pb) {
    mcpt_status st = validate_problem(pb);
    if (st != MCPT_OK) return st;
    if (pb->memory != MCPT_HOST) return fail(MCPT_ERR_INVALID, "served requests take host memory");
    int64_t e = 0;
    for (int x = 0; x < pb->n_mono; ++x) {
        const int o = pb->n_occ[x], nv = pb->n_vir[x];
        double omax = -INFINITY, vmin = INFINITY;
        for (int i = 0; i < o + nv; ++i) {
            const double ei = pb->eps[e + i];
            if (!std::isfinite(ei)) return fail(MCPT_ERR_NONFINITE, "non-finite orbital energy");
            if (i < o) omax = std::max(omax, ei);
            else vmin = std::min(vmin, ei);
        }
        if (!(omax < vmin))
            return fail(MCPT_ERR_INVALID, "monomer " + std::to_string(x) +
                                              ": max occupied energy >= min virtual energy (denominator >= 0)");
        e += o + nv;
    }
    return MCPT_OK;
}

// Copy of a large caller array into a pinned pool block (or, with the pool
// full, new pageable memory), split over threads: memory bandwidth per thread
// and, for new pages, their first touch set the cost.
HostBuf copy_of(const double* src, int64_t n, PinnedPool& pool) {
    const size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(double);
    double* p = pool.take(bytes);
    HostBuf dst = p ? HostBuf(p, &pool) : HostBuf(new double[std::max<int64_t>(n, 1)], nullptr);
    if (!p) pool.count_pageable();
    const int64_t chunk = int64_t(8) << 20;   // 64 MiB
    const int nt = (int)std::min<int64_t>(8, (n + chunk - 1) / chunk);
    if (nt <= 1) {
        if (n) std::memcpy(dst.get(), src, n * sizeof(double));
        return dst;
    }
    std::vector<std::thread> th;
    double* d = dst.get();
    for (int t = 0; t < nt; ++t) {
        const int64_t b = n * t / nt, e = n * (t + 1) / nt;
        th.emplace_back([d, src, b, e] { std::memcpy(d + b, src + b, (e - b) * sizeof(double)); });
    }
    for (auto& t : th) t.join();
    return dst;
}

mcpt_status start_server(mcpt_ctx* c) {
    Server& S = *c->server;
    if (!S.workers.empty()) return MCPT_OK;
    for (int w = 0; w < 2 * S.params.workers; ++w) {
        auto x = std::make_unique<Exec>();
        mcpt_status st = exec_init(c, *x);
        if (st != MCPT_OK) {
            exec_free(c, *x);
            for (auto& e : S.execs) exec_free(c, *e);
            for (auto& e : S.uploads) exec_free(c, *e);
            S.execs.clear();
            S.uploads.clear();
            return st;
        }
        (w < S.params.workers ? S.execs : S.uploads).push_back(std::move(x));
    }
    for (int w = 0; w < S.params.workers; ++w) S.workers.emplace_back(worker_loop, c, w);
    return MCPT_OK;
}

Server& server_of(mcpt_ctx* c) {
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->server) c->server = std::make_unique<Server>();
    return *c->server;
}

}  // namespace

void serve_stop(mcpt_ctx* c) {
    if (!c->server) return;
    Server& S = *c->server;
    {
        std::lock_guard<std::mutex> g(c->mu);
        S.stop = true;
        for (uint64_t t : S.queue) {
            Request* r = S.reqs[t].get();
            r->state = 2;
            r->sum.status = MCPT_ERR_INVALID;
            r->error = "context destroyed before the request ran";
        }
        S.queue.clear();
        S.cv.notify_all();
        S.done_cv.notify_all();
    }
    for (auto& t : S.workers) t.join();
    S.workers.clear();
    for (auto& x : S.execs) exec_free(c, *x);
    for (auto& x : S.uploads) exec_free(c, *x);
    S.execs.clear();
    S.uploads.clear();
}

bool serve_owns(mcpt_ctx* c, uint64_t ticket) {
    std::lock_guard<std::mutex> g(c->mu);
    return c->server && c->server->reqs.count(ticket) != 0;
}

mcpt_status serve_energy(mcpt_ctx* c, uint64_t ticket, double* e_m2, double* de_m2, double* e_d2, double* t_amp) {
    Resident* R = nullptr;
    int q = 0;
    {
        std::lock_guard<std::mutex> g(c->mu);
        auto it = c->server->reqs.find(ticket);
        if (it == c->server->reqs.end()) return fail(MCPT_ERR_UNKNOWN_ID, "unknown ticket");
        Request* r = it->second.get();
        if (r->state != 2) return fail(MCPT_PENDING, "request is still queued or running");
        if (!r->batch) return fail(MCPT_ERR_INVALID, "request has no result: " + r->error);
        R = c->res[r->batch].get();
        q = r->cluster;
    }
    return slice_results(c, c->main, R, q, e_m2, de_m2, e_d2, t_amp);
}

mcpt_status serve_release(mcpt_ctx* c, uint64_t ticket) {
    uint64_t drop = 0;
    {
        std::lock_guard<std::mutex> g(c->mu);
        Server& S = *c->server;
        auto it = S.reqs.find(ticket);
        if (it == S.reqs.end()) return fail(MCPT_ERR_UNKNOWN_ID, "unknown ticket");
        Request* r = it->second.get();
        if (r->state == 1) return fail(MCPT_PENDING, "request is running; release it once it is done");
        if (r->state == 0) S.queue.erase(std::find(S.queue.begin(), S.queue.end(), ticket));
        if (r->state == 2 && r->batch) {
            Resident* R = c->res[r->batch].get();
            if (--R->refs == 0) drop = r->batch;
        }
        S.reqs.erase(it);
    }
    if (drop) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->main.stream);
        release_resident(c, drop);
    }
    std::lock_guard<std::mutex> g(c->mu);
    c->server->cv.notify_all();   // memory or the queue head changed
    return MCPT_OK;
}

}  // namespace mcpt

using namespace mcpt;

extern "C" {

mcpt_status mcpt_serve_config(mcpt_ctx* c, int32_t workers, int32_t max_batch, int64_t max_batch_pairs) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    if (workers < 1 || workers > 16) return fail(MCPT_ERR_INVALID, "workers must be in [1, 16]");
    if (max_batch < 1 || max_batch > 4096) return fail(MCPT_ERR_INVALID, "max_batch must be in [1, 4096]");
    if (max_batch_pairs < 1) return fail(MCPT_ERR_INVALID, "max_batch_pairs must be >= 1");
    Server& S = server_of(c);
    std::lock_guard<std::mutex> g(c->mu);
    if (!S.workers.empty()) return fail(MCPT_ERR_INVALID, "the scheduler is already running");
    S.params.workers = workers;
    S.params.max_batch = max_batch;
    S.params.max_batch_pairs = max_batch_pairs;
    return MCPT_OK;
}

mcpt_status mcpt_serve_tick_mode(mcpt_ctx* c, int32_t mode) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    if (mode < MCPT_SERVE_BATCH_END || mode > MCPT_SERVE_JOIN_AT_TICKS)
        return fail(MCPT_ERR_INVALID, "mode must be MCPT_SERVE_BATCH_END, _RETIRE_AT_TICKS or _JOIN_AT_TICKS");
    Server& S = server_of(c);
    std::lock_guard<std::mutex> g(c->mu);
    if (!S.workers.empty()) return fail(MCPT_ERR_INVALID, "the scheduler is already running");
    S.params.tick_mode = mode;
    return MCPT_OK;
}

mcpt_status mcpt_serve_staging(mcpt_ctx* c, uint64_t bytes) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    Server& S = server_of(c);
    std::lock_guard<std::mutex> g(c->mu);
    if (!S.workers.empty()) return fail(MCPT_ERR_INVALID, "the scheduler is already running");
    S.pool.set_cap((size_t)bytes);
    return MCPT_OK;
}

mcpt_status mcpt_submit(mcpt_ctx* c, const mcpt_problem* prob, const mcpt_options* opts, uint64_t* ticket) {
    if (!c || !ticket) return fail(MCPT_ERR_INVALID, "ctx or ticket is NULL");
    mcpt_status st = validate_options(opts);
    if (st != MCPT_OK) return st;
    if ((st = check_request(prob)) != MCPT_OK) return st;
    try {
        auto r = std::make_unique<Request>();
        const mcpt_problem& p = *prob;
        int64_t ne = 0, nk = 0, nv = 0;
        for (int x = 0; x < p.n_mono; ++x) {
            ne += p.n_occ[x] + p.n_vir[x];
            nk += (int64_t)p.n_occ[x] * p.n_occ[x] * p.n_vir[x] * p.n_vir[x];
        }
        for (int64_t k = 0; k < p.n_pair; ++k) {
            const int x = p.pair[2 * k], y = p.pair[2 * k + 1];
            nv += (int64_t)p.n_occ[x] * p.n_vir[x] * p.n_occ[y] * p.n_vir[y];
        }
        r->n_occ.assign(p.n_occ, p.n_occ + p.n_mono);
        r->n_vir.assign(p.n_vir, p.n_vir + p.n_mono);
        r->pair.assign(p.pair ? p.pair : nullptr, p.pair ? p.pair + 2 * p.n_pair : nullptr);
        r->eps.assign(p.eps, p.eps + ne);
        Server& S = server_of(c);
        r->k_intra = copy_of(p.k_intra, nk, S.pool);
        r->v_dimer = copy_of(p.v_dimer, nv, S.pool);
        int64_t nt = 0;
        for (int x = 0; x < p.n_mono; ++x) nt += (int64_t)p.n_occ[x] * p.n_vir[x] * p.n_occ[x] * p.n_vir[x];
        if (opts->warm_t) r->warm_t.assign(opts->warm_t, opts->warm_t + nt);
        r->prob = mcpt_problem{p.n_mono, r->n_occ.data(), r->n_vir.data(), r->eps.data(), r->k_intra.get(),
                               p.n_pair, r->pair.empty() ? nullptr : r->pair.data(),
                               nv ? r->v_dimer.get() : nullptr, MCPT_HOST};
        r->opts = *opts;
        r->opts.warm_t = opts->warm_t ? r->warm_t.data() : nullptr;
        r->footprint = footprint(&r->prob, 1, opts->precision);
        r->size_class = size_class(r->prob);
        r->t_submit = now_s();
        std::lock_guard<std::mutex> g(c->mu);
        if (r->footprint > c->budget)
            return fail(MCPT_ERR_ADMISSION, "request needs " + std::to_string(r->footprint) +
                                                " bytes of HBM; the budget is " + std::to_string(c->budget));
        if (S.stop) return fail(MCPT_ERR_INVALID, "context is shutting down");
        if ((st = start_server(c)) != MCPT_OK) return st;
        r->ticket = c->next_id++;
        *ticket = r->ticket;
        S.queue.push_back(r->ticket);
        S.reqs[r->ticket] = std::move(r);
        S.cv.notify_all();
        return MCPT_OK;
    } catch (const std::exception& e) {
        return fail(MCPT_ERR_NOMEM, std::string("host exception: ") + e.what());
    }
}

mcpt_status mcpt_poll(mcpt_ctx* c, uint64_t ticket, mcpt_summary* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->server) return fail(MCPT_ERR_UNKNOWN_ID, "unknown ticket");
    auto it = c->server->reqs.find(ticket);
    if (it == c->server->reqs.end()) return fail(MCPT_ERR_UNKNOWN_ID, "unknown ticket");
    const Request* r = it->second.get();
    if (r->state != 2) return MCPT_PENDING;
    if (out) *out = r->sum;
    if (r->sum.status != MCPT_OK) fail(MCPT_OK, r->error);
    return MCPT_OK;
}

mcpt_status mcpt_wait(mcpt_ctx* c, uint64_t ticket, int32_t timeout_ms, mcpt_summary* out) {
    if (!c) return fail(MCPT_ERR_INVALID, "ctx is NULL");
    std::unique_lock<std::mutex> lk(c->mu);
    if (!c->server) return fail(MCPT_ERR_UNKNOWN_ID, "unknown ticket");
    Server& S = *c->server;
    auto ready = [&] {
        auto it = S.reqs.find(ticket);
        return it == S.reqs.end() || it->second->state == 2;
    };
    if (timeout_ms < 0) S.done_cv.wait(lk, ready);
    else if (!S.done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return MCPT_PENDING;
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(MCPT_ERR_UNKNOWN_ID, "unknown ticket");
    if (out) *out = it->second->sum;
    if (it->second->sum.status != MCPT_OK) fail(MCPT_OK, it->second->error);
    return MCPT_OK;
}

mcpt_status mcpt_serve_stats(mcpt_ctx* c, mcpt_serve_counters* out) {
    if (!c || !out) return fail(MCPT_ERR_INVALID, "ctx or out is NULL");
    std::lock_guard<std::mutex> g(c->mu);
    *out = mcpt_serve_counters{};
    out->budget = c->budget;
    out->bytes_in_use = c->in_use;
    out->bytes_reserved = c->reserved;
    if (!c->server) return MCPT_OK;
    const Server& S = *c->server;
    out->batches = S.batches;
    out->completed = S.served;
    out->queued = (int32_t)S.queue.size();
    out->running_batches = S.busy;
    out->workers = (int32_t)S.workers.size();
    for (const auto& kv : S.reqs) out->tickets += 1;
    out->staging_pinned_bytes = S.pool.held();
    out->staged_pageable = S.pool.pageable();
    out->joined_at_ticks = S.joined;
    return MCPT_OK;
}

}  // extern "C"
