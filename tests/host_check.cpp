// Exercises the host-only runtime (paper_1409_2700_amd/csrc/host.cpp) on the CPU:
// problem validation, the orbital-energy check, the device-footprint arithmetic,
// the tuning-table parser and the serving scheduler's batch formation, including
// malformed and edge-case inputs.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py; exits non-zero on a
// failed check, and the sanitizers abort on any memory or UB error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../paper_1409_2700_amd/csrc/host.hpp"

using namespace mcpt;

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

struct Owned {   // a problem whose arrays it owns
    std::vector<int32_t> occ, vir, pair;
    std::vector<double> eps, k, v;
    mcpt_problem p{};
    void finish() {
        size_t ne = 0, nk = 0, nv = 0;
        for (size_t x = 0; x < occ.size(); ++x) {
            ne += occ[x] + vir[x];
            nk += (size_t)occ[x] * occ[x] * vir[x] * vir[x];
        }
        const int n = (int)occ.size();
        for (size_t q = 0; q < pair.size() / 2; ++q) {   // invalid pairs (for the error cases) get no block
            const int x = pair[2 * q], y = pair[2 * q + 1];
            if (x >= 0 && y >= 0 && x < n && y < n)
                nv += (size_t)occ[x] * vir[x] * occ[y] * vir[y];
        }
        eps.assign(ne, 0.0);
        size_t off = 0;
        for (size_t x = 0; x < occ.size(); ++x) {
            for (int i = 0; i < occ[x]; ++i) eps[off++] = -1.0 + 0.01 * i;
            for (int a = 0; a < vir[x]; ++a) eps[off++] = 0.5 + 0.01 * a;
        }
        k.assign(std::max<size_t>(nk, 1), 0.0);
        v.assign(std::max<size_t>(nv, 1), 0.0);
        p = mcpt_problem{(int32_t)occ.size(), occ.data(), vir.data(), eps.data(), k.data(),
                         (int64_t)(pair.size() / 2), pair.empty() ? nullptr : pair.data(), v.data(), MCPT_HOST};
    }
};

static Owned chain(int n, int o, int v) {
    Owned w;
    w.occ.assign(n, o);
    w.vir.assign(n, v);
    for (int x = 0; x + 1 < n; ++x) {
        w.pair.push_back(x);
        w.pair.push_back(x + 1);
    }
    w.finish();
    return w;
}

static void test_errors() {
    clear_error();
    CHECK(last_error_text().empty());
    CHECK(fail(MCPT_ERR_INVALID, "bad") == MCPT_ERR_INVALID);
    prefix_error("cluster 3: ");
    CHECK(last_error_text() == "cluster 3: bad");
    clear_error();
    CHECK(last_error_text().empty());
}

static void test_validate() {
    Owned ok = chain(4, 2, 3);
    CHECK(validate_problem(&ok.p) == MCPT_OK);
    CHECK(validate_problem(nullptr) == MCPT_ERR_INVALID);
    mcpt_problem b = ok.p;
    b.n_mono = 0;
    CHECK(validate_problem(&b) == MCPT_ERR_INVALID);
    b = ok.p;
    b.eps = nullptr;
    CHECK(validate_problem(&b) == MCPT_ERR_INVALID);
    b = ok.p;
    b.n_pair = -1;
    CHECK(validate_problem(&b) == MCPT_ERR_INVALID);
    b = ok.p;
    b.pair = nullptr;
    CHECK(validate_problem(&b) == MCPT_ERR_INVALID);
    b = ok.p;
    b.memory = 7;
    CHECK(validate_problem(&b) == MCPT_ERR_INVALID);
    Owned w = chain(3, 2, 3);
    w.pair = {0, 3};   // out of range
    w.finish();
    CHECK(validate_problem(&w.p) == MCPT_ERR_INVALID);
    w.pair = {1, 1};   // X == Y
    w.finish();
    CHECK(validate_problem(&w.p) == MCPT_ERR_INVALID);
    w.pair = {0, 1, 2, 0, 1, 0};   // (1, 0) duplicates (0, 1)
    w.finish();
    CHECK(validate_problem(&w.p) == MCPT_ERR_INVALID);
    CHECK(last_error_text().find("pair 2") != std::string::npos);
    w.pair = {-1, 0};
    w.finish();
    CHECK(validate_problem(&w.p) == MCPT_ERR_INVALID);
    Owned big = chain(2, 1, 1);
    big.occ[1] = 65;
    big.vir[1] = 64;   // o v = 4160 > 4096
    big.pair.clear();
    big.finish();
    CHECK(validate_problem(&big.p) == MCPT_ERR_INVALID);
    Owned zero = chain(2, 2, 2);
    zero.vir[0] = 0;
    CHECK(validate_problem(&zero.p) == MCPT_ERR_INVALID);
    Owned single = chain(1, 1, 1);   // one monomer, no pairs
    CHECK(validate_problem(&single.p) == MCPT_OK);
}

static void test_energies() {
    Owned w = chain(3, 2, 3);
    CHECK(check_energies(w.eps.data(), &w.p) == MCPT_OK);
    std::vector<double> e = w.eps;
    e[5 + 1] = NAN;   // second monomer's first virtual... any non-finite value
    CHECK(check_energies(e.data(), &w.p) == MCPT_ERR_NONFINITE);
    e = w.eps;
    e[1] = 0.6;       // occupied above the first virtual of monomer 0
    CHECK(check_energies(e.data(), &w.p) == MCPT_ERR_INVALID);
    e = w.eps;
    e[1] = 0.5;       // equal: denominator zero
    CHECK(check_energies(e.data(), &w.p) == MCPT_ERR_INVALID);
    e = w.eps;
    e[e.size() - 1] = INFINITY;
    CHECK(check_energies(e.data(), &w.p) == MCPT_ERR_NONFINITE);
}

static void test_footprint() {
    const LayoutSizes ls{64, 32, 48, 16, 4096, 16, 32};
    Owned w = chain(5, 5, 27);
    const size_t f64 = footprint(&w.p, 1, MCPT_FP64, ls);
    const size_t f32 = footprint(&w.p, 1, MCPT_FP32, ls), b16 = footprint(&w.p, 1, MCPT_BF16, ls);
    CHECK(f64 % 256 == 0 && f32 > f64 && b16 > f64);
    // the V block of four 135 x 135 pairs and five 144 x 144 matrices per monomer are in it
    CHECK(f64 >= (size_t)8 * 4 * 135 * 135 + (size_t)5 * 8 * 5 * 144 * 144);
    Owned two[2] = {chain(5, 5, 27), chain(3, 8, 56)};
    mcpt_problem ps[2] = {two[0].p, two[1].p};
    CHECK(footprint(ps, 2, MCPT_FP64, ls) > footprint(ps, 1, MCPT_FP64, ls));
    Owned single = chain(1, 1, 1);
    CHECK(footprint(&single.p, 1, MCPT_BF16, ls) > 0);
    Owned large = chain(200, 8, 56);   // no overflow of the 64-bit sums
    CHECK(footprint(&large.p, 1, MCPT_FP32, ls) > (size_t)8 * 199 * 448 * 448);
}

static void test_tune_parser() {
    const int shapes[] = {2, 8, 1, 3, 8, 1, 4, 8, 2, 2, 16, 1};
    std::map<std::string, int> out;
    CHECK(parse_tune_table("a/b 3 8 1\n\nc 2 16 1\n", shapes, 4, &out) == MCPT_OK);
    CHECK(out.size() == 2 && out["a/b"] == 1 && out["c"] == 3);
    CHECK(parse_tune_table("", shapes, 4, &out) == MCPT_OK && out.size() == 2);
    CHECK(parse_tune_table("x 3 8", shapes, 4, &out) == MCPT_ERR_INVALID);
    CHECK(parse_tune_table("x 9 9 9\n", shapes, 4, &out) == MCPT_ERR_INVALID);
    CHECK(parse_tune_table("y 3 8 1\nbad line\n", shapes, 4, &out) == MCPT_ERR_INVALID);
    CHECK(out.size() == 2);   // nothing added by a failed parse
    std::string longkey(600, 'k');
    CHECK(parse_tune_table((longkey + " 3 8 1\n").c_str(), shapes, 4, &out) == MCPT_ERR_INVALID);
    std::string k511(511, 'q');
    CHECK(parse_tune_table((k511 + " 2 8 1").c_str(), shapes, 4, &out) == MCPT_ERR_INVALID);   // line too long
    CHECK(parse_tune_table("z 2 8 1", shapes, 4, &out) == MCPT_OK && out["z"] == 0);   // no final newline
    CHECK(parse_tune_table(nullptr, shapes, 4, &out) == MCPT_ERR_INVALID);
    CHECK(parse_tune_table("a 1 2 3", shapes, 0, &out) == MCPT_ERR_INVALID);
}

static void test_batches() {
    std::mt19937_64 rng(14092700);
    mcpt_options base{};
    base.tol = 1e-10;
    base.max_sweeps = 200;
    mcpt_options other = base;
    other.precision = MCPT_FP32;
    const double warm = 0.0;
    mcpt_options warm_opts = base;
    warm_opts.warm_t = &warm;
    for (int trial = 0; trial < 2000; ++trial) {
        const int n = (int)(rng() % 40);
        std::vector<QueuedRequest> q;
        for (int i = 0; i < n; ++i) {
            const int kind = (int)(rng() % 10);
            q.push_back({(size_t)(1 + rng() % 1000), (int64_t)(rng() % 5000), (int)(20 + rng() % 6),
                         kind == 0 ? &other : (kind == 1 && i == 0 && trial % 7 == 0 ? &warm_opts : &base)});
        }
        const size_t free_b = (size_t)(rng() % 8000);
        const int max_batch = 1 + (int)(rng() % 16);
        const int64_t max_pairs = (int64_t)(rng() % 20000);
        const std::vector<size_t> g = form_batch(q, free_b, max_batch, max_pairs);
        if (q.empty() || q[0].footprint > free_b) {
            CHECK(g.empty());
            continue;
        }
        CHECK(!g.empty() && g[0] == 0);
        size_t fp = 0;
        int64_t pairs = 0;
        for (size_t k = 0; k < g.size(); ++k) {
            CHECK(g[k] < q.size());
            if (k) CHECK(g[k] > g[k - 1]);
            fp += q[g[k]].footprint;
            pairs += q[g[k]].n_pair;
            if (k) {
                CHECK(same_options(*q[g[k]].opts, *q[0].opts));
                CHECK(std::abs(q[g[k]].size_class - q[0].size_class) <= 1);
            }
        }
        CHECK(fp <= free_b);
        CHECK((int)g.size() <= max_batch);
        if (g.size() > 1) CHECK(pairs <= max_pairs + q[0].n_pair);
        if (q[0].opts->warm_t) CHECK(g.size() == 1);
    }
    CHECK(form_batch({}, 100, 4, 100).empty());
    mcpt_options det = base;
    det.deterministic = 1;
    CHECK(!same_options(base, det));
}

// Admission at sweep ticks into a running FP64 batch: the head of the queue, in order, while
// each request is compatible, priced at twice its footprint, and within the batch's request and
// pair limits; the first that does not qualify ends the run.
static void test_joins() {
    std::mt19937_64 rng(27001409);
    mcpt_options base{};
    base.tol = 1e-10;
    base.max_sweeps = 200;
    mcpt_options lowp = base, det = base, graph = base;
    lowp.precision = MCPT_BF16;
    det.deterministic = 1;
    graph.graph = 1;
    const double warm = 0.0;
    mcpt_options warm_opts = base;
    warm_opts.warm_t = &warm;
    CHECK(joinable(base));
    mcpt_options none = base;
    none.max_sweeps = 0;
    CHECK(!joinable(lowp) && !joinable(det) && !joinable(graph) && !joinable(warm_opts) && !joinable(none));
    const mcpt_options* kinds[5] = {&base, &lowp, &det, &graph, &warm_opts};
    for (int trial = 0; trial < 2000; ++trial) {
        const int n = (int)(rng() % 40);
        std::vector<QueuedRequest> q;
        for (int i = 0; i < n; ++i) {
            const int kind = (int)(rng() % 8);
            q.push_back({(size_t)(1 + rng() % 1000), (int64_t)(rng() % 5000), (int)(20 + rng() % 6),
                         kind < 4 ? kinds[kind] : (kind == 4 ? kinds[4] : &base)});
        }
        const mcpt_options& batch = trial % 5 == 0 ? *kinds[rng() % 5] : base;
        const size_t free_b = (size_t)(rng() % 8000);
        const int cls = (int)(20 + rng() % 6);
        const int live = (int)(rng() % 8);
        const int max_batch = 1 + (int)(rng() % 16);
        const int64_t live_pairs = (int64_t)(rng() % 10000);
        const int64_t max_pairs = (int64_t)(rng() % 40000);
        const size_t live_bytes = trial % 3 == 0 ? (size_t)(rng() % 3000) : 0;
        const std::vector<size_t> g =
            join_batch(q, free_b, batch, cls, live, live_pairs, live_bytes, max_batch, max_pairs);
        if (!joinable(batch)) {
            CHECK(g.empty());
            continue;
        }
        if (live_bytes) {   // the same scan without the copy rule: taken whole, or not at all
            const std::vector<size_t> h = join_batch(q, free_b, batch, cls, live, live_pairs, 0, max_batch, max_pairs);
            size_t fp = 0;
            for (size_t k : h) fp += q[k].footprint;
            CHECK(fp >= live_bytes ? g == h : g.empty());
            if (g.empty()) continue;
        }
        size_t used = 0;
        int64_t pairs = live_pairs;
        for (size_t k = 0; k < g.size(); ++k) {
            CHECK(g[k] < q.size());
            if (k) CHECK(g[k] > g[k - 1]);
            const QueuedRequest& r = q[g[k]];
            CHECK(same_options(*r.opts, batch) && joinable(*r.opts));
            CHECK(std::abs(r.size_class - cls) <= 1);
            used += 2 * r.footprint;
            pairs += r.n_pair;
        }
        CHECK(used <= free_b);
        CHECK(pairs <= std::max(max_pairs, live_pairs));
        CHECK(live + (int)g.size() <= std::max(max_batch, live));
        // the joiners are the head of the queue, in order, up to the first that does not qualify
        for (size_t k = 0; k < g.size(); ++k) CHECK(g[k] == k);
        if (g.size() < q.size() && live + (int)g.size() < max_batch) {
            const QueuedRequest& r = q[g.size()];
            CHECK(!same_options(*r.opts, batch) || std::abs(r.size_class - cls) > 1 || pairs + r.n_pair > max_pairs ||
                  2 * r.footprint > free_b - used);
        }
    }
    CHECK(join_batch({}, 100, base, 20, 0, 0, 0, 4, 100).empty());
}

static void test_size_class() {
    Owned w = chain(3, 5, 27);
    const int c = size_class(w.p);
    // two 135 x 135 pairs: 2 x 4 x 135^2 x 270 flops
    CHECK(c == (int)std::floor(std::log2(2.0 * 4.0 * 135.0 * 135.0 * 270.0)));
    Owned one = chain(1, 2, 2);
    CHECK(size_class(one.p) == 0);
}

int main() {
    test_errors();
    test_validate();
    test_energies();
    test_footprint();
    test_tune_parser();
    test_batches();
    test_joins();
    test_size_class();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
