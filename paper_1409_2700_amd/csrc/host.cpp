// Host-only parts of the runtime (see host.hpp): plain C++, no HIP.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <unordered_set>

namespace mcpt {

namespace {
thread_local std::string g_err;
}

mcpt_status fail(mcpt_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

const std::string& last_error_text() { return g_err; }

void prefix_error(const std::string& prefix) { g_err = prefix + g_err; }

void clear_error() { g_err.clear(); }

mcpt_status validate_problem(const mcpt_problem* pb) {
    if (!pb) return fail(MCPT_ERR_INVALID, "problem is NULL");
    if (pb->n_mono < 1) return fail(MCPT_ERR_INVALID, "n_mono must be >= 1");
    if (!pb->n_occ || !pb->n_vir || !pb->eps || !pb->k_intra)
        return fail(MCPT_ERR_INVALID, "n_occ, n_vir, eps and k_intra must be non-NULL");
    if (pb->n_pair < 0) return fail(MCPT_ERR_INVALID, "n_pair must be >= 0");
    if (pb->n_pair > 0 && (!pb->pair || !pb->v_dimer))
        return fail(MCPT_ERR_INVALID, "pair and v_dimer must be non-NULL when n_pair > 0");
    if (pb->memory != MCPT_HOST && pb->memory != MCPT_DEVICE)
        return fail(MCPT_ERR_INVALID, "memory must be MCPT_HOST or MCPT_DEVICE");
    for (int x = 0; x < pb->n_mono; ++x) {
        const int o = pb->n_occ[x], v = pb->n_vir[x];
        if (o < 1 || v < 1) return fail(MCPT_ERR_INVALID, "monomer " + std::to_string(x) + ": o, v must be >= 1");
        if ((int64_t)o * v > 4096)
            return fail(MCPT_ERR_INVALID, "monomer " + std::to_string(x) + ": o*v > 4096 not supported");
    }
    std::unordered_set<uint64_t> seen;
    seen.reserve((size_t)pb->n_pair * 2);
    for (int64_t p = 0; p < pb->n_pair; ++p) {
        const int x = pb->pair[2 * p], y = pb->pair[2 * p + 1];
        if (x < 0 || y < 0 || x >= pb->n_mono || y >= pb->n_mono)
            return fail(MCPT_ERR_INVALID, "pair " + std::to_string(p) + " out of range");
        if (x == y) return fail(MCPT_ERR_INVALID, "pair " + std::to_string(p) + " has X == Y");
        const uint64_t key = ((uint64_t)std::min(x, y) << 32) | (uint32_t)std::max(x, y);
        if (!seen.insert(key).second)
            return fail(MCPT_ERR_INVALID, "pair " + std::to_string(p) + " duplicates an earlier pair");
    }
    return MCPT_OK;
}

mcpt_status check_energies(const double* eps, const mcpt_problem* pb) {
    int64_t off = 0;
    for (int x = 0; x < pb->n_mono; ++x) {
        const int o = pb->n_occ[x], v = pb->n_vir[x];
        double omax = -INFINITY, vmin = INFINITY;
        for (int k = 0; k < o + v; ++k) {
            const double e = eps[off + k];
            if (!std::isfinite(e))
                return fail(MCPT_ERR_NONFINITE, "non-finite orbital energy of monomer " + std::to_string(x));
            if (k < o) omax = std::max(omax, e);
            else vmin = std::min(vmin, e);
        }
        if (!(omax < vmin))
            return fail(MCPT_ERR_INVALID, "monomer " + std::to_string(x) +
                                              ": max occupied energy >= min virtual energy (denominator >= 0)");
        off += o + v;
    }
    return MCPT_OK;
}

size_t footprint(const mcpt_problem* pbs, int n, int precision, const LayoutSizes& ls) {
    int64_t n_mono = 0, n_pair = 0, dif = 0, raw = 0, mat = 0, v = 0, vlo = 0, mlo = 0;
    const int kc = precision == MCPT_FP64 ? 0 : (precision == MCPT_BF16 ? ls.chunk_bf16 : ls.chunk_fp32);
    const int64_t t = ls.tile;
    auto ld = [kc](int64_t m) { return (m + kc - 1) / kc * kc; };
    auto pad = [t](int64_t m) { return (m + t - 1) / t * t; };
    for (int q = 0; q < n; ++q) {
        const mcpt_problem& p = pbs[q];
        for (int x = 0; x < p.n_mono; ++x) {
            const int64_t nx = (int64_t)p.n_occ[x] * p.n_vir[x], np = pad(nx);
            dif += np;
            raw += nx * nx;
            mat += np * np;
            if (kc) mlo += np * ld(nx);
        }
        for (int64_t k = 0; k < p.n_pair; ++k) {
            const int x = p.pair[2 * k], y = p.pair[2 * k + 1];
            const int64_t nx = (int64_t)p.n_occ[x] * p.n_vir[x], ny = (int64_t)p.n_occ[y] * p.n_vir[y];
            v += nx * ny;
            if (kc) vlo += pad(nx) * ld(ny) + pad(ny) * ld(nx);
        }
        n_mono += p.n_mono;
        n_pair += p.n_pair;
    }
    auto r = [](int64_t bytes) { return (size_t)((std::max<int64_t>(bytes, 1) + 255) / 256 * 256); };
    size_t b = r(n_mono * ls.mono_desc) + r(std::max<int64_t>(n_pair, 1) * ls.pair_desc) + r(8 * dif) +
               r(8 * raw) + 5 * r(8 * mat) + r(8 * std::max<int64_t>(v, 1)) + 3 * r(8 * n_mono) +
               r(8 * std::max<int64_t>(n_pair, 1)) + r((int64_t)n * ls.cl_state) +
               r(8 * (int64_t)n * ls.max_sweeps) + 2 * r(8 * (int64_t)(n + 1)) + r(4 * (int64_t)n);
    if (kc) {
        const int64_t es = precision == MCPT_BF16 ? 2 : 4;
        b += r(es * vlo) + r(es * mlo) + r(8 * std::max<int64_t>(n_pair, 1)) + r(8 * n_mono) + 2 * r(8 * mat);
        if (precision == MCPT_BF16) b += r(8 * mat);   // two FP32 G buffers
    }
    return b;
}

mcpt_status parse_tune_table(const char* text, const int* shapes, int n_shapes,
                             std::map<std::string, int>* out) {
    if (!text || !out) return fail(MCPT_ERR_INVALID, "text or out is NULL");
    std::map<std::string, int> add;
    const std::string t(text);
    size_t pos = 0;
    while (pos < t.size()) {
        size_t e = t.find('\n', pos);
        if (e == std::string::npos) e = t.size();
        const std::string line = t.substr(pos, e - pos);
        pos = e + 1;
        if (line.empty()) continue;
        char key[512];
        int sb = 0, nw = 0, pd = 0;
        if (line.size() >= sizeof(key) || std::sscanf(line.c_str(), "%511s %d %d %d", key, &sb, &nw, &pd) != 4)
            return fail(MCPT_ERR_INVALID, "bad tuning line: " + line);
        int v = -1;
        for (int k = 0; k < n_shapes; ++k)
            if (shapes[3 * k] == sb && shapes[3 * k + 1] == nw && shapes[3 * k + 2] == pd) v = k;
        if (v < 0)
            return fail(MCPT_ERR_INVALID, "no tile variant " + std::to_string(sb) + " x " + std::to_string(nw) +
                                              " depth " + std::to_string(pd));
        add[key] = v;
    }
    for (const auto& kv : add) (*out)[kv.first] = kv.second;
    return MCPT_OK;
}

bool same_options(const mcpt_options& a, const mcpt_options& b) {
    return a.tol == b.tol && a.max_sweeps == b.max_sweeps && a.precision == b.precision && a.polish == b.polish &&
           a.check_every == b.check_every && a.inner_sweeps == b.inner_sweeps && a.graph == b.graph &&
           a.deterministic == b.deterministic && !a.warm_t && !b.warm_t;
}

int size_class(const mcpt_problem& p) {
    double f = 0.0;
    for (int64_t k = 0; k < p.n_pair; ++k) {
        const double nx = (double)p.n_occ[p.pair[2 * k]] * p.n_vir[p.pair[2 * k]];
        const double ny = (double)p.n_occ[p.pair[2 * k + 1]] * p.n_vir[p.pair[2 * k + 1]];
        f += 4.0 * nx * ny * (nx + ny);
    }
    return f > 1.0 ? (int)std::floor(std::log2(f)) : 0;
}

std::vector<size_t> form_batch(const std::vector<QueuedRequest>& queue, size_t free_bytes, int max_batch,
                               int64_t max_batch_pairs) {
    std::vector<size_t> group;
    if (queue.empty() || queue[0].footprint > free_bytes) return group;
    const QueuedRequest& head = queue[0];
    size_t reserve = 0;
    int64_t pairs = 0;
    for (size_t i = 0; i < queue.size(); ++i) {
        const QueuedRequest& r = queue[i];
        const bool first = group.empty();
        if (!first && ((int)group.size() >= max_batch || !same_options(*r.opts, *head.opts) ||
                       std::abs(r.size_class - head.size_class) > 1 || pairs + r.n_pair > max_batch_pairs))
            continue;
        if (!first && reserve + r.footprint > free_bytes) break;
        group.push_back(i);
        reserve += r.footprint;
        pairs += r.n_pair;
        if (head.opts->warm_t) break;   // a warm start runs alone
    }
    return group;
}

bool joinable(const mcpt_options& o) {
    return o.precision == MCPT_FP64 && !o.graph && !o.deterministic && !o.warm_t && o.max_sweeps > 0;
}

std::vector<size_t> join_batch(const std::vector<QueuedRequest>& queue, size_t free_bytes, const mcpt_options& batch,
                               int batch_class, int live, int64_t live_pairs, size_t live_bytes, int max_batch,
                               int64_t max_batch_pairs) {
    std::vector<size_t> take;
    if (!joinable(batch)) return take;
    size_t used = 0;
    int64_t pairs = live_pairs;
    int n = live;
    for (size_t i = 0; i < queue.size() && n < max_batch; ++i) {
        const QueuedRequest& r = queue[i];
        if (!same_options(*r.opts, batch) || std::abs(r.size_class - batch_class) > 1 ||
            pairs + r.n_pair > max_batch_pairs || r.footprint > (free_bytes - used) / 2)
            break;
        take.push_back(i);
        used += 2 * r.footprint;
        pairs += r.n_pair;
        ++n;
    }
    if (used / 2 < live_bytes) take.clear();   // copying the unfinished clusters would cost more than the joiners
    return take;
}

}  // namespace mcpt
