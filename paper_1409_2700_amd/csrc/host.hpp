// Host-only parts of the runtime: error text, problem validation, device
// footprint, the tuning-table parser and the serving scheduler's batch
// formation.  Plain C++ with no HIP dependency, so the same translation unit
// (host.cpp) is linked into the library and built for the CPU alone by the
// sanitizer test.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/mcpt.h"

namespace mcpt {

// Thread-local message of the last error (mcpt_last_error).
mcpt_status fail(mcpt_status s, const std::string& msg);
const std::string& last_error_text();
void prefix_error(const std::string& prefix);
void clear_error();

// Sizes, counts and indices of a problem (host arrays n_occ, n_vir, pair):
// MCPT_ERR_INVALID with a message naming the first violation.
mcpt_status validate_problem(const mcpt_problem* pb);
// Orbital energies (o then v per monomer, host copy): every value finite and
// every monomer's highest occupied below its lowest virtual, so that every
// denominator of Eqs. 60-61 is negative.
mcpt_status check_energies(const double* eps, const mcpt_problem* pb);

// Byte sizes the device layout takes, from the structs of the HIP side.
struct LayoutSizes {
    int64_t mono_desc, pair_desc, cl_state;
    int tile, max_sweeps;
    int chunk_fp32, chunk_bf16;   // k chunk that rows of reduced-precision operands are padded to
};
// Device bytes an upload of clusters pbs[0..n-1] allocates (and, for a reduced
// precision, the copies its first run adds), each allocation rounded to 256 B.
size_t footprint(const mcpt_problem* pbs, int n, int precision, const LayoutSizes& ls);

// Tuning table: one "key sb nw pd" line per entry ('\n' separated, blank lines
// skipped); shapes[3k..3k+2] = sb, nw, pd of variant k.  On success *out gains
// key -> variant; a malformed line or an unknown shape is MCPT_ERR_INVALID and
// leaves *out unchanged.
mcpt_status parse_tune_table(const char* text, const int* shapes, int n_shapes,
                             std::map<std::string, int>* out);

// Serving: options under which requests may share a batch, and the log2 size
// class of a request's pair-phase flops.
bool same_options(const mcpt_options& a, const mcpt_options& b);
int size_class(const mcpt_problem& p);

// One queued request as the scheduler sees it.
struct QueuedRequest {
    size_t footprint;
    int64_t n_pair;
    int size_class;
    const mcpt_options* opts;
};
// The requests (queue positions, in order) a free worker takes: the head if it
// fits in free_bytes, then later requests with the head's options, within one
// size class of it, while the batch stays within max_batch requests,
// max_batch_pairs pairs and free_bytes; the scan stops at the first compatible
// request that no longer fits, and a head with a warm start runs alone.
std::vector<size_t> form_batch(const std::vector<QueuedRequest>& queue, size_t free_bytes, int max_batch,
                               int64_t max_batch_pairs);

// Serving at sweep ticks: the queued requests that join a running FP64 batch whose clusters
// run with options `batch` and whose first request had size class batch_class, now holding
// `live` unfinished requests with live_pairs pairs.  Joiners are taken from the head of the
// queue, in order, while each has the batch's options (FP64 plain sweeps, at least one: no
// reduced precision, graphs, deterministic accumulation or warm start), a size class within one
// of batch_class, and room in max_batch, max_batch_pairs and free_bytes, where each costs twice
// its footprint (its upload, then its copy in the merged batch).  The first request that does
// not qualify ends the run, so a request a running batch cannot take is never overtaken by joins:
// the batches drain and a free worker takes it.  A join copies the unfinished clusters
// (live_bytes of footprint) into the merged batch: it happens only when the joiners' footprint
// is at least that, i.e. near the end of a batch, where merging fills launches that its last
// clusters alone would leave mostly idle.
bool joinable(const mcpt_options& o);
std::vector<size_t> join_batch(const std::vector<QueuedRequest>& queue, size_t free_bytes, const mcpt_options& batch,
                               int batch_class, int live, int64_t live_pairs, size_t live_bytes, int max_batch,
                               int64_t max_batch_pairs);

}  // namespace mcpt
