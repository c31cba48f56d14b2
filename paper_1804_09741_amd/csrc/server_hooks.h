// Internal hooks between prepared batches and the request server (not part
// of the C ABI): the work-unit range of each graph of a planned batch and
// the collection of one graph's histogram.
#pragma once

#include <vector>

#include "internal.h"

namespace mk {

// First work unit of every graph of a batch after mk_batch_create (its
// sizing plan), plus the total: ng + 1 values.  Blocks.
int batch_unit_begins(mk_batch *b, std::vector<uint32_t> *out);

// Finish graph gi's histogram (the core method's division) and copy it to
// host memory on copy_stream once its units are known to be done.
int batch_collect_graph(mk_batch *b, int gi, uint64_t *hist, hipStream_t copy_stream);

// Device side of batch_unit_begins: out[gi] = first unit of graph gi,
// out[ng] = the number of units.
int launch_unit_begins(const DevGraph *d_graphs, int ng, const uint32_t *slot_off,
                       uint32_t total_slots, const uint32_t *counters, uint32_t *out,
                       hipStream_t stream);

}  // namespace mk
