// Internal entry points of the batch used by the serving engine (not part of
// the C interface): one environment's internal state as an opaque snapshot,
// and the row layout of the caller-order arrays.
#pragma once
#include <stdint.h>

#include "../../include/mpm.h"

namespace mpmx {

// floats of a snapshot of env's current particles (state, caller ids)
int64_t env_snapshot_floats(const mpm_batch* b, int env);
// copies env's internal state (held as F - I, in its current sorted order)
// into the DEVICE buffer dst (env_snapshot_floats floats) on the batch's
// stream; *steps receives env's clock
int env_snapshot(mpm_batch* b, int env, float* dst, int64_t* steps);
// the inverse: env's particles and clock as they were when the snapshot was
// taken (env's particle count must be unchanged); drops any record
int env_restore(mpm_batch* b, int env, const float* src, int64_t steps);
// first row of env in the concatenation of the current counts
int64_t env_row_offset(const mpm_batch* b, int env);
// the batch's stream
void* batch_stream(const mpm_batch* b);

}  // namespace mpmx
