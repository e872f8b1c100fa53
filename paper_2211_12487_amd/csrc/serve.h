// Hooks of the TT-ICE engine for the serving layer (server.hip), internal to
// the library: one grouped level-1 launch over the increments of several
// streams (Algorithm 1's first projection, eq:first_resid), then each
// stream's update continues from its own level-1 results.
#pragma once

#include "../../include/ttice.h"
#include "kernels.h"

namespace ttice {

// Doubles of every state's K-split workspace (partials of the products that
// split K: up to 3 slices of a 1400 x 512 output at level 6 of the order-8
// stream); the server's footprint estimate counts it.
constexpr int64_t kSplitKDoubles = (int64_t)1 << 22;

// Level 1 of the state's Algorithm 1 updates always takes the fused
// projection with one column per lane (alone or grouped: the same values).
void serve_mark(ttice_state* st);
// Rank bounds r_0 .. r_d (rb, d + 1 entries) of a stream of at most T
// tensors, and the state's core capacities capped at them (a reservation
// computed from the bounds then covers every allocation of its cores).
void serve_rank_bounds(int32_t d, const int64_t* dims, int64_t T, int64_t* rb);
void serve_limit(ttice_state* st, int64_t max_tensors);
// Prepares ttice_update(st, batch, n, dtype) up to its level-1 projection
// (workspace, padding of the last core) and returns 1 with that launch's
// arguments in *desc and its group key in *key (equal keys: one grouped
// launch may hold both), or 0 when the update must run as a plain
// ttice_update (not Algorithm 1, not served, a launch that does not apply,
// or an error, which the plain call reports).  The state's stream must be
// the one the grouped launch goes to.
int serve_capture(ttice_state* st, const void* batch, int64_t n, int32_t dtype, ProjDesc* desc, int32_t* key);
// ttice_update after the captured level-1 launch has been made (ordered
// before this call's work on the state's stream).
int serve_update_after(ttice_state* st, const void* batch, int64_t n, int32_t dtype, ttice_update_info* info);
// One launch for g.n captured projections of equal key.
hipError_t serve_group_launch(hipStream_t s, int32_t key, const ProjGroup& g);

}  // namespace ttice
