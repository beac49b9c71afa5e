// prop_launch.h -- host-callable launchers of the propagation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "prop_layout.h"

namespace prop {

hipError_t launch_init(const Problem& P, hipStream_t s);
hipError_t launch_pack(const Problem& P, const double* lb, const double* ub, hipStream_t s);
hipError_t launch_unpack(const Problem& P, double* lb, double* ub, hipStream_t s);
hipError_t persistent_occupancy(int* blocks_per_cu, bool nnz_split);
hipError_t launch_persistent(const Problem& P, int max_rounds, int grid, hipStream_t s);
hipError_t launch_start(const Problem& P, int max_rounds, hipStream_t s);
// Queues one round: the matrix kernel (bracketed by e0 / e1 when they are
// not null), the long-row kernel, the commit and, in marked rounds, the
// mark kernel.  The kernels take the round number and limit from the
// control block (set by the start kernel and each commit), so the same
// launches can be captured once and replayed.
hipError_t launch_round(const Problem& P, hipStream_t s, hipEvent_t e0, hipEvent_t e1);

// Batched nodes: pack / unpack nodes [k0, k0 + cnt) of the caller's
// node-major arrays, round-0 decision for such a range (whole = the range is
// the whole batch), and one round of every active node.
hipError_t launch_pack_batch(const Problem& P, const Batch& Bt, const double* lb, const double* ub,
                             int k0, int cnt, hipStream_t s);
hipError_t launch_unpack_batch(const Problem& P, const Batch& Bt, double* lb, double* ub, int k0,
                               int cnt, hipStream_t s);
hipError_t launch_start_batch(const Problem& P, const Batch& Bt, int max_rounds, int k0, int cnt,
                              bool whole, hipStream_t s);
hipError_t launch_round_batch(const Problem& P, const Batch& Bt, hipStream_t s);
// Marked batches from a parent fixed point: stamps, for round 1, the rows of
// the variables whose start bounds differ from the parent's (per group).
hipError_t launch_seed_batch(const Problem& P, const Batch& Bt, hipStream_t s);
// Marked single runs from a parent fixed point: the same for one bound vector.
hipError_t launch_seed(const Problem& P, hipStream_t s);
// Normalises (integer rounding) and relabels a parent fixed point into
// P.parent; sets the control block's invalid flag for a bad bound.
hipError_t launch_set_parent(const Problem& P, double2* parent, const double* lb,
                             const double* ub, hipStream_t s);
// Compaction of a batch: slot moves (moves[q].x -> moves[q].y, device
// array) and unpacking of listed slots (pairs[q] = (slot, caller's row)).
hipError_t launch_move_batch(const Problem& P, const Batch& Bt, const int2* moves, int count,
                             hipStream_t s);
hipError_t launch_unpack_slots(const Problem& P, const Batch& Bt, double* lb, double* ub,
                               const int2* pairs, int count, hipStream_t s);

// Serving: one round of every instance listed in step S (device copy; H is
// the host copy it was uploaded from, for the grid sizes).
hipError_t launch_srv_round(const SrvInst* I, SrvStep* S, const SrvStep& H, hipStream_t s);

}  // namespace prop
