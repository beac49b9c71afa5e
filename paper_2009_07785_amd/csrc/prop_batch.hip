// prop_batch.hip -- gfx950 kernels for many bound vectors of one problem:
// batched branch-and-bound nodes and the serving engine's slots.  Nodes
// come in groups of 8 whose (l, u) pairs share one 128-byte line per
// variable; a group with more than kLoopNodes active nodes runs with
// node-parallel lanes, a smaller one node after node in the single-run
// shape.  Every node's results are those of its own single run.
#include <hip/hip_runtime.h>

#include "prop_device.h"
#include "prop_launch.h"
#include "prop_layout.h"

#pragma clang fp contract(off)

namespace prop {

// ---------------------------------------------------------------------------
// batched nodes (one problem, many bound vectors): every node runs exactly
// the arithmetic of a single run; nodes that finished are masked out
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t group_mask(const Batch& Bt, int g) {
  uint32_t mask = 0;
#pragma unroll
  for (int t = 0; t < kNodeGroup; ++t) {
    const int k = g * kNodeGroup + t;
    if (k < Bt.nodes && Bt.active[k]) mask |= 1u << t;
  }
  return mask;
}

// Nodes of group g whose rows all take the exact sums (a tiny bound).
__device__ __forceinline__ uint32_t group_exact(const Batch& Bt, int g) {
  uint32_t mask = 0;
#pragma unroll
  for (int t = 0; t < kNodeGroup; ++t) {
    const int k = g * kNodeGroup + t;
    if (k < Bt.nodes && Bt.tiny[k]) mask |= 1u << t;
  }
  return mask;
}

// Packs nodes [k0, k0 + cnt) from node-major arrays (row q = node k0 + q).
// One thread takes one variable of one group of 8 nodes and writes its
// nodes' pairs of that variable's 128-byte line itself, so a full group
// writes whole lines; reads stay coalesced (consecutive threads, consecutive
// variables of one node row).
__global__ __launch_bounds__(kBlock) void k_pack_batch(Problem P, Batch Bt,
                                                       const double* __restrict__ ulb,
                                                       const double* __restrict__ uub, int k0,
                                                       int cnt) {
  const int g0 = k0 / kNodeGroup;
  const int groups = (k0 + cnt - 1) / kNodeGroup - g0 + 1;
  const size_t total = (size_t)groups * P.n;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int g = g0 + (int)(i / (size_t)P.n);
    const int v = (int)(i - (size_t)(g - g0) * P.n);
    const int kb = max(k0, g * kNodeGroup);
    const int ke = min(k0 + cnt, (g + 1) * kNodeGroup);
    const int32_t j = P.perm[v];
    const bool is_int = P.vtype[j] != 0;
    double2* const la = Bt.gA[g] + (size_t)j * kNodeGroup;
    double2* const lb2 = Bt.gB[g] + (size_t)j * kNodeGroup;
    for (int k = kb; k < ke; ++k) {
      const size_t src = (size_t)(k - k0) * P.n + v;
      double l = ulb[src], u = uub[src];
      const bool bad = __builtin_isnan(l) || __builtin_isnan(u) || l == __builtin_inf() ||
                       u == -__builtin_inf() ||
                       (!is_inf(l) && __builtin_fabs(l) > PROP_HUGE) ||
                       (!is_inf(u) && __builtin_fabs(u) > PROP_HUGE);
      if (bad) __hip_atomic_store(&Bt.invalid[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (is_int) {
        l = __builtin_ceil(l - P.eps_int);
        u = __builtin_floor(u + P.eps_int);
      }
      l = l + 0.0;
      u = u + 0.0;
      const double2 b = make_double2(l, u);
      la[k % kNodeGroup] = b;
      lb2[k % kNodeGroup] = b;
      if (tiny_bound(l) || tiny_bound(u))
        __hip_atomic_store(&Bt.tiny[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (domain_empty(is_int, l, u, P.feas_tol))
        __hip_atomic_store(&Bt.infeasible[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Unpacks nodes [k0, k0 + cnt) into node-major arrays (row q = node k0 + q).
__global__ __launch_bounds__(kBlock) void k_unpack_batch(Problem P, Batch Bt,
                                                         double* __restrict__ ulb,
                                                         double* __restrict__ uub, int k0,
                                                         int cnt) {
  const size_t total = (size_t)cnt * P.n;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int q = (int)(i / (size_t)P.n);
    const int k = k0 + q;
    const int v = (int)(i - (size_t)q * P.n);
    const size_t src = (size_t)P.perm[v] * kNodeGroup + (k % kNodeGroup);
    const double2 b = Bt.gA[k / kNodeGroup][src];
    ulb[i] = b.x;
    uub[i] = b.y;
  }
}

// Block-wide count of active nodes after a status update; sets ctrl->done.
__device__ __forceinline__ void batch_set_done(const Problem& P, uint32_t my_active) {
  uint32_t dummy = 0;
  block_sum2(my_active, dummy);
  if (threadIdx.x == 0) {
    P.ctrl->done = my_active == 0 ? 1u : 0u;
    P.ctrl->active_nodes = my_active;
  }
}

// Slot moves of the batch driver's compaction: for move q, node slot
// moves[q].x (active) goes to slot moves[q].y (free): its pairs (A and B
// are equal after a commit) and its per-slot state; the source slot becomes
// inactive.  Sources and destinations are disjoint.
__global__ __launch_bounds__(kBlock) void k_move_batch(Problem P, Batch Bt,
                                                       const int2* __restrict__ moves, int count) {
  const size_t total = (size_t)count * P.n;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int q = (int)(i / (size_t)P.n);
    const size_t j = i - (size_t)q * P.n;
    const int s = moves[q].x, d = moves[q].y;
    const double2 b = Bt.gA[s / kNodeGroup][j * kNodeGroup + (s % kNodeGroup)];
    Bt.gA[d / kNodeGroup][j * kNodeGroup + (d % kNodeGroup)] = b;
    Bt.gB[d / kNodeGroup][j * kNodeGroup + (d % kNodeGroup)] = b;
  }
  // marked batches: a group's stamps do not cover nodes moved into it, so
  // every group processes every row in the next round
  if (Bt.row_mark && blockIdx.x == 0)
    for (int g = threadIdx.x; g < Bt.groups; g += blockDim.x) Bt.gall[g] = 1;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < (size_t)count; q += stride) {
    const int s = moves[q].x, d = moves[q].y;
    Bt.status[d] = Bt.status[s];
    Bt.rounds[d] = Bt.rounds[s];
    Bt.maxr[d] = Bt.maxr[s];
    Bt.tiny[d] = Bt.tiny[s];
    Bt.tiny[s] = 0;
    Bt.changed[d] = 0;
    Bt.infeasible[d] = 0;
    Bt.invalid[d] = 0;
    Bt.active[d] = 1;
    Bt.active[s] = 0;
  }
}

// Unpacks slot pairs[q].x into row pairs[q].y of node-major arrays.
__global__ __launch_bounds__(kBlock) void k_unpack_slots(Problem P, Batch Bt,
                                                         double* __restrict__ ulb,
                                                         double* __restrict__ uub,
                                                         const int2* __restrict__ pairs,
                                                         int count) {
  const size_t total = (size_t)count * P.n;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int q = (int)(i / (size_t)P.n);
    const int v = (int)(i - (size_t)q * P.n);
    const int k = pairs[q].x;
    const size_t src = (size_t)P.perm[v] * kNodeGroup + (k % kNodeGroup);
    const double2 b = Bt.gA[k / kNodeGroup][src];
    const size_t dst = (size_t)pairs[q].y * P.n + v;
    ulb[dst] = b.x;
    uub[dst] = b.y;
  }
}

// One block: round-0 decision for nodes [k0, k0 + cnt); with `whole`, the
// done flag reflects the whole batch, otherwise it is cleared (a node joins
// a running batch).
__global__ __launch_bounds__(kBlock) void k_start_batch(Problem P, Batch Bt, int max_rounds,
                                                        int k0, int cnt, int whole) {
  uint32_t act = 0;
  for (int k = k0 + threadIdx.x; k < k0 + cnt; k += blockDim.x) {
    uint32_t a = 0;
    if (Bt.invalid[k]) {
      Bt.status[k] = kInvalidInput;
    } else if (Bt.infeasible[k] || P.instance_infeasible) {
      Bt.status[k] = kInfeasible;
    } else if (max_rounds == 0) {
      Bt.status[k] = kMaxRounds;
    } else {
      Bt.status[k] = kMaxRounds;
      a = 1;
    }
    Bt.rounds[k] = 0;
    Bt.maxr[k] = max_rounds;
    Bt.active[k] = a;
    if (!a) Bt.tiny[k] = 0;
    Bt.changed[k] = 0;
    Bt.infeasible[k] = 0;
    Bt.invalid[k] = 0;
    if (Bt.live) Bt.live[k] = 1;
    // serving: a slot that joins a running group forces the group's next
    // round over every row (its own first round must see them all)
    if (!whole && a && Bt.row_mark) Bt.gall[k / kNodeGroup] = 1;
    act += a;
  }
  if (whole && Bt.row_mark) {
    // marked batches: round 1 processes every row unless a parent seeds it
    const int groups = (k0 + cnt + kNodeGroup - 1) / kNodeGroup;
    for (int g = threadIdx.x; g < groups; g += blockDim.x) {
      Bt.gall[g] = 1;
      Bt.gcnt[g] = 0;
    }
    if (threadIdx.x == 0) P.ctrl->round = 1;
  }
  if (whole) batch_set_done(P, act);
  else if (threadIdx.x == 0) P.ctrl->done = 0;
}

// ---- bodies shared by the batch kernels and the serving kernels ----------

// One wave: work unit `unit` (long-row segment, then chunk) of group g.
// Marked rounds of a batch: whether group g skips unstamped rows in the
// current round, and the group's stamps.
__device__ __forceinline__ bool group_marked(const Problem& P, const Batch& Bt, int g, int& r,
                                             const int32_t*& marks) {
  if (!Bt.row_mark || Bt.gall[g]) return false;
  r = __hip_atomic_load(&P.ctrl->round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  marks = Bt.row_mark + (size_t)g * P.n_rows;
  return true;
}

// kMarks: kernels whose groups may run marked rounds (the batch driver's,
// and the serving engine's when the server marks); without it the
// registers of the marking paths are not allocated.
template <bool kMarks>
__device__ __forceinline__ void round_unit(const Problem& P, const Batch& Bt, int unit, int g) {
  if (unit >= P.n_segs + P.n_chunks) return;
  const uint32_t mask = group_mask(Bt, g);
  if (!mask) return;
  // with few active nodes, node-parallel lanes would mostly idle: loop over
  // the active nodes with the single-run shape instead
  const bool few = __builtin_popcount(mask) <= kLoopNodes;
  const uint32_t exact = group_exact(Bt, g);
  int r = 0;
  const int32_t* marks = nullptr;
  const bool marked = kMarks && group_marked(P, Bt, g, r, marks);
  if (unit < P.n_segs) {
    if (few)
      seg_phase1<kSrcPairs>(P, unit, Bt.gA[g], kNodeGroup, mask, Bt.partials, Bt.nodes,
                        g * kNodeGroup, marked, r, marks);
    else
      seg_phase1_nodes(P, unit, Bt.gA[g], mask, Bt.partials, Bt.nodes, g * kNodeGroup, marked, r,
                       marks);
  } else {
    if (few)
      chunk_dispatch<kSrcPairs>(P, unit - P.n_segs, Bt.gA[g], Bt.gB[g], kNodeGroup, mask, exact,
                            marked, r, marks);
    else
      chunk_round_nodes(P, P.chunks[unit - P.n_segs], Bt.gA[g], Bt.gB[g], mask, exact, marked, r,
                        marks);
  }
}

// One wave: phase 2 of segment s for node k.  With row states (kRowStates
// and a buffer: the batch driver's), the state of the segment's row comes
// from the row-state kernel; otherwise the wave combines the row's
// partials itself (the serving engine, the allocation-free entry point).
template <bool kMarks, bool kRowStates = false>
__device__ __forceinline__ void long_unit(const Problem& P, const Batch& Bt, int s, int k) {
  if (s >= P.n_segs || !Bt.active[k]) return;
  const int g = k / kNodeGroup;
  int r = 0;
  const int32_t* marks = nullptr;
  const bool marked = kMarks && group_marked(P, Bt, g, r, marks);
  if (kRowStates && Bt.row_state) {
    const SegDesc sd = P.segs[s];
    if (marked && marks[sd.row] != r) return;
    const RowState R = Bt.row_state[(size_t)sd.first * Bt.nodes + k];
    seg_revisit<true, kSrcPairs>(P, s, sd, R, Bt.gA[g], Bt.gB[g], kNodeGroup, k % kNodeGroup,
                                 Bt.partials, Bt.nodes, k);
    return;
  }
  seg_phase2<true>(P, s, Bt.gA[g], Bt.gB[g], kNodeGroup, k % kNodeGroup, Bt.partials, Bt.nodes, k,
                   Bt.tiny[k] != 0, marked, r, marks);
}

// One wave: the state of long row i (first segment long_first[i]) for
// node k, stored at that segment.  A long row of nseg segments has nseg
// phase-2 waves per node; combining its partials once here instead of in
// each of them reads nseg partials per node instead of nseg^2 (and sums an
// uncertain row's exact sums once).  The grid has a wave per (long row,
// node): one per (segment, node) would mostly exit at once, and for 256
// nodes of the 1,000,000 x 500,000 instance (3,038 segments, 595 long
// rows) its dispatch alone took 176 us a launch.
__device__ __forceinline__ void row_state_unit(const Problem& P, const Batch& Bt, int i, int k) {
  if (!Bt.active[k]) return;
  const int s = Bt.long_first[i];
  const SegDesc sd = P.segs[s];
  const int g = k / kNodeGroup;
  int r = 0;
  const int32_t* marks = nullptr;
  if (group_marked(P, Bt, g, r, marks) && marks[sd.row] != r) return;
  const RowState R = seg_row_state(P, sd, Bt.gA[g], kNodeGroup, k % kNodeGroup, Bt.partials,
                                   Bt.nodes, k, Bt.tiny[k] != 0);
  if ((threadIdx.x & (kWave - 1)) == 0) Bt.row_state[(size_t)s * Bt.nodes + k] = R;
}

// The 8 variable bits of a wave's ballot over 8 variables x 8 nodes (lane
// v * 8 + t): bit v set when any node t has its bit set.
__device__ __forceinline__ uint32_t var_bits(uint64_t bits) {
  uint32_t byte = 0;
#pragma unroll
  for (int v = 0; v < 8; ++v) byte |= (uint32_t)(((bits >> (8 * v)) & 0xffull) != 0) << v;
  return byte;
}

// Block bx of nbx over group g's (variable, node) pairs: copy changed pairs
// B -> A, count them and check their domains per node (ch, inf: shared).
__device__ __forceinline__ void commit_part(const Problem& P, const Batch& Bt, int g, uint32_t bx,
                                            uint32_t nbx, uint32_t* ch, uint32_t* inf) {
  if (threadIdx.x < kNodeGroup) {
    ch[threadIdx.x] = 0;
    inf[threadIdx.x] = 0;
  }
  __syncthreads();
  const uint32_t mask = group_mask(Bt, g);
  if (mask) {
    double2* A = Bt.gA[g];
    double2* B = Bt.gB[g];
    // a wave's 64 pairs are 8 variables x 8 nodes: one touch byte
    uint8_t* const touch = touch_of(P, B, kNodeGroup);
    const size_t total = (size_t)P.n * kNodeGroup;
    const size_t stride = (size_t)nbx * blockDim.x;
    for (size_t e = (size_t)bx * blockDim.x + threadIdx.x; e < total; e += stride) {
      const uint32_t t = (uint32_t)(e % kNodeGroup);
      bool chg = false;
      const bool hit = touch[e / kWave] != 0;
      if (hit && (threadIdx.x & (kWave - 1)) == 0) touch[e / kWave] = 0;
      if (hit && ((mask >> t) & 1u)) {
        const double2 a = A[e];
        const double2 b = B[e];
        if (a.x != b.x || a.y != b.y) {
          chg = true;
          A[e] = b;
          atomicAdd(&ch[t], 1u);
          if (tiny_bound(b.x) || tiny_bound(b.y))
            __hip_atomic_store(&Bt.tiny[g * kNodeGroup + t], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          if (domain_empty(P.vtype[e / kNodeGroup] != 0, b.x, b.y, P.feas_tol)) inf[t] = 1;
        }
      }
      if (Bt.chg) {
        // marked rounds: the wave's 64 pairs are 8 variables x 8 nodes;
        // byte e / 64 of the group's bitmap gets one bit per variable
        // changed in any node (each byte has one writer per round)
        const uint32_t byte = var_bits(__ballot(chg));
        if ((threadIdx.x & (kWave - 1)) == 0)
          reinterpret_cast<uint8_t*>(Bt.chg + (size_t)g * ((P.n + kWave - 1) / kWave))[e / kWave] =
              (uint8_t)byte;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kNodeGroup) {
    const int k = g * kNodeGroup + threadIdx.x;
    if (ch[threadIdx.x])
      __hip_atomic_fetch_add(&Bt.changed[k], ch[threadIdx.x], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    if (inf[threadIdx.x])
      __hip_atomic_store(&Bt.infeasible[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Appends slot k's outcome to the step's completion list; a slot that finds
// the list full stays unreported (live) and is reported in a later round.
__device__ __forceinline__ void report_slot(const Batch& Bt, SrvStep* S, int inst, int k) {
  const uint32_t i = atomicAdd(&S->n_done, 1u);
  if (i < (uint32_t)kSrvStepDone) {
    S->done[i].inst = inst;
    S->done[i].slot = k;
    S->done[i].status = Bt.status[k];
    S->done[i].rounds = Bt.rounds[k];
    Bt.live[k] = 0;
  }
}

// One block: status of every active node after the round it just ran (its
// own round count: nodes may have joined at different times).  With a step
// (serving), finished slots are reported, including slots that finished at
// their start and slots a full list left unreported.
__device__ __forceinline__ void end_slots(const Problem& P, const Batch& Bt, SrvStep* S,
                                          int inst) {
  uint32_t act = 0;
  for (int k = threadIdx.x; k < Bt.nodes; k += blockDim.x) {
    if (!Bt.active[k]) {
      if (S && Bt.live[k]) report_slot(Bt, S, inst, k);
      continue;
    }
    const int r = Bt.rounds[k] + 1;
    const int max_rounds = Bt.maxr[k];
    uint32_t a = 0;
    Bt.rounds[k] = r;
    if (Bt.infeasible[k]) {
      Bt.status[k] = kInfeasible;
    } else if (Bt.changed[k] == 0) {
      Bt.status[k] = kConverged;
    } else if (r >= max_rounds) {
      Bt.status[k] = kMaxRounds;
    } else {
      a = 1;
    }
    Bt.active[k] = a;
    Bt.changed[k] = 0;
    Bt.infeasible[k] = 0;
    if (!a) Bt.tiny[k] = 0;
    act += a;
    if (S && !a) report_slot(Bt, S, inst, k);
  }
  batch_set_done(P, act);
}

// ---- batch kernels (one problem) ------------------------------------------
// Waves are numbered group-major: the waves in flight at any time work on
// one or two groups, whose bound lines (128 bytes per variable, 64 MB for
// 500,000 variables) then stay in the caches while the matrix streams past,
// once per group.  Numbered unit-major, every group's lines would be in use
// at once and each gather would go to HBM.
// Four waves per SIMD (at most 128 VGPRs): the node-parallel lanes are
// VALU-bound and need the resident waves to hide their gathers; left
// unconstrained the compiler takes 148 VGPRs (three waves), and 256 nodes
// of the 1,000,000 x 500,000 instance take 490 ms instead of 438.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_round_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const int64_t units = (int64_t)P.n_segs + P.n_chunks;
  if (units == 0) return;
  const int g = (int)(wid / units);
  if (g >= Bt.groups) return;
  round_unit<true>(P, Bt, (int)(wid - (int64_t)g * units), g);
}

// Row states: one wave per (long row, node).
__global__ __launch_bounds__(kBlock) void k_row_state_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  if (Bt.n_long == 0) return;
  const int k = (int)(wid / Bt.n_long);
  if (k >= Bt.nodes) return;
  row_state_unit(P, Bt, (int)(wid - (int64_t)k * Bt.n_long), k);
}

__global__ __launch_bounds__(kBlock) void k_round_long_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  if (P.n_segs == 0) return;
  const int k = (int)(wid / P.n_segs);
  if (k >= Bt.nodes) return;
  long_unit<true, true>(P, Bt, (int)(wid - (int64_t)k * P.n_segs), k);
}

// Commit per (variable, node) of group blockIdx.y, with per-node counts.
__global__ __launch_bounds__(kBlock) void k_commit_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  __shared__ uint32_t ch[kNodeGroup], inf[kNodeGroup];
  commit_part(P, Bt, blockIdx.y, blockIdx.x, gridDim.x, ch, inf);
}

__global__ __launch_bounds__(kBlock) void k_end_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  if (Bt.row_mark && threadIdx.x == 0) P.ctrl->round = P.ctrl->round + 1;
  end_slots(P, Bt, nullptr, 0);
}

// Marked batches, after the commit of the current round (offset 1) or after
// the parent seeding (offset 0): for every group with active nodes, stamps
// the rows of its changed variables with the round they are processed in,
// one thread per piece of <= kMarkPiece rows of a variable (blockIdx.y is
// the group).  A group that changed more than n / kMarkAllDiv variables
// processes every row instead (stamping them would cost more).
__device__ __forceinline__ void mark_group(const Problem& P, const Batch& Bt, int g, uint32_t bx,
                                           uint32_t nbx, int offset) {
  if (!group_mask(Bt, g)) return;
  uint32_t count = 0;
  if (offset == 0) {
    count = Bt.gcnt[g];
  } else {
#pragma unroll
    for (int t = 0; t < kNodeGroup; ++t) {
      const int k = g * kNodeGroup + t;
      if (k < Bt.nodes && Bt.active[k]) count += Bt.changed[k];
    }
  }
  const bool all = count > (uint32_t)(P.n / kMarkAllDiv);
  if (bx == 0 && threadIdx.x == 0) Bt.gall[g] = all ? 1u : 0u;
  if (all) return;
  const int next = __hip_atomic_load(&P.ctrl->round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) +
                   offset;
  const uint64_t* bits = Bt.chg + (size_t)g * ((P.n + kWave - 1) / kWave);
  int32_t* marks = Bt.row_mark + (size_t)g * P.n_rows;
  const int64_t stride = (int64_t)nbx * blockDim.x;
  for (int64_t q = (int64_t)bx * blockDim.x + threadIdx.x; q < P.n_pieces; q += stride) {
    const int32_t v = P.piece_var[q];
    if (!((bits[v / kWave] >> (v % kWave)) & 1ull)) continue;
    const int64_t start = P.piece_off[q];
    const int64_t stop = P.var_ptr[v + 1] < start + kMarkPiece ? P.var_ptr[v + 1] : start + kMarkPiece;
    for (int64_t i = start; i < stop; ++i) marks[P.var_rows[i]] = next;
  }
}

__global__ __launch_bounds__(kBlock) void k_mark_batch(Problem P, Batch Bt, int offset) {
  if (u32_load(&P.ctrl->done)) return;
  mark_group(P, Bt, blockIdx.y, blockIdx.x, gridDim.x, offset);
}

// Marked batches from a parent fixed point: bit v of group g's bitmap is set
// when variable v's start bounds differ from the parent's in any active node
// of the group; gcnt counts those variables.  Round 1 then processes only
// the rows of those variables (k_mark_batch, offset 0).
__global__ __launch_bounds__(kBlock) void k_seed_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  const int g = blockIdx.y;
  const uint32_t mask = group_mask(Bt, g);
  if (!mask) return;
  const double2* A = Bt.gA[g];
  uint8_t* bytes = reinterpret_cast<uint8_t*>(Bt.chg + (size_t)g * ((P.n + kWave - 1) / kWave));
  const size_t total = (size_t)P.n * kNodeGroup;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  uint32_t count = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const uint32_t t = (uint32_t)(e % kNodeGroup);
    bool diff = false;
    if ((mask >> t) & 1u) {
      const double2 a = A[e];
      const double2 b = P.parent[e / kNodeGroup];
      diff = a.x != b.x || a.y != b.y;
    }
    const uint32_t byte = var_bits(__ballot(diff));
    if ((threadIdx.x & (kWave - 1)) == 0) {
      bytes[e / kWave] = (uint8_t)byte;
      count += __builtin_popcount(byte);
    }
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && count)
    __hip_atomic_fetch_add(&Bt.gcnt[g], count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- serving kernels: every instance of a step in one launch per phase -----

// Entry of the step holding work item x of a phase (0 round waves, 1
// long-row waves, 2 commit blocks): the last entry whose first item is <= x.
__device__ __forceinline__ int step_entry(const SrvStep* S, int64_t x, int which) {
  int lo = 0, hi = S->n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const SrvEntry& E = S->e[mid];
    const int64_t base = which == 0   ? E.round_base
                         : which == 1 ? E.long_base
                         : which == 2 ? E.commit_base
                                      : E.mark_base;
    if (base <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ Batch step_batch(const SrvInst* I, const SrvEntry& E) {
  Batch Bt = I[E.inst].bt;
  Bt.groups = E.groups;
  Bt.nodes = E.groups * kNodeGroup;
  return Bt;
}

template <bool kMarks>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_srv_round(
    const SrvInst* __restrict__ I, const SrvStep* __restrict__ S) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  if (wid >= S->round_total) return;
  const SrvEntry E = S->e[step_entry(S, wid, 0)];
  const Problem P = I[E.inst].P;
  if (u32_load(&P.ctrl->done)) return;
  const Batch Bt = step_batch(I, E);
  // group-major within the instance, as in k_round_batch
  const int64_t local = wid - E.round_base;
  const int64_t units = (int64_t)P.n_segs + P.n_chunks;
  if (units == 0) return;
  const int g = (int)(local / units);
  round_unit<kMarks>(P, Bt, (int)(local - (int64_t)g * units), g);
}

template <bool kMarks>
__global__ __launch_bounds__(kBlock) void k_srv_long(const SrvInst* __restrict__ I,
                                                     const SrvStep* __restrict__ S) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  if (wid >= S->long_total) return;
  const SrvEntry E = S->e[step_entry(S, wid, 1)];
  const Problem P = I[E.inst].P;
  if (u32_load(&P.ctrl->done)) return;
  const Batch Bt = step_batch(I, E);
  const int64_t local = wid - E.long_base;
  if (P.n_segs == 0) return;
  const int k = (int)(local / P.n_segs);
  long_unit<kMarks>(P, Bt, (int)(local - (int64_t)k * P.n_segs), k);
}

__global__ __launch_bounds__(kBlock) void k_srv_commit(const SrvInst* __restrict__ I,
                                                       const SrvStep* __restrict__ S) {
  __shared__ uint32_t ch[kNodeGroup], inf[kNodeGroup];
  if ((int64_t)blockIdx.x >= S->commit_total) return;
  const SrvEntry E = S->e[step_entry(S, blockIdx.x, 2)];
  const Problem P = I[E.inst].P;
  if (u32_load(&P.ctrl->done)) return;
  const Batch Bt = step_batch(I, E);
  const int local = (int)((int64_t)blockIdx.x - E.commit_base);
  const int g = local / E.commit_blocks;
  commit_part(P, Bt, g, local - g * E.commit_blocks, E.commit_blocks, ch, inf);
}

// Marked rounds of the instances that mark, after the commit: stamps the
// rows of each group's changed variables with the next round (mark_group).
__global__ __launch_bounds__(kBlock) void k_srv_mark(const SrvInst* __restrict__ I,
                                                     const SrvStep* __restrict__ S) {
  if ((int64_t)blockIdx.x >= S->mark_total) return;
  const SrvEntry E = S->e[step_entry(S, blockIdx.x, 3)];
  if (E.mark_blocks == 0) return;
  const Problem P = I[E.inst].P;
  if (u32_load(&P.ctrl->done)) return;
  const Batch Bt = step_batch(I, E);
  const int local = (int)((int64_t)blockIdx.x - E.mark_base);
  const int g = local / E.mark_blocks;
  if (g >= E.groups) return;
  mark_group(P, Bt, g, local - g * E.mark_blocks, E.mark_blocks, 1);
}

// One block per entry.  No early exit on the done flag: slots finished at
// their start, or left unreported by a full list, are reported here.  A
// marking instance counts its rounds in its control block (the stamps of
// the mark kernel name the next one).
__global__ __launch_bounds__(kBlock) void k_srv_end(const SrvInst* __restrict__ I,
                                                    SrvStep* __restrict__ S) {
  if ((int)blockIdx.x >= S->n) return;
  const SrvEntry E = S->e[blockIdx.x];
  const Problem P = I[E.inst].P;
  const Batch Bt = step_batch(I, E);
  if (Bt.row_mark && threadIdx.x == 0) P.ctrl->round = P.ctrl->round + 1;
  end_slots(P, Bt, S, E.inst);
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------
hipError_t launch_pack_batch(const Problem& P, const Batch& Bt, const double* lb, const double* ub,
                             int k0, int cnt, hipStream_t s) {
  const int64_t groups = (k0 + cnt - 1) / kNodeGroup - k0 / kNodeGroup + 1;
  hipLaunchKernelGGL(k_pack_batch, dim3(blocks_for(groups * P.n, kBlock, 16384)),
                     dim3(kBlock), 0, s, P, Bt, lb, ub, k0, cnt);
  return hipGetLastError();
}

hipError_t launch_unpack_batch(const Problem& P, const Batch& Bt, double* lb, double* ub, int k0,
                               int cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_batch, dim3(blocks_for((int64_t)cnt * P.n, kBlock, 16384)),
                     dim3(kBlock), 0, s, P, Bt, lb, ub, k0, cnt);
  return hipGetLastError();
}

hipError_t launch_start_batch(const Problem& P, const Batch& Bt, int max_rounds, int k0, int cnt,
                              bool whole, hipStream_t s) {
  hipLaunchKernelGGL(k_start_batch, dim3(1), dim3(kBlock), 0, s, P, Bt, max_rounds, k0, cnt,
                     whole ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_round_batch(const Problem& P, const Batch& Bt, hipStream_t s) {
  const int64_t waves = (int64_t)(P.n_chunks + P.n_segs) * Bt.groups;
  hipLaunchKernelGGL(k_round_batch, dim3(blocks_for(waves, kWavesPerBlock, 1 << 30)),
                     dim3(kBlock), 0, s, P, Bt);
  if (P.n_segs && Bt.row_state)
    hipLaunchKernelGGL(k_row_state_batch,
                       dim3(blocks_for((int64_t)Bt.n_long * Bt.nodes, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P, Bt);
  if (P.n_segs)
    hipLaunchKernelGGL(k_round_long_batch,
                       dim3(blocks_for((int64_t)P.n_segs * Bt.nodes, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P, Bt);
  hipLaunchKernelGGL(k_commit_batch,
                     dim3(blocks_for((int64_t)P.n * kNodeGroup, kBlock, 256), Bt.groups),
                     dim3(kBlock), 0, s, P, Bt);
  if (Bt.row_mark)
    hipLaunchKernelGGL(k_mark_batch, dim3(blocks_for(P.n_pieces, kBlock, 1024), Bt.groups),
                       dim3(kBlock), 0, s, P, Bt, 1);
  hipLaunchKernelGGL(k_end_batch, dim3(1), dim3(kBlock), 0, s, P, Bt);
  return hipGetLastError();
}

hipError_t launch_seed_batch(const Problem& P, const Batch& Bt, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_batch,
                     dim3(blocks_for((int64_t)P.n * kNodeGroup, kBlock, 256), Bt.groups),
                     dim3(kBlock), 0, s, P, Bt);
  hipLaunchKernelGGL(k_mark_batch, dim3(blocks_for(P.n_pieces, kBlock, 1024), Bt.groups),
                     dim3(kBlock), 0, s, P, Bt, 0);
  return hipGetLastError();
}

hipError_t launch_move_batch(const Problem& P, const Batch& Bt, const int2* moves, int count,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_move_batch,
                     dim3(blocks_for((int64_t)count * (P.n > 1 ? P.n : 1), kBlock, 4096)),
                     dim3(kBlock), 0, s, P, Bt, moves, count);
  return hipGetLastError();
}

hipError_t launch_unpack_slots(const Problem& P, const Batch& Bt, double* lb, double* ub,
                               const int2* pairs, int count, hipStream_t s) {
  if (count <= 0 || P.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_slots, dim3(blocks_for((int64_t)count * P.n, kBlock, 4096)),
                     dim3(kBlock), 0, s, P, Bt, lb, ub, pairs, count);
  return hipGetLastError();
}

hipError_t launch_srv_round(const SrvInst* I, SrvStep* S, const SrvStep& H, hipStream_t s) {
  if (H.n == 0) return hipSuccess;
  const dim3 rgrid(blocks_for(H.round_total, kWavesPerBlock, 1 << 30));
  if (H.mark_total) hipLaunchKernelGGL(k_srv_round<true>, rgrid, dim3(kBlock), 0, s, I, S);
  else hipLaunchKernelGGL(k_srv_round<false>, rgrid, dim3(kBlock), 0, s, I, S);
  if (H.long_total) {
    const dim3 lgrid(blocks_for(H.long_total, kWavesPerBlock, 1 << 30));
    if (H.mark_total) hipLaunchKernelGGL(k_srv_long<true>, lgrid, dim3(kBlock), 0, s, I, S);
    else hipLaunchKernelGGL(k_srv_long<false>, lgrid, dim3(kBlock), 0, s, I, S);
  }
  hipLaunchKernelGGL(k_srv_commit, dim3(blocks_for(H.commit_total, 1, 1 << 30)), dim3(kBlock), 0,
                     s, I, S);
  if (H.mark_total)
    hipLaunchKernelGGL(k_srv_mark, dim3(blocks_for(H.mark_total, 1, 1 << 30)), dim3(kBlock), 0,
                       s, I, S);
  hipLaunchKernelGGL(k_srv_end, dim3(H.n), dim3(kBlock), 0, s, I, S);
  return hipGetLastError();
}

}  // namespace prop
