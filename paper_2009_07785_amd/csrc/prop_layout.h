// prop_layout.h -- device data layout shared by the host runtime and the
// gfx950 kernels of the propagation library: the control block, the
// problem and batch descriptors the kernels take by value, and the serving
// step tables.  The matrix tiles (chunks, long-row segments) and the
// layout constants are in prop_tiles.h.
#pragma once

#include <stdint.h>

#include "prop_tiles.h"

namespace prop {

// The commit kernel's blocks report their totals in two levels: into one of
// kCommitGroups group words (kCommitGroup blocks each, one 128-byte line
// apart), and the last block of a group into Ctrl::commit_word, so that no
// word sees more than 32 returning atomics per round.
constexpr int kCommitGroup = 32;
constexpr int kCommitGroups = 32;
constexpr int kCommitMaxBlocks = kCommitGroup * kCommitGroups;
constexpr int kGroupWordStride = 16;  // uint64 words per group word's line

// Device control block of one problem.
struct Ctrl {
  uint64_t commit_word;    // packed per-round commit totals (see the kernels)
  uint32_t infeasible;     // set when an input domain is empty
  uint32_t invalid;        // set when a bound fails validation
  int32_t status;
  int32_t rounds;
  uint32_t done;           // loop finished
  int32_t round;           // next round to run
  uint32_t tiny;           // a bound of this run has 0 < |b| < 2^-906 (exact sums for every row)
  uint32_t bar_gen;        // grid barrier generation
  uint32_t abort;          // barrier wait gave up (device timeout)
  uint32_t mark_all;       // marked rounds: the next round processes every row
  int32_t max_rounds;      // round limit of the current run
  uint32_t active_nodes;   // batches: nodes still active after the last round
  uint32_t pad[2];
};

// Everything a kernel needs, passed by value.
struct Problem {
  // matrix
  const double* vals;
  const int32_t* cols;
  const ChunkDesc* chunks;
  const SegDesc* segs;
  SegPartial* partials;
  const double* lhs;        // internal row order
  const double* rhs;
  const uint8_t* vtype;     // internal variable order
  const int32_t* perm;      // perm[user var] = internal var
  int32_t n_chunks;         // chunks, or nnz-split waves (nnz_split != 0)
  int32_t n_segs;
  int32_t n;
  int32_t instance_infeasible;
  int32_t nnz_split;        // the layout is nnz-split (prop_tiles.h)
  int32_t pad_nz;
  const uint8_t* wave_flags; // nnz-split: [n_chunks][64] row starts per lane
  // state: bnd[0] = start-of-round bounds, bnd[1] = candidate target
  // (followed by its touch bytes, see touch_bytes)
  double2* bnd[2];
  uint16_t* codes;          // [n] compact code of bnd[0] per variable (prop_device.h)
  // single-precision store (store32 != 0): every bound is kept on the grid
  // of zero, the infinities and the normal singles, rounded outward, and
  // b32 holds bnd[0] as singles (the same values) for the gathers
  float2* b32;              // [n]
  int32_t store32;
  double2* stripes;         // [kStripes][n_hot] candidate targets of hot variables
  int32_t n_hot;
  int32_t pad_hot;
  Ctrl* ctrl;
  uint64_t* commit_grp;     // [kCommitGroups * kGroupWordStride] commit group words
  // parameters
  double eps_int, cont_rel_tol, feas_tol;
  // marked rounds (marking != 0): a row is processed in round r only when
  // row_mark[row] == r, i.e. one of its variables changed in round r - 1
  int32_t marking;
  int32_t n_rows;           // rows of the internal order (chunk rows, then long rows)
  int32_t* row_mark;        // [n_rows]
  const int64_t* var_ptr;   // [n + 1] rows of each variable, internal orders
  const int32_t* var_rows;
  uint64_t* chg_bits;       // [ceil(n / 64)] variables changed in the current round
  const int32_t* piece_var; // [n_pieces] variable of each piece of <= kMarkPiece rows
  const int64_t* piece_off; // [n_pieces] first entry of the piece in var_rows
  int64_t n_pieces;
  // marked runs from a parent: the parent's bounds (a fixed point of this
  // problem's propagation, integer-rounded, internal order), else null
  const double2* parent;    // [n]
};

// Rows of a variable that one thread of the mark kernel stamps; a round
// that changed more than n / kMarkAllDiv variables runs the next round over
// every row instead.
constexpr int kMarkPiece = 64;
constexpr int kMarkAllDiv = 32;

// Touch bytes.  Every block of candidate targets (a single run's bnd[1],
// n pairs; a batch group's B, n x 8 pairs) is followed by touch_bytes(n)
// bytes: byte i is set when a candidate was written for one of variables
// 8i .. 8i + 7 (in any node of the block) in the current round, and the
// commit reads only the pairs of touched variables and clears the bytes.
// A byte set with nothing written costs a compare; every write sets its
// byte before the commit runs, so none is missed.  A block holds
// max(n, 1) x nodes pairs; the size keeps 64-variable words whole and
// the next block 256-byte aligned.
inline __host__ __device__ size_t touch_bytes(int32_t n) {
  const size_t words = ((size_t)(n > 0 ? n : 1) + 63) / 64;
  return (words * 8 + 255) / 256 * 256;
}

// Batch of branch-and-bound nodes sharing one problem.  Bounds of node
// k = 8 g + t for variable j sit at A[(g * n + j) * 8 + t]: the 8 nodes of a
// group share each variable's 128-byte line.
constexpr int kNodeGroup = 8;
// a group with at most this many active nodes runs them one after another
constexpr int kLoopNodes = 2;

// State of a long row for one node after its segments' partials are
// combined (prop_device.h); batches keep one per (first segment, node).
struct RowState;
constexpr int kRowStateBytes = 48;

// Node slots in groups of kNodeGroup; each group's bound pairs live in their
// own [n][8] block so that groups can be allocated and released one by one.
struct Batch {
  double2* const* gA;      // [groups] -> start-of-round bounds of the group, [n][8]
  double2* const* gB;      // [groups] -> candidate targets, same layout
  SegPartial* partials;    // [segments][nodes]
  // [segments][nodes] long-row states, filled at a row's first segment by
  // a kernel of its own so that a row's partials are combined once per node
  // (null: every segment combines them itself, as single runs do)
  RowState* row_state;
  const int32_t* long_first;  // [n_long] first segment of each long row (with row_state)
  int32_t n_long;
  uint32_t* active;        // [nodes] still propagating
  int32_t* status;         // [nodes]
  int32_t* rounds;         // [nodes]
  uint32_t* changed;       // [nodes] pairs changed in the current round
  uint32_t* infeasible;    // [nodes] empty domain seen
  uint32_t* invalid;       // [nodes] bound failed validation (cleared by the start kernel)
  int32_t* maxr;           // [nodes] round limit of each node
  uint32_t* live;          // [nodes] serving only (else null): finished, not yet reported
  uint32_t* tiny;          // [nodes] a bound of the node's run has 0 < |b| < 2^-906
  // marked rounds of batches (null when off): a group processes a row in
  // round r only when row_mark[g * n_rows + row] == r, unless gall[g] is set
  int32_t* row_mark;       // [groups][n_rows]
  uint64_t* chg;           // [groups][ceil(n / 64)] variables changed in any node of the group
  uint32_t* gall;          // [groups] the group's next round processes every row
  uint32_t* gcnt;          // [groups] variables that differ from the parent (seeded runs)
  int32_t nodes;
  int32_t groups;
};

// ---------------------------------------------------------------------------
// Serving: one launch per phase covers every instance with running slots.
// ---------------------------------------------------------------------------
struct SrvInst {           // per instance, device resident
  Problem P;               // matrix of the instance, control block of the server's
  Batch bt;                // slot state (nodes / groups are set per step)
};

struct SrvDone {           // a slot whose request finished
  int32_t inst, slot, status, rounds;
};

struct SrvEntry {          // an instance in a step, with the first work item of each phase
  int32_t inst, groups;
  int64_t round_base;      // waves of the round kernel
  int64_t long_base;       // waves of the long-row kernel
  int64_t commit_base;     // blocks of the commit kernel
  int64_t mark_base;       // blocks of the mark kernel (marked rounds)
  int32_t commit_blocks;   // commit blocks per group
  int32_t mark_blocks;     // mark blocks per group, 0 when the instance is unmarked
};

constexpr int kSrvStepDone = 512;     // completions a step can report (more wait a round)
constexpr int kSrvMaxInstances = 256;

struct SrvStep {
  int32_t n;               // entries
  uint32_t n_done;         // completions reported (may exceed kSrvStepDone)
  int64_t round_total, long_total, commit_total, mark_total;
  SrvDone done[kSrvStepDone];
  SrvEntry e[kSrvMaxInstances];
};

}  // namespace prop
