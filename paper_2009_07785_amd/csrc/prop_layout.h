// prop_layout.h -- device data layout shared by the host runtime and the
// gfx950 kernels of the propagation library.
//
// Matrix layout ("chunks").  Rows are grouped by length.  A row of L <= 1024
// entries gets K = 1, 2, 4, ..., 64 lanes of a 64-lane wave, the smallest K
// with ceil(L / K) <= 16; a chunk is one wave's tile of 64 / K rows of the
// same K.  Inside a chunk, entry p of row r sits at lane r * K + p % K and
// step p / K, stored at offset step * 64 + lane: every step is one
// contiguous 64-entry load of values (512 B) and columns (256 B).  W, the
// chunk's number of steps, is the largest ceil(L / K) of its rows; shorter
// rows are padded with zero coefficients.  Rows are sorted by length inside
// each K class so the padding stays small.
//
// Rows with more than 1024 entries are "long": their entries stay in CSR
// order, split into segments of 1024 (one wave, 16 steps), and a round
// handles them in two phases (partial sums per segment, then candidates per
// segment once all partial sums of the row exist).
//
// Variables are relabelled by decreasing column degree so the bounds of
// the most used variables share cache lines.  Bounds live as (lb, ub)
// pairs, one 16-byte load per entry, in two arrays: the start-of-round
// bounds (read only during a round) and the candidate target (atomic max /
// min), reconciled by a commit pass at the end of every round.
#pragma once

#include <stdint.h>

namespace prop {

constexpr int kWave = 64;        // lanes per wavefront on gfx950
constexpr int kMaxSteps = 16;    // steps per wave tile
constexpr int kSegLen = kWave * kMaxSteps;  // entries per long-row segment
constexpr int kBlock = 256;      // threads per workgroup (4 waves)
constexpr int kWavesPerBlock = kBlock / kWave;

// A stored column word holds the (relabelled) variable in bits 0-30 and
// the variable's integrality in bit 31.
constexpr int32_t kColMask = 0x7fffffff;

// Candidates for the most used variables (relabelled to 0 .. n_hot-1) go
// to kStripes copies of their bound pairs, copy = block index mod kStripes,
// instead of one shared pair; the commit merges the copies.  Rows of a
// power-law matrix send tens of thousands of candidates to one such
// variable in a round, and same-address atomics serialise.
constexpr int kStripes = 64;
constexpr int kMaxHot = 8192;
constexpr int kHotDegree = 512;

// run outcome codes (match PROP_CONVERGED / PROP_INFEASIBLE / PROP_MAX_ROUNDS)
constexpr int kConverged = 0;
constexpr int kInfeasible = 1;
constexpr int kMaxRounds = 2;
constexpr int kInvalidInput = -1;  // batch node status: an input bound failed validation

// One chunk of short/medium rows.
struct ChunkDesc {
  int32_t off64;   // data offset in units of 64 entries
  int32_t row0;    // first (internal) row of the chunk
  int32_t meta;    // bits 0-2: log2 K, bits 8-15: W, bits 16-23: rows in chunk
  int32_t pad;
};

// One segment of a long row.
struct SegDesc {
  int64_t off;     // data offset (entries) of the segment
  int32_t row;     // internal row index (lhs / rhs)
  int32_t len;     // entries in the segment (<= kSegLen)
  int32_t first;   // index of the row's first segment
  int32_t nseg;    // segments of the row
  int32_t pad0, pad1;
};

// Per-segment partial sums of a long row, written in phase 1 of a round.
struct SegPartial {
  double min_hi, min_lo;   // double-double finite part of the min activity
  double max_hi, max_lo;   // same for the max activity
  double tmin, tmax;       // largest per-side skip threshold of the segment's entries
  int32_t min_inf, max_inf;
  double err;              // error bound of both double-doubles (prop_sum.h)
};

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
  int32_t n_chunks;
  int32_t n_segs;
  int32_t n;
  int32_t instance_infeasible;
  // state: bnd[0] = start-of-round bounds, bnd[1] = candidate target
  double2* bnd[2];
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
};

// Rows of a variable that one thread of the mark kernel stamps; a round
// that changed more than n / kMarkAllDiv variables runs the next round over
// every row instead.
constexpr int kMarkPiece = 64;
constexpr int kMarkAllDiv = 32;

// Batch of branch-and-bound nodes sharing one problem.  Bounds of node
// k = 8 g + t for variable j sit at A[(g * n + j) * 8 + t]: the 8 nodes of a
// group share each variable's 128-byte line.
constexpr int kNodeGroup = 8;
// a group with at most this many active nodes runs them one after another
constexpr int kLoopNodes = 2;

// Node slots in groups of kNodeGroup; each group's bound pairs live in their
// own [n][8] block so that groups can be allocated and released one by one.
struct Batch {
  double2* const* gA;      // [groups] -> start-of-round bounds of the group, [n][8]
  double2* const* gB;      // [groups] -> candidate targets, same layout
  SegPartial* partials;    // [segments][nodes]
  uint32_t* active;        // [nodes] still propagating
  int32_t* status;         // [nodes]
  int32_t* rounds;         // [nodes]
  uint32_t* changed;       // [nodes] pairs changed in the current round
  uint32_t* infeasible;    // [nodes] empty domain seen
  uint32_t* invalid;       // [nodes] bound failed validation (cleared by the start kernel)
  int32_t* maxr;           // [nodes] round limit of each node
  uint32_t* live;          // [nodes] serving only (else null): finished, not yet reported
  uint32_t* tiny;          // [nodes] a bound of the node's run has 0 < |b| < 2^-906
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
  int32_t commit_blocks;   // commit blocks per group
  int32_t pad;
};

constexpr int kSrvStepDone = 512;     // completions a step can report (more wait a round)
constexpr int kSrvMaxInstances = 256;

struct SrvStep {
  int32_t n;               // entries
  uint32_t n_done;         // completions reported (may exceed kSrvStepDone)
  int64_t round_total, long_total, commit_total;
  SrvDone done[kSrvStepDone];
  SrvEntry e[kSrvMaxInstances];
};

}  // namespace prop
