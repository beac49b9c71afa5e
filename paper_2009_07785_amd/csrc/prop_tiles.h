// prop_tiles.h -- the matrix tiles and constants of the device layout,
// free of HIP types so that the host layout builder also compiles (and
// runs under the sanitizers) without the HIP toolchain.
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

// The nnz-split layout (merge-path style load balancing; an alternative to
// the length-class chunks, chosen at create).  Rows in input order are
// packed into waves of at most kNzEntries entries and kNzMaxRows rows, with
// no sorting by length; rows longer than kNzEntries go to segments.  Lane l
// of a wave owns the wave's entries l * kNzSteps .. l * kNzSteps + 7 in CSR
// order, stored step-major (entry k of lane l at k * 64 + l) so that every
// step is one contiguous load; a flag byte per lane marks the entries that
// start a row.  Rows may span lanes: a segmented scan over the lanes joins
// their pieces.
constexpr int kNzSteps = 8;
constexpr int kNzEntries = kWave * kNzSteps;
constexpr int kNzMaxRows = 256;

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
  double emin, emax;       // error bounds of the two double-doubles (prop_sum.h)
};

}  // namespace prop
