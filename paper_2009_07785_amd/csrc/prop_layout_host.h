// prop_layout_host.h -- the host side of the device layout: from a CSR
// matrix to the chunk / segment tiles, the variable relabelling, the row
// order and the rows of every variable (prop_tiles.h describes the layout).
// Plain C++ with no HIP types: prop_create uploads what it builds, and the
// CPU tests run it under the address and undefined-behaviour sanitizers.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "prop.h"
#include "prop_tiles.h"

namespace prop {

struct HostLayout {
  int64_t nnz = 0;                 // nonzero coefficients (explicit zeros dropped)
  int64_t stored = 0;              // stored entries (chunk padding, long rows to 64)
  int64_t chunk_entries = 0;       // entries of the chunk region (long rows follow)
  bool instance_infeasible = false;
  std::vector<int32_t> perm;       // perm[user var] = internal var
  std::vector<uint8_t> vtype;      // per internal var
  std::vector<double> vals;        // [stored]
  std::vector<int32_t> cols;       // [stored] column words
  std::vector<ChunkDesc> chunks;   // chunks, or the waves of the nnz-split layout
  std::vector<uint8_t> wave_flags; // nnz-split: [chunks][64] row starts per lane (bit = step)
  std::vector<SegDesc> segs;
  std::vector<double> lhs, rhs;    // internal row order (chunk rows, then long rows)
  int32_t n_rows = 0;              // internal rows
  int32_t n_long_rows = 0;
  int32_t n_hot = 0;               // leading internal vars with degree >= kHotDegree
  std::vector<int64_t> var_ptr;    // [n + 1] rows of each internal var ...
  std::vector<int32_t> var_rows;   // ... in internal row numbers
};

// Builds the layout of a validated matrix with `steps` entries per lane of a
// short row (4, 8 or 16).  Returns false with a message when an internal
// consistency check fails or the matrix does not fit the layout.
// kind 1 builds the nnz-split layout instead (prop_tiles.h; `steps` then
// only matters for the chunk consistency checks).
bool layout_build(const prop_csr* A, const double* lhs, const double* rhs,
                  const uint8_t* vartype, int steps, HostLayout* out, std::string* err,
                  int kind = 0);

}  // namespace prop
