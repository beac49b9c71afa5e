// prop_layout_host.cpp -- builds the device layout of prop_tiles.h on the
// host (see prop_layout_host.h).
#include "prop_layout_host.h"

#include <algorithm>
#include <numeric>

namespace prop {

namespace {

int ceil_log2(int64_t x) {
  int k = 0;
  while ((int64_t(1) << k) < x) ++k;
  return k;
}

}  // namespace

bool layout_build(const prop_csr* A, const double* lhs, const double* rhs,
                  const uint8_t* vartype, int steps, HostLayout* out, std::string* err) {
  const int32_t m = A->m, n = A->n;
  // nonzero entries per row and per column
  std::vector<int64_t> len(m, 0);
  std::vector<int64_t> deg(n, 0);
  int64_t nnz = 0;
  for (int32_t i = 0; i < m; ++i)
    for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
      if (A->vals[k] != 0.0) {
        ++len[i];
        ++deg[A->col_idx[k]];
        ++nnz;
      }
  out->nnz = nnz;
  bool infeasible = false;
  for (int32_t i = 0; i < m && !infeasible; ++i) {
    if (lhs[i] > rhs[i]) infeasible = true;
    if (len[i] == 0 && (lhs[i] > 0.0 || rhs[i] < 0.0)) infeasible = true;
  }
  out->instance_infeasible = infeasible;

  // Relabelling: the hot variables (degree >= kHotDegree, at most kMaxHot,
  // the most used first), then the other integer variables, then the other
  // continuous ones, each part by decreasing degree.  The activity pass
  // gathers the 2-byte bound codes of integer variables and the 16-byte
  // pairs of continuous ones, so keeping each class contiguous keeps each
  // gathered array dense.
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
  int32_t n_hot = 0;
  while (n_hot < n && n_hot < kMaxHot && deg[order[n_hot]] >= kHotDegree) ++n_hot;
  std::stable_partition(order.begin() + n_hot, order.end(),
                        [&](int32_t j) { return vartype[j] != 0; });
  std::vector<int32_t> perm(n);
  for (int32_t q = 0; q < n; ++q) perm[order[q]] = q;
  std::vector<uint8_t> vtype(n);
  for (int32_t j = 0; j < n; ++j) vtype[perm[j]] = vartype[j];
  auto col_word = [&](int32_t j) {
    return (int32_t)((uint32_t)perm[j] | (vartype[j] ? 0x80000000u : 0u));
  };

  // rows by lanes-per-row class; long rows apart
  std::vector<std::vector<int32_t>> cls(7);
  std::vector<int32_t> longs;
  for (int32_t i = 0; i < m; ++i) {
    if (len[i] == 0) continue;
    // rows of at most 64 lanes x `steps` entries go to chunks, longer ones
    // to 1024-entry segments
    if (len[i] > (int64_t)kWave * steps) {
      longs.push_back(i);
      continue;
    }
    const int64_t lanes = (len[i] + steps - 1) / steps;
    cls[ceil_log2(lanes)].push_back(i);
  }
  struct Chunk {
    int klog, W, nrows;
    size_t first;  // index into the class's sorted row list
  };
  std::vector<Chunk> chunks;
  for (int k = 0; k <= 6; ++k) {
    auto& rows = cls[k];
    std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) { return len[a] > len[b]; });
    const int per = kWave >> k;
    for (size_t q = 0; q < rows.size(); q += per) {
      const int nr = (int)std::min<size_t>(per, rows.size() - q);
      const int W = (int)((len[rows[q]] + (1 << k) - 1) >> k);
      chunks.push_back({k, W, nr, q});
    }
  }
  // heaviest tiles first
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& a, const Chunk& b) {
    return a.W != b.W ? a.W > b.W : a.klog > b.klog;
  });

  int64_t stored = 0;
  for (auto& c : chunks) stored += (int64_t)kWave * c.W;
  const int64_t chunk_entries = stored;
  for (int32_t i : longs) stored += (len[i] + kWave - 1) / kWave * kWave;
  if (chunk_entries / kWave > INT32_MAX) { *err = "matrix too large for the layout"; return false; }
  out->stored = stored;
  out->chunk_entries = chunk_entries;

  std::vector<double> h_vals(stored, 0.0);
  std::vector<int32_t> h_cols(stored, 0);
  std::vector<ChunkDesc> h_chunks;
  h_chunks.reserve(chunks.size());
  std::vector<double> h_lhs, h_rhs;
  h_lhs.reserve(m);
  h_rhs.reserve(m);
  int64_t off = 0;
  int32_t next_row = 0;
  for (auto& c : chunks) {
    const auto& rows = cls[c.klog];
    const int K = 1 << c.klog;
    ChunkDesc d;
    d.off64 = (int32_t)(off / kWave);
    d.row0 = next_row;
    d.meta = c.klog | (c.W << 8) | (c.nrows << 16);
    d.pad = 0;
    h_chunks.push_back(d);
    for (int q = 0; q < c.nrows; ++q) {
      const int32_t i = rows[c.first + q];
      h_lhs.push_back(lhs[i] + 0.0);
      h_rhs.push_back(rhs[i] + 0.0);
      int64_t pos = 0;
      for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
        if (A->vals[k] == 0.0) continue;
        const int64_t lane = (int64_t)q * K + pos % K;
        const int64_t step = pos / K;
        const int64_t idx = off + step * kWave + lane;
        h_vals[idx] = A->vals[k];
        h_cols[idx] = col_word(A->col_idx[k]);
        ++pos;
      }
    }
    next_row += c.nrows;
    off += (int64_t)kWave * c.W;
  }
  std::vector<SegDesc> h_segs;
  for (int32_t i : longs) {
    const int32_t row = next_row++;
    h_lhs.push_back(lhs[i] + 0.0);
    h_rhs.push_back(rhs[i] + 0.0);
    const int32_t first = (int32_t)h_segs.size();
    const int32_t nseg = (int32_t)((len[i] + kSegLen - 1) / kSegLen);
    for (int32_t s = 0; s < nseg; ++s) {
      SegDesc d;
      d.off = off + (int64_t)s * kSegLen;
      d.row = row;
      d.len = (int32_t)std::min<int64_t>(kSegLen, len[i] - (int64_t)s * kSegLen);
      d.first = first;
      d.nseg = nseg;
      d.pad0 = d.pad1 = 0;
      h_segs.push_back(d);
    }
    int64_t pos = 0;
    for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
      if (A->vals[k] == 0.0) continue;
      h_vals[off + pos] = A->vals[k];
      h_cols[off + pos] = col_word(A->col_idx[k]);
      ++pos;
    }
    off += (len[i] + kWave - 1) / kWave * kWave;
  }
  out->n_long_rows = (int32_t)longs.size();

  // every index a kernel forms must stay inside the arrays built above
  const int64_t n_rows_internal = next_row;
  for (const ChunkDesc& d : h_chunks) {
    const int W = (d.meta >> 8) & 0xff, nr = (d.meta >> 16) & 0xff, kl = d.meta & 7;
    if (W < 1 || W > steps || nr < 1 || nr > (kWave >> kl) ||
        (int64_t)d.off64 * kWave + (int64_t)W * kWave > chunk_entries || d.row0 < 0 ||
        d.row0 + nr > n_rows_internal)
      { *err = "internal layout check failed (chunk)"; return false; }
  }
  for (const SegDesc& d : h_segs) {
    if (d.len < 1 || d.len > kSegLen || d.off < chunk_entries || d.off + d.len > stored ||
        d.first < 0 || d.first + d.nseg > (int32_t)h_segs.size() || d.row < 0 ||
        d.row >= n_rows_internal)
      { *err = "internal layout check failed (segment)"; return false; }
  }
  for (int64_t q = 0; q < stored; ++q)
    if ((n > 0 && (h_cols[q] & kColMask) >= n) || (n == 0 && stored > 0))
      { *err = "internal layout check failed (column)"; return false; }
  if ((int64_t)h_lhs.size() != n_rows_internal)
    { *err = "internal layout check failed (rows)"; return false; }

  // rows of each variable in the internal orders, for marked rounds
  {
    std::vector<int64_t>& vp = out->var_ptr;
    std::vector<int32_t>& vr = out->var_rows;
    vp.assign((size_t)n + 1, 0);
    auto each_entry = [&](auto&& fn) {
      for (const ChunkDesc& d : h_chunks) {
        const int W = (d.meta >> 8) & 0xff, kl = d.meta & 7;
        const int64_t b = (int64_t)d.off64 * kWave;
        for (int64_t q = 0; q < (int64_t)W * kWave; ++q)
          if (h_vals[b + q] != 0.0) fn(h_cols[b + q] & kColMask, d.row0 + (int32_t)((q % kWave) >> kl));
      }
      for (const SegDesc& d : h_segs)
        for (int64_t q = d.off; q < d.off + d.len; ++q)
          if (h_vals[q] != 0.0) fn(h_cols[q] & kColMask, d.row);
    };
    each_entry([&](int32_t v, int32_t) { ++vp[(size_t)v + 1]; });
    for (int32_t j = 0; j < n; ++j) vp[(size_t)j + 1] += vp[j];
    vr.assign((size_t)vp[n], 0);
    std::vector<int64_t> fill(vp.begin(), vp.end() - 1);
    each_entry([&](int32_t v, int32_t row) { vr[(size_t)fill[v]++] = row; });
  }

  out->n_hot = n_hot;
  out->n_rows = (int32_t)n_rows_internal;
  out->perm = std::move(perm);
  out->vtype = std::move(vtype);
  out->vals = std::move(h_vals);
  out->cols = std::move(h_cols);
  out->chunks = std::move(h_chunks);
  out->segs = std::move(h_segs);
  out->lhs = std::move(h_lhs);
  out->rhs = std::move(h_rhs);
  return true;
}

}  // namespace prop
