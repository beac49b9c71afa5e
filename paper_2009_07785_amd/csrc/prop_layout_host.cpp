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
                  const uint8_t* vartype, int steps, HostLayout* out, std::string* err,
                  int kind) {
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

  // rows by lanes-per-row class; long rows apart (nnz-split waves: rows
  // longer than a wave's entries)
  const int64_t long_above = kind == 1 ? (int64_t)kNzEntries : (int64_t)kWave * steps;
  std::vector<std::vector<int32_t>> cls(7);
  std::vector<int32_t> longs;
  std::vector<int32_t> shorts;  // nnz-split: short rows in input order
  for (int32_t i = 0; i < m; ++i) {
    if (len[i] == 0) continue;
    // rows of at most 64 lanes x `steps` entries go to chunks, longer ones
    // to 1024-entry segments
    if (len[i] > long_above) {
      longs.push_back(i);
      continue;
    }
    if (kind == 1) {
      shorts.push_back(i);
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

  // nnz-split waves: consecutive short rows, in input order, packed into
  // waves of at most kNzEntries entries and kNzMaxRows rows
  int64_t chunk_entries_all = chunk_entries;
  struct NzWave {
    size_t first, count;  // range of `shorts`
  };
  std::vector<NzWave> nzw;
  if (kind == 1) {
    size_t q = 0;
    while (q < shorts.size()) {
      NzWave w{q, 0};
      int64_t fill = 0;
      while (q < shorts.size() && w.count < (size_t)kNzMaxRows &&
             fill + len[shorts[q]] <= (int64_t)kNzEntries) {
        fill += len[shorts[q]];
        ++w.count;
        ++q;
      }
      nzw.push_back(w);
    }
    stored = (int64_t)nzw.size() * kNzEntries;
    for (int32_t i : longs) stored += (len[i] + kWave - 1) / kWave * kWave;
    if ((int64_t)nzw.size() * kNzEntries / kWave > INT32_MAX)
      { *err = "matrix too large for the layout"; return false; }
    out->stored = stored;
    out->chunk_entries = chunk_entries_all = (int64_t)nzw.size() * kNzEntries;
  }

  std::vector<double> h_vals(stored, 0.0);
  std::vector<int32_t> h_cols(stored, 0);
  std::vector<ChunkDesc> h_chunks;
  h_chunks.reserve(kind == 1 ? nzw.size() : chunks.size());
  std::vector<uint8_t> h_wflags;
  std::vector<double> h_lhs, h_rhs;
  h_lhs.reserve(m);
  h_rhs.reserve(m);
  int64_t off = 0;
  int32_t next_row = 0;
  // nnz-split: entry q of a wave (CSR order within the wave) belongs to lane
  // q / kNzSteps, step q % kNzSteps, stored at step * 64 + lane; bit k of a
  // lane's flag byte marks the first entry of a row
  for (const NzWave& w : nzw) {
    ChunkDesc d;
    d.off64 = (int32_t)(off / kWave);
    d.row0 = next_row;
    d.meta = 0;
    d.pad = (int32_t)w.count;  // rows of the wave
    h_chunks.push_back(d);
    const size_t f0 = h_wflags.size();
    h_wflags.resize(f0 + kWave, 0);
    int64_t q = 0;
    for (size_t t = 0; t < w.count; ++t) {
      const int32_t i = shorts[w.first + t];
      h_lhs.push_back(lhs[i] + 0.0);
      h_rhs.push_back(rhs[i] + 0.0);
      bool first = true;
      for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
        if (A->vals[k] == 0.0) continue;
        const int64_t ln = q / kNzSteps, st = q % kNzSteps;
        const int64_t idx = off + st * kWave + ln;
        h_vals[idx] = A->vals[k];
        h_cols[idx] = col_word(A->col_idx[k]);
        if (first) h_wflags[f0 + (size_t)ln] |= (uint8_t)(1u << st);
        first = false;
        ++q;
      }
    }
    next_row += (int32_t)w.count;
    off += kNzEntries;
  }
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
    if (kind == 1) {
      if (d.pad < 1 || d.pad > kNzMaxRows ||
          (int64_t)d.off64 * kWave + kNzEntries > chunk_entries_all || d.row0 < 0 ||
          d.row0 + d.pad > n_rows_internal)
        { *err = "internal layout check failed (nnz-split wave)"; return false; }
      continue;
    }
    const int W = (d.meta >> 8) & 0xff, nr = (d.meta >> 16) & 0xff, kl = d.meta & 7;
    if (W < 1 || W > steps || nr < 1 || nr > (kWave >> kl) ||
        (int64_t)d.off64 * kWave + (int64_t)W * kWave > chunk_entries || d.row0 < 0 ||
        d.row0 + nr > n_rows_internal)
      { *err = "internal layout check failed (chunk)"; return false; }
  }
  if (kind == 1) {
    // a wave's first entry starts a row, and its flags name its rows
    for (size_t c = 0; c < h_chunks.size(); ++c) {
      int starts = 0;
      for (int l = 0; l < kWave; ++l) starts += __builtin_popcount(h_wflags[c * kWave + l]);
      if (!(h_wflags[c * kWave] & 1u) || starts != h_chunks[c].pad)
        { *err = "internal layout check failed (nnz-split flags)"; return false; }
    }
  }
  for (const SegDesc& d : h_segs) {
    if (d.len < 1 || d.len > kSegLen || d.off < chunk_entries_all || d.off + d.len > stored ||
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
      for (size_t c = 0; kind == 1 && c < h_chunks.size(); ++c) {
        const ChunkDesc& d = h_chunks[c];
        const int64_t b = (int64_t)d.off64 * kWave;
        int32_t local = -1;
        for (int64_t q = 0; q < kNzEntries; ++q) {
          const int64_t ln = q / kNzSteps, st = q % kNzSteps;
          if ((h_wflags[c * kWave + (size_t)ln] >> st) & 1u) ++local;
          const int64_t idx = b + st * kWave + ln;
          if (h_vals[idx] != 0.0) fn(h_cols[idx] & kColMask, d.row0 + local);
        }
      }
      for (const ChunkDesc& d : h_chunks) {
        if (kind == 1) break;
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
  out->wave_flags = std::move(h_wflags);
  out->segs = std::move(h_segs);
  out->lhs = std::move(h_lhs);
  out->rhs = std::move(h_rhs);
  return true;
}

}  // namespace prop
