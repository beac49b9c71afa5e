// layout_check.cpp -- runs the library's host layout builder
// (prop_layout_host.cpp) on a CSR matrix read from raw files, for every
// layout step count, and checks that the layout holds exactly the matrix's
// nonzeros: the multiset of (relabelled variable, coefficient) pairs, the
// rows of every variable, the row sides in the internal order and the tile
// descriptors.  Built with the address and undefined-behaviour sanitizers
// by the CPU tests.  Usage: layout_check <dir>; exit status 0 on success.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "prop_layout_host.h"

using namespace prop;

template <typename T>
static std::vector<T> load(const std::string& dir, const char* name) {
  std::string path = dir + "/" + name;
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path.c_str());
    exit(2);
  }
  fseek(f, 0, SEEK_END);
  const long bytes = ftell(f);
  fseek(f, 0, SEEK_SET);
  std::vector<T> v((size_t)bytes / sizeof(T));
  if (!v.empty() && fread(v.data(), sizeof(T), v.size(), f) != v.size()) exit(2);
  fclose(f);
  return v;
}

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      return 1;                                                       \
    }                                                                 \
  } while (0)

static int check_steps(const prop_csr& A, const std::vector<double>& lhs,
                       const std::vector<double>& rhs, const std::vector<uint8_t>& vt, int steps) {
  HostLayout L;
  std::string err;
  CHECK(layout_build(&A, lhs.data(), rhs.data(), vt.data(), steps, &L, &err));
  const int32_t m = A.m, n = A.n;
  // the input's nonzeros as (internal variable, coefficient bits)
  std::vector<std::pair<int32_t, uint64_t>> want, got;
  std::vector<int64_t> deg(n > 0 ? n : 1, 0);
  int64_t nnz = 0;
  for (int32_t i = 0; i < m; ++i)
    for (int64_t k = A.row_ptr[i]; k < A.row_ptr[i + 1]; ++k) {
      if (A.vals[k] == 0.0) continue;
      uint64_t bits;
      memcpy(&bits, &A.vals[k], 8);
      want.push_back({L.perm[A.col_idx[k]], bits});
      ++deg[A.col_idx[k]];
      ++nnz;
    }
  CHECK(L.nnz == nnz);
  CHECK((int64_t)L.vals.size() == L.stored && (int64_t)L.cols.size() == L.stored);
  for (int64_t q = 0; q < L.stored; ++q) {
    if (L.vals[q] == 0.0) continue;
    const int32_t v = L.cols[q] & kColMask;
    CHECK(v >= 0 && v < n);
    CHECK(((L.cols[q] < 0) ? 1 : 0) == L.vtype[v]);  // integrality bit
    uint64_t bits;
    memcpy(&bits, &L.vals[q], 8);
    got.push_back({v, bits});
  }
  std::sort(want.begin(), want.end());
  std::sort(got.begin(), got.end());
  CHECK(want == got);
  // relabelling: a permutation, types carried along, decreasing degree
  std::vector<int32_t> inv(n > 0 ? n : 1, -1);
  for (int32_t j = 0; j < n; ++j) {
    CHECK(L.perm[j] >= 0 && L.perm[j] < n && inv[L.perm[j]] < 0);
    inv[L.perm[j]] = j;
    CHECK(L.vtype[L.perm[j]] == vt[j]);
  }
  // hot prefix, then integer variables, then continuous ones, each part by
  // decreasing degree
  CHECK(L.n_hot >= 0 && L.n_hot <= n && L.n_hot <= kMaxHot);
  for (int32_t q = 0; q < L.n_hot; ++q) CHECK(deg[inv[q]] >= kHotDegree);
  for (int32_t q = L.n_hot; q < n; ++q) {
    CHECK(deg[inv[q]] < kHotDegree || L.n_hot == kMaxHot);
    if (q + 1 < n) {
      if (q + 1 == L.n_hot) continue;
      const bool same = L.vtype[q] == L.vtype[q + 1];
      CHECK(same ? deg[inv[q]] >= deg[inv[q + 1]] : (L.vtype[q] != 0 && L.vtype[q + 1] == 0));
    }
  }
  for (int32_t q = 1; q < L.n_hot; ++q) CHECK(deg[inv[q - 1]] >= deg[inv[q]]);
  // rows of every variable
  CHECK((int64_t)L.var_ptr.size() == (int64_t)n + 1 && L.var_ptr[n] == nnz);
  for (int32_t v = 0; v < n; ++v) CHECK(L.var_ptr[v + 1] - L.var_ptr[v] == deg[inv[v]]);
  for (int32_t r : L.var_rows) CHECK(r >= 0 && r < L.n_rows);
  // tiles inside the arrays; every internal row has sides from some input row
  CHECK((int64_t)L.lhs.size() == L.n_rows && (int64_t)L.rhs.size() == L.n_rows);
  for (const ChunkDesc& d : L.chunks) {
    const int W = (d.meta >> 8) & 0xff, nr = (d.meta >> 16) & 0xff, kl = d.meta & 7;
    CHECK(W >= 1 && W <= steps && nr >= 1 && nr <= (kWave >> kl));
    CHECK((int64_t)d.off64 * kWave + (int64_t)W * kWave <= L.chunk_entries);
    CHECK(d.row0 >= 0 && d.row0 + nr <= L.n_rows);
  }
  int64_t long_entries = 0;
  for (const SegDesc& d : L.segs) {
    CHECK(d.len >= 1 && d.len <= kSegLen && d.off >= L.chunk_entries && d.off + d.len <= L.stored);
    CHECK(d.first >= 0 && d.first + d.nseg <= (int32_t)L.segs.size());
    CHECK(d.row >= 0 && d.row < L.n_rows);
    long_entries += d.len;
  }
  int64_t long_nnz = 0;
  int32_t long_rows = 0;
  for (int32_t i = 0; i < m; ++i) {
    int64_t len = 0;
    for (int64_t k = A.row_ptr[i]; k < A.row_ptr[i + 1]; ++k) len += A.vals[k] != 0.0;
    if (len > (int64_t)kWave * steps) {
      long_nnz += len;
      ++long_rows;
    }
  }
  CHECK(long_entries == long_nnz && L.n_long_rows == long_rows);
  std::vector<std::pair<double, double>> sides_in, sides_out;
  for (int32_t i = 0; i < m; ++i)
    if (A.row_ptr[i + 1] > A.row_ptr[i]) {
      bool any = false;
      for (int64_t k = A.row_ptr[i]; k < A.row_ptr[i + 1]; ++k) any |= A.vals[k] != 0.0;
      if (any) sides_in.push_back({lhs[i] + 0.0, rhs[i] + 0.0});
    }
  for (int32_t r = 0; r < L.n_rows; ++r) sides_out.push_back({L.lhs[r], L.rhs[r]});
  std::sort(sides_in.begin(), sides_in.end());
  std::sort(sides_out.begin(), sides_out.end());
  CHECK(sides_in == sides_out);
  return 0;
}

// The nnz-split layout: each internal short row, read back from its wave
// through the flag bytes (entry q of a wave at step q % 8, lane q / 8), holds
// exactly the input row's nonzeros in order, with its sides, rows in input
// order; long rows go to segments as in the chunk layout.
static int check_nnz_split(const prop_csr& A, const std::vector<double>& lhs,
                           const std::vector<double>& rhs, const std::vector<uint8_t>& vt) {
  const int32_t m = A.m, n = A.n;
  HostLayout L;
  std::string err;
  CHECK(layout_build(&A, lhs.data(), rhs.data(), vt.data(), 16, &L, &err, 1));
  CHECK((int64_t)L.wave_flags.size() == (int64_t)L.chunks.size() * kWave);
  CHECK(L.chunk_entries == (int64_t)L.chunks.size() * kNzEntries);
  std::vector<int32_t> inv(n > 0 ? n : 1, -1);
  for (int32_t j = 0; j < n; ++j) inv[L.perm[j]] = j;
  // the short rows in input order
  std::vector<int32_t> shorts;
  for (int32_t i = 0; i < m; ++i) {
    int64_t len = 0;
    for (int64_t k = A.row_ptr[i]; k < A.row_ptr[i + 1]; ++k) len += A.vals[k] != 0.0;
    if (len > 0 && len <= kNzEntries) shorts.push_back(i);
  }
  size_t next = 0;
  for (size_t c = 0; c < L.chunks.size(); ++c) {
    const ChunkDesc& d = L.chunks[c];
    CHECK(d.pad >= 1 && d.pad <= kNzMaxRows && d.row0 == (int32_t)next);
    std::vector<std::vector<std::pair<int32_t, double>>> rows((size_t)d.pad);
    int32_t local = -1;
    for (int64_t q = 0; q < kNzEntries; ++q) {
      const int64_t ln = q / kNzSteps, st = q % kNzSteps;
      if ((L.wave_flags[c * kWave + (size_t)ln] >> st) & 1u) ++local;
      CHECK(local >= 0 && local < d.pad);
      const int64_t idx = (int64_t)d.off64 * kWave + st * kWave + ln;
      CHECK(idx >= 0 && idx < L.chunk_entries);
      if (L.vals[idx] == 0.0) continue;
      const int32_t v = L.cols[idx] & kColMask;
      CHECK(v >= 0 && v < n);
      CHECK(((L.cols[idx] < 0) ? 1 : 0) == L.vtype[v]);
      rows[(size_t)local].push_back({inv[v], L.vals[idx]});
    }
    CHECK(local == d.pad - 1);
    for (int32_t r = 0; r < d.pad; ++r, ++next) {
      CHECK(next < shorts.size());
      const int32_t i = shorts[next];
      std::vector<std::pair<int32_t, double>> want;
      for (int64_t k = A.row_ptr[i]; k < A.row_ptr[i + 1]; ++k)
        if (A.vals[k] != 0.0) want.push_back({A.col_idx[k], A.vals[k]});
      CHECK(rows[(size_t)r] == want);
      CHECK(L.lhs[(size_t)(d.row0 + r)] == lhs[i] + 0.0 && L.rhs[(size_t)(d.row0 + r)] == rhs[i] + 0.0);
    }
  }
  CHECK(next == shorts.size());
  for (const SegDesc& sd : L.segs)
    CHECK(sd.len >= 1 && sd.len <= kSegLen && sd.off >= L.chunk_entries && sd.off + sd.len <= L.stored);
  // rows of every variable: each entry's row counted once
  CHECK((int64_t)L.var_ptr.size() == (int64_t)n + 1);
  for (int32_t r : L.var_rows) CHECK(r >= 0 && r < L.n_rows);
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  const std::string dir = argv[1];
  const std::vector<int64_t> dims = load<int64_t>(dir, "dims");
  const std::vector<int64_t> rp = load<int64_t>(dir, "row_ptr");
  const std::vector<int32_t> col = load<int32_t>(dir, "col_idx");
  const std::vector<double> val = load<double>(dir, "vals");
  const std::vector<double> lhs = load<double>(dir, "lhs");
  const std::vector<double> rhs = load<double>(dir, "rhs");
  const std::vector<uint8_t> vt = load<uint8_t>(dir, "vartype");
  prop_csr A;
  A.m = (int32_t)dims[0];
  A.n = (int32_t)dims[1];
  A.nnz = dims[2];
  A.row_ptr = rp.data();
  A.col_idx = col.data();
  A.vals = val.data();
  for (int steps : {4, 8, 16}) {
    const int rc = check_steps(A, lhs, rhs, vt, steps);
    if (rc) {
      fprintf(stderr, "steps = %d\n", steps);
      return rc;
    }
  }
  if (check_nnz_split(A, lhs, rhs, vt)) {
    fprintf(stderr, "nnz-split layout\n");
    return 1;
  }
  printf("layout ok: %d x %d, %lld nonzeros\n", A.m, A.n, (long long)A.nnz);
  return 0;
}
