// host_sum.cpp -- CPU replay of the GPU kernels' activity summation, built
// from the library's own prop_sum.h, for the CPU tests: the same
// double-double updates in the same lane orders (chunk lanes, node-parallel
// slots, long-row segments), the same butterfly combines, the same
// certification and exact fixed-point fallback.  Test infrastructure only.
#include <stdint.h>

#include <vector>

#include "prop_sum.h"

#pragma clang fp contract(off)

using prop::DD;

namespace {

struct Lane {
  DD s{0.0, 0.0};
  double err = 0.0;
};

// Butterfly over `levels` xor levels of the index bits starting at `shift`:
// lane i combines with lane i ^ (1 << (shift + level)), both ending equal.
void butterfly(std::vector<Lane>& L, int shift, int levels) {
  for (int i = 0; i < levels; ++i) {
    const size_t off = (size_t)1 << (shift + i);
    std::vector<Lane> old = L;
    for (size_t k = 0; k < L.size(); ++k) {
      const Lane& y = old[k ^ off];
      prop::dd_add(L[k].s, L[k].err, y.s.hi, y.s.lo, y.err);
    }
  }
}

double exact_sum(const double* a, const double* b, int64_t n) {
  int64_t W[prop::kAccDigits] = {0};
  for (int64_t p = 0; p < n; ++p) {
    int d;
    uint32_t c[5];
    bool neg;
    if (!prop::product_digits(a[p], b[p], d, c, neg)) continue;
    for (int i = 0; i < 5; ++i) W[d + i] += neg ? -(int64_t)c[i] : (int64_t)c[i];
  }
  return prop::digits_round(W);
}

double finish(const Lane& x, const double* a, const double* b, int64_t n, int32_t* certified) {
  double out;
  const bool ok = prop::dd_round(x.s.hi, x.s.lo, x.err, out);
  *certified = ok ? 1 : 0;
  return ok ? out : exact_sum(a, b, n);
}

}  // namespace

extern "C" {

// Exact sum of a[p] * b[p] rounded once, through the fixed-point digits only.
double hs_exact_sum(const double* a, const double* b, int64_t n) { return exact_sum(a, b, n); }

// One row of a chunk with K lanes (K a power of two <= 64): entry p at lane
// p % K, step p / K; every lane sums its steps in order, then the K lanes
// combine by xor butterfly.
double hs_chunk_rowsum(const double* a, const double* b, int64_t n, int32_t K,
                       int32_t* certified) {
  std::vector<Lane> L((size_t)K);
  for (int64_t p = 0; p < n; ++p) {
    Lane& x = L[(size_t)(p % K)];
    prop::dd_add_prod(x.s, a[p], b[p], x.err);
  }
  int klog = 0;
  while ((1 << klog) < K) ++klog;
  butterfly(L, 0, klog);
  return finish(L[0], a, b, n, certified);
}

// The same row (K >= 16) on node-parallel lanes: entry slot e (0..7) sums
// the row's lanes e, e + 8, ... (lane order), each lane's steps in order;
// then the 8 slots combine by xor butterfly.
double hs_nodes_rowsum(const double* a, const double* b, int64_t n, int32_t K,
                       int32_t* certified) {
  std::vector<Lane> S(8);
  const int64_t steps = (n + K - 1) / K;
  for (int e = 0; e < 8; ++e)
    for (int32_t lane = e; lane < K; lane += 8)
      for (int64_t w = 0; w < steps; ++w) {
        const int64_t p = w * K + lane;
        if (p < n) prop::dd_add_prod(S[(size_t)e].s, a[p], b[p], S[(size_t)e].err);
      }
  butterfly(S, 0, 3);
  return finish(S[0], a, b, n, certified);
}

// A long row: 1024-entry segments; within a segment entry q at lane q % 64
// (nodes = 0) or at slot q % 8 (nodes = 1), summed in order, combined by
// butterfly into the segment's partial; then lane s of a 64-lane wave adds
// partials s, s + 64, ... in order and the 64 lanes combine by butterfly.
double hs_long_rowsum(const double* a, const double* b, int64_t n, int32_t nodes,
                      int32_t* certified) {
  const int64_t seg = 1024;
  std::vector<Lane> parts;
  for (int64_t s0 = 0; s0 < n; s0 += seg) {
    const int64_t len = n - s0 < seg ? n - s0 : seg;
    const int lanes = nodes ? 8 : 64;
    std::vector<Lane> L((size_t)lanes);
    for (int64_t q = 0; q < len; ++q) {
      Lane& x = L[(size_t)(q % lanes)];
      prop::dd_add_prod(x.s, a[s0 + q], b[s0 + q], x.err);
    }
    butterfly(L, 0, nodes ? 3 : 6);
    parts.push_back(L[0]);
  }
  std::vector<Lane> L(64);
  for (size_t q = 0; q < parts.size(); ++q) {
    Lane& x = L[q % 64];
    prop::dd_add(x.s, x.err, parts[q].s.hi, parts[q].s.lo, parts[q].err);
  }
  butterfly(L, 0, 6);
  return finish(L[0], a, b, n, certified);
}

}  // extern "C"
