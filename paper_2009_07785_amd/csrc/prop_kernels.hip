// prop_kernels.hip -- gfx950 kernels of one synchronous propagation round
// (Sofranac, Gleixner, Pokutta, arXiv 2009.07785, Algorithms 2 and 3) and
// the drivers that repeat rounds on the device.
//
// Bounds live in two arrays of (lb, ub) pairs: A holds the bounds as they
// stood at the start of the round and is only read during it; B starts
// equal to A and receives the candidates.  One round:
//   1. every row's min / max activity from A: finite parts as exact-product
//      double-double sums (rounded once at the end), plus the counts of
//      infinite contributions (Definition 1; Sec. 3.4);
//   2. per entry the candidates of Step 3 (eqs. bound_candidates_pos / _neg),
//      rounded inward for integer variables, each one IEEE operation in the
//      order (beta - activity) / a + bound;
//   3. a candidate that beats the start-of-round bound (the pre-check of
//      Sec. 3.5) goes to B with an FP64 atomic max (lower) / min (upper);
//      the atomics return nothing, so no wave waits on them (Algorithm 3);
//   4. commit: every variable whose pair in B differs from A is copied to A,
//      counted, and its domain checked for emptiness; the last block to
//      finish decides the round's status from one packed counter.
//
// Work units: a "chunk" is one wave's tile of short/medium rows, laid out so
// each of up to 16 steps is one contiguous 64-entry load; a row of K lanes
// sums its entries lane by lane, then across its K lanes.  Rows longer than
// 1024 entries are split into 1024-entry segments: phase 1 writes a partial
// sum per segment, phase 2 combines all partials of the row in a fixed order
// and handles the segment's candidates.
//
// Before any candidate arithmetic an entry side is skipped when the row's
// slack s on that side (rhs - min activity, or max activity - lhs) proves
// that its candidate cannot count.  For a > 0 on the rhs side the candidate
// is c = RN(RN(s / a) + l) and counts when c < V, V the point below which an
// upper bound must move (u itself for integers, up to the eps_int rounding;
// u - tau * max(1, |u|) for continuous variables, evaluated exactly as the
// significance test does).  If s > RN(RN(|a| * W) * (1 + 2^-39)) with
// W = RN(V - l) > 0, then s > |a| * (V - l) * (1 + 2^-40) in exact terms, so
// RN(s / a) > V - l and c >= V: the candidate cannot count.  The other three
// sign / side combinations are mirror images; integers use W = u - l, where
// c >= u already rules out floor(c + eps_int) < u.  A skipped side is thus
// exactly one whose candidate the oracle would also have discarded.
#include <hip/hip_runtime.h>

#include "prop_launch.h"
#include "prop_layout.h"

#pragma clang fp contract(off)

namespace prop {

#define PROP_HUGE 0x1p200
#define PROP_SKIP_MARGIN (1.0 + 0x1p-39)
#define PROP_SKIP_FLOOR 0x1p-900

// ---------------------------------------------------------------------------
// exact-product double-double accumulation
// ---------------------------------------------------------------------------
struct DD {
  double hi, lo;
};

// s += a * b: the product is split exactly into p + ep (FMA), p is added to
// s.hi with an error-free two-sum, and both error terms go to s.lo.
__device__ __forceinline__ void dd_add_prod(DD& s, double a, double b) {
  double p = a * b;
  double ep = __builtin_fma(a, b, -p);
  double t = s.hi + p;
  double z = t - s.hi;
  double e = (s.hi - (t - z)) + (p - z);
  s.hi = t;
  s.lo = s.lo + (e + ep);
}

// s += (yhi, ylo); symmetric in its two operands, so both lanes of a
// butterfly exchange end with identical bits.
__device__ __forceinline__ void dd_add(DD& s, double yhi, double ylo) {
  double t = s.hi + yhi;
  double z = t - s.hi;
  double e = (s.hi - (t - z)) + (yhi - z);
  s.hi = t;
  s.lo = (s.lo + ylo) + e;
}

__device__ __forceinline__ double dd_value(const DD& s) { return (s.hi + s.lo) + 0.0; }

// Combines the partial sums of the 2^klog lanes of each row (klog is the
// same in every lane of the wave, so the branches are uniform).
__device__ __forceinline__ void group_reduce(DD& smin, DD& smax, int& cmin, int& cmax, int klog) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    if (i >= klog) break;
    const int off = 1 << i;
    double a = __shfl_xor(smin.hi, off, kWave);
    double b = __shfl_xor(smin.lo, off, kWave);
    double c = __shfl_xor(smax.hi, off, kWave);
    double d = __shfl_xor(smax.lo, off, kWave);
    int e = __shfl_xor(cmin, off, kWave);
    int f = __shfl_xor(cmax, off, kWave);
    dd_add(smin, a, b);
    dd_add(smax, c, d);
    cmin += e;
    cmax += f;
  }
}

__device__ __forceinline__ bool is_inf(double x) { return __builtin_isinf(x); }

// Contribution of one entry to both activities.
__device__ __forceinline__ void accumulate(double a, double l, double u, DD& smin, DD& smax,
                                           int& cmin, int& cmax) {
  const double bmin = a > 0.0 ? l : u;
  const double bmax = a > 0.0 ? u : l;
  const bool imin = is_inf(bmin);
  const bool imax = is_inf(bmax);
  cmin += (a != 0.0 && imin) ? 1 : 0;
  cmax += (a != 0.0 && imax) ? 1 : 0;
  dd_add_prod(smin, a, imin ? 0.0 : bmin);
  dd_add_prod(smax, a, imax ? 0.0 : bmax);
}

// Skip threshold of one side of an entry: the candidate that side yields
// cannot count (be applied) when the row's slack on that side exceeds the
// returned value.  `upper` says which bound the side would tighten.  The
// width used is the distance from the other bound to the point where a
// candidate starts to count: u - l for integers, and for continuous
// variables the same expressions the significance test evaluates
// (u - tau * max(1, |u|) for an upper bound, l + tau * max(1, |l|) for a
// lower one).  With that width W > 0 the threshold is |a| * W with a
// 1 + 2^-39 margin, which covers the rounding of these three operations and
// of the candidate's own s / a and + bound (see the file header).  W <= 0
// means the candidate cannot count while the slack is >= 0, encoded as the
// threshold -2^-1074 (slack > -2^-1074 <=> slack >= 0).  An infinite bound
// to tighten counts every finite candidate: threshold +inf.
__device__ __forceinline__ double side_threshold(double a, double l, double u, bool is_int,
                                                 bool upper, double tau) {
  double w;
  if (upper) {
    if (u == __builtin_inf()) return __builtin_inf();
    if (is_int) {
      w = u - l;
    } else {
      const double s = __builtin_fabs(u) > 1.0 ? __builtin_fabs(u) : 1.0;
      w = (u - tau * s) - l;
    }
  } else {
    if (l == -__builtin_inf()) return __builtin_inf();
    if (is_int) {
      w = u - l;
    } else {
      const double s = __builtin_fabs(l) > 1.0 ? __builtin_fabs(l) : 1.0;
      w = u - (l + tau * s);
    }
  }
  if (!(w > 0.0)) return -0x1p-1074;
  const double thr = (__builtin_fabs(a) * w) * PROP_SKIP_MARGIN;
  return thr >= PROP_SKIP_FLOOR ? thr : __builtin_inf();
}

__device__ __forceinline__ bool domain_empty(bool is_int, double l, double u, double feas_tol) {
  if (is_int) return l > u;
  double s = __builtin_fabs(l) > __builtin_fabs(u) ? __builtin_fabs(l) : __builtin_fabs(u);
  if (s < 1.0) s = 1.0;
  return (l - u) > feas_tol * s;
}

// Fire-and-forget FP64 atomics (the result is unused, so no wave waits).
__device__ __forceinline__ void atomic_max_f64(double* p, double v) {
  (void)__hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_min_f64(double* p, double v) {
  (void)__hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Row-level quantities every entry of a row needs.
struct RowState {
  double minfin, maxfin;
  int cmin, cmax;
  bool min_side, max_side;  // the rhs / lhs side can yield candidates
  double smn;               // rhs - min activity
  double smx;               // lhs - max activity
};

__device__ __forceinline__ RowState make_row_state(const DD& smin, const DD& smax, int cmin,
                                                   int cmax, double lhs, double rhs) {
  RowState R;
  R.minfin = dd_value(smin);
  R.maxfin = dd_value(smax);
  R.cmin = cmin;
  R.cmax = cmax;
  R.min_side = (rhs < __builtin_inf()) && cmin <= 1;
  R.max_side = (lhs > -__builtin_inf()) && cmax <= 1;
  R.smn = rhs - R.minfin;
  R.smx = lhs - R.maxfin;
  return R;
}

// Which sides of entry (a, column word cw; start-of-round l, u) need the
// candidate arithmetic.  The rhs side works through the min activity and
// tightens u when a > 0, l when a < 0; the lhs side the other way round.
// With one infinite contribution only its owner gets a candidate.
__device__ __forceinline__ void entry_sides(const RowState& R, double a, double l, double u,
                                            int32_t cw, double tau, bool& dmin, bool& dmax) {
  dmin = dmax = false;
  if (a == 0.0) return;
  const bool is_int = cw < 0;
  const bool pos = a > 0.0;
  if (R.min_side) {
    if (R.cmin == 0) dmin = !(R.smn > side_threshold(a, l, u, is_int, pos, tau));
    else dmin = is_inf(pos ? l : u);
  }
  if (R.max_side) {
    if (R.cmax == 0) dmax = !((-R.smx) > side_threshold(a, l, u, is_int, !pos, tau));
    else dmax = is_inf(pos ? u : l);
  }
}

__device__ __forceinline__ bool entry_wanted(const RowState& R, double a, double l, double u,
                                             int32_t cw, double tau) {
  bool dmin, dmax;
  entry_sides(R, a, l, u, cw, tau, dmin, dmax);
  return dmin || dmax;
}

// Candidates of one entry (a, column word cw) with start-of-round bounds
// (l, u); the column word holds the variable in bits 0-30 and its
// integrality in bit 31.
// `nxt` points at this node's first pair; variable j's pair is nxt[j * stride].
// With `striped`, variables below P.n_hot write to this block's stripe copy.
__device__ __forceinline__ void entry_candidates(const Problem& P, const RowState& R, double a,
                                                 double l, double u, int32_t cw,
                                                 double2* __restrict__ nxt, uint32_t stride,
                                                 bool striped) {
  bool dmin, dmax;
  entry_sides(R, a, l, u, cw, P.cont_rel_tol, dmin, dmax);
  if (!(dmin || dmax)) return;
  const int32_t var = cw & kColMask;
  size_t j = (size_t)var * stride;
  if (striped && var < P.n_hot) {
    nxt = P.stripes + (size_t)(blockIdx.x % kStripes) * P.n_hot;
    j = (size_t)var;
  }
  const bool is_int = cw < 0;
  const double bmin = a > 0.0 ? l : u;
  const double bmax = a > 0.0 ? u : l;

  double lc = 0.0, uc = 0.0;
  bool hl = false, hu = false;
  if (dmin) {  // rhs side: (rhs - min act) / a (+ b_min when no infinity)
    double t = R.smn / a;
    if (R.cmin == 0) t = t + bmin;
    if (a > 0.0) { uc = t; hu = true; } else { lc = t; hl = true; }
  }
  if (dmax) {  // lhs side: (lhs - max act) / a (+ b_max when no infinity)
    double t = R.smx / a;
    if (R.cmax == 0) t = t + bmax;
    if (a > 0.0) { lc = t; hl = true; } else { uc = t; hu = true; }
  }
  if (hl) {
    double c = is_int ? __builtin_ceil(lc - P.eps_int) : lc;
    c = c + 0.0;
    if (__builtin_fabs(c) <= PROP_HUGE) {
      bool sig;
      if (l == -__builtin_inf()) sig = true;
      else if (is_int) sig = c > l;
      else {
        double s = __builtin_fabs(l) > 1.0 ? __builtin_fabs(l) : 1.0;
        sig = c > l + P.cont_rel_tol * s;
      }
      if (sig) atomic_max_f64(&nxt[j].x, c);
    }
  }
  if (hu) {
    double c = is_int ? __builtin_floor(uc + P.eps_int) : uc;
    c = c + 0.0;
    if (__builtin_fabs(c) <= PROP_HUGE) {
      bool sig;
      if (u == __builtin_inf()) sig = true;
      else if (is_int) sig = c < u;
      else {
        double s = __builtin_fabs(u) > 1.0 ? __builtin_fabs(u) : 1.0;
        sig = c < u - P.cont_rel_tol * s;
      }
      if (sig) atomic_min_f64(&nxt[j].y, c);
    }
  }
}

// Skip code of one entry side for the chunk filter: a float c with
// "slack >= c" implying "slack > thr" (thr from side_threshold), so a side
// skipped by the code is one the exact test skips too.  Finite thresholds
// round up to the next float strictly above them; thresholds below 2^-100
// map to 2^-100 (no subnormal floats are involved); W <= 0 (skipped iff the
// slack is >= 0) maps to 0; "never skip" stays +inf.
__device__ __forceinline__ float skip_code(double thr) {
  if (thr < 0.0) return 0.0f;
  if (!(thr < __builtin_inf())) return __builtin_inff();
  if (thr < 0x1p-100) return 0x1p-100f;
  float f = (float)thr;
  if ((double)f <= thr) f = __int_as_float(__float_as_int(f) + 1);
  return f;
}

// Both skip codes of an entry: the rhs side (through the min activity) and
// the lhs side (through the max activity).  NaN marks the entry whose bound
// makes that side's activity infinite: with exactly one infinite
// contribution only that entry gets a candidate.
__device__ __forceinline__ void entry_codes(double a, double l, double u, int32_t cw, double tau,
                                            float& emin, float& emax) {
  const bool is_int = cw < 0, pos = a > 0.0;
  const double bmin = pos ? l : u, bmax = pos ? u : l;
  emin = is_inf(bmin) ? __builtin_nanf("") : skip_code(side_threshold(a, l, u, is_int, pos, tau));
  emax = is_inf(bmax) ? __builtin_nanf("") : skip_code(side_threshold(a, l, u, is_int, !pos, tau));
}

// Conservative form of entry_sides from the codes: true for every entry
// with a side that entry_sides would keep.  Entries without a coefficient
// carry -inf codes and never pass.
__device__ __forceinline__ bool entry_passes(const RowState& R, float emin, float emax) {
  bool p = false;
  if (R.min_side) p |= R.cmin == 0 ? !(R.smn >= (double)emin) : __builtin_isnan(emin);
  if (R.max_side) p |= R.cmax == 0 ? !((-R.smx) >= (double)emax) : __builtin_isnan(emax);
  return p;
}

// ---------------------------------------------------------------------------
// one chunk: activities and candidates for 64/K rows, K lanes per row
//
// Bound arrays are addressed as base[var * stride + node]: stride 1 for a
// single problem, 8 for a batch (8 nodes share each variable's cache line).
// Per active node (bit t of node_mask) each step loads its coefficient and
// column word, gathers the bounds, adds the entry to the activities and
// keeps only the entry's two skip codes; after the row reduction, the
// entries whose codes do not rule them out reload their data and go through
// the exact candidate test.  Holding two floats per step instead of the
// entry's coefficient, column and bounds keeps the wave's register count,
// and with it the number of resident waves hiding the gather latency, in
// line with a plain sparse product.  In a batch, nodes after the first find
// the chunk's matrix data in cache.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chunk_round(const Problem& P, const ChunkDesc cd,
                                            const double2* __restrict__ cur,
                                            double2* __restrict__ nxt, uint32_t stride,
                                            uint32_t node_mask) {
  const int lane = threadIdx.x & (kWave - 1);
  const int klog = cd.meta & 7;
  const int W = (cd.meta >> 8) & 0xff;
  const int nrows = (cd.meta >> 16) & 0xff;
  const int r = lane >> klog;
  const size_t base = (size_t)cd.off64 * kWave + lane;
  const bool row_ok = r < nrows;
  const int row = cd.row0 + (row_ok ? r : 0);
  const double lhs = P.lhs[row], rhs = P.rhs[row];
  for (uint32_t mask = node_mask; mask; mask &= mask - 1) {
    const uint32_t t = __builtin_ctz(mask);
    float emin[kMaxSteps], emax[kMaxSteps];
    DD smin = {0.0, 0.0}, smax = {0.0, 0.0};
    int cmin = 0, cmax = 0;
#pragma unroll
    for (int w = 0; w < kMaxSteps; ++w) {
      emin[w] = -__builtin_inff();
      emax[w] = -__builtin_inff();
      if (w < W) {
        const size_t e = base + (size_t)w * kWave;
        // a single run reads the matrix once: stream it past the caches
        const double a = stride == 1 ? __builtin_nontemporal_load(P.vals + e) : P.vals[e];
        const int32_t cw = stride == 1 ? __builtin_nontemporal_load(P.cols + e) : P.cols[e];
        if (a != 0.0) {
          const double2 b = cur[(size_t)(cw & kColMask) * stride + t];
          accumulate(a, b.x, b.y, smin, smax, cmin, cmax);
          entry_codes(a, b.x, b.y, cw, P.cont_rel_tol, emin[w], emax[w]);
        }
      }
    }
    group_reduce(smin, smax, cmin, cmax, klog);
    if (!row_ok) continue;
    const RowState R = make_row_state(smin, smax, cmin, cmax, lhs, rhs);
    if (!(R.min_side || R.max_side)) continue;
    // a step no lane needs is skipped by the wave
#pragma unroll
    for (int w = 0; w < kMaxSteps; ++w) {
      if (w < W && entry_passes(R, emin[w], emax[w])) {
        const size_t e = base + (size_t)w * kWave;
        const double a = P.vals[e];
        const int32_t cw = P.cols[e];
        const double2 b = cur[(size_t)(cw & kColMask) * stride + t];
        entry_candidates(P, R, a, b.x, b.y, cw, nxt + t, stride, stride == 1);
      }
    }
  }
}

__device__ __forceinline__ void chunk_dispatch(const Problem& P, int c, const double2* cur,
                                               double2* nxt, uint32_t stride,
                                               uint32_t node_mask) {
  chunk_round(P, P.chunks[c], cur, nxt, stride, node_mask);
}

// ---------------------------------------------------------------------------
// node-parallel lanes for batches of 8 nodes
//
// In a batch the 8 nodes of a group keep each variable's (l, u) pairs in one
// 128-byte line ([n][8] layout).  Lane e * 8 + t serves entry slot e of an
// 8-entry block for node t, so the 8 lanes of an entry read one line with a
// single request and the matrix data is read once for the group.  The
// chunk layout is the single-run one: a 64-entry step is walked as 8 blocks
// of 8 entry lanes.  Rows of K <= 8 lanes sit inside one block (their lanes
// are the block's slots, summed in the single-run order); rows of K >= 16
// lanes span K / 8 blocks, whose entries each slot sums one after another.
//
// Instead of one code per entry, a lane keeps the largest skip code of its
// entries per side (and whether it holds the entry that owns the side's
// only infinite contribution): "slack >= largest code" skips every entry of
// the lane, so only lanes with an entry that may count revisit their
// entries, with the exact test.
// ---------------------------------------------------------------------------
struct LaneAcc {
  DD smin, smax;
  int cmin, cmax;
  float amin, amax;  // largest finite skip code per side
  bool omin, omax;   // holds the owner of the side's infinite contribution
};

__device__ __forceinline__ void lane_acc_init(LaneAcc& L) {
  L.smin = {0.0, 0.0};
  L.smax = {0.0, 0.0};
  L.cmin = L.cmax = 0;
  L.amin = L.amax = -__builtin_inff();
  L.omin = L.omax = false;
}

// Entries idx0 + k * dk (k < count, 1 <= count <= N) for node t: loads of
// the group, then its gathers, then the arithmetic.  Indices past count
// re-read the last entry and contribute nothing.
template <int N>
__device__ __forceinline__ void node_entries(const Problem& P, const double2* __restrict__ cur,
                                             uint32_t t, bool on, size_t idx0, size_t dk,
                                             int count, LaneAcc& L) {
  double av[N];
  int32_t cv[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const size_t idx = idx0 + (size_t)(k < count ? k : count - 1) * dk;
    av[k] = P.vals[idx];
    cv[k] = P.cols[idx];
  }
  double2 bv[N];
#pragma unroll
  for (int k = 0; k < N; ++k) bv[k] = cur[(size_t)(cv[k] & kColMask) * kNodeGroup + t];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k < count && on && av[k] != 0.0) {
      accumulate(av[k], bv[k].x, bv[k].y, L.smin, L.smax, L.cmin, L.cmax);
      float c1, c2;
      entry_codes(av[k], bv[k].x, bv[k].y, cv[k], P.cont_rel_tol, c1, c2);
      if (__builtin_isnan(c1)) L.omin = true;
      else L.amin = c1 > L.amin ? c1 : L.amin;
      if (__builtin_isnan(c2)) L.omax = true;
      else L.amax = c2 > L.amax ? c2 : L.amax;
    }
  }
}

// Sums over the entry slots of a row: xor over the slot bits (lane bits 3..)
// below `levels`, with the symmetric combine.
__device__ __forceinline__ void slot_reduce(LaneAcc& L, int levels) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= levels) break;
    const int off = 8 << i;
    double a = __shfl_xor(L.smin.hi, off, kWave);
    double b = __shfl_xor(L.smin.lo, off, kWave);
    double c = __shfl_xor(L.smax.hi, off, kWave);
    double d = __shfl_xor(L.smax.lo, off, kWave);
    int e = __shfl_xor(L.cmin, off, kWave);
    int f = __shfl_xor(L.cmax, off, kWave);
    dd_add(L.smin, a, b);
    dd_add(L.smax, c, d);
    L.cmin += e;
    L.cmax += f;
  }
}

__device__ __forceinline__ bool lane_may_pass(const RowState& R, const LaneAcc& L) {
  bool p = false;
  if (R.min_side) p |= R.cmin == 0 ? !(R.smn >= (double)L.amin) : L.omin;
  if (R.max_side) p |= R.cmax == 0 ? !((-R.smx) >= (double)L.amax) : L.omax;
  return p;
}

__device__ __forceinline__ void chunk_round_nodes(const Problem& P, const ChunkDesc cd,
                                                  const double2* __restrict__ cur,
                                                  double2* __restrict__ nxt, uint32_t node_mask) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t t = lane & (kNodeGroup - 1);
  const int e = lane >> 3;
  const bool on = (node_mask >> t) & 1u;
  const int klog = cd.meta & 7;
  const int W = (cd.meta >> 8) & 0xff;
  const int nrows = (cd.meta >> 16) & 0xff;
  const int QB = klog > 3 ? 1 << (klog - 3) : 1;       // 8-entry blocks per row block
  const int per_block = klog > 3 ? 1 : 8 >> klog;      // rows per row block
  const int nblocks = (nrows + per_block - 1) / per_block;
  const size_t base = (size_t)cd.off64 * kWave;
  for (int rb = 0; rb < nblocks; ++rb) {
    const int r = klog > 3 ? rb : rb * per_block + (e >> klog);
    LaneAcc L;
    lane_acc_init(L);
    for (int qq = 0; qq < QB; ++qq) {
      const size_t l = (size_t)(rb * QB + qq) * 8 + e;
      for (int w0 = 0; w0 < W; w0 += 8)
        node_entries<8>(P, cur, t, on, base + (size_t)w0 * kWave + l, kWave,
                        W - w0 < 8 ? W - w0 : 8, L);
    }
    slot_reduce(L, klog > 3 ? 3 : klog);
    if (r >= nrows || !on) continue;
    const int row = cd.row0 + r;
    const RowState R = make_row_state(L.smin, L.smax, L.cmin, L.cmax, P.lhs[row], P.rhs[row]);
    if (!lane_may_pass(R, L)) continue;
    for (int qq = 0; qq < QB; ++qq) {
      const size_t l = (size_t)(rb * QB + qq) * 8 + e;
      for (int w = 0; w < W; ++w) {
        const size_t idx = base + (size_t)w * kWave + l;
        const double a = P.vals[idx];
        if (a == 0.0) continue;
        const int32_t cw = P.cols[idx];
        const double2 b = cur[(size_t)(cw & kColMask) * kNodeGroup + t];
        entry_candidates(P, R, a, b.x, b.y, cw, nxt + t, kNodeGroup, false);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// long rows: partials live at partials[segment * pstride + node]
// ---------------------------------------------------------------------------
__device__ __forceinline__ void seg_phase1(const Problem& P, int s,
                                           const double2* __restrict__ cur, uint32_t stride,
                                           uint32_t node_mask, SegPartial* parts,
                                           uint32_t pstride, uint32_t node0) {
  const int lane = threadIdx.x & (kWave - 1);
  const SegDesc sd = P.segs[s];
  double a[kMaxSteps];
  int32_t jj[kMaxSteps];
#pragma unroll
  for (int w = 0; w < kMaxSteps; ++w) {
    const int p = w * kWave + lane;
    a[w] = 0.0;
    jj[w] = 0;
    if (p < sd.len) {
      a[w] = __builtin_nontemporal_load(P.vals + sd.off + p);
      jj[w] = __builtin_nontemporal_load(P.cols + sd.off + p);
    }
  }
  for (uint32_t mask = node_mask; mask; mask &= mask - 1) {
    const uint32_t t = __builtin_ctz(mask);
    DD smin = {0.0, 0.0}, smax = {0.0, 0.0};
    int cmin = 0, cmax = 0;
    double tmin = -0x1p-1074, tmax = -0x1p-1074;  // per-side skip thresholds
#pragma unroll
    for (int w = 0; w < kMaxSteps; ++w) {
      if (a[w] != 0.0) {
        const double2 b = cur[(size_t)(jj[w] & kColMask) * stride + t];
        accumulate(a[w], b.x, b.y, smin, smax, cmin, cmax);
        const bool is_int = jj[w] < 0, pos = a[w] > 0.0;
        const double t1 = side_threshold(a[w], b.x, b.y, is_int, pos, P.cont_rel_tol);
        const double t2 = side_threshold(a[w], b.x, b.y, is_int, !pos, P.cont_rel_tol);
        tmin = t1 > tmin ? t1 : tmin;
        tmax = t2 > tmax ? t2 : tmax;
      }
    }
    group_reduce(smin, smax, cmin, cmax, 6);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double o1 = __shfl_xor(tmin, off, kWave);
      const double o2 = __shfl_xor(tmax, off, kWave);
      tmin = o1 > tmin ? o1 : tmin;
      tmax = o2 > tmax ? o2 : tmax;
    }
    if (lane == 0) {
      SegPartial q;
      q.min_hi = smin.hi;
      q.min_lo = smin.lo;
      q.max_hi = smax.hi;
      q.max_lo = smax.lo;
      q.tmin = tmin;
      q.tmax = tmax;
      q.min_inf = cmin;
      q.max_inf = cmax;
      q.pad0 = q.pad1 = 0;
      parts[(size_t)s * pstride + node0 + t] = q;
    }
  }
}

// Phase 1 of a segment for the 8 nodes of a group (node-parallel lanes):
// slot e sums entries e, e + 8, e + 16, ... of the segment for node t.
__device__ __forceinline__ void seg_phase1_nodes(const Problem& P, int s,
                                                 const double2* __restrict__ cur,
                                                 uint32_t node_mask, SegPartial* parts,
                                                 uint32_t pstride, uint32_t node0) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t t = lane & (kNodeGroup - 1);
  const int e = lane >> 3;
  const bool on = (node_mask >> t) & 1u;
  const SegDesc sd = P.segs[s];
  const int nblk = (sd.len + 7) / 8;  // the region is padded to whole 64-entry steps
  LaneAcc L;
  lane_acc_init(L);
  double tmin = -0x1p-1074, tmax = -0x1p-1074;
  for (int i0 = 0; i0 < nblk; i0 += 8) {
    const int count = nblk - i0 < 8 ? nblk - i0 : 8;
    // same loads and gathers as node_entries, keeping the double thresholds
    double av[8];
    int32_t cv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t idx = (size_t)sd.off + (size_t)(i0 + (k < count ? k : count - 1)) * 8 + e;
      av[k] = P.vals[idx];
      cv[k] = P.cols[idx];
    }
    double2 bv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) bv[k] = cur[(size_t)(cv[k] & kColMask) * kNodeGroup + t];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < count && on && av[k] != 0.0) {
        const double2 b = bv[k];
        accumulate(av[k], b.x, b.y, L.smin, L.smax, L.cmin, L.cmax);
        const bool is_int = cv[k] < 0, pos = av[k] > 0.0;
        const double t1 = side_threshold(av[k], b.x, b.y, is_int, pos, P.cont_rel_tol);
        const double t2 = side_threshold(av[k], b.x, b.y, is_int, !pos, P.cont_rel_tol);
        tmin = t1 > tmin ? t1 : tmin;
        tmax = t2 > tmax ? t2 : tmax;
      }
    }
  }
  slot_reduce(L, 3);
#pragma unroll
  for (int off = 8; off < kWave; off <<= 1) {
    const double o1 = __shfl_xor(tmin, off, kWave);
    const double o2 = __shfl_xor(tmax, off, kWave);
    tmin = o1 > tmin ? o1 : tmin;
    tmax = o2 > tmax ? o2 : tmax;
  }
  if (e == 0 && on) {
    SegPartial q;
    q.min_hi = L.smin.hi;
    q.min_lo = L.smin.lo;
    q.max_hi = L.smax.hi;
    q.max_lo = L.smax.lo;
    q.tmin = tmin;
    q.tmax = tmax;
    q.min_inf = L.cmin;
    q.max_inf = L.cmax;
    q.pad0 = q.pad1 = 0;
    parts[(size_t)s * pstride + node0 + t] = q;
  }
}

__device__ __forceinline__ void seg_phase2(const Problem& P, int s,
                                           const double2* __restrict__ cur,
                                           double2* __restrict__ nxt, uint32_t stride, uint32_t t,
                                           const SegPartial* parts, uint32_t pstride,
                                           uint32_t node) {
  const int lane = threadIdx.x & (kWave - 1);
  const SegDesc sd = P.segs[s];
  DD smin = {0.0, 0.0}, smax = {0.0, 0.0};
  int cmin = 0, cmax = 0;
  for (int q = lane; q < sd.nseg; q += kWave) {
    const SegPartial pp = parts[(size_t)(sd.first + q) * pstride + node];
    dd_add(smin, pp.min_hi, pp.min_lo);
    dd_add(smax, pp.max_hi, pp.max_lo);
    cmin += pp.min_inf;
    cmax += pp.max_inf;
  }
  group_reduce(smin, smax, cmin, cmax, 6);
  const RowState R = make_row_state(smin, smax, cmin, cmax, P.lhs[sd.row], P.rhs[sd.row]);
  const SegPartial own = parts[(size_t)s * pstride + node];
  bool need = false;
  if (R.min_side) need |= (R.cmin == 0) ? !(R.smn > own.tmin) : (own.min_inf > 0);
  if (R.max_side) need |= (R.cmax == 0) ? !((-R.smx) > own.tmax) : (own.max_inf > 0);
  if (!need) return;
  for (int p = lane; p < sd.len; p += kWave) {
    const double a = P.vals[sd.off + p];
    if (a == 0.0) continue;
    const int32_t cw = P.cols[sd.off + p];
    const double2 b = cur[(size_t)(cw & kColMask) * stride + t];
    if (entry_wanted(R, a, b.x, b.y, cw, P.cont_rel_tol))
      entry_candidates(P, R, a, b.x, b.y, cw, nxt + t, stride, stride == 1);
  }
}

// ---------------------------------------------------------------------------
// commit: copy changed pairs B -> A, count them, check their domains
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t u32_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-thread part over a grid-stride range.
__device__ __forceinline__ void commit_range(const Problem& P, uint32_t tid, uint32_t nthreads,
                                             uint32_t& changed, uint32_t& infeasible) {
  double2* A = P.bnd[0];
  double2* B = P.bnd[1];
  for (uint32_t v = tid; v < (uint32_t)P.n; v += nthreads) {
    const double2 a = A[v];
    double2 b;
    if (v < (uint32_t)P.n_hot) {
      // a hot variable's candidates sit in its stripe copies (B is not a
      // target for it): merge them into the committed pair, reset them
      b = a;
      double2* st = P.stripes + v;
#pragma unroll 8
      for (int c = 0; c < kStripes; ++c) {
        const double2 q = st[(size_t)c * P.n_hot];
        b.x = q.x > b.x ? q.x : b.x;
        b.y = q.y < b.y ? q.y : b.y;
      }
#pragma unroll 8
      for (int c = 0; c < kStripes; ++c)
        st[(size_t)c * P.n_hot] = make_double2(-__builtin_inf(), __builtin_inf());
    } else {
      b = B[v];
    }
    if (a.x != b.x || a.y != b.y) {
      A[v] = b;
      B[v] = b;
      ++changed;
      if (domain_empty(P.vtype[v] != 0, b.x, b.y, P.feas_tol)) infeasible = 1;
    }
  }
}

// Block-wide sums; every thread gets the totals.
__device__ __forceinline__ void block_sum2(uint32_t& x, uint32_t& y) {
  __shared__ uint32_t sx[kWavesPerBlock], sy[kWavesPerBlock];
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    x += __shfl_xor(x, off, kWave);
    y += __shfl_xor(y, off, kWave);
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sx[wave] = x;
    sy[wave] = y;
  }
  __syncthreads();
  x = 0;
  y = 0;
#pragma unroll
  for (int q = 0; q < kWavesPerBlock; ++q) {
    x += sx[q];
    y += sy[q];
  }
}

// Status after round r from the round's totals (single thread).
__device__ __forceinline__ void end_of_round(const Problem& P, int r, int max_rounds,
                                             uint32_t changed, uint32_t infeasible) {
  Ctrl* C = P.ctrl;
  C->round = r + 1;
  if (infeasible) {
    C->status = kInfeasible;
    C->rounds = r;
    C->done = 1;
  } else if (changed == 0) {
    C->status = kConverged;
    C->rounds = r;
    C->done = 1;
  } else if (r >= max_rounds) {
    C->status = kMaxRounds;
    C->rounds = r;
    C->done = 1;
  }
}

// Round-0 decision, shared by all drivers (single thread).
__device__ __forceinline__ void start_status(const Problem& P, int max_rounds) {
  Ctrl* C = P.ctrl;
  C->round = 1;
  if (u32_load(&C->invalid) || u32_load(&C->infeasible) || P.instance_infeasible) {
    C->status = kInfeasible;
    C->rounds = 0;
    C->done = 1;
  } else if (max_rounds == 0) {
    C->status = kMaxRounds;
    C->rounds = 0;
    C->done = 1;
  }
}

// packed commit counter: bits 0-31 changed pairs, 32-47 blocks that saw an
// empty domain, 48-63 blocks finished
constexpr uint64_t kCommitBlock = 1ull << 48;
constexpr uint64_t kCommitInf = 1ull << 32;

// ---------------------------------------------------------------------------
// grid barrier for the persistent driver (sense-reversing, bounded wait)
// ---------------------------------------------------------------------------
#define PROP_SPIN_LIMIT (1u << 26)

// What the last block to arrive at a barrier does before releasing the rest.
enum BarrierAction { kActNone = 0, kActStart = 1, kActEndRound = 2 };

// All threads of all blocks call this.  The action runs on the last
// arriving block's thread 0 before the others are released.  Returns false
// when the wait gave up (every block then leaves its loop).
__device__ __forceinline__ bool grid_barrier(const Problem& P, int action, int r, int max_rounds) {
  Ctrl* C = P.ctrl;
  __syncthreads();
  __shared__ uint32_t ok_shared;
  if (threadIdx.x == 0) {
    __threadfence();
    uint32_t ok = 1;
    const uint32_t g = __hip_atomic_load(&C->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t prev =
        __hip_atomic_fetch_add(&C->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
      if (action == kActStart) {
        start_status(P, max_rounds);
      } else if (action == kActEndRound) {
        const uint64_t w =
            __hip_atomic_load(&C->commit_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        end_of_round(P, r, max_rounds, (uint32_t)w, (uint32_t)((w >> 32) & 0xffff));
        __hip_atomic_store(&C->commit_word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_store(&C->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&C->bar_gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&C->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > PROP_SPIN_LIMIT ||
            __hip_atomic_load(&C->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(&C->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
    ok_shared = ok;
  }
  __syncthreads();
  return ok_shared != 0;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_init(Problem P) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl* C = P.ctrl;
    C->commit_word = 0;
    C->infeasible = 0;
    C->invalid = 0;
    C->status = kMaxRounds;
    C->rounds = 0;
    C->done = 0;
    C->round = 1;
    C->bar_count = 0;
    C->bar_gen = 0;
    C->abort = 0;
  }
}

// Validate, integer-round and relabel the caller's bounds into both arrays.
__global__ __launch_bounds__(kBlock) void k_pack(Problem P, const double* __restrict__ ulb,
                                                 const double* __restrict__ uub) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)P.n; v += stride) {
    double l = ulb[v], u = uub[v];
    const bool bad = __builtin_isnan(l) || __builtin_isnan(u) || l == __builtin_inf() ||
                     u == -__builtin_inf() ||
                     (!is_inf(l) && __builtin_fabs(l) > PROP_HUGE) ||
                     (!is_inf(u) && __builtin_fabs(u) > PROP_HUGE);
    if (bad) __hip_atomic_store(&P.ctrl->invalid, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t j = P.perm[v];
    const bool is_int = P.vtype[j] != 0;
    if (is_int) {
      l = __builtin_ceil(l - P.eps_int);
      u = __builtin_floor(u + P.eps_int);
    }
    l = l + 0.0;
    u = u + 0.0;
    const double2 b = make_double2(l, u);
    P.bnd[0][j] = b;
    P.bnd[1][j] = b;
    if (domain_empty(is_int, l, u, P.feas_tol))
      __hip_atomic_store(&P.ctrl->infeasible, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kBlock) void k_reset_stripes(Problem P) {
  const size_t total = (size_t)kStripes * P.n_hot;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    P.stripes[i] = make_double2(-__builtin_inf(), __builtin_inf());
}

__global__ __launch_bounds__(kBlock) void k_unpack(Problem P, double* __restrict__ ulb,
                                                   double* __restrict__ uub) {
  const double2* src = P.bnd[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)P.n; v += stride) {
    const double2 b = src[P.perm[v]];
    ulb[v] = b.x;
    uub[v] = b.y;
  }
}

// ---- persistent driver: every round inside one cooperative launch -------
__global__ __launch_bounds__(kBlock) void k_persistent(Problem P, int max_rounds) {
  Ctrl* C = P.ctrl;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gwave = blockIdx.x * kWavesPerBlock + wave;
  const int nwaves = gridDim.x * kWavesPerBlock;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nthreads = gridDim.x * blockDim.x;
  const double2* A = P.bnd[0];
  double2* B = P.bnd[1];

  if (!grid_barrier(P, kActStart, 0, max_rounds)) return;
  if (u32_load(&C->done)) return;

  for (int r = 1; r <= max_rounds; ++r) {
    for (int c = gwave; c < P.n_chunks; c += nwaves) chunk_dispatch(P, c, A, B, 1, 1);
    if (P.n_segs) {
      for (int s = gwave; s < P.n_segs; s += nwaves) seg_phase1(P, s, A, 1, 1, P.partials, 1, 0);
      if (!grid_barrier(P, kActNone, r, max_rounds)) return;
      for (int s = gwave; s < P.n_segs; s += nwaves)
        seg_phase2(P, s, A, B, 1, 0, P.partials, 1, 0);
    }
    if (!grid_barrier(P, kActNone, r, max_rounds)) return;
    uint32_t changed = 0, infeasible = 0;
    commit_range(P, tid, nthreads, changed, infeasible);
    block_sum2(changed, infeasible);
    if (threadIdx.x == 0 && (changed || infeasible))
      __hip_atomic_fetch_add(&C->commit_word,
                             (uint64_t)changed | (infeasible ? kCommitInf : 0ull),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(P, kActEndRound, r, max_rounds)) return;
    if (u32_load(&C->done)) return;
  }
}

// ---- stream / host drivers: one launch per phase, early exit when done ----
__global__ void k_start(Problem P, int max_rounds) {
  if (blockIdx.x == 0 && threadIdx.x == 0) start_status(P, max_rounds);
}

__global__ __launch_bounds__(kBlock) void k_round(Problem P) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = blockIdx.x * kWavesPerBlock + wave;
  if (item < P.n_segs) seg_phase1(P, item, P.bnd[0], 1, 1, P.partials, 1, 0);
  else if (item - P.n_segs < P.n_chunks)
    chunk_dispatch(P, item - P.n_segs, P.bnd[0], P.bnd[1], 1, 1);
}

__global__ __launch_bounds__(kBlock) void k_round_long(Problem P) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = blockIdx.x * kWavesPerBlock + wave;
  if (s < P.n_segs) seg_phase2(P, s, P.bnd[0], P.bnd[1], 1, 0, P.partials, 1, 0);
}

// Commit of round r; the last block to finish decides the status.
__global__ __launch_bounds__(kBlock) void k_commit(Problem P, int r, int max_rounds) {
  Ctrl* C = P.ctrl;
  if (u32_load(&C->done)) return;
  uint32_t changed = 0, infeasible = 0;
  commit_range(P, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, changed,
               infeasible);
  block_sum2(changed, infeasible);
  if (threadIdx.x == 0) {
    const uint64_t add = kCommitBlock | (uint64_t)changed | (infeasible ? kCommitInf : 0ull);
    const uint64_t old =
        __hip_atomic_fetch_add(&C->commit_word, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((old >> 48) == gridDim.x - 1u) {
      const uint64_t tot = old + add;
      end_of_round(P, r, max_rounds, (uint32_t)tot, (uint32_t)((tot >> 32) & 0xffff));
      __hip_atomic_store(&C->commit_word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}


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

// Packs nodes [k0, k0 + cnt) from node-major arrays (row q = node k0 + q).
__global__ __launch_bounds__(kBlock) void k_pack_batch(Problem P, Batch Bt,
                                                       const double* __restrict__ ulb,
                                                       const double* __restrict__ uub, int k0,
                                                       int cnt) {
  const size_t total = (size_t)cnt * P.n;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int q = (int)(i / (size_t)P.n);
    const int k = k0 + q;
    const int v = (int)(i - (size_t)q * P.n);
    double l = ulb[i], u = uub[i];
    const bool bad = __builtin_isnan(l) || __builtin_isnan(u) || l == __builtin_inf() ||
                     u == -__builtin_inf() ||
                     (!is_inf(l) && __builtin_fabs(l) > PROP_HUGE) ||
                     (!is_inf(u) && __builtin_fabs(u) > PROP_HUGE);
    if (bad) __hip_atomic_store(&Bt.invalid[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t j = P.perm[v];
    const bool is_int = P.vtype[j] != 0;
    if (is_int) {
      l = __builtin_ceil(l - P.eps_int);
      u = __builtin_floor(u + P.eps_int);
    }
    l = l + 0.0;
    u = u + 0.0;
    const size_t dst = (size_t)j * kNodeGroup + (k % kNodeGroup);
    const double2 b = make_double2(l, u);
    Bt.gA[k / kNodeGroup][dst] = b;
    Bt.gB[k / kNodeGroup][dst] = b;
    if (domain_empty(is_int, l, u, P.feas_tol))
      __hip_atomic_store(&Bt.infeasible[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  if (threadIdx.x == 0) P.ctrl->done = my_active == 0 ? 1u : 0u;
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
    Bt.changed[k] = 0;
    Bt.infeasible[k] = 0;
    Bt.invalid[k] = 0;
    act += a;
  }
  if (whole) batch_set_done(P, act);
  else if (threadIdx.x == 0) P.ctrl->done = 0;
}

__global__ __launch_bounds__(kBlock) void k_round_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const int unit = (int)(wid / Bt.groups);
  const int g = (int)(wid - (int64_t)unit * Bt.groups);
  if (unit >= P.n_segs + P.n_chunks) return;
  const uint32_t mask = group_mask(Bt, g);
  if (!mask) return;
  // with few active nodes, node-parallel lanes would mostly idle: loop over
  // the active nodes with the single-run shape instead
  const bool few = __builtin_popcount(mask) <= kLoopNodes;
  if (unit < P.n_segs) {
    if (few)
      seg_phase1(P, unit, Bt.gA[g], kNodeGroup, mask, Bt.partials, Bt.nodes, g * kNodeGroup);
    else
      seg_phase1_nodes(P, unit, Bt.gA[g], mask, Bt.partials, Bt.nodes, g * kNodeGroup);
  } else {
    if (few)
      chunk_dispatch(P, unit - P.n_segs, Bt.gA[g], Bt.gB[g], kNodeGroup, mask);
    else
      chunk_round_nodes(P, P.chunks[unit - P.n_segs], Bt.gA[g], Bt.gB[g], mask);
  }
}

__global__ __launch_bounds__(kBlock) void k_round_long_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  const int s = (int)(wid / Bt.nodes);
  const int k = (int)(wid - (int64_t)s * Bt.nodes);
  if (s >= P.n_segs || !Bt.active[k]) return;
  const int g = k / kNodeGroup;
  seg_phase2(P, s, Bt.gA[g], Bt.gB[g], kNodeGroup, k % kNodeGroup, Bt.partials, Bt.nodes, k);
}

// Commit per (variable, node) of group blockIdx.y, with per-node counts.
__global__ __launch_bounds__(kBlock) void k_commit_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  __shared__ uint32_t ch[kNodeGroup], inf[kNodeGroup];
  if (threadIdx.x < kNodeGroup) {
    ch[threadIdx.x] = 0;
    inf[threadIdx.x] = 0;
  }
  __syncthreads();
  const int g = blockIdx.y;
  const uint32_t mask = group_mask(Bt, g);
  if (mask) {
    double2* A = Bt.gA[g];
    const double2* B = Bt.gB[g];
    const size_t total = (size_t)P.n * kNodeGroup;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
      const uint32_t t = (uint32_t)(e % kNodeGroup);
      if (!((mask >> t) & 1u)) continue;
      const double2 a = A[e];
      const double2 b = B[e];
      if (a.x != b.x || a.y != b.y) {
        A[e] = b;
        atomicAdd(&ch[t], 1u);
        if (domain_empty(P.vtype[e / kNodeGroup] != 0, b.x, b.y, P.feas_tol)) inf[t] = 1;
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

// One block: per-node status after the round each active node just ran
// (node k's own round count: nodes may have joined at different times).
__global__ __launch_bounds__(kBlock) void k_end_batch(Problem P, Batch Bt) {
  if (u32_load(&P.ctrl->done)) return;
  uint32_t act = 0;
  for (int k = threadIdx.x; k < Bt.nodes; k += blockDim.x) {
    if (!Bt.active[k]) continue;
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
    act += a;
  }
  batch_set_done(P, act);
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------
static int blocks_for(int64_t items, int per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

hipError_t launch_init(const Problem& P, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_pack(const Problem& P, const double* lb, const double* ub, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(blocks_for(P.n, kBlock, 4096)), dim3(kBlock), 0, s, P, lb, ub);
  if (P.n_hot)
    hipLaunchKernelGGL(k_reset_stripes, dim3(blocks_for((int64_t)kStripes * P.n_hot, kBlock, 1024)),
                       dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_unpack(const Problem& P, double* lb, double* ub, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(blocks_for(P.n, kBlock, 4096)), dim3(kBlock), 0, s, P, lb,
                     ub);
  return hipGetLastError();
}

hipError_t persistent_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent, kBlock, 0);
}

hipError_t launch_persistent(const Problem& P, int max_rounds, int grid, hipStream_t s) {
  Problem p = P;
  void* args[] = {(void*)&p, (void*)&max_rounds};
  return hipLaunchCooperativeKernel((const void*)k_persistent, dim3(grid), dim3(kBlock), args, 0,
                                    s);
}

hipError_t launch_start(const Problem& P, int max_rounds, hipStream_t s) {
  hipLaunchKernelGGL(k_start, dim3(1), dim3(64), 0, s, P, max_rounds);
  return hipGetLastError();
}

hipError_t launch_round(const Problem& P, int r, int max_rounds, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  const int items = P.n_chunks + P.n_segs;
  if (e0) hipEventRecord(e0, s);
  hipLaunchKernelGGL(k_round, dim3(blocks_for(items, kWavesPerBlock, 1 << 30)), dim3(kBlock), 0,
                     s, P);
  if (e1) hipEventRecord(e1, s);
  if (P.n_segs)
    hipLaunchKernelGGL(k_round_long, dim3(blocks_for(P.n_segs, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P);
  // at most 65535 blocks: the packed commit counter keeps 16 bits per field
  hipLaunchKernelGGL(k_commit, dim3(blocks_for(P.n, kBlock, 1024)), dim3(kBlock), 0, s, P, r,
                     max_rounds);
  return hipGetLastError();
}

hipError_t launch_pack_batch(const Problem& P, const Batch& Bt, const double* lb, const double* ub,
                             int k0, int cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_batch, dim3(blocks_for((int64_t)cnt * P.n, kBlock, 16384)),
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
  if (P.n_segs)
    hipLaunchKernelGGL(k_round_long_batch,
                       dim3(blocks_for((int64_t)P.n_segs * Bt.nodes, kWavesPerBlock, 1 << 30)),
                       dim3(kBlock), 0, s, P, Bt);
  hipLaunchKernelGGL(k_commit_batch,
                     dim3(blocks_for((int64_t)P.n * kNodeGroup, kBlock, 256), Bt.groups),
                     dim3(kBlock), 0, s, P, Bt);
  hipLaunchKernelGGL(k_end_batch, dim3(1), dim3(kBlock), 0, s, P, Bt);
  return hipGetLastError();
}

}  // namespace prop
