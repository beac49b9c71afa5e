// prop_device.h -- device functions of one synchronous propagation round
// (Sofranac, Gleixner, Pokutta, arXiv 2009.07785, Algorithms 2 and 3),
// shared by the single-run kernels (prop_kernels.hip) and the batched ones
// (prop_batch.hip); every function is inlined into the kernels using it.
// The two kernel files are separate translation units so that the register
// allocation of each kernel depends only on its own paths.
//
// Bounds live in two arrays of (lb, ub) pairs: A holds the bounds as they
// stood at the start of the round and is only read during it; B starts
// equal to A and receives the candidates.  One round:
//   1. every row's min / max activity from A: finite parts as the exact sum
//      of the products rounded once (prop_sum.h: a double-double with an
//      exact error bound, and a fixed-point sum for the rows that bound
//      cannot certify), plus the counts of infinite contributions
//      (Definition 1; Sec. 3.4);
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
#pragma once

#include <hip/hip_runtime.h>

#include "prop_layout.h"
#include "prop_sum.h"

#pragma clang fp contract(off)

namespace prop {

#define PROP_HUGE 0x1p200
#define PROP_SKIP_MARGIN (1.0 + 0x1p-39)
#define PROP_SKIP_FLOOR 0x1p-900

// Combines the partial sums of the 2^klog lanes of each row (klog is the
// same in every lane of the wave, so the branches are uniform); emin / emax
// are the lanes' error bounds of the two sums (see prop_sum.h).
__device__ __forceinline__ void group_reduce(DD& smin, DD& smax, double& emin, double& emax,
                                             int& cmin,
                                             int& cmax, int klog) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    if (i >= klog) break;
    const int off = 1 << i;
    double a = __shfl_xor(smin.hi, off, kWave);
    double b = __shfl_xor(smin.lo, off, kWave);
    double c = __shfl_xor(smax.hi, off, kWave);
    double d = __shfl_xor(smax.lo, off, kWave);
    double f = __shfl_xor(emin, off, kWave);
    double f2 = __shfl_xor(emax, off, kWave);
    int g = __shfl_xor(cmin, off, kWave);
    int h = __shfl_xor(cmax, off, kWave);
    dd_add(smin, emin, a, b, f);
    dd_add(smax, emax, c, d, f2);
    cmin += g;
    cmax += h;
  }
}

__device__ __forceinline__ bool is_inf(double x) { return __builtin_isinf(x); }

// Lane 0's value of x in every lane.
__device__ __forceinline__ double lane0_f64(double x) {
  const uint64_t v = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 0);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 0);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Contribution of one entry to both activities; mmin / mmax are the lane's
// error bounds of the two sums (dd_add_prod).
__device__ __forceinline__ void accumulate(double a, double l, double u, DD& smin, DD& smax,
                                           int& cmin, int& cmax, double& mmin, double& mmax) {
  const double bmin = a > 0.0 ? l : u;
  const double bmax = a > 0.0 ? u : l;
  const bool imin = is_inf(bmin);
  const bool imax = is_inf(bmax);
  cmin += (a != 0.0 && imin) ? 1 : 0;
  cmax += (a != 0.0 && imax) ? 1 : 0;
  dd_add_prod(smin, a, imin ? 0.0 : bmin, mmin);
  dd_add_prod(smax, a, imax ? 0.0 : bmax, mmax);
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
// Straight-line code: every case is computed with the same operations in
// the same order as its own branch would, and selected at the end, so the
// wave runs no divergent branches here.
__device__ __forceinline__ double side_threshold(double a, double l, double u, bool is_int,
                                                 bool upper, double tau) {
  const double bnd = upper ? u : l;  // the bound a candidate would tighten
  const double s = __builtin_fabs(bnd) > 1.0 ? __builtin_fabs(bnd) : 1.0;
  const double wc = upper ? (u - tau * s) - l : u - (l + tau * s);
  const double w = is_int ? u - l : wc;
  double thr = (__builtin_fabs(a) * w) * PROP_SKIP_MARGIN;
  thr = thr >= PROP_SKIP_FLOOR ? thr : __builtin_inf();
  thr = w > 0.0 ? thr : -0x1p-1074;
  // u = +inf (upper) or l = -inf (lower): every finite candidate counts
  return is_inf(bnd) ? __builtin_inf() : thr;
}

__device__ __forceinline__ bool domain_empty(bool is_int, double l, double u, double feas_tol) {
  if (is_int) return l > u;
  double s = __builtin_fabs(l) > __builtin_fabs(u) ? __builtin_fabs(l) : __builtin_fabs(u);
  if (s < 1.0) s = 1.0;
  return (l - u) > feas_tol * s;
}

// ---------------------------------------------------------------------------
// compact bound codes (single runs)
//
// Beside the (l, u) pairs of the start-of-round bounds, a single run keeps a
// 2-byte code per variable that the activity pass gathers for integer
// variables instead of the 16-byte pair: the low byte holds l and the high
// byte u as signed 8-bit integers, with -127 standing for l = -inf and 127
// for u = +inf.  A variable whose bounds do not fit (a bound outside
// [-126, 126] or not an integer, or any continuous variable) has the escape
// code (low byte -128), and its entries gather the pair.  Every code decodes
// to the exact doubles of the pair; the pack kernel writes the codes and the
// commit rewrites the code of every variable it changes.  With 2 bytes per
// variable instead of 16 the bounds that most entries gather take an eighth
// of the cache space, and a 64-lane gather touches that many fewer lines.
// ---------------------------------------------------------------------------
constexpr uint16_t kCodeEscape = 0x0080;

__device__ __forceinline__ uint16_t bound_code(bool is_int, double l, double u) {
  const bool lok = l == -__builtin_inf() || (l >= -126.0 && l <= 126.0 && l == __builtin_floor(l));
  const bool uok = u == __builtin_inf() || (u >= -126.0 && u <= 126.0 && u == __builtin_floor(u));
  if (!(is_int && lok && uok)) return kCodeEscape;
  const int lb = l == -__builtin_inf() ? -127 : (int)l;
  const int ub = u == __builtin_inf() ? 127 : (int)u;
  return (uint16_t)((uint32_t)(lb & 0xff) | ((uint32_t)(ub & 0xff) << 8));
}

// Bounds of a code; false for the escape code (the pair must be gathered).
__device__ __forceinline__ bool decode_code(uint16_t w, double& l, double& u) {
  const int lb = (int)(int8_t)(w & 0xff);
  const int ub = (int)(int8_t)(w >> 8);
  l = lb == -127 ? -__builtin_inf() : (double)lb;
  u = ub == 127 ? __builtin_inf() : (double)ub;
  return lb != -128;
}

// ---------------------------------------------------------------------------
// Single-precision bound store (Problem::store32; Sec. 4.5 of the paper runs
// the whole method in single precision and loses correctness).  Here the
// arithmetic stays FP64; only the stored bounds move to the grid of zero,
// the infinities and the normal singles, rounded outward: a lower bound to
// the largest grid member not above it, an upper bound to the smallest not
// below it.  Outward rounding only loosens a bound, so every point the FP64
// store keeps is kept; integers below 2^24 are grid members.  The rounding
// happens at the pack and at every commit, before the change test.
// ---------------------------------------------------------------------------
// Each result is taken from a branch of its own, never by negating the
// other direction's result: a zero then comes from the literal +0, and no
// sign change is left for the compiler to fold into a later conversion.
// Near a representable single, the conversion to nearest is at most one
// grid step off; a normal single's neighbour is one step of its bit pattern
// (towards zero the magnitude shrinks, away from it it grows).
__device__ __forceinline__ float store_down32(double x) {
  float f;
  if (is_inf(x)) f = x > 0.0 ? __builtin_inff() : -__builtin_inff();
  else if (x > (double)__FLT_MAX__) f = __FLT_MAX__;
  else if (x < -(double)__FLT_MAX__) f = -__builtin_inff();
  else if (x >= 0.0 && x < (double)__FLT_MIN__) f = 0.0f;  // both zeros too
  else if (x < 0.0 && x > -(double)__FLT_MIN__) f = -__FLT_MIN__;
  else {
    f = (float)x;
    if ((double)f > x) f = __int_as_float(__float_as_int(f) + (f > 0.0f ? -1 : 1));
  }
  return f;
}

__device__ __forceinline__ float store_up32(double x) {
  float f;
  if (is_inf(x)) f = x > 0.0 ? __builtin_inff() : -__builtin_inff();
  else if (x < -(double)__FLT_MAX__) f = -__FLT_MAX__;
  else if (x > (double)__FLT_MAX__) f = __builtin_inff();
  else if (x <= 0.0 && x > -(double)__FLT_MIN__) f = 0.0f;  // both zeros too
  else if (x > 0.0 && x < (double)__FLT_MIN__) f = __FLT_MIN__;
  else {
    f = (float)x;
    if ((double)f < x) f = __int_as_float(__float_as_int(f) + (f > 0.0f ? 1 : -1));
  }
  return f;
}

// Fire-and-forget FP64 atomics (the result is unused, so no wave waits).
__device__ __forceinline__ void atomic_max_f64(double* p, double v) {
  (void)__hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_min_f64(double* p, double v) {
  (void)__hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Touch bytes of the candidate block whose first pair is nxt (n x stride
// pairs; prop_layout.h).
__device__ __forceinline__ uint8_t* touch_of(const Problem& P, double2* nxt, uint32_t stride) {
  return reinterpret_cast<uint8_t*>(nxt + (size_t)(P.n > 0 ? P.n : 1) * stride);
}

// Row-level quantities every entry of a row needs.
struct RowState {
  double minfin, maxfin;
  int cmin, cmax;
  bool min_side, max_side;  // the rhs / lhs side can yield candidates
  bool uncertain;           // a side in use needs the exact path
  double smn;               // rhs - min activity
  double smx;               // lhs - max activity
};
static_assert(sizeof(RowState) == kRowStateBytes, "RowState size (batch row-state buffers)");

// Row state from the reduced double-doubles; `force` sends the row to the
// exact path whatever the certification says (a tiny bound is in play).
__device__ __forceinline__ RowState make_row_state(const DD& smin, const DD& smax, double emin,
                                                   double emax,
                                                   int cmin, int cmax, double lhs, double rhs,
                                                   bool force) {
  RowState R;
  const bool okmin = dd_round(smin.hi, smin.lo, emin, R.minfin);
  const bool okmax = dd_round(smax.hi, smax.lo, emax, R.maxfin);
  R.cmin = cmin;
  R.cmax = cmax;
  R.min_side = (rhs < __builtin_inf()) && cmin <= 1;
  R.max_side = (lhs > -__builtin_inf()) && cmax <= 1;
  R.uncertain = force || (R.min_side && !okmin) || (R.max_side && !okmax);
  R.smn = rhs - R.minfin;
  R.smx = lhs - R.maxfin;
  return R;
}

__device__ __forceinline__ void set_exact(RowState& R, double mn, double mx, double lhs,
                                          double rhs) {
  R.minfin = mn;
  R.maxfin = mx;
  R.smn = rhs - mn;
  R.smx = lhs - mx;
  R.uncertain = false;
}

// ---------------------------------------------------------------------------
// exact path (rows the fast sums cannot certify; see prop_sum.h)
//
// The lanes holding the row's entries add their exact products into two
// digit arrays in LDS (min and max activity) with 64-bit integer atomics,
// and one lane rounds them.  The wave runs it for one row at a time; its
// other lanes wait.  Rows get here when their double-double sum lies within
// its error bound of a rounding boundary, so this path is rare.
// ---------------------------------------------------------------------------
struct ExactScratch {
  int64_t w[2][kAccDigits];
  double out[2];
};

__device__ __forceinline__ ExactScratch& exact_scratch() {
  __shared__ ExactScratch sc[kWavesPerBlock];
  return sc[threadIdx.x >> 6];
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void exact_clear(ExactScratch& X) {
  const int lane = threadIdx.x & (kWave - 1);
  if (lane < kAccDigits) {
    X.w[0][lane] = 0;
    X.w[1][lane] = 0;
  }
  wave_sync();
}

__device__ __forceinline__ void lds_add_product(int64_t* W, double a, double b) {
  int d;
  uint32_t c[5];
  bool neg;
  if (!product_digits(a, b, d, c, neg)) return;
#pragma unroll
  for (int i = 0; i < 5; ++i)
    if (c[i])
      atomicAdd(reinterpret_cast<unsigned long long*>(&W[d + i]),
                neg ? (unsigned long long)(-(int64_t)c[i]) : (unsigned long long)c[i]);
}

// One entry's exact products into both digit arrays (infinite bounds are
// counted elsewhere and contribute no finite part).
__device__ __forceinline__ void exact_entry(ExactScratch& X, double a, double l, double u) {
  if (a == 0.0) return;
  const double bmin = a > 0.0 ? l : u;
  const double bmax = a > 0.0 ? u : l;
  if (!is_inf(bmin)) lds_add_product(X.w[0], a, bmin);
  if (!is_inf(bmax)) lds_add_product(X.w[1], a, bmax);
}

// After every lane has added: `leader` rounds both sums; every lane gets them.
__device__ __forceinline__ void exact_finish(ExactScratch& X, bool leader, double& mn,
                                             double& mx) {
  wave_sync();
  if (leader) {
    X.out[0] = digits_round(X.w[0]);
    X.out[1] = digits_round(X.w[1]);
  }
  wave_sync();
  mn = X.out[0];
  mx = X.out[1];
  wave_sync();
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
// With `striped`, variables below P.n_hot write to this block's stripe copy
// (the commit merges them); for every variable with a side that may
// count, the variable's touch byte is set (`touch`: the block's, from
// touch_of).
__device__ __forceinline__ void entry_candidates(const Problem& P, const RowState& R, double a,
                                                 double l, double u, int32_t cw,
                                                 double2* __restrict__ nxt, uint32_t stride,
                                                 bool striped, uint8_t* __restrict__ touch) {
  bool dmin, dmax;
  entry_sides(R, a, l, u, cw, P.cont_rel_tol, dmin, dmax);
  if (!(dmin || dmax)) return;
  const int32_t var = cw & kColMask;
  size_t j = (size_t)var * stride;
  if (striped && var < P.n_hot) {
    nxt = P.stripes + (size_t)(blockIdx.x % kStripes) * P.n_hot;
    j = (size_t)var;
  }
  // set before the candidates are known: a byte set with nothing written
  // only costs the commit a compare
  touch[var >> 3] = 1;
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

struct LaneAcc {
  DD smin, smax;
  double emin, emax;  // error bounds of the two sums (prop_sum.h)
  int cmin, cmax;
  double tmin, tmax;  // largest skip threshold per side (side_threshold)
  bool omin, omax;    // holds the owner of the side's infinite contribution
};

__device__ __forceinline__ void lane_acc_init(LaneAcc& L) {
  L.smin = {0.0, 0.0};
  L.smax = {0.0, 0.0};
  L.emin = L.emax = 0.0;
  L.cmin = L.cmax = 0;
  L.tmin = L.tmax = -__builtin_inf();
  L.omin = L.omax = false;
}

// One entry's thresholds into the lane's per-side maxima (side_threshold);
// an entry whose bound makes a side's activity infinite owns that side's
// only infinite contribution when the row has exactly one.
__device__ __forceinline__ void lane_thresholds(LaneAcc& L, double a, double l, double u,
                                                bool is_int, double tau) {
  const bool pos = a > 0.0;
  const double t1 = side_threshold(a, l, u, is_int, pos, tau);
  const double t2 = side_threshold(a, l, u, is_int, !pos, tau);
  L.tmin = t1 > L.tmin ? t1 : L.tmin;
  L.tmax = t2 > L.tmax ? t2 : L.tmax;
  L.omin |= is_inf(pos ? l : u);
  L.omax |= is_inf(pos ? u : l);
}

__device__ __forceinline__ bool lane_may_pass(const RowState& R, const LaneAcc& L) {
  bool p = false;
  if (R.min_side) p |= R.cmin == 0 ? !(R.smn > L.tmin) : L.omin;
  if (R.max_side) p |= R.cmax == 0 ? !((-R.smx) > L.tmax) : L.omax;
  return p;
}

// ---------------------------------------------------------------------------
// one chunk: activities and candidates for 64/K rows, K lanes per row
//
// Bound arrays are addressed as base[var * stride + node]: stride 1 for a
// single problem, 8 for a batch (8 nodes share each variable's cache line).
// Per active node (bit t of node_mask) each step loads its coefficient and
// column word, gathers the bounds (a single run gathers the 2-byte codes of
// integer variables), adds the entry to the activities and folds its skip
// thresholds into the lane's per-side maxima; after the row reduction, only
// lanes whose maxima do not rule out every entry reload their entries and
// run the exact candidate test.  Keeping two doubles per lane instead of
// anything per step keeps the wave's register count, and with it the
// number of resident waves hiding the gather latency, in line with a plain
// sparse product.  In a batch, nodes after the first find the chunk's
// matrix data in cache.
// ---------------------------------------------------------------------------
// Exact path for row rr of a chunk (lanes rr * K .. rr * K + K - 1) and
// node t: the exactly rounded activities replace the row state of those
// lanes, which then run the candidates of their entries.
__device__ __forceinline__ void exact_chunk_row(const Problem& P, const ChunkDesc cd, int rr,
                                                const double2* __restrict__ cur,
                                                double2* __restrict__ nxt, uint32_t stride,
                                                uint32_t t, RowState& R, double lhs,
                                                double rhs) {
  const int lane = threadIdx.x & (kWave - 1);
  const int klog = cd.meta & 7;
  const int W = (cd.meta >> 8) & 0xff;
  const size_t base = (size_t)cd.off64 * kWave + lane;
  const bool mine = (lane >> klog) == rr;
  ExactScratch& X = exact_scratch();
  exact_clear(X);
  if (mine) {
    for (int w = 0; w < W; ++w) {
      const size_t e = base + (size_t)w * kWave;
      const double a = P.vals[e];
      if (a == 0.0) continue;
      const double2 b = cur[(size_t)(P.cols[e] & kColMask) * stride + t];
      exact_entry(X, a, b.x, b.y);
    }
  }
  double mn, mx;
  exact_finish(X, lane == (rr << klog), mn, mx);
  if (!mine) return;
  set_exact(R, mn, mx, lhs, rhs);
  if (!(R.min_side || R.max_side)) return;
  for (int w = 0; w < W; ++w) {
    const size_t e = base + (size_t)w * kWave;
    const double a = P.vals[e];
    if (a == 0.0) continue;
    const int32_t cw = P.cols[e];
    const double2 b = cur[(size_t)(cw & kColMask) * stride + t];
    entry_candidates(P, R, a, b.x, b.y, cw, nxt + t, stride, stride == 1,
                     touch_of(P, nxt, stride));
  }
}

// Steps of a chunk handled together in the activity pass: their
// coefficients and column words are loaded first, then their bounds are
// gathered, then they are added, so a wave waits for two memory round trips
// per kStepGroup steps instead of three per step (one more for integer
// variables whose code escapes): groups of 2 measured 416 us per round on
// the 5,000,000 x 2,000,000 instance, against 431 for 1 and 434 for 4.
// Padding entries (zero coefficient) hold column 0, a valid variable, so
// their gathers need no guard; they contribute nothing.
constexpr int kStepGroup = 2;
static_assert(kStepGroup == 1 || kStepGroup == 2 || kStepGroup == 4,
              "lane_steps handles remainders of up to 3 steps");

// Where the activity pass finds start-of-round bounds: the pair arrays
// (batches), integer variables' codes and the FP64 pairs of the rest (single
// runs), or codes and the single-precision copies (single runs with the
// single-precision store; the copies hold the pairs' exact values).
constexpr int kSrcPairs = 0;
constexpr int kSrcCodes = 1;
constexpr int kSrcCodes32 = 2;

// Bounds of variable word cw for node t, from the pairs or, with kSrcCodes32,
// from the single-precision copies.
template <int kSrc>
__device__ __forceinline__ double2 pair_of(const double2* __restrict__ cur,
                                           const float2* __restrict__ c32, int32_t cw,
                                           uint32_t stride, uint32_t t) {
  if (kSrc == kSrcCodes32) {
    const float2 f = c32[cw & kColMask];
    return make_double2((double)f.x, (double)f.y);
  }
  return cur[(size_t)(cw & kColMask) * stride + t];
}

// Start-of-round bounds of N entries (column words cv): with codes, an
// integer variable's 2-byte code (its pair only on escape) and a continuous
// variable's pair; otherwise the pairs.  All first gathers are issued before
// any escape gather.
template <int N, int kSrc>
__device__ __forceinline__ void gather_bounds(const double2* __restrict__ cur,
                                              const float2* __restrict__ c32,
                                              const uint16_t* __restrict__ codes,
                                              const int32_t* cv, uint32_t stride, uint32_t t,
                                              double2* bv) {
  if (kSrc != kSrcPairs) {
    bool pair[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      pair[k] = cv[k] >= 0;
      if (!pair[k]) {
        const uint16_t w = codes[cv[k] & kColMask];
        pair[k] = !decode_code(w, bv[k].x, bv[k].y);
      }
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
      if (pair[k]) bv[k] = pair_of<kSrc>(cur, c32, cv[k], stride, t);
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) bv[k] = cur[(size_t)(cv[k] & kColMask) * stride + t];
  }
}

template <int N, int kSrc>
__device__ __forceinline__ void chunk_steps(const Problem& P, const double2* __restrict__ cur,
                                            const uint16_t* __restrict__ codes, uint32_t stride,
                                            uint32_t t, size_t e0, LaneAcc& L) {
  double av[N];
  int32_t cv[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const size_t e = e0 + (size_t)k * kWave;
    // a single run reads the matrix once: stream it past the caches
    av[k] = stride == 1 ? __builtin_nontemporal_load(P.vals + e) : P.vals[e];
    cv[k] = stride == 1 ? __builtin_nontemporal_load(P.cols + e) : P.cols[e];
  }
  double2 bv[N];
  gather_bounds<N, kSrc>(cur, P.b32, codes, cv, stride, t, bv);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (av[k] != 0.0) {
      accumulate(av[k], bv[k].x, bv[k].y, L.smin, L.smax, L.cmin, L.cmax, L.emin, L.emax);
      lane_thresholds(L, av[k], bv[k].x, bv[k].y, cv[k] < 0, P.cont_rel_tol);
    }
  }
}

// The activity pass over W steps of one lane, starting at entry e0.
template <int kSrc>
__device__ __forceinline__ void lane_steps(const Problem& P, const double2* __restrict__ cur,
                                           const uint16_t* __restrict__ codes, uint32_t stride,
                                           uint32_t t, size_t e0, int W, LaneAcc& L) {
  int w0 = 0;
  for (; w0 + kStepGroup <= W; w0 += kStepGroup)
    chunk_steps<kStepGroup, kSrc>(P, cur, codes, stride, t, e0 + (size_t)w0 * kWave, L);
  // W is the same in every lane
  switch (W - w0) {
    case 3: chunk_steps<3, kSrc>(P, cur, codes, stride, t, e0 + (size_t)w0 * kWave, L); break;
    case 2: chunk_steps<2, kSrc>(P, cur, codes, stride, t, e0 + (size_t)w0 * kWave, L); break;
    case 1: chunk_steps<1, kSrc>(P, cur, codes, stride, t, e0 + (size_t)w0 * kWave, L); break;
    default: break;
  }
}

// With `marked` (marked rounds), rows whose stamp in `marks` is not r are
// skipped: none of their variables changed in the previous round, so their
// activities and candidates are those of that round, which changed nothing.
// Bit t of `exact_mask` sends every row of node t to the exact path (a tiny
// bound is in play).
//
// Each lane keeps, besides its sums, the largest skip threshold of its
// entries per side and whether it holds the owner of a side's infinite
// contribution (LaneAcc): "slack > largest threshold" skips every entry of
// the lane exactly as the per-entry test would, so only lanes holding an
// entry that may count revisit their entries, with the exact test.
template <int kSrc>
__device__ __forceinline__ void chunk_round(const Problem& P, const ChunkDesc cd,
                                            const double2* __restrict__ cur,
                                            double2* __restrict__ nxt, uint32_t stride,
                                            uint32_t node_mask, uint32_t exact_mask,
                                            bool marked = false, int r_round = 0,
                                            const int32_t* marks = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  const int klog = cd.meta & 7;
  const int W = (cd.meta >> 8) & 0xff;
  const int nrows = (cd.meta >> 16) & 0xff;
  const int r = lane >> klog;
  const size_t base = (size_t)cd.off64 * kWave + lane;
  const bool row_ok = r < nrows;
  const int row = cd.row0 + (row_ok ? r : 0);
  const bool want = !marked || (row_ok && marks[row] == r_round);
  if (marked && __ballot(want) == 0) return;
  const double lhs = P.lhs[row], rhs = P.rhs[row];
  for (uint32_t mask = node_mask; mask; mask &= mask - 1) {
    const uint32_t t = __builtin_ctz(mask);
    LaneAcc L;
    lane_acc_init(L);
    if (want) lane_steps<kSrc>(P, cur, P.codes, stride, t, base, W, L);
    group_reduce(L.smin, L.smax, L.emin, L.emax, L.cmin, L.cmax, klog);
    RowState R = make_row_state(L.smin, L.smax, L.emin, L.emax, L.cmin, L.cmax, lhs, rhs,
                                (exact_mask >> t) & 1u);
    const bool live = row_ok && want;
    if (live && !R.uncertain && lane_may_pass(R, L)) {
      // four entries at a time: loads, then gathers, then the exact tests
      for (int w0 = 0; w0 < W; w0 += 4) {
        const int cnt = W - w0 < 4 ? W - w0 : 4;
        double av[4];
        int32_t cv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const size_t e = base + (size_t)(w0 + (k < cnt ? k : cnt - 1)) * kWave;
          av[k] = P.vals[e];
          cv[k] = P.cols[e];
        }
        double2 bv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) bv[k] = pair_of<kSrc>(cur, P.b32, cv[k], stride, t);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < cnt && av[k] != 0.0)
            entry_candidates(P, R, av[k], bv[k].x, bv[k].y, cv[k], nxt + t, stride, stride == 1,
                             touch_of(P, nxt, stride));
      }
    }
    // rows the fast sums cannot certify, one at a time with the whole wave
    uint64_t need = __ballot(live && R.uncertain && (lane & ((1 << klog) - 1)) == 0);
    while (need) {
      exact_chunk_row(P, cd, __builtin_ctzll(need) >> klog, cur, nxt, stride, t, R, lhs, rhs);
      need &= need - 1;
    }
  }
}

// kSrc: where the activity pass reads bounds (kSrcPairs for batches, which
// pass their own bound arrays; kSrcCodes / kSrcCodes32 for single runs).
template <int kSrc>
__device__ __forceinline__ void chunk_dispatch(const Problem& P, int c, const double2* cur,
                                               double2* nxt, uint32_t stride,
                                               uint32_t node_mask, uint32_t exact_mask,
                                               bool marked = false, int r_round = 0,
                                               const int32_t* marks = nullptr) {
  chunk_round<kSrc>(P, P.chunks[c], cur, nxt, stride, node_mask, exact_mask, marked, r_round,
                      marks);
}

// ---------------------------------------------------------------------------
// nnz-split waves (single runs; layout in prop_tiles.h)
//
// Lane l walks its 8 consecutive entries, which may hold the end of a row
// begun in earlier lanes (the head piece), whole rows, and the start of a
// row that may go on in later lanes (the open piece).  Whole rows are
// finished as they end.  An inclusive segmented scan over the lanes adds
// the open pieces of a row (a segment starts at the lane where the row
// starts), so the lane where a row ends holds all of it but its own head
// piece; each row's state (slacks, counts, sides) is computed by the lane
// where it ends and handed to the lanes holding its other pieces.  Every
// piece then runs the exact candidate test when the lane's per-piece
// thresholds do not rule it out.  A row the fast sums cannot certify sends
// the whole wave to the exact fixed-point sums, row by row.
// ---------------------------------------------------------------------------
struct Sums {
  DD smin, smax;
  double emin, emax;
  int cmin, cmax;
};

__device__ __forceinline__ Sums sums_of(const LaneAcc& L) {
  return Sums{L.smin, L.smax, L.emin, L.emax, L.cmin, L.cmax};
}

// x = y + x, y the earlier part of the row
__device__ __forceinline__ void sums_prepend(Sums& x, const Sums& y) {
  dd_add(x.smin, x.emin, y.smin.hi, y.smin.lo, y.emin);
  dd_add(x.smax, x.emax, y.smax.hi, y.smax.lo, y.emax);
  x.cmin += y.cmin;
  x.cmax += y.cmax;
}

__device__ __forceinline__ Sums sums_shfl_up(const Sums& x, int d) {
  Sums y;
  y.smin.hi = __shfl_up(x.smin.hi, d, kWave);
  y.smin.lo = __shfl_up(x.smin.lo, d, kWave);
  y.smax.hi = __shfl_up(x.smax.hi, d, kWave);
  y.smax.lo = __shfl_up(x.smax.lo, d, kWave);
  y.emin = __shfl_up(x.emin, d, kWave);
  y.emax = __shfl_up(x.emax, d, kWave);
  y.cmin = __shfl_up(x.cmin, d, kWave);
  y.cmax = __shfl_up(x.cmax, d, kWave);
  return y;
}

__device__ __forceinline__ RowState sums_state(const Sums& x, double lhs, double rhs, bool force) {
  return make_row_state(x.smin, x.smax, x.emin, x.emax, x.cmin, x.cmax, lhs, rhs, force);
}

// Row state in three words for a shuffle: the counts matter only as 0, 1 or
// more (a side with two infinite contributions yields no candidates).
__device__ __forceinline__ int state_bits(const RowState& R) {
  const int c0 = R.cmin < 2 ? R.cmin : 2, c1 = R.cmax < 2 ? R.cmax : 2;
  return c0 | (c1 << 2) | ((int)R.min_side << 4) | ((int)R.max_side << 5) |
         ((int)R.uncertain << 6);
}

__device__ __forceinline__ RowState state_from(double smn, double smx, int bits) {
  RowState R{};
  R.smn = smn;
  R.smx = smx;
  R.cmin = bits & 3;
  R.cmax = (bits >> 2) & 3;
  R.min_side = (bits >> 4) & 1;
  R.max_side = (bits >> 5) & 1;
  R.uncertain = (bits >> 6) & 1;
  return R;
}

// The exact candidate test over the lane's entries k0 .. k1 - 1 (one row).
__device__ __forceinline__ void nz_piece_candidates(const Problem& P, const RowState& R,
                                                    size_t base, int k0, int k1,
                                                    const double2* __restrict__ cur,
                                                    double2* __restrict__ nxt) {
  for (int k = k0; k < k1; ++k) {
    const size_t e = base + (size_t)k * kWave;
    const double a = P.vals[e];
    if (a == 0.0) continue;
    const int32_t cw = P.cols[e];
    const double2 b = cur[cw & kColMask];
    entry_candidates(P, R, a, b.x, b.y, cw, nxt, 1, true, touch_of(P, nxt, 1));
  }
}

// A row that lies in one lane, entries k0 .. k1 - 1, has ended: its state,
// and its candidates when the thresholds allow.  Returns true when the
// fast sums cannot certify it.
__device__ __forceinline__ bool nz_finish_row(const Problem& P, const LaneAcc& L, int row,
                                              size_t base, int k0, int k1,
                                              const double2* __restrict__ cur,
                                              double2* __restrict__ nxt, bool force) {
  const RowState R = sums_state(sums_of(L), P.lhs[row], P.rhs[row], force);
  if (R.uncertain) return true;
  if (lane_may_pass(R, L)) nz_piece_candidates(P, R, base, k0, k1, cur, nxt);
  return false;
}

// Exact path of an nnz-split wave: every row in turn, the lanes holding its
// entries adding their exact products into LDS digits.
__device__ void nz_wave_exact(const Problem& P, const ChunkDesc cd, size_t base, uint32_t flags,
                              int first_row, const double2* __restrict__ cur,
                              double2* __restrict__ nxt) {
  const int lane = threadIdx.x & (kWave - 1);
  ExactScratch& X = exact_scratch();
  for (int r = 0; r < cd.pad; ++r) {
    exact_clear(X);
    int row = first_row, cmin = 0, cmax = 0;
    for (int k = 0; k < kNzSteps; ++k) {
      if (k > 0 && ((flags >> k) & 1u)) ++row;
      if (row != r) continue;
      const size_t e = base + (size_t)k * kWave;
      const double a = P.vals[e];
      if (a == 0.0) continue;
      const double2 b = cur[P.cols[e] & kColMask];
      exact_entry(X, a, b.x, b.y);
      cmin += is_inf(a > 0.0 ? b.x : b.y) ? 1 : 0;
      cmax += is_inf(a > 0.0 ? b.y : b.x) ? 1 : 0;
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      cmin += __shfl_xor(cmin, off, kWave);
      cmax += __shfl_xor(cmax, off, kWave);
    }
    double mn, mx;
    exact_finish(X, lane == 0, mn, mx);
    const double lhs = P.lhs[cd.row0 + r], rhs = P.rhs[cd.row0 + r];
    RowState R{};
    R.cmin = cmin;
    R.cmax = cmax;
    R.min_side = (rhs < __builtin_inf()) && cmin <= 1;
    R.max_side = (lhs > -__builtin_inf()) && cmax <= 1;
    set_exact(R, mn, mx, lhs, rhs);
    if (!(R.min_side || R.max_side)) continue;
    row = first_row;
    for (int k = 0; k < kNzSteps; ++k) {
      if (k > 0 && ((flags >> k) & 1u)) ++row;
      if (row != r) continue;
      const size_t e = base + (size_t)k * kWave;
      const double a = P.vals[e];
      if (a == 0.0) continue;
      const int32_t cw = P.cols[e];
      const double2 b = cur[cw & kColMask];
      entry_candidates(P, R, a, b.x, b.y, cw, nxt, 1, true, touch_of(P, nxt, 1));
    }
  }
}

__device__ __forceinline__ void nz_wave_round(const Problem& P, int w,
                                              const double2* __restrict__ cur,
                                              double2* __restrict__ nxt, bool force_exact) {
  const int lane = threadIdx.x & (kWave - 1);
  const ChunkDesc cd = P.chunks[w];
  const size_t base = (size_t)cd.off64 * kWave + lane;
  const uint32_t flags = P.wave_flags[(size_t)w * kWave + lane];
  // rows started in earlier lanes (exclusive scan of the flag counts)
  const int own = __builtin_popcount(flags);
  int pre = own;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(pre, d, kWave);
    if (lane >= d) pre += y;
  }
  pre -= own;
  const bool starts = flags != 0;
  const bool head_open = !(flags & 1u);  // the first entry continues an earlier row
  const int first_row = (flags & 1u) ? pre : pre - 1;
  int row = first_row, kstart = 0, head_end = 0;
  LaneAcc acc, head;
  lane_acc_init(acc);
  lane_acc_init(head);
  bool redo = force_exact;
  // activity pass, two steps' loads before their gathers
#pragma unroll
  for (int k0 = 0; k0 < kNzSteps; k0 += 2) {
    double av[2];
    int32_t cv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const size_t e = base + (size_t)(k0 + k) * kWave;
      av[k] = __builtin_nontemporal_load(P.vals + e);
      cv[k] = __builtin_nontemporal_load(P.cols + e);
    }
    double2 bv[2];
    gather_bounds<2, kSrcCodes>(cur, nullptr, P.codes, cv, 1, 0, bv);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int kk = k0 + k;
      if (kk > 0 && ((flags >> kk) & 1u)) {
        // the piece kstart .. kk - 1 ends: the head piece, or a whole row
        if (kstart == 0 && head_open) {
          head = acc;
          head_end = kk;
        } else {
          redo |= nz_finish_row(P, acc, cd.row0 + row, base, kstart, kk, cur, nxt, force_exact);
        }
        lane_acc_init(acc);
        ++row;
        kstart = kk;
      }
      if (av[k] != 0.0) {
        accumulate(av[k], bv[k].x, bv[k].y, acc.smin, acc.smax, acc.cmin, acc.cmax, acc.emin,
                   acc.emax);
        lane_thresholds(acc, av[k], bv[k].x, bv[k].y, cv[k] < 0, P.cont_rel_tol);
      }
    }
  }
  // open pieces joined over the lanes: a segment starts where its row starts
  Sums x = sums_of(acc);
  bool f = starts;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const Sums y = sums_shfl_up(x, d);
    const bool fy = __shfl_up((int)f, d, kWave) != 0;
    if (lane >= d && !f) {
      sums_prepend(x, y);
      f = fy;
    }
  }
  // rows ending here: the open row when the next lane starts a new row (or
  // this is the last lane), and the head row (its earlier pieces are the
  // previous lane's scan)
  const uint32_t next_flags = __shfl_down(flags, 1, kWave);
  const bool ends = lane == kWave - 1 || (next_flags & 1u);
  const Sums carry = sums_shfl_up(x, 1);
  RowState rt{}, rh{};
  if (ends) rt = sums_state(x, P.lhs[cd.row0 + row], P.rhs[cd.row0 + row], force_exact);
  const bool has_head = starts && head_open;
  if (has_head) {
    Sums h = sums_of(head);
    sums_prepend(h, carry);
    rh = sums_state(h, P.lhs[cd.row0 + pre - 1], P.rhs[cd.row0 + pre - 1], force_exact);
  }
  // the open row's state from the lane where it ends: the first lane from
  // here on where it ends (`ends`), or the first later lane that starts a
  // row (the open row is that lane's head row)
  const uint64_t m_end = __ballot(ends), m_start = __ballot(starts);
  const uint64_t ge = ~0ull << lane;
  const uint64_t gt = lane == kWave - 1 ? 0ull : ~0ull << (lane + 1);
  const int j = __builtin_ctzll((m_end & ge) | (m_start & gt));
  const double h_smn = __shfl(rh.smn, j, kWave), h_smx = __shfl(rh.smx, j, kWave);
  const int h_bits = __shfl(state_bits(rh), j, kWave);
  const double t_smn = __shfl(rt.smn, j, kWave), t_smx = __shfl(rt.smx, j, kWave);
  const int t_bits = __shfl(state_bits(rt), j, kWave);
  const bool via_head = j > lane && ((m_start >> j) & 1ull);
  const RowState ro = via_head ? state_from(h_smn, h_smx, h_bits) : state_from(t_smn, t_smx, t_bits);
  if (has_head) {
    if (rh.uncertain) redo = true;
    else if (lane_may_pass(rh, head)) nz_piece_candidates(P, rh, base, 0, head_end, cur, nxt);
  }
  if (ro.uncertain) redo = true;
  else if (lane_may_pass(ro, acc)) nz_piece_candidates(P, ro, base, kstart, kNzSteps, cur, nxt);
  if (__ballot(redo)) nz_wave_exact(P, cd, base, flags, first_row, cur, nxt);
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
// Instead of one code per entry, a lane keeps the largest skip threshold of
// its entries per side (and whether it holds the entry that owns the side's
// only infinite contribution): "slack > largest threshold" skips every
// entry of the lane, exactly as the per-entry test would, so only lanes
// with an entry that may count revisit their entries, with the exact test.
// ---------------------------------------------------------------------------
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
      accumulate(av[k], bv[k].x, bv[k].y, L.smin, L.smax, L.cmin, L.cmax, L.emin, L.emax);
      lane_thresholds(L, av[k], bv[k].x, bv[k].y, cv[k] < 0, P.cont_rel_tol);
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
    double f = __shfl_xor(L.emin, off, kWave);
    double f2 = __shfl_xor(L.emax, off, kWave);
    int g = __shfl_xor(L.cmin, off, kWave);
    int h = __shfl_xor(L.cmax, off, kWave);
    dd_add(L.smin, L.emin, a, b, f);
    dd_add(L.smax, L.emax, c, d, f2);
    L.cmin += g;
    L.cmax += h;
  }
}

// Exact path for one (row, node) of node-parallel lanes: row block rb,
// node t0, entry slot e0 of the leading lane.  The pair's lanes get the
// exactly rounded activities and run the candidates of their entries.
__device__ __forceinline__ void exact_nodes_row(const Problem& P, const ChunkDesc cd, int rb,
                                                uint32_t t0, int e0,
                                                const double2* __restrict__ cur,
                                                double2* __restrict__ nxt, RowState& R,
                                                double lhs, double rhs) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t t = lane & (kNodeGroup - 1);
  const int e = lane >> 3;
  const int klog = cd.meta & 7;
  const int W = (cd.meta >> 8) & 0xff;
  const int QB = klog > 3 ? 1 << (klog - 3) : 1;
  const size_t base = (size_t)cd.off64 * kWave;
  ExactScratch& X = exact_scratch();
  exact_clear(X);
  const bool mine = t == t0 && (klog > 3 || (e >> klog) == (e0 >> klog));
  if (mine) {
    for (int qq = 0; qq < QB; ++qq) {
      const size_t l = (size_t)(rb * QB + qq) * 8 + e;
      for (int w = 0; w < W; ++w) {
        const size_t idx = base + (size_t)w * kWave + l;
        const double a = P.vals[idx];
        if (a == 0.0) continue;
        const double2 b = cur[(size_t)(P.cols[idx] & kColMask) * kNodeGroup + t];
        exact_entry(X, a, b.x, b.y);
      }
    }
  }
  double mn, mx;
  exact_finish(X, lane == e0 * 8 + (int)t0, mn, mx);
  if (!mine) return;
  set_exact(R, mn, mx, lhs, rhs);
  if (!(R.min_side || R.max_side)) return;
  for (int qq = 0; qq < QB; ++qq) {
    const size_t l = (size_t)(rb * QB + qq) * 8 + e;
    for (int w = 0; w < W; ++w) {
      const size_t idx = base + (size_t)w * kWave + l;
      const double a = P.vals[idx];
      if (a == 0.0) continue;
      const int32_t cw = P.cols[idx];
      const double2 b = cur[(size_t)(cw & kColMask) * kNodeGroup + t];
      entry_candidates(P, R, a, b.x, b.y, cw, nxt + t, kNodeGroup, false,
                       touch_of(P, nxt, kNodeGroup));
    }
  }
}

// Steps of a long chunk that node-parallel lanes load, gather and add as one
// group: 6 keeps k_round_batch within 128 VGPRs without spills (8 spilled).
constexpr int kNodeSteps = 6;

__device__ __forceinline__ void chunk_round_nodes(const Problem& P, const ChunkDesc cd,
                                                  const double2* __restrict__ cur,
                                                  double2* __restrict__ nxt, uint32_t node_mask,
                                                  uint32_t exact_mask, bool marked = false,
                                                  int r_round = 0,
                                                  const int32_t* marks = nullptr) {
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
    // marked rounds: a row block none of whose rows is stamped is skipped
    if (marked && __ballot(r < nrows && marks[cd.row0 + r] == r_round) == 0) continue;
    LaneAcc L;
    lane_acc_init(L);
    for (int qq = 0; qq < QB; ++qq) {
      const size_t l = (size_t)(rb * QB + qq) * 8 + e;
      // the chunk's step count W is the same in every lane: short chunks
      // (most rows have a few entries) take a narrower body, so no wave
      // issues loads and gathers for steps it does not have
      if (W <= 2) {
        node_entries<2>(P, cur, t, on, base + l, kWave, W, L);
      } else if (W <= 4) {
        node_entries<4>(P, cur, t, on, base + l, kWave, W, L);
      } else {
        for (int w0 = 0; w0 < W; w0 += kNodeSteps)
          node_entries<kNodeSteps>(P, cur, t, on, base + (size_t)w0 * kWave + l, kWave,
                                   W - w0 < kNodeSteps ? W - w0 : kNodeSteps, L);
      }
    }
    slot_reduce(L, klog > 3 ? 3 : klog);
    const int row = cd.row0 + (r < nrows ? r : 0);
    const bool live = r < nrows && on && (!marked || marks[row] == r_round);
    const double lhs = P.lhs[row], rhs = P.rhs[row];
    RowState R = make_row_state(L.smin, L.smax, L.emin, L.emax, L.cmin, L.cmax, lhs, rhs,
                                (exact_mask >> t) & 1u);
    if (live && !R.uncertain && lane_may_pass(R, L)) {
      for (int qq = 0; qq < QB; ++qq) {
        const size_t l = (size_t)(rb * QB + qq) * 8 + e;
        // four entries at a time: loads, then gathers, then the exact tests
        // (two memory round trips per four entries instead of three each)
        for (int w0 = 0; w0 < W; w0 += 4) {
          const int cnt = W - w0 < 4 ? W - w0 : 4;
          double av[4];
          int32_t cv[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const size_t idx = base + (size_t)(w0 + (k < cnt ? k : cnt - 1)) * kWave + l;
            av[k] = P.vals[idx];
            cv[k] = P.cols[idx];
          }
          double2 bv[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) bv[k] = cur[(size_t)(cv[k] & kColMask) * kNodeGroup + t];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < cnt && av[k] != 0.0)
              entry_candidates(P, R, av[k], bv[k].x, bv[k].y, cv[k], nxt + t, kNodeGroup, false,
                               touch_of(P, nxt, kNodeGroup));
        }
      }
    }
    // (row, node) pairs the fast sums cannot certify, one at a time with the
    // whole wave, led by the row's first entry slot
    const bool lead = klog > 3 ? e == 0 : (e & ((1 << klog) - 1)) == 0;
    uint64_t need = __ballot(live && lead && R.uncertain);
    while (need) {
      const int ll = __builtin_ctzll(need);
      exact_nodes_row(P, cd, rb, ll & (kNodeGroup - 1), ll >> 3, cur, nxt, R, lhs, rhs);
      need &= need - 1;
    }
  }
}

// ---------------------------------------------------------------------------
// long rows: partials live at partials[segment * pstride + node]
// ---------------------------------------------------------------------------
template <int kSrc>
__device__ __forceinline__ void seg_phase1(const Problem& P, int s,
                                           const double2* __restrict__ cur, uint32_t stride,
                                           uint32_t node_mask, SegPartial* parts,
                                           uint32_t pstride, uint32_t node0, bool marked = false,
                                           int r_round = 0, const int32_t* marks = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  const SegDesc sd = P.segs[s];
  if (marked && marks[sd.row] != r_round) return;
  // the segment's region is padded to whole 64-entry steps (zero
  // coefficients, column 0), so it is walked like a chunk of one 64-lane row
  const int W = (sd.len + kWave - 1) / kWave;
  const size_t base = (size_t)sd.off + lane;
  for (uint32_t mask = node_mask; mask; mask &= mask - 1) {
    const uint32_t t = __builtin_ctz(mask);
    LaneAcc L;
    lane_acc_init(L);
    lane_steps<kSrc>(P, cur, P.codes, stride, t, base, W, L);
    group_reduce(L.smin, L.smax, L.emin, L.emax, L.cmin, L.cmax, 6);
    double tmin = L.tmin, tmax = L.tmax;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double o1 = __shfl_xor(tmin, off, kWave);
      const double o2 = __shfl_xor(tmax, off, kWave);
      tmin = o1 > tmin ? o1 : tmin;
      tmax = o2 > tmax ? o2 : tmax;
    }
    if (lane == 0) {
      SegPartial q;
      q.min_hi = L.smin.hi;
      q.min_lo = L.smin.lo;
      q.max_hi = L.smax.hi;
      q.max_lo = L.smax.lo;
      q.tmin = tmin;
      q.tmax = tmax;
      q.min_inf = L.cmin;
      q.max_inf = L.cmax;
      q.emin = L.emin;
      q.emax = L.emax;
      parts[(size_t)s * pstride + node0 + t] = q;
    }
  }
}

// Phase 1 of a segment for the 8 nodes of a group (node-parallel lanes):
// slot e sums entries e, e + 8, e + 16, ... of the segment for node t.
__device__ __forceinline__ void seg_phase1_nodes(const Problem& P, int s,
                                                 const double2* __restrict__ cur,
                                                 uint32_t node_mask, SegPartial* parts,
                                                 uint32_t pstride, uint32_t node0,
                                                 bool marked = false, int r_round = 0,
                                                 const int32_t* marks = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t t = lane & (kNodeGroup - 1);
  const int e = lane >> 3;
  const bool on = (node_mask >> t) & 1u;
  const SegDesc sd = P.segs[s];
  if (marked && marks[sd.row] != r_round) return;
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
        accumulate(av[k], b.x, b.y, L.smin, L.smax, L.cmin, L.cmax, L.emin, L.emax);
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
    q.emin = L.emin;
    q.emax = L.emax;
    parts[(size_t)s * pstride + node0 + t] = q;
  }
}

// kBatchLoads (kernels that run phase 2 on its own): when a segment needs
// its candidates, each lane takes its entries kSegBatch at a time, loading
// all their coefficients and column words, then gathering all their bounds,
// then testing them, so the lane waits for two memory round trips per
// kSegBatch entries instead of three per entry.  Positions past the
// segment's end gather variable 0's pair and are skipped like padding.
constexpr int kSegBatch = 4;

// Exact path of a long row for node t: the wave sums all of the row's
// entries (its segments are stored one after another).
__device__ __forceinline__ void exact_long_row(const Problem& P, const SegDesc sd,
                                            const double2* __restrict__ cur, uint32_t stride,
                                            uint32_t t, double& mn, double& mx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t start = P.segs[sd.first].off;
  const int64_t len = (int64_t)(sd.nseg - 1) * kSegLen + P.segs[sd.first + sd.nseg - 1].len;
  ExactScratch& X = exact_scratch();
  exact_clear(X);
  for (int64_t p = lane; p < len; p += kWave) {
    const double a = P.vals[start + p];
    if (a == 0.0) continue;
    const double2 b = cur[(size_t)(P.cols[start + p] & kColMask) * stride + t];
    exact_entry(X, a, b.x, b.y);
  }
  exact_finish(X, lane == 0, mn, mx);
}

// Phase 2, first half: the state of the long row of segment descriptor sd
// for node t from all of the row's segment partials, combined in segment
// order (and the exact sums when the fast sums cannot certify it, or with
// force_exact).  The same in every lane after the full-wave reduction.
__device__ __forceinline__ RowState seg_row_state(const Problem& P, const SegDesc& sd,
                                                  const double2* __restrict__ cur,
                                                  uint32_t stride, uint32_t t,
                                                  const SegPartial* parts, uint32_t pstride,
                                                  uint32_t node, bool force_exact) {
  const int lane = threadIdx.x & (kWave - 1);
  DD smin = {0.0, 0.0}, smax = {0.0, 0.0};
  double emin = 0.0, emax = 0.0;
  int cmin = 0, cmax = 0;
  for (int q = lane; q < sd.nseg; q += kWave) {
    const SegPartial pp = parts[(size_t)(sd.first + q) * pstride + node];
    dd_add(smin, emin, pp.min_hi, pp.min_lo, pp.emin);
    dd_add(smax, emax, pp.max_hi, pp.max_lo, pp.emax);
    cmin += pp.min_inf;
    cmax += pp.max_inf;
  }
  if (sd.nseg <= 8) {
    // the partials sit in lanes 0-7 (zeros beyond): three levels, then
    // lane 0's sums for the whole wave
    group_reduce(smin, smax, emin, emax, cmin, cmax, 3);
    smin.hi = lane0_f64(smin.hi);
    smin.lo = lane0_f64(smin.lo);
    smax.hi = lane0_f64(smax.hi);
    smax.lo = lane0_f64(smax.lo);
    emin = lane0_f64(emin);
    emax = lane0_f64(emax);
    cmin = __builtin_amdgcn_readlane(cmin, 0);
    cmax = __builtin_amdgcn_readlane(cmax, 0);
  } else {
    group_reduce(smin, smax, emin, emax, cmin, cmax, 6);
  }
  const double lhs = P.lhs[sd.row], rhs = P.rhs[sd.row];
  RowState R = make_row_state(smin, smax, emin, emax, cmin, cmax, lhs, rhs, force_exact);
  if (R.uncertain) {
    double mn, mx;
    exact_long_row(P, sd, cur, stride, t, mn, mx);
    set_exact(R, mn, mx, lhs, rhs);
  }
  return R;
}

// Whether a segment whose partial is `own` may hold a counting entry of
// its row (state R): its largest skip thresholds do not rule one out, or
// it owns a side's only infinite contribution.
__device__ __forceinline__ bool seg_needs(const RowState& R, const SegPartial& own) {
  bool need = false;
  if (R.min_side) need |= (R.cmin == 0) ? !(R.smn > own.tmin) : (own.min_inf > 0);
  if (R.max_side) need |= (R.cmax == 0) ? !((-R.smx) > own.tmax) : (own.max_inf > 0);
  return need;
}

// Phase 2, second half: the candidates of segment s (descriptor sd) for
// node t given its row's state, when the segment's own largest skip
// thresholds do not rule out a counting entry.
template <bool kBatchLoads, int kSrc>
__device__ __forceinline__ void seg_revisit(const Problem& P, int s, const SegDesc& sd,
                                            const RowState& R, const double2* __restrict__ cur,
                                            double2* __restrict__ nxt, uint32_t stride,
                                            uint32_t t, const SegPartial* parts,
                                            uint32_t pstride, uint32_t node) {
  const int lane = threadIdx.x & (kWave - 1);
  if (!seg_needs(R, parts[(size_t)s * pstride + node])) return;
  if (kBatchLoads) {
    for (int w0 = 0; w0 < kSegLen / kWave; w0 += kSegBatch) {
      if (w0 * kWave >= sd.len) break;
      double av[kSegBatch];
      int32_t cv[kSegBatch];
#pragma unroll
      for (int w = 0; w < kSegBatch; ++w) {
        const int p = lane + (w0 + w) * kWave;
        av[w] = p < sd.len ? P.vals[sd.off + p] : 0.0;
        cv[w] = p < sd.len ? P.cols[sd.off + p] : 0;
      }
      double2 bv[kSegBatch];
#pragma unroll
      for (int w = 0; w < kSegBatch; ++w) bv[w] = pair_of<kSrc>(cur, P.b32, cv[w], stride, t);
#pragma unroll
      for (int w = 0; w < kSegBatch; ++w)
        if (av[w] != 0.0 && entry_wanted(R, av[w], bv[w].x, bv[w].y, cv[w], P.cont_rel_tol))
          entry_candidates(P, R, av[w], bv[w].x, bv[w].y, cv[w], nxt + t, stride, stride == 1,
                           touch_of(P, nxt, stride));
    }
    return;
  }
  for (int p = lane; p < sd.len; p += kWave) {
    const double a = P.vals[sd.off + p];
    if (a == 0.0) continue;
    const int32_t cw = P.cols[sd.off + p];
    const double2 b = pair_of<kSrc>(cur, P.b32, cw, stride, t);
    if (entry_wanted(R, a, b.x, b.y, cw, P.cont_rel_tol))
      entry_candidates(P, R, a, b.x, b.y, cw, nxt + t, stride, stride == 1,
                       touch_of(P, nxt, stride));
  }
}

// Phase 2 of segment s for node t: its row's state, then its candidates.
// Every segment of a row computes the row state itself (no wave waits on
// another; an uncertain row's exact sums are then summed once per segment).
template <bool kBatchLoads = false, int kSrc = kSrcPairs>
__device__ __forceinline__ void seg_phase2(const Problem& P, int s,
                                           const double2* __restrict__ cur,
                                           double2* __restrict__ nxt, uint32_t stride, uint32_t t,
                                           const SegPartial* parts, uint32_t pstride,
                                           uint32_t node, bool force_exact, bool marked = false,
                                           int r_round = 0, const int32_t* marks = nullptr) {
  const SegDesc sd = P.segs[s];
  if (marked && marks[sd.row] != r_round) return;
  const RowState R = seg_row_state(P, sd, cur, stride, t, parts, pstride, node, force_exact);
  seg_revisit<kBatchLoads, kSrc>(P, s, sd, R, cur, nxt, stride, t, parts, pstride, node);
}

// ---------------------------------------------------------------------------
// commit: copy changed pairs B -> A, count them, check their domains
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t u32_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Commit of one variable from its merged candidate pair b (b already holds
// the start-of-round pair folded in).
__device__ __forceinline__ bool commit_one(const Problem& P, uint32_t v, double2 a, double2 b,
                                           uint32_t& changed, uint32_t& infeasible) {
  float2 s32;
  if (P.store32) {
    s32 = make_float2(store_down32(b.x), store_up32(b.y));
    const double2 raw = b;
    b = make_double2((double)s32.x, (double)s32.y);
    if (a.x == b.x && a.y == b.y) {
      // a gain smaller than a grid step: nothing changes, and the candidate
      // target goes back to the start-of-round pair
      if (raw.x != a.x || raw.y != a.y) P.bnd[1][v] = a;
      return false;
    }
  }
  if (a.x == b.x && a.y == b.y) return false;
  const bool is_int = P.vtype[v] != 0;
  P.bnd[0][v] = b;
  P.bnd[1][v] = b;
  P.codes[v] = bound_code(is_int, b.x, b.y);
  if (P.store32) P.b32[v] = s32;
  ++changed;
  if (tiny_bound(b.x) || tiny_bound(b.y))
    __hip_atomic_store(&P.ctrl->tiny, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (domain_empty(is_int, b.x, b.y, P.feas_tol)) infeasible = 1;
  return true;
}

// First part of the commit: variables [0, H), H = n_hot rounded up to a
// multiple of 64 (at most n), eight lanes per variable.  Each lane takes
// the max / min over eight of a hot variable's stripe copies (and resets
// them); lane 0 of the eight also takes the variable's pair in B.  Three
// butterfly steps combine the eight lanes (max and min are exact, so the
// grouping does not matter) and lane 0 commits.  A wave covers eight
// variables, one touch byte: with kTouch, a wave whose byte is clear skips
// its variables (their stripes still hold the reset values and B equals
// A) and a wave whose byte is set clears it.  In marked rounds the wave
// stores the eight changed flags as one byte of the bitmap; the general
// part starts at H, so no bitmap word has two writers.
__device__ __forceinline__ uint32_t hot_end(const Problem& P) {
  if (P.n_hot <= 0) return 0;
  const uint32_t h = ((uint32_t)P.n_hot + kWave - 1) / kWave * kWave;
  return h < (uint32_t)P.n ? h : (uint32_t)P.n;
}

template <bool kTouch>
__device__ __forceinline__ void commit_hot(const Problem& P, uint32_t tid, uint32_t nthreads,
                                           uint32_t& changed, uint32_t& infeasible) {
  const uint32_t H = hot_end(P);
  const uint32_t items = H * 8u;
  const uint32_t lane = tid & (kWave - 1);
  uint8_t* const touch = kTouch ? touch_of(P, P.bnd[1], 1) : nullptr;
  for (uint32_t q0 = tid - lane; q0 < items; q0 += nthreads) {
    const uint32_t q = q0 + lane;
    if (kTouch) {
      // variables q0 / 8 .. q0 / 8 + 7: touch byte q0 / 64
      if (touch[q0 / kWave] == 0) {
        if (P.marking && lane == 0) reinterpret_cast<uint8_t*>(P.chg_bits)[q0 / kWave] = 0;
        continue;
      }
      if (lane == 0) touch[q0 / kWave] = 0;
    }
    const bool ok = q < items;
    const uint32_t v = ok ? q >> 3 : 0;
    const uint32_t g = q & 7;
    double lo = -__builtin_inf(), hi = __builtin_inf();
    if (ok && g == 0) {
      const double2 b = P.bnd[1][v];
      lo = b.x;
      hi = b.y;
    }
    if (ok && v < (uint32_t)P.n_hot) {
      double2* st = P.stripes + v + (size_t)g * 8 * P.n_hot;
      double2 c[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) c[k] = st[(size_t)k * P.n_hot];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        lo = c[k].x > lo ? c[k].x : lo;
        hi = c[k].y < hi ? c[k].y : hi;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        st[(size_t)k * P.n_hot] = make_double2(-__builtin_inf(), __builtin_inf());
    }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
      const double olo = __shfl_xor(lo, off, kWave);
      const double ohi = __shfl_xor(hi, off, kWave);
      lo = olo > lo ? olo : lo;
      hi = ohi < hi ? ohi : hi;
    }
    bool chg = false;
    if (ok && g == 0) chg = commit_one(P, v, P.bnd[0][v], make_double2(lo, hi), changed, infeasible);
    if (P.marking) {
      const uint64_t bits = __ballot(chg);
      if (lane == 0) {
        uint32_t byte = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) byte |= (uint32_t)((bits >> (8 * k)) & 1u) << k;
        // variables q0 / 8 .. q0 / 8 + 7: byte q0 / 64 of the little-endian bitmap
        reinterpret_cast<uint8_t*>(P.chg_bits)[q0 / kWave] = (uint8_t)byte;
      }
    }
  }
}

// Second part: variables [H, n), a wave taking kCommitUnroll consecutive
// 64-variable words per step of a grid-stride loop.  With kTouch, a word's
// eight touch bytes (one 64-bit load) say whether any of its variables got
// a candidate this round; only touched words load their pairs, all of the
// step's before any is compared, and their touch bytes are cleared.
// Without it (the persistent kernel, whose registers have no room for the
// touch pointer) every word is compared and the bytes stay set, which
// costs the next per-round commit one compare per word.  In marked rounds
// the wave also stores each word's changed flags as one word of the
// round's bitmap; the loop keeps the lanes of a wave together for that.
constexpr int kCommitUnroll = 2;

template <bool kTouch>
__device__ __forceinline__ void commit_range(const Problem& P, uint32_t tid, uint32_t nthreads,
                                             uint32_t& changed, uint32_t& infeasible) {
  commit_hot<kTouch>(P, tid, nthreads, changed, infeasible);
  const uint32_t lane = tid & (kWave - 1);
  const uint32_t n = (uint32_t)P.n;
  uint64_t* const touch =
      kTouch ? reinterpret_cast<uint64_t*>(touch_of(P, P.bnd[1], 1)) : nullptr;
  const uint64_t step = (uint64_t)nthreads * kCommitUnroll;
  for (uint64_t v0 = hot_end(P) + (uint64_t)(tid - lane) * kCommitUnroll; v0 < n; v0 += step) {
    bool hit[kCommitUnroll];
#pragma unroll
    for (int k = 0; k < kCommitUnroll; ++k) {
      const uint64_t w0 = v0 + (uint64_t)k * kWave;
      hit[k] = w0 < n && (!kTouch || touch[w0 / kWave] != 0);
    }
    double2 a[kCommitUnroll], b[kCommitUnroll];
#pragma unroll
    for (int k = 0; k < kCommitUnroll; ++k) {
      const uint64_t v = v0 + (uint64_t)k * kWave + lane;
      if (hit[k] && v < n) {
        a[k] = P.bnd[0][v];
        b[k] = P.bnd[1][v];
      }
    }
#pragma unroll
    for (int k = 0; k < kCommitUnroll; ++k) {
      const uint64_t w0 = v0 + (uint64_t)k * kWave;
      const uint64_t v = w0 + lane;
      bool chg = false;
      if (hit[k]) {
        if (v < n) chg = commit_one(P, (uint32_t)v, a[k], b[k], changed, infeasible);
        if (kTouch && lane == 0) touch[w0 / kWave] = 0;
      }
      if (P.marking && w0 < n) {
        const uint64_t bits = __ballot(chg);
        if (lane == 0) P.chg_bits[w0 / kWave] = bits;
      }
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
  if (P.marking) C->mark_all = changed > (uint32_t)(P.n / kMarkAllDiv) ? 1u : 0u;
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
//
// Arrival is counted in two levels, as by the commit kernel: block b adds
// to group word b mod G (G = min(blocks, kCommitGroups)), and the last
// block of a group adds the group's total to the control word, so no word
// sees more than ceil(blocks / G) returning atomics per barrier.  `add` is
// the block's packed commit total (changed pairs, infeasible flag), summed
// along: the end-of-round action reads the round's totals from the count.
//
// Ordering uses fences around relaxed atomics, one release and one acquire
// per block: on this chip an agent-scope release writes back the XCD's L2
// and an acquire invalidates it, so acquire loads in the polling loop would
// empty the L2 of every XCD over and over while other blocks still work.
// A block's writes before its release fence reach the last block of its
// group (acquire fence after the group's count is complete), whose release
// fence passes them on through the control word to the last block overall,
// whose release fence before the generation store passes everything to the
// waiters' acquire fence after they see the new generation.
__device__ __forceinline__ bool grid_barrier(const Problem& P, int action, int r, int max_rounds,
                                             uint64_t add = 0) {
  Ctrl* C = P.ctrl;
  __syncthreads();
  __shared__ uint32_t ok_shared;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    uint32_t ok = 1;
    // the generation cannot advance before this block has arrived
    const uint32_t g = __hip_atomic_load(&C->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t ngroups = gridDim.x < (uint32_t)kCommitGroups ? gridDim.x : kCommitGroups;
    const uint32_t grp = blockIdx.x % ngroups;
    const uint32_t in_grp = (gridDim.x - 1u - grp) / ngroups + 1u;
    uint64_t* gw = P.commit_grp + (size_t)grp * kGroupWordStride;
    const uint64_t mine = kCommitBlock | add;
    const uint64_t gold = __hip_atomic_fetch_add(gw, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool last = false;
    uint64_t tot = 0;
    if ((gold >> 48) == in_grp - 1u) {
      // the group is complete: reset its word (its blocks touch it again
      // only after this barrier's release) and report the group's total
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      const uint64_t gtot = gold + mine;
      __hip_atomic_store(gw, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t old =
          __hip_atomic_fetch_add(&C->commit_word, gtot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      tot = old + gtot;
      last = (tot >> 48) == gridDim.x;
    }
    if (last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (action == kActStart) {
        start_status(P, max_rounds);
      } else if (action == kActEndRound) {
        end_of_round(P, r, max_rounds, (uint32_t)tot, (uint32_t)((tot >> 32) & 0xffff));
      }
      __hip_atomic_store(&C->commit_word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&C->bar_gen, g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&C->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > PROP_SPIN_LIMIT ||
            __hip_atomic_load(&C->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(&C->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ok_shared = ok;
  }
  __syncthreads();
  return ok_shared != 0;
}

// Blocks for `items` work items of `per_block` each, at least 1, at most `cap`.
static inline int blocks_for(int64_t items, int per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace prop
