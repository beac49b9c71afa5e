// prop_sum.h -- the activity sums of Definition 1 (with the infinity counts
// of Sec. 3.4), computed as the exact sum of the products rounded once to
// the nearest double (ties to even), whatever the order of the terms.
//
// Fast path: every lane sums its products as a double-double (hi, lo): the
// product is split exactly with an FMA, hi takes an error-free two-sum, and
// lo collects both error terms.  The two additions into lo can round; each
// one's rounding error is itself computed exactly with a two-sum, and err
// collects their magnitudes.  Lanes and partial sums combine with dd_add,
// which does the same for its own two roundings and adds both operands'
// err.  Each of the two sums of a row (min and max activity) keeps its own
// err.  So |S - (hi + lo)| <= sum of the collected errors, S the exact sum
// of the row's products, and err is that sum computed in floating point
// (nonnegative terms: at most (k - 1)u relative below the true sum for k
// terms, u = 2^-53; exact while the terms are below 2^-1021).  dd_round
// checks whether every real number within that distance of hi + lo rounds
// to the same double as hi + lo; if so that double is RN(S).  When no
// addition rounded at all, err is 0 and hi + lo is S itself, which covers
// exact ties (frequent with +-1 coefficients and short mantissas; an a
// priori bound such as 2^-53 |lo| would refuse those ties).  Only when S
// may lie on the other side of a rounding boundary than hi + lo (as with
// 2^53 + 1 + 2^-60, where lo loses the 2^-60) does the row need the exact
// path below.
//
// The FMA split is exact when the product's last bit is not below 2^-1074.
// With coefficients of magnitude in [2^-64, 2^64] that holds for every
// bound that is 0 or of magnitude at least 2^-906; a bound of smaller
// nonzero magnitude sends its rows to the exact path (PROP_TINY_BOUND).
//
// Exact path: a fixed-point integer sum.  A product is ma * mb * 2^(ea+eb)
// with 53-bit integers ma, mb; its 106-bit integer lands at bit
// ea + eb + kAccBias of an array of 32-bit digits, each digit accumulated
// in a signed 64-bit word (2^31 additions cannot overflow it).  The
// position never drops below 2^-1190 (bounds down to 2^-1074, coefficients
// down to 2^-64) and the sum stays below 2^297 (bounds up to 2^200,
// coefficients up to 2^64, at most 2^31 terms), so 48 digits cover it.
// digits_round normalises the carries and rounds once, to nearest even,
// with subnormal results handled.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace prop {

struct DD {
  double hi, lo;
};

// Bounds below this magnitude (and nonzero) may make a product's FMA split
// inexact; their rows take the exact path.
#define PROP_TINY_BOUND 0x1p-906

__host__ __device__ __forceinline__ bool tiny_bound(double b) {
  return b != 0.0 && __builtin_fabs(b) < PROP_TINY_BOUND;
}

// Rounding error of c = RN(x + y), exactly (two-sum).
__host__ __device__ __forceinline__ double two_sum_err(double x, double y, double c) {
  const double z = c - x;
  return (x - (c - z)) + (y - z);
}

// s += a * b; err += the magnitudes of the two roundings into s.lo.
__host__ __device__ __forceinline__ void dd_add_prod(DD& s, double a, double b, double& err) {
  const double p = a * b;
  const double ep = __builtin_fma(a, b, -p);
  const double t = s.hi + p;
  const double e = two_sum_err(s.hi, p, t);
  const double x = e + ep;
  const double l = s.lo + x;
  err = err + (__builtin_fabs(two_sum_err(e, ep, x)) + __builtin_fabs(two_sum_err(s.lo, x, l)));
  s.hi = t;
  s.lo = l;
}

// s += (yhi, ylo), yerr the operand's own bound.  Symmetric in its two
// operands (two-sum errors and commutative additions), so both lanes of a
// butterfly exchange end with identical bits.
__host__ __device__ __forceinline__ void dd_add(DD& s, double& err, double yhi, double ylo,
                                                double yerr) {
  const double t = s.hi + yhi;
  const double e = two_sum_err(s.hi, yhi, t);
  const double v = s.lo + ylo;
  const double l = v + e;
  err = (err + yerr) +
        (__builtin_fabs(two_sum_err(s.lo, ylo, v)) + __builtin_fabs(two_sum_err(v, e, l)));
  s.hi = t;
  s.lo = l;
}

__host__ __device__ __forceinline__ uint64_t f64_bits(double x) {
  return __builtin_bit_cast(uint64_t, x);
}
__host__ __device__ __forceinline__ double f64_from(uint64_t b) {
  return __builtin_bit_cast(double, b);
}

// Rounds the double-double (hi, lo), whose distance to the exact sum is at
// most err (up to the rounding of err's own sum), to *out = RN(hi + lo).
// Returns true when that is provably the exact sum rounded to nearest even.
__host__ __device__ __forceinline__ bool dd_round(double hi, double lo, double err, double& out) {
  const double s = hi + lo;
  out = s + 0.0;
  if (err == 0.0) return true;  // no addition into lo rounded: hi + lo is exact
  const double t = two_sum_err(hi, lo, s);  // hi + lo = s + t exactly
  // E >= the true error: err's own sum of at most 2^22 terms is low by less
  // than 2^-30 relative (and exact below 2^-1021)
  const double E = err + err * 0x1p-30;
  if (s == 0.0) return false;
  const uint64_t bits = f64_bits(s) & 0x7fffffffffffffffull;
  const uint64_t expo = bits >> 52;
  // ulp of |s| (the gap to the next larger magnitude)
  double ulp;
  if (expo > 52) ulp = f64_from((expo - 52) << 52);
  else ulp = f64_from(1ull << (expo > 0 ? expo - 1 : 0));
  // gap to the next smaller magnitude: half the ulp at a power of two
  const bool pow2 = (bits & 0x000fffffffffffffull) == 0 && expo > 1;
  const double gap_dn = pow2 ? ulp * 0.5 : ulp;
  const bool away = t != 0.0 && ((t < 0.0) == (s < 0.0));
  const double half = (away ? ulp : gap_dn) * 0.5;
  // |t| + E < half, with room for the rounding of half - |t|
  return E < 0.5 * (half - __builtin_fabs(t));
}

// ---------------------------------------------------------------------------
// exact path: fixed-point digits
// ---------------------------------------------------------------------------
constexpr int kAccDigits = 48;   // 32-bit digits, bits [0, 1536)
constexpr int kAccBias = 1216;   // bit position of 2^0

// 53-bit integer significand and exponent of a finite nonzero double:
// |x| = m * 2^e.
__host__ __device__ __forceinline__ void split_f64(double x, uint64_t& m, int& e) {
  const uint64_t bits = f64_bits(x) & 0x7fffffffffffffffull;
  const int expo = (int)(bits >> 52);
  const uint64_t frac = bits & 0x000fffffffffffffull;
  if (expo == 0) {  // subnormal
    m = frac;
    e = -1074;
  } else {
    m = frac | (1ull << 52);
    e = expo - 1075;
  }
}

// The exact product a * b (both finite) as up to five 32-bit chunks c[0..4]
// to be added (neg: subtracted) at digits d .. d + 4.  Returns false for a
// zero product.
__host__ __device__ __forceinline__ bool product_digits(double a, double b, int& d,
                                                        uint32_t c[5], bool& neg) {
  if (a == 0.0 || b == 0.0) return false;
  uint64_t ma, mb;
  int ea, eb;
  split_f64(a, ma, ea);
  split_f64(b, mb, eb);
  neg = (a < 0.0) != (b < 0.0);
  const unsigned __int128 p = (unsigned __int128)ma * mb;  // < 2^106
  const int pos = ea + eb + kAccBias;                      // >= 26
  d = pos >> 5;
  const int sh = pos & 31;
  const uint64_t lo = (uint64_t)p, hi = (uint64_t)(p >> 64);
  const uint64_t w0 = lo << sh;
  const uint64_t w1 = (hi << sh) | (sh ? lo >> (64 - sh) : 0);
  const uint64_t w2 = sh ? hi >> (64 - sh) : 0;
  c[0] = (uint32_t)w0;
  c[1] = (uint32_t)(w0 >> 32);
  c[2] = (uint32_t)w1;
  c[3] = (uint32_t)(w1 >> 32);
  c[4] = (uint32_t)w2;
  return true;
}

// Bit q of the normalised magnitude digits (stored in the low 32 bits of W).
__host__ __device__ __forceinline__ uint32_t digit_bit(const int64_t* W, int q) {
  if (q < 0) return 0;
  return (uint32_t)(((uint64_t)W[q >> 5] >> (q & 31)) & 1u);
}

// Normalises the digit words in place and returns the value they hold
// (sum of W[k] * 2^(32k - kAccBias)), rounded once to nearest even.
__host__ __device__ inline double digits_round(int64_t* W) {
  // carries: afterwards W[k] in [0, 2^32), sign in the final carry
  int64_t carry = 0;
#pragma unroll 1
  for (int k = 0; k < kAccDigits; ++k) {
    const int64_t v = W[k] + carry;
    W[k] = (int64_t)(uint32_t)v;
    carry = v >> 32;  // arithmetic shift: floor division
  }
  const bool neg = carry < 0;
  if (neg) {  // magnitude of the two's complement value
    uint64_t c = 1;
#pragma unroll 1
    for (int k = 0; k < kAccDigits; ++k) {
      const uint64_t v = (uint64_t)(uint32_t)~(uint32_t)W[k] + c;
      W[k] = (int64_t)(uint32_t)v;
      c = v >> 32;
    }
  }
  int top = kAccDigits - 1;
  while (top >= 0 && W[top] == 0) --top;
  if (top < 0) return 0.0;
  int h = top * 32 + 31;
  while (!digit_bit(W, h)) --h;
  // lowest kept bit: 53 significant bits, or 2^-1074 for a subnormal result
  int q = h - 52;
  if (q < kAccBias - 1074) q = kAccBias - 1074;
  uint64_t sig = 0;
#pragma unroll 1
  for (int b = h; b >= q; --b) sig = (sig << 1) | digit_bit(W, b);
  const uint32_t rbit = digit_bit(W, q - 1);
  uint32_t sticky = 0;
  if (q - 2 >= 0) {
    const int qd = (q - 2) >> 5;
    const uint32_t below = (uint32_t)(((uint64_t)1 << (((q - 2) & 31) + 1)) - 1);
    sticky = ((uint32_t)W[qd] & below) != 0;
#pragma unroll 1
    for (int k = 0; k < qd && !sticky; ++k) sticky = W[k] != 0;
  }
  if (rbit && (sticky || (sig & 1u))) ++sig;
  const double r = __builtin_ldexp((double)sig, q - kAccBias);
  return (neg ? -r : r) + 0.0;
}

}  // namespace prop
