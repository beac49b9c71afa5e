/*
 * prop_oracle.c -- sequential CPU oracle for activity-based domain
 * propagation of linear constraints  lhs <= A x <= rhs,  l <= x <= u.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or constant with the GPU library; the two are built
 * separately and neither includes or links the other.
 *
 * What it computes (Sofranac, Gleixner, Pokutta, "Accelerating Domain
 * Propagation: an Efficient GPU-Parallel Algorithm over Sparse Matrices"):
 *
 *   - minimum / maximum activity of every row (Sec. 1.1, Definition 1,
 *     eq. minactivities / maxactivities), split into a finite part and a
 *     count of infinite contributions (Sec. 3.4, "Numerical Considerations
 *     for Computing Activities");
 *   - per nonzero the bound candidates of Step 3 (Sec. 1.1,
 *     eq. bound_candidates_pos / bound_candidates_neg), with integer
 *     rounding of Step 3's last sentence;
 *   - the synchronous round of Algorithm 2 (Sec. 2.3): all activities come
 *     from the bounds as they stood at the start of the round, every
 *     candidate is compared against those start-of-round bounds (Sec. 3.5),
 *     and the best candidate per variable wins (max for lower bounds, min
 *     for upper bounds; Algorithm 3);
 *   - rounds repeat until no bound changes, a domain becomes empty, or the
 *     round limit is hit (Sec. 1.1 last paragraphs, Algorithm 2's while).
 *
 * Readings where the paper is silent (all stated once more in the design
 * notes of the repository):
 *   R1  the activity sum is the exact real sum of the products a_k * b_k,
 *       rounded once to the nearest double (ties to even); the paper fixes
 *       no summation order and notes the sums are parallel reductions, so
 *       the order-free value is the definition written out;
 *   R2  explicit zero coefficients contribute nothing and get no candidate;
 *   R3  one infinite contribution: the candidate of the variable that owns
 *       it is (beta - finite_part) / a, without the "+ b" term (Sec. 3.4);
 *       two or more: no candidate from that side of the row;
 *   R4  integer candidates: lower = ceil(c - eps_int), upper =
 *       floor(c + eps_int); every candidate gets "+ 0.0" so -0.0 never
 *       appears;
 *   R5  a candidate counts ("is significant") when, against the
 *       start-of-round bound b: b infinite -> any finite candidate;
 *       integer -> strictly better; continuous -> better by more than
 *       cont_rel_tol * max(1, |b|)  (the threshold termination of Sec. 1.1);
 *   R6  a candidate whose magnitude exceeds 2^200, or is not finite, is
 *       dropped (the domain of valid input values ends at 2^200);
 *   R7  a variable's domain is empty when, for integers, l > u, and for
 *       continuous variables, l - u > feas_tol * max(1, |l|, |u|);
 *   R8  rounds counted include the last, change-free round; the status is
 *       decided at the end of every round, infeasibility first;
 *   R9  before round 1 the integer bounds are rounded as in R4, and the run
 *       stops with status INFEASIBLE after 0 rounds when an input domain is
 *       empty (R7), some row has lhs > rhs, or an empty row excludes 0;
 *   R12 (numbered as in the design notes, whose R10 and R11 state the
 *       synchronous update and the IEEE infinities this file also follows)
 *       single-precision bound store (orc_run_store with 32; Sec. 4.5 runs
 *       the whole method in single precision and reports results that are
 *       no longer correct): all arithmetic stays as in R1-R9, but every
 *       bound is kept as a member of F = {0, -inf, +inf} together with the
 *       normal single-precision numbers, rounded outward: a lower bound to
 *       the largest member of F not above it, an upper bound to the
 *       smallest member not below it.  This applies to the input bounds
 *       after R9's integer rounding and to every bound a round commits,
 *       before the round decides whether anything changed.  Outward
 *       rounding only loosens bounds, so a point the FP64 store keeps is
 *       kept (integers up to 2^24 are members of F and stay exact).
 *
 * Build:  gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_CONVERGED 0
#define ORC_INFEASIBLE 1
#define ORC_MAX_ROUNDS 2

#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Largest magnitude of a usable finite value (R6): 2^200. */
static double orc_huge(void) { return ldexp(1.0, 200); }

/* ------------------------------------------------------------------ */
/* Exact accumulation of a sum of products (reading R1).                */
/*                                                                      */
/* A finite double is m * 2^e with an integer |m| < 2^53 and            */
/* e >= -1126 (subnormals included, via frexp).  A product of two of    */
/* them is an integer below 2^106 times 2^(ea+eb).  All such products   */
/* are added exactly into a fixed-point integer whose least significant */
/* bit is 2^-ACC_OFF; positive and negative products go to separate     */
/* magnitudes, subtracted once at the end, and the difference is        */
/* rounded once to the nearest double, ties to even.                    */
/* ------------------------------------------------------------------ */
#define ACC_OFF 2304
#define ACC_LIMBS 140 /* 140 * 32 = 4480 bits */

typedef struct {
  uint32_t mag[2][ACC_LIMBS]; /* [0] positive products, [1] negative */
  int lo, hi;                 /* limb range touched since clear */
} exact_acc;

static void acc_clear(exact_acc* A) {
  if (A->hi >= A->lo) {
    size_t nb = (size_t)(A->hi - A->lo + 1) * sizeof(uint32_t);
    memset(&A->mag[0][A->lo], 0, nb);
    memset(&A->mag[1][A->lo], 0, nb);
  }
  A->lo = ACC_LIMBS;
  A->hi = -1;
}

static void acc_init(exact_acc* A) {
  memset(A, 0, sizeof(*A));
  A->lo = ACC_LIMBS;
  A->hi = -1;
}

/* x = m * 2^e with m an integer, 0 < m < 2^53; x finite and nonzero. */
static void split_double(double x, uint64_t* m, int* e) {
  int k;
  double f = frexp(fabs(x), &k); /* f in [0.5, 1) */
  *m = (uint64_t)ldexp(f, 53);
  *e = k - 53;
}

static void acc_add_product(exact_acc* A, double a, double b) {
  if (a == 0.0 || b == 0.0) return;
  uint64_t ma, mb;
  int ea, eb;
  split_double(a, &ma, &ea);
  split_double(b, &mb, &eb);
  int side = ((a < 0.0) != (b < 0.0)) ? 1 : 0;
  unsigned __int128 p = (unsigned __int128)ma * mb; /* < 2^106 */
  int pos = ea + eb + ACC_OFF;                      /* >= 52 */
  int limb = pos >> 5, sh = pos & 31;
  unsigned __int128 lo = p << sh;                   /* low 128 bits */
  uint32_t hi = sh ? (uint32_t)(p >> (128 - sh)) : 0u;
  uint32_t* L = A->mag[side];
  uint64_t carry = 0;
  for (int i = 0; i < 4; i++) {
    uint64_t s = (uint64_t)L[limb + i] + (uint32_t)(lo >> (32 * i)) + carry;
    L[limb + i] = (uint32_t)s;
    carry = s >> 32;
  }
  uint64_t s = (uint64_t)L[limb + 4] + hi + carry;
  L[limb + 4] = (uint32_t)s;
  carry = s >> 32;
  int i = limb + 5;
  while (carry) {
    s = (uint64_t)L[i] + carry;
    L[i] = (uint32_t)s;
    carry = s >> 32;
    i++;
  }
  if (limb < A->lo) A->lo = limb;
  if (i - 1 > A->hi) A->hi = i - 1;
  if (limb + 4 > A->hi) A->hi = limb + 4;
}

static int bit_at(const uint32_t* M, int idx) {
  if (idx < 0) return 0;
  return (int)((M[idx >> 5] >> (idx & 31)) & 1u);
}

/* Round the exact value (mag[0] - mag[1]) * 2^-ACC_OFF to nearest even. */
static double acc_round(exact_acc* A) {
  if (A->hi < A->lo) return 0.0;
  int lo = A->lo, hi = A->hi;
  uint32_t* P = A->mag[0];
  uint32_t* N = A->mag[1];
  int cmp = 0;
  for (int i = hi; i >= lo; i--) {
    if (P[i] != N[i]) {
      cmp = P[i] > N[i] ? 1 : -1;
      break;
    }
  }
  if (cmp == 0) return 0.0;
  uint32_t D[ACC_LIMBS];
  memset(D, 0, sizeof(D));
  const uint32_t* X = cmp > 0 ? P : N;
  const uint32_t* Y = cmp > 0 ? N : P;
  int64_t borrow = 0;
  for (int i = lo; i <= hi; i++) {
    int64_t d = (int64_t)X[i] - (int64_t)Y[i] - borrow;
    borrow = d < 0 ? 1 : 0;
    D[i] = (uint32_t)(d + (borrow << 32));
  }
  int top = hi;
  while (D[top] == 0) top--;
  int h = top * 32 + 31;
  while (!((D[top] >> (h & 31)) & 1u)) h--;
  /* least significant kept bit: 53 bits for normal results, 2^-1074 for
     subnormal ones */
  int q = h - 52;
  if (q < ACC_OFF - 1074) q = ACC_OFF - 1074;
  uint64_t sig = 0;
  for (int b = h; b >= q; b--) sig = (sig << 1) | (uint64_t)bit_at(D, b);
  int rbit = bit_at(D, q - 1);
  int sticky = 0;
  for (int b = q - 2; b >= lo * 32 && !sticky; b--) sticky = bit_at(D, b);
  if (rbit && (sticky || (sig & 1u))) sig++;
  double r = ldexp((double)sig, q - ACC_OFF);
  return cmp > 0 ? r : -r;
}

/* Exact dot product rounded once; exported for the oracle's own pins. */
double orc_exact_dot(const double* a, const double* b, int64_t k) {
  exact_acc* A = (exact_acc*)malloc(sizeof(exact_acc));
  if (!A) return NAN;
  acc_init(A);
  for (int64_t i = 0; i < k; i++) acc_add_product(A, a[i], b[i]);
  double r = acc_round(A) + 0.0;
  free(A);
  return r;
}

/* ------------------------------------------------------------------ */
/* Problem description and validation                                   */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t m, n;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  const double* lhs;
  const double* rhs;
  const uint8_t* vartype; /* 0 continuous, 1 integer */
} orc_problem;

typedef struct {
  double eps_int, cont_rel_tol, feas_tol;
  int store32; /* R12 */
} orc_params;

static int valid_value(double x) { return isfinite(x) && fabs(x) <= orc_huge(); }

/* Checks the input domain: finite coefficients with 2^-64 <= |a| <= 2^64 or
   exactly zero, column indices in range and distinct within a row, lhs and
   rhs either infinite in the harmless direction or finite within 2^200,
   vartype 0 or 1. */
static int orc_validate_problem(const orc_problem* P) {
  if (P->m < 0 || P->n < 0) return ORC_EINVAL;
  if (P->row_ptr[0] != 0) return ORC_EINVAL;
  for (int32_t i = 0; i < P->m; i++)
    if (P->row_ptr[i + 1] < P->row_ptr[i]) return ORC_EINVAL;
  double amin = ldexp(1.0, -64), amax = ldexp(1.0, 64);
  int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * (size_t)(P->n > 0 ? P->n : 1));
  if (!seen) return ORC_ENOMEM;
  for (int32_t j = 0; j < P->n; j++) seen[j] = -1;
  int rc = 0;
  for (int32_t i = 0; i < P->m && rc == 0; i++) {
    for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; k++) {
      int32_t j = P->col[k];
      double a = P->val[k];
      if (j < 0 || j >= P->n || seen[j] == i) { rc = ORC_EINVAL; break; }
      seen[j] = i;
      if (!isfinite(a)) { rc = ORC_EINVAL; break; }
      if (a != 0.0 && (fabs(a) < amin || fabs(a) > amax)) { rc = ORC_EINVAL; break; }
    }
    double l = P->lhs[i], r = P->rhs[i];
    if (isnan(l) || isnan(r)) rc = ORC_EINVAL;
    if (l == INFINITY || r == -INFINITY) rc = ORC_EINVAL;
    if (isfinite(l) && !valid_value(l)) rc = ORC_EINVAL;
    if (isfinite(r) && !valid_value(r)) rc = ORC_EINVAL;
  }
  for (int32_t j = 0; j < P->n && rc == 0; j++)
    if (P->vartype[j] > 1) rc = ORC_EINVAL;
  free(seen);
  return rc;
}

static int orc_validate_bounds(const orc_problem* P, const double* lb, const double* ub) {
  for (int32_t j = 0; j < P->n; j++) {
    double l = lb[j], u = ub[j];
    if (isnan(l) || isnan(u)) return ORC_EINVAL;
    if (l == INFINITY || u == -INFINITY) return ORC_EINVAL;
    if (isfinite(l) && !valid_value(l)) return ORC_EINVAL;
    if (isfinite(u) && !valid_value(u)) return ORC_EINVAL;
  }
  return 0;
}

/* Reading R12: the largest member of F not above x (x not NaN). */
static double store_down(double x) {
  if (isinf(x) || x == 0.0) return x + 0.0;
  if (x > FLT_MAX) return FLT_MAX;
  if (x < -FLT_MAX) return -INFINITY;
  if (x > 0.0 && x < FLT_MIN) return 0.0;
  if (x < 0.0 && x > -FLT_MIN) return -FLT_MIN;
  float f = (float)x; /* nearest: at most one step of the grid away */
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return (double)f;
}

/* Reading R12: the smallest member of F not below x. */
static double store_up(double x) { return -store_down(-x) + 0.0; }

/* Exported for the oracle's own pins. */
double orc_store_down(double x) { return store_down(x); }
double orc_store_up(double x) { return store_up(x); }

/* Reading R7. */
static int domain_empty(int is_int, double l, double u, double feas_tol) {
  if (is_int) return l > u;
  double s = fabs(l) > fabs(u) ? fabs(l) : fabs(u);
  if (s < 1.0) s = 1.0;
  return (l - u) > feas_tol * s;
}

/* Reading R9, the parts that depend on the rows only. */
static int rows_infeasible(const orc_problem* P) {
  for (int32_t i = 0; i < P->m; i++) {
    if (P->lhs[i] > P->rhs[i]) return 1;
    int empty = 1;
    for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; k++)
      if (P->val[k] != 0.0) { empty = 0; break; }
    if (empty && (P->lhs[i] > 0.0 || P->rhs[i] < 0.0)) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Activities (Definition 1 with the infinity counts of Sec. 3.4)       */
/* ------------------------------------------------------------------ */
static void row_activity(const orc_problem* P, int32_t i, const double* L, const double* U,
                         exact_acc* amin, exact_acc* amax, double* minfin, int64_t* mininf,
                         double* maxfin, int64_t* maxinf) {
  acc_clear(amin);
  acc_clear(amax);
  int64_t cmin = 0, cmax = 0;
  for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; k++) {
    double a = P->val[k];
    if (a == 0.0) continue; /* R2 */
    int32_t j = P->col[k];
    /* min activity takes l_j when a > 0, u_j otherwise; max the reverse */
    double bmin = a > 0.0 ? L[j] : U[j];
    double bmax = a > 0.0 ? U[j] : L[j];
    if (isinf(bmin)) cmin++;
    else acc_add_product(amin, a, bmin);
    if (isinf(bmax)) cmax++;
    else acc_add_product(amax, a, bmax);
  }
  *minfin = acc_round(amin) + 0.0;
  *maxfin = acc_round(amax) + 0.0;
  *mininf = cmin;
  *maxinf = cmax;
}

int orc_activities(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col,
                   const double* val, const double* L, const double* U, double* minfin,
                   int64_t* mininf, double* maxfin, int64_t* maxinf) {
  orc_problem P = {m, n, row_ptr, col, val, NULL, NULL, NULL};
  exact_acc* A = (exact_acc*)malloc(2 * sizeof(exact_acc));
  if (!A) return ORC_ENOMEM;
  acc_init(&A[0]);
  acc_init(&A[1]);
  for (int32_t i = 0; i < m; i++)
    row_activity(&P, i, L, U, &A[0], &A[1], &minfin[i], &mininf[i], &maxfin[i], &maxinf[i]);
  free(A);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Candidates (Step 3, eqs. bound_candidates_pos / _neg; Sec. 3.4)      */
/* ------------------------------------------------------------------ */

/* The bound a side of row i implies for variable j:
     (beta - act_fin) / a + b_j   when the activity has no infinite part,
     (beta - act_fin) / a         when j owns its only infinite part (R3).
   Returns 0 when the side gives nothing. */
static int side_term(double beta, double act_fin, int64_t act_inf, double a, double b, double* out) {
  if (!isfinite(beta)) return 0;
  double t;
  if (act_inf == 0) {
    t = beta - act_fin;
    t = t / a;
    t = t + b;
  } else if (act_inf == 1 && isinf(b)) {
    t = beta - act_fin;
    t = t / a;
  } else {
    return 0;
  }
  *out = t;
  return 1;
}

static int near_integer(double c, double eps) {
  double r = nearbyint(c);
  return fabs(c - r) <= eps + 1e-9;
}

/* One lower-bound candidate against the start-of-round bound Lj (R4-R6).
   Returns 1 and the rounded value when it counts. */
static int lower_counts(double c, int is_int, double Lj, const orc_params* prm, double* out,
                        int64_t* flags) {
  if (is_int) {
    if (isfinite(c) && near_integer(c, prm->eps_int)) (*flags)++;
    c = ceil(c - prm->eps_int);
  }
  c = c + 0.0;
  if (!(fabs(c) <= orc_huge())) return 0;
  int sig;
  if (Lj == -INFINITY) sig = 1;
  else if (is_int) sig = c > Lj;
  else {
    double s = fabs(Lj) > 1.0 ? fabs(Lj) : 1.0;
    sig = c > Lj + prm->cont_rel_tol * s;
  }
  if (sig) *out = c;
  return sig;
}

static int upper_counts(double c, int is_int, double Uj, const orc_params* prm, double* out,
                        int64_t* flags) {
  if (is_int) {
    if (isfinite(c) && near_integer(c, prm->eps_int)) (*flags)++;
    c = floor(c + prm->eps_int);
  }
  c = c + 0.0;
  if (!(fabs(c) <= orc_huge())) return 0;
  int sig;
  if (Uj == INFINITY) sig = 1;
  else if (is_int) sig = c < Uj;
  else {
    double s = fabs(Uj) > 1.0 ? fabs(Uj) : 1.0;
    sig = c < Uj - prm->cont_rel_tol * s;
  }
  if (sig) *out = c;
  return sig;
}

/* ------------------------------------------------------------------ */
/* One synchronous round (Algorithm 2 with the start-of-round snapshot  */
/* of Sec. 3.5 and the max/min resolution of Algorithm 3)                */
/* ------------------------------------------------------------------ */
static int round_impl(const orc_problem* P, const orc_params* prm, const double* L,
                      const double* U, double* Ln, double* Un, int* changed, int* infeasible,
                      int64_t* flags, exact_acc* A) {
  for (int32_t j = 0; j < P->n; j++) {
    Ln[j] = L[j];
    Un[j] = U[j];
  }
  for (int32_t i = 0; i < P->m; i++) {
    double minfin, maxfin;
    int64_t mininf, maxinf;
    row_activity(P, i, L, U, &A[0], &A[1], &minfin, &mininf, &maxfin, &maxinf);
    for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; k++) {
      double a = P->val[k];
      if (a == 0.0) continue;
      int32_t j = P->col[k];
      int is_int = P->vartype[j] == 1;
      double bmin = a > 0.0 ? L[j] : U[j];
      double bmax = a > 0.0 ? U[j] : L[j];
      double tmin = 0.0, tmax = 0.0, c;
      /* the rhs side works through the min activity, the lhs side through
         the max activity; for a > 0 they bound x_j from above / below, for
         a < 0 from below / above (eqs. bound_candidates_pos / _neg) */
      int has_min = side_term(P->rhs[i], minfin, mininf, a, bmin, &tmin);
      int has_max = side_term(P->lhs[i], maxfin, maxinf, a, bmax, &tmax);
      double lc_raw = 0, uc_raw = 0;
      int has_l = 0, has_u = 0;
      if (a > 0.0) {
        if (has_min) { uc_raw = tmin; has_u = 1; }
        if (has_max) { lc_raw = tmax; has_l = 1; }
      } else {
        if (has_min) { lc_raw = tmin; has_l = 1; }
        if (has_max) { uc_raw = tmax; has_u = 1; }
      }
      if (has_l && lower_counts(lc_raw, is_int, L[j], prm, &c, flags))
        if (c > Ln[j]) Ln[j] = c;
      if (has_u && upper_counts(uc_raw, is_int, U[j], prm, &c, flags))
        if (c < Un[j]) Un[j] = c;
    }
  }
  int ch = 0, inf = 0;
  for (int32_t j = 0; j < P->n; j++) {
    if (prm->store32) {
      Ln[j] = store_down(Ln[j]);
      Un[j] = store_up(Un[j]);
    }
    if (Ln[j] != L[j] || Un[j] != U[j]) ch = 1;
    if (domain_empty(P->vartype[j] == 1, Ln[j], Un[j], prm->feas_tol)) inf = 1;
  }
  *changed = ch;
  *infeasible = inf;
  return 0;
}

static void fill_params(orc_params* prm, double eps_int, double cont_rel_tol, double feas_tol) {
  prm->eps_int = eps_int;
  prm->cont_rel_tol = cont_rel_tol;
  prm->feas_tol = feas_tol;
  prm->store32 = 0;
}

/* One round from (L, U) to (Ln, Un); no entry normalisation. */
int orc_round(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
              const double* lhs, const double* rhs, const uint8_t* vartype, double eps_int,
              double cont_rel_tol, double feas_tol, const double* L, const double* U, double* Ln,
              double* Un, int32_t* changed, int32_t* infeasible, int64_t* flags) {
  orc_problem P = {m, n, row_ptr, col, val, lhs, rhs, vartype};
  orc_params prm;
  fill_params(&prm, eps_int, cont_rel_tol, feas_tol);
  int rc = orc_validate_problem(&P);
  if (rc) return rc;
  rc = orc_validate_bounds(&P, L, U);
  if (rc) return rc;
  exact_acc* A = (exact_acc*)malloc(2 * sizeof(exact_acc));
  if (!A) return ORC_ENOMEM;
  acc_init(&A[0]);
  acc_init(&A[1]);
  int ch = 0, inf = 0;
  *flags = 0;
  round_impl(&P, &prm, L, U, Ln, Un, &ch, &inf, flags, A);
  free(A);
  *changed = ch;
  *infeasible = inf;
  return 0;
}

/* Integer rounding of the input bounds (R9). */
static void normalize_bounds(const orc_problem* P, const orc_params* prm, double* lb, double* ub) {
  for (int32_t j = 0; j < P->n; j++) {
    if (P->vartype[j] == 1) {
      lb[j] = ceil(lb[j] - prm->eps_int);
      ub[j] = floor(ub[j] + prm->eps_int);
    }
    lb[j] = lb[j] + 0.0;
    ub[j] = ub[j] + 0.0;
    if (prm->store32) {
      lb[j] = store_down(lb[j]);
      ub[j] = store_up(ub[j]);
    }
  }
}

/* Full run: lb/ub in, tightened lb/ub out (unspecified when INFEASIBLE). */
static int run_impl(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col,
                    const double* val, const double* lhs, const double* rhs,
                    const uint8_t* vartype, double eps_int, double cont_rel_tol, double feas_tol,
                    int store32, double* lb, double* ub, int32_t max_rounds, int32_t* status,
                    int32_t* rounds, int64_t* flags) {
  orc_problem P = {m, n, row_ptr, col, val, lhs, rhs, vartype};
  orc_params prm;
  fill_params(&prm, eps_int, cont_rel_tol, feas_tol);
  prm.store32 = store32;
  if (max_rounds < 0) return ORC_EINVAL;
  int rc = orc_validate_problem(&P);
  if (rc) return rc;
  rc = orc_validate_bounds(&P, lb, ub);
  if (rc) return rc;
  *flags = 0;
  *rounds = 0;
  if (rows_infeasible(&P)) {
    *status = ORC_INFEASIBLE;
    return 0;
  }
  normalize_bounds(&P, &prm, lb, ub);
  for (int32_t j = 0; j < n; j++) {
    if (domain_empty(vartype[j] == 1, lb[j], ub[j], feas_tol)) {
      *status = ORC_INFEASIBLE;
      return 0;
    }
  }
  if (max_rounds == 0) {
    *status = ORC_MAX_ROUNDS;
    return 0;
  }
  double* Ln = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* Un = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  exact_acc* A = (exact_acc*)malloc(2 * sizeof(exact_acc));
  if (!Ln || !Un || !A) {
    free(Ln);
    free(Un);
    free(A);
    return ORC_ENOMEM;
  }
  acc_init(&A[0]);
  acc_init(&A[1]);
  *status = ORC_MAX_ROUNDS;
  *rounds = max_rounds;
  for (int32_t r = 1; r <= max_rounds; r++) {
    int ch = 0, inf = 0;
    round_impl(&P, &prm, lb, ub, Ln, Un, &ch, &inf, flags, A);
    memcpy(lb, Ln, sizeof(double) * (size_t)n);
    memcpy(ub, Un, sizeof(double) * (size_t)n);
    if (inf) {
      *status = ORC_INFEASIBLE;
      *rounds = r;
      break;
    }
    if (!ch) {
      *status = ORC_CONVERGED;
      *rounds = r;
      break;
    }
  }
  free(Ln);
  free(Un);
  free(A);
  return 0;
}

int orc_run(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
            const double* lhs, const double* rhs, const uint8_t* vartype, double eps_int,
            double cont_rel_tol, double feas_tol, double* lb, double* ub, int32_t max_rounds,
            int32_t* status, int32_t* rounds, int64_t* flags) {
  return run_impl(m, n, row_ptr, col, val, lhs, rhs, vartype, eps_int, cont_rel_tol, feas_tol, 0,
                  lb, ub, max_rounds, status, rounds, flags);
}

/* The same run with the bound store of R12: store_bits 64 (doubles, as
   orc_run) or 32 (single precision, rounded outward). */
int orc_run_store(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col,
                  const double* val, const double* lhs, const double* rhs,
                  const uint8_t* vartype, double eps_int, double cont_rel_tol, double feas_tol,
                  int32_t store_bits, double* lb, double* ub, int32_t max_rounds,
                  int32_t* status, int32_t* rounds, int64_t* flags) {
  if (store_bits != 32 && store_bits != 64) return ORC_EINVAL;
  return run_impl(m, n, row_ptr, col, val, lhs, rhs, vartype, eps_int, cont_rel_tol, feas_tol,
                  store_bits == 32, lb, ub, max_rounds, status, rounds, flags);
}

/* ------------------------------------------------------------------ */
/* Sequential propagation with constraint marking (Algorithm 1).        */
/* Rows are visited in order; a row's activities come from the current */
/* bounds, a tightening is visible at once to every later row, and the  */
/* rows holding a tightened variable are marked for the next sweep.     */
/* Used to pin the limit point the synchronous rounds reach (Sec. 1.1:  */
/* the fixed-point iteration has a unique limit).                        */
/* ------------------------------------------------------------------ */
int orc_run_seq(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col,
                const double* val, const double* lhs, const double* rhs, const uint8_t* vartype,
                double eps_int, double cont_rel_tol, double feas_tol, double* lb, double* ub,
                int32_t max_sweeps, int32_t* status, int32_t* sweeps) {
  orc_problem P = {m, n, row_ptr, col, val, lhs, rhs, vartype};
  orc_params prm;
  fill_params(&prm, eps_int, cont_rel_tol, feas_tol);
  if (max_sweeps < 0) return ORC_EINVAL;
  int rc = orc_validate_problem(&P);
  if (rc) return rc;
  rc = orc_validate_bounds(&P, lb, ub);
  if (rc) return rc;
  *sweeps = 0;
  if (rows_infeasible(&P)) {
    *status = ORC_INFEASIBLE;
    return 0;
  }
  normalize_bounds(&P, &prm, lb, ub);
  for (int32_t j = 0; j < n; j++)
    if (domain_empty(vartype[j] == 1, lb[j], ub[j], feas_tol)) {
      *status = ORC_INFEASIBLE;
      return 0;
    }
  if (max_sweeps == 0) {
    *status = ORC_MAX_ROUNDS;
    return 0;
  }
  /* column view of A for the marking step */
  int64_t nnz = row_ptr[m];
  int64_t* cptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* crow = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint8_t* mark = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  exact_acc* A = (exact_acc*)malloc(2 * sizeof(exact_acc));
  if (!cptr || !crow || !fill || !mark || !A) {
    free(cptr); free(crow); free(fill); free(mark); free(A);
    return ORC_ENOMEM;
  }
  for (int64_t k = 0; k < nnz; k++) cptr[col[k] + 1]++;
  for (int32_t j = 0; j < n; j++) cptr[j + 1] += cptr[j];
  for (int32_t j = 0; j < n; j++) fill[j] = cptr[j];
  for (int32_t i = 0; i < m; i++)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) crow[fill[col[k]]++] = i;
  acc_init(&A[0]);
  acc_init(&A[1]);
  memset(mark, 1, (size_t)m);
  int64_t dummy = 0;
  *status = ORC_MAX_ROUNDS;
  *sweeps = max_sweeps;
  for (int32_t s = 1; s <= max_sweeps; s++) {
    int ch = 0;
    for (int32_t i = 0; i < m; i++) {
      if (!mark[i]) continue;
      mark[i] = 0;
      double minfin, maxfin;
      int64_t mininf, maxinf;
      row_activity(&P, i, lb, ub, &A[0], &A[1], &minfin, &mininf, &maxfin, &maxinf);
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
        double a = val[k];
        if (a == 0.0) continue;
        int32_t j = col[k];
        int is_int = vartype[j] == 1;
        double bmin = a > 0.0 ? lb[j] : ub[j];
        double bmax = a > 0.0 ? ub[j] : lb[j];
        double tmin = 0.0, tmax = 0.0, c;
        int has_min = side_term(rhs[i], minfin, mininf, a, bmin, &tmin);
        int has_max = side_term(lhs[i], maxfin, maxinf, a, bmax, &tmax);
        double lc = 0, uc = 0;
        int hl = 0, hu = 0;
        if (a > 0.0) {
          if (has_min) { uc = tmin; hu = 1; }
          if (has_max) { lc = tmax; hl = 1; }
        } else {
          if (has_min) { lc = tmin; hl = 1; }
          if (has_max) { uc = tmax; hu = 1; }
        }
        int tightened = 0;
        if (hl && lower_counts(lc, is_int, lb[j], &prm, &c, &dummy)) { lb[j] = c; tightened = 1; }
        if (hu && upper_counts(uc, is_int, ub[j], &prm, &c, &dummy)) { ub[j] = c; tightened = 1; }
        if (tightened) {
          ch = 1;
          for (int64_t q = cptr[j]; q < cptr[j + 1]; q++) mark[crow[q]] = 1;
        }
      }
    }
    int inf = 0;
    for (int32_t j = 0; j < n; j++)
      if (domain_empty(vartype[j] == 1, lb[j], ub[j], feas_tol)) inf = 1;
    if (inf) { *status = ORC_INFEASIBLE; *sweeps = s; break; }
    if (!ch) { *status = ORC_CONVERGED; *sweeps = s; break; }
  }
  free(cptr); free(crow); free(fill); free(mark); free(A);
  return 0;
}
