/*
 * cpu_seq.c -- the paper's sequential CPU baseline: domain propagation with
 * constraint marking (Sofranac, Gleixner, Pokutta, Sec. 2.1, Algorithm 1),
 * in plain double arithmetic, for speed comparisons.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY, like the oracle beside it, with
 * which it shares no code.  It is not the oracle: its activities are plain
 * left-to-right double sums in CSR order (the paper's sequential code sums
 * that way), not exactly rounded ones, so its bounds agree with the
 * oracle's within a tolerance only.
 *
 * Algorithm 1, as the paper gives it:
 *   - every constraint starts marked; sweeps visit the marked constraints
 *     in order, unmarking each;
 *   - a constraint's min / max activities (Definition 1, with the infinity
 *     counts of Sec. 3.4) come from the bounds as they are at that moment,
 *     so tightenings found earlier in the sweep are already visible;
 *   - "can the constraint propagate": a side (rhs through the min activity,
 *     lhs through the max activity) is used only if it is finite, has at
 *     most one infinite contribution, and is not redundant (max activity
 *     <= rhs, resp. min activity >= lhs, Sec. 1.1 Step 1);
 *   - "can the variable be tightened": a side skips a variable whose whole
 *     domain width times |a| fits in the side's slack (the candidate cannot
 *     beat the bound);
 *   - candidates (eqs. bound_candidates_pos / _neg), integer rounding and
 *     the significance threshold follow the same readings as the oracle
 *     (see its header); a tightened bound is written at once, and every
 *     constraint holding the variable is marked (a column view of A);
 *   - a sweep that tightens nothing ends the run (converged); an empty
 *     domain after a sweep ends it as infeasible.
 * The paper's listing reuses its loop flag when deciding whether to mark a
 * variable's constraints; here only a variable that was tightened marks
 * them.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CS_CONVERGED 0
#define CS_INFEASIBLE 1
#define CS_MAX_ROUNDS 2

typedef struct {
  int32_t m, n;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  const double* lhs;
  const double* rhs;
  const uint8_t* vartype;
  int64_t* cptr; /* column view: rows of variable j at crow[cptr[j] .. cptr[j+1]) */
  int32_t* crow;
  uint8_t* mark;
} cs_problem;

/* Builds the column view (untimed set-up, as the paper times propagation
   only).  The arrays are borrowed: the caller keeps them alive. */
cs_problem* cs_create(int32_t m, int32_t n, const int64_t* row_ptr, const int32_t* col,
                      const double* val, const double* lhs, const double* rhs,
                      const uint8_t* vartype) {
  cs_problem* P = (cs_problem*)calloc(1, sizeof(cs_problem));
  if (!P) return NULL;
  P->m = m;
  P->n = n;
  P->row_ptr = row_ptr;
  P->col = col;
  P->val = val;
  P->lhs = lhs;
  P->rhs = rhs;
  P->vartype = vartype;
  int64_t nnz = row_ptr[m];
  P->cptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  P->crow = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  P->mark = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!P->cptr || !P->crow || !P->mark || !fill) {
    free(fill);
    free(P->cptr);
    free(P->crow);
    free(P->mark);
    free(P);
    return NULL;
  }
  for (int64_t k = 0; k < nnz; k++) P->cptr[col[k] + 1]++;
  for (int32_t j = 0; j < n; j++) P->cptr[j + 1] += P->cptr[j];
  for (int32_t j = 0; j < n; j++) fill[j] = P->cptr[j];
  for (int32_t i = 0; i < m; i++)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) P->crow[fill[col[k]]++] = i;
  free(fill);
  return P;
}

void cs_destroy(cs_problem* P) {
  if (!P) return;
  free(P->cptr);
  free(P->crow);
  free(P->mark);
  free(P);
}

static int empty_domain(int is_int, double l, double u, double feas_tol) {
  if (is_int) return l > u;
  double s = fabs(l) > fabs(u) ? fabs(l) : fabs(u);
  if (s < 1.0) s = 1.0;
  return (l - u) > feas_tol * s;
}

/* A candidate against the current bound: integer rounding, drop beyond
   2^200, significance (the oracle's readings R4-R6). */
static int better_lower(double c, int is_int, double l, double eps, double tol, double* out) {
  if (is_int) c = ceil(c - eps);
  c = c + 0.0;
  if (!(fabs(c) <= 0x1p200)) return 0;
  int sig;
  if (l == -INFINITY) sig = 1;
  else if (is_int) sig = c > l;
  else sig = c > l + tol * (fabs(l) > 1.0 ? fabs(l) : 1.0);
  if (sig) *out = c;
  return sig;
}

static int better_upper(double c, int is_int, double u, double eps, double tol, double* out) {
  if (is_int) c = floor(c + eps);
  c = c + 0.0;
  if (!(fabs(c) <= 0x1p200)) return 0;
  int sig;
  if (u == INFINITY) sig = 1;
  else if (is_int) sig = c < u;
  else sig = c < u - tol * (fabs(u) > 1.0 ? fabs(u) : 1.0);
  if (sig) *out = c;
  return sig;
}

/* Propagates lb/ub in place.  Returns 0; *status and *sweeps as the oracle's
   run (sweeps count the last, change-free one).  Entry normalisation and
   the round-0 checks are the oracle's (reading R9). */
int cs_run(cs_problem* P, double eps_int, double cont_rel_tol, double feas_tol, double* lb,
           double* ub, int32_t max_sweeps, int32_t* status, int32_t* sweeps) {
  const int32_t m = P->m, n = P->n;
  *sweeps = 0;
  for (int32_t i = 0; i < m; i++) {
    int empty = P->row_ptr[i] == P->row_ptr[i + 1];
    for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1] && empty; k++)
      if (P->val[k] != 0.0) empty = 0;
    if (P->lhs[i] > P->rhs[i] || (empty && (P->lhs[i] > 0.0 || P->rhs[i] < 0.0))) {
      *status = CS_INFEASIBLE;
      return 0;
    }
  }
  for (int32_t j = 0; j < n; j++) {
    if (P->vartype[j]) {
      lb[j] = ceil(lb[j] - eps_int);
      ub[j] = floor(ub[j] + eps_int);
    }
    lb[j] += 0.0;
    ub[j] += 0.0;
    if (empty_domain(P->vartype[j], lb[j], ub[j], feas_tol)) {
      *status = CS_INFEASIBLE;
      return 0;
    }
  }
  if (max_sweeps == 0) {
    *status = CS_MAX_ROUNDS;
    return 0;
  }
  memset(P->mark, 1, (size_t)(m > 0 ? m : 1));
  *status = CS_MAX_ROUNDS;
  *sweeps = max_sweeps;
  for (int32_t s = 1; s <= max_sweeps; s++) {
    int found = 0;
    for (int32_t i = 0; i < m; i++) {
      if (!P->mark[i]) continue;
      P->mark[i] = 0;
      const int64_t k0 = P->row_ptr[i], k1 = P->row_ptr[i + 1];
      double amin = 0.0, amax = 0.0;
      int64_t cmin = 0, cmax = 0;
      for (int64_t k = k0; k < k1; k++) {
        const double a = P->val[k];
        if (a == 0.0) continue;
        const int32_t j = P->col[k];
        const double bmin = a > 0.0 ? lb[j] : ub[j];
        const double bmax = a > 0.0 ? ub[j] : lb[j];
        if (isinf(bmin)) cmin++;
        else amin = amin + a * bmin;
        if (isinf(bmax)) cmax++;
        else amax = amax + a * bmax;
      }
      const double rhs = P->rhs[i], lhs = P->lhs[i];
      /* can the constraint propagate */
      const int use_r = isfinite(rhs) && cmin <= 1 && !(cmax == 0 && amax <= rhs);
      const int use_l = isfinite(lhs) && cmax <= 1 && !(cmin == 0 && amin >= lhs);
      if (!use_r && !use_l) continue;
      const double sr = rhs - amin, sl = amax - lhs; /* slacks */
      for (int64_t k = k0; k < k1; k++) {
        const double a = P->val[k];
        if (a == 0.0) continue;
        const int32_t j = P->col[k];
        const int is_int = P->vartype[j] != 0;
        const double l = lb[j], u = ub[j];
        const double bmin = a > 0.0 ? l : u, bmax = a > 0.0 ? u : l;
        const double wa = fabs(a) * (u - l); /* inf for an unbounded domain */
        double cr = 0.0, cl = 0.0;
        int hr = 0, hl = 0;
        /* can the variable be tightened, then the side's candidate */
        if (use_r && !(cmin == 0 && sr > wa * (1.0 + 1e-12))) {
          if (cmin == 0) {
            cr = (rhs - amin) / a + bmin;
            hr = 1;
          } else if (isinf(bmin)) {
            cr = (rhs - amin) / a;
            hr = 1;
          }
        }
        if (use_l && !(cmax == 0 && sl > wa * (1.0 + 1e-12))) {
          if (cmax == 0) {
            cl = (lhs - amax) / a + bmax;
            hl = 1;
          } else if (isinf(bmax)) {
            cl = (lhs - amax) / a;
            hl = 1;
          }
        }
        if (!hr && !hl) continue;
        /* a > 0: the rhs side bounds x from above, the lhs side from below;
           a < 0 the reverse */
        double cand_lo = 0.0, cand_up = 0.0;
        int has_lo = 0, has_up = 0;
        if (a > 0.0) {
          if (hr) { cand_up = cr; has_up = 1; }
          if (hl) { cand_lo = cl; has_lo = 1; }
        } else {
          if (hr) { cand_lo = cr; has_lo = 1; }
          if (hl) { cand_up = cl; has_up = 1; }
        }
        double c;
        int tightened = 0;
        if (has_lo && better_lower(cand_lo, is_int, lb[j], eps_int, cont_rel_tol, &c)) {
          lb[j] = c;
          tightened = 1;
        }
        if (has_up && better_upper(cand_up, is_int, ub[j], eps_int, cont_rel_tol, &c)) {
          ub[j] = c;
          tightened = 1;
        }
        if (tightened) {
          found = 1;
          for (int64_t q = P->cptr[j]; q < P->cptr[j + 1]; q++) P->mark[P->crow[q]] = 1;
        }
      }
    }
    int inf = 0;
    for (int32_t j = 0; j < n && !inf; j++)
      inf = empty_domain(P->vartype[j], lb[j], ub[j], feas_tol);
    if (inf) {
      *status = CS_INFEASIBLE;
      *sweeps = s;
      return 0;
    }
    if (!found) {
      *status = CS_CONVERGED;
      *sweeps = s;
      return 0;
    }
  }
  return 0;
}
