"""Pins of the oracle against facts fixed by the paper and by mathematics.

Every check takes an ``oracle.Oracle`` so the same checks can also run
against deliberately broken oracle builds (``test_oracle_mutants.py``):
each plausible mistake must make at least one check fail.

None of these checks re-types the oracle's formulas; they compare it with
exact rational arithmetic, hand-derived closed forms, brute-force
enumeration, a linear-programming projection, algebraic invariants of the
method, and the sequential algorithm's limit point.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np

import oracle as oracle_mod
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(v):
    if isinstance(v, str):
        return {"inf": math.inf, "-inf": -math.inf}[v]
    return float(v)


def load_closed_forms():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        return json.load(f)["cases"]


def case_instance(c):
    n = len(c["lb"])
    return synth.from_rows(
        c["rows"], [_num(v) for v in c["lhs"]], [_num(v) for v in c["rhs"]],
        [_num(v) for v in c["lb"]], [_num(v) for v in c["ub"]], c["vartype"], n=n,
        name=c["name"])


def case_params(c):
    p = oracle_mod.Params()
    for k, v in c.get("params", {}).items():
        setattr(p, k, float(v))
    return p


# ---------------------------------------------------------------------------
# exact activity sums (reading: the exact sum rounded once)
# ---------------------------------------------------------------------------
def _exact(a, b):
    s = sum((Fraction(x) * Fraction(y) for x, y in zip(a, b)), Fraction(0))
    return float(s) + 0.0


def check_exact_dot_special(orc):
    two = 2.0
    cases = [
        ([1e100, 1.0, -1e100], [1.0, 1.0, 1.0], 1.0),  # cancellation
        ([two**53, 1.0], [1.0, 1.0], two**53),  # exact tie -> even
        ([two**53, 1.0, two**-60], [1.0, 1.0, 1.0], two**53 + 2),  # above the tie
        ([two**53, 3.0], [1.0, 1.0], two**53 + 4),  # tie 2^53+3 -> even (2^53+4)
        ([two**-1074, two**-1074], [1.0, 1.0], two**-1073),  # subnormals
        ([1e-300], [1e-300], 0.0),  # underflow to zero
        ([0.1, 0.2, -0.3], [1.0, 1.0, 1.0], _exact([0.1, 0.2, -0.3], [1, 1, 1])),
        ([3.0, -2.0], [0.5, 0.75], 0.0),
        ([], [], 0.0),
        ([-1.0], [0.0], 0.0),
    ]
    for a, b, want in cases:
        got = orc.exact_dot(np.array(a, dtype=float), np.array(b, dtype=float))
        assert got == want and math.copysign(1, got) == math.copysign(1, want), (a, b, got, want)


def check_exact_dot_random(orc, trials=300, seed=7):
    rng = np.random.default_rng(seed)
    for t in range(trials):
        k = int(rng.integers(1, 40))
        mant = rng.uniform(-1, 1, size=(2, k))
        ex = rng.integers(-60, 60, size=(2, k))
        if t % 3 == 0:
            ex = rng.integers(-500, 500, size=(2, k))
        a = np.ldexp(mant[0], ex[0])
        b = np.ldexp(mant[1], ex[1])
        if t % 5 == 0:  # force heavy cancellation
            a = np.concatenate([a, -a[: k // 2]])
            b = np.concatenate([b, b[: k // 2]])
        got = orc.exact_dot(a, b)
        want = _exact(a, b)
        assert got == want, (t, got, want)


def check_activities_exact_rows(orc):
    """Every row's activity equals the exact rational sum, rounded once."""
    inst = synth.config0()
    L, U = inst.lb.copy(), inst.ub.copy()
    # tighten a few bounds to non-trivial fractional values
    rng = np.random.default_rng(3)
    cont = np.nonzero((inst.vartype == 0) & np.isfinite(L) & np.isfinite(U))[0]
    L[cont] = L[cont] + rng.uniform(0, 10, size=cont.size) / 3.0
    mnf, mni, mxf, mxi = orc.activities(inst, L, U)
    for i in range(0, inst.m, 7):
        sl = slice(inst.row_ptr[i], inst.row_ptr[i + 1])
        a = inst.vals[sl]
        j = inst.col_idx[sl]
        bmin = np.where(a > 0, L[j], U[j])
        bmax = np.where(a > 0, U[j], L[j])
        fin_min = np.isfinite(bmin)
        fin_max = np.isfinite(bmax)
        assert mni[i] == np.count_nonzero(~fin_min)
        assert mxi[i] == np.count_nonzero(~fin_max)
        assert mnf[i] == _exact(a[fin_min], bmin[fin_min]), i
        assert mxf[i] == _exact(a[fin_max], bmax[fin_max]), i


def check_activities_spmv(orc):
    """With finite bounds, min act = A+ l + A- u and max act = A+ u + A- l
    (the SpMV form of Sec. 3.1), checked with scipy's sparse product."""
    import scipy.sparse as sp

    inst = synth.config1(1)
    fin = np.isfinite(inst.lb) & np.isfinite(inst.ub)
    L = np.where(fin, inst.lb, -5.0)
    U = np.where(fin, inst.ub, 7.0)
    A = sp.csr_matrix((inst.vals, inst.col_idx, inst.row_ptr), shape=(inst.m, inst.n))
    Ap = A.maximum(0)
    An = A.minimum(0)
    mn_ref = Ap @ L + An @ U
    mx_ref = Ap @ U + An @ L
    scale = abs(A) @ np.maximum(np.abs(L), np.abs(U))
    mnf, mni, mxf, mxi = orc.activities(inst, L, U)
    assert not mni.any() and not mxi.any()
    assert np.all(np.abs(mnf - mn_ref) <= 1e-13 * scale + 1e-300)
    assert np.all(np.abs(mxf - mx_ref) <= 1e-13 * scale + 1e-300)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
def check_closed_forms(orc):
    for c in load_closed_forms():
        inst = case_instance(c)
        r = orc.run(inst, inst.lb, inst.ub, c["max_rounds"], case_params(c), c.get("store", 64))
        e = c["expect"]
        assert (r.status, r.rounds) == (e["status"], e["rounds"]), (c["name"], r.status, r.rounds)
        if "lb" in e:
            want_lb = np.array([_num(v) for v in e["lb"]])
            want_ub = np.array([_num(v) for v in e["ub"]])
            if "ub_exact" in e:
                want_ub[:] = 2.0 + 98.0 * 2.0**-25
            if "lb_exact" in e:
                want_lb[:] = -(2.0 + 98.0 * 2.0**-25)
            assert np.array_equal(r.lb, want_lb), (c["name"], r.lb, want_lb)
            assert np.array_equal(r.ub, want_ub), (c["name"], r.ub, want_ub)
        if "min_flags" in e:
            assert r.flags >= e["min_flags"], (c["name"], r.flags)


def cascade_instance(m):
    """x_{k+1} - x_k >= 0 for k = 1..m; x_1 in [5,10], the rest in [0,10]."""
    rows = [[(k, -1.0), (k + 1, 1.0)] for k in range(m)]
    lb = np.zeros(m + 1)
    lb[0] = 5.0
    ub = np.full(m + 1, 10.0)
    return synth.from_rows(rows, np.zeros(m), np.full(m, np.inf), lb, ub, np.ones(m + 1), n=m + 1,
                           name=f"cascade{m}")


def check_cascade(orc):
    """The cascading pattern of Sec. 2.2: round k tightens only x_{k+1}, so
    synchronous rounds need m of them (plus the change-free last round)."""
    for m in (1, 2, 7, 30):
        inst = cascade_instance(m)
        r = orc.run(inst, inst.lb, inst.ub, 100)
        assert (r.status, r.rounds) == (oracle_mod.CONVERGED, m + 1), (m, r.status, r.rounds)
        assert np.all(r.lb == 5.0) and np.all(r.ub == 10.0)
        # after k rounds exactly x_1..x_{k+1} have lower bound 5
        k = max(1, m // 2)
        rk = orc.run(inst, inst.lb, inst.ub, k)
        assert rk.status == oracle_mod.MAX_ROUNDS and rk.rounds == k
        assert np.all(rk.lb[: k + 1] == 5.0) and np.all(rk.lb[k + 1:] == 0.0)
    inst = cascade_instance(99)
    r = orc.run(inst, inst.lb, inst.ub, 100)
    assert (r.status, r.rounds) == (oracle_mod.CONVERGED, 100)
    inst = cascade_instance(100)
    r = orc.run(inst, inst.lb, inst.ub, 100)
    assert (r.status, r.rounds) == (oracle_mod.MAX_ROUNDS, 100)
    # the sequential order of Algorithm 1 takes the whole cascade in one sweep
    s = orc.run_seq(inst, inst.lb, inst.ub, 100)
    assert (s.status, s.rounds) == (oracle_mod.CONVERGED, 2)
    assert np.all(s.lb == 5.0)


# ---------------------------------------------------------------------------
# soundness and tightness
# ---------------------------------------------------------------------------
def _feasible_points(inst):
    lo = inst.lb.astype(int)
    hi = inst.ub.astype(int)
    A = np.zeros((inst.m, inst.n))
    for i in range(inst.m):
        sl = slice(inst.row_ptr[i], inst.row_ptr[i + 1])
        A[i, inst.col_idx[sl]] = inst.vals[sl]
    grids = [range(lo[j], hi[j] + 1) for j in range(inst.n)]
    pts = np.array(list(itertools.product(*grids)), dtype=float)
    act = pts @ A.T  # small integers: exact
    ok = np.all((act >= inst.lhs) & (act <= inst.rhs), axis=1)
    return pts[ok]


def check_brute_force_integer(orc, count=60):
    """Every integer point of the box that satisfies all rows stays inside
    the propagated bounds; INFEASIBLE only when there is no such point."""
    n_inf = n_feas = 0
    for s in range(count):
        inst = synth.random_small(s, m=int(3 + s % 5), n=int(3 + s % 4), box=4, slack=3.0)
        pts = _feasible_points(inst)
        r = orc.run(inst, inst.lb, inst.ub, 100)
        assert r.status != oracle_mod.MAX_ROUNDS, s
        if r.status == oracle_mod.INFEASIBLE:
            assert pts.shape[0] == 0, (s, "infeasible but has points")
            n_inf += 1
            continue
        n_feas += 1
        if pts.shape[0]:
            assert np.all(pts >= r.lb - 1e-12) and np.all(pts <= r.ub + 1e-12), s
            # the bounds are integral for integer variables
            assert np.all(r.lb == np.ceil(r.lb)) and np.all(r.ub == np.floor(r.ub))
    assert n_feas > 0


def check_single_row_projection(orc, count=40):
    """For one continuous row over a finite box, the propagated bounds are the
    exact projection of the feasible set onto each coordinate (linear
    programming: min and max of x_j)."""
    from scipy.optimize import linprog

    for s in range(count):
        rng = np.random.default_rng(1000 + s)
        n = int(rng.integers(2, 6))
        a = rng.integers(1, 6, size=n) * np.where(rng.random(n) < 0.5, -1, 1).astype(float)
        lo = rng.integers(-5, 1, size=n).astype(float)
        hi = lo + rng.integers(1, 8, size=n)
        x0 = lo + rng.random(n) * (hi - lo)
        s0 = float(a @ x0)
        lhs = s0 - float(rng.integers(0, 3)) if rng.random() < 0.8 else -np.inf
        rhs = s0 + float(rng.integers(0, 3)) if rng.random() < 0.8 else np.inf
        inst = synth.from_rows([[(j, a[j]) for j in range(n)]], [lhs], [rhs], lo, hi,
                               np.zeros(n), n=n)
        r = orc.run(inst, lo, hi, 100, oracle_mod.Params(cont_rel_tol=0.0))
        assert r.status == oracle_mod.CONVERGED, s
        A_ub, b_ub = [], []
        if np.isfinite(rhs):
            A_ub.append(a); b_ub.append(rhs)
        if np.isfinite(lhs):
            A_ub.append(-a); b_ub.append(-lhs)
        for j in range(n):
            c = np.zeros(n); c[j] = 1.0
            kw = dict(A_ub=np.array(A_ub) if A_ub else None, b_ub=np.array(b_ub) if b_ub else None,
                      bounds=list(zip(lo, hi)), method="highs")
            lo_j = linprog(c, **kw).fun
            hi_j = -linprog(-c, **kw).fun
            assert abs(r.lb[j] - lo_j) <= 1e-9 * max(1, abs(lo_j)), (s, j, r.lb[j], lo_j)
            assert abs(r.ub[j] - hi_j) <= 1e-9 * max(1, abs(hi_j)), (s, j, r.ub[j], hi_j)


def check_x0_contained(orc):
    """The point every row was drawn around stays inside the bounds."""
    for inst in (synth.config0(), synth.config0(1)):
        r = orc.run(inst, inst.lb, inst.ub, 100)
        assert r.status == oracle_mod.CONVERGED
        tol = 1e-6 * np.maximum(1.0, np.abs(inst.x0))
        assert np.all(r.lb - tol <= inst.x0) and np.all(inst.x0 <= r.ub + tol)
        assert np.all(r.lb >= np.where(inst.vartype == 1, np.ceil(inst.lb), inst.lb))
        assert np.all(r.ub <= inst.ub)


# ---------------------------------------------------------------------------
# invariants of the method
# ---------------------------------------------------------------------------
def check_idempotent_and_resume(orc):
    inst = synth.config0()
    r = orc.run(inst, inst.lb, inst.ub, 100)
    assert r.status == oracle_mod.CONVERGED and r.rounds > 3
    again = orc.run(inst, r.lb, r.ub, 100)
    assert (again.status, again.rounds) == (oracle_mod.CONVERGED, 1)
    assert np.array_equal(again.lb, r.lb) and np.array_equal(again.ub, r.ub)
    # rounds are a Markov chain in (l, u): k rounds then the rest = all
    k = r.rounds // 2
    a = orc.run(inst, inst.lb, inst.ub, k)
    assert (a.status, a.rounds) == (oracle_mod.MAX_ROUNDS, k)
    b = orc.run(inst, a.lb, a.ub, 100)
    assert b.status == oracle_mod.CONVERGED and a.rounds + b.rounds == r.rounds
    assert np.array_equal(b.lb, r.lb) and np.array_equal(b.ub, r.ub)
    # the round function agrees with the run
    Ln, Un, ch, inf, _ = orc.round_(inst, a.lb, a.ub)
    a1 = orc.run(inst, inst.lb, inst.ub, k + 1)
    assert ch and not inf
    assert np.array_equal(Ln, a1.lb) and np.array_equal(Un, a1.ub)


def check_monotone(orc):
    inst = synth.config0(2)
    r = orc.run(inst, inst.lb, inst.ub, 3)
    lb0 = np.where(inst.vartype == 1, np.ceil(inst.lb - 1e-6), inst.lb)
    assert np.all(r.lb >= lb0) and np.all(r.ub <= inst.ub)
    Ln, Un, _, _, _ = orc.round_(inst, r.lb, r.ub)
    assert np.all(Ln >= r.lb) and np.all(Un <= r.ub)


def _permute(inst, row_perm=None, col_perm=None, within_row_rev=False):
    """Same system with rows reordered, variables relabelled (new index of old
    variable j is col_perm[j]) and/or every row's entries reversed."""
    m, n = inst.m, inst.n
    rp = row_perm if row_perm is not None else np.arange(m)
    cp = col_perm if col_perm is not None else np.arange(n)
    rows = []
    for i in rp:
        sl = slice(inst.row_ptr[i], inst.row_ptr[i + 1])
        ent = list(zip(cp[inst.col_idx[sl]].tolist(), inst.vals[sl].tolist()))
        if within_row_rev:
            ent = ent[::-1]
        rows.append(ent)
    inv = np.empty(n, dtype=np.int64)
    inv[cp] = np.arange(n)
    return synth.from_rows(rows, inst.lhs[rp], inst.rhs[rp], inst.lb[inv], inst.ub[inv],
                           inst.vartype[inv], n=n)


def check_permutation_invariance(orc):
    """Synchronous rounds do not depend on the order of rows, of variables,
    or of entries within a row (App. B studies the order's effect on speed):
    with exactly rounded activities the results are bitwise identical."""
    inst = synth.config0(3)
    base = orc.run(inst, inst.lb, inst.ub, 100)
    rng = np.random.default_rng(11)
    rperm = rng.permutation(inst.m)
    cperm = rng.permutation(inst.n)
    p = _permute(inst, rperm, cperm, within_row_rev=True)
    r = orc.run(p, p.lb, p.ub, 100)
    assert (r.status, r.rounds) == (base.status, base.rounds)
    assert np.array_equal(r.lb[cperm], base.lb) and np.array_equal(r.ub[cperm], base.ub)


def check_sequential_limit_point(orc, count=40):
    """On bounded pure-integer systems the fixed-point iteration has one limit
    (Sec. 1.1); Algorithm 1's order must reach the same bounds."""
    same = 0
    for s in range(count):
        inst = synth.random_small(500 + s, m=int(4 + s % 6), n=int(4 + s % 5), box=6, slack=4.0)
        a = orc.run(inst, inst.lb, inst.ub, 200)
        b = orc.run_seq(inst, inst.lb, inst.ub, 200)
        assert a.status != oracle_mod.MAX_ROUNDS and b.status != oracle_mod.MAX_ROUNDS
        assert a.status == b.status, s
        if a.status == oracle_mod.CONVERGED:
            assert np.array_equal(a.lb, b.lb) and np.array_equal(a.ub, b.ub), s
            assert b.rounds <= a.rounds, s
            same += 1
    assert same > count // 2


def check_validation(orc):
    base = synth.from_rows([[(0, 1.0), (1, 1.0)]], [-np.inf], [3.0], [0, 0], [5, 5], [1, 1], n=2)
    ok = orc.run(base, base.lb, base.ub, 10)
    assert ok.status == oracle_mod.CONVERGED

    def bad(**kw):
        inst = synth.from_rows(kw.get("rows", [[(0, 1.0), (1, 1.0)]]), kw.get("lhs", [-np.inf]),
                               kw.get("rhs", [3.0]), kw.get("lb", [0, 0]), kw.get("ub", [5, 5]),
                               kw.get("vt", [1, 1]), n=2)
        try:
            orc.run(inst, inst.lb, inst.ub, 10)
        except oracle_mod.OracleError:
            return True
        return False

    assert bad(rows=[[(0, np.nan), (1, 1.0)]])
    assert bad(rows=[[(0, 1.0), (0, 1.0)]])  # duplicate column
    assert bad(rows=[[(0, 1.0), (2, 1.0)]])  # column out of range
    assert bad(rows=[[(0, 1e-30), (1, 1.0)]])  # coefficient below 2^-64
    assert bad(lhs=[np.inf])
    assert bad(rhs=[-np.inf])
    assert bad(lb=[np.inf, 0])
    assert bad(ub=[0, -np.inf])
    assert bad(lb=[np.nan, 0])
    assert bad(ub=[0, 1e70])  # beyond 2^200
    assert bad(vt=[2, 1])


# ---------------------------------------------------------------------------
# single-precision bound store, rounded outward (reading R12)
# ---------------------------------------------------------------------------
F32_MIN = float(np.finfo(np.float32).tiny)  # smallest normal single
F32_MAX = float(np.finfo(np.float32).max)


def _in_store_grid(x):
    """x is 0, an infinity, or a normal single-precision number."""
    if x == 0.0 or math.isinf(x):
        return True
    if not F32_MIN <= abs(x) <= F32_MAX:
        return False
    return float(np.float32(x)) == x


def _grid_next(f, up):
    """The neighbour of grid member f in the given direction (the grid skips
    the subnormal singles)."""
    if up:
        if f == -math.inf:
            return -F32_MAX
        if f == -F32_MIN:
            return 0.0
        if f == 0.0:
            return F32_MIN
        if f == F32_MAX:
            return math.inf
        return float(np.nextafter(np.float32(f), np.float32(np.inf)))
    return -_grid_next(-f, True)


def _store_probe_values(seed=5, count=6000):
    rng = np.random.default_rng(seed)
    vals = [0.0, -0.0, math.inf, -math.inf, F32_MIN, -F32_MIN, F32_MAX, -F32_MAX,
            F32_MIN / 2, -F32_MIN / 2, 5e-324, -5e-324, F32_MAX * (1 + 2.0**-30), 1e39, -1e39,
            0.1, 0.9, 1.9999999, 1.0 + 2.0**-30, 16777217.0, -16777217.0, 2.0**200, -2.0**200]
    # random doubles over the whole exponent range a bound may take
    e = rng.integers(-160, 161, size=count)
    m = 1.0 + rng.random(count)
    sgn = np.where(rng.random(count) < 0.5, -1.0, 1.0)
    vals += list(sgn * np.ldexp(m, e))
    # singles, and the doubles next to them and halfway between two of them
    f = np.float32(np.ldexp(m[:1500], np.clip(e[:1500], -120, 120)) * sgn[:1500])
    for x in f.astype(np.float64):
        vals += [x, np.nextafter(x, np.inf), np.nextafter(x, -np.inf)]
        y = float(np.nextafter(np.float32(x), np.float32(np.inf)))
        vals.append((x + y) / 2)
    # integers near 2^24, where the singles stop being every integer
    vals += [float(2**24 + k) for k in range(-3, 6)]
    return [float(v) for v in vals]


def check_store_grid(orc):
    """The store's roundings, by their definition: down(x) is a grid member
    not above x whose upper neighbour is above x, up(x) the mirror image;
    grid members map to themselves."""
    for x in _store_probe_values():
        d, u = orc.store_down(x), orc.store_up(x)
        assert _in_store_grid(d) and _in_store_grid(u), (x, d, u)
        assert d <= x <= u, (x, d, u)
        if not math.isinf(x):
            assert _grid_next(d, True) > x, (x, d)
            assert _grid_next(u, False) < x, (x, u)
        if _in_store_grid(x):
            assert d == x == u, (x, d, u)
        assert not (d == 0.0 and math.copysign(1.0, d) < 0), x
        assert not (u == 0.0 and math.copysign(1.0, u) < 0), x


def check_store_integer_identity(orc, count=40):
    """Integer bounds below 2^24 are grid members: on pure-integer systems the
    single-precision store gives the FP64 store's results bitwise."""
    for s in range(count):
        inst = synth.random_small(700 + s, m=int(3 + s % 6), n=int(3 + s % 5), box=8, slack=4.0)
        a = orc.run(inst, inst.lb, inst.ub, 200)
        b = orc.run(inst, inst.lb, inst.ub, 200, store=32)
        assert (a.status, a.rounds) == (b.status, b.rounds), s
        if a.status != oracle_mod.INFEASIBLE:
            assert np.array_equal(a.lb, b.lb) and np.array_equal(a.ub, b.ub), s


def check_store_sound(orc, count=40):
    """Outward rounding only loosens: on one continuous row over a box the
    stored bounds contain the exact projection (linear programming) and stay
    within a few single-precision steps of it; feasible integer points stay
    inside; every stored bound is a grid member."""
    from scipy.optimize import linprog

    for s in range(count):
        rng = np.random.default_rng(3000 + s)
        n = int(rng.integers(2, 6))
        a = rng.integers(1, 6, size=n) * np.where(rng.random(n) < 0.5, -1, 1).astype(float)
        lo = rng.integers(-5, 1, size=n).astype(float) + 0.1 * rng.integers(0, 10, size=n)
        hi = lo + rng.integers(1, 8, size=n) + 0.3
        x0 = lo + rng.random(n) * (hi - lo)
        s0 = float(a @ x0)
        lhs = s0 - 0.7 * float(rng.integers(0, 3))
        rhs = s0 + 0.7 * float(rng.integers(0, 3))
        inst = synth.from_rows([[(j, a[j]) for j in range(n)]], [lhs], [rhs], lo, hi,
                               np.zeros(n), n=n)
        r = orc.run(inst, lo, hi, 100, oracle_mod.Params(cont_rel_tol=0.0), store=32)
        assert r.status == oracle_mod.CONVERGED, s
        assert all(_in_store_grid(v) for v in np.concatenate([r.lb, r.ub])), s
        kw = dict(A_ub=np.array([a, -a]), b_ub=np.array([rhs, -lhs]), bounds=list(zip(lo, hi)),
                  method="highs")
        for j in range(n):
            c = np.zeros(n)
            c[j] = 1.0
            lo_j = linprog(c, **kw).fun
            hi_j = -linprog(-c, **kw).fun
            tol = 1e-9 * max(1.0, abs(lo_j), abs(hi_j))
            assert r.lb[j] <= lo_j + tol and r.ub[j] >= hi_j - tol, (s, j)
            assert r.lb[j] >= lo_j - 1e-4 and r.ub[j] <= hi_j + 1e-4, (s, j, r.lb[j], lo_j)
    for s in range(count):
        inst = synth.random_small(900 + s, m=int(3 + s % 5), n=int(3 + s % 4), box=4, slack=3.0)
        pts = _feasible_points(inst)
        r = orc.run(inst, inst.lb, inst.ub, 100, store=32)
        if r.status == oracle_mod.INFEASIBLE:
            assert pts.shape[0] == 0, s
        elif pts.shape[0]:
            assert np.all(pts >= r.lb) and np.all(pts <= r.ub), s
    for inst in (synth.config0(), synth.config0(1)):
        r = orc.run(inst, inst.lb, inst.ub, 100, store=32)
        assert r.status == oracle_mod.CONVERGED
        tol = 1e-6 * np.maximum(1.0, np.abs(inst.x0))
        assert np.all(r.lb - tol <= inst.x0) and np.all(inst.x0 <= r.ub + tol)
        assert all(_in_store_grid(v) for v in np.concatenate([r.lb, r.ub]))


ALL_CHECKS = [
    check_exact_dot_special,
    check_exact_dot_random,
    check_activities_exact_rows,
    check_activities_spmv,
    check_closed_forms,
    check_cascade,
    check_brute_force_integer,
    check_single_row_projection,
    check_x0_contained,
    check_idempotent_and_resume,
    check_monotone,
    check_permutation_invariance,
    check_sequential_limit_point,
    check_validation,
    check_store_grid,
    check_store_integer_identity,
    check_store_sound,
]
