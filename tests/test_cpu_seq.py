"""The sequential baseline (Algorithm 1 with constraint marking, plain double
sums; oracle/cpu_seq.c) against what the paper and the mathematics fix
(CPU only).

It is not the oracle, and its sums are not exactly rounded, so the
closed forms that pin exact rounding are left out.  Where the iteration has
one limit point that both orders reach in finitely many steps (bounded
integer systems, Sec. 1.1), its bounds must be the oracle's; elsewhere they
agree within the propagation's own threshold.
"""
import numpy as np

import oracle
import oracle_pins as pins
import synth

TOL = 1e-9


def close(a, b, tol=TOL):
    both_inf = np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))
    fin = np.isfinite(a) & np.isfinite(b)
    ok = both_inf.copy()
    ok[fin] = np.abs(a[fin] - b[fin]) <= tol + tol * np.abs(b[fin])
    return bool(ok.all())


def test_closed_forms():
    for c in pins.load_closed_forms():
        if c["name"].startswith("exact_sum"):
            continue  # plain sums round differently on purpose
        if c.get("store", 64) != 64:
            continue  # the sequential baseline keeps its bounds in FP64
        inst = pins.case_instance(c)
        e = c["expect"]
        cs = oracle.CpuSeq(inst)
        r, _ = cs.run(inst.lb, inst.ub, 0 if c["max_rounds"] == 0 else 1000,
                      pins.case_params(c))
        name = c["name"]
        assert r.status == e["status"], (name, r.status)
        if "lb" not in e or r.status == oracle.INFEASIBLE:
            continue
        want_lb = np.array([pins._num(v) for v in e["lb"]])
        want_ub = np.array([pins._num(v) for v in e["ub"]])
        if c["name"].startswith("geometric_cycle"):
            # the threshold stops both orders near the limit 2 (resp. -2)
            want_ub[:] = np.where(np.isfinite(want_ub) & (want_ub > 1), 2.0, want_ub)
            want_lb[:] = np.where(np.isfinite(want_lb) & (want_lb < -1), -2.0, want_lb)
            assert close(r.lb, want_lb, 1e-5) and close(r.ub, want_ub, 1e-5), (name, r.lb, r.ub)
        else:
            assert close(r.lb, want_lb) and close(r.ub, want_ub), (name, r.lb, r.ub)


def test_cascade_in_one_sweep():
    """Sec. 2.2: the sequential order takes the whole cascade in one sweep
    (plus the change-free one), where synchronous rounds need m + 1."""
    for m in (1, 7, 100):
        inst = pins.cascade_instance(m)
        r, _ = oracle.CpuSeq(inst).run(inst.lb, inst.ub, 100)
        assert (r.status, r.rounds) == (oracle.CONVERGED, 2)
        assert np.all(r.lb == 5.0)


def test_limit_point_bounded_integer():
    """Bounded pure-integer systems: the oracle's limit point, exactly, in
    no more sweeps than the synchronous rounds."""
    same = 0
    for s in range(60):
        inst = synth.random_small(900 + s, m=int(4 + s % 6), n=int(4 + s % 5), box=6, slack=4.0)
        a = oracle.run(inst, inst.lb, inst.ub, 200)
        b, _ = oracle.CpuSeq(inst).run(inst.lb, inst.ub, 200)
        assert a.status == b.status, s
        if a.status == oracle.CONVERGED:
            assert np.array_equal(a.lb, b.lb) and np.array_equal(a.ub, b.ub), s
            assert b.rounds <= a.rounds, s
            same += 1
    assert same > 30


def test_brute_force_soundness():
    """Every feasible integer point of small boxes stays inside the bounds;
    INFEASIBLE only when there is none."""
    for s in range(40):
        inst = synth.random_small(1200 + s, m=int(3 + s % 5), n=int(3 + s % 4), box=5,
                                  int_frac=1.0)
        pts = pins._feasible_points(inst)
        r, _ = oracle.CpuSeq(inst).run(inst.lb, inst.ub, 200)
        if r.status == oracle.INFEASIBLE:
            assert pts.shape[0] == 0, s
            continue
        assert np.all(pts >= r.lb - 1e-9) and np.all(pts <= r.ub + 1e-9), s


def test_config0_within_threshold():
    """Mixed integer / continuous: both orders stop near the same limit; the
    integer bounds agree and the continuous ones within the relative
    threshold's reach."""
    inst = synth.config0()
    a = oracle.run(inst, inst.lb, inst.ub, 100)
    b, _ = oracle.CpuSeq(inst).run(inst.lb, inst.ub, 1000)
    assert a.status == b.status == oracle.CONVERGED
    integer = inst.vartype == 1
    assert np.array_equal(a.lb[integer], b.lb[integer]) and np.array_equal(a.ub[integer],
                                                                         b.ub[integer])
    assert close(a.lb, b.lb, 1e-3) and close(a.ub, b.ub, 1e-3)
    assert b.rounds < a.rounds
