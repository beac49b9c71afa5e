"""GPU parity: the HIP library (through its C ABI) against the oracle.

Bar: status and rounds identical; bounds bitwise identical (activities are
exactly rounded on both sides and every other step is the same IEEE
operation, so no tolerance is needed; the comparison helper still reports
the largest deviation for diagnosis).  Runs go through every round-loop
driver; the graph driver replays its captured rounds many times per run,
with other drivers' runs in between.
"""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest
from bitwise import differing, same_bits

import oracle
import oracle_pins as pins
import synth

pytestmark = pytest.mark.gpu

LOOPS = ("persistent", "stream", "host", "graph", "graph_all")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def lib(torch_cuda):
    from paper_2009_07785_amd import binding

    return binding


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same(tag, got, ref):
    """Bitwise equality of status, rounds and (unless infeasible) bounds."""
    res, lb, ub = got
    assert (res.status, res.rounds) == (ref.status, ref.rounds), (
        f"{tag}: status/rounds {res.status}/{res.rounds} vs oracle {ref.status}/{ref.rounds}")
    if ref.status == oracle.INFEASIBLE:
        return
    for name, g, r in (("lb", lb, ref.lb), ("ub", ub, ref.ub)):
        bad = differing(g, r)
        if bad.size:
            fin = np.isfinite(g[bad]) & np.isfinite(r[bad])
            dev = np.max(np.abs(g[bad][fin] - r[bad][fin])) if fin.any() else math.inf
            raise AssertionError(f"{tag}: {name} differs at {bad.size} vars (first {bad[:5]}, "
                                 f"max |diff| {dev})")


def gpu_run(lib, inst, lb, ub, max_rounds, loop="persistent", params=None):
    kw = {}
    if params is not None:
        kw = dict(eps_int=params.eps_int, cont_rel_tol=params.cont_rel_tol,
                  feas_tol=params.feas_tol)
    with lib.Problem.from_instance(inst, **kw) as p:
        p.set_loop(loop)
        return p.run(lb, ub, max_rounds)


def check_against_oracle(lib, inst, max_rounds=100, params=None, loops=LOOPS, lb=None, ub=None):
    lb = inst.lb if lb is None else lb
    ub = inst.ub if ub is None else ub
    ref = oracle.run(inst, lb, ub, max_rounds, params)
    # candidates within eps_int of an integer before rounding: flagged and
    # counted; the comparison stays bitwise for them too
    say(f"  {inst.name}: oracle {oracle.STATUS_NAMES[ref.status]}"
        f" after {ref.rounds} rounds, near-integer candidates flagged: {ref.flags}")
    for loop in loops:
        say(f"  {inst.name} loop={loop} max_rounds={max_rounds}")
        assert_same(f"{inst.name}/{loop}", gpu_run(lib, inst, lb, ub, max_rounds, loop, params), ref)
    return ref


def test_closed_forms(lib):
    for c in pins.load_closed_forms():
        inst = pins.case_instance(c)
        check_against_oracle(lib, inst, c["max_rounds"], pins.case_params(c))


def test_config0(lib):
    ref = check_against_oracle(lib, synth.config0())
    assert ref.status == oracle.CONVERGED and ref.rounds > 5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_layout_mix(lib, seed):
    """Every lanes-per-row class, ragged tails and long rows that tighten."""
    ref = check_against_oracle(lib, synth.layout_mix(seed))
    assert ref.status == oracle.CONVERGED


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_code_edges(lib, seed):
    """Integer bounds on both sides of the compact codes' range [-126, 126],
    at its edges and infinite, moving into it as the rounds tighten them:
    codes decode to the pairs' exact values and escaped variables gather
    their pairs, so the results stay the oracle's bitwise."""
    inst = synth.code_edges(seed)
    ref = check_against_oracle(lib, inst)
    assert ref.status == oracle.CONVERGED and ref.rounds > 5
    for steps in (4, 16):
        with lib.Problem.from_instance(inst, steps=steps) as p:
            assert_same(f"{inst.name}/steps={steps}", p.run(inst.lb, inst.ub, 100), ref)


def test_nnz_split_layout(lib):
    """The nnz-split layout (rows in input order packed into 512-entry waves,
    8 consecutive entries per lane, rows spanning lanes joined by a
    segmented scan, longer rows in segments) gives the oracle's results
    bitwise on every driver."""
    insts = [synth.config0(), synth.layout_mix(0), synth.layout_mix(1), synth.code_edges(0),
             synth.config1(1), synth.config3_matrix(50_000, 25_000), pins.cascade_instance(99)]
    insts += [synth.random_small(s, m=int(3 + s % 9), n=int(3 + s % 7), box=6,
                                 int_frac=[1.0, 0.5, 0.0][s % 3], inf_frac=0.2 * (s % 2))
              for s in range(12)]
    for c in pins.load_closed_forms():
        insts.append((pins.case_instance(c), c["max_rounds"], pins.case_params(c)))
    for item in insts:
        inst, max_rounds, params = item if isinstance(item, tuple) else (item, 100, None)
        ref = oracle.run(inst, inst.lb, inst.ub, max_rounds, params)
        kw = {} if params is None else dict(eps_int=params.eps_int,
                                            cont_rel_tol=params.cont_rel_tol,
                                            feas_tol=params.feas_tol)
        with lib.Problem.from_instance(inst, layout=1, **kw) as p:
            assert p.info()["layout"] == 1
            for loop in LOOPS:
                p.set_loop(loop)
                assert_same(f"{inst.name}/nnz-split/{loop}", p.run(inst.lb, inst.ub, max_rounds),
                            ref)
            p.set_marking(True)
            p.set_loop("stream")
            assert_same(f"{inst.name}/nnz-split/marked", p.run(inst.lb, inst.ub, max_rounds), ref)
    # batches and serving refuse the layout
    with lib.Problem.from_instance(synth.config0(), layout=1) as p:
        with pytest.raises(lib.PropError):
            p.run_batch(np.stack([synth.config0().lb] * 2), np.stack([synth.config0().ub] * 2), 10)


def test_powerlaw_hot_variables(lib):
    """Power-law columns: dozens of variables above the degree at which the
    kernels spread their candidate targets over stripe copies."""
    inst = synth.config3_matrix(50_000, 25_000)
    deg = np.bincount(inst.col_idx, minlength=inst.n)
    assert (deg >= 512).sum() >= 10
    ref = check_against_oracle(lib, inst)
    assert ref.rounds >= 3  # slow continuous convergence: the root hits the round limit
    nodes = [synth.node_bounds(inst, 21_000 + k) for k in range(4)]
    for lb, ub in nodes:
        check_against_oracle(lib, inst, lb=lb, ub=ub, loops=("stream",))


def test_random_small(lib):
    for s in range(40):
        inst = synth.random_small(s, m=int(3 + s % 9), n=int(3 + s % 7), box=6,
                                  int_frac=[1.0, 0.5, 0.0][s % 3], inf_frac=0.2 * (s % 2))
        check_against_oracle(lib, inst, loops=("persistent",) if s % 4 else LOOPS)


def test_cascade_round_counts(lib):
    for m, want in ((99, (oracle.CONVERGED, 100)), (100, (oracle.MAX_ROUNDS, 100))):
        inst = pins.cascade_instance(m)
        ref = check_against_oracle(lib, inst)
        assert (ref.status, ref.rounds) == want


def test_resume_and_idempotence(lib):
    inst = synth.config0(1)
    res, lb, ub = gpu_run(lib, inst, inst.lb, inst.ub, 100)
    assert res.status == oracle.CONVERGED
    k = res.rounds // 2
    r1, lb1, ub1 = gpu_run(lib, inst, inst.lb, inst.ub, k)
    r2, lb2, ub2 = gpu_run(lib, inst, lb1, ub1, 100)
    assert r1.status == oracle.MAX_ROUNDS and r1.rounds + r2.rounds == res.rounds
    assert same_bits(lb2, lb) and same_bits(ub2, ub)
    r3, lb3, ub3 = gpu_run(lib, inst, lb, ub, 100)
    assert (r3.status, r3.rounds) == (oracle.CONVERGED, 1)
    assert same_bits(lb3, lb) and same_bits(ub3, ub)


def test_config1_suite(lib):
    for k in (1, 50):
        inst = synth.config1(k)
        ref = check_against_oracle(lib, inst, loops=("persistent", "stream"))
        if k % 50 == 0:
            assert ref.status == oracle.INFEASIBLE
        else:
            assert ref.status == oracle.CONVERGED


def test_limit_point_matches_sequential(lib):
    """Bounded pure-integer systems have one limit point (Sec. 1.1): the
    GPU's synchronous rounds end at the bounds of the sequential Algorithm 1
    with marking (plain double sums in CSR order), in no fewer rounds than
    its sweeps; the large-instance version of this check is the rounds
    study of bench.py."""
    same = 0
    with_seq = 0
    for s in range(40):
        inst = synth.random_small(2_900 + s, m=int(4 + s % 6), n=int(4 + s % 5), box=6, slack=4.0)
        seq, _ = oracle.CpuSeq(inst).run(inst.lb, inst.ub, 200)
        with lib.Problem.from_instance(inst) as p:
            p.set_loop("graph_all" if s % 2 else "stream")
            res, lb, ub = p.run(inst.lb, inst.ub, 200)
        assert res.status == seq.status, s
        if seq.status == oracle.CONVERGED:
            assert same_bits(lb, seq.lb) and same_bits(ub, seq.ub), s
            assert seq.rounds <= res.rounds, s
            same += 1
        with_seq += 1
    assert same > 20, (same, with_seq)


def test_determinism_device_path(lib, torch_cuda):
    torch = torch_cuda
    inst = synth.config1(1)
    outs = []
    with lib.Problem.from_instance(inst) as p:
        for _ in range(3):
            d_lb = torch.tensor(inst.lb, dtype=torch.float64, device="cuda")
            d_ub = torch.tensor(inst.ub, dtype=torch.float64, device="cuda")
            res = p.run_device(d_lb, d_ub, 100)
            outs.append((res.status, res.rounds, d_lb.cpu().numpy(), d_ub.cpu().numpy()))
    for o in outs[1:]:
        assert o[:2] == outs[0][:2]
        assert same_bits(o[2], outs[0][2]) and same_bits(o[3], outs[0][3])


def test_edge_cases(lib):
    # no rows: one change-free round
    inst = synth.from_rows([], [], [], [0.0, -1.0], [1.0, 2.0], [1, 0], n=2)
    check_against_oracle(lib, inst)
    # only empty rows, compatible with 0, and one incompatible
    inst = synth.from_rows([[], []], [-1.0, -np.inf], [0.0, 3.0], [0.0], [5.0], [1], n=1)
    check_against_oracle(lib, inst)
    inst = synth.from_rows([[], []], [0.5, -np.inf], [1.0, 3.0], [0.0], [5.0], [1], n=1)
    check_against_oracle(lib, inst)
    # zero round limit, fractional integer bounds
    inst = synth.from_rows([[(0, 2.0)]], [-np.inf], [5.0], [0.3], [9.7], [1], n=1)
    check_against_oracle(lib, inst, max_rounds=0)
    check_against_oracle(lib, inst, max_rounds=1)
    # explicit zeros and a variable in no row
    inst = synth.from_rows([[(0, 0.0), (1, 3.0)], [(1, 1.0), (2, -2.0)]], [-np.inf, 0.0],
                           [4.0, np.inf], [-np.inf, 0.0, -5.0, 7.0], [np.inf, 10.0, 5.0, 9.0],
                           [0, 1, 0, 1], n=4)
    check_against_oracle(lib, inst)


def test_layout_steps(lib):
    """Every layout (4, 8 or 16 entries per lane; longer rows to segments)
    gives the oracle's results bitwise."""
    for inst in (synth.config0(), synth.layout_mix(0), synth.layout_mix(1), synth.config1(1)):
        ref = oracle.run(inst, inst.lb, inst.ub, 100)
        for steps in (4, 8, 16):
            with lib.Problem.from_instance(inst, steps=steps) as p:
                assert p.info()["steps"] == steps
                for loop in ("stream", "persistent"):
                    p.set_loop(loop)
                    say(f"  {inst.name} steps={steps} loop={loop}")
                    assert_same(f"{inst.name}/steps{steps}/{loop}", p.run(inst.lb, inst.ub, 100),
                                ref)


def test_autotune_records_layout(lib):
    inst = synth.config0(3)
    steps = lib.autotune(inst, inst.lb, inst.ub, 100)
    assert steps in (4, 8, 16)
    with lib.Problem.from_instance(inst) as p:  # steps = 0: the tuned value
        assert p.info()["steps"] == steps
        assert_same("tuned", p.run(inst.lb, inst.ub, 100), oracle.run(inst, inst.lb, inst.ub, 100))


def test_marked_rounds(lib):
    """Marked rounds give bitwise the results of unmarked ones (and of the
    oracle), with the stream and the host driver; the persistent driver
    ignores the switch."""
    cases = [synth.config0(), synth.config1(1), synth.layout_mix(0), synth.layout_mix(2),
             synth.config3_matrix(50_000, 25_000), pins.cascade_instance(99)]
    for inst in cases:
        ref = oracle.run(inst, inst.lb, inst.ub, 100)
        with lib.Problem.from_instance(inst) as p:
            p.set_marking(True)
            for loop in ("stream", "host", "graph", "graph_all", "persistent"):
                p.set_loop(loop)
                say(f"  marked {inst.name} loop={loop}")
                assert_same(f"marked {inst.name}/{loop}", p.run(inst.lb, inst.ub, 100), ref)
            # nodes of a search: marked rounds from fixed bounds, then again
            # after switching marking off and on
            for k in range(3 if inst.x0 is not None else 0):
                lb, ub = synth.node_bounds(inst, 31_000 + k, frac_hi=0.2, only_int=False)
                r1 = oracle.run(inst, lb, ub, 100)
                p.set_loop("stream")
                assert_same(f"marked node {inst.name}/{k}", p.run(lb, ub, 100), r1)
                p.set_marking(False)
                assert_same(f"unmarked node {inst.name}/{k}", p.run(lb, ub, 100), r1)
                p.set_marking(True)


def test_invalid_bounds_rejected(lib):
    inst = synth.config0()
    with lib.Problem.from_instance(inst) as p:
        for bad in (np.nan, np.inf):
            lb = inst.lb.copy()
            lb[5] = bad
            with pytest.raises(lib.PropError) as e:
                p.run(lb, inst.ub, 10)
            assert e.value.code == lib.EINVAL
        ub = inst.ub.copy()
        ub[3] = -np.inf
        with pytest.raises(lib.PropError):
            p.run(inst.lb, ub, 10)
        # the problem stays usable after a rejected call
        res, _, _ = p.run(inst.lb, inst.ub, 100)
        assert res.status == oracle.CONVERGED


# ---------------------------------------------------------------------------
# full-size config 2 (5M x 2M, ~52M nonzeros): every round against the
# oracle's, through the SHA-256 of the bounds after that round
# (tests/golden/config2_rounds.json, written by make_round_hashes.py from
# the oracle alone), plus properties of the final state
# ---------------------------------------------------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def bounds_sha(lb, ub):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(lb, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(ub, dtype="<f8").tobytes())
    return h.hexdigest()


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def big(lib):
    say("generating config2 (5,000,000 x 2,000,000)")
    inst = synth.cached("config2", synth.config2)
    say(f"config2: nnz={inst.nnz}; creating the device problem")
    p = lib.Problem.from_instance(inst)
    yield inst, p
    p.close()


def test_config2_every_round(lib, big):
    """Round r of the GPU run (max_rounds = r) leaves exactly the bounds of
    the oracle's round r, for every round of the run; the first differing
    round is named."""
    inst, p = big
    g = load_golden("config2_rounds.json")
    R = g["rounds"]
    assert R >= 2
    for r in range(1, R + 1):
        res, lb, ub = p.run(inst.lb, inst.ub, r)
        want = (g["status"], R) if r == R else (oracle.MAX_ROUNDS, r)
        assert (res.status, res.rounds) == want, f"round {r}: {res.status}/{res.rounds} vs {want}"
        assert bounds_sha(lb, ub) == g["sha"][r], f"bounds differ from the oracle's after round {r}"
    say(f"config2: {R} rounds, every one equal to the oracle's")
    # x0 stays inside the final bounds
    tol = 1e-6 * np.maximum(1.0, np.abs(inst.x0))
    assert np.all(lb - tol <= inst.x0) and np.all(inst.x0 <= ub + tol)
    # the full run (all drivers) ends in the same state
    for loop in LOOPS:
        p.set_loop(loop)
        res, lb, ub = p.run(inst.lb, inst.ub, 100)
        assert (res.status, res.rounds) == (g["status"], R), loop
        assert bounds_sha(lb, ub) == g["sha"][R], loop
    p.set_loop("stream")


def test_config2_marked_full_run(lib, big):
    """Marked rounds on the full instance: the oracle's final state."""
    inst, p = big
    g = load_golden("config2_rounds.json")
    p.set_marking(True)
    try:
        res1, lb1, ub1 = p.run(inst.lb, inst.ub, 100)
    finally:
        p.set_marking(False)
    assert (res1.status, res1.rounds) == (g["status"], g["rounds"])
    assert bounds_sha(lb1, ub1) == g["sha"][g["rounds"]]


def test_config2_store32(lib, big):
    """The single-precision bound store on the full instance: every round's
    bounds equal to the oracle's under the same store, and the full run on
    every driver."""
    inst, p = big
    g = load_golden("config2_store32.json")
    R = g["rounds"]
    p.set_store(32)
    try:
        p.set_loop("stream")
        for r in range(1, R + 1):
            res, lb, ub = p.run(inst.lb, inst.ub, r)
            want = (g["status"], R) if r == R else (oracle.MAX_ROUNDS, r)
            assert (res.status, res.rounds) == want, f"store32 round {r}"
            assert bounds_sha(lb, ub) == g["sha"][r], f"store32: bounds differ after round {r}"
        for loop in LOOPS:
            p.set_loop(loop)
            res, lb, ub = p.run(inst.lb, inst.ub, 100)
            assert (res.status, res.rounds) == (g["status"], R), loop
            assert bounds_sha(lb, ub) == g["sha"][R], f"store32/{loop}: bounds differ"
    finally:
        p.set_store(64)
        p.set_loop("stream")
    say(f"config2 store32: {R} rounds, every one equal to the oracle's")


def test_config2_nnz_split(lib, big):
    """The nnz-split layout on the full instance: every 4th round and the
    final state equal to the oracle's stored hashes."""
    inst, _ = big
    g = load_golden("config2_rounds.json")
    R = g["rounds"]
    with lib.Problem.from_instance(inst, layout=1) as p:
        for r in list(range(1, R, 4)) + [R]:
            res, lb, ub = p.run(inst.lb, inst.ub, r)
            want = (g["status"], R) if r == R else (oracle.MAX_ROUNDS, r)
            assert (res.status, res.rounds) == want, f"round {r}"
            assert bounds_sha(lb, ub) == g["sha"][r], f"nnz-split: bounds differ after round {r}"
    say(f"config2 nnz-split: rounds 1, 5, ..., {R} equal to the oracle's")


def test_round_limits_all_drivers(lib):
    """Round limits below, at and across the drivers' batch of 4 rounds, with
    and without marking: status and rounds exact, bounds bitwise."""
    inst = synth.config0()
    with lib.Problem.from_instance(inst) as p:
        for mr in (0, 1, 2, 3, 4, 5, 7, 9):
            ref = oracle.run(inst, inst.lb, inst.ub, mr)
            for marking in (False, True):
                p.set_marking(marking)
                for loop in LOOPS:
                    p.set_loop(loop)
                    assert_same(f"limit {mr} marking={marking} {loop}", p.run(inst.lb, inst.ub, mr),
                                ref)


def test_empty_and_degenerate_shapes(lib, torch_cuda):
    """No rows, no variables, a single 3,000-entry row (three long-row
    segments) and a variable in every row, through single runs, marked runs,
    batches and the device path."""
    torch = torch_cuda
    rng = np.random.default_rng(5)
    cases = [
        synth.from_rows([], [], [], [0.0, -1.0, 0.0], [1.0, 2.0, 4.0], [1, 0, 1], n=3),
        synth.from_rows([[(0, 1.0), (1, -1.0)]] * 3, [-1.0, 0.0, -np.inf], [1.0, 2.0, 0.5],
                        [-3.0, 0.0], [3.0, 1.0], [1, 0], n=2),
    ]
    n = 3000
    row = [(j, float(rng.integers(1, 4))) for j in range(n)]
    cases.append(synth.from_rows([row], [-np.inf], [10.0], np.zeros(n), np.full(n, 5.0),
                                 np.ones(n), n=n))
    cases.append(synth.from_rows([], [], [], [], [], [], n=0))
    # variable 0 in every row of a small system
    rows = [[(0, 1.0), (1 + i, 1.0)] for i in range(40)]
    cases.append(synth.from_rows(rows, [-np.inf] * 40, [3.0] * 40, np.zeros(41),
                                 np.full(41, 10.0), np.ones(41), n=41))
    for inst in cases:
        ref = oracle.run(inst, inst.lb, inst.ub, 100)
        with lib.Problem.from_instance(inst) as p:
            for marking in (False, True):
                p.set_marking(marking)
                for loop in ("stream", "graph", "graph_all", "host"):
                    p.set_loop(loop)
                    assert_same(f"{inst.name} {loop} marking={marking}",
                                p.run(inst.lb, inst.ub, 100), ref)
            if inst.n:
                lbs = np.stack([inst.lb] * 3)
                ubs = np.stack([inst.ub] * 3)
                d_lb = torch.tensor(lbs, dtype=torch.float64, device="cuda")
                d_ub = torch.tensor(ubs, dtype=torch.float64, device="cuda")
                res = p.run_batch_device(d_lb, d_ub, 100)
                for k in range(3):
                    assert (res[k].status, res[k].rounds) == (ref.status, ref.rounds)
                    if ref.status != oracle.INFEASIBLE:
                        assert same_bits(d_lb[k].cpu().numpy(), ref.lb)
                        assert same_bits(d_ub[k].cpu().numpy(), ref.ub)
