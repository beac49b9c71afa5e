"""Writes the round-by-round expectations of the full-size workloads.

For the 5,000,000 x 2,000,000 power-law instance and for 8 of the 256
branch-and-bound nodes of the 1,000,000 x 500,000 instance: the oracle's
final status and round count, and a SHA-256 of the bounds (lb then ub,
little-endian float64 in the caller's variable order) after every round.
Only the oracle and the input generators are called.  A round is the
oracle's synchronous round applied to the bounds the previous one left;
the oracle's own run with the same round limit gives the same state (the
resume property its pins check).

    python tests/golden/make_round_hashes.py config2   # ~6 s per round
    python tests/golden/make_round_hashes.py config3

With ``config2_store32`` it writes the same round-by-round trace of the
5,000,000 x 2,000,000 instance under the oracle's single-precision bound
store: each round is the oracle's run of one round from the bounds the
previous one left (those are integer-rounded and on the store's grid
already, so the run's entry normalisation leaves them unchanged).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

CONFIG3_NODES = (0, 5, 37, 64, 101, 150, 203, 255)


def bounds_sha(lb, ub) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(lb, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(ub, dtype="<f8").tobytes())
    return h.hexdigest()


def round_trace(inst, lb, ub, max_rounds=100, log=print):
    """Status, rounds and the bounds' hash after each round (round 0: the
    oracle's entry normalisation)."""
    start = oracle.run(inst, lb, ub, 0)  # validation and integer rounding only
    if start.status == oracle.INFEASIBLE:
        return {"status": start.status, "rounds": 0, "sha": [bounds_sha(start.lb, start.ub)]}
    L, U = start.lb, start.ub
    shas = [bounds_sha(L, U)]
    status, rounds = oracle.MAX_ROUNDS, max_rounds
    for r in range(1, max_rounds + 1):
        t0 = time.perf_counter()
        L, U, changed, infeasible, _ = oracle.round_(inst, L, U)
        shas.append(bounds_sha(L, U))
        log(f"  round {r}: changed={changed} infeasible={infeasible} "
            f"({time.perf_counter() - t0:.1f} s)")
        if infeasible:
            status, rounds = oracle.INFEASIBLE, r
            break
        if not changed:
            status, rounds = oracle.CONVERGED, r
            break
    return {"status": status, "rounds": rounds, "sha": shas}


def store32_trace(inst, lb, ub, max_rounds=100, log=print):
    """round_trace under the single-precision bound store."""
    start = oracle.run(inst, lb, ub, 0, store=32)
    if start.status == oracle.INFEASIBLE:
        return {"status": start.status, "rounds": 0, "sha": [bounds_sha(start.lb, start.ub)]}
    L, U = start.lb, start.ub
    shas = [bounds_sha(L, U)]
    status, rounds = oracle.MAX_ROUNDS, max_rounds
    for r in range(1, max_rounds + 1):
        t0 = time.perf_counter()
        one = oracle.run(inst, L, U, 1, store=32)
        changed = not (np.array_equal(one.lb, L) and np.array_equal(one.ub, U))
        L, U = one.lb, one.ub
        shas.append(bounds_sha(L, U))
        log(f"  round {r}: status={one.status} ({time.perf_counter() - t0:.1f} s)")
        if one.status == oracle.INFEASIBLE:
            status, rounds = oracle.INFEASIBLE, r
            break
        if one.status == oracle.CONVERGED:
            assert not changed
            status, rounds = oracle.CONVERGED, r
            break
    return {"status": status, "rounds": rounds, "sha": shas}


def main(which: str):
    if which == "config2":
        inst = synth.config2()
        out = {"workload": f"{inst.name}: {inst.m} x {inst.n}, {inst.nnz} nnz, root bounds",
               "max_rounds": 100, **round_trace(inst, inst.lb, inst.ub)}
        path = os.path.join(HERE, "config2_rounds.json")
    elif which == "config2_store32":
        inst = synth.config2()
        out = {"workload": f"{inst.name}: {inst.m} x {inst.n}, {inst.nnz} nnz, root bounds, "
                           "single-precision bound store",
               "max_rounds": 100, "store": 32, **store32_trace(inst, inst.lb, inst.ub)}
        path = os.path.join(HERE, "config2_store32.json")
    elif which == "config3":
        inst = synth.config3_matrix()
        lbs, ubs = synth.config3_nodes(inst, 256)
        nodes = {}
        for k in CONFIG3_NODES:
            print(f"node {k}", flush=True)
            nodes[str(k)] = round_trace(inst, lbs[k], ubs[k])
        out = {"workload": f"{inst.name}: {inst.m} x {inst.n}, {inst.nnz} nnz, nodes of "
                           "synth.config3_nodes(inst, 256)",
               "max_rounds": 100, "nodes": nodes}
        path = os.path.join(HERE, "config3_nodes.json")
    else:
        raise SystemExit(f"unknown workload {which}")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print(f"wrote {path}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "config2")
