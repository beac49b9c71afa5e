"""Benchmark: synchronous domain propagation on the large single-instance
workload (5,000,000 rows x 2,000,000 variables, ~52M nonzeros, power-law
row lengths and column degrees).

A step is one full propagation run -- every round until no bound changes --
from the root bounds, with the matrix and the bounds already in HBM.  The
printed JSON line carries:
  value      nonzeros processed per second, summed over rounds
             (nnz * rounds * steps / timed seconds);
  roofline   algorithmic bytes of the round-loop launch (rounds x
             (12 nnz + 20 m + 33 n + 4)) over its average duration, measured
             with HIP events on the launch stream, against 8 TB/s HBM;
  cpu_baseline  the CPU oracle (single thread) on a bounded sample: one
             synchronous round over the full instance.
Progress goes to stderr; stdout gets the one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "nnz processed/s per round & HBM GB/s; batched B&B nodes/s vs one-at-a-time"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(inst, skip: bool, min_seconds: float = 10.0, max_rounds: int = 4):
    """Synchronous oracle rounds over the whole instance from the root
    bounds, single thread, until at least `min_seconds` have passed (at most
    `max_rounds` rounds, fewer if the run ends sooner)."""
    if skip:
        return None
    import numpy as np

    import oracle

    lb = np.where(inst.vartype == 1, np.ceil(inst.lb - 1e-6), inst.lb) + 0.0
    ub = np.where(inst.vartype == 1, np.floor(inst.ub + 1e-6), inst.ub) + 0.0
    try:
        os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})
    except (AttributeError, OSError):
        pass
    log(f"oracle: synchronous rounds over the full instance (single thread, >= {min_seconds} s)")
    t0 = time.perf_counter()
    rounds = flags = 0
    while rounds < max_rounds:
        lb, ub, changed, infeasible, f = oracle.round_(inst, lb, ub)
        rounds += 1
        flags += f
        if not changed or infeasible or time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    return {
        "value": rounds * inst.nnz / dt,
        "unit": "nnz/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the first {rounds} synchronous rounds of the full {inst.m}x{inst.n} instance "
                  f"({inst.nnz} nnz) from the root bounds: {dt:.2f} s",
        "host_cpu": host_cpu_model(),
        "host_nproc": os.cpu_count(),
        "near_integer_candidates": int(flags),
    }


def cpu_seq_compare(skip: bool, max_rounds: int, suite: int = 10):
    """The paper's comparison: sequential propagation with constraint
    marking (Algorithm 1) on one host core against full GPU runs of the
    synchronous rounds, on the 200,000 x 100,000 lognormal instance.  Two
    sequential codes are timed: the paper's kind (plain double sums in CSR
    order, cpu_seq.c) and the oracle's Algorithm 1 (exactly rounded sums,
    several times slower).  Over the first `suite` seeds of that family the
    synchronous round counts are set against the sequential sweep counts
    (the paper's rounds study: 4.4 synchronous rounds vs 3.1 sequential
    on average)."""
    if skip:
        return None
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2009_07785_amd import Problem

    inst = synth.cached("config1_1", synth.config1, 1)
    log("cpu_seq: sequential Algorithm 1 on the 200,000 x 100,000 instance")
    seq = oracle.CpuSeq(inst)
    t_plain = []
    for _ in range(3):
        res_plain, dt = seq.run(inst.lb, inst.ub)
        t_plain.append(dt)
    seq.close()
    t0 = time.perf_counter()
    res_exact = oracle.run_seq(inst, inst.lb, inst.ub)
    t_exact = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    from paper_2009_07785_amd import autotune

    steps = autotune(inst, inst.lb, inst.ub, max_rounds)  # layout for this shape
    prob = Problem.from_instance(inst)
    root_lb = torch.tensor(inst.lb, dtype=torch.float64, device=dev)
    root_ub = torch.tensor(inst.ub, dtype=torch.float64, device=dev)
    d_lb, d_ub = torch.empty_like(root_lb), torch.empty_like(root_ub)
    ts = []
    for i in range(6):
        d_lb.copy_(root_lb)
        d_ub.copy_(root_ub)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = prob.run_device(d_lb, d_ub, max_rounds)
        torch.cuda.synchronize()
        if i:
            ts.append(time.perf_counter() - t0)
    prob.close()
    t_gpu = float(np.median(ts))
    # rounds study over a suite of seeds (feasible ones; every 50th seed of
    # the family is made infeasible)
    sync_rounds, seq_sweeps = [], []
    for k in range(1, suite + 1):
        ik = synth.cached(f"config1_{k}", synth.config1, k)
        with Problem.from_instance(ik) as pk:
            rk = pk.run(ik.lb, ik.ub, max_rounds)[0]
        cs = oracle.CpuSeq(ik)
        rs, _ = cs.run(ik.lb, ik.ub)
        cs.close()
        if rk.status == 0 and rs.status == 0:
            sync_rounds.append(rk.rounds)
            seq_sweeps.append(rs.rounds)
    out = {"workload": f"config1: {inst.m}x{inst.n}, {inst.nnz} nnz, from the root bounds",
           "cores": 1, "gpu_run_ms": t_gpu * 1e3, "gpu_rounds": r.rounds, "layout_steps": steps,
           "cpu_seq": {"kind": "Algorithm 1 with marking, plain double sums (the paper's kind)",
                       "seconds": float(np.median(t_plain)), "sweeps": res_plain.rounds,
                       "speedup_gpu_vs_cpu_seq": float(np.median(t_plain)) / t_gpu},
           "oracle_seq": {"kind": "the oracle's Algorithm 1, exactly rounded sums",
                          "seconds": t_exact, "sweeps": res_exact.rounds,
                          "speedup_gpu_vs_oracle_seq": t_exact / t_gpu},
           "rounds_study": {"seeds": f"config1 seeds 1..{suite}, converged on both",
                            "instances": len(sync_rounds),
                            "synchronous_rounds_mean": float(np.mean(sync_rounds)),
                            "sequential_sweeps_mean": float(np.mean(seq_sweeps)),
                            "ratio": float(np.mean(sync_rounds)) / float(np.mean(seq_sweeps))}}
    log(f"cpu_seq: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--max-rounds", type=int, default=100)
    ap.add_argument("--loop", default="stream",
                    choices=["persistent", "stream", "host", "graph", "graph_all"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-seq", action="store_true",
                    help="skip the sequential-propagation comparison on the medium instance")
    ap.add_argument("--no-loop-compare", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 2,000 x 1,000 and 200,000 x 100,000 single-instance lines")
    ap.add_argument("--no-layouts", action="store_true",
                    help="skip the nnz-split layout comparison")
    ap.add_argument("--store", type=int, default=64, choices=[64, 32],
                    help="bound store of the timed runs: 64 (doubles) or 32 (single "
                         "precision, rounded outward; FP64 arithmetic either way)")
    ap.add_argument("--no-store32", action="store_true",
                    help="skip the single-precision bound store comparison")
    ap.add_argument("--no-children", action="store_true",
                    help="skip the branch-and-bound children leg (marked rounds from a parent)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched branch-and-bound node comparison")
    ap.add_argument("--batch-nodes", type=int, default=256)
    ap.add_argument("--no-marked", action="store_true",
                    help="skip the marked-rounds leg (rows without changed variables skipped)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg (open-loop requests over 64 resident instances)")
    ap.add_argument("--serving-scale", type=float, default=1.0,
                    help="row-count scale of the 64 serving instances (1.0 = ~386M nnz)")
    ap.add_argument("--serving-seconds", type=float, default=60.0)
    ap.add_argument("--serving-rate-below", type=float, default=400.0,
                    help="a second, shorter phase at a rate the server sustains (0: none)")
    ap.add_argument("--serving-seconds-below", type=float, default=20.0)
    ap.add_argument("--serving-rounds-per-step", type=int, default=0,
                    help="rounds the server queues between status reads (0: its default, 1)")
    ap.add_argument("--serving-marking", type=int, default=1, choices=[0, 1],
                    help="marked rounds per group of serving slots (results unchanged)")
    ap.add_argument("--serving-max-slots", type=int, default=256,
                    help="slots per instance (requests of one instance running at once)")
    ap.add_argument("--serving-max-pending", type=int, default=1024,
                    help="requests held before submissions are refused (admission control)")
    ap.add_argument("--serving-rate", type=float, default=2000.0, help="requests per second")
    ap.add_argument("--serving-budget-gib", type=float, default=64.0)
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_config2.json"),
                    help="HBM traffic per launch measured with rocprofv3 counters (JSON)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (the reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        # a plain elementwise kernel that reads and writes exactly BYTES each
        # (dst = src + 1): what FETCH_SIZE / WRITE_SIZE report for it gives
        # the counters' scale
        import torch

        n = args.copy_calibration // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"kernel": "elementwise add", "bytes_read": n * 8, "bytes_written": n * 8,
                          "launches": 5}))
        return

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path; "
              "the value is one GPU's throughput", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2009_07785_amd import Problem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log("generating the 5,000,000 x 2,000,000 power-law instance")
    t0 = time.perf_counter()
    inst = synth.cached("config2", synth.config2)
    log(f"generated: nnz={inst.nnz} in {time.perf_counter() - t0:.1f} s; building device problem")
    t0 = time.perf_counter()
    prob = Problem.from_instance(inst)
    info = prob.info()
    log(f"device problem ready in {time.perf_counter() - t0:.1f} s: {info}")
    prob.set_loop(args.loop)
    prob.set_kernel_timing(args.loop != "persistent")
    prob.set_store(args.store)

    root_lb = torch.tensor(inst.lb, dtype=torch.float64, device=dev)
    root_ub = torch.tensor(inst.ub, dtype=torch.float64, device=dev)
    d_lb = torch.empty_like(root_lb)
    d_ub = torch.empty_like(root_ub)
    stream = torch.cuda.current_stream(dev)

    def step():
        d_lb.copy_(root_lb)
        d_ub.copy_(root_ub)
        return prob.run_device(d_lb, d_ub, args.max_rounds, stream)

    for i in range(args.warmup):
        r = step()
        log(f"warmup {i + 1}/{args.warmup}: {r.status_name} after {r.rounds} rounds, "
            f"loop {prob.last_timing()[0]:.3f} ms")

    loop_ms, total_ms, kern_ms, kern_n, rounds = [], [], [], [], set()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step()
        lm, tm = prob.last_timing()
        km, kn = prob.last_kernel_timing()
        loop_ms.append(lm)
        total_ms.append(tm)
        kern_ms.append(km)
        kern_n.append(kn)
        rounds.add((r.status, r.rounds))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f} s; status/rounds {sorted(rounds)}")
    assert len(rounds) == 1, "runs disagree"
    status, nrounds = rounds.pop()

    nnz = info["nnz"]
    alg_round = info["alg_bytes_round"]
    value = nnz * nrounds * args.steps / elapsed
    loop_avg_ms = float(np.mean(loop_ms))
    loop_GBps = alg_round * nrounds / (loop_avg_ms * 1e-3) / 1e9
    # dominant kernel: the per-round matrix kernel; per launch it reads the
    # matrix (12 B per nonzero), the row sides and row pointers (20 B per
    # row) and every variable's bounds and type once (17 B per variable);
    # the commit kernel accounts for the remaining 16 B per variable
    m_, n_ = info["m"], info["n"]
    kern_bytes = 12 * nnz + 20 * m_ + 17 * n_
    if sum(kern_n):
        kern_avg_ms = float(np.sum(kern_ms) / np.sum(kern_n))
        achieved = kern_bytes / (kern_avg_ms * 1e-3) / 1e9
        kern_name = "k_round (per-round matrix kernel: activities, candidates, atomics)"
    else:
        kern_avg_ms = loop_avg_ms
        achieved = loop_GBps
        kern_name = "k_persistent (all rounds of one run in one cooperative launch)"

    traffic = None
    if os.path.exists(args.traffic):
        with open(args.traffic) as f:
            tr = json.load(f)
        if (tr.get("kernel_source_sha") == kernel_source_sha()
                and tr.get("bound_store", 64) == args.store):
            traffic = tr.get("bytes_per_launch")

    loops = {}
    if not args.no_loop_compare:
        for mode in ("persistent", "stream", "host", "graph", "graph_all"):
            prob.set_loop(mode)
            ts = []
            for _ in range(3):
                rr = step()
                ts.append(prob.last_timing()[0])
            loops[mode] = {"loop_ms": float(np.median(ts)), "rounds": rr.rounds}
        prob.set_loop(args.loop)
        log(f"round-loop drivers: {loops}")

    # marked rounds (rows whose variables did not change are skipped; same
    # results): an extension of the paper's method, reported beside it
    marked = None
    if not args.no_marked:
        prob.set_loop("stream")
        ref_lb, ref_ub = d_lb.clone(), d_ub.clone()
        step()
        ref_lb.copy_(d_lb)
        ref_ub.copy_(d_ub)
        prob.set_marking(True)
        ts, same = [], True
        for _ in range(max(3, min(args.steps, 10))):
            rr = step()
            ts.append(prob.last_timing()[0])
            same &= (rr.status, rr.rounds) == (status, nrounds)
            same &= bool(torch.equal(d_lb, ref_lb) and torch.equal(d_ub, ref_ub))
        prob.set_marking(False)
        prob.set_loop(args.loop)
        mm = float(np.median(ts))
        marked = {"loop_ms": mm, "speedup_vs_unmarked": loop_avg_ms / mm,
                  "effective_nnz_per_s": nnz * nrounds / (mm * 1e-3),
                  "identical_results": same}
        log(f"marked rounds: {marked}")

    small = None if args.no_small else small_configs(args.max_rounds)
    layouts = None if args.no_layouts else layout_compare(args.max_rounds, inst)
    store32 = None if args.no_store32 else store_compare(prob, inst, args.max_rounds)
    prob.set_store(args.store)
    prob.set_loop(args.loop)
    prob.set_kernel_timing(args.loop != "persistent")

    batch = None if args.no_batch else batched_nodes(args.batch_nodes, args.max_rounds)
    children = None if args.no_children else children_nodes(args.batch_nodes, args.max_rounds)

    serve = None
    if not args.no_serving:
        serve = serving(args.serving_scale, args.serving_seconds, args.serving_rate,
                        int(args.serving_budget_gib * (1 << 30)), args.serving_max_pending,
                        args.serving_rate_below, args.serving_seconds_below,
                        args.serving_max_slots, marking=bool(args.serving_marking),
                        rounds_per_step=args.serving_rounds_per_step)

    # the CPU baseline leg: the oracle's synchronous rounds on config2 and,
    # as the paper's own comparison, its sequential Algorithm 1 on config1
    base = cpu_baseline(inst, args.no_cpu_baseline)
    if base is not None:
        base["sequential_algorithm1"] = cpu_seq_compare(args.no_cpu_seq, args.max_rounds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "config2: single instance, 5,000,000 x 2,000,000, power-law rows "
                        "(pdf exponent 2.2, cap 200,000) and column degrees",
            "m": inst.m, "n": inst.n, "nnz": nnz, "max_rounds": args.max_rounds,
            "loop": args.loop, "parallelism": "single GPU", "layout_steps": info["steps"],
            "bound_store": args.store,
        },
        "status": ["CONVERGED", "INFEASIBLE", "MAX_ROUNDS"][status],
        "rounds": nrounds,
        "loop_ms": loop_avg_ms,
        "pack_run_unpack_ms": float(np.mean(total_ms)),
        "alg_bytes_per_round": alg_round,
        "loop_alg_GBps": loop_GBps,
        "loop_frac": loop_GBps / HBM_PEAK_GBS,
        "roofline": {
            "bound": "hbm",
            "kernel": kern_name,
            "kernel_avg_ms": kern_avg_ms,
            "alg_bytes_per_launch": kern_bytes if sum(kern_n) else alg_round * nrounds,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
        },
        "round_loops": loops,
        "marked": marked,
        "small_configs": small,
        "layouts": layouts,
        "store32": store32,
        "batched": batch,
        "children": children,
        "serving": serve,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    prob.close()


def small_configs(max_rounds: int, reps: int = 20):
    """The two smaller single-instance workloads: 2,000 x 1,000 (latency:
    microseconds per round and per run) and 200,000 x 100,000 (nonzeros per
    second and fraction of the HBM roofline), full runs from the root bounds
    with the bounds resident on the device, median of `reps` runs per
    round-loop driver; the figures are the fastest driver's."""
    import numpy as np
    import torch

    import synth
    from paper_2009_07785_amd import Problem

    dev = torch.device("cuda:0")
    out = {}
    for key, fn, args in (("config0", synth.config0, ()), ("config1", synth.config1, (1,))):
        inst = synth.cached(key + "_bench", fn, *args)
        prob = Problem.from_instance(inst)
        info = prob.info()
        root_lb = torch.tensor(inst.lb, dtype=torch.float64, device=dev)
        root_ub = torch.tensor(inst.ub, dtype=torch.float64, device=dev)
        d_lb, d_ub = torch.empty_like(root_lb), torch.empty_like(root_ub)
        per_loop = {}
        for loop in ("stream", "graph", "graph_all", "host", "persistent"):
            prob.set_loop(loop)
            loop_ms = []
            for i in range(reps + 2):
                d_lb.copy_(root_lb)
                d_ub.copy_(root_ub)
                r = prob.run_device(d_lb, d_ub, max_rounds)
                if i >= 2:
                    loop_ms.append(prob.last_timing()[0])
            per_loop[loop] = float(np.median(loop_ms))
        prob.close()
        best = min(per_loop, key=per_loop.get)
        ms = per_loop[best]
        gbps = info["alg_bytes_round"] * r.rounds / (ms * 1e-3) / 1e9
        out[key] = {"workload": f"{inst.name}: {inst.m}x{inst.n}, {info['nnz']} nnz, root bounds",
                    "rounds": r.rounds, "loop": best, "layout_steps": info["steps"],
                    "run_us": ms * 1e3, "us_per_round": ms * 1e3 / r.rounds,
                    "nnz_per_s": info["nnz"] * r.rounds / (ms * 1e-3),
                    "alg_GBps": gbps, "frac": gbps / HBM_PEAK_GBS,
                    "run_us_per_loop": {k: v * 1e3 for k, v in per_loop.items()}}
    log(f"small configs: {out}")
    return out


def layout_compare(max_rounds: int, inst2, reps: int = 6):
    """The nnz-split layout (merge-path style: rows in input order packed
    into 512-entry waves, 8 consecutive entries per lane, rows spanning
    lanes joined by a segmented scan) against the default length-class
    chunks, on the 5,000,000 x 2,000,000 and 200,000 x 100,000 instances:
    round-kernel time per launch and full-run time, identical results
    required."""
    import numpy as np
    import torch

    import synth
    from paper_2009_07785_amd import Problem

    dev = torch.device("cuda:0")
    out = {}
    for key in ("config2", "config1"):
        inst = inst2 if key == "config2" else synth.cached("config1_bench", synth.config1, 1)
        res = {}
        for name, kw in (("chunks", {}), ("nnz_split", {"layout": 1})):
            p = Problem.from_instance(inst, **kw)
            p.set_loop("stream")
            p.set_kernel_timing(True)
            rl = torch.tensor(inst.lb, dtype=torch.float64, device=dev)
            ru = torch.tensor(inst.ub, dtype=torch.float64, device=dev)
            dl, du = torch.empty_like(rl), torch.empty_like(ru)
            lm, km, kn = [], [], []
            for i in range(reps + 1):
                dl.copy_(rl)
                du.copy_(ru)
                r = p.run_device(dl, du, max_rounds)
                if i:
                    lm.append(p.last_timing()[0])
                    a, b = p.last_kernel_timing()
                    km.append(a)
                    kn.append(b)
            res[name] = {"loop_ms": float(np.median(lm)),
                         "round_kernel_us": 1e3 * float(np.sum(km)) / max(1, int(np.sum(kn))),
                         "stored_entries": p.info()["nnz_stored"],
                         "result": (r.status, r.rounds, dl.cpu().numpy().tobytes(),
                                    du.cpu().numpy().tobytes())}
            p.close()
        same = res["chunks"].pop("result") == res["nnz_split"].pop("result")
        out[key] = {**res, "identical_results": same,
                    "nnz_split_over_chunks": res["nnz_split"]["loop_ms"] / res["chunks"]["loop_ms"]}
    log(f"layouts: {out}")
    return out


def store_compare(prob2, inst2, max_rounds: int, reps: int = 6):
    """The single-precision bound store (FP64 arithmetic, bounds kept as
    singles rounded outward) against the FP64 store, on the 5,000,000 x
    2,000,000 and 200,000 x 100,000 instances: round-kernel time per launch,
    run time, rounds, and how far the final bounds moved (outward rounding
    only loosens, so the single-precision results are never tighter where
    the runs otherwise agree)."""
    import numpy as np
    import torch

    import synth
    from paper_2009_07785_amd import Problem

    dev = torch.device("cuda:0")
    out = {}
    for key in ("config2", "config1"):
        if key == "config2":
            inst, p = inst2, prob2
        else:
            inst = synth.cached("config1_bench", synth.config1, 1)
            p = Problem.from_instance(inst)
        p.set_loop("stream")
        p.set_kernel_timing(True)
        rl = torch.tensor(inst.lb, dtype=torch.float64, device=dev)
        ru = torch.tensor(inst.ub, dtype=torch.float64, device=dev)
        dl, du = torch.empty_like(rl), torch.empty_like(ru)
        res, final = {}, {}
        for bits in (64, 32):
            p.set_store(bits)
            lm, km, kn, seen = [], [], [], set()
            for i in range(reps + 1):
                dl.copy_(rl)
                du.copy_(ru)
                r = p.run_device(dl, du, max_rounds)
                seen.add((r.status, r.rounds, hash(dl.cpu().numpy().tobytes()),
                          hash(du.cpu().numpy().tobytes())))
                if i:
                    lm.append(p.last_timing()[0])
                    a, b = p.last_kernel_timing()
                    km.append(a)
                    kn.append(b)
            res[f"f{bits}"] = {"loop_ms": float(np.median(lm)),
                               "round_kernel_us": 1e3 * float(np.sum(km)) / max(1, int(np.sum(kn))),
                               "status": ["CONVERGED", "INFEASIBLE", "MAX_ROUNDS"][r.status],
                               "rounds": r.rounds, "repeatable": len(seen) == 1}
            final[bits] = (dl.cpu().numpy(), du.cpu().numpy())
        p.set_store(64)
        if key != "config2":
            p.close()
        (l64, u64), (l32, u32) = final[64], final[32]
        is_int = inst.vartype != 0
        dlb, dub = l32 != l64, u32 != u64
        fin = np.isfinite(l64) & np.isfinite(u64) & np.isfinite(l32) & np.isfinite(u32)
        w64 = np.where(fin, u64 - l64, 0.0)
        w32 = np.where(fin, u32 - l32, 0.0)
        rel = np.where(fin & (w64 > 0), (w32 - w64) / np.maximum(w64, 1e-300), 0.0)
        out[key] = {**res,
                    "bounds_differing": int(dlb.sum() + dub.sum()),
                    "integer_bounds_differing": int((dlb & is_int).sum() + (dub & is_int).sum()),
                    "looser_or_equal": bool(np.all(l32 <= l64) and np.all(u32 >= u64)),
                    "bounds_tighter_than_f64": int((l32 > l64).sum() + (u32 < u64).sum()),
                    "max_rel_width_increase": float(rel.max()) if rel.size else 0.0,
                    "f32_over_f64_round_kernel": res["f32"]["round_kernel_us"]
                    / res["f64"]["round_kernel_us"]}
    log(f"store32: {out}")
    return out


def batched_nodes(count: int, max_rounds: int):
    """Branch-and-bound nodes on the 1,000,000 x 500,000 power-law matrix:
    `count` bound vectors (1-5% of the integer variables fixed each),
    propagated in one batched run and as `count` separate runs, with the
    results required to be identical."""
    import numpy as np
    import torch

    import synth
    from paper_2009_07785_amd import Problem

    dev = torch.device("cuda:0")
    log("generating the 1,000,000 x 500,000 matrix and the node bounds")
    inst = synth.cached("config3", synth.config3_matrix)
    lbs, ubs = synth.config3_nodes(inst, count)
    prob = Problem.from_instance(inst)
    D_lb = torch.tensor(lbs, dtype=torch.float64, device=dev)
    D_ub = torch.tensor(ubs, dtype=torch.float64, device=dev)
    s_lb = torch.empty(inst.n, dtype=torch.float64, device=dev)
    s_ub = torch.empty_like(s_lb)
    out_lb = torch.empty_like(D_lb)
    out_ub = torch.empty_like(D_ub)
    stream = torch.cuda.current_stream(dev)

    def one_at_a_time():
        res = []
        for k in range(count):
            s_lb.copy_(D_lb[k])
            s_ub.copy_(D_ub[k])
            res.append(prob.run_device(s_lb, s_ub, max_rounds, stream))
            out_lb[k].copy_(s_lb)
            out_ub[k].copy_(s_ub)
        return res

    def batched():
        b_lb = D_lb.clone()
        b_ub = D_ub.clone()
        return prob.run_batch_device(b_lb, b_ub, max_rounds, stream), b_lb, b_ub

    one_at_a_time()
    batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = one_at_a_time()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    bat, b_lb, b_ub = batched()
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    same_status = all((a.status, a.rounds) == (b.status, b.rounds) for a, b in zip(seq, bat))
    feas = torch.tensor([r.status != 1 for r in seq], device=dev)
    same_bounds = bool(torch.all(torch.where(feas[:, None], (b_lb == out_lb) & (b_ub == out_ub),
                                             True)).item())
    # the same with marked rounds (rows whose variables did not change in
    # the previous round are skipped; per group of 8 nodes in the batch)
    prob.set_marking(True)
    one_at_a_time()
    batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_m = one_at_a_time()
    torch.cuda.synchronize()
    t_seq_m = time.perf_counter() - t0
    same_m = all((a.status, a.rounds) == (b.status, b.rounds) for a, b in zip(seq, seq_m))
    same_m &= bool(torch.all(torch.where(feas[:, None], (b_lb == out_lb) & (b_ub == out_ub),
                                         True)).item())
    t0 = time.perf_counter()
    bat_m, m_lb, m_ub = batched()
    torch.cuda.synchronize()
    t_bat_m = time.perf_counter() - t0
    prob.set_marking(False)
    same_m &= all((a.status, a.rounds) == (b.status, b.rounds) for a, b in zip(seq, bat_m))
    same_m &= bool(torch.all(torch.where(feas[:, None], (m_lb == b_lb) & (m_ub == b_ub),
                                         True)).item())
    statuses = {}
    for r in seq:
        statuses[r.status_name] = statuses.get(r.status_name, 0) + 1
    rounds = [r.rounds for r in seq]
    out = {
        "workload": f"config3: {inst.m}x{inst.n} power-law matrix ({inst.nnz} nnz), {count} "
                    "nodes fixing 1-5% of the integer variables",
        "nodes": count,
        "batched_nodes_per_s": count / t_bat,
        "one_at_a_time_nodes_per_s": count / t_seq,
        "speedup": t_seq / t_bat,
        "batched_ms": t_bat * 1e3,
        "one_at_a_time_ms": t_seq * 1e3,
        "rounds_max": max(rounds),
        "rounds_mean": float(np.mean(rounds)),
        "statuses": statuses,
        "identical_results": bool(same_status and same_bounds),
        "marked": {"batched_ms": t_bat_m * 1e3, "one_at_a_time_ms": t_seq_m * 1e3,
                   "speedup": t_seq_m / t_bat_m, "batched_vs_plain_one_at_a_time": t_seq / t_bat_m,
                   "identical_results": bool(same_m)},
    }
    log(f"batched nodes: {out}")
    prob.close()
    return out


def children_nodes(count: int, max_rounds: int):
    """Branch-and-bound children on the 1,000,000 x 500,000 power-law
    matrix: the root's fixed point is the parent, and children 2i, 2i + 1
    split the domain of one unfixed integer variable at its middle.  The
    children run one at a time and batched, each without and with marked
    rounds seeded from the parent (round 1 then processes only the rows of
    the branched variable); all four give identical results."""
    import numpy as np
    import torch

    import synth
    from paper_2009_07785_amd import Problem

    dev = torch.device("cuda:0")
    inst = synth.cached("config3", synth.config3_matrix)
    prob = Problem.from_instance(inst)
    d_plb = torch.tensor(inst.lb, dtype=torch.float64, device=dev)
    d_pub = torch.tensor(inst.ub, dtype=torch.float64, device=dev)
    root = prob.run_device(d_plb, d_pub, 1000)
    log(f"children: root {root.status_name} after {root.rounds} rounds")
    if root.status != 0:
        prob.close()
        return {"skipped": f"the root did not converge ({root.status_name})"}
    plb, pub = d_plb.cpu().numpy(), d_pub.cpu().numpy()
    lbs, ubs = synth.branch_children(plb, pub, inst.vartype, count, 4100)
    D_lb = torch.tensor(lbs, dtype=torch.float64, device=dev)
    D_ub = torch.tensor(ubs, dtype=torch.float64, device=dev)
    s_lb = torch.empty(inst.n, dtype=torch.float64, device=dev)
    s_ub = torch.empty_like(s_lb)
    stream = torch.cuda.current_stream(dev)

    def one_at_a_time():
        out_lb, out_ub, res = torch.empty_like(D_lb), torch.empty_like(D_ub), []
        for k in range(count):
            s_lb.copy_(D_lb[k])
            s_ub.copy_(D_ub[k])
            res.append(prob.run_device(s_lb, s_ub, max_rounds, stream))
            out_lb[k].copy_(s_lb)
            out_ub[k].copy_(s_ub)
        return res, out_lb, out_ub

    def batched():
        b_lb, b_ub = D_lb.clone(), D_ub.clone()
        return prob.run_batch_device(b_lb, b_ub, max_rounds, stream), b_lb, b_ub

    out, ref = {}, None
    for key, fn, marked in (("one_at_a_time", one_at_a_time, False),
                            ("one_at_a_time_marked", one_at_a_time, True),
                            ("batched", batched, False), ("batched_marked", batched, True)):
        prob.set_marking(marked)
        prob.set_parent(d_plb, d_pub) if marked else prob.set_parent(None, None)
        fn()  # warm-up (workspace, marking data)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, lb, ub = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        got = ([(r.status, r.rounds) for r in res], lb, ub)
        if ref is None:
            ref = got
            same = True
        else:
            feas = torch.tensor([st != 1 for st, _ in ref[0]], device=dev)
            same = got[0] == ref[0] and bool(torch.all(torch.where(
                feas[:, None], (got[1] == ref[1]) & (got[2] == ref[2]), True)).item())
        out[key] = {"ms": dt * 1e3, "nodes_per_s": count / dt, "identical_to_first": same}
    prob.set_marking(False)
    prob.set_parent(None, None)
    prob.close()
    rounds = [r for _, r in ref[0]]
    out.update({"workload": f"config3 matrix {inst.m}x{inst.n} ({inst.nnz} nnz): {count} "
                            "children of the root's fixed point, each pair splitting one "
                            "integer variable's domain",
                "root_rounds": root.rounds, "children_rounds_mean": float(np.mean(rounds)),
                "children_rounds_max": int(max(rounds))})
    log(f"children: {out}")
    return out


def serving(scale: float, seconds: float, rate: float, budget: int, max_pending: int,
            rate_below: float = 0.0, seconds_below: float = 0.0, max_slots: int = 256,
            variants: int = 8, max_rounds: int = 50, verify: int = 1000, marking: bool = False,
            rounds_per_step: int = 0):
    """Open-loop serving: Poisson arrivals at `rate` per second for `seconds`,
    each request a bound vector (0-5% of all variables fixed to a feasible
    point's values) on one of 64 resident instances drawn uniformly.  A
    request that finds `max_pending` requests held is refused at submission
    (admission control: the server sheds load instead of queueing without
    bound).  A consumer thread collects results as they finish; at least
    `verify` of them, spread over the run, are compared bitwise with the
    same request run alone.  Latency is the server's (submission to result
    ready)."""
    import queue
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import synth
    from paper_2009_07785_amd import Problem, binding

    log(f"generating the 64 serving instances (scale {scale})")
    t0 = time.perf_counter()
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else os.cpu_count() or 1))
    pool = synth.config4_pool(scale=scale, workers=workers)
    total_nnz = int(sum(i.nnz for i in pool))
    log(f"generated {total_nnz} nnz in {time.perf_counter() - t0:.1f} s; creating problems")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:  # prop_create releases the GIL in ctypes
        probs = list(ex.map(Problem.from_instance, pool))
    log(f"serving pool ready in {time.perf_counter() - t0:.1f} s")
    # `variants` distinct requests per instance; arrivals pick one by seed
    bounds = [[synth.request_bounds(inst, 1000 * k + v) for v in range(variants)]
              for k, inst in enumerate(pool)]
    alone = [[probs[k].run(lb, ub, max_rounds) for lb, ub in bounds[k]]
             for k in range(len(pool))]
    srv = binding.Server(budget, max_slots=max_slots, max_pending=max_pending, marking=marking,
                         rounds_per_step=rounds_per_step)
    for p in probs:
        srv.add_instance(p)
    # warm the server: one request per instance
    for k in range(len(pool)):
        lb, ub = bounds[k][0]
        t = srv.submit(k, lb, ub, max_rounds)
        srv.wait(t, pool[k].n, timeout_ms=120_000, bounds=False)

    def phase(rate_, seconds_, seed_offset):
        arrivals = synth.config4_requests(pool, rate=rate_, duration=seconds_,
                                          seed_offset=seed_offset)
        log(f"serving: {len(arrivals)} arrivals over {seconds_} s at {rate_:g} req/s")
        srv.reset_stats()
        every = max(1, len(arrivals) // (4 * verify))
        tickets = queue.Queue()
        counts = {"refused": 0, "verified": 0, "verified_ok": 0, "collected": 0}
        lock = threading.Lock()
        lag = [0.0]
        n_prod = 4  # submissions validate and copy 2n doubles: several threads keep up
        start = [0.0]

        def producer(j):
            for i in range(j, len(arrivals), n_prod):
                ta, k, seed = arrivals[i]
                now = time.perf_counter() - start[0]
                if ta > now:
                    time.sleep(ta - now)
                elif now - ta > lag[0]:
                    lag[0] = now - ta
                v = seed % variants
                lb, ub = bounds[k][v]
                try:
                    tickets.put((srv.submit(k, lb, ub, max_rounds), k, v, i % every == 0))
                except binding.PropError as e:
                    if e.code != binding.EBUSY:
                        raise
                    with lock:
                        counts["refused"] += 1
            tickets.put(None)

        def consumer():
            done = 0
            while True:
                item = tickets.get()
                if item is None:
                    done += 1
                    if done == n_prod:
                        return
                    continue
                t, k, v, check = item
                res, lb, ub = srv.wait(t, pool[k].n, timeout_ms=300_000, bounds=check)
                counts["collected"] += 1
                if check:
                    r1, lb1, ub1 = alone[k][v]
                    same = (res.status, res.rounds) == (r1.status, r1.rounds) and (
                        r1.status == 1 or (np.array_equal(lb, lb1) and np.array_equal(ub, ub1)))
                    counts["verified"] += 1
                    counts["verified_ok"] += bool(same)

        th_p = [threading.Thread(target=producer, args=(j,)) for j in range(n_prod)]
        th_c = threading.Thread(target=consumer)
        t_start = time.perf_counter()
        start[0] = t_start
        th_c.start()
        for th in th_p:
            th.start()
        for th in th_p:
            th.join()
        th_c.join()
        wall = time.perf_counter() - t_start
        st = srv.stats()
        out = {
            "offered": len(arrivals),
            "offered_per_s": len(arrivals) / seconds_,
            "seconds": seconds_,
            "admitted": len(arrivals) - counts["refused"],
            "refused_busy": counts["refused"],
            "completed": st["completed"],
            "req_per_s": st["req_per_s"],
            "served_per_s_wall": counts["collected"] / wall,
            "p50_ms": st["p50_ms"],
            "p99_ms": st["p99_ms"],
            "mean_ms": st["mean_ms"],
            "max_ms": st["max_ms"],
            "verified": counts["verified"],
            "verified_fraction": counts["verified_ok"] / max(1, counts["verified"]),
            "submit_lag_max_ms": lag[0] * 1e3,
            "peak_device_bytes": st["peak_device_bytes"],
            "round_steps": st["steps"],
        }
        log(f"serving at {rate_:g} req/s: {out}")
        return out

    main = phase(rate, seconds, 0)
    below = phase(rate_below, seconds_below, 1) if rate_below > 0 else None
    srv.close()
    for p in probs:
        p.close()
    rounds = [r[0].rounds for row in alone for r in row]
    out = {
        "workload": f"config4: 64 instances at row scale {scale} ({total_nnz} nnz resident), "
                    f"open-loop Poisson arrivals, 0-5% of the variables fixed per request, "
                    f"max_rounds {max_rounds}",
        **main,
        "max_pending": max_pending,
        "max_slots": max_slots,
        "marking": marking,
        "rounds_per_step": rounds_per_step or 1,
        "budget_bytes": budget,
        "verified_against": "the same request run alone (prop_run), bitwise, on a sample spread "
                            "over the run",
        "alone_rounds_mean": float(np.mean(rounds)),
        "below_capacity": below,
    }
    return out


def kernel_source_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in ("prop_kernels.hip", "prop_device.h", "prop_layout.h", "prop_sum.h",
                 "prop_tiles.h"):
        with open(os.path.join(ROOT, "paper_2009_07785_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
