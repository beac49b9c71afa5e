"""CPU code under the address and undefined-behaviour sanitizers (CPU only).

- The oracle and the sequential baseline, rebuilt with
  -fsanitize=address,undefined, run the oracle's pins and the baseline's
  runs in a child process that preloads the sanitizer runtimes.
- The library's host layout builder (prop_layout_host.cpp, no HIP) is
  built with the same sanitizers into a checker that rebuilds the layout
  of several matrices for every step count and checks it against the input.
Any sanitizer report aborts the child with a nonzero status.
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2009_07785_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _runtime(name):
    path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


@pytest.fixture(scope="module")
def build_dir():
    with tempfile.TemporaryDirectory(prefix="san_") as d:
        yield d


CHILD = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import numpy as np
import oracle, oracle_pins, synth
orc = oracle.Oracle({lib!r})
for check in oracle_pins.ALL_CHECKS:
    check(orc)
oracle._SEQ_LIB_PATH = {seq!r}
for inst in (synth.config0(), synth.layout_mix(0), synth.hard_sums(0, tiny=True)):
    r, _ = oracle.CpuSeq(inst).run(inst.lb, inst.ub, 1000)
    assert r.status in (0, 1, 2)
print("sanitized oracle ok")
"""


def test_oracle_under_sanitizers(build_dir):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    lib = os.path.join(build_dir, "liboracle_san.so")
    seq = os.path.join(build_dir, "libcpuseq_san.so")
    for src, out in ((oracle.SOURCE, lib), (oracle.SEQ_SOURCE, seq)):
        subprocess.check_call(["gcc", *SAN, "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-std=gnu11", "-o", out, src, "-lm"])
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    code = CHILD.format(root=ROOT, tests=HERE, lib=lib, seq=seq)
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=900)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-6000:]
    assert "sanitized oracle ok" in res.stdout


def _write(inst, d):
    os.makedirs(d, exist_ok=True)
    np.array([inst.m, inst.n, inst.nnz], dtype=np.int64).tofile(os.path.join(d, "dims"))
    for name, dt in (("row_ptr", np.int64), ("col_idx", np.int32), ("vals", np.float64),
                     ("lhs", np.float64), ("rhs", np.float64), ("vartype", np.uint8)):
        np.ascontiguousarray(getattr(inst, name), dtype=dt).tofile(os.path.join(d, name))


def test_layout_builder_under_sanitizers(build_dir):
    exe = os.path.join(build_dir, "layout_check")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-Wall", "-I", CSRC, "-I",
                           os.path.join(ROOT, "include"), os.path.join(HERE, "layout_check.cpp"),
                           os.path.join(CSRC, "prop_layout_host.cpp"), "-o", exe])
    cases = [synth.config0(), synth.layout_mix(0), synth.layout_mix(2), synth.hard_sums(1),
             synth.config3_matrix(50_000, 25_000),
             synth.from_rows([], [], [], [0.0, 1.0], [1.0, 2.0], [1, 0], n=2),
             synth.from_rows([[], [(0, 0.0)]], [-1.0, -np.inf], [0.0, 3.0], [0.0], [5.0], [1], n=1),
             synth.from_rows([], [], [], [], [], [], n=0)]
    cases += [synth.random_small(s, m=int(3 + s % 9), n=int(3 + s % 7), box=6) for s in range(6)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    for k, inst in enumerate(cases):
        d = os.path.join(build_dir, f"case{k}")
        _write(inst, d)
        res = subprocess.run([exe, d], env=env, capture_output=True, text=True, timeout=600)
        assert res.returncode == 0, (inst.name, res.stdout[-2000:], res.stderr[-6000:])
        assert "layout ok" in res.stdout
