"""The GPU kernels' activity summation, replayed on the CPU (CPU only).

``host_sum.cpp`` compiles the library's own ``prop_sum.h`` for the host and
runs it in the lane orders of the kernels: rows of K lanes in a chunk, the
node-parallel slots of batches, and long rows in 1024-entry segments.  Every
result must be the exact sum rounded once, as the oracle computes it with
its own fixed-point accumulator: either the double-double fast path
certified it, or the row went to the exact fixed-point path.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle_pins as pins

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2009_07785_amd", "csrc")
BUILD = os.path.join(HERE, "_build")


@pytest.fixture(scope="module")
def hs():
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, "libhostsum.so")
    src = os.path.join(HERE, "host_sum.cpp")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-I", CSRC, src, "-o", out])
    lib = ctypes.CDLL(out)
    P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    for name, args in (("hs_chunk_rowsum", [P, P, i64, i32, P]),
                       ("hs_nodes_rowsum", [P, P, i64, i32, P]),
                       ("hs_long_rowsum", [P, P, i64, i32, P]),
                       ("hs_exact_sum", [P, P, i64])):
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_double
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def all_orders(hs, a, b):
    """(name, value, certified) for every lane order the kernels use."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = a.size
    out = []
    c = ctypes.c_int32(0)
    for K in (1, 2, 4, 8, 16, 32, 64):
        out.append((f"chunk K={K}", hs.hs_chunk_rowsum(_p(a), _p(b), n, K, ctypes.byref(c)),
                    c.value))
        if K >= 16:
            out.append((f"nodes K={K}", hs.hs_nodes_rowsum(_p(a), _p(b), n, K, ctypes.byref(c)),
                        c.value))
    for nodes in (0, 1):
        out.append((f"long nodes={nodes}",
                    hs.hs_long_rowsum(_p(a), _p(b), n, nodes, ctypes.byref(c)), c.value))
    out.append(("digits", hs.hs_exact_sum(_p(a), _p(b), n), 0))
    return out


def check_all(hs, orc, a, b, tag=""):
    want = orc.exact_dot(a, b)
    for name, got, _ in all_orders(hs, a, b):
        assert got == want and np.signbit(got) == np.signbit(want), (tag, name, got, want)


def test_special_cases(hs, orc):
    two = 2.0
    cases = [
        ([1e100, 1.0, -1e100], [1.0, 1.0, 1.0]),
        ([two**53, 1.0], [1.0, 1.0]),
        ([two**53, 1.0, two**-60], [1.0, 1.0, 1.0]),
        ([two**53, 3.0], [1.0, 1.0]),
        ([two**-1074, two**-1074], [1.0, 1.0]),
        ([1e-300], [1e-300]),
        ([0.1, 0.2, -0.3], [1.0, 1.0, 1.0]),
        ([3.0, -2.0], [0.5, 0.75]),
        ([], []),
        ([-1.0], [0.0]),
        ([two**64, -two**64, two**-64], [two**200, two**200, two**-1074]),
        ([1.0, -1.0], [two**-1022, two**-1022 + two**-1074]),
    ]
    for a, b in cases:
        check_all(hs, orc, np.array(a, float), np.array(b, float), (a, b))


def test_counterexample_goes_exact(hs, orc):
    """x1 + x2 + x3 with bounds (2^53, 1, 2^-60): the double-double sum is
    2^53 + 1 + (lost 2^-60), a tie the fast path cannot resolve; the
    certification must refuse it so the exact path gives 2^53 + 2."""
    a = np.ones(3)
    b = np.array([2.0**53, 1.0, 2.0**-60])
    c = ctypes.c_int32(-1)
    got = hs.hs_chunk_rowsum(_p(a), _p(b), 3, 1, ctypes.byref(c))
    assert c.value == 0
    assert got == 2.0**53 + 2 == orc.exact_dot(a, b)
    for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1], [1, 0, 2], [2, 1, 0]):
        check_all(hs, orc, a[perm], b[perm], perm)


def in_domain(a, b):
    """The library's input domain: coefficients 0 or of magnitude in
    [2^-64, 2^64], bounds of magnitude at most 2^200 (the pins of the
    oracle also probe wider exponents, which only the oracle accepts)."""
    a, b = np.abs(np.asarray(a, float)), np.abs(np.asarray(b, float))
    return bool(np.all((a == 0) | ((a >= 2.0**-64) & (a <= 2.0**64))) and np.all(b <= 2.0**200))


def test_oracle_pin_cases(hs, orc):
    """The oracle's own exact-sum pins, through every kernel order (those
    inside the library's input domain)."""
    seen = [0]

    class Shim:
        def exact_dot(self, a, b):
            want = orc.exact_dot(a, b)
            if in_domain(a, b):
                seen[0] += 1
                for name, got, _ in all_orders(hs, a, b):
                    assert got == want, (name, got, want)
            return want

    pins.check_exact_dot_special(Shim())
    pins.check_exact_dot_random(Shim(), trials=200, seed=11)
    assert seen[0] >= 100


def _mant(rng, k):
    """Signed mantissas in [0.5, 1): exponents alone decide the magnitude."""
    return rng.choice([-1.0, 1.0], k) * rng.uniform(0.5, 1.0, k)


def test_random_wide_range(hs, orc):
    rng = np.random.default_rng(5)
    for t in range(300):
        k = int(rng.integers(1, 300))
        a = np.ldexp(_mant(rng, k), rng.integers(-60, 60, k))
        b = np.ldexp(_mant(rng, k), rng.integers(-300, 190, k))
        if t % 4 == 0:
            a = np.concatenate([a, -a[: k // 2]])
            b = np.concatenate([b, b[: k // 2]])
        check_all(hs, orc, a, b, t)


def _near_tie_case(rng):
    """Terms whose exact sum lies on, or a tiny distance from, the midpoint
    between two doubles, spread over terms of mixed magnitude."""
    e = int(rng.integers(-40, 60))
    big = np.ldexp(float(rng.integers(2**52, 2**53)), e - 52)
    half = np.ldexp(1.0, e - 53)  # half an ulp of big
    off = [0.0, np.ldexp(1.0, e - 53 - int(rng.integers(5, 120)))][int(rng.integers(0, 2))]
    off *= [-1.0, 1.0][int(rng.integers(0, 2))]
    parts = [big, half, off]
    # split the big term into pieces that cancel partly
    junk = np.ldexp(rng.uniform(-1, 1, 4), rng.integers(e - 20, e + 20, 4))
    parts += list(junk) + list(-junk)
    parts = np.array(parts)
    rng.shuffle(parts)
    return parts, np.ones(parts.size)


def test_near_ties(hs, orc):
    rng = np.random.default_rng(9)
    refused = 0
    for t in range(400):
        a, b = _near_tie_case(rng)
        check_all(hs, orc, a, b, t)
        refused += sum(1 for name, _, c in all_orders(hs, a, b) if name != "digits" and c == 0)
    assert refused > 0  # the certification does send such rows to the exact path


def test_exact_digits_against_fractions(hs):
    rng = np.random.default_rng(2)
    for t in range(200):
        k = int(rng.integers(1, 30))
        a = np.ldexp(_mant(rng, k), rng.integers(-63, 65, k))
        b = np.ldexp(_mant(rng, k), rng.integers(-1074, 201, k))
        want = float(sum((Fraction(x) * Fraction(y) for x, y in zip(a, b)), Fraction(0))) + 0.0
        got = hs.hs_exact_sum(_p(np.ascontiguousarray(a)), _p(np.ascontiguousarray(b)), k)
        assert got == want, (t, got, want)


def test_certified_fast_path_is_common(hs, orc):
    """On ordinary data the fast path certifies nearly every row."""
    rng = np.random.default_rng(4)
    refused = total = 0
    for t in range(200):
        k = int(rng.integers(2, 60))
        a = rng.choice([-1.0, 1.0], k) * np.where(rng.random(k) < 0.7, 1.0,
                                                    rng.uniform(0, 100, k))
        b = rng.uniform(-1e3, 1e3, k)
        for name, got, c in all_orders(hs, a, b):
            if name != "digits":
                total += 1
                refused += c == 0
    assert refused <= total // 100
