"""Seeded generators for the synthetic workloads.

The paper's test bed (MIPLIB 2017) is not available here, so these
instances stand in for its shapes: short rows with a heavy tail, a few
very dense "connecting" rows, skewed column degrees and a mix of binary,
integer and continuous variables (the shape effects of Sec. 3.6 of the
paper).  Every row's sides are drawn around a random point x0 so that the
root problem is feasible unless a config asks otherwise.

Workloads (sizes and distributions):
  config0  2,000 x 1,000, 10 distinct uniform columns per row, integer
           coefficients in [-10, 10] \\ {0}; 50% binary, 30% integer [0,100],
           20% continuous [-1e3, 1e3] (5% of those with one infinite bound).
  config1  200,000 x 100,000; row lengths max(1, rint(LogNormal(ln 6, 1)))
           plus 0.1% dense rows of 5,000; coefficients 70% +-1, 30%
           U[-100, 100]; a suite of seeds, every 50th made infeasible (one
           row's rhs set 1-10 below its minimum over the root box).
  config2  5,000,000 x 2,000,000; row lengths floor(Pareto) with pdf exponent
           2.2, minimum 2, capped at 200,000; column weights from the same
           law and each row's distinct columns drawn in proportion to them;
           40% binary / 30% integer / 30% continuous.
  config3  1,000,000 x 500,000 matrix drawn as config2, plus 256 node bound
           vectors, each fixing 1-5% of the integer variables (to x0, or in a
           quarter of the nodes to random values).
  config4  64 instances of log-uniform size in [1e4, 2e6] rows drawn as
           config1, plus a Poisson request stream fixing 0-5% of the vars.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

BASE_SEED = 200907785

INF = np.inf


@dataclass
class Instance:
    name: str
    m: int
    n: int
    row_ptr: np.ndarray  # int64 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: np.ndarray  # float64 [nnz]
    lhs: np.ndarray  # float64 [m]
    rhs: np.ndarray  # float64 [m]
    vartype: np.ndarray  # uint8 [n], 0 continuous, 1 integer
    lb: np.ndarray  # float64 [n]
    ub: np.ndarray  # float64 [n]
    x0: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# small hand-built systems
# --------------------------------------------------------------------------
def from_rows(rows, lhs, rhs, lb, ub, vartype=None, n=None, name="hand") -> Instance:
    """Build an instance from rows given as lists of (column, coefficient)."""
    if n is None:
        n = len(lb)
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    cols, vals = [], []
    for i, r in enumerate(rows):
        for j, a in r:
            cols.append(j)
            vals.append(a)
        row_ptr[i + 1] = len(cols)
    vt = np.zeros(n, np.uint8) if vartype is None else np.asarray(vartype, dtype=np.uint8)
    return Instance(
        name=name, m=len(rows), n=n, row_ptr=row_ptr,
        col_idx=np.asarray(cols, dtype=np.int32), vals=np.asarray(vals, dtype=np.float64),
        lhs=np.asarray(lhs, dtype=np.float64), rhs=np.asarray(rhs, dtype=np.float64),
        vartype=vt, lb=np.asarray(lb, dtype=np.float64).copy(),
        ub=np.asarray(ub, dtype=np.float64).copy())


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def _variables(rng, n, frac_bin, frac_int, frac_inf_of_cont):
    nb = int(round(n * frac_bin))
    ni = int(round(n * frac_int))
    nc = n - nb - ni
    kind = np.concatenate([np.zeros(nb, np.int8), np.ones(ni, np.int8), np.full(nc, 2, np.int8)])
    kind = rng.permutation(kind)
    vartype = (kind != 2).astype(np.uint8)
    lb = np.where(kind == 0, 0.0, np.where(kind == 1, 0.0, -1e3))
    ub = np.where(kind == 0, 1.0, np.where(kind == 1, 100.0, 1e3))
    x0 = np.empty(n)
    x0[kind == 0] = rng.integers(0, 2, size=nb)
    x0[kind == 1] = rng.integers(0, 101, size=ni)
    x0[kind == 2] = rng.uniform(-1e3, 1e3, size=nc)
    cont = np.nonzero(kind == 2)[0]
    k_inf = int(round(nc * frac_inf_of_cont))
    if k_inf:
        pick = rng.choice(cont, size=k_inf, replace=False)
        side = rng.random(k_inf) < 0.5
        lb[pick[side]] = -INF
        ub[pick[~side]] = INF
    return vartype, lb.astype(np.float64), ub.astype(np.float64), x0


def _distinct_columns(rng, lengths, n, cum_weights=None):
    """Per row, `lengths[i]` distinct columns, drawn uniformly or in proportion
    to weights.  Draws repeat until each row holds enough distinct columns,
    which is sampling without replacement in proportion to the weights."""
    lengths = np.asarray(lengths, dtype=np.int64)
    m = lengths.size
    if np.any(lengths > n):
        raise ValueError("row longer than the number of columns")

    def draw(k):
        if cum_weights is None:
            return rng.integers(0, n, size=k, dtype=np.int64)
        # sorted queries keep the binary search cache-friendly; the shuffle
        # afterwards restores independent draws in random order
        u = np.sort(rng.random(k)) * cum_weights[-1]
        idx = np.minimum(np.searchsorted(cum_weights, u, side="right"), n - 1).astype(np.int64)
        rng.shuffle(idx)
        return idx

    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    keys = np.unique(rows * n + draw(rows.size))
    del rows
    done = []
    while keys.size:
        krow = keys // n
        cnt = np.bincount(krow, minlength=m)
        fin = cnt[krow] == lengths[krow]
        done.append(keys[fin])
        keys = keys[~fin]
        if keys.size == 0:
            break
        act = np.unique(keys // n)
        d = lengths[act] - cnt[act]
        new_rows = np.repeat(act, d)
        keys = np.unique(np.concatenate([keys, new_rows * n + draw(new_rows.size)]))
    allk = np.concatenate(done) if done else np.zeros(0, np.int64)
    allk.sort()
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    assert allk.size == row_ptr[-1]
    return row_ptr, (allk % n).astype(np.int32)


def _coeffs_mixed(rng, k):
    """70% +-1 (sign 50/50), 30% uniform in [-100, 100] (exact zero redrawn)."""
    unit = rng.random(k) < 0.7
    sign = np.where(rng.random(k) < 0.5, -1.0, 1.0)
    v = np.where(unit, sign, rng.uniform(-100.0, 100.0, size=k))
    z = np.nonzero(v == 0.0)[0]
    while z.size:
        v[z] = rng.uniform(-100.0, 100.0, size=z.size)
        z = z[v[z] == 0.0]
    return v


def _coeffs_int(rng, k):
    mag = rng.integers(1, 11, size=k).astype(np.float64)
    return np.where(rng.random(k) < 0.5, -mag, mag)


def _row_dot(row_ptr, col, vals, x):
    """Plain row-wise dot products a_i . x used to place the row sides."""
    prod = vals * x[col]
    m = row_ptr.size - 1
    out = np.zeros(m)
    nonempty = row_ptr[1:] > row_ptr[:-1]
    if prod.size:
        sums = np.add.reduceat(prod, row_ptr[:-1][nonempty])
        out[nonempty] = sums
    return out


def _sides(rng, s, frac_one_sided=0.1):
    m = s.size
    lhs = s - rng.uniform(0.0, 20.0, size=m)
    rhs = s + rng.uniform(0.0, 20.0, size=m)
    one = rng.random(m) < frac_one_sided
    drop_l = rng.random(m) < 0.5
    lhs[one & drop_l] = -INF
    rhs[one & ~drop_l] = INF
    return lhs, rhs


def _make_infeasible(rng, inst: Instance):
    """Set one row's rhs below its minimum over the root box: the row is
    chosen among rows whose minimising bounds (l_j for a_j > 0, u_j for
    a_j < 0) are all finite, rhs becomes that minimum minus U[1, 10] and
    lhs becomes -inf.  The margin of at least 1 is far above the rounding
    of the float sum taken here, so the row excludes the whole box."""
    lengths = inst.row_lengths()
    a = inst.vals
    bmin = np.where(a > 0, inst.lb[inst.col_idx], inst.ub[inst.col_idx])
    ok_nnz = np.isfinite(bmin).astype(np.int64)
    ok_rows = np.add.reduceat(ok_nnz, inst.row_ptr[:-1]) == lengths
    cand = np.nonzero(ok_rows & (lengths > 0))[0]
    i = int(rng.choice(cand))
    sl = slice(inst.row_ptr[i], inst.row_ptr[i + 1])
    low = float(np.sum(a[sl] * bmin[sl]))
    inst.rhs[i] = low - rng.uniform(1.0, 10.0)
    inst.lhs[i] = -INF
    inst.meta["infeasible_row"] = i
    return inst


def _pareto_lengths(rng, m, lmin=2.0, cap=200_000, tail=1.2):
    # numpy's pareto(a) + 1 is the classical Pareto with tail index a; a pdf
    # exponent of 2.2 is tail index 1.2
    x = (rng.pareto(tail, size=m) + 1.0) * lmin
    return np.minimum(np.floor(x), cap).astype(np.int64)


# --------------------------------------------------------------------------
# configs
# --------------------------------------------------------------------------
def config0(seed_offset: int = 0) -> Instance:
    rng = _rng(BASE_SEED + 0 + seed_offset)
    m, n = 2000, 1000
    vartype, lb, ub, x0 = _variables(rng, n, 0.5, 0.3, 0.05)
    row_ptr, col = _distinct_columns(rng, np.full(m, 10), n)
    vals = _coeffs_int(rng, col.size)
    lhs, rhs = _sides(rng, _row_dot(row_ptr, col, vals, x0))
    return Instance("config0", m, n, row_ptr, col, vals, lhs, rhs, vartype, lb, ub, x0)


def _lognormal_instance(rng, m, n, name, dense_len=5000, dense_frac=0.001):
    vartype, lb, ub, x0 = _variables(rng, n, 0.5, 0.3, 0.05)
    n_dense = int(round(m * dense_frac))
    lengths = np.maximum(1, np.rint(rng.lognormal(np.log(6.0), 1.0, size=m))).astype(np.int64)
    lengths = np.minimum(lengths, n)
    if n_dense:
        lengths[rng.choice(m, size=n_dense, replace=False)] = min(dense_len, n)
    row_ptr, col = _distinct_columns(rng, lengths, n)
    vals = _coeffs_mixed(rng, col.size)
    lhs, rhs = _sides(rng, _row_dot(row_ptr, col, vals, x0))
    return Instance(name, m, n, row_ptr, col, vals, lhs, rhs, vartype, lb, ub, x0)


def config1(k: int = 1) -> Instance:
    """Member k of the config-1 suite (seed BASE_SEED + 100 + k); members with
    k % 50 == 0 get one infeasible row."""
    rng = _rng(BASE_SEED + 100 + k)
    inst = _lognormal_instance(rng, 200_000, 100_000, f"config1[{k}]")
    if k % 50 == 0:
        _make_infeasible(rng, inst)
    return inst


def _powerlaw_instance(rng, m, n, name, lmin=2.0):
    vartype, lb, ub, x0 = _variables(rng, n, 0.4, 0.3, 0.05)
    lengths = np.minimum(_pareto_lengths(rng, m, lmin=lmin), n)
    w = np.minimum((rng.pareto(1.2, size=n) + 1.0) * lmin, 200_000.0)
    cum = np.cumsum(w)
    row_ptr, col = _distinct_columns(rng, lengths, n, cum_weights=cum)
    vals = _coeffs_mixed(rng, col.size)
    lhs, rhs = _sides(rng, _row_dot(row_ptr, col, vals, x0))
    return Instance(name, m, n, row_ptr, col, vals, lhs, rhs, vartype, lb, ub, x0)


def config2(m: int = 5_000_000, n: int = 2_000_000) -> Instance:
    rng = _rng(BASE_SEED + 2)
    return _powerlaw_instance(rng, m, n, f"config2[{m}x{n}]")


def config3_matrix(m: int = 1_000_000, n: int = 500_000) -> Instance:
    rng = _rng(BASE_SEED + 3)
    return _powerlaw_instance(rng, m, n, f"config3[{m}x{n}]")


def node_bounds(inst: Instance, seed: int, frac_lo=0.01, frac_hi=0.05, only_int=True,
                random_share=0.25):
    """Root bounds with a random fraction of the variables fixed.  A node
    either fixes every chosen variable to its x0 value (x0 stays feasible) or,
    with probability `random_share`, fixes the chosen integer variables to
    uniform integers in their range (such nodes are usually infeasible);
    continuous variables, when included, are fixed to x0_j."""
    rng = _rng(seed)
    lb = inst.lb.copy()
    ub = inst.ub.copy()
    frac = rng.uniform(frac_lo, frac_hi)
    random_node = rng.random() < random_share
    pool = np.nonzero(inst.vartype == 1)[0] if only_int else np.arange(inst.n)
    k = int(round(frac * pool.size))
    if k == 0:
        return lb, ub
    pick = rng.choice(pool, size=k, replace=False)
    is_int = inst.vartype[pick] == 1
    lo = np.where(np.isfinite(lb[pick]), lb[pick], -1e3)
    hi = np.where(np.isfinite(ub[pick]), ub[pick], 1e3)
    rand_int = np.minimum(np.floor(lo + rng.random(k) * (hi - lo + 1.0)), hi)
    val = np.where(is_int & random_node, rand_int, inst.x0[pick])
    lb[pick] = val
    ub[pick] = val
    return lb, ub


def branch_children(parent_lb, parent_ub, vartype, count: int, seed: int, per_child: int = 1):
    """Branch-and-bound children of a node whose bounds are (parent_lb,
    parent_ub): child 2i and 2i + 1 split the domain of the same unfixed
    integer variables (`per_child` of them) at the middle, the first keeping
    the lower half, the second the upper half.  Returns (lbs, ubs) of shape
    (count, n)."""
    rng = _rng(seed)
    lbs = np.repeat(np.asarray(parent_lb, dtype=np.float64)[None, :], count, axis=0)
    ubs = np.repeat(np.asarray(parent_ub, dtype=np.float64)[None, :], count, axis=0)
    free = np.nonzero((vartype == 1) & (parent_lb < parent_ub) & np.isfinite(parent_lb)
                      & np.isfinite(parent_ub))[0]
    if free.size == 0:
        return lbs, ubs
    for i in range(0, count, 2):
        pick = rng.choice(free, size=min(per_child, free.size), replace=False)
        mid = np.floor((parent_lb[pick] + parent_ub[pick]) / 2.0)
        ubs[i, pick] = mid
        if i + 1 < count:
            lbs[i + 1, pick] = mid + 1.0
    return lbs, ubs


def config3_nodes(inst: Instance, count: int = 256):
    lbs = np.empty((count, inst.n))
    ubs = np.empty((count, inst.n))
    for k in range(count):
        lbs[k], ubs[k] = node_bounds(inst, BASE_SEED + 3000 + k)
    return lbs, ubs


def _config4_instance(args):
    k, mk = args
    mk = max(int(mk), 10)
    nk = max(mk // 2, 5)
    sub = _rng(BASE_SEED + 4000 + k)
    return _lognormal_instance(sub, mk, nk, f"config4[{k}]", dense_len=min(5000, nk))


def config4_pool(count: int = 64, m_lo: float = 1e4, m_hi: float = 2e6, scale: float = 1.0,
                 workers: int = 1):
    """The serving pool; `scale` shrinks every instance (tests use < 1).
    Every instance has its own seed, so `workers` processes may generate
    them side by side with the same result."""
    rng = _rng(BASE_SEED + 4)
    ms = np.rint(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi), size=count)) * scale)
    jobs = list(enumerate(ms.astype(np.int64)))
    if workers <= 1:
        return [_config4_instance(j) for j in jobs]
    import multiprocessing as mp

    # largest first, so that the big instances do not finish last
    order = sorted(range(count), key=lambda k: -int(ms[k]))
    with mp.get_context("fork").Pool(workers) as pool:
        made = pool.map(_config4_instance, [jobs[k] for k in order], chunksize=1)
    out = [None] * count
    for k, inst in zip(order, made):
        out[k] = inst
    return out


def config4_requests(pool, rate: float = 2000.0, duration: float = 60.0, seed_offset: int = 0):
    """Open-loop Poisson arrivals: list of (arrival_time_s, instance_id, node_seed)."""
    rng = _rng(BASE_SEED + 4 + 1_000_000 + seed_offset)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append((t, int(rng.integers(0, len(pool))), int(rng.integers(0, 2**62))))
    return out


def request_bounds(inst: Instance, node_seed: int):
    """A serving request: 0-5% of all variables fixed to their x0 values."""
    return node_bounds(inst, node_seed, frac_lo=0.0, frac_hi=0.05, only_int=False,
                       random_share=0.0)


def random_small(seed: int, m: int, n: int, max_len: int = 6, int_frac: float = 1.0,
                 box: int = 5, inf_frac: float = 0.0, coef: int = 5, one_sided: float = 0.1,
                 slack: float = 3.0) -> Instance:
    """Tiny random systems for brute force and property checks: integer
    coefficients in [-coef, coef] \\ {0}, boxes of at most `box` + 1 values."""
    rng = _rng(BASE_SEED + 900_000 + seed)
    vartype = (rng.random(n) < int_frac).astype(np.uint8)
    lo = rng.integers(-box, 1, size=n).astype(np.float64)
    hi = lo + rng.integers(0, box + 1, size=n)
    x0 = lo + np.floor(rng.random(n) * (hi - lo + 1))
    x0 = np.minimum(x0, hi)
    cont = vartype == 0
    x0[cont] = lo[cont] + rng.random(cont.sum()) * (hi[cont] - lo[cont])
    lb, ub = lo.copy(), hi.copy()
    if inf_frac > 0:
        inf = rng.random(n) < inf_frac
        side = rng.random(n) < 0.5
        lb[inf & side] = -INF
        ub[inf & ~side] = INF
    lengths = rng.integers(1, min(max_len, n) + 1, size=m)
    row_ptr, col = _distinct_columns(rng, lengths, n)
    mag = rng.integers(1, coef + 1, size=col.size).astype(np.float64)
    vals = np.where(rng.random(col.size) < 0.5, -mag, mag)
    s = _row_dot(row_ptr, col, vals, x0)
    lhs = s - np.floor(rng.random(m) * slack)
    rhs = s + np.floor(rng.random(m) * slack)
    one = rng.random(m) < one_sided
    dl = rng.random(m) < 0.5
    lhs[one & dl] = -INF
    rhs[one & ~dl] = INF
    return Instance(f"small[{seed}]", m, n, row_ptr, col, vals, lhs, rhs, vartype, lb, ub, x0)


def code_edges(seed: int = 0, n: int = 4000, m: int = 6000) -> Instance:
    """Integer variables whose bounds sit on both sides of the small-integer
    range [-126, 126] (and at its edges, and infinite), continuous ones
    mixed in, rows of 1-12 entries plus some of 300-2,000 entries, small
    integer coefficients and sides close to a feasible point, so that
    propagation moves integer bounds into the range and across its edges."""
    rng = _rng(BASE_SEED + 800_000 + seed)
    inf = INF
    lows = np.array([-inf, -300.0, -128.0, -127.0, -126.0, -125.0, -3.0, 0.0, 1.0, 120.0,
                     125.0, 126.0, 127.0, 200.0])
    widths = np.array([0.0, 1.0, 2.0, 5.0, 30.0, 130.0, 253.0, 260.0, 600.0, inf])
    vartype = (rng.random(n) < 0.85).astype(np.uint8)
    lb = lows[rng.integers(0, lows.size, n)]
    free_lo = np.isinf(lb)
    ub = np.where(free_lo, rng.choice([-126.0, 0.0, 126.0, 127.0, 1000.0, inf], n),
                  np.where(free_lo, 0.0, lb) + widths[rng.integers(0, widths.size, n)])
    cont = vartype == 0
    shift = rng.random(n) * 0.5  # fractional bounds for the continuous variables
    lb = np.where(cont & ~np.isinf(lb), lb + shift, lb)
    ub = np.where(cont & ~np.isinf(ub), ub + shift, ub)
    # a finite point inside every box
    flo = np.where(np.isinf(lb), np.where(np.isinf(ub), 0.0, ub - 50.0), lb)
    fhi = np.where(np.isinf(ub), flo + 50.0, ub)
    x0 = flo + np.floor(rng.random(n) * (fhi - flo + 1))
    x0 = np.minimum(x0, fhi)
    x0[cont] = flo[cont] + rng.random(cont.sum()) * (fhi[cont] - flo[cont])
    lengths = rng.integers(1, 13, size=m)
    lengths[rng.random(m) < 0.004] = rng.integers(300, 2000, size=1)[0]
    row_ptr, col = _distinct_columns(rng, lengths, n)
    mag = rng.integers(1, 6, size=col.size).astype(np.float64)
    vals = np.where(rng.random(col.size) < 0.5, -mag, mag)
    s = _row_dot(row_ptr, col, vals, x0)
    lhs = s - np.floor(rng.random(m) * 12)
    rhs = s + np.floor(rng.random(m) * 12)
    one = rng.random(m) < 0.2
    dl = rng.random(m) < 0.5
    lhs[one & dl] = -INF
    rhs[one & ~dl] = INF
    return Instance(f"code_edges[{seed}]", m, n, row_ptr, col, vals, lhs, rhs, vartype, lb, ub, x0)


def layout_mix(seed: int = 0, copies: int = 3) -> Instance:
    """Rows of every length class a wave tile distinguishes (1 .. 1024 entries,
    ragged within each class) plus rows longer than 1024 entries, some of them
    built so that they do tighten bounds: a cardinality row forcing 3,000
    binaries to 0, and a row whose only infinite contribution belongs to one
    free variable."""
    rng = _rng(BASE_SEED + 700_000 + seed)
    n = 20_000
    vartype, lb, ub, x0 = _variables(rng, n, 0.4, 0.3, 0.1)
    lens = [1, 2, 3, 5, 8, 15, 16, 17, 24, 31, 32, 33, 47, 63, 64, 65, 100, 127, 128, 129,
            200, 255, 256, 257, 400, 511, 512, 513, 700, 1000, 1023, 1024, 1025, 1500, 2047,
            2048, 2049, 3000, 5000]
    lengths = np.array(lens * copies + list(rng.integers(1, 40, size=400)), dtype=np.int64)
    lengths = rng.permutation(lengths)
    row_ptr, col = _distinct_columns(rng, lengths, n - 5001)
    vals = _coeffs_mixed(rng, col.size)
    lhs, rhs = _sides(rng, _row_dot(row_ptr, col, vals, x0))
    # special long rows over variables no other row touches
    base = n - 5001
    card = np.arange(base, base + 3000)
    vartype[card] = 1
    lb[card], ub[card] = 0.0, 1.0
    x0[card] = 0.0
    grp = np.arange(base + 3000, base + 5000)
    vartype[grp] = 1
    lb[grp], ub[grp] = 0.0, 1.0
    free = n - 1
    vartype[free] = 0
    lb[free], ub[free] = -INF, INF
    x0[free] = 10.0
    extra_rows = [(card, np.ones(card.size), -INF, 0.0),
                  (np.concatenate([grp, [free]]), np.ones(grp.size + 1), 5.0, INF)]
    rp = list(row_ptr)
    cols = [col]
    vs = [vals]
    lh, rh = list(lhs), list(rhs)
    for c, v, lo_, hi_ in extra_rows:
        cols.append(c.astype(np.int32))
        vs.append(v)
        rp.append(rp[-1] + c.size)
        lh.append(lo_)
        rh.append(hi_)
    return Instance(f"layout_mix[{seed}]", len(rp) - 1, n, np.array(rp, dtype=np.int64),
                    np.concatenate(cols).astype(np.int32), np.concatenate(vs),
                    np.array(lh), np.array(rh), vartype, lb, ub, x0)


def _hard_terms(rng, kind: int):
    """Coefficients and bound values whose products sum to a value on, or a
    tiny distance from, the midpoint between two doubles, or cancel to a
    small remainder: the sums a double-double accumulator cannot round
    correctly on its own.  Magnitudes stay inside the library's input domain
    (coefficients in [2^-64, 2^64], bounds up to 2^200)."""
    two = 2.0
    if kind == 0:  # 2^53 + 1 + 2^-60 and relatives: the tie hides in the lost bits
        k = int(rng.integers(0, 60))
        a = [1.0, 1.0, 1.0]
        b = [two ** (53 + k), two**k, two ** (k - int(rng.integers(55, 110)))]
    elif kind == 1:  # exact tie, rounds to even
        k = int(rng.integers(-30, 30))
        a = [1.0, 1.0]
        b = [two ** (53 + k) + 2 * float(rng.integers(0, 4)) * two**k, two**k]
    elif kind == 2:  # cancellation of large terms around a small remainder
        big = np.ldexp(rng.uniform(0.5, 1.0), int(rng.integers(100, 190)))
        small = np.ldexp(rng.uniform(0.5, 1.0), int(rng.integers(-60, 60)))
        a = [1.0, -1.0, 1.0]
        b = [big, big, small]
    else:  # near-midpoint sums of mixed-magnitude pieces
        e = int(rng.integers(-40, 60))
        big = np.ldexp(float(rng.integers(2**52, 2**53)), e - 52)
        half = np.ldexp(1.0, e - 53)
        off = np.ldexp(1.0, e - 53 - int(rng.integers(5, 100))) * rng.choice([-1.0, 0.0, 1.0])
        junk = list(np.ldexp(rng.uniform(0.5, 1.0, 3), rng.integers(e - 20, e + 20, 3)))
        b = [big, half, off] + junk + [-x for x in junk]
        b = [x for x in b if x != 0.0]
        a = [1.0] * len(b)
    # spread each term over a coefficient and a bound: a * b stays exact
    a = np.array(a, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    sh = rng.integers(-8, 9, size=a.size)
    a = np.ldexp(a, sh)
    b = np.ldexp(b, -sh)
    return a, b


def hard_sums(seed: int = 0, count: int = 64,
              lengths=(3, 7, 20, 60, 130, 300, 900, 2500), tiny: bool = False) -> Instance:
    """Rows whose min activity is a hard sum (see _hard_terms), one row per
    case, padded to each of `lengths` entries with variables in [0, 1] (zero
    contribution to the min activity) so that every lanes-per-row class and
    the long-row segments see them.  Each term owns a continuous variable:
    a > 0 gets lower bound b (upper +inf), a < 0 upper bound b (lower -inf),
    so the min activity is exactly the sum of the terms.  rhs sits a few
    units above it; every candidate of the row depends on the activity's
    last bits.  With `tiny`, one term per row uses a bound of magnitude below
    2^-906 (the products a kernel cannot split exactly with an FMA)."""
    rng = _rng(BASE_SEED + 800_000 + seed)
    rows, lhs, rhs, lb, ub = [], [], [], [], []
    n = 0
    for c in range(count):
        a, b = _hard_terms(rng, c % 4)
        if tiny:
            a = np.append(a, np.ldexp(rng.uniform(1.0, 2.0), int(rng.integers(-60, 60))))
            b = np.append(b, np.ldexp(rng.uniform(0.5, 1.0), int(rng.integers(-1074, -907))))
        L = int(lengths[c % len(lengths)])
        pad = max(0, L - a.size)
        row = []
        for x, y in zip(a, b):
            row.append((n, float(x)))
            if x > 0:
                lb.append(float(y))
                ub.append(INF)
            else:
                lb.append(-INF)
                ub.append(float(y))
            n += 1
        for _ in range(pad):
            row.append((n, 1.0))
            lb.append(0.0)
            ub.append(1.0)
            n += 1
        row = [row[q] for q in rng.permutation(len(row))]
        rows.append(row)
        # the products are exact by construction, so fsum places rhs just
        # above the row's exact sum
        s0 = math.fsum(float(x) * float(y) for x, y in zip(a, b))
        scale = max(abs(s0), 1.0)
        lhs.append(-INF)
        rhs.append(s0 + float(rng.integers(1, 6)) * float(np.spacing(scale)))
    return from_rows(rows, lhs, rhs, lb, ub, np.zeros(n, np.uint8), n=n,
                     name=f"hard_sums[{seed}{',tiny' if tiny else ''}]")


# --------------------------------------------------------------------------
# optional on-disk cache (directory from PROP_SYNTH_CACHE), so one process can
# reuse what an earlier one generated
# --------------------------------------------------------------------------
_FIELDS = ("row_ptr", "col_idx", "vals", "lhs", "rhs", "vartype", "lb", "ub", "x0")


def cached(key: str, fn, *args, **kw) -> Instance:
    import os

    d = os.environ.get("PROP_SYNTH_CACHE")
    if not d:
        return fn(*args, **kw)
    path = os.path.join(d, key + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        arrs = {f: z[f] for f in _FIELDS}
        return Instance(str(z["name"]), int(z["m"]), int(z["n"]), x0=arrs.pop("x0"), **arrs)
    inst = fn(*args, **kw)
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, name=np.array(inst.name), m=np.array(inst.m), n=np.array(inst.n),
             **{f: getattr(inst, f) for f in _FIELDS})
    os.replace(tmp, path)
    return inst
