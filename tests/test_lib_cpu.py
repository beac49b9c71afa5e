"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol the header declares, and rejects invalid input before touching the
device."""
import math
import os
import re

import numpy as np
import pytest

from paper_2009_07785_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "prop.h")).read()
    return sorted(set(re.findall(r"\b(prop_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = _declared()
    assert set(names) == set(b.EXPORTED)
    for name in names:
        assert hasattr(b.lib, name), name


def _base():
    # rows: x0 + x1 <= 3 ; x1 - x2 >= -1
    return dict(csr=(2, 3, [0, 2, 4], [0, 1, 1, 2], [1.0, 1.0, 1.0, -1.0]),
                lhs=[-math.inf, -1.0], rhs=[3.0, math.inf], vt=[1, 1, 0])


def _rc(**over):
    d = _base()
    d.update(over)
    rc, _ = b.create_raw(d["csr"], d["lhs"], d["rhs"], d["vt"], d.get("params"))
    return rc


def test_valid_input_reaches_device_stage():
    rc = _rc()
    if rc == b.OK:
        pytest.skip("a GPU is present; the no-device path is not exercised")
    assert rc == b.EDEVICE, b.last_error()


@pytest.mark.parametrize("over,why", [
    (dict(csr=(2, 3, [0, 2, 4], [0, 1, 1, 2], [1.0, np.nan, 1.0, -1.0])), "NaN coefficient"),
    (dict(csr=(2, 3, [0, 2, 4], [0, 1, 1, 2], [1.0, np.inf, 1.0, -1.0])), "infinite coefficient"),
    (dict(csr=(2, 3, [0, 2, 4], [0, 0, 1, 2], [1.0, 1.0, 1.0, -1.0])), "repeated column"),
    (dict(csr=(2, 3, [0, 2, 4], [0, 3, 1, 2], [1.0, 1.0, 1.0, -1.0])), "column out of range"),
    (dict(csr=(2, 3, [0, 2, 4], [0, -1, 1, 2], [1.0, 1.0, 1.0, -1.0])), "negative column"),
    (dict(csr=(2, 3, [0, 3, 4], [0, 1, 1, 2], [1.0, 1.0, 1.0, -1.0])), "row_ptr[m] != nnz"),
    (dict(csr=(2, 3, [1, 2, 4], [0, 1, 1, 2], [1.0, 1.0, 1.0, -1.0])), "row_ptr[0] != 0"),
    (dict(csr=(2, 3, [0, 2, 4], [0, 1, 1, 2], [1e-30, 1.0, 1.0, -1.0])), "tiny coefficient"),
    (dict(csr=(2, 3, [0, 2, 4], [0, 1, 1, 2], [1e30, 1.0, 1.0, -1.0])), "huge coefficient"),
    (dict(lhs=[math.inf, -1.0]), "lhs = +inf"),
    (dict(rhs=[3.0, -math.inf]), "rhs = -inf"),
    (dict(rhs=[np.nan, math.inf]), "NaN rhs"),
    (dict(rhs=[1e70, math.inf]), "rhs beyond 2^200"),
    (dict(vt=[1, 2, 0]), "vartype 2"),
    (dict(params=(0.5, 1e-6, 1e-6)), "eps_int >= 0.5"),
    (dict(params=(1e-6, -1.0, 1e-6)), "negative cont_rel_tol"),
    (dict(params=(1e-6, 1e-6, np.nan)), "NaN feas_tol"),
    (dict(params=(1e-6, 1e-6, 1e-6, 5)), "layout steps 5"),
    (dict(params=(1e-6, 1e-6, 1e-6, 0, 2)), "layout 2"),
])
def test_invalid_input_rejected(over, why):
    assert _rc(**over) == b.EINVAL, why
    assert b.last_error() != ""


def test_decreasing_row_ptr_rejected():
    rc, _ = b.create_raw((2, 3, [0, 3, 2], [0, 1, 2], [1.0, 1.0, 1.0]), [0, 0], [1, 1], [0, 0, 0])
    assert rc == b.EINVAL


def test_null_out_pointer():
    import ctypes

    d = _base()
    m, n, rp, ci, va = d["csr"]
    rp, ci, va = (np.asarray(rp, np.int64), np.asarray(ci, np.int32), np.asarray(va, np.float64))
    csr = b._Csr(m, n, 4, b._ptr(rp).value, b._ptr(ci).value, b._ptr(va).value)
    lh = np.asarray(d["lhs"], np.float64)
    rh = np.asarray(d["rhs"], np.float64)
    vt = np.asarray(d["vt"], np.uint8)
    assert b.lib.prop_create(ctypes.byref(csr), b._ptr(lh), b._ptr(rh), b._ptr(vt), None,
                             None) == b.EINVAL


def test_null_problem_calls():
    import ctypes

    res = b._Result()
    assert b.lib.prop_run(None, None, None, 10, ctypes.byref(res)) == b.EINVAL
    assert b.lib.prop_run_batch(None, 1, None, None, 10, ctypes.byref(res)) == b.EINVAL
    assert b.lib.prop_set_loop(None, 0) == b.EINVAL
    assert b.lib.prop_set_store(None, 32) == b.EINVAL
    b.lib.prop_destroy(None)


def test_server_argument_checks():
    """prop_srv_create / submit / poll reject bad arguments without a device."""
    import ctypes

    for cfg, why in (((0,), "zero budget"), ((1 << 20, 7), "slots not a multiple of 8"),
                     ((1 << 20, 0, 65), "rounds_per_step > 64"),
                     ((1 << 20, 0, 0, -1), "negative max_pending")):
        rc, _ = b.srv_create_raw(*cfg)
        assert rc == b.EINVAL, why
    rc, h = b.srv_create_raw(1 << 20)
    assert rc == b.OK, b.last_error()
    try:
        t = ctypes.c_int64()
        assert b.lib.prop_srv_submit(h, 0, None, None, 5, ctypes.byref(t)) == b.EINVAL
        assert b.lib.prop_srv_submit(h, 0, None, None, -1, ctypes.byref(t)) == b.EINVAL
        assert b.lib.prop_srv_poll(h, 1, None, None, None) == b.EINVAL
        assert b.lib.prop_srv_wait(h, 1, 0, None, None, None) == b.EINVAL
        assert b.lib.prop_srv_add_instance(h, None, ctypes.byref(ctypes.c_int32())) == b.EINVAL
        st = b._SrvStats()
        assert b.lib.prop_srv_get_stats(h, ctypes.byref(st)) == b.OK
        assert st.submitted == 0 and st.device_bytes == 0
        assert b.lib.prop_srv_reset_stats(h) == b.OK
    finally:
        b.lib.prop_srv_destroy(h)
    b.lib.prop_srv_destroy(None)


def test_autotune_argument_checks():
    import ctypes

    d = _base()
    m, n, rp, ci, va = d["csr"]
    rp = np.asarray(rp, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int32)
    va = np.asarray(va, dtype=np.float64)
    csr = b._Csr(m, n, int(rp[-1]), b._ptr(rp).value, b._ptr(ci).value, b._ptr(va).value)
    lh = np.asarray(d["lhs"], dtype=np.float64)
    rh = np.asarray(d["rhs"], dtype=np.float64)
    vt = np.asarray(d["vt"], dtype=np.uint8)
    lb = np.zeros(n)
    ub = np.ones(n)
    out = ctypes.c_int32()
    args = (ctypes.byref(csr), b._ptr(lh), b._ptr(rh), b._ptr(vt), None, b._ptr(lb), b._ptr(ub))
    assert b.lib.prop_autotune(*args, 10, None) == b.EINVAL
    assert b.lib.prop_autotune(*args, -1, ctypes.byref(out)) == b.EINVAL
    bad = va.copy()
    bad[0] = np.nan
    csr_bad = b._Csr(m, n, int(rp[-1]), b._ptr(rp).value, b._ptr(ci).value, b._ptr(bad).value)
    assert b.lib.prop_autotune(ctypes.byref(csr_bad), *args[1:], 10, ctypes.byref(out)) == b.EINVAL
