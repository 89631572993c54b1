"""C-ABI checks that need no GPU: every symbol declared in include/qsv.h is
exported by libqsv.so, the library's standard gate matrices agree with the
oracle's textbook ones, and argument validation rejects bad calls on the host
before any device work."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2502_11385_amd import qsv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "qsv.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert len(names) >= 15
    lib = qsv.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(qsv.EXPORTED)


@pytest.mark.parametrize("name,params", [
    ("h", ()), ("x", ()), ("y", ()), ("z", ()), ("s", ()), ("sdg", ()),
    ("p", (0.3,)), ("u3", (0.1, 2.5, -1.2)), ("u3", (math.pi, 0, math.pi))])
def test_gate_matrix_matches_oracle(name, params):
    want = oracle.gate_spec(name, (0,), params)[2]
    got = qsv.gate_matrix(name, params)
    assert np.max(np.abs(got - want)) < 1e-15


def test_gate_matrix_errors():
    with pytest.raises(qsv.QsvError) as e:
        qsv.gate_matrix("nope")
    assert e.value.status == qsv.QSV_ERR_UNSUPPORTED
    with pytest.raises(qsv.QsvError) as e:
        qsv.gate_matrix("u3", (1.0,))
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG


def _status(fn, *args):
    return fn(*args)


def test_alloc_validation_without_device():
    lib = qsv.lib()
    h = C.c_void_p()
    assert lib.qsv_alloc(0, qsv.QSV_C64, None, C.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert lib.qsv_alloc(35, qsv.QSV_C64, None, C.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert lib.qsv_alloc(10, 3, None, C.byref(h)) == qsv.QSV_ERR_UNSUPPORTED
    assert lib.qsv_alloc(10, qsv.QSV_C64, None, None) == qsv.QSV_ERR_INVALID_ARG
    assert lib.qsv_wrap(10, qsv.QSV_C64, None, 1 << 20, None,
                        C.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert lib.qsv_wrap(10, qsv.QSV_C64, 0x1008, 1 << 20, None,
                        C.byref(h)) == qsv.QSV_ERR_INVALID_ARG  # misaligned
    assert lib.qsv_wrap(10, qsv.QSV_C64, 0x1000, 100, None,
                        C.byref(h)) == qsv.QSV_ERR_INVALID_ARG  # too small
    assert "buffer smaller" in qsv.last_error()


def test_null_state_calls():
    lib = qsv.lib()
    assert lib.qsv_free(None) == qsv.QSV_OK
    assert lib.qsv_init_basis(None, 0) == qsv.QSV_ERR_INVALID_ARG
    assert lib.qsv_sync(None) == qsv.QSV_ERR_INVALID_ARG
    d = C.c_double()
    assert lib.qsv_norm(None, C.byref(d)) == qsv.QSV_ERR_INVALID_ARG
    assert lib.qsv_apply_fused(None, None, None) == qsv.QSV_ERR_INVALID_ARG


def _circ(gates):
    c = qsv.Circuit()
    for t, ctl, m in gates:
        c.add(t, m, ctl)
    return c


X = np.array([[0, 1], [1, 0]], complex)


@pytest.mark.parametrize("bad,msg", [
    ([([5], [], X)], "out of range"),
    ([([1], [1], X)], "duplicate"),
    ([([0, 1, 2, 3, 4, 5], [], np.eye(64))], "k must be"),
    ([([0], [], np.array([[np.nan, 0], [0, 1]]))], "non-finite"),
])
def test_plan_validation(bad, msg):
    c = _circ(bad)
    with pytest.raises(qsv.QsvError) as e:
        qsv.plan_describe(c, 5)
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    assert msg in str(e.value)


def test_plan_option_validation():
    c = _circ([([0], [], X)])
    with pytest.raises(qsv.QsvError) as e:
        qsv.plan_describe(c, 8, opts=qsv.fuse_opts(strategy=9))
    assert e.value.status == qsv.QSV_ERR_UNSUPPORTED
    for kw in (dict(tile_log2=20), dict(k_max=7), dict(reg_log2=2),
               dict(reg_log2=6), dict(tile_log2=13, reg_log2=3)):
        with pytest.raises(qsv.QsvError) as e:
            qsv.plan_describe(c, 8, opts=qsv.fuse_opts(**kw))
        assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    with pytest.raises(qsv.QsvError) as e:
        qsv.plan_describe(c, 8, prec=7)
    assert e.value.status == qsv.QSV_ERR_UNSUPPORTED


def test_plan_program_stats_diagonal_flops():
    # CZ multiplies the quarter of the amplitudes with both bits 1; a
    # general one-qubit diagonal multiplies every amplitude (6 flops each)
    Z = np.diag([1, -1]).astype(complex)
    rz = np.diag([np.exp(-0.3j), np.exp(0.3j)])
    opts = qsv.fuse_opts(strategy=qsv.PLAN_TILED)
    st = qsv.plan_program_stats(_circ([([1], [0], Z)]), 8, qsv.QSV_C64, opts)
    assert st["tile_flops"] == 6 * 64
    st = qsv.plan_program_stats(_circ([([2], [], rz)]), 8, qsv.QSV_C64, opts)
    assert st["tile_flops"] == 6 * 256


def test_plan_program_stats_validation():
    c = _circ([([0], [], X), ([1], [0], X)])
    st = qsv.plan_program_stats(c, 8, qsv.QSV_C64,
                                qsv.fuse_opts(strategy=qsv.PLAN_TILED))
    assert st["passes"] == 1 and st["tile_passes"] == 1
    assert st["tile_ops"] >= 1 and st["phase_blocks"] == 0
    # X changes every amplitude, CX the half whose control is 1: one 2x2
    # complex row each (14 flops)
    assert st["tile_flops"] == 14 * 256 + 14 * 128
    with pytest.raises(qsv.QsvError) as e:
        qsv.plan_program_stats(c, 8, prec=7)
    assert e.value.status == qsv.QSV_ERR_UNSUPPORTED
    for n in (0, 35):
        with pytest.raises(qsv.QsvError) as e:
            qsv.plan_program_stats(c, n)
        assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    out = np.zeros(8, np.uint64)
    import ctypes as C
    st = c.struct()
    assert qsv._lib.qsv_plan_program_stats(
        C.byref(st), 8, qsv.QSV_C64, None,
        out.ctypes.data_as(C.POINTER(C.c_uint64)), 8) == qsv.QSV_ERR_INVALID_ARG
    assert qsv._lib.qsv_plan_program_stats(
        C.byref(st), 8, qsv.QSV_C64, None, None, 1) == qsv.QSV_ERR_INVALID_ARG
