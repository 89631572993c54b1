"""Batch API validation on the host (no GPU needed): bad variants are
rejected before any device call."""
import ctypes as C

import numpy as np
import pytest

from circuits import BatchCircuit, Gate, batch_variants
from paper_2502_11385_amd import qsv


def _try(variants, **kw):
    with pytest.raises(qsv.QsvError) as e:
        qsv.Batch(variants, **kw)
    return e.value


def test_rejects_bad_variants():
    good = batch_variants(2, seed=1, wmin=8, wmax=9, dmin=2, dmax=3)
    bad_w = [BatchCircuit(3, 1, [Gate("h", (0,))])]
    assert _try(bad_w).status == qsv.QSV_ERR_INVALID_ARG
    bad_q = [BatchCircuit(8, 1, [Gate("h", (9,))])]
    assert "out of range" in str(_try(bad_q))
    dup = [BatchCircuit(8, 1, [Gate("h", (0,))], [(1, "0"), (1, "+")])]
    assert "duplicate" in str(_try(dup))
    badlab = [BatchCircuit(8, 1, [Gate("h", (0,))], [], [(2, "Z")])]
    with pytest.raises(KeyError):
        qsv.Batch(badlab)
    assert _try(good, tile_log2=14).status == qsv.QSV_ERR_INVALID_ARG
    assert _try(good, reg_log2=5, prec=qsv.QSV_C128).status == \
        qsv.QSV_ERR_INVALID_ARG
    assert _try(good, prec=9).status == qsv.QSV_ERR_UNSUPPORTED


def test_empty_batch_rejected():
    h = C.c_void_p()
    assert qsv.lib().qsv_batch_create(None, 0, 1, None, None,
                                      C.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert qsv.lib().qsv_batch_free(None) == qsv.QSV_OK
