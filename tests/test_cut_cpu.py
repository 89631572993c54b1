"""Cut reconstruction entry points without a GPU: specification checks and
workspace sizes (host-side validation; nothing is launched on an error)."""
import ctypes as C

import numpy as np
import pytest

from circuits import cut_chain, cut_variants
from paper_2502_11385_amd import qsv


class _Sub:
    def __init__(self, width, out_qubit, cut_in, cut_out):
        self.width, self.out_qubit = width, out_qubit
        self.cut_in, self.cut_out = cut_in, cut_out


def _ok_subs():
    return [_Sub(2, [0, -1], [-1, -1], [-1, 0]),
            _Sub(2, [1, 2], [0, -1], [-1, -1])]


def test_workspace_bytes_of_a_chain():
    prob = cut_chain((3, 4, 3), 1, 1)
    spec = qsv.CutSpec(prob.n, prob.n_cuts, prob.subs)
    nb = spec.workspace_bytes()
    # term vectors: 4^1*2^2 + 4^2*2^3 + 4^1*2^3 doubles, plus tables
    assert nb >= 8 * (16 + 128 + 32)
    assert nb < 8 * (16 + 128 + 32) + 4096 + 8 * (3 + 12 + 4) + 8 * 16 * 3


@pytest.mark.parametrize("mutate,msg", [
    (lambda s: s[1].cut_in.__setitem__(0, -1), "downstream"),
    (lambda s: s[0].out_qubit.__setitem__(1, 1), "exactly once"),
    (lambda s: s[1].out_qubit.__setitem__(1, 0), "measured twice"),
    (lambda s: s[1].out_qubit.__setitem__(1, 7), "out of range"),
    (lambda s: s[1].cut_in.__setitem__(0, 3), "out of range"),
])
def test_bad_specifications_are_rejected(mutate, msg):
    subs = _ok_subs()
    mutate(subs)
    spec = qsv.CutSpec(3, 1, subs)
    with pytest.raises(qsv.QsvError) as e:
        spec.workspace_bytes()
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    assert msg in str(e.value)


def test_same_subcircuit_cut_is_rejected():
    subs = [_Sub(3, [0, 1, -1], [-1, 0, -1], [-1, -1, 0])]
    with pytest.raises(qsv.QsvError) as e:
        qsv.CutSpec(2, 1, subs).workspace_bytes()
    assert "different subcircuits" in str(e.value)


def test_offsets_outside_the_buffer_are_rejected_before_any_launch():
    subs = _ok_subs()
    spec = qsv.CutSpec(3, 1, subs)
    nb = spec.workspace_bytes()
    off = np.array([0, 4, 8, 12, 16, 20, 24], np.uint64)   # 3 + 4 variants
    fake = 0x10000  # never dereferenced: validation fails first
    L = qsv.lib()
    st = L.qsv_cut_reconstruct(C.byref(spec._s), fake, 1, 27,
                               off.ctypes.data_as(C.POINTER(C.c_uint64)),
                               fake, nb, fake, None)
    assert st == qsv.QSV_ERR_INVALID_ARG and "outside" in qsv.last_error()
    st = L.qsv_cut_reconstruct(C.byref(spec._s), fake, 1, 28,
                               off.ctypes.data_as(C.POINTER(C.c_uint64)),
                               fake, nb - 8, fake, None)
    assert st == qsv.QSV_ERR_INVALID_ARG and "workspace" in qsv.last_error()


def test_variant_counts_follow_the_canonical_order():
    prob = cut_chain((2, 1, 3), 1, 2)
    assert [len(cut_variants(s)) for s in prob.subs] == [3, 12, 4]
