"""Server admission checks that need no GPU: requests larger than the HBM
budget are rejected at submission, invalid requests are refused before any
device work, and an idle server starts and stops cleanly."""
import numpy as np
import pytest

from circuits import layered_circuit
from paper_2502_11385_amd import qsv


def test_budget_reject_and_validation():
    s = qsv.Server(budget_bytes=1 << 20)          # 1 MiB budget
    small = qsv.Circuit.from_gates(layered_circuit(18, 1, 1))
    with pytest.raises(qsv.QsvError) as e:
        s.submit(18, small)                          # 2 MiB state alone
    assert e.value.status == qsv.QSV_ERR_BUDGET
    bad = qsv.Circuit().add([5], np.eye(2))
    with pytest.raises(qsv.QsvError) as e:
        s.submit(4, bad)
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    with pytest.raises(qsv.QsvError) as e:
        s.submit(40, qsv.Circuit())
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    with pytest.raises(qsv.QsvError) as e:
        s.submit(8, qsv.Circuit(), prec=5)
    assert e.value.status == qsv.QSV_ERR_UNSUPPORTED
    st = s.stats()
    assert st["rejected"] == 1 and st["submitted"] == 0
    s.close()


def test_server_options_validation():
    with pytest.raises(qsv.QsvError):
        qsv.Server(n_streams=99)
    with pytest.raises(qsv.QsvError):
        qsv.Server(small_width=40)
    qsv.Server().close()
