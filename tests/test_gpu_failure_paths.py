"""Failure paths, forced from the host (no kernel is made to fault):

* an allocation failure returns QSV_ERR_OUT_OF_MEMORY and leaves no state
  behind, or leaves an existing state's amplitudes as they were;
* a failed device call turns only its own state failed (sticky), while
  other states keep working;
* a queued server request can be cancelled, and a wait can time out.
"""
import numpy as np
import pytest

from circuits import layered_circuit

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu
C64, C128 = qsv.QSV_C64, qsv.QSV_C128
X = np.array([[0, 1], [1, 0]], complex)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def _clear_injection():
    yield
    qsv.debug_inject(1, 0)
    qsv.debug_inject(2, 0)


def test_state_allocation_failure_leaves_nothing():
    qsv.debug_inject(1, 1)
    with pytest.raises(qsv.QsvError) as e:
        qsv.State(12, C64)
    assert e.value.status == qsv.QSV_ERR_OUT_OF_MEMORY
    s = qsv.State(12, C64)          # the next allocation succeeds
    s.init_basis(9)
    assert np.argmax(np.abs(s.get())) == 9
    s.free()


def test_scratch_allocation_failure_keeps_the_state():
    s = qsv.State(12, C128)
    s.init_basis(1234)
    qsv.debug_inject(1, 1)          # the norm's scratch cannot be allocated
    with pytest.raises(qsv.QsvError) as e:
        s.norm()
    assert e.value.status == qsv.QSV_ERR_OUT_OF_MEMORY
    got = s.get()
    assert got[1234] == 1 and np.count_nonzero(got) == 1
    assert s.norm() == 1.0          # and the state still works
    s.free()


def test_failed_device_call_poisons_only_its_state():
    a, b = qsv.State(10, C64), qsv.State(10, C64)
    a.init_basis(3)
    b.init_basis(5)
    qsv.debug_inject(2, 1)
    with pytest.raises(qsv.QsvError) as e:
        a.apply_gate([0], X)
    assert e.value.status == qsv.QSV_ERR_DEVICE
    qsv.debug_inject(2, 0)
    with pytest.raises(qsv.QsvError) as e:   # sticky
        a.init_basis(0)
    assert e.value.status == qsv.QSV_ERR_DEVICE
    b.apply_gate([0], X)
    got = b.get()
    assert got[4] == 1 and np.count_nonzero(got) == 1
    a.free()
    b.free()


def test_server_cancel_and_timeout():
    srv = qsv.Server(serial=True)
    # a long first request holds the device; the others wait in the queue
    t1 = srv.submit(28, qsv.Circuit.from_gates(layered_circuit(28, 30, 1)),
                    C128)
    small = qsv.Circuit.from_gates(layered_circuit(10, 5, 2))
    t2 = srv.submit(10, small, C64)
    t3 = srv.submit(10, small, C64, shots=100, seed=3)
    srv.cancel(t3)
    with pytest.raises(qsv.QsvError) as e:
        srv.wait(t2, timeout=0.0)
    assert e.value.status == qsv.QSV_ERR_TIMEOUT
    with pytest.raises(qsv.QsvError) as e:
        srv.wait(t3)
    assert e.value.status == qsv.QSV_ERR_CANCELLED
    srv.release(t3)
    p1, info1 = srv.wait(t1, copy=False)
    assert info1["status"] == 0
    p2, info2 = srv.wait(t2, timeout=60.0)
    assert abs(float(np.sum(p2, dtype=np.float64)) - 1) < 1e-5
    with pytest.raises(qsv.QsvError) as e:   # finished: nothing to cancel
        srv.cancel(t2)
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    with pytest.raises(qsv.QsvError) as e:
        srv.wait(t2, timeout=-1.0)
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    srv.release(t1)
    srv.release(t2)
    st = srv.stats()
    assert st["completed"] == 3
    srv.close()
