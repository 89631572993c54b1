"""Randomised parity sweep: seeded random gate lists of every form the
library accepts (dense 1..5-target unitaries with 0..2 controls, unitary
diagonals on 1..5 qubits with and without controls, masked phases,
non-unitary diagonals), random plan options within the documented ranges,
both precisions, against the oracle applying every gate in order.

Tolerances: 1e-12 (complex128) and 1e-6 (complex64) absolute per
amplitude."""
import numpy as np
import pytest

import oracle
from circuits import random_state
from diag_programs import random_gates, random_opts

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu

C64, C128 = qsv.QSV_C64, qsv.QSV_C128
TOL = {C64: 1e-6, C128: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("seed", range(96))
def test_random_program(seed):
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(6, 17))
    prec = C64 if seed % 2 == 0 else C128
    gl = random_gates(n, int(rng.integers(20, 160)), rng)
    o = random_opts(rng, prec == C128)
    circ = qsv.Circuit()
    want = random_state(n, seed)
    v = want.copy()
    for u, t, c in gl:
        circ.add(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    s = qsv.State(n, prec)
    s.set(v)
    s.apply_fused(circ, qsv.fuse_opts(**o))
    got = s.get().astype(np.complex128)
    s.free()
    # non-unitary diagonals can grow the amplitudes: compare relative to the
    # largest expected magnitude
    scale = max(1.0, float(np.max(np.abs(want))))
    err = float(np.max(np.abs(got - want))) / scale
    assert err <= TOL[prec], f"n={n} prec={prec} opts={o}: {err:.3e}"
