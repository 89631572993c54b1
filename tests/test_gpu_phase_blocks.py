"""Phase blocks on the GPU: diagonal-heavy programs run by the tile kernel
(runs of diagonal gates applied as one phase polynomial) against the
oracle applying every gate in order.

Tolerances as for every amplitude parity test: 1e-12 (complex128) and
1e-6 (complex64) absolute per amplitude."""
import numpy as np
import pytest

import oracle
from circuits import qft_style_circuit, random_state
from diag_programs import diagonal_heavy

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu

C64, C128 = qsv.QSV_C64, qsv.QSV_C128
TOL = {C64: 1e-6, C128: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


OPTS = {
    "L8": dict(strategy=qsv.PLAN_TILED, tile_log2=8, low_qubits=2),
    "L10_rb3": dict(strategy=qsv.PLAN_TILED, tile_log2=10, low_qubits=3,
                    reg_log2=3),
    "L9_rb5": dict(strategy=qsv.PLAN_TILED, tile_log2=9, reg_log2=5),
    "default": dict(strategy=qsv.PLAN_TILED),
}


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("oname", list(OPTS))
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_diagonal_heavy_programs(prec, oname, seed):
    if prec == C128 and oname == "L9_rb5":
        pytest.skip("reg_log2 = 5 is complex64 only")
    n = 14
    gl = diagonal_heavy(n, 400, 300 + seed)
    circ = qsv.Circuit()
    want = random_state(n, 40 + seed)
    v = want.copy()
    for u, t, c in gl:
        circ.add(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    opts = qsv.fuse_opts(**OPTS[oname])
    s = qsv.State(n, prec)
    s.set(v)
    s.apply_fused(circ, opts)
    got = s.get().astype(np.complex128)
    st = s.plan_stats()
    s.free()
    err = np.max(np.abs(got - want))
    assert err <= TOL[prec], f"max |da| = {err:.3e}"
    assert st["phase_blocks"] > 0 and st["block_gates"] > 100


@pytest.mark.parametrize("prec", [C64, C128])
def test_qft_ladder_blocks_20q(prec):
    """QFT ladder plus tail layers at 20 qubits (several tiles, outer
    qubits in most terms) against the oracle."""
    n = 20
    x, gates = qft_style_circuit(n, 11, tail_layers=2)
    want = oracle.simulate(n, gates, init=x)
    s = qsv.State(n, prec)
    s.init_basis(x)
    s.apply_fused(qsv.Circuit.from_gates(gates))
    got = s.get().astype(np.complex128)
    st = s.plan_stats()
    s.free()
    err = np.max(np.abs(got - want))
    assert err <= TOL[prec], f"max |da| = {err:.3e}"
    assert st["block_gates"] > 100
