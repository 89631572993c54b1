"""Top-k outcomes and Pauli expectation values on the GPU against the
oracle, on seeded input states uploaded to the device (both sides read the
same amplitudes)."""
import numpy as np
import pytest

import oracle
from circuits import ghz_circuit, random_state

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu

C64, C128 = qsv.QSV_C64, qsv.QSV_C128
DT = {C64: np.complex64, C128: np.complex128}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _state(psi, prec):
    n = int(np.log2(psi.size))
    s = qsv.State(n, prec)
    s.set(psi.astype(DT[prec]))
    return s


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("n,k,seed", [(8, 1, 1), (12, 10, 2), (16, 1000, 3),
                                      (20, 65536, 4), (10, 1024, 5)])
def test_top_k_random_states(prec, n, k, seed):
    psi = random_state(n, seed).astype(DT[prec])
    s = _state(psi, prec)
    idx, p = s.top_k(k)
    s.free()
    widx, wp = oracle.top_k(oracle.probs_of_amplitudes(psi), k)
    assert idx.tolist() == widx.tolist()
    assert p.tolist() == wp.tolist()          # same FP64 evaluation


@pytest.mark.parametrize("prec", [C64, C128])
def test_top_k_ties_resolved_by_index(prec):
    n = 14
    rng = np.random.default_rng(9)
    # few distinct magnitudes: large groups of equal probabilities
    psi = (rng.integers(1, 5, 1 << n) * np.exp(1j * rng.integers(0, 4, 1 << n)
                                                * np.pi / 2)).astype(DT[prec])
    s = _state(psi, prec)
    for k in (1, 7, 3000, 1 << n):
        idx, p = s.top_k(k)
        widx, wp = oracle.top_k(oracle.probs_of_amplitudes(psi), k)
        assert idx.tolist() == widx.tolist(), k
        assert p.tolist() == wp.tolist()
    s.free()


def test_top_k_uniform_superposition():
    n = 16
    s = qsv.State(n, C128)
    s.init_basis(0)
    c = qsv.Circuit()
    for q in range(n):
        c.add_named("h", [q])
    s.apply_fused(c)
    idx, p = s.top_k(100)
    psi = s.get()
    s.free()
    widx, wp = oracle.top_k(oracle.probs_of_amplitudes(psi), 100)
    assert idx.tolist() == widx.tolist()
    assert np.allclose(p, 2.0 ** -n, rtol=1e-12, atol=0)


def test_top_k_bounds_rejected():
    s = qsv.State(6, C64)
    s.init_basis(0)
    for k in (0, 65, 1 << 20):
        with pytest.raises(qsv.QsvError) as e:
            s.top_k(k)
        assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    s.free()


TERMS = [{0: "Z"}, {3: "X"}, {1: "Y"}, {0: "X", 1: "X"}, {2: "Y", 5: "Z"},
         {0: "Y", 4: "Y"}, {0: "Y", 1: "Y", 2: "Y"}, {q: "Z" for q in range(9)},
         {1: "X", 3: "Y", 6: "Z", 8: "X"}, {}]


@pytest.mark.parametrize("prec,tol", [(C64, 2e-6), (C128, 1e-12)])
def test_pauli_expectations_random_state(prec, tol):
    n = 9
    psi = random_state(n, 12).astype(DT[prec])
    s = _state(psi, prec)
    got = s.expectation(TERMS)
    s.free()
    for term, g in zip(TERMS, got):
        want = oracle.pauli_expectation(psi.astype(np.complex128), n, term)
        assert abs(g - want) < tol, (term, g, want)


def test_pauli_expectations_ghz_closed_forms():
    n = 20
    s = qsv.State(n, C128)
    s.init_basis(0)
    s.apply_fused(qsv.Circuit.from_gates(ghz_circuit(n)))
    got = s.expectation([{0: "Z", 19: "Z"}, {q: "X" for q in range(n)},
                         {0: "Y", 1: "Y", **{q: "X" for q in range(2, n)}},
                         {5: "Z"}])
    s.free()
    assert np.allclose(got, [1.0, 1.0, -1.0, 0.0], atol=1e-12)


def test_pauli_mask_beyond_n_rejected():
    s = qsv.State(5, C64)
    s.init_basis(0)
    with pytest.raises(qsv.QsvError) as e:
        s.expectation([{7: "Z"}])
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    s.free()


@pytest.mark.parametrize("n,prec", [(34, C64), (33, C128)])
def test_outputs_at_full_width(n, prec):
    """Every output of the widest states on a state with a closed form: a
    basis state x with H on three qubits (8 outcomes of probability 1/8).
    Norm, FP32 probability vector (sampled entries), Pauli expectations
    (<Z_q> = (-1)^{x_q} off the H qubits, <X_q> = (-1)^{x_q} and <Z_q> = 0
    on them),
    top-8, marginal of the top 10 qubits and shots."""
    torch.cuda.empty_cache()
    rng = np.random.default_rng(n + 100)
    x = int(rng.integers(0, 1 << n, dtype=np.uint64))
    hq = [1, 20, n - 1]
    zq = 7
    base = x & ~sum(1 << q for q in hq)
    support = sorted(base | sum(((v >> j) & 1) << q for j, q in enumerate(hq))
                     for v in range(8))
    tol = 1e-6 if prec == C64 else 1e-12
    s = qsv.State(n, prec)
    try:
        s.init_basis(x)
        h = qsv.gate_matrix("h")
        for q in hq:
            s.apply_gate([q], h)
        assert abs(s.norm() - 1.0) < tol
        ev = s.expectation([{zq: "Z"}, {hq[1]: "X"}, {hq[1]: "Z"},
                            {hq[0]: "X", hq[2]: "X", zq: "Z"}])
        def sg(q):
            return -1.0 if (x >> q) & 1 else 1.0
        # H|b> has <X> = (-1)^b and <Z> = 0; an untouched qubit <Z> = (-1)^b
        assert np.allclose(ev, [sg(zq), sg(hq[1]), 0.0,
                                sg(hq[0]) * sg(hq[2]) * sg(zq)], atol=tol)
        idx, p = s.top_k(8)
        assert sorted(int(i) for i in idx) == support
        assert np.allclose(p, 0.125, atol=tol)
        marg = s.marginal(list(range(n - 10, n)))
        want = np.zeros(1024)
        for i in support:
            want[i >> (n - 10)] += 0.125
        assert np.max(np.abs(marg - want)) < tol
        shots = s.sample(4096, 77)
        assert set(int(v) for v in shots) <= set(support)
        probs = s.probabilities(fp64=False)
        pick = torch.tensor(support + [support[0] ^ (1 << zq), 0, (1 << n) - 1],
                            device="cuda")
        got = probs[pick].cpu().numpy().astype(np.float64)
        want = [0.125] * 8 + [0.0] + [0.125 if i in support else 0.0
                                      for i in (0, (1 << n) - 1)]
        assert np.allclose(got, want, atol=1e-7)
        del probs
    finally:
        s.free()
        torch.cuda.empty_cache()
