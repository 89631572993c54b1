"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances (absolute, per amplitude): 1e-12 for complex128, 1e-6 for
complex64, plus total-variation distance <= 1e-4 on complex64 probabilities.
Inputs are seeded random normalised states and the synthetic workloads; the
oracle computes every expected value from the same seeds.
"""
import math

import numpy as np
import pytest

import oracle
from circuits import (Gate, bv_circuit, ghz_circuit, inverse_circuit,
                      layered_circuit, qft_style_circuit, random_state)

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu

C64, C128 = qsv.QSV_C64, qsv.QSV_C128
TOL = {C64: 1e-6, C128: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _random_unitary(dim, rng):
    z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _check_amps(got, want, prec, what=""):
    err = np.max(np.abs(got.astype(np.complex128) - want))
    assert err <= TOL[prec], f"{what}: max |da| = {err:.3e}"
    if prec == C64:
        pg = np.abs(got.astype(np.complex128)) ** 2
        tv = 0.5 * np.sum(np.abs(pg - np.abs(want) ** 2))
        assert tv <= 1e-4, f"{what}: TV = {tv:.3e}"
    return err


def _state(n, prec, init):
    s = qsv.State(n, prec)
    if isinstance(init, np.ndarray):
        s.set(init)
    else:
        s.init_basis(int(init))
    return s


# ---------------------------------------------------------------- a1


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("n,x", [(1, 1), (3, 5), (10, 0), (10, 1023),
                                 (17, 99999)])
def test_init_basis(prec, n, x):
    s = _state(n, prec, x)
    want = np.zeros(1 << n, complex)
    want[x] = 1
    assert np.array_equal(s.get().astype(complex), want)
    s.free()


# ---------------------------------------------------------------- a2-a4


@pytest.mark.parametrize("prec", [C64, C128])
def test_dense_1q_every_target(prec):
    n = 13
    rng = np.random.default_rng(1)
    v = random_state(n, 2)
    s = _state(n, prec, v)
    want = v.copy()
    for t in range(n):
        u = _random_unitary(2, rng)
        s.apply_gate([t], u)
        want = oracle.apply_gate(want, n, u, [t])
    _check_amps(s.get(), want, prec, "1q sweep")


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("k,c", [(1, 1), (1, 2), (1, 3), (2, 0), (2, 1),
                                 (3, 0), (3, 2), (4, 0), (4, 1), (5, 0)])
def test_dense_k_targets_with_controls(prec, k, c):
    n = 12
    rng = np.random.default_rng(10 * k + c)
    v = random_state(n, k + c)
    s = _state(n, prec, v)
    want = v.copy()
    for trial in range(4):
        qs = [int(q) for q in rng.choice(n, k + c, replace=False)]
        if trial == 0:   # put the lowest and the highest qubit in the gate
            rest = [q for q in qs if q not in (0, n - 1)]
            qs = ([0] + rest + [n - 1])[:k + c] if k + c > 1 else [0]
        u = _random_unitary(1 << k, rng)
        s.apply_gate(qs[:k], u, qs[k:])
        want = oracle.apply_gate(want, n, u, qs[:k], qs[k:])
    _check_amps(s.get(), want, prec, f"k={k} c={c}")


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_dense_with_low_controls(prec, k):
    """Controls on the low qubits, which the complex64 kernel tests per lane
    (writing untouched amplitudes back, or not storing them), alone, mixed
    with one another and with higher controls, targets low and high,
    against the oracle."""
    n = 13
    rng = np.random.default_rng(70 + k)
    v = random_state(n, 71 + k)
    s = _state(n, prec, v)
    want = v.copy()
    control_sets = [[0], [1], [2], [3], [4], [5], [0, 3], [3, 6], [1, 2],
                    [2, 9], [3, 4], [4, 7], [0, 1, 2, 3]]
    for cs in control_sets:
        free = [q for q in range(n) if q not in cs]
        for ts in (free[:k], free[-k:],
                   [int(q) for q in rng.choice(free, k, replace=False)]):
            u = _random_unitary(1 << k, rng)
            s.apply_gate(ts, u, cs)
            want = oracle.apply_gate(want, n, u, ts, cs)
        _check_amps(s.get(), want, prec, f"k={k} controls={cs}")


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("k,c", [(2, 0), (2, 1), (2, 2), (3, 0), (3, 1)])
def test_dense_with_qubit0_in_every_target_slot(prec, k, c):
    """k = 2, 3 gates with qubit 0 as each of their targets in turn (the
    complex64 kernel moves qubit 0's adjacent amplitude pairs as one 16-byte
    access, taking qubit 0 as the lowest matrix bit: for k = 2 the host
    swaps the targets and the matrix bits when qubit 0 comes second),
    with and without controls, 14 qubits, against the oracle."""
    n = 14
    rng = np.random.default_rng(700 + 10 * k + c)
    v = random_state(n, 70 + k + c)
    s = _state(n, prec, v)
    want = v.copy()
    for slot in range(k):
        others = [int(q) for q in rng.choice(np.arange(1, n), k - 1 + c,
                                             replace=False)]
        tq = others[:k - 1]
        tq.insert(slot, 0)
        cq = others[k - 1:]
        u = _random_unitary(1 << k, rng)
        s.apply_gate(tq, u, cq)
        want = oracle.apply_gate(want, n, u, tq, cq)
    _check_amps(s.get(), want, prec, f"k={k} c={c}")
    s.free()


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("k", [4, 5])
def test_dense_k4_k5_matrix_cores_20q(prec, k):
    """Control-free 4- and 5-target gates (the matrix-core path) on 20
    qubits with targets in every order, including the lowest and highest
    qubit."""
    n = 20
    rng = np.random.default_rng(40 + k)
    v = random_state(n, 50 + k)
    s = _state(n, prec, v)
    want = v.copy()
    for trial in range(5):
        qs = [int(q) for q in rng.choice(n, k, replace=False)]
        if trial == 0:
            mid = [q for q in qs if q not in (0, n - 1)][:k - 2]
            qs = [n - 1] + mid + [0]
        u = _random_unitary(1 << k, rng)
        s.apply_gate(qs, u)
        want = oracle.apply_gate(want, n, u, qs, [])
    _check_amps(s.get(), want, prec, f"k={k}")
    s.free()


@pytest.mark.parametrize("prec", [C64, C128])
def test_diagonal_gates(prec):
    n = 11
    rng = np.random.default_rng(4)
    v = random_state(n, 5)
    s = _state(n, prec, v)
    want = v.copy()
    cases = [
        ([3], [7], np.diag([1, -1])),                   # CZ
        ([0], [10], np.diag([1, np.exp(0.3j)])),        # CP
        ([5], [], np.diag([1, 1j])),                    # S
        ([2], [], np.diag([np.exp(-0.2j), np.exp(0.2j)])),  # RZ (table)
        ([1, 9], [], np.diag(np.exp(1j * rng.uniform(0, 6, 4)))),
        ([4, 6, 8], [0], np.diag([1] * 7 + [-1])),      # masked, k=3
        ([10, 0, 5], [], np.diag(np.exp(1j * rng.uniform(0, 6, 8)))),
    ]
    for t, c, u in cases:
        s.apply_gate(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    _check_amps(s.get(), want, prec, "diagonal")


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 13])
def test_diagonal_gates_small_and_ragged(prec, n):
    """Every placement of a diagonal gate's fixed and target bits, the low
    ones tested per lane, on states smaller than one wave and on one that
    spans many work-groups."""
    rng = np.random.default_rng(40 + n)
    v = random_state(n, 41 + n)
    s = _state(n, prec, v)
    want = v.copy()
    for q in range(n):
        u = np.diag([1, np.exp(1j * rng.uniform(0, 6))])     # masked phase
        s.apply_gate([q], u)
        want = oracle.apply_gate(want, n, u, [q], [])
        u = np.diag(np.exp(1j * rng.uniform(0, 6, 2)))       # table
        s.apply_gate([q], u)
        want = oracle.apply_gate(want, n, u, [q], [])
        for c in range(n):
            if c == q:
                continue
            u = np.diag([1, -1])                               # CZ
            s.apply_gate([q], u, [c])
            want = oracle.apply_gate(want, n, u, [q], [c])
            u = np.diag(np.exp(1j * rng.uniform(0, 6, 2)))   # controlled RZ
            s.apply_gate([q], u, [c])
            want = oracle.apply_gate(want, n, u, [q], [c])
    _check_amps(s.get(), want, prec, f"diagonal n={n}")


# ---------------------------------------------------------------- a5-a8

STRATS = {
    "plain": qsv.fuse_opts(strategy=qsv.PLAN_PLAIN),
    "tiled": qsv.fuse_opts(strategy=qsv.PLAN_TILED),
    "tiled_L10_rb5": qsv.fuse_opts(strategy=qsv.PLAN_TILED, tile_log2=10,
                                   reg_log2=5, low_qubits=3),
    "tiled_L13": qsv.fuse_opts(strategy=qsv.PLAN_TILED, tile_log2=13),
    "tiled_rb3": qsv.fuse_opts(strategy=qsv.PLAN_TILED, reg_log2=3),
    "tiled_L9_rb3": qsv.fuse_opts(strategy=qsv.PLAN_TILED, tile_log2=9,
                                  reg_log2=3, low_qubits=3),
    "tiled_L8": qsv.fuse_opts(strategy=qsv.PLAN_TILED, tile_log2=8,
                              low_qubits=2),
    "fused5": qsv.fuse_opts(strategy=qsv.PLAN_FUSED, k_max=5),
    "fused4": qsv.fuse_opts(strategy=qsv.PLAN_FUSED, k_max=4),
    "fused3": qsv.fuse_opts(strategy=qsv.PLAN_FUSED, k_max=3),
    "fused2": qsv.fuse_opts(strategy=qsv.PLAN_FUSED, k_max=2),
    "auto": None,
}


def _mixed(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 9))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        ang = tuple(float(v) for v in rng.uniform(0, 2 * math.pi, 3))
        out.append([Gate("u3", (a,), ang), Gate("h", (a,)), Gate("s", (a,)),
                    Gate("p", (a,), ang[:1]), Gate("cx", (a, b)),
                    Gate("cz", (a, b)), Gate("cp", (a, b), ang[1:2]),
                    Gate("x", (a,)), Gate("sdg", (a,))][kind])
    return out


CIRCUITS = {
    "layered12": (12, lambda: layered_circuit(12, 20, 12)),
    "ghz12": (12, lambda: ghz_circuit(12)),
    "mixed14": (14, lambda: _mixed(14, 300, 7)),
    "qft15": (15, lambda: qft_style_circuit(15, 15, tail_layers=3)[1]),
    "layered17": (17, lambda: layered_circuit(17, 12, 17)),
}


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("strat", list(STRATS))
@pytest.mark.parametrize("cname", list(CIRCUITS))
def test_apply_fused_parity(prec, strat, cname):
    n, make = CIRCUITS[cname]
    gates = make()
    v = random_state(n, 21)
    s = _state(n, prec, v)
    if prec == C128 and strat == "tiled_L10_rb5":
        # 32 complex128 registers per thread do not fit the register file
        with pytest.raises(qsv.QsvError) as e:
            s.apply_fused(qsv.Circuit.from_gates(gates), STRATS[strat])
        assert e.value.status == qsv.QSV_ERR_INVALID_ARG
        return
    want = oracle.simulate(n, gates, init=v)
    s.apply_fused(qsv.Circuit.from_gates(gates), STRATS[strat])
    _check_amps(s.get(), want, prec, f"{cname}/{strat}")
    st = s.plan_stats()
    assert st["gates"] == len(gates)
    s.free()


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("strat", ["plain", "tiled", "fused5"])
def test_fused_dense_multi_qubit_gates(prec, strat):
    """Gate lists that mix 2..5-target dense gates with 1-qubit gates."""
    n = 12
    rng = np.random.default_rng(3)
    c = qsv.Circuit()
    want = random_state(n, 4)
    s = _state(n, prec, want)
    for i in range(40):
        k = int(rng.integers(1, 6)) if i % 3 == 0 else 1
        cc = int(rng.integers(0, 2)) if k <= 3 else 0
        qs = [int(q) for q in rng.choice(n, k + cc, replace=False)]
        u = _random_unitary(1 << k, rng)
        c.add(qs[:k], u, qs[k:])
        want = oracle.apply_gate(want, n, u, qs[:k], qs[k:])
    s.apply_fused(c, STRATS[strat])
    _check_amps(s.get(), want, prec, strat)


@pytest.mark.parametrize("prec", [C64, C128])
def test_empty_and_tiny(prec):
    for n in (1, 2, 5):
        v = random_state(n, n)
        s = _state(n, prec, v)
        s.apply_fused(qsv.Circuit())
        _check_amps(s.get(), v, prec, "empty")
        g = _mixed(n, 20, n) if n > 1 else [Gate("h", (0,)), Gate("s", (0,))]
        s.apply_fused(qsv.Circuit.from_gates(g))
        _check_amps(s.get(), oracle.simulate(n, g, init=v), prec, f"n={n}")


# ---------------------------------------------------------------- configs


def test_config1_12q_c128_plain_probabilities():
    n = 12
    gates = layered_circuit(12, 20, 12)
    want = oracle.probabilities(oracle.simulate(n, gates))
    s = _state(n, C128, 0)
    s.apply_fused(qsv.Circuit.from_gates(gates), STRATS["plain"])
    p = s.probabilities(fp64=True).cpu().numpy()
    assert np.max(np.abs(p - want)) <= 1e-12
    g = _state(n, C128, 0)
    g.apply_fused(qsv.Circuit.from_gates(ghz_circuit(n)), STRATS["plain"])
    pg = g.probabilities(fp64=True).cpu().numpy()
    assert abs(pg[0] - 0.5) < 1e-15 and abs(pg[-1] - 0.5) < 1e-15
    assert np.max(np.abs(pg[1:-1])) == 0.0


@pytest.fixture(scope="module")
def oracle_20q():
    gates = layered_circuit(20, 40, 30)
    return gates, oracle.simulate(20, gates)


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("strat", ["plain", "tiled", "fused5"])
def test_config2_20q_instance(oracle_20q, prec, strat):
    gates, want = oracle_20q
    s = _state(20, prec, 0)
    s.apply_fused(qsv.Circuit.from_gates(gates), STRATS[strat])
    err = _check_amps(s.get(), want, prec, strat)
    print(f"20q depth-40 {strat} prec={prec}: max|da|={err:.3e}")
    s.free()


# ---------------------------------------------------------------- a9-a11


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("n", [1, 6, 12, 15])
def test_probabilities_and_norm(prec, n):
    v = random_state(n, 30 + n)
    s = _state(n, prec, v)
    got_amps = s.get().astype(np.complex128)
    p64 = s.probabilities(fp64=True).cpu().numpy()
    p32 = s.probabilities(fp64=False).cpu().numpy()
    want = oracle.probabilities(v)
    tol = 1e-15 if prec == C128 else 2e-7
    assert np.max(np.abs(p64 - want)) <= tol * max(1.0, want.max()) + 1e-16
    assert np.max(np.abs(p32 - want)) <= 1e-6 * want.max() + 1e-12
    nv = s.norm()
    assert abs(nv - oracle.norm(v)) <= (1e-14 if prec == C128 else 1e-6)
    # the norm of the stored amplitudes, summed exactly
    assert abs(nv - oracle.norm(got_amps)) <= 1e-14
    # bitwise reproducible
    assert s.norm() == nv


@pytest.mark.parametrize("prec", [C64, C128])
def test_renormalize(prec):
    n = 10
    v = 3.0 * random_state(n, 8)
    s = _state(n, prec, v)
    before = s.renormalize()
    assert abs(before - 9.0) < 1e-5
    assert abs(s.norm() - 1.0) < (1e-14 if prec == C128 else 1e-6)


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("qubits", [[0], [13], [0, 1, 2], [13, 12, 11, 10],
                                    [3, 9, 0, 7, 12], list(range(14)),
                                    [5, 2, 11, 8, 1, 13, 0, 6, 10, 4]])
def test_marginal(prec, qubits):
    n = 14
    v = random_state(n, 41)
    s = _state(n, prec, v)
    got = s.marginal(qubits)
    want = oracle.marginal(oracle.probabilities(v), n, qubits)
    tol = 1e-14 if prec == C128 else 1e-6
    assert np.max(np.abs(got - want)) <= tol
    assert np.array_equal(s.marginal(qubits), got)   # deterministic


def test_marginal_bv():
    secret = [1, 0, 1, 1, 0, 0, 1, 0, 1, 1, 1]
    m = len(secret)
    s = _state(m + 1, C64, 0)
    s.apply_fused(qsv.Circuit.from_gates(bv_circuit(secret)))
    marg = s.marginal(list(range(m)))
    key = sum(b << i for i, b in enumerate(secret))
    assert abs(marg[key] - 1.0) < 1e-6


def _check_samples(got, p_oracle, seed, delta):
    """Index-for-index equality with the oracle except where u_j * total
    falls within delta of a CDF boundary between the two answers."""
    want = oracle.sample(p_oracle, len(got), seed)
    c = np.cumsum(p_oracle)
    t = oracle.uniforms(seed, len(got)) * c[-1]
    bad = np.nonzero(got != want)[0]
    for j in bad:
        lo, hi = sorted((int(got[j]), int(want[j])))
        assert hi < len(p_oracle)
        near = np.min(np.abs(c[lo:hi] - t[j])) if hi > lo else 0.0
        assert near <= delta, (j, got[j], want[j], near)
    return len(bad)


@pytest.mark.parametrize("prec", [C64, C128])
def test_sample_matches_oracle(prec):
    n = 12
    gates = layered_circuit(n, 10, 5)
    psi = oracle.simulate(n, gates)
    p = oracle.probabilities(psi)
    s = _state(n, prec, 0)
    s.apply_fused(qsv.Circuit.from_gates(gates))
    shots, seed = 20000, 1000003
    got = s.sample(shots, seed)
    assert got.dtype == np.uint64 and got.max() < (1 << n)
    delta = 1e-9 if prec == C128 else 2e-4
    bad = _check_samples(got, p, seed, delta)
    assert bad <= (2 if prec == C128 else 20)
    assert np.array_equal(s.sample(shots, seed), got)


def test_sample_ghz_and_sparse():
    n = 16
    s = _state(n, C64, 0)
    s.apply_fused(qsv.Circuit.from_gates(ghz_circuit(n)))
    got = s.sample(5000, 7)
    assert set(np.unique(got).tolist()) == {0, (1 << n) - 1}
    b = _state(n, C128, 12345)
    assert np.all(b.sample(100, 1) == 12345)
    for m in (1, 3, 7):
        t = _state(m, C64, (1 << m) - 1)
        assert np.all(t.sample(64, 2) == (1 << m) - 1)


def test_sample_chi_square_20q(oracle_20q):
    gates, psi = oracle_20q
    p = oracle.probabilities(psi)
    s = _state(20, C64, 0)
    s.apply_fused(qsv.Circuit.from_gates(gates))
    shots = 400_000
    got = s.sample(shots, 99)
    hi = (got >> np.uint64(14)).astype(np.int64)     # top 6 qubits
    counts = np.bincount(hi, minlength=64)
    expect = shots * oracle.marginal(p, 20, list(range(14, 20)))
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < 63 + 5 * math.sqrt(2 * 63)


# ---------------------------------------------------------------- full width


@pytest.mark.parametrize("prec", [C64, C128])
def test_round_trip_30q(prec):
    """30-qubit depth-40 circuit then its inverse returns |x> (tiled plan)."""
    n, x = 30, 123456789
    gates = layered_circuit(n, 40, 30)
    s = _state(n, prec, x)
    circ = qsv.Circuit.from_gates(gates + inverse_circuit(gates))
    s.apply_fused(circ, STRATS["tiled"])
    nv = s.norm()
    marg = s.marginal(list(range(n - 10, n)))
    tol = 1e-4 if prec == C64 else 1e-10
    assert abs(nv - 1.0) < tol
    assert abs(marg[x >> (n - 10)] - 1.0) < tol
    low = s.marginal(list(range(10)))
    assert abs(low[x & 1023] - 1.0) < tol
    mid = s.marginal(list(range(10, 20)))
    assert abs(mid[(x >> 10) & 1023] - 1.0) < tol
    s.free()


@pytest.mark.parametrize("n,prec", [(30, C64), (30, C128), (33, C128),
                                    (34, C64)])
def test_qft_closed_form_full_width(n, prec):
    """QFT ladder on |x> at full width against the closed form
    psi[z] = 2^(-n/2) exp(2 pi i x rev_n(z) / 2^n) on sampled z."""
    x, gates = qft_style_circuit(n, n, tail_layers=0)
    dt = torch.complex64 if prec == C64 else torch.complex128
    buf = torch.empty(1 << n, dtype=dt, device="cuda")
    s = qsv.State(n, prec, tensor=buf)
    s.init_basis(x)
    s.apply_fused(qsv.Circuit.from_gates(gates))
    s.sync()
    rng = np.random.default_rng(n)
    z = rng.integers(0, 1 << n, size=4096, dtype=np.int64)
    got = buf[torch.from_numpy(z).cuda()].cpu().numpy().astype(np.complex128)
    rev = np.array([int(format(int(v), f"0{n}b")[::-1], 2) for v in z],
                   dtype=object)
    ph = np.array([((x * int(r)) % (1 << n)) / (1 << n) for r in rev],
                  dtype=np.float64)
    want = np.exp(2j * math.pi * ph) / math.sqrt(1 << n)
    # relative to the amplitudes' size 2^(-n/2) (7.6e-6 at 34 qubits)
    tol = (1e-4 if prec == C64 else 1e-10) / math.sqrt(1 << n)
    err = np.max(np.abs(got - want))
    assert err <= tol, f"max |da| = {err:.3e}, bound {tol:.3e}"
    s.free()
    del buf
    torch.cuda.empty_cache()


def test_c64_vs_c128_30q_depth40():
    """Full-size workload in the benchmark's launch configuration: complex64
    against complex128 on the GPU (labelled GPU-vs-GPU), via the top-10
    marginal, plus norms."""
    n = 30
    gates = layered_circuit(n, 40, 30)
    circ = qsv.Circuit.from_gates(gates)
    res = {}
    for prec in (C64, C128):
        s = _state(n, prec, 0)
        s.apply_fused(circ, STRATS["tiled"])
        res[prec] = (s.marginal(list(range(20, 30))), s.norm())
        s.free()
    m64, n64 = res[C64]
    m128, n128 = res[C128]
    assert abs(n128 - 1.0) < 1e-10 and abs(n64 - 1.0) < 1e-4
    assert 0.5 * np.sum(np.abs(m64 - m128)) < 1e-4
