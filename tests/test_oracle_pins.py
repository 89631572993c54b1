"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Each test checks the oracle against something other than itself: textbook
special cases, closed forms (GHZ, Bernstein-Vazirani, QFT), invariants
(norm, circuit followed by its inverse), brute force over the full 2^n x 2^n
matrix, the paper's decomposition identities (eqs 3.1-3.6), its cut
reconstruction rule (eq 3.7 and the worked example of Section III.A), its
Table III, and published SplitMix64 outputs.
"""
import math
import os

import numpy as np
import pytest

import oracle
from circuits import (Gate, bv_circuit, ghz_circuit, inverse_circuit,
                      layered_circuit, qft_style_circuit, random_state)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mat(name, *params):
    return oracle.gate_spec(name, (0,) if name not in ("cx", "cz", "cp")
                            else (0, 1), params)[2]


# --------------------------------------------------------------------------
# gate matrices


def test_u3_special_cases():
    # U3(pi, 0, pi) = X; U3(pi/2, 0, pi) = H; U3(0, 0, l) = P(l)
    assert np.allclose(_mat("u3", math.pi, 0, math.pi), [[0, 1], [1, 0]],
                       atol=1e-15)
    s = 1 / math.sqrt(2)
    assert np.allclose(_mat("u3", math.pi / 2, 0, math.pi),
                       [[s, s], [s, -s]], atol=1e-15)
    assert np.allclose(_mat("u3", 0, 0, 0.7), np.diag([1, np.exp(0.7j)]))
    # U3(t, -pi/2, pi/2) = RX(t) = [[c, -is], [-is, c]]
    t = 0.9
    c, sn = math.cos(t / 2), math.sin(t / 2)
    assert np.allclose(_mat("u3", t, -math.pi / 2, math.pi / 2),
                       [[c, -1j * sn], [-1j * sn, c]])


def test_fixed_gate_algebra():
    h, x, z, s, sdg = (_mat(g) for g in ("h", "x", "z", "s", "sdg"))
    y = _mat("y")
    assert np.allclose(h @ h, np.eye(2))
    assert np.allclose(s @ s, z)
    assert np.allclose(s @ sdg, np.eye(2))
    assert np.allclose(h @ z @ h, x)
    assert np.allclose(1j * x @ z, y)       # Y = iXZ
    for m in (h, x, z, s, sdg, y, _mat("u3", 1.1, 2.2, 3.3)):
        assert np.allclose(m.conj().T @ m, np.eye(2), atol=1e-15)


# --------------------------------------------------------------------------
# brute force: whole-circuit unitary built entry by entry


def _mixed_small_circuit(n, seed):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(6 * n):
        kind = rng.integers(0, 9 if n > 1 else 6)
        a, b = (int(v) for v in rng.choice(n, 2, replace=False)) \
            if n > 1 else (0, 0)
        ang = [float(v) for v in rng.uniform(0, 2 * math.pi, 3)]
        gates.append({0: Gate("u3", (a,), tuple(ang)),
                      1: Gate("h", (a,)), 2: Gate("x", (a,)),
                      3: Gate("s", (a,)), 4: Gate("sdg", (a,)),
                      5: Gate("p", (a,), (ang[0],)),
                      6: Gate("cx", (a, b)), 7: Gate("cz", (a, b)),
                      8: Gate("cp", (a, b), (ang[1],))}[int(kind)])
    return gates


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_simulate_matches_full_unitary(n):
    gates = _mixed_small_circuit(n, 100 + n)
    u = oracle.full_unitary(n, gates)
    for x in (0, (1 << n) - 1, (1 << n) // 3):
        psi = oracle.simulate(n, gates, init=x)
        assert np.max(np.abs(psi - u[:, x])) < 1e-12
    v = random_state(n, 7)
    assert np.max(np.abs(oracle.simulate(n, gates, init=v) - u @ v)) < 1e-12


def _random_unitary(dim, rng):
    z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("k,c", [(1, 0), (1, 2), (2, 0), (2, 1), (3, 0),
                                 (3, 2), (4, 1), (5, 0)])
def test_apply_gate_general_matches_embedding(k, c):
    n = 7
    rng = np.random.default_rng(10 * k + c)
    for trial in range(3):
        qs = [int(v) for v in rng.choice(n, k + c, replace=False)]
        t, ctl = qs[:k], qs[k:]
        u = _random_unitary(1 << k, rng)
        v = random_state(n, trial)
        got = oracle.apply_gate(v, n, u, t, ctl)
        want = oracle.embed(n, u, t, ctl) @ v
        assert np.max(np.abs(got - want)) < 1e-13


def test_full_unitary_n10_spot():
    # the north-star's n <= 10 brute force, on a short circuit at n = 10
    n = 10
    gates = _mixed_small_circuit(n, 5)[:12]
    u = oracle.full_unitary(n, gates)
    assert np.allclose(u.conj().T @ u, np.eye(1 << n), atol=1e-12)
    psi = oracle.simulate(n, gates, init=37)
    assert np.max(np.abs(psi - u[:, 37])) < 1e-12


def test_nontarget_amplitudes_untouched_by_controlled_gate():
    n = 5
    v = random_state(n, 3)
    u = _random_unitary(2, np.random.default_rng(0))
    out = oracle.apply_gate(v, n, u, [2], [0, 4])
    for i in range(1 << n):
        if not ((i & 1) and (i >> 4) & 1):
            assert out[i] == v[i]


# --------------------------------------------------------------------------
# closed forms


def test_ghz_12():
    n = 12
    p = oracle.probabilities(oracle.simulate(n, ghz_circuit(n)))
    assert abs(p[0] - 0.5) < 1e-15 and abs(p[-1] - 0.5) < 1e-15
    assert np.all(p[1:-1] == 0.0)


@pytest.mark.parametrize("secret", [[1, 0, 1, 1, 0, 1, 0, 0, 1],
                                    [0] * 6, [1] * 7])
def test_bernstein_vazirani(secret):
    m = len(secret)
    p = oracle.probabilities(oracle.simulate(m + 1, bv_circuit(secret)))
    marg = oracle.marginal(p, m + 1, list(range(m)))
    s = sum(b << i for i, b in enumerate(secret))
    assert abs(marg[s] - 1.0) < 1e-12
    assert abs(marg.sum() - 1.0) < 1e-12


def _bitrev(z, n):
    return int(format(z, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("n,x", [(3, 5), (6, 41), (8, 200)])
def test_qft_ladder_closed_form(n, x):
    _, gates = qft_style_circuit(n, seed=1, tail_layers=0)
    psi = oracle.simulate(n, gates, init=x)
    z = np.arange(1 << n)
    rev = np.array([_bitrev(int(v), n) for v in z])
    want = np.exp(2j * math.pi * x * rev / (1 << n)) / math.sqrt(1 << n)
    assert np.max(np.abs(psi - want)) < 1e-12


# --------------------------------------------------------------------------
# invariants


def test_norm_after_every_gate_12q():
    oracle.simulate(12, layered_circuit(12, 20, seed=12), check_norm=True)


@pytest.mark.parametrize("n,x", [(10, 0), (10, 777), (9, 300)])
def test_round_trip(n, x):
    g = layered_circuit(n, 8, seed=n)
    _, q = qft_style_circuit(n, seed=3, tail_layers=2)
    g = g + q + _mixed_small_circuit(n, 9)
    psi = oracle.simulate(n, g + inverse_circuit(g), init=x)
    assert abs(abs(psi[x]) - 1.0) < 1e-12
    assert np.max(np.abs(np.delete(psi, x))) < 1e-12


# --------------------------------------------------------------------------
# reductions


def test_marginal_brute_force():
    n = 7
    p = oracle.probabilities(random_state(n, 11))
    for qubits in ([3], [0, 6], [5, 1, 2], [6, 5, 4, 3, 2, 1, 0]):
        m = len(qubits)
        want = np.zeros(1 << m)
        for i in range(1 << n):
            j = sum(((i >> q) & 1) << l for l, q in enumerate(qubits))
            want[j] += p[i]
        assert np.max(np.abs(oracle.marginal(p, n, qubits) - want)) < 1e-15
    assert np.array_equal(oracle.marginal(p, n, list(range(n))), p)


def test_norm_is_exact_sum():
    p = np.array([1e16, 1.0, -1e16, 1.0])
    psi = np.sqrt(np.abs(p)).astype(np.complex128)
    assert oracle.norm(psi) == math.fsum(np.abs(p).tolist())
    assert oracle.norm(np.full(1 << 10, 2.0 ** -5, np.complex128)) == 1.0


# --------------------------------------------------------------------------
# sampling


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        want = [int(l) for l in f if l.strip() and not l.startswith("#")]
    assert [oracle.splitmix64(1234567, j) for j in range(5)] == want


def test_uniforms_in_unit_interval():
    u = oracle.uniforms(99, 20000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    # the 53-bit grid
    assert np.all(u * 2.0 ** 53 == np.floor(u * 2.0 ** 53))


def test_sample_inverse_cdf_rule():
    p = np.array([0.25, 0.0, 0.5, 0.25])
    s = oracle.sample(p, 4000, seed=5)
    u = oracle.uniforms(5, 4000)
    want = np.where(u < 0.25, 0, np.where(u < 0.75, 2, 3))
    assert np.array_equal(s, want)
    assert not np.any(s == 1)


def test_sample_chi_square():
    n = 8
    p = oracle.probabilities(oracle.simulate(n, layered_circuit(n, 6, 2)))
    shots = 200_000
    s = oracle.sample(p, shots, seed=17)
    counts = np.bincount(s.astype(np.int64), minlength=1 << n)
    expected = shots * p
    keep = expected > 5
    chi2 = np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep])
    dof = keep.sum() - 1
    # 5-sigma bound for a chi-square with dof degrees of freedom
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_sample_ghz_only_two_outcomes():
    n = 10
    p = oracle.probabilities(oracle.simulate(n, ghz_circuit(n)))
    s = oracle.sample(p, 5000, seed=3)
    assert set(np.unique(s).tolist()) == {0, (1 << n) - 1}


# --------------------------------------------------------------------------
# cut variants: eqs 3.1-3.6 and the reconstruction rule


PAULI = {"I": np.eye(2, dtype=complex),
         "X": np.array([[0, 1], [1, 0]], dtype=complex),
         "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
         "Z": np.array([[1, 0], [0, -1]], dtype=complex)}


def _prepared(label):
    """The oracle's cut-input state |label> (from its prologue gates)."""
    return oracle.simulate(1, oracle.cut_prologue([(0, label)]))


def test_pauli_decomposition_eq_3_1():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    rec = sum(np.trace(a @ PAULI[k]) * PAULI[k] for k in "IXYZ") / 2
    assert np.allclose(rec, a)


def test_eigenbasis_decomposition_eq_3_2_with_prologue_states():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    proj = {lab: np.outer(_prepared(lab), _prepared(lab).conj())
            for lab in ("0", "1", "+", "+i")}
    tr = {k: np.trace(a @ PAULI[k]) for k in "IXYZ"}
    a1 = (tr["I"] + tr["Z"]) * proj["0"]
    a2 = (tr["I"] - tr["Z"]) * proj["1"]
    a3 = tr["X"] * (2 * proj["+"] - proj["0"] - proj["1"])
    a4 = tr["Y"] * (2 * proj["+i"] - proj["0"] - proj["1"])
    assert np.allclose((a1 + a2 + a3 + a4) / 2, a)
    # with |-> in place of |+i> (the alternative reading) the identity fails
    minus = np.array([1, -1]) / math.sqrt(2)
    a4m = tr["Y"] * (2 * np.outer(minus, minus) - proj["0"] - proj["1"])
    assert not np.allclose((a1 + a2 + a3 + a4m) / 2, a)


@pytest.mark.parametrize("basis,eig", [("X", "+"), ("Y", "+i")])
def test_epilogue_maps_plus_one_eigenstate_to_zero(basis, eig):
    psi = oracle.simulate(1, oracle.cut_prologue([(0, eig)]) +
                          oracle.cut_epilogue([(0, basis)]))
    assert abs(abs(psi[0]) - 1.0) < 1e-15


def test_cut_reconstruction_identity():
    """Cut one wire of a 4-qubit circuit and rebuild the full distribution.

    The uncut circuit is U_A on qubits (0, 1) followed by U_B on (1, 2, 3):
    wire 1 is cut between them.  Subcircuit 1 has qubits (0, 1) with qubit 1
    measured in I/X/Y; subcircuit 2 has the cut wire as its qubit 0
    (initialised in 0/1/+/+i) and original qubits 2, 3 as its qubits 1, 2.
    The rebuild follows Section III.A: shot attribution (eq 3.7) gives
    p_{1,i}, the initialisation terms give p_{2,i}, and the uncut
    probability is one half of the sum over i of their Kronecker products.
    """
    from circuits.generators import _layers, _rng
    ua = _layers(_rng(31), 2, 3, "mixed")                    # qubits 0, 1
    ub = _layers(_rng(32), 3, 3, "mixed")                    # local 0, 1, 2
    ub_full = [Gate(g.name, tuple(q + 1 for q in g.qubits), g.params)
               for g in ub]
    p_full = oracle.probabilities(oracle.simulate(4, ua + ub_full))

    def sub1(basis):
        g = ua + oracle.cut_epilogue([(1, basis)])
        return oracle.probabilities(oracle.simulate(2, g)).reshape(2, 2)

    def sub2(init):
        g = oracle.cut_prologue([(0, init)]) + ub
        return oracle.probabilities(oracle.simulate(3, g)).reshape(4, 2)

    # subcircuit 1: axis 0 = cut qubit (bit 1), axis 1 = qubit 0
    pI, pX, pY = sub1("I"), sub1("X"), sub1("Y")
    p11 = pI[0] + pI[1] + (pI[0] - pI[1])     # I and Z, same readout
    p12 = pI[0] + pI[1] - (pI[0] - pI[1])
    p13 = pX[0] - pX[1]
    p14 = pY[0] - pY[1]
    # subcircuit 2: index = (q2_local1,2 bits) * 2 + cut bit; drop the cut
    # qubit's position by summing over it (it is an input only, measured as
    # part of the output qubits of the original circuit: original qubit 1)
    q0, q1, qp, qi = sub2("0"), sub2("1"), sub2("+"), sub2("+i")
    p21, p22 = q0, q1
    p23 = 2 * qp - q0 - q1
    p24 = 2 * qi - q0 - q1
    # original index bits: q0 from sub1, q1..q3 from sub2 (local 0..2)
    rebuilt = np.zeros(16)
    for i in range(16):
        b0 = i & 1
        rest = i >> 1                 # local index of subcircuit 2
        r2, c2 = rest >> 1, rest & 1
        rebuilt[i] = 0.5 * (p11[b0] * p21[r2, c2] + p12[b0] * p22[r2, c2] +
                            p13[b0] * p23[r2, c2] + p14[b0] * p24[r2, c2])
    assert np.max(np.abs(rebuilt - p_full)) < 1e-14


@pytest.mark.parametrize("widths,depth,seed", [
    ((3, 3), 3, 11), ((3, 4, 3), 3, 12), ((2, 3, 3, 2), 2, 13),
    ((3, 1, 3), 2, 14), ((2, 1, 1, 3), 2, 15), ((5,), 4, 16)])
def test_cut_chain_reconstruction_matches_uncut(widths, depth, seed):
    """The multi-cut rebuild (every cut by the one-cut rule) from oracle
    variant vectors equals the uncut circuit's distribution."""
    from circuits import cut_chain, cut_variants
    prob = cut_chain(widths, depth, seed)
    vp = [[oracle.variant_probabilities(v) for v in cut_variants(sub)]
          for sub in prob.subs]
    rec = oracle.cut_reconstruct(prob, vp)
    full = oracle.probabilities(oracle.simulate(prob.n, prob.uncut))
    assert np.max(np.abs(rec - full)) < 1e-13


def test_cut_reconstruction_detects_wrong_variant():
    """Swapping the X- and Y-basis variants of the upstream subcircuit (or
    dropping the X/Y terms) breaks the rebuild."""
    from circuits import cut_chain, cut_variants
    prob = cut_chain((3, 3), 3, 21)
    vp = [[oracle.variant_probabilities(v) for v in cut_variants(sub)]
          for sub in prob.subs]
    full = oracle.probabilities(oracle.simulate(prob.n, prob.uncut))
    bad = [list(vp[0]), vp[1]]
    bad[0][1], bad[0][2] = vp[0][2], vp[0][1]     # X <-> Y readout
    assert np.max(np.abs(oracle.cut_reconstruct(prob, bad) - full)) > 1e-3
    flat = [list(vp[0]), vp[1]]
    flat[0][1] = flat[0][2] = np.full_like(vp[0][1], 0.25)  # no X/Y signal
    assert np.max(np.abs(oracle.cut_reconstruct(prob, flat) - full)) > 1e-3


# --------------------------------------------------------------------------
# qubit permutation


def test_permute_qubits_brute_force_and_gate_relabelling():
    n = 6
    rng = np.random.default_rng(11)
    psi = random_state(n, 11)
    for _ in range(5):
        perm = rng.permutation(n).tolist()
        got = oracle.permute_qubits(psi, n, perm)
        want = np.zeros_like(psi)
        for i in range(1 << n):
            j = 0
            for q in range(n):
                j |= ((i >> q) & 1) << perm[q]
            want[j] = psi[i]
        assert np.array_equal(got, want)
        # a gate on qubit q before relabelling acts on perm[q] after it
        u = oracle.gate_spec("u3", (2,), (0.3, 1.1, -0.4))[2]
        a = oracle.permute_qubits(oracle.apply_gate(psi, n, u, (2,)), n, perm)
        b = oracle.apply_gate(oracle.permute_qubits(psi, n, perm), n, u,
                              (perm[2],))
        assert np.max(np.abs(a - b)) < 1e-15
        inv = [0] * n
        for q in range(n):
            inv[perm[q]] = q
        assert np.array_equal(oracle.permute_qubits(got, n, inv), psi)


# --------------------------------------------------------------------------
# outputs: top-k probabilities and Pauli expectation values


def test_top_k_against_python_sort_with_ties():
    rng = np.random.default_rng(3)
    p = rng.integers(0, 7, 200) / 8.0          # many equal values
    for k in (1, 5, 37, 200):
        idx, val = oracle.top_k(p, k)
        want = sorted(range(200), key=lambda i: (-p[i], i))[:k]
        assert idx.tolist() == want
        assert val.tolist() == [p[i] for i in want]


def test_probs_of_amplitudes_rounding():
    a = np.array([0.1 + 0.7j, 1e-9 - 3e-9j], dtype=np.complex128)
    want = [(0.1 * 0.1) + (0.7 * 0.7), (1e-9 * 1e-9) + (3e-9 * 3e-9)]
    assert oracle.probs_of_amplitudes(a).tolist() == want
    a32 = a.astype(np.complex64)
    re, im = float(a32[0].real), float(a32[0].imag)
    assert oracle.probs_of_amplitudes(a32)[0] == re * re + im * im


def test_pauli_expectations_closed_forms():
    n = 4
    ghz = oracle.simulate(n, ghz_circuit(n))
    assert abs(oracle.pauli_expectation(ghz, n, {0: "Z", 3: "Z"}) - 1) < 1e-14
    assert abs(oracle.pauli_expectation(ghz, n, {0: "Z"})) < 1e-14
    assert abs(oracle.pauli_expectation(
        ghz, n, {q: "X" for q in range(n)}) - 1) < 1e-14
    # GHZ: <Y Y X X> = -1 (two Y factors give i^2 on the |1111> -> |0000> term)
    assert abs(oracle.pauli_expectation(
        ghz, n, {0: "Y", 1: "Y", 2: "X", 3: "X"}) + 1) < 1e-14
    # one qubit: the Bloch vector of a0|0> + a1|1>
    rng = np.random.default_rng(4)
    v = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    v /= np.linalg.norm(v)
    bloch = (2 * (np.conj(v[0]) * v[1]).real, 2 * (np.conj(v[0]) * v[1]).imag,
             abs(v[0]) ** 2 - abs(v[1]) ** 2)
    for lab, want in zip("XYZ", bloch):
        assert abs(oracle.pauli_expectation(v, 1, {0: lab}) - want) < 1e-14


def test_pauli_z_matches_marginal():
    n = 6
    psi = random_state(n, 8)
    for q in range(n):
        m = oracle.marginal(oracle.probabilities(psi), n, [q])
        assert abs(oracle.pauli_expectation(psi, n, {q: "Z"}) -
                   (m[0] - m[1])) < 1e-14


# --------------------------------------------------------------------------
# Table III


def test_table_iii_state_bytes():
    with open(os.path.join(GOLDEN, "table3_state_memory.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for w, printed in rows:
        gb = oracle.state_bytes(int(w)) / 1e9
        mant, _, exp = printed.partition("e")
        scale = 10.0 ** int(exp) if exp else 1.0
        decimals = len(mant.split(".")[1])
        trunc = math.floor(gb / scale * 10 ** decimals) / 10 ** decimals
        assert abs(trunc - float(mant)) < 1e-9, (w, printed, gb)
