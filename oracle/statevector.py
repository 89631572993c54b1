"""Plain complex128 state-vector oracle (NumPy).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

What it computes, and where the paper defines it:

* The state is the 2^n complex amplitude vector that full-circuit execution
  stores (Section III.B, "single or double precision complex numbers");
  here always complex128.  Index convention: little-endian, bit q of the
  index is the value of qubit q (the convention of the probability vector the
  evaluator returns, Section IV.A, Evaluator).
* A gate with matrix U (2^k x 2^k, row index r = sum_j bit_j(r) 2^j over the
  targets t_0..t_{k-1}) and controls C acts on every coset where all control
  bits are 1: psi'[i_r] = sum_s U[r, s] psi[i_s]; all other amplitudes are
  unchanged.
* The output is the probability vector p_i = |psi_i|^2 (Section IV.A,
  Evaluator), marginals over specified qubits (Builder and Verifier), and
  shots drawn from p (Section III.A, shot attribution).
* Cut variants: inputs initialised in {|0>, |1>, |+>, |+i>} and outputs
  measured in the I, X or Y basis, the eigenbasis terms of eqs 3.2-3.6.

Gate matrices are the textbook ones; u3 is the OpenQASM 2 / Qiskit U3, which
the paper uses (u1/u3 in the cache-blocking example, Section III.B) without
defining it.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

_S2 = 1.0 / math.sqrt(2.0)

# ---------------------------------------------------------------------------
# Gate definitions (names as produced by ``circuits.generators``)


def _u3(theta: float, phi: float, lam: float) -> np.ndarray:
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
                    dtype=np.complex128)


def _phase(lam: float) -> np.ndarray:
    return np.array([[1.0, 0.0], [0.0, np.exp(1j * lam)]], dtype=np.complex128)


_FIXED = {
    "h": np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128),
    "x": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "s": np.array([[1, 0], [0, 1j]], dtype=np.complex128),
    "sdg": np.array([[1, 0], [0, -1j]], dtype=np.complex128),
}


def gate_spec(name: str, qubits: Sequence[int], params: Sequence[float] = ()
              ) -> Tuple[Tuple[int, ...], Tuple[int, ...], np.ndarray]:
    """(targets, controls, matrix) of a named gate.

    cx(c, t) is X on t controlled by c; cz(a, b) is Z on b controlled by a;
    cp(a, b; l) is P(l) on b controlled by a (CZ and CP are symmetric).
    """
    if name in _FIXED:
        return (qubits[0],), (), _FIXED[name]
    if name == "u3":
        return (qubits[0],), (), _u3(*params)
    if name == "p":
        return (qubits[0],), (), _phase(params[0])
    if name == "cx":
        return (qubits[1],), (qubits[0],), _FIXED["x"]
    if name == "cz":
        return (qubits[1],), (qubits[0],), _FIXED["z"]
    if name == "cp":
        return (qubits[1],), (qubits[0],), _phase(params[0])
    raise ValueError(f"unknown gate {name!r}")


# ---------------------------------------------------------------------------
# Gate application


def apply_gate(psi: np.ndarray, n: int, u: np.ndarray,
               targets: Sequence[int], controls: Sequence[int] = ()) -> np.ndarray:
    """Return U (controlled on ``controls``) applied to ``targets`` of psi.

    psi is viewed as an n-axis tensor of shape (2,)*n in C order, so axis
    n-1-q holds qubit q.  The control-satisfied slice is selected with index
    1 on every control axis, and U is contracted with the target axes.
    """
    k = len(targets)
    if u.shape != (1 << k, 1 << k):
        raise ValueError("matrix shape does not match the number of targets")
    qs = list(targets) + list(controls)
    if len(set(qs)) != len(qs) or any(q < 0 or q >= n for q in qs):
        raise ValueError("bad qubit list")
    t = psi.reshape((2,) * n).copy()
    idx = [slice(None)] * n
    for c in controls:
        idx[n - 1 - c] = 1
    idx = tuple(idx)
    sub = t[idx]                                   # axes: remaining qubits
    # axis positions of the targets inside ``sub``
    remaining = [a for a in range(n) if a not in {n - 1 - c for c in controls}]
    tax = [remaining.index(n - 1 - q) for q in targets]
    # U as a tensor: axes (r_{k-1}, .., r_0, s_{k-1}, .., s_0)
    ut = u.reshape((2,) * (2 * k))
    s_axes = list(range(2 * k - 1, k - 1, -1))     # s_0 .. s_{k-1}
    out = np.tensordot(ut, sub, axes=(s_axes, tax))
    # out axes: r_{k-1}..r_0 followed by the non-target axes of sub in order;
    # output axis a holds r_{k-1-a}, which belongs at target (k-1-a)'s axis.
    src = list(range(k))
    dst = [tax[k - 1 - a] for a in range(k)]
    t[idx] = np.moveaxis(out, src, dst)
    return t.reshape(-1)


def _initial(n: int, init) -> np.ndarray:
    if init is None:
        init = 0
    if isinstance(init, (int, np.integer)):
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[int(init)] = 1.0
        return psi
    psi = np.array(init, dtype=np.complex128).reshape(-1)
    if psi.size != 1 << n:
        raise ValueError("initial state has the wrong length")
    return psi.copy()


def simulate(n: int, gates: Iterable, init=0, check_norm: bool = False
             ) -> np.ndarray:
    """Apply a gate list (``circuits.Gate`` records) to |init> (or a vector)."""
    psi = _initial(n, init)
    for g in gates:
        targets, controls, u = gate_spec(g.name, g.qubits, g.params)
        psi = apply_gate(psi, n, u, targets, controls)
        if check_norm:
            nv = norm(psi)
            if abs(nv - 1.0) > 1e-12:
                raise AssertionError(f"norm {nv!r} after gate {g}")
    return psi


# ---------------------------------------------------------------------------
# Reductions


def probabilities(psi: np.ndarray) -> np.ndarray:
    """p_i = |psi_i|^2 in float64."""
    return psi.real * psi.real + psi.imag * psi.imag


def norm(psi: np.ndarray) -> float:
    """Sum of p_i, exactly rounded (math.fsum)."""
    return math.fsum(probabilities(psi).tolist())


def marginal(p: np.ndarray, n: int, qubits: Sequence[int]) -> np.ndarray:
    """P[j] = sum of p_i over i whose bit qubits[l] equals bit l of j.

    qubits[0] is the least significant bit of j.  The sum over the other
    qubits is taken with NumPy's sum over tensor axes.
    """
    m = len(qubits)
    if len(set(qubits)) != m or any(q < 0 or q >= n for q in qubits):
        raise ValueError("bad qubit list")
    t = p.reshape((2,) * n)
    keep_axes = [n - 1 - q for q in qubits]
    drop = tuple(a for a in range(n) if a not in keep_axes)
    red = t.sum(axis=drop) if drop else t
    # remaining axes are in increasing axis order; reorder so that the axis
    # of qubits[m-1] comes first (most significant) and qubits[0] last.
    order_now = sorted(keep_axes)
    want = [n - 1 - q for q in reversed(qubits)]
    red = np.transpose(red, [order_now.index(a) for a in want])
    return np.ascontiguousarray(red).reshape(-1)


# ---------------------------------------------------------------------------
# Brute force: the full 2^n x 2^n unitary, entry by entry (small n only)


def embed(n: int, u: np.ndarray, targets: Sequence[int],
          controls: Sequence[int] = ()) -> np.ndarray:
    """The full 2^n x 2^n matrix of one (controlled) gate, entry by entry.

    Entry (i, j) is U[r(i), r(j)] when i and j agree on every non-target bit
    and all control bits of j are 1 (r(.) reads the target bits, targets[0]
    least significant); it is delta(i, j) when some control bit of j is 0;
    and 0 otherwise.  This construction is independent of ``apply_gate``'s
    tensor contraction.
    """
    dim = 1 << n
    tmask = sum(1 << q for q in targets)
    cmask = sum(1 << q for q in controls)
    idx = np.arange(dim, dtype=np.int64)
    r = np.zeros(dim, dtype=np.int64)
    for b, q in enumerate(targets):
        r |= ((idx >> q) & 1) << b
    i = idx[:, None]
    j = idx[None, :]
    same_rest = (i & ~tmask) == (j & ~tmask)
    ctrl_on = (j & cmask) == cmask
    e = np.where(same_rest & ctrl_on, u[r[:, None], r[None, :]], 0.0)
    e = e + np.where(~ctrl_on & (i == j), 1.0, 0.0)
    return e.astype(np.complex128)


def full_unitary(n: int, gates: Iterable) -> np.ndarray:
    """Product of the gates' embedded 2^n x 2^n matrices (small n only).

    Each item is a ``circuits.Gate`` or a (matrix, targets, controls) triple.
    """
    total = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        if isinstance(g, tuple):
            u, targets, controls = g
        else:
            targets, controls, u = gate_spec(g.name, g.qubits, g.params)
        total = embed(n, np.asarray(u, dtype=np.complex128), targets,
                      controls) @ total
    return total


# ---------------------------------------------------------------------------
# Sampling (Steele, Lea & Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014: the SplitMix64 output function)

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, j: int) -> int:
    """Output number j (0-based) of the SplitMix64 stream started at seed."""
    z = (seed + (j + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniforms(seed: int, count: int) -> np.ndarray:
    """u_j = (splitmix64(seed, j) >> 11) * 2^-53 for j = 0..count-1."""
    return np.array([(splitmix64(seed, j) >> 11) * 2.0 ** -53
                     for j in range(count)], dtype=np.float64)


def sample(p: np.ndarray, shots: int, seed: int) -> np.ndarray:
    """Draw j: the least i with C(i) > u_j * C(2^n - 1), C = cumsum(p)."""
    c = np.cumsum(p)
    t = uniforms(seed, shots) * c[-1]
    return np.searchsorted(c, t, side="right").astype(np.uint64)


def permute_qubits(psi: np.ndarray, n: int, perm) -> np.ndarray:
    """Relabel qubits: qubit q becomes qubit perm[q], i.e. the amplitude of
    index i moves to the index whose bit perm[q] is bit q of i."""
    t = np.asarray(psi).reshape((2,) * n)
    # axis n-1-q holds qubit q; new axis n-1-perm[q] must hold old qubit q
    src_axis_for_new = [0] * n
    for q in range(n):
        src_axis_for_new[n - 1 - perm[q]] = n - 1 - q
    return np.transpose(t, src_axis_for_new).reshape(-1).copy()


def top_k(p: np.ndarray, k: int):
    """The k largest entries of p: (indices, values), by value descending and
    by index ascending among equal values."""
    p = np.asarray(p, dtype=np.float64)
    order = np.lexsort((np.arange(p.size), -p))[:k]
    return order.astype(np.uint64), p[order]


def probs_of_amplitudes(psi: np.ndarray) -> np.ndarray:
    """|a|^2 as re*re + im*im, each product and the sum rounded separately
    in FP64 (the key on which a top-k selection decides)."""
    re = np.real(psi).astype(np.float64)
    im = np.imag(psi).astype(np.float64)
    return re * re + im * im


def pauli_expectation(psi: np.ndarray, n: int, paulis) -> float:
    """<psi| P |psi> for P = product over {qubit: 'X' | 'Y' | 'Z'}, by
    applying P's one-qubit matrices to a copy of psi."""
    mats = {"X": np.array([[0, 1], [1, 0]], dtype=complex),
            "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
            "Z": np.array([[1, 0], [0, -1]], dtype=complex)}
    phi = np.asarray(psi, dtype=complex).copy()
    for q, lab in paulis.items():
        phi = apply_gate(phi, n, mats[lab], (q,))
    return float(np.vdot(psi, phi).real)


# ---------------------------------------------------------------------------
# Cut variants (Section III.A, eqs 3.2-3.6)


def cut_prologue(inputs: Sequence[Tuple[int, str]]) -> List:
    """Gates preparing cut-input qubits in |0>, |1>, |+> or |+i>.

    |1> = X|0>, |+> = H|0>, |+i> = (|0> + i|1>)/sqrt 2 = S H |0>.
    """
    from circuits.generators import Gate
    out = []
    for q, lab in inputs:
        if lab == "0":
            continue
        if lab == "1":
            out.append(Gate("x", (q,)))
        elif lab == "+":
            out.append(Gate("h", (q,)))
        elif lab == "+i":
            out += [Gate("h", (q,)), Gate("s", (q,))]
        else:
            raise ValueError(lab)
    return out


def cut_epilogue(outputs: Sequence[Tuple[int, str]]) -> List:
    """Basis rotations before a computational-basis readout.

    I (and Z): nothing.  X: H, which maps |+> to |0>.  Y: S-dagger then H,
    which maps |+i> to |0>.
    """
    from circuits.generators import Gate
    out = []
    for q, lab in outputs:
        if lab == "I":
            continue
        if lab == "X":
            out.append(Gate("h", (q,)))
        elif lab == "Y":
            out += [Gate("sdg", (q,)), Gate("h", (q,))]
        else:
            raise ValueError(lab)
    return out


def variant_probabilities(circ) -> np.ndarray:
    """Probability vector of one ``circuits.BatchCircuit`` variant."""
    gates = cut_prologue(circ.cut_inputs) + list(circ.gates) + \
        cut_epilogue(circ.cut_outputs)
    return probabilities(simulate(circ.width, gates))


def cut_term_vectors(sub, variant_probs) -> dict:
    """The per-term vectors of one subcircuit (Section III.A).

    ``variant_probs[v]`` is the probability vector of variant v in the
    canonical order of ``circuits.cut_variants``.  A term assigns each of the
    subcircuit's cut ends one of the four indices i = 1..4 of the one-cut
    identity (written 0..3 here):

    * downstream end (the cut's initialised qubit): p_{2,1} = p(|0>),
      p_{2,2} = p(|1>), p_{2,3} = 2 p(|+>) - p(|0>) - p(|1>),
      p_{2,4} = 2 p(|+i>) - p(|0>) - p(|1>)  (eqs 3.3-3.6);
    * upstream end (the cut's measured qubit), by shot attribution (eq 3.7):
      p_{1,1} = I + Z and p_{1,2} = I - Z from the I-basis readout, p_{1,3}
      = X and p_{1,4} = Y from the X and Y readouts, where I sums both
      outcomes and Z, X, Y weigh outcome 1 by -1.

    Returns {term tuple over the ends (canonical end order): vector over the
    subcircuit's output qubits, bit i = i-th output qubit in local order}.
    """
    import itertools
    w = sub.width
    ends = []
    for j in range(w):
        if sub.cut_in[j] >= 0:
            ends.append(("in", j))
        if sub.cut_out[j] >= 0:
            ends.append(("out", j))
    radix = [4 if k == "in" else 3 for k, _ in ends]
    outs = [j for j in range(w) if sub.out_qubit[j] >= 0]
    init_mix = {0: [(0, 1.0)], 1: [(1, 1.0)],
                2: [(2, 2.0), (0, -1.0), (1, -1.0)],
                3: [(3, 2.0), (0, -1.0), (1, -1.0)]}
    basis_of = {0: 0, 1: 0, 2: 1, 3: 2}             # I, I, X, Y
    weight = {0: (2.0, 0.0), 1: (0.0, 2.0), 2: (1.0, -1.0), 3: (1.0, -1.0)}
    result = {}
    for t in itertools.product(range(4), repeat=len(ends)):
        # expand the initialisation mixtures into (variant digits, coef)
        choices = []
        for (kind, j), ti in zip(ends, t):
            choices.append(init_mix[ti] if kind == "in"
                           else [(basis_of[ti], 1.0)])
        acc = np.zeros(1 << len(outs))
        for combo in itertools.product(*choices):
            v, mult, coef = 0, 1, 1.0
            for (digit, c), r in zip(combo, radix):
                v += digit * mult
                mult *= r
                coef *= c
            # (2,)*w tensor, axis w-1-j <-> local qubit j
            tens = np.asarray(variant_probs[v], dtype=np.float64).reshape(
                (2,) * w)
            for (kind, j), ti in zip(ends, t):
                if kind == "out":
                    wv = np.zeros((2,) * w)
                    sl0 = [slice(None)] * w
                    sl1 = [slice(None)] * w
                    sl0[w - 1 - j] = 0
                    sl1[w - 1 - j] = 1
                    wv[tuple(sl0)] = weight[ti][0]
                    wv[tuple(sl1)] = weight[ti][1]
                    tens = tens * wv
            # sum out the measured cut qubits, keep outputs
            summed = [w - 1 - j for kind, j in ends if kind == "out"]
            red = tens.sum(axis=tuple(summed)) if summed else tens
            # remaining axes are the outputs in descending local order
            acc += coef * red.reshape(-1)
        result[t] = acc
    return result


def cut_reconstruct(problem, variant_probs) -> np.ndarray:
    """Probability vector of the uncut circuit from its subcircuits' variants.

    p(x) = (1/2)^K sum over term assignments (i_1..i_K) of the product over
    subcircuits of their term vectors at x's bits (Section III.A, the one-cut
    rule applied to every cut).  ``variant_probs[s][v]`` as in
    ``cut_term_vectors``.
    """
    import itertools
    n, K = problem.n, problem.n_cuts
    x = np.arange(1 << n, dtype=np.int64)
    per_sub = []
    for s, sub in enumerate(problem.subs):
        terms = cut_term_vectors(sub, variant_probs[s])
        ends = []
        for j in range(sub.width):
            if sub.cut_in[j] >= 0:
                ends.append(sub.cut_in[j])
            if sub.cut_out[j] >= 0:
                ends.append(sub.cut_out[j])
        outs = [sub.out_qubit[j] for j in range(sub.width)
                if sub.out_qubit[j] >= 0]
        y = np.zeros_like(x)
        for i, q in enumerate(outs):
            y |= ((x >> q) & 1) << i
        per_sub.append((ends, terms, y))
    p = np.zeros(1 << n)
    for tk in itertools.product(range(4), repeat=K):
        prod = np.ones(1 << n)
        for ends, terms, y in per_sub:
            prod = prod * terms[tuple(tk[c] for c in ends)][y]
        p += prod
    return p * 0.5 ** K


# ---------------------------------------------------------------------------


def state_bytes(n: int, bytes_per_amplitude: int = 16) -> int:
    """Bytes of a 2^n-amplitude state (Table III uses 16 B complex128)."""
    return bytes_per_amplitude << n
