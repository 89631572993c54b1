"""Seeded gate-list generators for the synthetic workloads.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in a fixed,
documented order so that the oracle and the HIP path see identical inputs.

Gate records use these names (qubit tuples in the order shown):

  ``h(q)``, ``x(q)``, ``s(q)``, ``sdg(q)``, ``p(q; lam)``,
  ``u3(q; theta, phi, lam)``, ``cx(control, target)``, ``cz(a, b)``,
  ``cp(a, b; lam)``.

The paper's benchmark suites (Adder, AQFT, BV, HWEA, Supremacy; Section V.B)
are not reproduced; these circuits only take their shapes: widths 10-34,
sparse layered structure, subcircuit widths of the order of Tables I-II,
and thousands of cut variants per run (4^K growth, Section VI).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _brick_pairs(n: int, layer: int) -> List[Tuple[int, int]]:
    """Nearest-neighbour pairs (i, i+1), i = layer % 2, layer % 2 + 2, ..."""
    return [(i, i + 1) for i in range(layer % 2, n - 1, 2)]


def _layers(rng: np.random.Generator, n: int, depth: int,
            entangler: str = "cz") -> List[Gate]:
    """``depth`` layers: U3 on every qubit, then a brick wall of 2-qubit gates.

    Angles are drawn as one array of shape (depth, n, 3), i.e. in
    (layer, qubit, theta -> phi -> lambda) order, uniform on [0, 2 pi).
    With ``entangler == "mixed"`` each pair is CZ or CNOT with probability 1/2;
    those coin flips are drawn after all angles, in (layer, pair) order.
    """
    angles = rng.uniform(0.0, TWO_PI, size=(depth, n, 3))
    coins = None
    if entangler == "mixed":
        n_pairs = sum(len(_brick_pairs(n, l)) for l in range(depth))
        coins = rng.integers(0, 2, size=n_pairs)
    gates: List[Gate] = []
    ci = 0
    for l in range(depth):
        for q in range(n):
            th, ph, la = angles[l, q]
            gates.append(Gate("u3", (q,), (float(th), float(ph), float(la))))
        for a, b in _brick_pairs(n, l):
            if entangler == "cz" or (coins is not None and coins[ci] == 0):
                gates.append(Gate("cz", (a, b)))
            else:
                gates.append(Gate("cx", (a, b)))
            ci += 1
    return gates


def layered_circuit(n: int, depth: int, seed: int) -> List[Gate]:
    """Layered random circuit: per layer U3 on all qubits then brick-wall CZ.

    Used for the 12-qubit depth-20 and the 30-qubit depth-40 workloads
    (and their 20-qubit parity instance with the same seed).
    """
    return _layers(_rng(seed), n, depth, "cz")


def ghz_circuit(n: int) -> List[Gate]:
    """H on qubit 0 then a CNOT chain q -> q+1."""
    return [Gate("h", (0,))] + [Gate("cx", (q, q + 1)) for q in range(n - 1)]


def bv_circuit(secret: Sequence[int]) -> List[Gate]:
    """Bernstein-Vazirani with data qubits 0..m-1 and ancilla m.

    ``secret[i]`` is the hidden bit for data qubit i.  The ancilla is put in
    |-> (X then H), the data register is put in |+>^m, one CNOT per set bit
    implements the oracle, and a final layer of H returns the secret.
    """
    m = len(secret)
    g = [Gate("x", (m,)), Gate("h", (m,))]
    g += [Gate("h", (q,)) for q in range(m)]
    g += [Gate("cx", (q, m)) for q in range(m) if secret[q]]
    g += [Gate("h", (q,)) for q in range(m)]
    return g


def qft_style_circuit(n: int, seed: int, tail_layers: int = 10):
    """QFT-style circuit on a random basis state.

    Draw order: first the basis index x ~ U{0 .. 2^n - 1}, then the angles of
    ``tail_layers`` U3+CZ layers.  The QFT part is, for j = n-1 down to 0:
    H(j), then CP(pi / 2^k) on (j-k, j) for k = 1..j; no final swaps.

    Returns (x, gates).
    """
    rng = _rng(seed)
    x = int(rng.integers(0, 1 << n, dtype=np.uint64))
    gates: List[Gate] = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("h", (j,)))
        for k in range(1, j + 1):
            gates.append(Gate("cp", (j - k, j), (math.pi / (1 << k),)))
    gates += _layers(rng, n, tail_layers, "cz")
    return x, gates


_SELF_INVERSE = {"h", "x", "cz", "cx"}


def inverse_circuit(gates: Sequence[Gate]) -> List[Gate]:
    """The inverse gate list: reversed order, each gate inverted.

    U3(t, p, l)^-1 = U3(-t, -l, -p); P(l)^-1 = P(-l); CP(l)^-1 = CP(-l);
    S^-1 = Sdg; H, X, CZ and CNOT are their own inverses.
    """
    out = []
    for g in reversed(gates):
        if g.name in _SELF_INVERSE:
            out.append(g)
        elif g.name == "u3":
            t, p, l = g.params
            out.append(Gate("u3", g.qubits, (-t, -l, -p)))
        elif g.name in ("p", "cp"):
            out.append(Gate(g.name, g.qubits, (-g.params[0],)))
        elif g.name == "s":
            out.append(Gate("sdg", g.qubits))
        elif g.name == "sdg":
            out.append(Gate("s", g.qubits))
        else:
            raise ValueError(f"no inverse rule for {g.name}")
    return out


def gate_counts(gates: Sequence[Gate]) -> dict:
    out: dict = {}
    for g in gates:
        out[g.name] = out.get(g.name, 0) + 1
    return out


def random_state(n: int, seed: int) -> np.ndarray:
    """A random normalised complex128 vector of length 2^n (Gaussian entries)."""
    rng = _rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.sqrt(np.vdot(v, v).real)


# --------------------------------------------------------------------------
# Cut-variant batches.
# Labels: init in {"0", "1", "+", "+i"} (Section III.A, eqs 3.3-3.6),
# measurement basis in {"I", "X", "Y"} (the three upstream variants).


INIT_LABELS = ("0", "1", "+", "+i")
BASIS_LABELS = ("I", "X", "Y")


@dataclass
class BatchCircuit:
    width: int
    depth: int
    gates: List[Gate]
    cut_inputs: List[Tuple[int, str]] = field(default_factory=list)
    cut_outputs: List[Tuple[int, str]] = field(default_factory=list)


def batch_variants(count: int = 4096, seed: int = 4096, wmin: int = 10,
                   wmax: int = 20, dmin: int = 10, dmax: int = 60
                   ) -> List[BatchCircuit]:
    """Ragged batch of subcircuit variants.

    Per circuit, in this draw order: width w ~ U{wmin..wmax}, depth
    d ~ U{dmin..dmax}, number of cut inputs a ~ U{1..3}, number of cut outputs
    b ~ U{1..3}; the a input qubits (without replacement) and their init labels
    (uniform over 4); the b output qubits (without replacement) and their
    basis labels (uniform over 3); then the body (U3 layers with a CZ/CNOT
    brick wall, coin per pair).
    """
    rng = _rng(seed)
    out = []
    for _ in range(count):
        w = int(rng.integers(wmin, wmax + 1))
        d = int(rng.integers(dmin, dmax + 1))
        a = int(rng.integers(1, 4))
        b = int(rng.integers(1, 4))
        qin = rng.choice(w, size=a, replace=False)
        lin = rng.integers(0, 4, size=a)
        qout = rng.choice(w, size=b, replace=False)
        lout = rng.integers(0, 3, size=b)
        body = _layers(rng, w, d, "mixed")
        out.append(BatchCircuit(
            w, d, body,
            [(int(q), INIT_LABELS[int(l)]) for q, l in zip(qin, lin)],
            [(int(q), BASIS_LABELS[int(l)]) for q, l in zip(qout, lout)]))
    return out


@dataclass
class ServeRequest:
    arrival_s: float
    width: int
    depth: int
    precision: str          # "c64" or "c128"
    want_samples: bool      # False: probability vector; True: samples
    shots: int
    seed: int               # circuit seed (layered_circuit) and sampler seed


def serve_trace(n_requests: int = 2000, rate_per_s: float = 100.0,
                seed: int = 5, wmin: int = 8, wmax: int = 28,
                dmin: int = 10, dmax: int = 100, shots: int = 10_000
                ) -> List[ServeRequest]:
    """Poisson request stream.

    Draw order per request: inter-arrival gap ~ Exp(rate), width, depth,
    precision (c64 with probability 0.8), output kind (samples with
    probability 0.5), circuit seed (63-bit).
    """
    rng = _rng(seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        w = int(rng.integers(wmin, wmax + 1))
        d = int(rng.integers(dmin, dmax + 1))
        prec = "c64" if rng.random() < 0.8 else "c128"
        samp = bool(rng.random() < 0.5)
        cs = int(rng.integers(0, 1 << 62))
        out.append(ServeRequest(t, w, d, prec, samp, shots, cs))
    return out


# ---------------------------------------------------------------------------
# Wire-cut problems (Section III.A): an uncut circuit made of subcircuits in a
# chain, consecutive subcircuits sharing one wire that is cut between them.


@dataclass
class CutSub:
    """One subcircuit of a cut problem, in its local qubit numbering.

    Per local qubit j: ``out_qubit[j]`` is the uncut qubit whose final value
    is measured at j (-1: none), ``cut_in[j]`` the cut whose downstream end
    initialises j (-1: none), ``cut_out[j]`` the cut whose upstream end is
    measured at j (-1: none).  Every local qubit is measured exactly once:
    as an output or as a cut's upstream end.
    """
    width: int
    depth: int
    gates: List[Gate]
    out_qubit: List[int]
    cut_in: List[int]
    cut_out: List[int]


@dataclass
class CutProblem:
    n: int                 # qubits of the uncut circuit
    n_cuts: int
    subs: List[CutSub]
    uncut: List[Gate]      # the same circuit without cuts, on n qubits


def cut_chain(widths: Sequence[int], depth: int, seed: int) -> CutProblem:
    """Chain of len(widths) subcircuits cut on len(widths) - 1 wires.

    Subcircuit s has its own qubits; for s > 0 its local qubit 0 is the wire
    coming from subcircuit s - 1 (cut s - 1, downstream end, measured at the
    end as that wire's uncut qubit), and for s < S - 1 its local qubit
    w_s - 1 is the wire going to subcircuit s + 1 (cut s, upstream end).  A
    middle subcircuit of width 1 is one wire cut on both sides: initialised
    by cut s - 1 and measured for cut s, with no output.  Uncut qubits are
    numbered in order of first appearance.  Bodies are drawn one after the
    other from one generator: per subcircuit, ``depth`` U3 layers with a
    CZ/CNOT brick wall (coin per pair).  The uncut circuit is the bodies in
    subcircuit order on the uncut qubits.
    """
    rng = _rng(seed)
    S = len(widths)
    subs: List[CutSub] = []
    uncut: List[Gate] = []
    nxt = 0
    wire_q = -1
    for s, w in enumerate(widths):
        if w < 1 or (S > 1 and w < 2 and s in (0, S - 1)):
            raise ValueError("end subcircuits of a chain need width >= 2")
        out_q, c_in, c_out, umap = [], [], [], []
        for j in range(w):
            if w == 1 and 0 < s < S - 1:       # a wire cut on both sides
                out_q.append(-1); c_in.append(s - 1); c_out.append(s)
                umap.append(wire_q)
            elif s > 0 and j == 0:             # incoming wire
                out_q.append(wire_q); c_in.append(s - 1); c_out.append(-1)
                umap.append(wire_q)
            elif s < S - 1 and j == w - 1:     # outgoing wire
                out_q.append(-1); c_in.append(-1); c_out.append(s)
                umap.append(nxt)
                wire_q = nxt
                nxt += 1
            else:
                out_q.append(nxt); c_in.append(-1); c_out.append(-1)
                umap.append(nxt)
                nxt += 1
        body = _layers(rng, w, depth, "mixed")
        subs.append(CutSub(w, depth, body, out_q, c_in, c_out))
        uncut += [Gate(g.name, tuple(umap[q] for q in g.qubits), g.params)
                  for g in body]
    return CutProblem(nxt, S - 1, subs, uncut)


def cut_variants(sub: CutSub) -> List[BatchCircuit]:
    """All variants of one subcircuit in the canonical order.

    The subcircuit's cut ends, in increasing local qubit order, are the
    digits of the variant index, the first end least significant: a
    downstream end (cut input) has 4 values, labels 0, 1, +, +i; an
    upstream end (cut output) has 3, bases I, X, Y.  A qubit that is both
    contributes its input digit first.
    """
    ends = []
    for j in range(sub.width):
        if sub.cut_in[j] >= 0:
            ends.append(("in", j))
        if sub.cut_out[j] >= 0:
            ends.append(("out", j))
    total = 1
    for kind, _ in ends:
        total *= 4 if kind == "in" else 3
    out = []
    for v in range(total):
        r = v
        ins, outs = [], []
        for kind, j in ends:
            if kind == "in":
                ins.append((j, INIT_LABELS[r % 4]))
                r //= 4
            else:
                outs.append((j, BASIS_LABELS[r % 3]))
                r //= 3
        out.append(BatchCircuit(sub.width, sub.depth, list(sub.gates), ins,
                                outs))
    return out

