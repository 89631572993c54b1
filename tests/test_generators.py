"""Seeded workload generators: determinism and the gate counts of each
workload (layered 12q/20q/30q, QFT-style 33q/34q, ragged cut variants,
serving trace)."""
import numpy as np

from circuits import (batch_variants, gate_counts, ghz_circuit,
                      layered_circuit, qft_style_circuit, serve_trace)


def test_layered_counts():
    assert gate_counts(layered_circuit(12, 20, 12)) == {"u3": 240, "cz": 110}
    assert gate_counts(layered_circuit(30, 40, 30)) == {"u3": 1200, "cz": 580}
    assert gate_counts(layered_circuit(20, 40, 30)) == {"u3": 800, "cz": 380}


def test_brick_wall_pairs():
    g = [x for x in layered_circuit(6, 2, 1) if x.name == "cz"]
    assert [x.qubits for x in g] == [(0, 1), (2, 3), (4, 5), (1, 2), (3, 4)]


def test_qft_counts():
    for n, want in ((34, {"h": 34, "cp": 561, "u3": 340, "cz": 165}),
                    (33, {"h": 33, "cp": 528, "u3": 330, "cz": 160})):
        x, g = qft_style_circuit(n, n)
        assert 0 <= x < (1 << n)
        assert gate_counts(g) == want


def test_qft_order():
    _, g = qft_style_circuit(3, 0, tail_layers=0)
    assert [(x.name, x.qubits) for x in g] == [
        ("h", (2,)), ("cp", (1, 2)), ("cp", (0, 2)),
        ("h", (1,)), ("cp", (0, 1)), ("h", (0,))]


def test_determinism():
    a = layered_circuit(10, 5, 7)
    b = layered_circuit(10, 5, 7)
    assert a == b
    assert layered_circuit(10, 5, 8) != a
    assert ghz_circuit(4)[0].name == "h"


def test_batch_variants_shape():
    vs = batch_variants(200, seed=4096)
    assert all(10 <= v.width <= 20 and 10 <= v.depth <= 60 for v in vs)
    for v in vs:
        qi = [q for q, _ in v.cut_inputs]
        qo = [q for q, _ in v.cut_outputs]
        assert 1 <= len(qi) <= 3 and len(set(qi)) == len(qi)
        assert 1 <= len(qo) <= 3 and len(set(qo)) == len(qo)
        assert all(0 <= q < v.width for q in qi + qo)
    names = {g.name for v in vs for g in v.gates}
    assert names == {"u3", "cz", "cx"}
    widths = np.array([v.width for v in vs])
    assert widths.min() == 10 and widths.max() == 20


def test_serve_trace():
    tr = serve_trace(500, rate_per_s=50.0, seed=5)
    t = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1 / 50.0) < 0.2 / 50.0
    frac64 = np.mean([r.precision == "c64" for r in tr])
    assert 0.7 < frac64 < 0.9
    assert all(8 <= r.width <= 28 and 10 <= r.depth <= 100 for r in tr)


def test_cut_chain_structure():
    from circuits import cut_chain, cut_variants
    prob = cut_chain((3, 4, 1, 3), 2, 9)
    # each cut joins two ends of one uncut qubit
    assert prob.n_cuts == 3 and prob.n == (3 + 4 + 1 + 3) - 3
    ins = [c for sub in prob.subs for c in sub.cut_in if c >= 0]
    outs = [c for sub in prob.subs for c in sub.cut_out if c >= 0]
    assert sorted(ins) == sorted(outs) == [0, 1, 2]
    outq = sorted(q for sub in prob.subs for q in sub.out_qubit if q >= 0)
    assert outq == list(range(prob.n))
    for sub in prob.subs:               # every local qubit measured once
        for j in range(sub.width):
            assert (sub.out_qubit[j] >= 0) != (sub.cut_out[j] >= 0)
    counts = [len(cut_variants(sub)) for sub in prob.subs]
    assert counts == [3, 12, 12, 4]
    v = cut_variants(prob.subs[1])
    # first end (local 0, input) is the least significant digit
    assert v[1].cut_inputs == [(0, "1")] and v[4].cut_outputs == [(3, "X")]

