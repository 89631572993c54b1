"""The host planner (no GPU): its pass list, replayed by the oracle, gives the
same state as the gate list in order; tile passes respect the tile's qubit
set and size; fused blocks respect k_max; the block products, multiplied in
NumPy here and applied by the oracle, reproduce the circuit."""
import math

import numpy as np
import pytest

import oracle
from circuits import Gate, layered_circuit, qft_style_circuit, random_state
from paper_2502_11385_amd import qsv
from diag_programs import diagonal_heavy, is_diagonal


def _mixed(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 8))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        ang = [float(v) for v in rng.uniform(0, 2 * math.pi, 3)]
        out.append([Gate("u3", (a,), tuple(ang)), Gate("h", (a,)),
                    Gate("s", (a,)), Gate("p", (a,), (ang[0],)),
                    Gate("cx", (a, b)), Gate("cz", (a, b)),
                    Gate("cp", (a, b), (ang[1],)), Gate("x", (a,))][kind])
    return out


def _specs(gates):
    return [oracle.gate_spec(g.name, g.qubits, g.params) for g in gates]


def _replay(n, specs, order, v):
    psi = v.copy()
    for gi in order:
        t, c, u = specs[gi]
        psi = oracle.apply_gate(psi, n, u, t, c)
    return psi


CASES = [
    ("layered", 8, lambda: layered_circuit(8, 6, 1)),
    ("layered14", 14, lambda: layered_circuit(14, 5, 2)),
    ("qft", 9, lambda: qft_style_circuit(9, 4, tail_layers=2)[1]),
    ("mixed", 10, lambda: _mixed(10, 120, 5)),
]


@pytest.mark.parametrize("strategy", [qsv.PLAN_PLAIN, qsv.PLAN_TILED,
                                      qsv.PLAN_FUSED])
@pytest.mark.parametrize("name,n,make", CASES)
def test_plan_order_is_equivalent(strategy, name, n, make):
    gates = make()
    circ = qsv.Circuit.from_gates(gates)
    for opts in (qsv.fuse_opts(strategy=strategy),
                 qsv.fuse_opts(strategy=strategy, tile_log2=8, k_max=3,
                               low_qubits=2, reg_log2=5)):
        gp, order, kinds, pq = qsv.plan_describe(circ, n, qsv.QSV_C64, opts)
        assert sorted(order.tolist()) == list(range(len(gates)))
        # passes are applied in order; gates of one pass are contiguous
        assert np.all(np.diff(gp[order]) >= 0)
        specs = _specs(gates)
        v = random_state(n, 3)
        want = _replay(n, specs, range(len(gates)), v)
        got = _replay(n, specs, order, v)
        assert np.max(np.abs(got - want)) < 1e-12
        if strategy == qsv.PLAN_PLAIN:
            assert len(kinds) == len(gates) and np.all(kinds == 1)


@pytest.mark.parametrize("name,n,make", CASES)
def test_tile_pass_structure(name, n, make):
    gates = make()
    circ = qsv.Circuit.from_gates(gates)
    for L, m in ((10, 5), (8, 2), (12, 4)):
        opts = qsv.fuse_opts(strategy=qsv.PLAN_TILED, tile_log2=L,
                             low_qubits=m)
        gp, order, kinds, pq = qsv.plan_describe(circ, n, qsv.QSV_C64, opts)
        Le = min(L, n)
        for p, mask in enumerate(pq):
            if kinds[p] != 2:
                continue
            mask = int(mask)
            assert bin(mask).count("1") == Le
            assert mask & ((1 << min(m, Le)) - 1) == (1 << min(m, Le)) - 1
        for gi, g in enumerate(gates):
            t, c, u = oracle.gate_spec(g.name, g.qubits, g.params)
            p = gp[gi]
            if kinds[p] == 2 and not np.allclose(u, np.diag(np.diag(u))):
                for q in t:   # dense targets must be tile qubits
                    assert int(pq[p]) >> q & 1


@pytest.mark.parametrize("kmax", [2, 3, 5])
@pytest.mark.parametrize("name,n,make", CASES)
def test_fused_blocks_reproduce_circuit(kmax, name, n, make):
    gates = make()
    circ = qsv.Circuit.from_gates(gates)
    opts = qsv.fuse_opts(strategy=qsv.PLAN_FUSED, k_max=kmax)
    gp, order, kinds, pq = qsv.plan_describe(circ, n, qsv.QSV_C128, opts)
    specs = _specs(gates)
    v = random_state(n, 9)
    want = _replay(n, specs, range(len(gates)), v)
    psi = v.copy()
    for p in range(len(kinds)):
        members = [gi for gi in order if gp[gi] == p]
        qs = [q for q in range(n) if int(pq[p]) >> q & 1]
        assert kinds[p] == 3 and len(qs) <= kmax
        k = len(qs)
        # block product in NumPy: embed each member on the block's qubits
        u = np.eye(1 << k, dtype=complex)
        for gi in members:
            t, c, g = specs[gi]
            assert set(t) | set(c) <= set(qs)
            u = oracle.embed(k, g, [qs.index(x) for x in t],
                             [qs.index(x) for x in c]) @ u
        psi = oracle.apply_gate(psi, n, u, qs)
    assert np.max(np.abs(psi - want)) < 1e-12


def test_pass_counts_30q_layered():
    gates = layered_circuit(30, 40, 30)
    circ = qsv.Circuit.from_gates(gates)
    _, _, kinds, _ = qsv.plan_describe(circ, 30, qsv.QSV_C64,
                                       qsv.fuse_opts(strategy=qsv.PLAN_TILED))
    # 1780 gates; the tiled plan needs far fewer full passes
    assert len(kinds) < 200
    _, _, fk, _ = qsv.plan_describe(circ, 30, qsv.QSV_C64,
                                    qsv.fuse_opts(strategy=qsv.PLAN_FUSED))
    assert len(fk) < 1780


def test_tiled_program_size_30q_layered():
    """Planner quality on the 30-qubit depth-40 layered circuit (1200 U3 +
    580 CZ), default options: the pass count and the op count of the tile
    program and its register segments are what the tile kernel's time
    follows (one HBM round trip, the tile's load and store and its re-layouts
    per pass, about 0.2 ms per dense op per 2^30 amplitudes), so none may
    grow.  Reached: 22 tile passes, 150 segments, 688 ops (tile qubits taken
    as the window of consecutive qubits that holds the most gates: 53 passes
    with the first qubits the gates ask for; U3s merged, CZs folded as mux
    ops, lone U3s deferred into the next op on their qubit, each CZ given to
    the side where it joins the most gates, and register segments built so
    that the side's gate comes first: 103 segments and 773 ops without)."""
    circ = qsv.Circuit.from_gates(layered_circuit(30, 40, 30))
    st = qsv.plan_program_stats(circ, 30, qsv.QSV_C64)
    assert st["passes"] == st["tile_passes"] <= 22
    assert st["segments"] <= 150
    assert 0 < st["tile_ops"] <= 688


# --------------------------------------------------------------------------
# the emitted tile program (register segments, folded diagonals, merged
# gates), executed on the host, against the oracle


def _cut_variant_gates(seed, w):
    from circuits import batch_variants
    v = batch_variants(1, seed=seed, wmin=w, wmax=w, dmin=6, dmax=6)[0]
    return (oracle.cut_prologue(v.cut_inputs) + list(v.gates) +
            oracle.cut_epilogue(v.cut_outputs))


EMU_CASES = CASES + [
    ("variant10", 10, lambda: _cut_variant_gates(3, 10)),
    ("variant12", 12, lambda: _cut_variant_gates(4, 12)),
    ("mixed12", 12, lambda: _mixed(12, 300, 17)),
]


@pytest.mark.parametrize("opts", [
    dict(), dict(tile_log2=8, low_qubits=2), dict(tile_log2=9, reg_log2=5),
    dict(tile_log2=10, low_qubits=3), dict(tile_log2=10, reg_log2=3)])
@pytest.mark.parametrize("name,n,make", EMU_CASES)
def test_emulated_tile_program_matches_oracle(name, n, make, opts):
    gates = make()
    v = random_state(n, 5)
    want = oracle.simulate(n, gates, init=v)
    got = qsv.debug_emulate_tiled(qsv.Circuit.from_gates(gates), n, v,
                                  qsv.fuse_opts(**opts))
    assert np.max(np.abs(got - want)) < 1e-12


def _random_mixed_with_diagonals(n, count, seed):
    """Gates of every kind the tile program handles: dense 1-qubit gates
    with 0-2 controls, masked phases and general 1-2 qubit diagonals."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 7))
        qs = [int(v) for v in rng.choice(n, 3, replace=False)]
        if kind <= 1:
            u = qsv.gate_matrix("u3", rng.uniform(0, 6, 3))
            out.append((u, qs[:1], qs[1:1 + kind]))
        elif kind == 2:
            out.append((qsv.gate_matrix("x"), qs[:1], qs[1:3]))   # Toffoli
        elif kind == 3:
            out.append((np.diag([1, -1]).astype(complex), qs[:1], qs[1:2]))
        elif kind == 4:
            out.append((np.diag(np.exp(1j * rng.uniform(0, 6, 2))), qs[:1],
                        []))
        elif kind == 5:
            out.append((np.diag(np.exp(1j * rng.uniform(0, 6, 4))), qs[:2],
                        []))
        else:
            out.append((np.diag([1, np.exp(1j * 0.7)]), qs[:1], qs[1:3]))
    return out


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("n,L", [(10, 8), (11, 9), (9, 9)])
def test_emulated_random_programs(seed, n, L):
    gl = _random_mixed_with_diagonals(n, 160, seed)
    circ = qsv.Circuit()
    want = random_state(n, seed)
    v = want.copy()
    for u, t, c in gl:
        circ.add(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    got = qsv.debug_emulate_tiled(circ, n, v,
                                  qsv.fuse_opts(tile_log2=L, low_qubits=2))
    assert np.max(np.abs(got - want)) < 1e-12


def _brick_cp(n, depth, seed):
    """U3 layers with brick-wall controlled phases of random angle and CZs:
    two-qubit diagonal gates that either neighbour's op can absorb."""
    rng = np.random.default_rng(seed)
    out = []
    for layer in range(depth):
        for q in range(n):
            out.append(Gate("u3", (q,), tuple(float(v) for v in
                                              rng.uniform(0, 2 * math.pi, 3))))
        for a in range(layer % 2, n - 1, 2):
            if rng.integers(0, 2):
                out.append(Gate("cp", (a, a + 1),
                                (float(rng.uniform(0, 2 * math.pi)),)))
            else:
                out.append(Gate("cz", (a, a + 1)))
    return out


@pytest.mark.parametrize("opts", [
    dict(), dict(tile_log2=10, low_qubits=2, reg_log2=3),
    dict(tile_log2=11, low_qubits=3, reg_log2=5),
    dict(tile_log2=8, low_qubits=2)])
@pytest.mark.parametrize("name,n,make", [
    ("layered16", 16, lambda: layered_circuit(16, 12, 8)),
    ("brick_cp16", 16, lambda: _brick_cp(16, 14, 9)),
    ("brick_cp16_deep", 16, lambda: _brick_cp(16, 24, 10)),
])
def test_steered_merges_match_oracle(name, n, make, opts):
    """Brick-wall circuits (16 qubits: the planner steers from there)
    whose two-qubit diagonal gates could go to either neighbour: the tile
    program, with each such gate given to the side where it joins the most
    one-target gates and the segments built and ordered to match, executed
    on the host, against the oracle; and it has fewer ops than one per
    one-target gate."""
    gates = make()
    v = random_state(n, 11)
    want = oracle.simulate(n, gates, init=v)
    o = qsv.fuse_opts(**opts)
    got = qsv.debug_emulate_tiled(qsv.Circuit.from_gates(gates), n, v, o)
    assert np.max(np.abs(got - want)) < 1e-12
    st = qsv.plan_program_stats(qsv.Circuit.from_gates(gates), n,
                                qsv.QSV_C64, o)
    n_u3 = sum(1 for g in gates if g.name == "u3")
    assert st["tile_ops"] < 0.75 * n_u3


# --------------------------------------------------------------------------
# phase blocks: runs of diagonal gates applied as one phase polynomial

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n,opts", [
    (10, dict(tile_log2=8, low_qubits=2)),
    (11, dict(tile_log2=9, low_qubits=3, reg_log2=5)),
    (12, dict(tile_log2=10, low_qubits=2, reg_log2=3)),
    (9, dict(tile_log2=9)),
])
def test_phase_blocks_emulated(seed, n, opts):
    """Diagonal-heavy random programs: the tile program (with phase blocks)
    executed on the host equals the gates applied one by one by the oracle;
    most diagonal gates land in phase blocks."""
    gl = diagonal_heavy(n, 240, 100 + seed)
    circ = qsv.Circuit()
    want = random_state(n, seed)
    v = want.copy()
    for u, t, c in gl:
        circ.add(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    o = qsv.fuse_opts(**opts)
    got = qsv.debug_emulate_tiled(circ, n, v, o)
    assert np.max(np.abs(got - want)) < 1e-12
    st = qsv.plan_program_stats(circ, n, qsv.QSV_C64, o)
    n_diag = sum(1 for u, _, _ in gl if is_diagonal(u))
    assert st["phase_blocks"] > 0
    assert st["block_gates"] > n_diag // 2


def test_phase_blocks_qft_ladder():
    """The QFT ladder's controlled phases go into phase blocks, and the
    program still reproduces the oracle."""
    n = 12
    _, gates = qft_style_circuit(n, 7, tail_layers=1)
    circ = qsv.Circuit.from_gates(gates)
    v = random_state(n, 2)
    want = oracle.simulate(n, gates, init=v)
    for opts in (dict(tile_log2=8, low_qubits=3), dict(tile_log2=10)):
        o = qsv.fuse_opts(**opts)
        got = qsv.debug_emulate_tiled(circ, n, v, o)
        assert np.max(np.abs(got - want)) < 1e-12
        st = qsv.plan_program_stats(circ, n, qsv.QSV_C64, o)
        n_cp = sum(1 for g in gates if g.name == "cp")
        assert st["block_gates"] >= n_cp // 2


def test_program_stats_match_describe():
    gates = layered_circuit(14, 6, 3)
    circ = qsv.Circuit.from_gates(gates)
    o = qsv.fuse_opts(strategy=qsv.PLAN_TILED, tile_log2=10)
    st = qsv.plan_program_stats(circ, 14, qsv.QSV_C64, o)
    _, _, kinds, _ = qsv.plan_describe(circ, 14, qsv.QSV_C64, o)
    assert st["passes"] == len(kinds)
    assert st["tile_passes"] == int(np.sum(kinds == 2))
    assert st["segments"] >= st["tile_passes"]


@pytest.mark.parametrize("seed", range(24))
def test_emulated_random_programs_random_options(seed):
    """Random gate lists of every accepted form under random tile options
    (tile size, register bits, low qubits), tile program run on the host,
    against the oracle applying every gate in order."""
    from diag_programs import random_gates, random_opts
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(6, 15))
    gl = random_gates(n, int(rng.integers(20, 160)), rng)
    o = random_opts(rng, False)
    o["strategy"] = qsv.PLAN_TILED
    circ = qsv.Circuit()
    want = random_state(n, seed)
    v = want.copy()
    for u, t, c in gl:
        circ.add(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    got = qsv.debug_emulate_tiled(circ, n, v, qsv.fuse_opts(**o))
    scale = max(1.0, float(np.max(np.abs(want))))
    assert np.max(np.abs(got - want)) / scale < 1e-12, o


@pytest.mark.parametrize("seed", range(6))
def test_emulated_random_programs_steered(seed):
    """Random gate lists of every accepted form on 16 qubits (from there
    the planner builds and orders segments for diagonal-gate ownership)
    under random tile options, tile program run on the host, against the
    oracle."""
    from diag_programs import random_gates, random_opts
    rng = np.random.default_rng(9100 + seed)
    n = 16
    gl = random_gates(n, int(rng.integers(80, 200)), rng)
    o = random_opts(rng, False)
    o["strategy"] = qsv.PLAN_TILED
    circ = qsv.Circuit()
    want = random_state(n, seed)
    v = want.copy()
    for u, t, c in gl:
        circ.add(t, u, c)
        want = oracle.apply_gate(want, n, np.asarray(u, complex), t, c)
    got = qsv.debug_emulate_tiled(circ, n, v, qsv.fuse_opts(**o))
    scale = max(1.0, float(np.max(np.abs(want))))
    assert np.max(np.abs(got - want)) / scale < 1e-12, o


@pytest.mark.parametrize("n,L", [(12, 13), (12, 12), (10, 12), (13, 13),
                                 (8, 8), (14, 12)])
def test_default_register_count_is_valid(n, L):
    """Circuits that fit one tile default to eight amplitudes per thread
    where the tile allows it (at most 512 threads); every default plans."""
    circ = qsv.Circuit.from_gates(layered_circuit(n, 4, 5))
    for prec in (qsv.QSV_C64, qsv.QSV_C128):
        st = qsv.plan_program_stats(circ, n, prec,
                                    qsv.fuse_opts(strategy=qsv.PLAN_TILED,
                                                  tile_log2=L))
        assert st["tile_passes"] >= 1
    v = random_state(n, 3)
    want = oracle.simulate(n, layered_circuit(n, 4, 5), init=v)
    if n <= 16:
        got = qsv.debug_emulate_tiled(circ, n, v, qsv.fuse_opts(tile_log2=L))
        assert np.max(np.abs(got - want)) < 1e-12


def test_planner_is_deterministic():
    """The same circuit plans to the same program every time (the steered
    search included), so a state's bits do not depend on the call."""
    gates = _brick_cp(16, 10, 21)
    circ = qsv.Circuit.from_gates(gates)
    v = random_state(16, 4)
    o = qsv.fuse_opts()
    a = qsv.plan_program_stats(circ, 16, qsv.QSV_C64, o)
    b = qsv.plan_program_stats(circ, 16, qsv.QSV_C64, o)
    assert a == b
    x = qsv.debug_emulate_tiled(circ, 16, v, o)
    y = qsv.debug_emulate_tiled(circ, 16, v, o)
    assert np.array_equal(x, y)
