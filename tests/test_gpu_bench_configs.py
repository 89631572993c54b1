"""Parity of the workloads bench.py times, as bench.py builds them.

* The 4096-variant cut batch (widths 10..20, depths 10..60, seed 4096),
  autotuned and replayed from a hipGraph: every variant of width <= 14 and
  a seeded 5 % of widths 15..20 against the oracle, complex64 tolerances
  (2e-6 per probability, total variation <= 1e-4 per variant).
* The QFT-style workload (ladder on a random basis state plus its 10 U3+CZ
  tail layers): its 20-qubit instances against the oracle (amplitudes and
  the top-10 marginal), and at full width (34 qubits complex64, 33 qubits
  complex128) the circuit followed by its inverse returns the basis state,
  checked through marginals that together cover every qubit.
The measured errors are printed (pytest -s) for the record.
"""
import numpy as np
import pytest

import oracle
import oracle_pool
from circuits import batch_variants, inverse_circuit, qft_style_circuit

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu
C64, C128 = qsv.QSV_C64, qsv.QSV_C128


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def bench_batch():
    """The batch as the bench builds and times it: the same generator call,
    autotune and graph replay, two launches over the same buffers."""
    vs = batch_variants(4096, seed=4096)
    b = qsv.Batch(vs, prec=C64, autotune=True, use_graph=True)
    out = b.output()
    b.launch(out)
    b.launch(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    offs = np.asarray(b.offsets).copy()
    st = b.stats()
    b.free()
    del out
    torch.cuda.empty_cache()
    return vs, got, offs, st


def _check_variants(vs, got, offs, idx):
    want = oracle_pool.pool_map(oracle_pool.variant_probabilities,
                                [vs[i] for i in idx])
    worst = worst_tv = 0.0
    for i, p_or in zip(idx, want):
        p = got[int(offs[i]):int(offs[i + 1])].astype(np.float64)
        assert p.shape == p_or.shape, i
        err = float(np.max(np.abs(p - p_or)))
        tv = 0.5 * float(np.sum(np.abs(p - p_or)))
        assert err <= 2e-6, (i, vs[i].width, err)
        assert tv <= 1e-4, (i, vs[i].width, tv)
        worst, worst_tv = max(worst, err), max(worst_tv, tv)
    return worst, worst_tv


def test_bench_batch_all_narrow_variants(bench_batch):
    vs, got, offs, st = bench_batch
    idx = [i for i, v in enumerate(vs) if v.width <= 14]
    assert len(idx) > 1500
    worst, tv = _check_variants(vs, got, offs, idx)
    print(f"\nbatch (tile_log2 {st['tile_log2']}, reg_log2 {st['reg_log2']}, "
          f"grid {st['grid']}): {len(idx)} variants of width <= 14, "
          f"max|dp| = {worst:.3e}, max TV = {tv:.3e}")


def _wide_sample(vs):
    """A seeded 5 % of the variants of widths 15..20."""
    wide = [i for i, v in enumerate(vs) if v.width >= 15]
    rng = np.random.default_rng(4096)
    return sorted(rng.choice(wide, size=max(1, len(wide) // 20),
                             replace=False).tolist())


@pytest.mark.parametrize("lo,hi", [(15, 17), (18, 19), (20, 20)])
def test_bench_batch_sampled_wide_variants(bench_batch, lo, hi):
    """The seeded 5 % sample of widths 15..20, checked in width bands (each
    band's oracle work stays within a test's time)."""
    vs, got, offs, _ = bench_batch
    idx = [i for i in _wide_sample(vs) if lo <= vs[i].width <= hi]
    assert idx
    worst, tv = _check_variants(vs, got, offs, idx)
    print(f"\nbatch: seeded 5 % of widths 15..20, band {lo}..{hi} "
          f"({len(idx)} variants), max|dp| = {worst:.3e}, max TV = {tv:.3e}")


@pytest.mark.parametrize("prec", [C64, C128])
@pytest.mark.parametrize("seed", [33, 34])
def test_qft_style_20q_instance(prec, seed):
    """The configured QFT-style construction (ladder + 10 tail layers) at
    20 qubits, default plan: amplitudes and the top-10 marginal."""
    n = 20
    x, gates = qft_style_circuit(n, seed)
    assert sum(1 for g in gates if g.name == "u3") == 10 * n
    want = oracle.simulate(n, gates, init=x)
    s = qsv.State(n, prec)
    s.init_basis(x)
    s.apply_fused(qsv.Circuit.from_gates(gates))
    got = s.get().astype(np.complex128)
    err = float(np.max(np.abs(got - want)))
    tol = 1e-6 if prec == C64 else 1e-12
    assert err <= tol
    pw = oracle.probabilities(want)
    if prec == C64:
        assert 0.5 * np.sum(np.abs(np.abs(got) ** 2 - pw)) <= 1e-4
    top = list(range(n - 10, n))
    m = s.marginal(top)
    merr = float(np.max(np.abs(m - oracle.marginal(pw, n, top))))
    assert merr <= (2e-6 if prec == C64 else 1e-12)
    print(f"\nqft-style 20q seed {seed} prec {prec}: max|da| = {err:.3e}, "
          f"top-10 marginal max|dP| = {merr:.3e}")
    s.free()


@pytest.mark.parametrize("n,prec", [(34, C64), (33, C128)])
def test_qft_style_round_trip_full_width(n, prec):
    """The benchmarked wide circuit (seed n) followed by its inverse returns
    |x>: marginals over qubits 0..9, 10..19, 20..29 and 30..n-1 are each one
    at x's bits, and the norm is one."""
    x, gates = qft_style_circuit(n, n)
    s = qsv.State(n, prec)
    s.init_basis(x)
    s.apply_fused(qsv.Circuit.from_gates(gates + inverse_circuit(gates)))
    tol = 1e-4 if prec == C64 else 1e-10
    nv = s.norm()
    assert abs(nv - 1.0) < tol
    worst = 0.0
    for lo in range(0, n, 10):
        qs = list(range(lo, min(n, lo + 10)))
        m = s.marginal(qs)
        j = (x >> lo) & ((1 << len(qs)) - 1)
        worst = max(worst, abs(m[j] - 1.0))
        assert abs(m[j] - 1.0) < tol, (lo, m[j])
    print(f"\nround trip {n}q prec {prec}: |norm-1| = {abs(nv - 1):.3e}, "
          f"max |1 - P(x bits)| = {worst:.3e}")
    s.free()
    torch.cuda.empty_cache()
