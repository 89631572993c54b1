"""Serving on the GPU: results of a mixed request stream match the oracle,
each result is the same alone and in the mix, and admission by bytes keeps
the reserved HBM within the budget while queueing the rest."""
import numpy as np
import pytest

import oracle
from circuits import layered_circuit

torch = pytest.importorskip("torch")
from paper_2502_11385_amd import qsv  # noqa: E402

pytestmark = pytest.mark.gpu
C64, C128 = qsv.QSV_C64, qsv.QSV_C128


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (width, depth, precision, shots)
MIX = [(8, 10, C64, 0), (12, 6, C128, 0), (9, 20, C64, 3000),
       (14, 5, C64, 0), (16, 4, C128, 2000), (21, 2, C64, 0),
       (10, 12, C128, 0), (13, 8, C64, 5000), (20, 2, C64, 0),
       (22, 1, C128, 4000), (7, 30, C64, 0), (15, 3, C64, 1000)]


def _circ(i, w, d):
    return layered_circuit(w, d, seed=100 + i)


def _run(server, reqs):
    tickets = [server.submit(w, qsv.Circuit.from_gates(_circ(i, w, d)), prec,
                             shots=shots, seed=7 + i)
               for i, (w, d, prec, shots) in enumerate(reqs)]
    out = []
    for t in tickets:
        data, info = server.wait(t)
        server.release(t)
        out.append((data, info))
    return out


def test_mixed_stream_matches_oracle():
    srv = qsv.Server()
    res = _run(srv, MIX)
    for i, ((w, d, prec, shots), (data, info)) in enumerate(zip(MIX, res)):
        assert info["status"] == 0
        p = oracle.probabilities(oracle.simulate(w, _circ(i, w, d)))
        if shots == 0:
            tol = 2e-6 if prec == C64 else 1e-12
            assert data.shape == (1 << w,)
            assert np.max(np.abs(data.astype(np.float64) - p)) <= tol, i
        else:
            want = oracle.sample(p, shots, 7 + i)
            c = np.cumsum(p)
            t = oracle.uniforms(7 + i, shots) * c[-1]
            delta = 1e-9 if prec == C128 else 2e-4
            for j in np.nonzero(data != want)[0]:
                lo, hi = sorted((int(data[j]), int(want[j])))
                assert np.min(np.abs(c[lo:hi] - t[j])) <= delta
        assert info["t_submit"] <= info["t_admit"] <= info["t_start"] <= \
            info["t_done"]
        assert info["batched"] == (w <= 20)
    st = srv.stats()
    assert st["completed"] == len(MIX)
    assert st["batch_launches"] >= 1 and st["single_launches"] >= 2
    srv.close()


def test_alone_equals_in_mix_bitwise():
    mixed = _run(qsv.Server(), MIX)
    for i, req in enumerate(MIX):
        srv = qsv.Server(serial=True)
        tk = srv.submit(req[0], qsv.Circuit.from_gates(_circ(i, req[0], req[1])),
                        req[2], shots=req[3], seed=7 + i)
        alone, _ = srv.wait(tk)
        srv.close()
        assert np.array_equal(alone, mixed[i][0]), i


def test_budget_queues_and_bounds_reserved_bytes():
    reqs = [(18, 4, C64, 0)] * 6 + [(19, 3, C128, 0)] * 3
    per = max((16 if p == C128 else 8) << w for w, _, p, _ in reqs)
    budget = 3 * per                           # a few at a time
    srv = qsv.Server(budget_bytes=budget)
    res = _run(srv, reqs)
    st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["peak_reserved_bytes"] <= budget
    admits = sorted(info["t_admit"] for _, info in res)
    dones = sorted(info["t_done"] for _, info in res)
    assert admits[-1] >= dones[0]     # the last admission waited for a finish
    for i, (w, d, prec, _) in enumerate(reqs):
        p = oracle.probabilities(oracle.simulate(w, _circ(i, w, d)))
        tol = 2e-6 if prec == C64 else 1e-12
        assert np.max(np.abs(res[i][0].astype(np.float64) - p)) <= tol
    srv.close()


def test_budget_counts_cached_device_memory():
    """Device memory the server keeps for reuse (pooled blocks, cached
    states) counts against the budget: a stream of wide requests of mixed
    widths and precisions never holds more than the budget plus a small
    fixed overhead, by the device's own free-memory count."""
    import threading
    gib = 1 << 30
    budget = int(3.5 * gib)
    reqs = [(27, 2, C128, 0), (28, 2, C64, 0), (26, 2, C128, 2000),
            (27, 2, C64, 0), (12, 4, C64, 0), (25, 3, C128, 0),
            (28, 1, C64, 1000)]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    low = [free0]
    stop = threading.Event()

    def poll():
        while not stop.is_set():
            low[0] = min(low[0], torch.cuda.mem_get_info()[0])
            stop.wait(0.0005)

    th = threading.Thread(target=poll, daemon=True)
    th.start()
    srv = qsv.Server(budget_bytes=budget)
    try:
        res = _run(srv, reqs)
        held = free0 - torch.cuda.mem_get_info()[0]
        st = srv.stats()
    finally:
        stop.set()
        th.join()
    overhead = 256 << 20
    assert free0 - low[0] <= budget + overhead, (free0 - low[0]) / gib
    assert held <= budget + overhead, held / gib
    assert st["completed"] == len(reqs) and st["idle_trims"] >= 1
    for i, (w, d, prec, shots) in enumerate(reqs):
        data, info = res[i]
        assert info["status"] == 0
        if shots:
            assert data.shape == (shots,) and int(data.max()) < (1 << w)
        else:
            assert abs(float(np.sum(data, dtype=np.float64)) - 1) < 1e-4
    w, d, prec, _ = reqs[4]
    p = oracle.probabilities(oracle.simulate(w, _circ(4, w, d)))
    assert np.max(np.abs(res[4][0].astype(np.float64) - p)) <= 2e-6
    srv.close()
