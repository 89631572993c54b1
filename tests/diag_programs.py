"""Seeded random gate programs for the parity tests (inputs only: gate
matrices as NumPy arrays with their target and control lists)."""
import math

import numpy as np


def _unitary2(rng):
    z = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def diagonal_heavy(n, count, seed, non_unitary=True):
    """Mostly diagonal gates of every form the tile program accepts (masked
    phases with 1-3 controls, unitary 1-2 qubit diagonals with and without
    controls, Z-rotations with their global phase, S/T, optionally a
    non-unitary diagonal now and then), with a dense 1-qubit gate about
    every tenth gate.  Returns [(matrix, targets, controls)]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 10))
        qs = [int(v) for v in rng.choice(n, 4, replace=False)]
        ph = np.exp(1j * rng.uniform(-7, 7, 4))
        if kind == 0:
            out.append((_unitary2(rng), qs[:1], []))
        elif kind == 1:       # CP / CCP / CCCP
            c = int(rng.integers(1, 4))
            out.append((np.diag([1, ph[0]]), qs[:1], qs[1:1 + c]))
        elif kind == 2:       # CZ
            out.append((np.diag([1, -1]).astype(complex), qs[:1], qs[1:2]))
        elif kind == 3:       # 1-qubit unitary diagonal
            out.append((np.diag(ph[:2]), qs[:1], []))
        elif kind == 4:       # 2-qubit unitary diagonal
            out.append((np.diag(ph), qs[:2], []))
        elif kind == 5:       # controlled 2-qubit unitary diagonal
            out.append((np.diag(ph), qs[:2], qs[2:3]))
        elif kind == 6:       # controlled 1-qubit diagonal
            out.append((np.diag(ph[:2]), qs[:1], qs[1:3]))
        elif kind == 7:       # RZ
            t = float(rng.uniform(-4, 4))
            out.append((np.diag([np.exp(-0.5j * t), np.exp(0.5j * t)]),
                        qs[:1], []))
        elif kind == 8 and non_unitary and rng.uniform() < 0.2:
            out.append((np.diag([1.25, 0.8j]), qs[:1], []))
        else:                 # S, T
            out.append((np.diag([1, np.exp(0.25j * math.pi *
                                           (1 + kind % 2))]), qs[:1], []))
    return out


def is_diagonal(u):
    u = np.asarray(u)
    return np.count_nonzero(u - np.diag(np.diag(u))) == 0


def _unitary(d, rng):
    """A Haar-random d x d unitary (QR of a complex Gaussian matrix)."""
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_gates(n, count, rng):
    """Gates of every form the library accepts: dense 1..5-target unitaries
    with 0..2 controls, unitary diagonals, masked phases and diagonals that
    are not phases.  Returns [(matrix, targets, controls)]."""
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 9))
        k = 1 if kind < 4 else int(rng.integers(1, 6))
        c = int(rng.integers(0, 3))
        c = min(c, n - k)
        qs = [int(v) for v in rng.choice(n, k + c, replace=False)]
        t, ctl = qs[:k], qs[k:]
        if kind <= 3:        # dense 1-qubit, 0..2 controls
            u = _unitary(2, rng)
        elif kind <= 5:      # dense k-qubit
            u = _unitary(1 << k, rng)
        elif kind == 6:      # unitary diagonal
            u = np.diag(np.exp(1j * rng.uniform(-7, 7, 1 << k)))
        elif kind == 7:      # masked phase
            d = np.ones(1 << k, complex)
            d[-1] = np.exp(1j * rng.uniform(-7, 7))
            u = np.diag(d)
        else:                # a diagonal that is not a phase
            u = np.diag(rng.uniform(0.5, 1.5, 1 << k) *
                        np.exp(1j * rng.uniform(-3, 3, 1 << k)))
        out.append((u, t, ctl))
    return out


def random_opts(rng, c128):
    """Plan options within the documented ranges (reg_log2 <= 4 for
    complex128, tile_log2 - reg_log2 <= 9)."""
    strategy = int(rng.integers(1, 4))          # plain, fused, tiled
    L = int(rng.integers(8, 14))
    rb = int(rng.integers(3, 5 if c128 else 6))
    rb = max(rb, L - 9)
    if c128:
        rb = min(rb, 4)
        L = min(L, rb + 9)
    low = int(rng.integers(0, min(L, 7)))
    kmax = int(rng.integers(1, 6))
    return dict(strategy=strategy, tile_log2=L, reg_log2=rb,
                low_qubits=low, k_max=kmax)
