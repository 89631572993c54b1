"""CPU oracle for the dense state-vector path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything under ``oracle/``; only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library: it builds its own gate matrices from gate names and angles and
applies them with plain NumPy complex128 arithmetic.

Every function is pinned by CPU tests against facts fixed by the paper or by
mathematics (closed forms, invariants, brute force); see ``tests/``.
"""
from .statevector import (  # noqa: F401
    gate_spec,
    apply_gate,
    simulate,
    probabilities,
    marginal,
    norm,
    full_unitary,
    embed,
    splitmix64,
    uniforms,
    sample,
    top_k,
    permute_qubits,
    probs_of_amplitudes,
    pauli_expectation,
    cut_prologue,
    cut_epilogue,
    variant_probabilities,
    cut_term_vectors,
    cut_reconstruct,
    state_bytes,
)
