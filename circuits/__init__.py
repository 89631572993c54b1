"""Seeded synthetic circuit generators.

This package only draws random numbers and lays out gate lists as
(name, qubits, params) records.  It contains none of the simulation
arithmetic: gate matrices, amplitudes, probabilities and the cut-variant
state preparations are built separately by the oracle (``oracle/``) and by
the HIP library (``paper_2502_11385_amd``).  Both sides consume the same
records, which is the only thing they share.
"""
from .generators import (  # noqa: F401
    Gate,
    BatchCircuit,
    CutSub,
    CutProblem,
    cut_chain,
    cut_variants,
    ServeRequest,
    layered_circuit,
    ghz_circuit,
    bv_circuit,
    qft_style_circuit,
    inverse_circuit,
    batch_variants,
    serve_trace,
    random_state,
    gate_counts,
)
