"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package generates inputs only: gate lists (random unitaries, angles, noise
strengths), request streams and measurement draws.  It applies no gate, forms
no probability and collapses nothing; the oracle and the HIP library each do
that arithmetic on their own.
"""
from .circuits import (  # noqa: F401
    Op, haar_unitary, layered_circuit, noisy_circuit, param_circuit,
    measurement_draws, gate_counts, product_layer, inverse, random_state,
    random_gate_ops, serving_requests, X, H, ry, rz, haar_unitary_k, random_kraus, random_multi_ops,
    paper_random_circuit, SQRT_X, SQRT_Y,
)
