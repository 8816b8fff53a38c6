"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This module draws random numbers and lays out gate lists as plain data.  It
holds none of the simulator's arithmetic: no gate matrix is built here (except
the Haar-random unitaries, which are inputs), and nothing here applies a gate
to a state.  Both the oracle and the HIP library consume these lists and build
their own matrices from (kind, qubits, theta).
"""
from .circuits import (Gate, GATE_KINDS, layered_circuit, brickwork_circuit, qft_circuit,
                       qaoa_circuit,
                       haar_unitary, fused_haar_circuit, gate_bench_set, random_matching,
                       serving_requests, Request)
from .states import gaussian_state_np, basis_state_np

__all__ = ["Gate", "GATE_KINDS", "layered_circuit", "brickwork_circuit", "qft_circuit", "qaoa_circuit",
           "haar_unitary", "fused_haar_circuit", "gate_bench_set", "random_matching",
           "serving_requests", "Request", "gaussian_state_np", "basis_state_np"]
