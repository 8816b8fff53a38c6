"""CPU oracle for the state-vector hot path (complex128, numpy).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.
"""
from . import brute, qaoa, sv_oracle
from .sv_oracle import (apply_gate, apply_matrix, apply_ops, apply_to_group, circuit_unitary,
                        gate_matrix, group_indices, named_matrix, norm2, permute_qubits, probs, run)

__all__ = ["brute", "qaoa", "sv_oracle", "apply_gate", "apply_matrix", "apply_ops", "apply_to_group",
           "circuit_unitary", "gate_matrix", "group_indices", "named_matrix", "norm2",
           "permute_qubits", "probs", "run"]
