"""Closed form of the complete-graph QAOA state (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP path at full size;
never imported by the product package.

QAOA (the second workload family of QueenV2, Sec. IV) on the complete graph
K_n with one angle per layer: H on every qubit, then per level RZZ(gamma) on
every pair and RX(theta) on every qubit.  Every layer commutes with every
permutation of the qubits, and so does |+>^n, so the state stays in the
symmetric subspace spanned by the Dicke states |D_w> (the normalised sum of
the C(n, w) basis states of Hamming weight w).  In that (n+1)-dimensional
space:
  * the cost layer multiplies |D_w> by exp(-i gamma E_w / 2), where
    E_w = sum_{a<b} s_a s_b = ((n - 2w)^2 - n) / 2 with s = 1 - 2x (the
    eigenvalue of Z_a Z_b is s_a s_b, and RZZ(g) = exp(-i g Z Z / 2));
  * the mixer is exp(-i theta S / 2) with S = sum_a X_a, which maps |D_w> to
    sqrt((w+1)(n-w)) |D_{w+1}> + sqrt(w(n-w+1)) |D_{w-1}> (a basis state of
    weight w+1 is reached from w+1 states of weight w).
Basis state x then has amplitude c_{w(x)} / sqrt(C(n, w(x))).
Pinned against the gate-by-gate oracle at small n in tests/test_oracle_pins.py.
"""
import math

import numpy as np
import scipy.linalg


def weight_amplitudes(n, levels):
    """Amplitude of a basis state of each Hamming weight 0..n after the QAOA
    circuit; levels = [(gamma, theta), ...] (RZZ angle, RX angle)."""
    w = np.arange(n + 1)
    binom = np.array([math.comb(n, int(k)) for k in w], dtype=np.float64)
    c = np.sqrt(binom) * 2.0 ** (-n / 2)  # |+>^n in the Dicke basis
    s = np.zeros((n + 1, n + 1))
    for k in range(n):
        s[k + 1, k] = s[k, k + 1] = math.sqrt((k + 1) * (n - k))
    energy = ((n - 2 * w) ** 2 - n) / 2.0
    c = c.astype(np.complex128)
    for gamma, theta in levels:
        c = np.exp(-0.5j * gamma * energy) * c
        c = scipy.linalg.expm(-0.5j * theta * s) @ c
    return c / np.sqrt(binom)


def levels_of(gates):
    """(gamma, theta) per level of a complete-graph QAOA gate list (the first
    RZZ angle and the RX angle of each level)."""
    out = []
    gamma = None
    for g in gates:
        if g.kind == "RZZ" and gamma is None:
            gamma = g.theta
        elif g.kind == "RX" and gamma is not None:
            out.append((gamma, g.theta))
            gamma = None
    return out
