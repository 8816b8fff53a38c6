"""Brute-force full-matrix constructions (small N only) used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/sv_oracle.py).  These build the full
2^N x 2^N operator of a gate by a different route from the oracle's
reshape/moveaxis path, so that a mistake in either shows up as a mismatch:

  * ``kron_1q``      -- Eq. 2 as a Kronecker product I (x) G (x) I, with qubit q
                        at weight 2^q;
  * ``full_matrix``  -- Eq. 2/3 for any k: entry (i, j) is U[r(i), r(j)] when i
                        and j agree outside the gate's bits, else 0, with the
                        local index r built from integer bit masks.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def kron_1q(g: np.ndarray, q: int, n: int) -> np.ndarray:
    """I_{2^(n-1-q)} (x) G (x) I_{2^q}: qubit q is bit q of the index."""
    left = np.eye(1 << (n - 1 - q), dtype=np.complex128)
    right = np.eye(1 << q, dtype=np.complex128)
    return np.kron(np.kron(left, np.asarray(g, dtype=np.complex128)), right)


def local_index(i: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    k = len(qubits)
    r = np.zeros_like(i)
    for m, q in enumerate(qubits):
        r |= ((i >> q) & 1) << (k - 1 - m)
    return r


def full_matrix(u: np.ndarray, qubits: Sequence[int], n: int) -> np.ndarray:
    dim = 1 << n
    mask = 0
    for q in qubits:
        mask |= 1 << int(q)
    i = np.arange(dim, dtype=np.int64)
    ri = local_index(i, qubits)
    rest = i & ~mask
    same = rest[:, None] == rest[None, :]
    full = np.where(same, np.asarray(u, dtype=np.complex128)[ri[:, None], ri[None, :]], 0.0)
    return full.astype(np.complex128)


def brute_probs(psi: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """Marginal by explicit loop over every basis index (small N only)."""
    m = len(qubits)
    out = np.zeros(1 << m, dtype=np.float64)
    for i in range(psi.size):
        b = 0
        for r, q in enumerate(qubits):
            b |= ((i >> q) & 1) << (m - 1 - r)
        out[b] += abs(psi[i]) ** 2
    return out
