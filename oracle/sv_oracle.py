"""Plain CPU state-vector simulator in complex128 -- the parity oracle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library; the only thing
both sides consume is the seeded gate lists of ``svgen`` (plain data).

What it computes is the plain definition of the method (QueenV2, Sec. II-A):
  * the state is 2^N complex amplitudes a_i with |phi> = sum_i a_i |i>  (Eq. 1);
  * a one-qubit gate G on qubit q maps every amplitude pair whose indices
    differ only in bit q, (a_{..0_q..}, a_{..1_q..}), to G times that pair  (Eq. 2);
  * a k-qubit gate is a 2^k x 2^k matrix applied in the same way to every group
    of 2^k amplitudes that differ only in its k bits; the CNOT example fixes the
    row order 0_i0_j, 0_i1_j, 1_i0_j, 1_i1_j, i.e. the first-listed qubit is the
    most significant bit of the local index  (Eq. 3);
  * a circuit is its gates applied in order.
Gate fusion, in-cache grouping and qubit reordering (Sec. II-B, III) only
regroup this exact arithmetic, so the oracle applies gates one by one.

Readings where the paper is silent (all also listed in the design notes):
  * qubit q <-> bit q (weight 2^q) of the index; "i-th bit" counts from the LSB;
  * probability of |i> is |a_i|^2 (amplitudes are complex);
  * named gates are the textbook ones; RZ(t) = exp(-i t Z / 2) (global phase kept);
  * marginal probabilities: output index bit (m-1-r) <-> qubits[r] (qubits[0] = MSB).

Pins: every function here is checked in tests/test_oracle_pins.py against
something other than itself (the printed Eq. 3 matrix, Kronecker-product and
integer-mask brute force, closed forms, numpy's inverse FFT, scipy's matrix
exponential, invariants).  No function is "parity unpinned".
"""
from __future__ import annotations

import math
from typing import Iterable, Optional, Sequence

import numpy as np

_SQ2 = 1.0 / math.sqrt(2.0)


def n_qubits_of(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.ndim != 1 or (1 << n) != psi.size:
        raise ValueError("state length must be a power of two")
    return n


# ---------------------------------------------------------------- gate matrices
def named_matrix(kind: str, theta: float = 0.0) -> np.ndarray:
    """Textbook matrices of the named gates, in the local row order of Eq. 3
    (first qubit = most significant).  The paper defines only the generic G of
    Eq. 2 and the CNOT of Eq. 3; the rest are the standard definitions."""
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    e = np.exp
    if kind == "H":
        return np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=np.complex128)
    if kind == "X":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if kind == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if kind == "Z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if kind == "S":
        return np.array([[1, 0], [0, 1j]], dtype=np.complex128)
    if kind == "T":
        return np.array([[1, 0], [0, e(1j * math.pi / 4)]], dtype=np.complex128)
    if kind == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if kind == "RY":
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if kind == "RZ":
        return np.array([[e(-0.5j * theta), 0], [0, e(0.5j * theta)]], dtype=np.complex128)
    if kind == "P":
        return np.array([[1, 0], [0, e(1j * theta)]], dtype=np.complex128)
    if kind == "CNOT":   # Eq. 3, qubits (control, target)
        return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
    if kind == "CZ":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if kind == "SWAP":
        return np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
    if kind == "CPHASE":
        return np.diag([1, 1, 1, e(1j * theta)]).astype(np.complex128)
    if kind == "RZZ":
        a, b = e(-0.5j * theta), e(0.5j * theta)
        return np.diag([a, b, b, a]).astype(np.complex128)
    raise ValueError(f"no named matrix for {kind!r}")


def gate_matrix(gate) -> np.ndarray:
    if gate.kind == "MATRIX":
        return np.asarray(gate.matrix, dtype=np.complex128)
    return named_matrix(gate.kind, gate.theta)


# ---------------------------------------------------------------- application
def apply_matrix(psi: np.ndarray, u: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """Eq. 2 / Eq. 3 generalised to k qubits: every group of 2^k amplitudes that
    differ only in bits ``qubits`` is multiplied by ``u``; ``qubits[0]`` is the
    most significant bit of the group's local index.

    The state is viewed as an N-dimensional 2x...x2 array in which axis a holds
    bit N-1-a; the gate's axes are moved to the front in the order of
    ``qubits`` so that a row-major reshape to (2^k, rest) puts qubits[0] in the
    most significant position; then one matrix product."""
    n = n_qubits_of(psi)
    qubits = [int(q) for q in qubits]
    k = len(qubits)
    if u.shape != (1 << k, 1 << k):
        raise ValueError("matrix size does not match qubit count")
    if len(set(qubits)) != k or any(q < 0 or q >= n for q in qubits):
        raise ValueError(f"bad qubits {qubits} for N={n}")
    t = psi.reshape((2,) * n)
    axes = [n - 1 - q for q in qubits]
    t = np.moveaxis(t, axes, list(range(k)))
    shape = t.shape
    t = (np.asarray(u, dtype=np.complex128) @ t.reshape(1 << k, -1)).reshape(shape)
    t = np.moveaxis(t, list(range(k)), axes)
    return np.ascontiguousarray(t).reshape(-1)


def apply_gate(psi: np.ndarray, gate) -> np.ndarray:
    return apply_matrix(psi, gate_matrix(gate), gate.qubits)


def run(gates: Iterable, n: Optional[int] = None, psi0: Optional[np.ndarray] = None) -> np.ndarray:
    """A circuit is its gates applied in list order, starting from |0..0> unless
    ``psi0`` is given."""
    if psi0 is None:
        if n is None:
            raise ValueError("need n or psi0")
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1.0
    else:
        psi = np.array(psi0, dtype=np.complex128, copy=True)
    for g in gates:
        psi = apply_gate(psi, g)
    return psi


def apply_ops(psi: np.ndarray, ops: Iterable) -> np.ndarray:
    """Apply (qubits, matrix) pairs in order -- used to replay a fusion plan."""
    for qubits, u in ops:
        psi = apply_matrix(psi, np.asarray(u), qubits)
    return psi


def circuit_unitary(gates: Sequence, n: int) -> np.ndarray:
    """The 2^n x 2^n unitary of a gate list: column j is the circuit applied to
    basis state |j>.  (Small n only.)"""
    dim = 1 << n
    cols = []
    for j in range(dim):
        e = np.zeros(dim, dtype=np.complex128)
        e[j] = 1.0
        cols.append(run(gates, psi0=e))
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------- sampled groups
def group_indices(base: int, qubits: Sequence[int]) -> np.ndarray:
    """Indices of the 2^k amplitudes of one gate group (Eq. 2/3): base has zeros
    at every bit in ``qubits``; local index r sets bit qubits[m] to bit (k-1-m)
    of r."""
    k = len(qubits)
    idx = np.full(1 << k, int(base), dtype=np.int64)
    for r in range(1 << k):
        for m, q in enumerate(qubits):
            if (r >> (k - 1 - m)) & 1:
                idx[r] += 1 << int(q)
    return idx


def apply_to_group(u: np.ndarray, amps: np.ndarray) -> np.ndarray:
    """Eq. 2/3 for one group: the new amplitudes are u times the old ones."""
    return np.asarray(u, dtype=np.complex128) @ np.asarray(amps, dtype=np.complex128)


# ---------------------------------------------------------------- readout
def norm2(psi: np.ndarray) -> float:
    """Sum of |a_i|^2 (the normalisation condition of Sec. II-A)."""
    return float(np.vdot(psi, psi).real)


def probs(psi: np.ndarray, qubits: Optional[Sequence[int]] = None) -> np.ndarray:
    """Probability |a_i|^2 of each basis state (Eq. 1), or the marginal over
    ``qubits`` with output index bit (m-1-r) <-> qubits[r]."""
    n = n_qubits_of(psi)
    p = (psi.real ** 2 + psi.imag ** 2).astype(np.float64)
    if qubits is None:
        return p
    qubits = [int(q) for q in qubits]
    t = p.reshape((2,) * n)
    axes = [n - 1 - q for q in qubits]
    t = np.moveaxis(t, axes, list(range(len(qubits))))
    return t.reshape(1 << len(qubits), -1).sum(axis=1)


def permute_qubits(psi: np.ndarray, dest: Sequence[int]) -> np.ndarray:
    """Physical qubit reordering (Sec. II-B): the amplitude at index i moves to
    the index whose bit dest[q] equals bit q of i, for every q."""
    n = n_qubits_of(psi)
    dest = [int(d) for d in dest]
    if sorted(dest) != list(range(n)):
        raise ValueError("dest must be a permutation")
    t = psi.reshape((2,) * n)
    # new axis (n-1-dest[q]) takes old axis (n-1-q)
    src_axes = [n - 1 - q for q in range(n)]
    dst_axes = [n - 1 - dest[q] for q in range(n)]
    t = np.moveaxis(t, src_axes, dst_axes)
    return np.ascontiguousarray(t).reshape(-1)
