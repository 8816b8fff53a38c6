"""Seeded gate-list generators (plain data; no gate arithmetic).

Qubit convention used throughout: qubit q is bit q (weight 2**q) of the state
index.  For a multi-qubit gate, ``qubits[0]`` is the most significant bit of the
gate's local matrix index, the row order printed for the CNOT example of
Sec. II-A (Eq. 3): rows 0_i0_j, 0_i1_j, 1_i0_j, 1_i1_j for qubits (i, j).
CNOT is (control, target).

Workloads (synthetic stand-ins for the paper's gate and circuit benchmarks of
Sec. IV; no dataset is involved):
  * ``layered_circuit``   -- layers of H/RX/RY/RZ on every qubit alternating
                             with CNOTs on a random disjoint matching
  * ``brickwork_circuit`` -- RX/RY/RZ on every qubit + CNOT brickwork
  * ``qft_circuit``       -- textbook QFT (the circuit family of Sec. IV-C)
  * ``fused_haar_circuit``-- Haar-random 5- and 6-qubit unitaries
  * ``gate_bench_set``    -- one gate per (kind, target) for the per-gate sweep
                             benchmark (the gate benchmark of Sec. IV-B)
  * ``serving_requests``  -- request stream for the continuous-batching loop
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

# Gate kinds understood by both the oracle and the library.  Parameterised
# kinds read ``theta`` (radians).  'MATRIX' carries an explicit 2^k x 2^k
# complex unitary; any other gate can be supplied that way (Sec. III-B: special
# gates are generated from the unitaries the simulator supports).
GATE_KINDS = ("MATRIX", "H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P",
              "CNOT", "CZ", "SWAP", "CPHASE", "RZZ")
_ARITY = {"H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "T": 1, "RX": 1, "RY": 1, "RZ": 1,
          "P": 1, "CNOT": 2, "CZ": 2, "SWAP": 2, "CPHASE": 2, "RZZ": 2}


@dataclass(eq=False)
class Gate:
    kind: str
    qubits: tuple
    theta: float = 0.0
    matrix: Optional[np.ndarray] = field(default=None, repr=False)

    def __post_init__(self):
        if self.kind not in GATE_KINDS:
            raise ValueError(f"unknown gate kind {self.kind!r}")
        self.qubits = tuple(int(q) for q in self.qubits)
        if self.kind == "MATRIX":
            if self.matrix is None:
                raise ValueError("MATRIX gate needs a matrix")
            d = 1 << len(self.qubits)
            m = np.asarray(self.matrix, dtype=np.complex128)
            if m.shape != (d, d):
                raise ValueError(f"matrix shape {m.shape} != {(d, d)}")
            self.matrix = m
        elif len(self.qubits) != _ARITY[self.kind]:
            raise ValueError(f"{self.kind} takes {_ARITY[self.kind]} qubits, got {self.qubits}")


def random_matching(n: int, rng: np.random.Generator):
    """Disjoint random qubit pairs (p[2m], p[2m+1]) from a permutation of range(n)."""
    p = rng.permutation(n)
    return [(int(p[2 * m]), int(p[2 * m + 1])) for m in range(n // 2)]


def layered_circuit(n: int, n_gates: Optional[int] = None, n_layer_pairs: Optional[int] = None,
                    seed: int = 1, rng: Optional[np.random.Generator] = None):
    """Rotation layer (each qubit: kind ~ U{H,RX,RY,RZ}, theta ~ U[0,2pi)) then a
    CNOT layer on a random disjoint matching (control = first of the pair),
    repeated.  Either truncated at exactly ``n_gates`` gates or ``n_layer_pairs``
    full (rotation, CNOT) layer pairs."""
    if rng is None:
        rng = np.random.default_rng(seed)
    if (n_gates is None) == (n_layer_pairs is None):
        raise ValueError("give exactly one of n_gates / n_layer_pairs")
    kinds = ("H", "RX", "RY", "RZ")
    gates = []
    pairs_done = 0
    while True:
        if n_layer_pairs is not None and pairs_done == n_layer_pairs:
            break
        ks = rng.integers(0, 4, size=n)
        ths = rng.uniform(0.0, 2.0 * math.pi, size=n)
        for q in range(n):
            kind = kinds[int(ks[q])]
            gates.append(Gate(kind, (q,), float(ths[q]) if kind != "H" else 0.0))
        for c, t in random_matching(n, rng):
            gates.append(Gate("CNOT", (c, t)))
        pairs_done += 1
        if n_gates is not None and len(gates) >= n_gates:
            return gates[:n_gates]
    return gates


def brickwork_circuit(n: int, depth: int, seed: int = 3):
    """Random layered circuit: every layer applies RX/RY/RZ (kind uniform,
    theta ~ U[0,2pi)) to all qubits, then CNOT brickwork -- pairs (2m, 2m+1) on
    even layers and (2m+1, 2m+2) on odd layers."""
    rng = np.random.default_rng(seed)
    kinds = ("RX", "RY", "RZ")
    gates = []
    for layer in range(depth):
        for q in range(n):
            kind = kinds[int(rng.integers(0, 3))]
            gates.append(Gate(kind, (q,), float(rng.uniform(0.0, 2.0 * math.pi))))
        start = layer % 2
        for a in range(start, n - 1, 2):
            gates.append(Gate("CNOT", (a, a + 1)))
    return gates


def qft_circuit(n: int):
    """Textbook quantum Fourier transform without approximation: for j from the
    top qubit down, H(j) then CPHASE(pi / 2^(j-k)) on (k, j) for k = j-1..0;
    finally SWAP(q, n-1-q).  Every controlled phase is kept, however small."""
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("H", (j,)))
        for k in range(j - 1, -1, -1):
            gates.append(Gate("CPHASE", (k, j), math.pi / float(1 << (j - k))))
    for q in range(n // 2):
        gates.append(Gate("SWAP", (q, n - 1 - q)))
    return gates


def qaoa_circuit(n: int, levels: int = 5, seed: int = 7):
    """QAOA on the complete graph K_n: H on every qubit, then per level a
    cost layer RZZ(gamma) on every pair (a, b), a < b, in lexicographic order,
    and a mixer layer RX(beta) on every qubit.  gamma ~ U[0, pi), beta ~
    U[0, pi/2) per level, drawn from the seed."""
    rng = np.random.default_rng(seed)
    gates = [Gate("H", (q,)) for q in range(n)]
    for _ in range(levels):
        gamma = float(rng.uniform(0.0, math.pi))
        beta = float(rng.uniform(0.0, 0.5 * math.pi))
        for a in range(n):
            for b in range(a + 1, n):
                gates.append(Gate("RZZ", (a, b), gamma))
        for q in range(n):
            gates.append(Gate("RX", (q,), 2.0 * beta))
    return gates


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random d x d unitary: QR of a complex Gaussian matrix with the phases
    of R's diagonal moved into Q (Mezzadri's correction)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[np.newaxis, :]


def fused_haar_circuit(n: int, n_gates: int, seed: int = 4, ks: Sequence[int] = (5, 6)):
    """Alternating k-qubit Haar-random unitaries (k cycles through ``ks``) on
    ordered random qubit sets ``rng.choice(n, k, replace=False)``."""
    rng = np.random.default_rng(seed)
    gates = []
    for g in range(n_gates):
        k = ks[g % len(ks)]
        qs = tuple(int(x) for x in rng.choice(n, k, replace=False))
        gates.append(Gate("MATRIX", qs, 0.0, haar_unitary(1 << k, rng)))
    return gates


GATE_BENCH_KINDS = ("H", "X", "RZ", "CNOT", "CZ", "SWAP", "CPHASE")


def gate_bench_set(n: int = 30, seed: int = 2, kinds: Sequence[str] = GATE_BENCH_KINDS):
    """One gate per (kind, target t in 0..n-1).  Two-qubit gates draw their
    partner uniformly from the other qubits: the CNOT control, the other
    CZ/CPHASE qubit, or the other SWAP qubit.  Angles ~ U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for kind in kinds:
        for t in range(n):
            theta = 0.0
            if kind in ("RZ", "CPHASE"):
                theta = float(rng.uniform(0.0, 2.0 * math.pi))
            if kind in ("CNOT", "CZ", "SWAP", "CPHASE"):
                p = int(rng.integers(0, n - 1))
                p = p + 1 if p >= t else p
                qs = (p, t) if kind == "CNOT" else (t, p)
            else:
                qs = (t,)
            out.append(Gate(kind, qs, theta))
    return out


@dataclass
class Request:
    """One circuit request of the serving workload."""
    rid: int
    n: int
    depth: int            # number of (rotation, CNOT) layer pairs
    seed: int             # seed of this request's circuit
    arrival_unit: float   # cumulative arrival time at rate 1 (scale by 1/lambda)

    def circuit(self):
        rng = np.random.default_rng(self.seed)
        return layered_circuit(self.n, n_layer_pairs=self.depth, rng=rng)


def serving_requests(count: int = 4096, seed: int = 5, n_range=(12, 26), depth_range=(20, 200)):
    """Request stream: n ~ U{n_range}, depth ~ U{depth_range} layer pairs, one
    circuit seed per request (SeedSequence(seed).spawn), Poisson arrivals at
    unit rate (exponential gaps; the caller scales time by 1/rate)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    ds = rng.integers(depth_range[0], depth_range[1] + 1, size=count)
    gaps = rng.exponential(1.0, size=count)
    arr = np.cumsum(gaps) - gaps[0]
    seeds = [int(s.generate_state(1)[0]) for s in np.random.SeedSequence(seed).spawn(count)]
    return [Request(i, int(ns[i]), int(ds[i]), seeds[i], float(arr[i])) for i in range(count)]
