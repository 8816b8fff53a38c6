"""Pins for the CPU oracle: each check ties the oracle to something other than
itself -- the CNOT matrix printed in Eq. 3, Kronecker-product and integer-mask
brute force (Eq. 2/3), closed forms, numpy's inverse FFT (QFT), scipy's matrix
exponential (named rotations), and invariants.  The mutation tests at the end
plant plausible mistakes in copies of the oracle's routines and check that the
pins catch every one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import brute
from oracle import sv_oracle as so
from svgen import (Gate, basis_state_np, brickwork_circuit, fused_haar_circuit, gate_bench_set,
                   gaussian_state_np, haar_unitary, layered_circuit, qaoa_circuit, qft_circuit, random_matching)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)


def load_eq3():
    rows = []
    with open(os.path.join(GOLDEN, "eq3_cnot.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows, dtype=complex)


def rand_unitary(d, rng):
    return haar_unitary(d, rng)


# ------------------------------------------------------------- reusable pins
def pin_eq3(apply_fn):
    """CNOT(control=1, target=0) at N=2: column j of the operator is the
    image of basis state j and must equal Eq. 3 exactly; embedded at N=5 with
    spectators it must map x -> x xor 2^t when bit c of x is set."""
    eq3 = load_eq3()
    cnot = so.named_matrix("CNOT")
    if not np.array_equal(cnot, eq3):
        return False
    cols = [apply_fn(basis_state_np(2, j), cnot, [1, 0]) for j in range(4)]
    if not np.array_equal(np.stack(cols, axis=1), eq3):
        return False
    n = 5
    for c, t in [(3, 1), (0, 4), (2, 3), (4, 0)]:
        for x in range(1 << n):
            out = apply_fn(basis_state_np(n, x), cnot, [c, t])
            y = x ^ (1 << t) if (x >> c) & 1 else x
            if not np.array_equal(out, basis_state_np(n, y)):
                return False
    return True


def pin_kron(apply_fn, seed=11):
    rng = np.random.default_rng(seed)
    for n in range(1, 8):
        for q in range(n):
            g = rand_unitary(2, rng)
            psi = gaussian_state_np(n, int(rng.integers(1 << 30)))
            ref = brute.kron_1q(g, q, n) @ psi
            if np.max(np.abs(apply_fn(psi, g, [q]) - ref)) > 1e-14:
                return False
    return True


def pin_full(apply_fn, seed=12, ns=(6, 8), ks=(2, 3, 4, 5, 6)):
    rng = np.random.default_rng(seed)
    for n in ns:
        for k in ks:
            if k > n:
                continue
            for _ in range(2):
                qs = [int(x) for x in rng.choice(n, k, replace=False)]
                u = rand_unitary(1 << k, rng)
                psi = gaussian_state_np(n, int(rng.integers(1 << 30)))
                ref = brute.full_matrix(u, qs, n) @ psi
                if np.max(np.abs(apply_fn(psi, u, qs) - ref)) > 1e-13:
                    return False
    return True


# ------------------------------------------------------------- Eq. 3
def test_eq3_golden_and_oracle():
    assert pin_eq3(so.apply_matrix)


def test_eq3_rows_embedded_order():
    """Spectators in random basis states: the four amplitudes of the group,
    listed in the order 0_i0_j, 0_i1_j, 1_i0_j, 1_i1_j, transform by Eq. 3."""
    rng = np.random.default_rng(3)
    eq3 = load_eq3()
    n = 6
    for _ in range(20):
        i, j = (int(x) for x in rng.choice(n, 2, replace=False))
        psi = gaussian_state_np(n, int(rng.integers(1 << 30)))
        out = oracle.run([Gate("CNOT", (i, j))], psi0=psi)
        base = int(rng.integers(0, 1 << n)) & ~((1 << i) | (1 << j))
        idx = [base, base | (1 << j), base | (1 << i), base | (1 << i) | (1 << j)]
        assert np.array_equal(out[idx], eq3 @ psi[idx])


# ------------------------------------------------------------- Eq. 2, k-qubit
def test_eq2_against_kronecker():
    assert pin_kron(so.apply_matrix)


def test_kqubit_against_integer_mask_full_matrix():
    assert pin_full(so.apply_matrix)


def test_kqubit_n10_k6():
    assert pin_full(so.apply_matrix, seed=21, ns=(10,), ks=(6,))


def test_brute_forces_agree():
    rng = np.random.default_rng(4)
    for n in range(1, 7):
        for q in range(n):
            g = rand_unitary(2, rng)
            assert np.array_equal(brute.full_matrix(g, [q], n), brute.kron_1q(g, q, n))
    # two-qubit gate on adjacent bits equals a Kronecker product with the
    # first-listed qubit as the more significant factor
    u = rand_unitary(4, rng)
    n = 5
    for q in range(n - 1):
        kron = np.kron(np.kron(np.eye(1 << (n - 2 - q)), u), np.eye(1 << q))
        assert np.allclose(brute.full_matrix(u, [q + 1, q], n), kron, atol=1e-15)


def test_group_indices_and_apply_to_group():
    rng = np.random.default_rng(5)
    n = 9
    for k in (1, 2, 3, 5):
        qs = [int(x) for x in rng.choice(n, k, replace=False)]
        u = rand_unitary(1 << k, rng)
        psi = gaussian_state_np(n, 7)
        out = so.apply_matrix(psi, u, qs)
        mask = sum(1 << q for q in qs)
        for base in rng.integers(0, 1 << n, size=10):
            base = int(base) & ~mask
            idx = so.group_indices(base, qs)
            assert np.max(np.abs(out[idx] - so.apply_to_group(u, psi[idx]))) < 1e-15


# ------------------------------------------------------------- QAOA
@pytest.mark.parametrize("n", [4, 7])
def test_qaoa_level_closed_form(n):
    """One QAOA level on the complete graph as a closed form: the cost layer
    multiplies basis state x by exp(-i gamma E / 2), E = sum_{a<b} s_a s_b =
    (M^2 - n) / 2 with s = 1 - 2 x and M = sum s (the Ising energy of K_n);
    the mixer is the n-fold tensor power of exp(-i beta X).  Checked against
    the oracle's gate-by-gate run from |0...0>."""
    gates = qaoa_circuit(n, 1, seed=3)
    gamma, two_beta = gates[n].theta, gates[-1].theta
    assert [g.kind for g in gates].count("RZZ") == n * (n - 1) // 2
    x = np.arange(1 << n)
    pop = np.array([bin(int(v)).count("1") for v in x])
    mag = n - 2 * pop
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=complex) * np.exp(-0.25j * gamma * (mag * mag - n))
    mix = scipy.linalg.expm(-0.5j * two_beta * PX)
    u = np.ones((1, 1), dtype=complex)
    for _ in range(n):
        u = np.kron(u, mix)
    ref = u @ psi
    assert np.max(np.abs(oracle.run(gates, psi0=basis_state_np(n, 0)) - ref)) < 1e-13


@pytest.mark.parametrize("n,levels", [(3, 1), (6, 3), (9, 5)])
def test_qaoa_symmetric_closed_form(n, levels):
    """The symmetric-subspace closed form of the complete-graph QAOA state
    (used at full size) against the gate-by-gate oracle on every amplitude,
    for several levels; the H-only and the no-level cases are |+>^n."""
    from oracle import qaoa
    gates = qaoa_circuit(n, levels, seed=20 + n)
    lv = qaoa.levels_of(gates)
    assert len(lv) == levels
    amp = qaoa.weight_amplitudes(n, lv)
    pop = np.array([bin(i).count("1") for i in range(1 << n)])
    ref = oracle.run(gates, psi0=basis_state_np(n, 0))
    assert np.max(np.abs(amp[pop] - ref)) < 1e-13
    assert np.max(np.abs(qaoa.weight_amplitudes(n, []) - 2.0 ** (-n / 2))) < 1e-15


# ------------------------------------------------------------- named gates
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, math.pi, 5.9])
def test_rotations_are_matrix_exponentials(theta):
    for kind, p in (("RX", PX), ("RY", PY), ("RZ", PZ)):
        ref = scipy.linalg.expm(-0.5j * theta * p)
        assert np.max(np.abs(so.named_matrix(kind, theta) - ref)) < 1e-14
    zz = np.kron(PZ, PZ)
    assert np.max(np.abs(so.named_matrix("RZZ", theta) - scipy.linalg.expm(-0.5j * theta * zz))) < 1e-14
    p11 = np.diag([0, 0, 0, 1]).astype(complex)
    assert np.max(np.abs(so.named_matrix("CPHASE", theta) - scipy.linalg.expm(1j * theta * p11))) < 1e-14
    assert np.max(np.abs(so.named_matrix("P", theta)
                         - np.exp(0.5j * theta) * so.named_matrix("RZ", theta))) < 1e-14


def test_fixed_gate_identities():
    m = so.named_matrix
    assert np.allclose(m("H"), (PX + PZ) / math.sqrt(2), atol=1e-16)
    assert np.array_equal(m("X"), PX) and np.array_equal(m("Y"), PY) and np.array_equal(m("Z"), PZ)
    assert np.allclose(m("S") @ m("S"), PZ, atol=1e-16)
    assert np.allclose(m("T") @ m("T"), m("S"), atol=1e-15)
    h2 = np.kron(np.eye(2), m("H"))      # H on the target (second, less significant) qubit
    assert np.allclose(h2 @ m("CNOT") @ h2, m("CZ"), atol=1e-15)
    assert np.allclose(m("CPHASE", math.pi), m("CZ"), atol=1e-15)
    # SWAP = CNOT(a,b) CNOT(b,a) CNOT(a,b), as a circuit on 2 qubits
    for a, b in ((1, 0), (0, 1)):
        u = so.circuit_unitary([Gate("CNOT", (a, b)), Gate("CNOT", (b, a)), Gate("CNOT", (a, b))], 2)
        assert np.array_equal(u, so.circuit_unitary([Gate("SWAP", (a, b))], 2))


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 4, 11])
def test_hadamard_all_uniform(n):
    psi = oracle.run([Gate("H", (q,)) for q in range(n)], n=n)
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15


@pytest.mark.parametrize("n", [2, 5, 12])
def test_ghz(n):
    gates = [Gate("H", (0,))] + [Gate("CNOT", (0, q)) for q in range(1, n)]
    psi = oracle.run(gates, n=n)
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


def test_x_on_basis_is_exact_bitflip():
    n = 7
    rng = np.random.default_rng(6)
    for _ in range(30):
        x = int(rng.integers(0, 1 << n))
        q = int(rng.integers(0, n))
        out = oracle.run([Gate("X", (q,))], psi0=basis_state_np(n, x))
        assert np.array_equal(out, basis_state_np(n, x ^ (1 << q)))


def test_rz_phases_on_plus_state():
    n, theta = 6, 0.77
    gates = [Gate("H", (q,)) for q in range(n)] + [Gate("RZ", (q,), theta) for q in range(n)]
    psi = oracle.run(gates, n=n)
    x = np.arange(1 << n)
    ones = np.array([bin(v).count("1") for v in x])
    ref = 2.0 ** (-n / 2) * np.exp(-0.5j * theta * (n - ones)) * np.exp(0.5j * theta * ones)
    assert np.max(np.abs(psi - ref)) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 5, 9, 12])
def test_qft_is_scaled_inverse_fft(n):
    dim = 1 << n
    gates = qft_circuit(n)
    assert len(gates) == n + n * (n - 1) // 2 + n // 2
    psi = gaussian_state_np(n, 100 + n)
    ref = math.sqrt(dim) * np.fft.ifft(psi)
    assert np.max(np.abs(oracle.run(gates, psi0=psi) - ref)) < 1e-13
    for x in (0, 1, dim - 1, dim // 3):
        y = np.arange(dim)
        closed = np.exp(2j * math.pi * x * y / dim) / math.sqrt(dim)
        assert np.max(np.abs(oracle.run(gates, psi0=basis_state_np(n, x)) - closed)) < 1e-13


# ------------------------------------------------------------- invariants
def test_norm_preserved_layered():
    gates = layered_circuit(10, n_gates=200, seed=1)
    psi = oracle.run(gates, n=10)
    assert abs(so.norm2(psi) - 1.0) < 1e-14 * 200


def test_inverse_restores():
    rng = np.random.default_rng(8)
    n = 8
    psi = gaussian_state_np(n, 9)
    gates = fused_haar_circuit(n, 6, seed=10, ks=(3, 4))
    fwd = oracle.run(gates, psi0=psi)
    inv = [Gate("MATRIX", g.qubits, 0.0, g.matrix.conj().T) for g in reversed(gates)]
    assert np.max(np.abs(oracle.run(inv, psi0=fwd) - psi)) < 1e-13


def test_involutions_exact():
    n = 7
    psi = gaussian_state_np(n, 12)
    for g in (Gate("X", (3,)), Gate("CNOT", (2, 5)), Gate("SWAP", (0, 6)), Gate("CZ", (1, 4)),
              Gate("Z", (2,)), Gate("Y", (5,))):
        once = oracle.run([g], psi0=psi)
        assert np.array_equal(oracle.run([g], psi0=once), psi)
    h = Gate("H", (4,))
    assert np.max(np.abs(oracle.run([h, h], psi0=psi) - psi)) < 1e-15


def test_circuit_unitary_is_product_of_full_matrices():
    n = 4
    gates = layered_circuit(n, n_gates=12, seed=13)
    u = so.circuit_unitary(gates, n)
    ref = np.eye(1 << n, dtype=complex)
    for g in gates:
        ref = brute.full_matrix(so.gate_matrix(g), g.qubits, n) @ ref
    assert np.max(np.abs(u - ref)) < 1e-14
    assert np.max(np.abs(u.conj().T @ u - np.eye(1 << n))) < 1e-14


# ------------------------------------------------------------- readout
def test_probs_against_loop():
    rng = np.random.default_rng(14)
    n = 7
    psi = gaussian_state_np(n, 15)
    assert np.max(np.abs(so.probs(psi) - np.abs(psi) ** 2)) < 1e-17
    for m in (0, 1, 2, 4, 7):
        qs = [int(x) for x in rng.choice(n, m, replace=False)]
        assert np.max(np.abs(so.probs(psi, qs) - brute.brute_probs(psi, qs))) < 1e-15
    assert abs(so.norm2(psi) - 1.0) < 1e-14


def test_permute_qubits():
    rng = np.random.default_rng(16)
    n = 7
    psi = gaussian_state_np(n, 17)
    dest = [int(x) for x in rng.permutation(n)]
    out = so.permute_qubits(psi, dest)
    for i in range(1 << n):
        j = 0
        for q in range(n):
            j |= ((i >> q) & 1) << dest[q]
        assert out[j] == psi[i]
    inv = [0] * n
    for q, d in enumerate(dest):
        inv[d] = q
    assert np.array_equal(so.permute_qubits(out, inv), psi)
    qs = [0, 3, 5]
    assert np.allclose(so.probs(psi, qs), so.probs(out, [dest[q] for q in qs]), atol=1e-16)


# ------------------------------------------------------------- input generators
def test_generators_shapes():
    c1 = layered_circuit(16, n_gates=200, seed=1)
    assert len(c1) == 200
    kinds = [g.kind for g in c1]
    assert kinds[:16].count("CNOT") == 0 and kinds[16:24] == ["CNOT"] * 8
    c3 = brickwork_circuit(32, 40, seed=3)
    assert len(c3) == 1900
    assert len(qft_circuit(32)) == 544
    pairs = random_matching(15, np.random.default_rng(0))
    flat = [q for p in pairs for q in p]
    assert len(pairs) == 7 and len(set(flat)) == 14
    gb = gate_bench_set(30, seed=2)
    assert len(gb) == 7 * 30
    for g in gb:
        assert len(set(g.qubits)) == len(g.qubits)
    rng = np.random.default_rng(1)
    for d in (32, 64):
        u = haar_unitary(d, rng)
        assert np.max(np.abs(u.conj().T @ u - np.eye(d))) < 1e-13


# ------------------------------------------------------------- mutation tests
def _mut_transposed(psi, u, qs):
    return so.apply_matrix(psi, np.asarray(u).T, qs)


def _mut_lsb_first(psi, u, qs):
    return so.apply_matrix(psi, u, list(reversed(qs)))


def _mut_conj(psi, u, qs):
    return so.apply_matrix(psi, np.conj(u), qs)


def _mut_msb_bits(psi, u, qs):
    n = so.n_qubits_of(psi)
    return so.apply_matrix(psi, u, [n - 1 - q for q in qs])


def _mut_drop_offdiag(psi, u, qs):
    return so.apply_matrix(psi, np.diag(np.diag(u)), qs)


@pytest.mark.parametrize("mutant", [_mut_transposed, _mut_lsb_first, _mut_conj, _mut_msb_bits,
                                    _mut_drop_offdiag])
def test_pins_catch_planted_mistakes(mutant):
    caught = (not pin_eq3(mutant)) or (not pin_kron(mutant)) or (not pin_full(mutant, ns=(6,), ks=(2, 3)))
    assert caught, f"{mutant.__name__} slipped through every pin"


def test_qft_pin_catches_sign_mistake():
    n = 6
    psi = gaussian_state_np(n, 1)
    wrong = [Gate("CPHASE", g.qubits, -g.theta) if g.kind == "CPHASE" else g for g in qft_circuit(n)]
    ref = math.sqrt(1 << n) * np.fft.ifft(psi)
    assert np.max(np.abs(oracle.run(wrong, psi0=psi) - ref)) > 1e-3
