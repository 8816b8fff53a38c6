"""GPU parity of the in-cache tile passes (LDS stages, qubit relabeling, fused
write-back permutations) and of the plan modes, against the oracle."""
import math

import numpy as np
import pytest

import oracle
from svgen import (Gate, basis_state_np, brickwork_circuit, gaussian_state_np, haar_unitary, layered_circuit,
                   qaoa_circuit, qft_circuit)
from tests.gpu_util import TOL, max_err, to_device, to_host

pytestmark = pytest.mark.gpu

DTYPES = ["c128", "c64"]


@pytest.fixture(scope="module")
def sv():
    import paper_2409_14697_amd as sv
    return sv


def mixed_circuit(n, count, seed):
    """Every gate kind, random qubits (controls and phase bits anywhere)."""
    rng = np.random.default_rng(seed)
    kinds1 = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P"]
    kinds2 = ["CNOT", "CZ", "SWAP", "CPHASE", "RZZ"]
    out = []
    for _ in range(count):
        if rng.random() < 0.5:
            out.append(Gate(kinds1[int(rng.integers(len(kinds1)))], (int(rng.integers(n)),),
                            float(rng.uniform(0, 2 * math.pi))))
        else:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append(Gate(kinds2[int(rng.integers(len(kinds2)))], (a, b), float(rng.uniform(0, 2 * math.pi))))
    return out


def run_plan(sv, n, dtype, psi, gates, opts):
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.apply_circuit(gates, opts)
    st.sync()
    out = to_host(t)
    st.close()
    return out, oracle.run(gates, psi0=host_in)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 6, 9])
@pytest.mark.parametrize("circuit", ["mixed", "layered", "brickwork", "qft"])
def test_pass_mode_circuits(sv, dtype, lds, circuit):
    n = 14
    gates = {"mixed": lambda: mixed_circuit(n, 300, 7),
             "layered": lambda: layered_circuit(n, n_gates=200, seed=1),
             "brickwork": lambda: brickwork_circuit(n, 10, seed=3),
             "qft": lambda: qft_circuit(n)}[circuit]()
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 21), gates, {"mode": "pass", "lds_qubits": lds})
    assert max_err(out, ref) <= TOL[dtype]


def ladder_circuit(n, seed):
    """Runs of phases that share one qubit (the QFT's controlled-phase
    ladders, generalised): random angles, CPHASE / CZ with the shared qubit on
    either side and the other qubit anywhere, phase gates on the shared qubit,
    runs of 1-20 broken by H / RX gates."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(12):
        j = int(rng.integers(n))
        out.append(Gate("H", (j,)))
        for _ in range(int(rng.integers(1, 21))):
            r = rng.random()
            if r < 0.15:
                out.append(Gate("P", (j,), float(rng.uniform(-7, 7))))
            elif r < 0.25:
                k = int(rng.choice([q for q in range(n) if q != j]))
                out.append(Gate("CZ", (j, k) if rng.random() < 0.5 else (k, j)))
            else:
                k = int(rng.choice([q for q in range(n) if q != j]))
                out.append(Gate("CPHASE", (j, k) if rng.random() < 0.5 else (k, j), float(rng.uniform(-7, 7))))
        out.append(Gate("RX", (int(rng.integers(n)),), float(rng.uniform(0, 6))))
    return out


def diagonal_run_circuit(n, seed):
    """Dense gates on a few qubits, then runs of diagonal gates among the same
    qubits (register bits of the stage): CZ, CPHASE, RZZ, RZ, Z, S, T, P."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(10):
        qs = [int(x) for x in rng.choice(n, 5, replace=False)]
        out += [Gate("RY", (q,), float(rng.uniform(0, 6))) for q in qs]
        for _ in range(int(rng.integers(2, 12))):
            kind = ["CZ", "CPHASE", "RZZ", "RZ", "Z", "S", "T", "P"][int(rng.integers(8))]
            if kind in ("CZ", "CPHASE", "RZZ"):
                a, b = (int(x) for x in rng.choice(qs, 2, replace=False))
                out.append(Gate(kind, (a, b), float(rng.uniform(-7, 7))))
            else:
                out.append(Gate(kind, (int(rng.choice(qs)),), float(rng.uniform(-7, 7))))
    return out


def phase_run_circuit(n, seed):
    """Runs of 3-60 phase gates on any qubits (RZZ, CPHASE, CZ, RZ, P, S, T, Z
    and random diagonal unitaries on one or two qubits), each run after H / RY
    gates on four random qubits, so that the run's qubits fall in registers,
    in the tile outside the registers and outside the tile."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(8):
        for q in rng.choice(n, 4, replace=False):
            out.append(Gate("H", (int(q),)) if rng.random() < 0.5 else Gate("RY", (int(q),), float(rng.uniform(0, 6))))
        for _ in range(int(rng.integers(3, 61))):
            kind = ["RZZ", "CPHASE", "CZ", "RZ", "P", "S", "T", "Z", "D1", "D2"][int(rng.integers(10))]
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            if kind == "D1":
                out.append(Gate("MATRIX", (a,), matrix=np.diag(np.exp(1j * rng.uniform(-7, 7, 2)))))
            elif kind == "D2":
                out.append(Gate("MATRIX", (a, b), matrix=np.diag(np.exp(1j * rng.uniform(-7, 7, 4)))))
            elif kind in ("RZZ", "CPHASE", "CZ"):
                out.append(Gate(kind, (a, b), float(rng.uniform(-7, 7))))
            else:
                out.append(Gate(kind, (a,), float(rng.uniform(-7, 7))))
    return out


def interleaved_phase_circuit(n, count, seed):
    """Two-qubit phase gates (RZZ, CPHASE, CZ) and RZ interleaved with H / RX
    on random qubits, so that runs of phase gates form only after the phase
    gates are moved past the gates on other qubits."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        r = rng.random()
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        if r < 0.6:
            out.append(Gate(["RZZ", "CPHASE", "CZ"][int(rng.integers(3))], (a, b), float(rng.uniform(-7, 7))))
        elif r < 0.7:
            out.append(Gate("RZ", (a,), float(rng.uniform(-7, 7))))
        elif r < 0.85:
            out.append(Gate("H", (a,)))
        else:
            out.append(Gate("RX", (a,), float(rng.uniform(0, 6))))
    return out


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 8])
def test_phase_gates_reordered(sv, dtype, lds):
    """Phase gates gathered past the gates they commute with (other qubits)
    and fused, against the oracle."""
    n = 15
    gates = interleaved_phase_circuit(n, 400, 8)
    opts = {"mode": "pass", "lds_qubits": lds}
    assert sum(lad for _, lad in sv.Plan(n, dtype, gates, opts).kernel_ops()) > 0
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 47), gates, opts)
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 7, 10])
@pytest.mark.parametrize("seed", [3, 4])
def test_phase_runs(sv, dtype, lds, seed):
    """Runs of phase gates fused into ladders, register factors and one
    quadratic phase over the other bits, against the oracle; the plan holds
    fused phase ops."""
    n = 15
    gates = phase_run_circuit(n, seed)
    opts = {"mode": "pass", "lds_qubits": lds}
    plan = sv.Plan(n, dtype, gates, opts)
    assert sum(lad for _, lad in plan.kernel_ops()) > 0
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 43 + seed), gates, opts)
    assert max_err(out, ref) <= TOL[dtype]


def single_qubit_layers(n, depth, family, seed):
    """Layers of single-qubit gates on every qubit (the family fixes which
    2x2 form a register stage needs: real, real-diagonal/imaginary
    off-diagonal, both mixed, or general complex), each followed by CNOTs
    on a random disjoint matching."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(depth):
        for q in range(n):
            th = float(rng.uniform(0, 2 * math.pi))
            if family == "real":
                kind = ("H", "RY")[int(rng.integers(2))]
            elif family == "imag":
                kind = ("RX", "Y")[int(rng.integers(2))]
            elif family == "mixed":
                kind = ("H", "RY", "RX", "Y")[int(rng.integers(4))]
            else:
                out.append(Gate("MATRIX", (q,), matrix=haar_unitary(2, rng)))
                continue
            out.append(Gate(kind, (q,), th))
        p = rng.permutation(n)
        out += [Gate("CNOT", (int(p[2 * i]), int(p[2 * i + 1]))) for i in range(n // 2)]
    return out


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("family", ["real", "imag", "mixed", "haar"])
@pytest.mark.parametrize("lds", list(range(4, 14)))
def test_tensor_product_layers(sv, dtype, family, lds):
    """A layer of single-qubit gates is applied by a register stage as the
    tensor product of one 2x2 per register bit (Sec. III-A's tensor product
    booster, own design); random layers of each form mixed with CNOTs at
    N=14, every tile size, against the oracle."""
    rb = 4 if dtype == "c128" else 5
    m_max = 12 if dtype == "c128" else 13
    if lds < rb or lds > m_max:
        pytest.skip("tile size outside this dtype's range")
    n = 14
    gates = single_qubit_layers(n, 6, family, seed=31 + lds)
    plan = sv.Plan(n, dtype, gates, {"mode": "pass", "lds_qubits": lds})
    # several single-qubit gates per stage: fewer stages than such gates
    stages = sum(p[3] for p in plan.passes(stages=True))
    plan.close()
    assert stages < 6 * n
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 5), gates, {"mode": "pass", "lds_qubits": lds})
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_phase_runs_across_permutations(sv, dtype):
    """Forty runs of RZZ on all pairs of qubits 2..15, each closed by CNOTs
    from every one of those qubits onto qubit 1.  A phase gate on a CNOT's
    control commutes with it, so a stage applies all forty runs as one fused
    phase before its register permutation: a few fixed-point items, not one
    item per gate; against the oracle."""
    n = 16
    rng = np.random.default_rng(12)
    gates = [Gate("H", (q,)) for q in range(n)]
    for _ in range(40):
        for a in range(2, n):
            for b in range(a + 1, n):
                gates.append(Gate("RZZ", (a, b), float(rng.uniform(-3, 3))))
        gates += [Gate("CNOT", (c, 1)) for c in range(2, n)]
    opts = {"mode": "pass"}
    kops, ladders = sv.Plan(n, dtype, gates, opts).kernel_ops()[-1]
    # the 560 CNOTs count one each; the 3640 phase gates a handful
    assert ladders > 0 and kops <= 560 + 20
    out, ref = run_plan(sv, n, dtype, basis_state_np(n, 0), gates, opts)
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 6, 9])
def test_qaoa_complete_graph(sv, dtype, lds):
    """Five QAOA levels on K_n from |0...0> (the H layer prepares |+>): every
    ZZ layer is one run of phase gates."""
    n = 16
    gates = qaoa_circuit(n, 5, seed=11)
    out, ref = run_plan(sv, n, dtype, basis_state_np(n, 0), gates, {"mode": "pass", "lds_qubits": lds})
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 8])
def test_register_diagonal_runs(sv, dtype, lds):
    """Runs of diagonal gates on register bits (one factor per register index)
    against the oracle."""
    n = 14
    gates = diagonal_run_circuit(n, 9)
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 41), gates, {"mode": "pass", "lds_qubits": lds})
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 7, 10])
@pytest.mark.parametrize("seed", [1, 2])
def test_phase_ladders(sv, dtype, lds, seed):
    """Phase ladders (one fixed-point angle sum per lane and tile) against the
    oracle, with the shared qubit's partners in registers, in the tile and
    outside it."""
    n = 15
    gates = ladder_circuit(n, seed)
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 30 + seed), gates, {"mode": "pass", "lds_qubits": lds})
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_pass_whole_state_tile(sv, dtype):
    """N at or below the tile size: one tile holds the whole state."""
    for n in (5, 9, 12):
        gates = mixed_circuit(n, 120, n)
        out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 2), gates, {"mode": "pass"})
        assert max_err(out, ref) <= TOL[dtype], n


@pytest.mark.parametrize("dtype", DTYPES)
def test_pass_permutation_exact(sv, dtype):
    """Only X, CNOT and SWAP: permutations of amplitudes, bitwise exact."""
    n = 15
    rng = np.random.default_rng(5)
    gates = []
    for _ in range(200):
        k = int(rng.integers(3))
        if k == 0:
            gates.append(Gate("X", (int(rng.integers(n)),)))
        else:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            gates.append(Gate("CNOT" if k == 1 else "SWAP", (a, b)))
    out, ref = run_plan(sv, n, dtype, gaussian_state_np(n, 3), gates, {"mode": "pass", "lds_qubits": 8})
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_qft_pass_mode_n20(sv, dtype):
    n = 20
    psi = gaussian_state_np(n, 9)
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.apply_circuit(qft_circuit(n), {"mode": "pass"})
    st.sync()
    ref = math.sqrt(1 << n) * np.fft.ifft(host_in)
    assert max_err(to_host(t), ref) <= TOL[dtype]
    st.close()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("mode", ["auto", "sweep", "pass"])
def test_modes_agree_layered_n16(sv, dtype, mode):
    n = 16
    gates = layered_circuit(n, n_gates=200, seed=1)
    out, ref = run_plan(sv, n, dtype, basis_state_np(n, 0), gates, {"mode": mode})
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_permute_qubits_bitwise(sv, dtype):
    """sv_permute_qubits against the oracle's index-bit permutation: random
    permutations, a reversal, a cyclic shift and the identity; bitwise."""
    from paper_2409_14697_amd import binding as B
    rng = np.random.default_rng(17)
    for n in (1, 2, 4, 5, 6, 9, 13, 14, 17, 20):
        perms = [list(rng.permutation(n)) for _ in range(2)]
        perms += [list(range(n - 1, -1, -1)), [(q + 1) % n for q in range(n)], list(range(n))]
        for dest in perms:
            t, host_in = to_device(gaussian_state_np(n, n), dtype)
            st = sv.StateVector(n, dtype, tensor=t, init=False)
            st.permute_qubits(dest)
            st.sync()
            ref = oracle.permute_qubits(host_in, dest)
            assert np.array_equal(to_host(t), ref), (n, dest)
            st.close()
    st = sv.StateVector(5, dtype)
    for bad in ([0, 1, 2, 3, 3], [0, 1, 2, 3, 5], [0, 1, 2, 3, -1]):
        with pytest.raises(B.SvError) as e:
            st.permute_qubits(bad)
        assert e.value.status == B.SV_ERR_QUBIT
    st.close()
