"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element
by element, on seeded inputs.  Bars: max |psi_gpu - psi_oracle| <= 1e-12 for
complex128 and <= 1e-5 for complex64; permutation and sign gates (X, CNOT,
SWAP, CZ) bitwise.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import sv_oracle as so
from svgen import (Gate, basis_state_np, brickwork_circuit, fused_haar_circuit, gaussian_state_np, haar_unitary,
                   layered_circuit, qft_circuit)
from tests.gpu_util import TOL, max_err, to_device, to_host

pytestmark = pytest.mark.gpu

DTYPES = ["c128", "c64"]
ONE_Q = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P"]
TWO_Q = ["CNOT", "CZ", "SWAP", "CPHASE", "RZZ"]
EXACT = {"X", "CNOT", "SWAP", "CZ"}


@pytest.fixture(scope="module")
def sv():
    import paper_2409_14697_amd as sv
    return sv


def run_gates(sv, n, dtype, psi, gates, circuit=False, opts=None):
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    if circuit:
        st.apply_circuit(gates, opts)
    else:
        for g in gates:
            st.apply_gate(g)
    st.sync()
    out = to_host(t)
    st.close()
    return out, oracle.run(gates, psi0=host_in)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 3, 9, 13])
def test_one_qubit_gates_every_target(sv, dtype, n):
    rng = np.random.default_rng(100 + n)
    psi = gaussian_state_np(n, 7 + n)
    for kind in ONE_Q:
        for t in range(n):
            g = Gate(kind, (t,), float(rng.uniform(0, 2 * math.pi)))
            out, ref = run_gates(sv, n, dtype, psi, [g])
            if kind in EXACT:
                assert np.array_equal(out, ref), (kind, t)
            else:
                assert max_err(out, ref) <= TOL[dtype], (kind, t, max_err(out, ref))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [2, 5, 11])
def test_two_qubit_gates_every_pair(sv, dtype, n):
    rng = np.random.default_rng(200 + n)
    psi = gaussian_state_np(n, 17 + n)
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    if len(pairs) > 40:
        pairs = [pairs[i] for i in rng.choice(len(pairs), 40, replace=False)] + [(0, 1), (1, 0), (0, n - 1),
                                                                                 (n - 1, 0)]
    for kind in TWO_Q:
        for a, b in pairs:
            g = Gate(kind, (a, b), float(rng.uniform(0, 2 * math.pi)))
            out, ref = run_gates(sv, n, dtype, psi, [g])
            if kind in EXACT:
                assert np.array_equal(out, ref), (kind, a, b)
            else:
                assert max_err(out, ref) <= TOL[dtype], (kind, a, b, max_err(out, ref))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_dense_matrix_gates(sv, dtype, k):
    rng = np.random.default_rng(300 + k)
    for n in (k, k + 3, 14):
        psi = gaussian_state_np(n, 3 + n)
        for _ in range(3):
            qs = tuple(int(x) for x in rng.choice(n, k, replace=False))
            g = Gate("MATRIX", qs, matrix=haar_unitary(1 << k, rng))
            out, ref = run_gates(sv, n, dtype, psi, [g])
            assert max_err(out, ref) <= TOL[dtype], (n, qs, max_err(out, ref))


@pytest.mark.parametrize("dtype", DTYPES)
def test_dense_low_and_high_bits(sv, dtype):
    """Gate bits at the bottom (coalescing edge), at the top, and both."""
    n = 15
    rng = np.random.default_rng(5)
    psi = gaussian_state_np(n, 2)
    for qs in ((0, 1, 2), (2, 0, 1), (14, 13, 12, 11, 10), (0, 14, 7, 1, 13, 3), (5, 4, 3, 2, 1, 0)):
        g = Gate("MATRIX", qs, matrix=haar_unitary(1 << len(qs), rng))
        out, ref = run_gates(sv, n, dtype, psi, [g])
        assert max_err(out, ref) <= TOL[dtype], qs


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kmax", [0, 5])
def test_layered_circuit_n16(sv, dtype, kmax):
    """N=16, 200 gates from |0..0> (layers of H/RX/RY/RZ alternating with CNOTs
    on random disjoint pairs)."""
    n = 16
    gates = layered_circuit(n, n_gates=200, seed=1)
    out, ref = run_gates(sv, n, dtype, basis_state_np(n, 0), gates, circuit=True,
                         opts={"max_fuse_qubits": kmax})
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_layered_gate_by_gate_n16(sv, dtype):
    n = 16
    gates = layered_circuit(n, n_gates=200, seed=1)
    out, ref = run_gates(sv, n, dtype, basis_state_np(n, 0), gates)
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [14, 24])
def test_qft_against_inverse_fft(sv, dtype, n):
    psi = gaussian_state_np(n, 9)
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.apply_circuit(qft_circuit(n))
    st.sync()
    ref = math.sqrt(1 << n) * np.fft.ifft(host_in)
    assert max_err(to_host(t), ref) <= TOL[dtype]


_BENCH_REF = {}


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("circuit", ["brickwork_d40", "qft"])
def test_circuit_benchmark_generators_n20(sv, dtype, circuit):
    """The circuit benchmark's generators (brickwork depth 40, seed 3; QFT) at
    N=20 in plan mode auto (fused MFMA sweeps, tile passes with phase ladders
    and register-diagonal runs), against the oracle on a Gaussian state."""
    n = 20
    gates = brickwork_circuit(n, 40, seed=3) if circuit == "brickwork_d40" else qft_circuit(n)
    psi = gaussian_state_np(n, 13)
    t, host_in = to_device(psi, dtype)
    key = (circuit, dtype)
    if key not in _BENCH_REF:
        _BENCH_REF[key] = oracle.run(gates, psi0=host_in)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.apply_circuit(gates, {"mode": "auto"})
    st.sync()
    assert max_err(to_host(t), _BENCH_REF[key]) <= TOL[dtype]
    st.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_haar_fused_circuit(sv, dtype):
    n = 12
    gates = fused_haar_circuit(n, 12, seed=4)
    out, ref = run_gates(sv, n, dtype, gaussian_state_np(n, 4), gates, circuit=True)
    assert max_err(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_create_init_and_basis(sv, dtype):
    import torch
    n = 10
    st = sv.StateVector(n, dtype)
    st.sync()
    assert np.array_equal(to_host(st.tensor), basis_state_np(n, 0))
    st.init_basis(777)
    st.sync()
    assert np.array_equal(to_host(st.tensor), basis_state_np(n, 777))
    st.close()
    import ctypes  # library-owned buffer through the raw ABI
    from paper_2409_14697_amd import binding as B
    h = ctypes.c_void_p()
    B.check(B.load_library().sv_create(12, B.SV_C128 if dtype == "c128" else B.SV_C64, None, None, 0,
                                       ctypes.byref(h)))
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    B.check(B.load_library().sv_measure_probs(h, None, 0, ctypes.c_void_p(out.data_ptr())))
    B.check(B.load_library().sv_sync(h))
    assert out.item() == 1.0
    B.check(B.load_library().sv_destroy(h))


@pytest.mark.parametrize("dtype", DTYPES)
def test_probs_and_norm(sv, dtype):
    rng = np.random.default_rng(12)
    for n in (3, 9, 18):
        psi = gaussian_state_np(n, n)
        t, host_in = to_device(psi, dtype)
        st = sv.StateVector(n, dtype, tensor=t, init=False)
        subsets = [[], list(range(n - 1, -1, -1)), [0], [n - 1], list(range(min(n, 16) - 1, -1, -1))]
        for m in (1, 2, min(n, 5)):
            subsets.append([int(x) for x in rng.choice(n, m, replace=False)])
        for qs in subsets:
            p1 = st.measure_probs(qs).cpu().numpy()
            p2 = st.measure_probs(qs).cpu().numpy()
            assert np.array_equal(p1, p2)  # fixed summation order
            ref = so.probs(host_in, qs) if qs else np.array([so.norm2(host_in)])
            assert np.max(np.abs(p1 - ref)) <= 1e-12, (n, qs)
        st.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_scale(sv, dtype):
    n = 11
    psi = gaussian_state_np(n, 1)
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.scale(0.5)
    st.sync()
    assert np.array_equal(to_host(t), host_in * 0.5)
    st.close()


def test_invalid_gate_leaves_state_untouched(sv):
    n = 6
    psi = gaussian_state_np(n, 3)
    t, host_in = to_device(psi, "c128")
    st = sv.StateVector(n, "c128", tensor=t, init=False)
    with pytest.raises(sv.SvError):
        st.apply_gate(Gate("H", (6,)))
    with pytest.raises(sv.SvError):
        st.apply_circuit([Gate("H", (0,)), Gate("CNOT", (2, 2))])
    st.sync()
    assert np.array_equal(to_host(t), host_in)
    st.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_degenerate_inputs(sv, dtype):
    """Empty circuits and plans change nothing; a state that is all zeros stays
    zero under renormalisation; n above the maximum is rejected."""
    from paper_2409_14697_amd import binding as B
    n = 7
    t, host_in = to_device(gaussian_state_np(n, 5), dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    before = to_host(t)
    for mode in ("auto", "sweep", "pass"):
        st.apply_circuit([], {"mode": mode})
    st.apply_plan(sv.Plan(n, dtype, [], {"mode": "pass"}))
    st.sync()
    assert np.array_equal(to_host(t), before)
    t.zero_()
    st.apply_circuit([Gate("MATRIX", (0, 1, 2), matrix=np.eye(8))],
                     {"mode": "sweep", "max_fuse_qubits": 0, "renorm_interval": 1})
    st.sync()
    assert np.array_equal(to_host(t), np.zeros(1 << n))
    st.close()
    import ctypes
    h = ctypes.c_void_p()
    code = B.SV_C128 if dtype == "c128" else B.SV_C64
    assert B.load_library().sv_create(35, code, None, None, 0, ctypes.byref(h)) == B.SV_ERR_ARG  # before allocating
    assert B.load_library().sv_create(0, code, None, None, 0, ctypes.byref(h)) == B.SV_ERR_ARG
