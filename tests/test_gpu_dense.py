"""GPU parity of the dense k-qubit kernels: FP64 MFMA (complex128), FP32 VALU
and FP32 MFMA (complex64), and the FP64 renormalisation of complex64 plans."""
import numpy as np
import pytest

import oracle
from svgen import Gate, fused_haar_circuit, gaussian_state_np, haar_unitary
from tests.gpu_util import TOL, max_err, to_device, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    import paper_2409_14697_amd as sv
    return sv


def run(sv, n, dtype, psi, gates, opts):
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.apply_circuit(gates, opts)
    st.sync()
    out = to_host(t)
    norm2 = st.norm2()
    st.close()
    return out, oracle.run(gates, psi0=host_in), norm2


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("variant", ["c128", "c64-valu", "c64-mfma"])
def test_dense_kernel_variants(sv, k, variant):
    dtype = "c128" if variant == "c128" else "c64"
    opts = {"mode": "sweep", "max_fuse_qubits": 0, "fp32_mfma": 1 if variant == "c64-mfma" else 0}
    rng = np.random.default_rng(40 + k)
    for n in (k, k + 4, 15):
        placements = [tuple(int(x) for x in rng.choice(n, k, replace=False)) for _ in range(3)]
        placements.append(tuple(range(k - 1, -1, -1)))          # the lowest bits, MSB first
        placements.append(tuple(range(n - k, n)))                # the highest bits, LSB first
        for qs in placements:
            g = Gate("MATRIX", qs, matrix=haar_unitary(1 << k, rng))
            out, ref, _ = run(sv, n, dtype, gaussian_state_np(n, n), [g], opts)
            assert max_err(out, ref) <= TOL[dtype], (variant, n, qs, max_err(out, ref))


@pytest.mark.parametrize("mfma", [0, 1])
def test_haar_circuit_c64(sv, mfma):
    n = 16
    gates = fused_haar_circuit(n, 40, seed=4)
    out, ref, _ = run(sv, n, "c64", gaussian_state_np(n, 4), gates,
                      {"mode": "sweep", "max_fuse_qubits": 0, "fp32_mfma": mfma})
    assert max_err(out, ref) <= TOL["c64"]


def test_renormalisation_fp64(sv):
    n = 14
    gates = fused_haar_circuit(n, 60, seed=7)
    out, ref, norm2 = run(sv, n, "c64", gaussian_state_np(n, 7), gates,
                          {"mode": "sweep", "max_fuse_qubits": 0, "renorm_interval": 10})
    assert max_err(out, ref) <= TOL["c64"]
    # the FP64 norm of the renormalised FP32 state is 1 to FP32 rounding of the scale
    assert abs(norm2 - 1.0) < 1e-6
    # and the scale itself is applied: start from a state scaled by 3
    t, _ = to_device(3.0 * gaussian_state_np(n, 8), "c64")
    st = sv.StateVector(n, "c64", tensor=t, init=False)
    st.apply_circuit(gates[:5], {"mode": "sweep", "max_fuse_qubits": 0, "renorm_interval": 5})
    assert abs(st.norm2() - 1.0) < 1e-6
    st.close()


def test_mfma_and_valu_agree_to_fp32(sv):
    n = 13
    rng = np.random.default_rng(3)
    g = Gate("MATRIX", (3, 9, 0, 12, 5, 7), matrix=haar_unitary(64, rng))
    a, ref, _ = run(sv, n, "c64", gaussian_state_np(n, 1), [g], {"mode": "sweep", "fp32_mfma": 1})
    b, _, _ = run(sv, n, "c64", gaussian_state_np(n, 1), [g], {"mode": "sweep", "fp32_mfma": 0})
    assert max_err(a, b) <= 2 * TOL["c64"] and max_err(a, ref) <= TOL["c64"]


@pytest.mark.parametrize("dtype,k", [("c128", 3), ("c128", 4), ("c128", 5), ("c128", 6),
                                     ("c64", 4), ("c64", 5), ("c64", 6)])
def test_dense_line_covering_placements(sv, dtype, k):
    """Placements with the highest qubits, and with the lowest physical bits
    (one 128-byte line) among the gate's qubits next to random higher ones:
    N=22, so that the persistent blocks loop over many column tiles (with the
    next tile's loads in flight); against the oracle."""
    n = 22
    rng = np.random.default_rng(70 + k)
    low = [0] if dtype == "c64" else [1, 0]  # member bits the lane groups own, at physical 0 (and 1)
    placements = [tuple(range(n - 1, n - 1 - k, -1)),                          # the highest bits, MSB first
                  tuple(int(x) for x in rng.choice(np.arange(6, n), k - len(low), replace=False)) + tuple(low)]
    for qs in placements:
        g = Gate("MATRIX", qs, matrix=haar_unitary(1 << k, rng))
        out, ref, _ = run(sv, n, dtype, gaussian_state_np(n, 5), [g], {"mode": "sweep", "max_fuse_qubits": 0})
        assert max_err(out, ref) <= TOL[dtype], (dtype, k, qs, max_err(out, ref))
