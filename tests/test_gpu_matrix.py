"""GPU parity of matrix passes: fused dense ops grouped by locality, each group
applied to every in-cache tile as matrix-core stages (gate fusion and in-cache
operation together, Sec. II-B / III-B), against the oracle."""
import numpy as np
import pytest

import oracle
from svgen import Gate, brickwork_circuit, gaussian_state_np, haar_unitary
from tests.gpu_util import TOL, max_err, to_device, to_host

pytestmark = pytest.mark.gpu

MATRIX_PASS = 4


@pytest.fixture(scope="module")
def sv():
    import paper_2409_14697_amd as sv
    return sv


def run(sv, n, dtype, psi, gates, opts):
    plan = sv.Plan(n, dtype, gates, opts)
    kinds = [k for k, _, _, _ in plan.passes(stages=True)]
    stages = [s for k, _, _, s in plan.passes(stages=True) if k == MATRIX_PASS]
    t, host_in = to_device(psi, dtype)
    st = sv.StateVector(n, dtype, tensor=t, init=False)
    st.apply_plan(plan)
    st.sync()
    out = to_host(t)
    st.close()
    plan.close()
    return out, oracle.run(gates, psi0=host_in), kinds, stages


def grouped_haar(n, rng, groups, per_group, kmin=3, kmax=5, pinned=4, free=9):
    """Haar gates in groups: each group's gates use the pinned low qubits and
    `free` other qubits of its own, so that a group fits one tile."""
    gates = []
    for _ in range(groups):
        pool = list(range(pinned)) + [int(x) for x in rng.choice(np.arange(pinned, n), free, replace=False)]
        for _ in range(per_group):
            k = int(rng.integers(kmin, kmax + 1))
            qs = tuple(int(x) for x in rng.choice(pool, k, replace=False))
            gates.append(Gate("MATRIX", qs, matrix=haar_unitary(1 << k, rng)))
    return gates


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [12, 13, 16])
def test_brickwork_matrix_mode(sv, dtype, n):
    """Layered rotations + CNOT bricks, fused to k <= 5 and grouped; the
    smallest states are one tile."""
    gates = brickwork_circuit(n, 12, seed=n)
    out, ref, kinds, stages = run(sv, n, dtype, gaussian_state_np(n, n), gates, {"mode": "matrix"})
    assert MATRIX_PASS in kinds and max(stages) >= 2, (kinds, stages)
    assert max_err(out, ref) <= TOL[dtype], max_err(out, ref)


@pytest.mark.parametrize("dtype,n", [("c64", 22), ("c128", 21), ("c64", 14), ("c128", 12)])
def test_grouped_haar_gates(sv, dtype, n):
    """Random 3..5-qubit unitaries in groups that fit one tile; at N = 22 / 21
    every block runs several tiles (more tiles than resident blocks)."""
    rng = np.random.default_rng(100 + n)
    pinned = 4 if dtype == "c64" else 3
    free = min(9, n - pinned)
    gates = grouped_haar(n, rng, groups=4, per_group=3, pinned=pinned, free=free)
    out, ref, kinds, stages = run(sv, n, dtype, gaussian_state_np(n, 3), gates,
                                  {"mode": "matrix", "max_fuse_qubits": 0})
    assert MATRIX_PASS in kinds and max(stages) >= 3, (kinds, stages)
    assert max_err(out, ref) <= TOL[dtype], max_err(out, ref)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_narrow_ops_widened(sv, dtype):
    """Ops of 1..4 qubits in a matrix pass run as the stage width's product
    (identity on the added tile bits); complex128 groups of ops of at most 4
    qubits run 16 x 16 stages."""
    n = 15
    rng = np.random.default_rng(7)
    gates = grouped_haar(n, rng, groups=3, per_group=4, kmin=1, kmax=4,
                         pinned=4 if dtype == "c64" else 3, free=8)
    out, ref, kinds, _ = run(sv, n, dtype, gaussian_state_np(n, 5), gates, {"mode": "matrix", "max_fuse_qubits": 0})
    assert MATRIX_PASS in kinds
    assert max_err(out, ref) <= TOL[dtype], max_err(out, ref)


def test_matrix_passes_in_auto_plan(sv):
    """The auto plan of a brickwork circuit uses matrix passes (complex64)."""
    n = 20
    gates = brickwork_circuit(n, 8, seed=2)
    out, ref, kinds, _ = run(sv, n, "c64", gaussian_state_np(n, 2), gates, {"mode": "auto"})
    assert kinds.count(MATRIX_PASS) >= 2, kinds
    assert max_err(out, ref) <= TOL["c64"], max_err(out, ref)


def test_renormalisation_counts_matrix_ops(sv):
    """complex64 plans renormalise after every R dense ops, matrix-pass ops included."""
    n = 14
    rng = np.random.default_rng(11)
    gates = grouped_haar(n, rng, groups=3, per_group=3)
    t, _ = to_device(2.0 * gaussian_state_np(n, 6), "c64")
    st = sv.StateVector(n, "c64", tensor=t, init=False)
    st.apply_circuit(gates, {"mode": "matrix", "max_fuse_qubits": 0, "renorm_interval": 4})
    assert abs(st.norm2() - 1.0) < 1e-6
    st.close()
