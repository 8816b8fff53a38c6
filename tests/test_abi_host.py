"""Host-side tests of the C ABI (no GPU needed): the library loads and exports
every function the headers declare; the planner (sv_fuse) validates its
input and its exported plan, replayed by the oracle, reproduces the circuit.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from oracle import sv_oracle as so
from paper_2409_14697_amd import binding as B
from svgen import (Gate, fused_haar_circuit, layered_circuit, qaoa_circuit, qft_circuit, brickwork_circuit,
                   gaussian_state_np, haar_unitary)


def test_library_exports_every_header_symbol():
    lib = B.load_library()
    names = B.header_symbols()
    assert "sv_create" in names and "sv_apply_gate" in names and "sv_measure_probs" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_version_and_defaults():
    assert "gfx950" in B.version()
    o = B.make_opts(None)
    assert o.max_fuse_qubits == 5 and o.reorder == 1 and o.fp32_mfma == 1 and o.mode == 0


def _fuse_err(n, gates, opts=None, dtype="c128"):
    with pytest.raises(B.SvError) as e:
        B.Plan(n, dtype, gates, opts)
    return e.value.status


def test_validation_errors():
    assert _fuse_err(4, [Gate("H", (4,))]) == B.SV_ERR_QUBIT
    assert _fuse_err(4, [Gate("CNOT", (1, 1))]) == B.SV_ERR_QUBIT
    assert _fuse_err(4, [Gate("H", (-1,))]) == B.SV_ERR_QUBIT
    assert _fuse_err(4, [Gate("H", (0,))], {"max_fuse_qubits": 7}) == B.SV_ERR_ARG
    assert _fuse_err(4, [Gate("H", (0,))], {"mode": 9}) == B.SV_ERR_ARG
    assert _fuse_err(0, []) == B.SV_ERR_ARG
    assert _fuse_err(35, []) == B.SV_ERR_ARG
    with pytest.raises(ValueError):
        B.Plan(4, "c32", [])
    # raw ABI: bad kind, nq mismatch, matrix gate without matrix, too many qubits
    lib = B.load_library()
    arr = (B.SvGate * 1)()
    h = ctypes.c_void_p()
    for kind, nq, q in ((99, 1, [0]), (B.KIND["H"], 2, [0, 1]), (B.KIND["MATRIX"], 1, [0]),
                        (B.KIND["MATRIX"], 7, [0, 1, 2, 3, 4, 5])):
        arr[0].kind, arr[0].nq = kind, nq
        for j in range(6):
            arr[0].q[j] = q[j] if j < len(q) else -1
        arr[0].m = None
        st = lib.sv_fuse(8, B.SV_C128, arr, 1, None, ctypes.byref(h))
        assert st == B.SV_ERR_ARG, (kind, nq, st)
        assert lib.sv_last_error()
    assert lib.sv_fuse(8, B.SV_C128, None, 1, None, ctypes.byref(h)) == B.SV_ERR_ARG
    assert lib.sv_fuse(8, B.SV_C128, None, 0, None, None) == B.SV_ERR_ARG
    assert lib.sv_plan_info(None, None, None) == B.SV_ERR_ARG
    assert lib.sv_measure_probs(None, None, 0, None) == B.SV_ERR_ARG
    assert lib.sv_apply_gate(None, None) == B.SV_ERR_ARG
    assert lib.sv_destroy(None) == B.SV_OK


def _replay(plan, n, psi):
    ops = [(q, m) for q, m, _ in plan.export()]
    return oracle.apply_ops(psi, ops)


@pytest.mark.parametrize("kmax", [0, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fusion_plan_replays_circuit(kmax, dtype):
    n = 10
    gates = layered_circuit(n, n_gates=120, seed=31)
    plan = B.Plan(n, dtype, gates, {"max_fuse_qubits": kmax})
    n_ops, n_passes = plan.info()
    assert n_ops <= len(gates)
    if kmax <= 1:
        assert n_ops == len(gates)
    psi = gaussian_state_np(n, 5)
    ref = oracle.run(gates, psi0=psi)
    out = _replay(plan, n, psi)
    assert np.max(np.abs(out - ref)) < 1e-13
    for q, m, ps in plan.export():
        assert len(q) <= max(kmax, 2) and len(set(q)) == len(q)
        assert np.max(np.abs(m.conj().T @ m - np.eye(m.shape[0]))) < 1e-13
        assert 0 <= ps < n_passes


@pytest.mark.parametrize("kmax", [2, 3, 5])
def test_forward_merge_replays_brickwork(kmax):
    """Ops that join a later op holding all their qubits (brickwork: the first
    rotations before each CNOT pair) still reproduce the circuit, and no
    single-qubit op is left once fusion may span a CNOT pair."""
    n = 11
    gates = brickwork_circuit(n, 8, seed=5)
    plan = B.Plan(n, "c128", gates, {"max_fuse_qubits": kmax, "mode": "sweep"})
    psi = gaussian_state_np(n, 6)
    ref = oracle.run(gates, psi0=psi)
    assert np.max(np.abs(_replay(plan, n, psi) - ref)) < 1e-13
    sizes = [len(q) for q, _, _ in plan.export()]
    assert all(k <= kmax for k in sizes)
    assert 1 not in sizes


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_phase_runs_fuse_qaoa(dtype):
    """Tile passes fold each QAOA cost layer (a run of n(n-1)/2 RZZ gates)
    into a few fixed-point phase ops per stage: far fewer kernel ops than
    gates, and phase functions in every pass that holds RZZ gates."""
    n = 20
    gates = qaoa_circuit(n, 5, seed=7)
    plan = B.Plan(n, dtype, gates, {"mode": "pass"})
    kops = plan.kernel_ops()
    assert sum(k for k, _ in kops) < len(gates) / 4
    rzz_pass = {ps for (q, m, ps) in plan.export() if len(q) == 2}
    assert rzz_pass and all(kops[ps][1] > 0 for ps in rzz_pass)


def test_fusion_reduces_ops():
    gates = brickwork_circuit(12, 6, seed=3)
    n5 = B.Plan(12, "c128", gates, {"max_fuse_qubits": 5, "mode": "sweep"}).info()[0]
    n0 = B.Plan(12, "c128", gates, {"max_fuse_qubits": 0, "mode": "sweep"}).info()[0]
    assert n0 == len(gates) and n5 < n0 / 3


CIRCUITS = {
    "layered": lambda n: layered_circuit(n, n_gates=160, seed=1),
    "brickwork": lambda n: brickwork_circuit(n, 8, seed=3),
    "qft": lambda n: qft_circuit(n),
    "haar": lambda n: fused_haar_circuit(n, 5, seed=4, ks=(2, 3, 5)),
}


@pytest.mark.parametrize("name", sorted(CIRCUITS))
@pytest.mark.parametrize("mode", ["pass", "auto", "sweep", "matrix"])
@pytest.mark.parametrize("lds", [0, 6, 9])
def test_pass_plans_replay_circuit(name, mode, lds):
    n = 12
    gates = CIRCUITS[name](n)
    plan = B.Plan(n, "c64", gates, {"mode": mode, "lds_qubits": lds})
    psi = gaussian_state_np(n, 8)
    assert np.max(np.abs(_replay(plan, n, psi) - oracle.run(gates, psi0=psi))) < 1e-13
    n_ops, n_passes = plan.info()
    passes = plan.passes()
    assert len(passes) == n_passes
    for kind, nops, nloc in passes:
        assert kind in (0, 1, 2, 3, 4)
        if kind in (1, 3):
            assert nloc == (lds or 12) or nloc == n
        if kind == 4:  # matrix passes: 64 KiB tiles whatever lds_qubits says
            assert nloc == min(n, 13)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_matrix_plans_group_local_ops(dtype):
    """Matrix-pass plans: exported ops replay the circuit (grouping moves an op
    only past ops on other qubits), every group fits one tile with the pinned
    low qubits, and each pass has one stage per op."""
    n, m, pin = 22, (13 if dtype == "c64" else 12), (4 if dtype == "c64" else 3)
    rng = np.random.default_rng(5)
    gates = []
    for _ in range(5):
        pool = list(range(pin)) + [int(x) for x in rng.choice(np.arange(pin, n), m - pin, replace=False)]
        for _ in range(3):
            k = int(rng.integers(2, 6))
            qs = tuple(int(x) for x in rng.choice(pool, k, replace=False))
            gates.append(Gate("MATRIX", qs, matrix=haar_unitary(1 << k, rng)))
    plan = B.Plan(n, dtype, gates, {"mode": "matrix", "max_fuse_qubits": 0})
    psi = gaussian_state_np(n, 2)
    assert np.max(np.abs(_replay(plan, n, psi) - oracle.run(gates, psi0=psi))) < 1e-12
    ex = plan.export()
    passes = plan.passes(stages=True)
    assert sum(1 for p in passes if p[0] == 4) >= 2
    for pi, (kind, nops, nloc, nst) in enumerate(passes):
        if kind != 4:
            continue
        assert nloc == m and nst == nops
        qs = set(range(pin))
        for q, _, p in ex:
            if p == pi:
                qs |= set(q)
        assert len(qs) <= m


def test_qft_swaps_become_relabels():
    n = 14
    plan = B.Plan(n, "c128", qft_circuit(n), {"mode": "pass", "lds_qubits": 8})
    ex = plan.export()
    swaps = [ps for q, m, ps in ex if len(q) == 2 and np.array_equal(m, so.named_matrix("SWAP"))]
    assert len(swaps) == n // 2 and all(ps == -1 for ps in swaps)
    kinds = [k for k, _, _ in plan.passes()]
    # the logical order is restored by the write-backs and at most a few
    # permutation-only passes; the replay checks the data ends in place
    assert set(kinds) <= {1, 3} and len(kinds) <= 5, kinds
    psi = gaussian_state_np(n, 4)
    assert np.max(np.abs(_replay(plan, n, psi) - oracle.run(qft_circuit(n), psi0=psi))) < 1e-12


def test_qft_n32_plan_needs_five_passes():
    """Gate blocks that leave local bits free for data on its way to its final
    position let the N=32 QFT (64 KiB tiles) restore the qubit order without
    a second permutation pass."""
    plan = B.Plan(32, "c64", qft_circuit(32), {"mode": "pass"})
    assert len(plan.passes()) <= 5, plan.passes()


def test_pass_plan_needs_few_passes_for_diagonal_ladders():
    # controlled phases need no locality: the QFT's passes are set by its H gates
    n = 20
    plan = B.Plan(n, "c64", qft_circuit(n), {"mode": "pass"})
    passes = plan.passes()
    assert len(passes) <= 4
    # two passes hold the H gates and their phase ladders (a third at most
    # holds the last few gates)
    assert sum(1 for k, ops, _ in passes if k == 1 and ops > 10) <= 2


def test_fusion_qft_and_haar():
    n = 9
    for gates in (qft_circuit(n), fused_haar_circuit(n, 8, seed=2, ks=(3, 4, 5, 6))):
        plan = B.Plan(n, "c128", gates, {"max_fuse_qubits": 6})
        psi = gaussian_state_np(n, 1)
        assert np.max(np.abs(_replay(plan, n, psi) - oracle.run(gates, psi0=psi))) < 1e-13


def test_export_matches_input_when_unfused():
    gates = [Gate("RX", (2,), 0.3), Gate("CNOT", (0, 3)), Gate("CPHASE", (1, 2), 1.1), Gate("RZZ", (0, 1), 0.7),
             Gate("MATRIX", (3, 0, 1), matrix=np.eye(8)[::-1])]
    plan = B.Plan(4, "c128", gates, {"max_fuse_qubits": 0})
    ex = plan.export()
    assert len(ex) == len(gates)
    for g, (q, m, _) in zip(gates, ex):
        assert q == g.qubits
        assert np.max(np.abs(m - so.gate_matrix(g))) < 1e-15


def test_named_gate_matrices_match_oracle_definitions():
    # the library builds its own matrices (C++, FP64); compare them entrywise
    for kind in ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P", "CNOT", "CZ", "SWAP", "CPHASE", "RZZ"):
        for theta in (0.0, 0.4, 2.9):
            nq = 2 if kind in ("CNOT", "CZ", "SWAP", "CPHASE", "RZZ") else 1
            g = Gate(kind, tuple(range(nq)), theta)
            (q, m, _), = B.Plan(3, "c128", [g], {"max_fuse_qubits": 0}).export()
            assert np.max(np.abs(m - so.gate_matrix(g))) < 1e-15, kind


@pytest.mark.parametrize("cap", [1, 7, 32])
def test_pass_op_cap_splits_passes_and_replays(cap):
    n = 12
    gates = layered_circuit(n, n_gates=300, seed=9)
    plan = B.Plan(n, "c128", gates, {"mode": "pass", "max_pass_ops": cap})
    psi = gaussian_state_np(n, 3)
    assert np.max(np.abs(_replay(plan, n, psi) - oracle.run(gates, psi0=psi))) < 1e-13
    for kind, nops, nloc in plan.passes():
        assert kind in (1, 3) and nops <= cap
    uncapped = B.Plan(n, "c128", gates, {"mode": "pass"}).info()[1]
    assert plan.info()[1] >= max(uncapped, len(gates) // cap)
    with pytest.raises(B.SvError):
        B.Plan(n, "c128", gates, {"mode": "pass", "max_pass_ops": -1})


def test_planning_time_is_bounded():
    # host planning must stay far below device time: ~8k gates at N=26 in well under a second
    import time
    from svgen import Request
    gates = Request(0, 26, 200, 7, 0.0).circuit()
    for mode in ("pass", "auto", "sweep"):
        t0 = time.perf_counter()
        plan = B.Plan(26, "c64", gates, {"mode": mode})
        dt = time.perf_counter() - t0
        assert plan.info()[0] > 0
        assert dt < 2.0, (mode, dt)


def test_pass_flops_count_each_gate_class():
    """Flops per amplitude: 8 * 2^k for a dense k-qubit op, 6 for a diagonal
    op, 0 for a permutation; the one-call array form equals the per-pass
    query, and a plan of one-qubit-merged sweeps counts what the tile-pass
    plan of the same circuit counts."""
    rng = np.random.default_rng(3)
    gates = [Gate("H", (0,)), Gate("RZ", (1,), 0.3), Gate("CNOT", (0, 2)), Gate("CZ", (1, 3)),
             Gate("RX", (2,), 0.7), Gate("MATRIX", (0, 1, 3), matrix=haar_unitary(8, rng)), Gate("SWAP", (1, 2))]
    plan = B.Plan(6, "c128", gates, {"mode": "sweep", "max_fuse_qubits": 0})
    flops = plan.pass_flops()
    assert flops == [16.0, 6.0, 0.0, 6.0, 16.0, 64.0, 0.0]
    lib = B.load_library()
    one = ctypes.c_double()
    for i, f in enumerate(flops):
        B.check(lib.sv_plan_pass_flops(plan._h, i, ctypes.byref(one)))
        assert one.value == f
    short = (ctypes.c_double * 3)()
    with pytest.raises(B.SvError):
        B.check(lib.sv_plan_flops(plan._h, short, 3))
    plan.close()
    lay = layered_circuit(16, n_layer_pairs=6, seed=2)
    tile = B.Plan(16, "c64", lay, {"mode": "pass"})
    light = B.Plan(16, "c64", lay, {"mode": "sweep", "max_fuse_qubits": 1})
    assert sum(tile.pass_flops()) == sum(light.pass_flops()) > 0
    tile.close()
    light.close()
    empty = B.Plan(4, "c64", [], {"mode": "auto"})
    assert empty.info() == (0, 0) and empty.pass_flops() == [] and empty.program_bytes() == 0
    empty.close()
