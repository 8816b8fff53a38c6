"""GPU tests of the serving form: the batched pass launch (sv_batcher_run) and
the continuous-batching loop.  Every served state is checked against the
oracle, and a request's result is the same whether it ran alone or in a mix
(the batched kernel reads only the request's own program and state)."""
import numpy as np
import pytest

import oracle
from svgen import brickwork_circuit, layered_circuit, qft_circuit, serving_requests
from tests.gpu_util import TOL, max_err, to_host

pytestmark = pytest.mark.gpu

PROB_TOL = {"c128": 1e-12, "c64": 4e-5}


@pytest.fixture(scope="module")
def sv():
    import paper_2409_14697_amd as sv
    return sv


def low_probs_ref(psi, n, k=16):
    k = min(n, k)
    return oracle.probs(psi, list(range(k - 1, -1, -1)))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("family", ["layered", "qft"])
def test_batched_pass_launch_matches_oracle_and_single_plans(sv, dtype, family):
    """Batched passes (one launch per step for all states) against the oracle
    and against the unbatched pass kernel; the QFT family runs the
    phase-ladder and register-diagonal ops through the batched kernel."""
    import torch
    ns = [6, 9, 12, 13, 14, 16, 17]
    if family == "qft":
        circuits = {n: qft_circuit(n) for n in ns}
    else:
        circuits = {n: layered_circuit(n, n_layer_pairs=5, seed=n) for n in ns}
    plans = {n: sv.Plan(n, dtype, circuits[n], {"mode": "pass", "max_pass_ops": 16}) for n in ns}
    progs = {n: sv.Program(plans[n]) for n in ns}
    states = {n: sv.StateVector(n, dtype) for n in ns}
    batcher = sv.Batcher()
    step = 0
    while True:
        live = [n for n in ns if step < progs[n].n_passes]
        if not live:
            break
        batcher.run([states[n] for n in live], [progs[n] for n in live], [step] * len(live))
        step += 1
    torch.cuda.synchronize()
    if family == "qft":
        assert any(lad for n in ns for _, lad in plans[n].kernel_ops())
    for n in ns:
        out = to_host(states[n].tensor)
        ref = oracle.run(circuits[n], n=n)
        assert max_err(out, ref) <= TOL[dtype], n
        # the unbatched pass kernel (sv_apply_plan) on the same plan
        single = sv.StateVector(n, dtype)
        single.apply_plan(plans[n])
        single.sync()
        assert max_err(to_host(single.tensor), out) <= TOL[dtype], n
        single.close()
    for n in ns:
        states[n].close()
        progs[n].close()
    batcher.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batched_steps_with_matrix_dense_and_sweep_passes(sv, dtype):
    """Programs of every pass kind in one batch: each step runs the tile and
    permutation passes of all states in one launch and every matrix, dense or
    sweep pass as a launch of its own.  Each state matches the oracle and,
    bitwise, the same plan applied alone."""
    import torch
    cases = [(9, "sweep", brickwork_circuit(9, 4, seed=1)),
             (14, "matrix", brickwork_circuit(14, 10, seed=2)),
             (16, "sweep", layered_circuit(16, n_layer_pairs=2, seed=3)),
             (17, "pass", layered_circuit(17, n_layer_pairs=4, seed=4)),
             (18, "matrix", brickwork_circuit(18, 10, seed=5)),
             (20, "auto", brickwork_circuit(20, 8, seed=6))]
    plans = [sv.Plan(n, dtype, g, {"mode": mode}) for n, mode, g in cases]
    kinds = {k for p in plans for k, _, _ in p.passes()}
    assert {0, 1, 2, 4} <= kinds, kinds  # sweep, tile, dense and matrix passes
    progs = [sv.Program(p) for p in plans]
    states = [sv.StateVector(n, dtype) for n, _, _ in cases]
    b = sv.Batcher()
    step = 0
    while True:
        live = [i for i in range(len(cases)) if step < progs[i].n_passes]
        if not live:
            break
        b.run([states[i] for i in live], [progs[i] for i in live], [step] * len(live))
        step += 1
    torch.cuda.synchronize()
    for i, (n, mode, g) in enumerate(cases):
        out = to_host(states[i].tensor)
        assert max_err(out, oracle.run(g, n=n)) <= TOL[dtype], (n, mode)
        single = sv.StateVector(n, dtype)
        single.apply_plan(plans[i])
        single.sync()
        assert np.array_equal(to_host(single.tensor), out), (n, mode)
        single.close()
    for x in states + progs + plans + [b]:
        x.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batcher_rejects_bad_batches(sv, dtype):
    from paper_2409_14697_amd import binding as B
    other = "c64" if dtype == "c128" else "c128"
    pa = sv.Program(sv.Plan(8, dtype, layered_circuit(8, n_layer_pairs=2, seed=1), {"mode": "pass"}))
    pb = sv.Program(sv.Plan(8, other, layered_circuit(8, n_layer_pairs=2, seed=1), {"mode": "pass"}))
    s8, s9 = sv.StateVector(8, dtype), sv.StateVector(9, dtype)
    s8o = sv.StateVector(8, other)
    before = to_host(s8.tensor)
    b = sv.Batcher()
    cases = [([s9], [pa], [0]),                       # program for 8 qubits, state of 9
             ([s8, s8o], [pa, pb], [0, 0]),           # mixed dtypes
             ([s8, s8], [pa, pa], [0, 0]),            # a state twice
             ([s8], [pa], [pa.n_passes]),             # pass index out of range
             ([s8], [pa], [-1])]
    for st, pr, ix in cases:
        with pytest.raises(B.SvError) as e:
            b.run(st, pr, ix)
        assert e.value.status == B.SV_ERR_ARG
    b.run([], [], [])  # an empty batch is a no-op
    import torch
    torch.cuda.synchronize()
    assert np.array_equal(to_host(s8.tensor), before)
    for x in (s8, s9, s8o, pa, pb, b):
        x.close()


def _serve(sv, dtype, requests, rate, budget=None, keep_states=True, max_active=64, matrix_qubits=24):
    from paper_2409_14697_amd import binding as B
    from paper_2409_14697_amd.serve import DeviceEngine, Server, free_budget, make_jobs
    jobs = make_jobs(requests, rate, B.make_gates)
    eng = DeviceEngine(dtype, keep_states=keep_states, max_pass_ops=24, matrix_qubits=matrix_qubits)
    srv = Server(eng, budget or free_budget(0.5), max_active=max_active, plan_workers=4)
    res = srv.run(jobs)
    eng.close()
    return res, jobs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("rate", [None, 3000.0])
def test_serving_loop_results_match_oracle(sv, dtype, rate):
    reqs = serving_requests(24, seed=11, n_range=(6, 15), depth_range=(2, 12))
    res, jobs = _serve(sv, dtype, reqs, rate)
    s = res.summary()
    assert s["completed"] == len(reqs) and s["errors"] == 0 and s["rejected"] == 0
    assert s["p99_ms"] >= s["p50_ms"] > 0
    tile = 13 if dtype == "c64" else 12  # qubits of one 64 KiB LDS tile
    for r, j in zip(reqs, jobs):
        ref = oracle.run(r.circuit(), n=r.n)
        assert max_err(to_host(j.handle["tensor"]), ref) <= TOL[dtype], (r.rid, r.n)
        assert max_err(j.probs, low_probs_ref(ref, r.n)) <= PROB_TOL[dtype], (r.rid, r.n)
        if r.n <= tile:  # the whole circuit in one LDS-resident pass: one launch
            assert j.n_passes == 1, (r.rid, r.n, j.n_passes)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_serving_loop_with_auto_plans(sv, dtype):
    """Requests of at least 15 qubits planned in mode AUTO (matrix, dense and
    sweep passes next to tile passes) served in one loop with smaller ones."""
    reqs = serving_requests(16, seed=12, n_range=(10, 19), depth_range=(4, 16))
    res, jobs = _serve(sv, dtype, reqs, None, matrix_qubits=15)
    s = res.summary()
    assert s["completed"] == len(reqs) and s["errors"] == 0 and s["rejected"] == 0
    assert any(r.n >= 15 for r in reqs)
    for r, j in zip(reqs, jobs):
        ref = oracle.run(r.circuit(), n=r.n)
        assert max_err(to_host(j.handle["tensor"]), ref) <= TOL[dtype], (r.rid, r.n)
        assert max_err(j.probs, low_probs_ref(ref, r.n)) <= PROB_TOL[dtype], (r.rid, r.n)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_serving_tiny_requests(sv, dtype):
    """Requests of 1..5 qubits (too small for a tile: their programs hold
    sweep and dense passes only; 1-2 qubits: no program bytes at all) served
    with 6..9-qubit ones, against the oracle."""
    from svgen.circuits import Request
    reqs = [Request(i, n, 3 + i % 4, 40 + i, 0.0) for i, n in enumerate((1, 2, 3, 4, 5, 1, 3, 5))]
    reqs += [Request(10 + i, n, 4, 60 + i, 0.0) for i, n in enumerate((6, 7, 8, 9))]
    res, jobs = _serve(sv, dtype, reqs, None)
    s = res.summary()
    assert s["completed"] == len(reqs) and s["errors"] == 0 and s["rejected"] == 0
    for r, j in zip(reqs, jobs):
        ref = oracle.run(r.circuit(), n=r.n)
        assert max_err(to_host(j.handle["tensor"]), ref) <= TOL[dtype], (r.rid, r.n)
        assert max_err(j.probs, low_probs_ref(ref, r.n)) <= PROB_TOL[dtype], (r.rid, r.n)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_serving_alone_equals_in_mix_bitwise(sv, dtype):
    reqs = serving_requests(16, seed=12, n_range=(6, 17), depth_range=(2, 10))
    _, mixed = _serve(sv, dtype, reqs, None)
    for r, j in zip(reqs[:8], mixed[:8]):
        _, alone = _serve(sv, dtype, [r], None)
        a = alone[0].handle["tensor"].cpu().numpy()
        b = j.handle["tensor"].cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), r.rid
        assert np.array_equal(alone[0].probs, j.probs), r.rid


def test_serving_under_a_tight_budget(sv):
    # a budget that holds only a few of the states at once forces queueing
    reqs = serving_requests(20, seed=13, n_range=(10, 16), depth_range=(2, 6))
    budget = 3 * (1 << 16) * 8 + (4 << 20)
    res, jobs = _serve(sv, "c64", reqs, 5000.0, budget=budget)
    s = res.summary()
    assert s["completed"] == len(reqs)
    assert res.peak_used <= budget
    for r, j in zip(reqs, jobs):
        assert max_err(to_host(j.handle["tensor"]), oracle.run(r.circuit(), n=r.n)) <= TOL["c64"]


def test_serving_rejects_a_request_larger_than_the_budget(sv):
    reqs = serving_requests(6, seed=14, n_range=(8, 10), depth_range=(2, 4))
    big = serving_requests(1, seed=15, n_range=(20, 20), depth_range=(2, 2))[0]
    big.rid = 99
    res, jobs = _serve(sv, "c64", reqs + [big], None, budget=64 << 20 >> 4)
    by = {j.rid: j for j in jobs}
    assert by[99].status == "rejected"
    assert all(by[r.rid].status == "done" for r in reqs)
