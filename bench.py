"""Benchmarks of the state-vector hot path on one MI355X.  Prints ONE JSON line.

Default run (the headline first, then the other two parts of the metric
"HBM GB/s per gate at N=30; circuit sec; served circuits/s + p99 latency"):

  * gate benchmark (the per-gate benchmark of QueenV2 Sec. IV-B, made
    concrete): a normalised complex Gaussian state of N=30 qubits in
    complex128 (16 GiB, the paper's FP64) and complex64 (8 GiB), seeded; each
    of H, X, RZ, CNOT, CZ, SWAP, CPHASE on every target qubit 0..29 (two-qubit
    partners drawn at random), one gate per sv_apply_gate call.  One step =
    the 210 gates on each state.  value = complex128 algorithmic bytes /
    kernel time (GB/s); complex64 is reported beside it.  A gate's algorithmic
    bytes are 2 * S * f, S the state size and f the fraction of 128-byte lines
    holding an amplitude the gate changes (1 for H/X/RZ; 1/2 or 1 for CNOT
    and SWAP; 1/4, 1/2 or 1 for CZ and CPHASE).
  * "circuit": N=32 complex64 (32 GiB) brickwork depth 40 + QFT with the
    planner's plans (Sec. IV-C circuit families), seconds and passes;
  * "precision": N=30, 2000 fused Haar 5/6-qubit gates (one seed), FP32 MFMA
    against FP64 on the same GPU, with errors;
  * "serving": continuous batching of random circuit requests (N 12..26),
    closed-loop throughput, Poisson arrivals at 0.8 x, p50 / p99 latency.

Every launch of the gate benchmark is bracketed by HIP events on the stream
the library launches on (torch's current stream, handed to sv_create), so
per-kernel average durations come from the same timed region.  Inputs are
resident in HBM before every timed region; no host transfer is timed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# vector (VALU) peaks: 256 CUs x 2.4 GHz; FP32 counts packed math, FP64 does not
PEAK_VALU_TFLOPS = {"c64": 157.3, "c128": 78.6}
# dense matrix-core peaks (no sparsity): FP32 and FP64 MFMA
PEAK_MFMA_TFLOPS = {"c64": 157.3, "c128": 78.6}
N_QUBITS = 30
LINE = 128  # bytes per memory read granule (FETCH_SIZE of sub-line subsets)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def line_qubits(dtype: str) -> int:
    """Qubits whose bit lies inside one 128-byte line."""
    return int(math.log2(LINE // (16 if dtype == "c128" else 8)))


def touched_fraction(gate, dtype: str) -> float:
    g = line_qubits(dtype)
    kind, qs = gate.kind, gate.qubits
    if kind in ("H", "X", "RZ"):
        return 1.0
    if kind == "CNOT":
        return 0.5 if qs[0] >= g else 1.0
    if kind == "SWAP":
        return 0.5 if (qs[0] >= g and qs[1] >= g) else 1.0
    if kind in ("CZ", "CPHASE"):
        return 2.0 ** -((qs[0] >= g) + (qs[1] >= g))
    raise ValueError(kind)


_ELEM = {"c128": "double __vector(2)", "c64x2": "float __vector(4)", "c64x1": "float __vector(2)",
         "c64": "float __vector(4)"}
_OPS = {"DENSE1": "OpDense1", "DENSE2": "OpDense2", "SWAP": "OpSwap", "PHASE": "OpPhase", "DIAG": "OpDiag",
        "SCALE": "OpScale"}
_KINDS = {"INTRA": 0, "LANE": 1, "REG": 2}


def kernel_symbol(key: str) -> str:
    """Template instantiation of a kernel identifier returned by
    sv_gate_kernel, as rocprofv3 lists it with namespaces removed."""
    parts = key.split("/")
    if parts[0] == "group":
        el, op, zv = parts[1], parts[2], parts[3]
        nz, nv = zv[1:].split("v")
        real = "double" if el == "c128" else "float"
        return f"k_group<{_ELEM[el]}, {nz}, {nv}, {_OPS[op]}<{real}> >"
    if parts[0] == "lane":
        el, k, kinds, z = parts[1], int(parts[2][1:]), parts[3].split("-"), int(parts[4][1:])
        ka = _KINDS[kinds[0]]
        kb = _KINDS[kinds[1]] if k == 2 else -1
        return f"k_low<{_ELEM[el]}, {k}, {ka}, {kb}, {z}>"
    return key


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sv_sweep.hip", "sv_device.h", "sv_kernels.h", "sv_gates.cpp"):  # the gate-sweep kernels and their arguments
        with open(os.path.join(ROOT, "paper_2409_14697_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def circuit_source_hash() -> str:
    """Hash of the sources that decide the circuit benchmark's kernels and plans."""
    h = hashlib.sha256()
    for f in ("sv_pass.hip", "sv_dense.hip", "sv_sweep.hip", "sv_tile_kernels.h", "sv_device.h", "sv_kernels.h",
              "sv_plan.cpp", "sv_passplan.cpp", "sv_gates.cpp"):
        with open(os.path.join(ROOT, "paper_2409_14697_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_circuit_traffic():
    """Per-kernel HBM bytes per launch of the circuit benchmark (committed
    rocprofv3 counter summary); None when absent or taken on other sources."""
    try:
        with open(os.path.join(ROOT, "profiles", "circuit_traffic_n32_c64.json")) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("source_hash") != circuit_source_hash():
        return None
    return {k: {"launches": v["launches"], "bytes_per_launch": v["bytes_per_launch"],
                "of_read_plus_write": v["of_read_plus_write"]} for k, v in d["kernels"].items()}


def load_traffic(kernel_key: str):
    """HBM bytes per launch of `kernel_key` from the committed rocprofv3 counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a copy kernel of known size);
    None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "gate_sweep_counters_n30.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel_key)
    return None if k is None else k.get("bytes_per_launch")


# ---------------------------------------------------------------- CPU baseline
def _host_info():
    """The host the oracle runs on: core counts, BLAS build, thread settings."""
    import numpy as np
    info = {"cpu_count": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["affinity"] = None
    try:
        cfg = np.show_config(mode="dicts")
        blas = cfg.get("Build Dependencies", {}).get("blas", {})
        info["blas"] = f"{blas.get('name', '?')} {blas.get('version', '')}".strip()
    except Exception:
        info["blas"] = "?"
    try:
        from threadpoolctl import threadpool_info
        pools = threadpool_info()
        info["blas_threads"] = max([p.get("num_threads", 1) for p in pools] or [1])
        info["blas_runtime"] = ", ".join(sorted({f"{p.get('internal_api')} {p.get('version')}" for p in pools}))
    except Exception:
        info["blas_threads"] = 1
    info["thread_env"] = {k: os.environ[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
                          if k in os.environ}
    return info


def _oracle_gate_rate(gates, n: int):
    """Oracle seconds and algorithmic GB/s over `gates` at N=n (complex128)."""
    import oracle
    from svgen import gaussian_state_np
    psi = gaussian_state_np(n, 2)
    total_bytes, total_t = 0.0, 0.0
    for g in gates:
        t0 = time.perf_counter()
        psi = oracle.apply_gate(psi, g)
        total_t += time.perf_counter() - t0
        total_bytes += 2.0 * (1 << n) * 16 * touched_fraction(g, "c128")
    return total_bytes / total_t / 1e9, total_t


def cpu_baseline(gates, n: int):
    """The oracle (numpy, complex128) on a bounded sample of the gate
    benchmark -- three of its gates at N=30 -- on the host cores, with all
    BLAS threads and with one; plus the seconds the oracle takes for the
    N=16, 200-gate parity circuit."""
    import oracle
    from svgen import layered_circuit
    host = _host_info()
    sample = [g for g in gates if (g.kind, g.qubits[-1]) in (("H", n - 1), ("CNOT", 0), ("CPHASE", n // 2))]
    gbs, secs = _oracle_gate_rate(sample, n)
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            gbs1, secs1 = _oracle_gate_rate(sample[:1], n)
        single = {"value": round(gbs1, 3), "unit": "GB/s", "cores": 1, "sample": f"{sample[0].kind}{sample[0].qubits} at N={n}",
                  "seconds": round(secs1, 2)}
    except Exception as e:  # threadpoolctl missing: say so
        single = {"error": str(e)}
    c1 = layered_circuit(16, n_gates=200, seed=1)
    t0 = time.perf_counter()
    oracle.run(c1, n=16)
    c1_s = time.perf_counter() - t0
    desc = ", ".join(f"{g.kind}{g.qubits}" for g in sample)
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": host["blas_threads"], "kind": "oracle",
            "sample": f"{len(sample)} gates of the set ({desc}) at N={n}, complex128, {secs:.1f} s",
            "single_thread": single, "c1_parity_circuit_s": round(c1_s, 4),
            "c1_workload": "N=16 complex128, 200-gate layered circuit (seed 1), all host threads",
            "host": host}


# ---------------------------------------------------------------- gate benchmark
def gates_bench(args):
    import torch

    import paper_2409_14697_amd as sv
    from svgen import gate_bench_set
    from svgen.states import gaussian_state_torch

    torch.cuda.set_device(0)
    n = args.n
    gates = gate_bench_set(n, seed=2)
    dtypes = [d for d in args.dtypes.split(",") if d]
    stream = torch.cuda.current_stream()
    per_kernel = {}   # (dtype, key) -> [bytes, seconds, launches]
    per_dtype = {}
    launch_min = {}   # dtype -> (GB/s, gate) of the slowest (gate, target) launch
    for dtype in dtypes:
        tdt = torch.complex128 if dtype == "c128" else torch.complex64
        psi = gaussian_state_torch(n, 2, tdt)
        st = sv.StateVector(n, dtype, tensor=psi, init=False, stream=stream)
        S = psi.numel() * psi.element_size()
        kernels = [sv.gate_kernel(n, dtype, g) for g in gates]
        for _ in range(args.warmup):
            for g in gates:
                st.apply_gate(g)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in gates]
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        durations = [0.0] * len(gates)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            for i, g in enumerate(gates):
                evs[i][0].record(stream)
                st.apply_gate(g)
                evs[i][1].record(stream)
            stream.synchronize()
            for i in range(len(gates)):
                durations[i] += evs[i][0].elapsed_time(evs[i][1]) * 1e-3
        stop.record(stream)
        torch.cuda.synchronize()
        wall = start.elapsed_time(stop) * 1e-3
        dbytes = 0.0
        worst = None
        for i, g in enumerate(gates):
            b = 2.0 * S * touched_fraction(g, dtype) * args.steps
            dbytes += b
            rate = b / durations[i] / 1e9
            if worst is None or rate < worst[0]:
                worst = (rate, f"{g.kind}{tuple(g.qubits)}")
            acc = per_kernel.setdefault((dtype, kernels[i]), [0.0, 0.0, 0])
            acc[0] += b
            acc[1] += durations[i]
            acc[2] += args.steps
        kern_s = sum(durations)
        per_dtype[dtype] = {"GB/s": round(dbytes / kern_s / 1e9, 1), "ms_per_step": round(1e3 * wall / args.steps, 3),
                            "gates_per_step": len(gates), "kernel_s": kern_s, "bytes": dbytes}
        launch_min[dtype] = {"GB/s": round(worst[0], 1), "gate": worst[1], "frac": round(worst[0] / PEAK_HBM_GBS, 4)}
        st.close()
        del psi
        torch.cuda.empty_cache()

    copy_gbs = None
    if args.copy_ceiling:
        src = torch.empty(1 << (n - 1), dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(src)
        sv.util_copy(dst, src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            sv.util_copy(dst, src)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 2.0 * src.numel() * 16 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
    head = "c128" if "c128" in per_dtype else dtypes[0]
    # dominant kernel of the headline dtype = the one with the most time in the timed region
    (_, dom_key), (dbytes, dsec, dl) = max(((k, v) for k, v in per_kernel.items() if k[0] == head),
                                           key=lambda kv: kv[1][1])
    achieved = dbytes / dsec / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": load_traffic(dom_key),
                "traffic_calibration": "FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000: the factors that turn the "
                                       "counters of the 16-byte copy kernel into its known bytes",
                "kernel": dom_key, "symbol": kernel_symbol(dom_key),
                "launches": dl, "avg_ms": round(1e3 * dsec / dl, 4),
                "algorithmic_bytes_per_launch": round(dbytes / dl)}
    out = {"value": per_dtype[head]["GB/s"], "head": head, "per_dtype": per_dtype, "launch_min": launch_min,
           "per_kernel": {f"{d}:{k}": {"GB/s": round(v[0] / v[1] / 1e9, 1), "launches": v[2], "ms": round(1e3 * v[1], 2)}
                          for (d, k), v in sorted(per_kernel.items())},
           "roofline": roofline, "copy_kernel_GBs": None if copy_gbs is None else round(copy_gbs, 1),
           "gates": gates}
    return out


# ---------------------------------------------------------------- circuits
def circuit_bench(args, n: int = 32):
    """Circuit benchmark: N=32 complex64 (32 GiB) random brickwork circuit of
    depth 40 (1900 gates) and the N=32 QFT (544 gates), planned once (gate
    fusion + in-cache tile passes, mode `args.mode`) and applied `steps`
    times after `warmup`.  The QFT runs on a seeded basis state and is
    checked against its closed form on 4096 sampled amplitudes."""
    import numpy as np
    import torch

    import paper_2409_14697_amd as sv
    from svgen import brickwork_circuit, qft_circuit

    torch.cuda.set_device(0)
    dtype = "c64"
    stream = torch.cuda.current_stream()
    st = sv.StateVector(n, dtype, stream=stream)
    S = (1 << n) * 8
    out = {}
    rng = np.random.default_rng(7)
    x0 = int(rng.integers(0, 1 << n))
    steps, warmup = args.circuit_steps, args.circuit_warmup
    for name, gates in (("brickwork_d40", brickwork_circuit(n, 40, seed=3)), ("qft", qft_circuit(n))):
        t0 = time.perf_counter()
        plan = sv.Plan(n, dtype, gates, {"mode": args.mode})
        plan_s = time.perf_counter() - t0
        kinds = [k for k, _, _ in plan.passes()]
        sweeps = len(kinds)
        init = x0 if name == "qft" else 0
        for _ in range(warmup):
            st.init_basis(init)
            st.apply_plan(plan)
        times = []
        for _ in range(steps):
            st.init_basis(init)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st.apply_plan(plan)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        sec = sum(times) / len(times)
        # matrix-core work of the dense passes: 8 * 2^(N+k) real flops per k-qubit op
        dense_flops = sum(8.0 * 2.0 ** (n + len(q)) for q, _, ps in plan.export() if ps >= 0 and len(q) >= 3)
        rec = {"seconds": round(sec, 5), "min_s": round(min(times), 5), "gates": len(gates),
               "ops": plan.info()[0], "passes": sweeps,
               "pass_kinds": {str(k): kinds.count(k) for k in sorted(set(kinds))},
               "plan_s": round(plan_s, 4),
               "mfma_algorithmic_frac": round(dense_flops / sec / (PEAK_MFMA_TFLOPS["c64"] * 1e12), 4)}
        hbm = {"bound": "hbm", "achieved": round(sweeps * 2 * S / sec / 1e9, 1), "peak": PEAK_HBM_GBS,
               "unit": "GB/s", "frac": round(sweeps * 2 * S / sec / 1e9 / PEAK_HBM_GBS, 4),
               "traffic": None, "bytes": "passes x read + write of the 32 GiB state"}
        mfma = {"bound": "mfma", "achieved": round(dense_flops / sec / 1e12, 2), "peak": PEAK_MFMA_TFLOPS["c64"],
                "unit": "TFLOP/s", "frac": rec["mfma_algorithmic_frac"], "traffic": None,
                "flops": "8 * 2^(N+k) per dense k-qubit op (k >= 3)"}
        # the nearer of the two bounds
        rec["roofline"] = mfma if mfma["frac"] > hbm["frac"] else hbm
        rec["roofline_hbm"] = hbm
        if name == "qft":
            ys = torch.from_numpy(rng.integers(0, 1 << n, size=4096)).cuda()
            got = st.tensor[ys].cpu().numpy().astype(np.complex128)
            y = ys.cpu().numpy().astype(np.float64)
            ref = np.exp(2j * np.pi * ((x0 * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
            rec["closed_form_max_err"] = float(np.max(np.abs(got - ref)))
        out[name] = rec
        plan.close()
    st.close()
    torch.cuda.empty_cache()
    total = sum(v["seconds"] for v in out.values())
    out["seconds"] = round(total, 5)
    out["config"] = {"workload": f"N={n} complex64, brickwork depth 40 (seed 3) + QFT", "mode": args.mode,
                     "steps": steps, "warmup": warmup}
    # HBM bytes per launch of each kernel from the committed counter runs
    # (a pass reads and writes the state once: of_read_plus_write = 1)
    if n == 32 and args.mode == "auto":
        out["kernel_traffic"] = load_circuit_traffic()
    return out


def qaoa_cpu_baseline(gates, n: int):
    """The oracle (numpy, complex128) on a bounded sample of the QAOA circuit:
    one RZZ and one RX of it at N=30 on the host cores, extrapolated to the
    whole gate list by gate kind (H costs what RX costs: one dense 2x2)."""
    import oracle
    from svgen import gaussian_state_np
    host = _host_info()
    psi = gaussian_state_np(n, 2)
    per_kind = {}
    for kind in ("RZZ", "RX"):
        g = next(g for g in gates if g.kind == kind)
        t0 = time.perf_counter()
        psi = oracle.apply_gate(psi, g)
        per_kind[kind] = time.perf_counter() - t0
    del psi
    per_kind["H"] = per_kind["RX"]
    est = sum(per_kind[g.kind] for g in gates)
    return {"value": round(est, 1), "unit": "s", "cores": host["blas_threads"], "kind": "oracle",
            "sample": f"one RZZ and one RX at N={n}, complex128 ({per_kind['RZZ'] + per_kind['RX']:.1f} s), "
                      f"scaled to the {len(gates)} gates by kind", "host": host}


def qaoa_bench(args):
    """QAOA benchmark: five levels on the complete graph K_N (N=30: 2175 RZZ,
    150 RX, 30 H) from |0..0>, complex128 (the paper's precision) and
    complex64, planned once (mode auto) and applied `steps` times after
    `warmup`.  Checks on 4096 sampled amplitudes: the state is symmetric under
    qubit permutations (equal amplitudes for a bit rotation of the index), and
    the two precisions agree."""
    import numpy as np
    import torch

    import paper_2409_14697_amd as sv
    from svgen import qaoa_circuit

    torch.cuda.set_device(0)
    n = args.n
    gates = qaoa_circuit(n, 5, seed=7)
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(9)
    xs = rng.integers(0, 1 << n, size=4096, dtype=np.int64)
    rot = ((xs << 7) | (xs >> (n - 7))) & ((1 << n) - 1)  # the same Hamming weight
    out, samples = {}, {}
    for dtype in ("c128", "c64"):
        st = sv.StateVector(n, dtype, stream=stream)
        t0 = time.perf_counter()
        plan = sv.Plan(n, dtype, gates, {"mode": args.mode})
        plan_s = time.perf_counter() - t0
        for _ in range(args.warmup):
            st.init_basis(0)
            st.apply_plan(plan)
        times = []
        for _ in range(args.steps):
            st.init_basis(0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st.apply_plan(plan)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        sec = sum(times) / len(times)
        got = st.tensor[torch.from_numpy(np.concatenate([xs, rot])).cuda()].cpu().numpy().astype(np.complex128)
        samples[dtype] = got[:4096]
        scale = float(np.max(np.abs(got)))
        n_passes = plan.info()[1]
        S = (1 << n) * (16 if dtype == "c128" else 8)
        kops = plan.kernel_ops()
        out[dtype] = {"seconds": round(sec, 5), "min_s": round(min(times), 5), "gates": len(gates),
                      "passes": n_passes, "kernel_ops": sum(k for k, _ in kops),
                      "phase_ops": sum(lad for _, lad in kops), "plan_s": round(plan_s, 4),
                      "sweep_GBs": round(n_passes * 2 * S / sec / 1e9, 1),
                      "symmetry_max_rel_err": float(np.max(np.abs(got[:4096] - got[4096:]))) / scale}
        st.close()
        plan.close()
        torch.cuda.empty_cache()
    out["c64_vs_c128_max_rel_err"] = float(np.max(np.abs(samples["c64"] - samples["c128"]))) / float(
        np.max(np.abs(samples["c128"])))
    achieved = out["c128"]["sweep_GBs"]
    rec = {"metric": f"QAOA seconds at N={n} (5 levels, complete graph, complex128)",
           "value": out["c128"]["seconds"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * out["c128"]["seconds"], 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"QAOA: N={n}, 5 levels on K_{n} (RZZ on all pairs + RX on all qubits, "
                                  f"angles from seed 7), complex128 and complex64", "mode": args.mode},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None},
           "qaoa": out}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = qaoa_cpu_baseline(gates, n)
    return rec


# ---------------------------------------------------------------- serving
def serve_cpu_baseline(requests, budget_s: float = 8.0):
    """The oracle on a bounded sample of the serving mix: for one request of
    each N in the mix, time its first few gates (at least 2, more while the
    per-N share of `budget_s` allows), extrapolate linearly to the request's
    full gate count, and weight by how often that N occurs.  Returns estimated
    oracle circuits/s over the whole mix."""
    import numpy as np

    from oracle import sv_oracle as so

    host = _host_info()
    by_n = {}
    for r in requests:
        by_n.setdefault(r.n, []).append(r)
    per_n = budget_s / max(1, len(by_n))
    total_s = 0.0
    timed = 0
    for n in sorted(by_n):
        rs = by_n[n]
        gates = rs[0].circuit()
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1.0
        t0 = time.perf_counter()
        k = 0
        while k < len(gates) and (k < 2 or time.perf_counter() - t0 < per_n):
            psi = so.apply_gate(psi, gates[k])
            k += 1
        per_gate = (time.perf_counter() - t0) / k
        timed += k
        mean_gates = sum(r.depth * (r.n + r.n // 2) for r in rs) / len(rs)  # N rotations + N/2 CNOTs per pair
        total_s += per_gate * mean_gates * len(rs)
    return {"value": round(len(requests) / total_s, 4), "unit": "circuits/s", "cores": host["blas_threads"],
            "kind": "oracle",
            "sample": f"oracle (numpy complex128) timed on the first gates of one request per N "
                      f"({timed} gates over N={min(by_n)}..{max(by_n)}), extrapolated linearly in gate count "
                      f"to the {len(requests)}-request mix", "host": host}


def _cpu_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def serve_roofline(st, dt):
    """Roofline of the batched step (the batched tile-pass kernel plus the
    launches of matrix, dense and sweep passes of the step): whichever of HBM
    bytes and VALU flops (both algorithmic: each state read and written once
    per pass, the gates' flops; per second of step time) is nearer its peak."""
    peak_flops = PEAK_VALU_TFLOPS[dt]
    hbm = st["GBs"] / PEAK_HBM_GBS
    alu = st["TFLOPs"] / peak_flops
    common = {"kernel": "batched step (k_pass_batch; k_mpass / dense / sweep launches)",
              "mean_launch_us": round(st["mean_launch_us"], 2),
              "hbm_frac": round(hbm, 4), "alu_frac": round(alu, 4)}
    if alu > hbm:
        return dict({"bound": "alu", "achieved": round(st["TFLOPs"], 2), "peak": peak_flops, "unit": "TFLOP/s",
                     "frac": round(alu, 4), "traffic": None}, **common)
    return dict({"bound": "hbm", "achieved": round(st["GBs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": round(hbm, 4), "traffic": None}, **common)


def _round(d):
    if d is None:
        return None
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def serve_bench(args, requests_by_dtype):
    """Serving form: a stream of circuit requests (N ~ U{12..nmax}, depth ~
    U{20..200} layer pairs of N rotations + N/2 CNOTs, Poisson arrivals)
    served by the continuous-batching loop, per dtype.  For each dtype: a
    closed-loop run (all requests at t=0) measures the saturated throughput X;
    the timed run replays the arrivals at rate 0.8 X."""
    from svgen import serving_requests
    from paper_2409_14697_amd.serve import marshal_requests, jobs_from_marshalled

    import torch

    from paper_2409_14697_amd.serve import DeviceEngine, Server, free_budget

    torch.cuda.set_device(0)
    out = {}
    for dt, count in requests_by_dtype:
        reqs = serving_requests(count, seed=5, n_range=(12, args.nmax), depth_range=(20, 200))
        t0 = time.perf_counter()
        marshalled = marshal_requests(reqs, workers=min(16, _cpu_threads()))
        prep_s = time.perf_counter() - t0

        def run(rate, budget=None, timed=False):
            eng = DeviceEngine(dt, time_launches=timed, matrix_qubits=args.matrix_qubits)
            srv = Server(eng, budget or free_budget(0.8), max_active=args.max_active,
                         plan_workers=min(16, _cpu_threads()))
            res = srv.run(jobs_from_marshalled(reqs, marshalled, rate))
            stats = eng.launch_stats() if timed else None
            eng.close()
            torch.cuda.synchronize()
            return res, stats
        # warm-up: allocator, kernels, planner threads
        warm = max(1, min(32, len(reqs) // 8))
        eng = DeviceEngine(dt, matrix_qubits=args.matrix_qubits)
        Server(eng, free_budget(0.8), plan_workers=4).run(jobs_from_marshalled(reqs[:warm], marshalled[:warm], None))
        eng.close()
        closed, _ = run(None)
        sat = closed.summary()["circuits_per_s"]
        lam = args.rate_fraction * sat
        timed, stats = run(lam, timed=True)
        rec = {"requests": count, "closed_loop": _round(closed.summary()), "rate_per_s": round(lam, 3),
               "poisson": _round(timed.summary()), "launch": _round(stats), "roofline": serve_roofline(stats, dt),
               "prep_s": round(prep_s, 2)}
        if args.contention_gib > 0:
            cont, _ = run(lam, budget=int(args.contention_gib * (1 << 30)))
            rec["contention"] = dict(_round(cont.summary()), budget_gib=args.contention_gib)
        out[dt] = rec
        log(f"serve {dt}: {count} requests, closed {sat:.1f}/s, poisson {timed.summary()['circuits_per_s']:.1f}/s "
            f"p99 {timed.summary()['p99_ms']:.1f} ms")
        if not args.no_cpu_baseline and "cpu_baseline" not in out:
            out["cpu_baseline"] = serve_cpu_baseline(reqs)
    out["config"] = {"workload": f"serving: requests N~U{{12..{args.nmax}}}, depth~U{{20..200}} layer pairs "
                                 f"(seed 5), Poisson arrivals at {args.rate_fraction} x closed-loop throughput, "
                                 f"budget 0.8 x free HBM, AUTO plans from N={args.matrix_qubits}"}
    return out


# ---------------------------------------------------------------- precision form
def _compare(a64, b128):
    """FP64 error metrics of a complex64 state against a complex128 one
    (chunked, on the device): max-abs, relative L2, infidelity, norm drift."""
    import torch
    step = 1 << 26
    max_abs, diff2, ref2, own2 = 0.0, 0.0, 0.0, 0.0
    inner = torch.zeros((), dtype=torch.complex128, device=b128.device)
    for s0 in range(0, b128.numel(), step):
        x = a64[s0:s0 + step].to(torch.complex128)
        y = b128[s0:s0 + step]
        d = x - y
        max_abs = max(max_abs, float(d.abs().max()))
        diff2 += float((d.real ** 2 + d.imag ** 2).sum())
        ref2 += float((y.real ** 2 + y.imag ** 2).sum())
        own2 += float((x.real ** 2 + x.imag ** 2).sum())
        inner += torch.vdot(y, x)
    fid = abs(complex(inner)) ** 2 / (ref2 * own2)
    return {"max_abs": max_abs, "rel_l2": math.sqrt(diff2 / ref2), "infidelity": 1.0 - fid,
            "norm_drift_fp32": own2 - 1.0, "norm_drift_fp64": ref2 - 1.0}


def precision_bench(args, seeds, n_gates, checkpoint):
    """Precision form: N=30, `n_gates` Haar-random 5- and 6-qubit unitaries on
    random ordered qubit sets; complex64 state with FP32 MFMA contractions
    (FP32 accumulation, FP64 renormalisation every `renorm` ops) against a
    complex128 state with the FP64 matrix-core kernel, same GPU, same seeded
    input.  Errors are taken at checkpoints; one record per seed."""
    import torch

    import paper_2409_14697_amd as sv
    from svgen import fused_haar_circuit
    from svgen.states import gaussian_state_torch

    torch.cuda.set_device(0)
    n = args.n
    stream = torch.cuda.current_stream()
    records = []
    t32_total = t64_total = 0.0
    flops = {"c64": 0.0, "c128": 0.0}
    for seed in seeds:
        gates = fused_haar_circuit(n, n_gates, seed=seed)
        gflops = sum(8.0 * 2.0 ** (n + len(g.qubits)) for g in gates)
        s128 = gaussian_state_torch(n, seed, torch.complex128)
        s64 = s128.to(torch.complex64)
        st64 = sv.StateVector(n, "c128", tensor=s128, init=False, stream=stream)
        st32 = sv.StateVector(n, "c64", tensor=s64, init=False, stream=stream)
        rec = {"seed": seed, "gates": len(gates), "checkpoints": []}
        t32 = t64 = 0.0
        for g0 in range(0, len(gates), checkpoint):
            part = gates[g0:g0 + checkpoint]
            for st, dtype in ((st32, "c64"), (st64, "c128")):
                opts = {"mode": "sweep", "max_fuse_qubits": 0}
                if dtype == "c64":
                    opts["renorm_interval"] = args.renorm
                plan = sv.Plan(n, dtype, part, opts)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                st.apply_plan(plan)
                e1.record(stream)
                torch.cuda.synchronize()
                plan.close()
                dt = e0.elapsed_time(e1) * 1e-3
                if dtype == "c64":
                    t32 += dt
                else:
                    t64 += dt
            m = _compare(s64, s128)
            m["after_gates"] = g0 + len(part)
            rec["checkpoints"].append({k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in m.items()})
        rec["fp32_mfma_s"] = round(t32, 4)
        rec["fp64_s"] = round(t64, 4)
        records.append(rec)
        t32_total += t32
        t64_total += t64
        flops["c64"] += gflops
        flops["c128"] += gflops
        st32.close()
        st64.close()
        del s64, s128
        torch.cuda.empty_cache()
    final_err = max(r["checkpoints"][-1]["max_abs"] for r in records)
    mfma32 = flops["c64"] / t32_total / 1e12
    mfma64 = flops["c128"] / t64_total / 1e12
    return {"fp32_mfma_s": round(t32_total / len(records), 4), "fp64_s": round(t64_total / len(records), 4),
            "fp32_max_abs_error": final_err, "bar_max_abs": 1e-5,
            "roofline_fp32": {"bound": "mfma", "achieved": round(mfma32, 2), "peak": PEAK_MFMA_TFLOPS["c64"],
                              "unit": "TFLOP/s", "frac": round(mfma32 / PEAK_MFMA_TFLOPS["c64"], 4),
                              "traffic": None, "flops": "8 * 2^(N+k) per k-qubit gate (real embedding)"},
            "roofline_fp64": {"bound": "mfma", "achieved": round(mfma64, 2), "peak": PEAK_MFMA_TFLOPS["c128"],
                              "unit": "TFLOP/s", "frac": round(mfma64 / PEAK_MFMA_TFLOPS["c128"], 4),
                              "traffic": None},
            "config": {"workload": f"precision form: N={n}, {n_gates} Haar unitaries alternating k=5/6 "
                                   f"(seeds {seeds}), renorm every {args.renorm}"},
            "records": records}


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 10 for gates, the gate benchmark's 10 repetitions; 3 otherwise)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=N_QUBITS)
    ap.add_argument("--dtypes", default="c128,c64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-ceiling", action="store_true", help="also time the 16-byte copy kernel")
    ap.add_argument("--extras", default="circuit,precision,serve",
                    help="default workload: parts of the metric run after the gate benchmark ('none' for none)")
    ap.add_argument("--circuit-steps", type=int, default=2)
    ap.add_argument("--circuit-warmup", type=int, default=1)
    ap.add_argument("--requests", type=int, default=None, help="serve workload: number of requests")
    ap.add_argument("--serve-default", default="c64:4096,c128:1024",
                    help="default workload's serving part: dtype:requests list")
    ap.add_argument("--nmax", type=int, default=26, help="serve workload: largest request N")
    ap.add_argument("--max-active", type=int, default=512, help="serve workload: slot cap")
    ap.add_argument("--matrix-qubits", type=int, default=24,
                    help="serve workload: requests of at least this many qubits use AUTO plans (0: tile passes only)")
    ap.add_argument("--rate-fraction", type=float, default=0.8, help="serve workload: arrival rate / saturated rate")
    ap.add_argument("--contention-gib", type=float, default=0.0,
                    help="serve workload: also run with this HBM budget (GiB)")
    ap.add_argument("--workload", default="gates", choices=["gates", "circuit", "precision", "serve", "qaoa"],
                    help="gates: the default line (gate benchmark + extras); circuit: N=32 circuits; "
                         "precision: FP32 MFMA vs FP64 fused Haar gates; serve: the serving form; qaoa")
    ap.add_argument("--gates", type=int, default=2000, help="precision workload: number of fused gates")
    ap.add_argument("--checkpoint", type=int, default=250, help="precision workload: gates between error checks")
    ap.add_argument("--seeds", default="4,5,6", help="precision workload: circuit seeds")
    ap.add_argument("--renorm", type=int, default=250, help="precision workload: FP64 renorm interval (0: off)")
    ap.add_argument("--mode", default="auto", choices=["auto", "pass", "sweep", "matrix"], help="plan mode (circuit and qaoa workloads)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the state-vector hot path here runs on a single MI355X "
              "(no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 10 if args.workload == "gates" else 3
    common = {"n_gpus": 1, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if args.workload == "circuit":
        args.circuit_steps, args.circuit_warmup = args.steps, args.warmup
        c = circuit_bench(args, n=32 if args.n == N_QUBITS else args.n)
        print(json.dumps(dict({"metric": "circuit seconds at N=32 (complex64)", "value": c["seconds"], "unit": "s",
                               "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * c["seconds"], 3),
                               "higher_is_better": False, "dtype": "f32", "config": c.pop("config"),
                               "roofline": c["brickwork_d40"]["roofline"], "circuits": c}, **common)))
        return
    if args.workload == "precision":
        p = precision_bench(args, [int(x) for x in args.seeds.split(",")], args.gates, args.checkpoint)
        print(json.dumps(dict({"metric": f"precision form: seconds for {args.gates} fused 5/6-qubit gates at N={args.n}, "
                                         "FP32 MFMA vs FP64", "value": p["fp32_mfma_s"], "unit": "s",
                               "steps": len(p["records"]), "warmup": 0, "ms_per_step": round(1e3 * p["fp32_mfma_s"], 3),
                               "higher_is_better": False, "dtype": "f32 (vs f64)", "config": p.pop("config"),
                               "roofline": p["roofline_fp32"], "precision": p}, **common)))
        return
    if args.workload == "serve":
        count = args.requests or 512
        s = serve_bench(args, [(d, count) for d in args.dtypes.split(",") if d])
        main_dt = "c64" if "c64" in s else args.dtypes.split(",")[0]
        summ = s[main_dt]["poisson"]
        line = dict({"metric": "served circuits/s", "value": summ["circuits_per_s"], "unit": "circuits/s",
                     "steps": summ["completed"], "warmup": 1,
                     "ms_per_step": round(1e3 / max(summ["circuits_per_s"], 1e-9), 3), "higher_is_better": True,
                     "dtype": "f32" if main_dt == "c64" else "f64",
                     "config": dict(s.pop("config"), requests=count, p99_ms=summ["p99_ms"], p50_ms=summ["p50_ms"]),
                     "roofline": s[main_dt]["roofline"], "serving": s}, **common)
        if "cpu_baseline" in s:
            line["cpu_baseline"] = s.pop("cpu_baseline")
        print(json.dumps(line))
        return
    if args.workload == "qaoa":
        print(json.dumps(qaoa_bench(args)))
        return

    # ---- default line: the gate benchmark (headline), then the other parts
    t_start = time.perf_counter()
    g = gates_bench(args)
    log(f"gates: c128 {g['per_dtype'].get('c128', {}).get('GB/s')} GB/s, c64 {g['per_dtype'].get('c64', {}).get('GB/s')} "
        f"GB/s ({time.perf_counter() - t_start:.0f} s)")
    gates = g.pop("gates")
    head = g["head"]
    out = dict({
        "metric": "HBM GB/s per gate at N=30 (gate sweep benchmark)",
        "value": g["value"],
        "unit": "GB/s",
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g["per_dtype"][head]["ms_per_step"],
        "higher_is_better": True,
        "dtype": {"c128": "f64", "c64": "f32"}[head],
        "config": {"workload": f"gate sweep benchmark: N={args.n}, Gaussian state (seed 2), H/X/RZ/CNOT/CZ/SWAP/CPHASE "
                               f"on every target (partners random, seed 2); value: {head}",
                   "n_qubits": args.n, "gates_per_step": len(gates), "dtypes": args.dtypes},
        "by_dtype": {d: {k: v for k, v in r.items() if k not in ("kernel_s", "bytes")} for d, r in g["per_dtype"].items()},
        "launch_min": g["launch_min"],
        "per_kernel": g["per_kernel"],
        "roofline": g["roofline"],
    }, **common)
    if g["copy_kernel_GBs"] is not None:
        out["copy_kernel_GBs"] = g["copy_kernel_GBs"]
    extras = [] if args.extras == "none" else [x for x in args.extras.split(",") if x]
    if "circuit" in extras:
        t0 = time.perf_counter()
        out["circuit"] = circuit_bench(args, n=32)
        log(f"circuit: {out['circuit']['seconds']} s ({time.perf_counter() - t0:.0f} s)")
    if "precision" in extras:
        t0 = time.perf_counter()
        out["precision"] = precision_bench(args, [4], args.gates, 500)
        log(f"precision: fp32 {out['precision']['fp32_mfma_s']} s, fp64 {out['precision']['fp64_s']} s "
            f"({time.perf_counter() - t0:.0f} s)")
    if "serve" in extras:
        t0 = time.perf_counter()
        plan = []
        for item in args.serve_default.split(","):
            d, c = item.split(":")
            plan.append((d, int(c)))
        out["serving"] = serve_bench(args, plan)
        log(f"serving ({time.perf_counter() - t0:.0f} s)")
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(gates, args.n)
        log(f"cpu baseline ({time.perf_counter() - t0:.0f} s)")
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
