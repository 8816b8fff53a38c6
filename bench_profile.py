"""Summarise rocprofv3 output of bench.py into profiles/ (host side, no GPU).

Inputs are the CSV directories of three profiled runs of bench.py:
  --trace : rocprofv3 --kernel-trace --stats -f csv -d <dir> -o bench -- python bench.py --extras none
  --fetch : rocprofv3 --pmc FETCH_SIZE -f csv -d <dir> -o bench -- python bench.py --steps 1 --warmup 0
            --no-cpu-baseline --copy-ceiling --extras none
  --write : the same with --pmc WRITE_SIZE
Subcommands `trace` (kernel-trace summary of any profiled run), `mfma`
(matrix-core utilisation of the dense kernels from a counter run) and
`circuit` (HBM traffic per launch of the circuit benchmark's kernels) write
their own summaries.
Outputs:
  profiles/gate_sweep_n30.md              per-kernel durations (kernel trace) and
                                          calibrated HBM traffic (counters)
  profiles/gate_sweep_counters_n30.json   bytes per launch, read by bench.py's
                                          roofline "traffic" field

Calibration: the copy kernel (sv_util_copy) moves a known number of bytes
(2^(N-1) complex128 elements read and written); FETCH_SIZE and WRITE_SIZE (KiB
per dispatch) are each scaled by known bytes / counter value for that kernel.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def short(name: str) -> str:
    """Kernel name without namespaces and argument list."""
    n = name.replace("void ", "", 1)
    n = n.replace("sv::(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def counters(d: str, counter: str):
    rows = list(csv.DictReader(open(os.path.join(d, "bench_counter_collection.csv"))))
    per = defaultdict(list)
    for r in rows:
        if r["Counter_Name"] == counter:
            per[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per


def trace_summary(argv):
    """Kernel-trace summary of any profiled bench.py run:
    bench_profile.py trace --dir D --out profiles/NAME.md --title T --cmd "C" [--result R.json]"""
    ap = argparse.ArgumentParser(prog="bench_profile.py trace")
    ap.add_argument("--dir", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--cmd", required=True, help="the profiled command, as run from the repository root")
    ap.add_argument("--result", help="the JSON line the profiled run printed (figures quoted in the summary)")
    ap.add_argument("--min-pct", type=float, default=0.5)
    args = ap.parse_args(argv)
    stats = list(csv.DictReader(open(os.path.join(args.dir, "bench_kernel_stats.csv"))))
    lines = [f"# {args.title}: rocprofv3 kernel trace", "",
             "Command (from the repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```", args.cmd, "```", "",
             f"## Kernels above {args.min_pct}% of GPU time", "",
             "| kernel | calls | avg us | min us | max us | total ms | total % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in stats:
        if float(r["Percentage"]) < args.min_pct:
            continue
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    if args.result:
        with open(args.result) as f:
            line = [l for l in f.read().splitlines() if l.startswith("{")][-1]
        res = json.loads(line)
        lines += ["", "## The profiled run's own report", "", "```",
                  json.dumps({k: res[k] for k in ("metric", "value", "unit", "roofline") if k in res}, indent=1),
                  "```"]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}")


SIMDS = 256 * 4        # MI355X: 256 CUs, 4 SIMDs each
CLOCK_HZ = 2.4e9       # peak engine clock
MATRIX_PEAK = {"float": 157.3e12, "double": 78.6e12}  # dense MFMA FP32 / FP64


def mfma_summary(argv):
    """Matrix-core utilisation of the dense fused kernels from one counter run:
    bench_profile.py mfma --dir D --n N --out profiles/NAME.md --title T --cmd "C"
    where the run collected SQ_VALU_MFMA_BUSY_CYCLES (summed over all SIMDs).
    Busy fraction = counter / (SIMDs x kernel duration x clock); the algorithmic
    rate counts 8 * 2^(N+k) real flops per k-qubit gate (the complex product
    by definition) against the dense matrix peak of the kernel's type; the
    three-product kernels (k_dense_3m) perform 6 * 2^(N+k) of them, the
    embedding kernels (k_dense_mfma) 8 * 2^(N+k)."""
    ap = argparse.ArgumentParser(prog="bench_profile.py mfma")
    ap.add_argument("--dir", required=True)
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--cmd", required=True)
    args = ap.parse_args(argv)
    rows = list(csv.DictReader(open(os.path.join(args.dir, "bench_counter_collection.csv"))))
    per = defaultdict(lambda: {"busy": [], "dur": []})
    seen = {}
    for r in rows:
        if r["Counter_Name"] != "SQ_VALU_MFMA_BUSY_CYCLES" or not any(
                k in r["Kernel_Name"] for k in ("k_dense_mfma", "k_dense_3m", "k_mpass")):
            continue
        key = (r["Dispatch_Id"], short(r["Kernel_Name"]))
        seen.setdefault(key, [0.0, (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9])
        seen[key][0] += float(r["Counter_Value"])
    for (_, name), (busy, dur) in seen.items():
        per[name]["busy"].append(busy)
        per[name]["dur"].append(dur)
    lines = [f"# {args.title}: matrix-core utilisation (rocprofv3 counters)", "",
             "Command (from the repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```", args.cmd, "```", "",
             f"Busy = SQ_VALU_MFMA_BUSY_CYCLES / ({SIMDS} SIMDs x duration x {CLOCK_HZ / 1e9:.1f} GHz). Algorithmic = "
             f"8 * 2^(N+k) flops per gate at N={args.n} / duration, against the dense matrix peak "
             "(FP32 157.3, FP64 78.6 TFLOP/s).", "",
             "| kernel | dispatches | avg ms | MFMA busy | algorithmic TFLOP/s | of matrix peak | performed TFLOP/s |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for name in sorted(per):
        d = per[name]
        k = int(name.split(",")[1].strip(" >"))
        rtype = name.split("<")[1].split(",")[0].strip()
        dur = statistics.mean(d["dur"])
        busy = statistics.mean(b / (SIMDS * t * CLOCK_HZ) for b, t in zip(d["busy"], d["dur"]))
        if "k_mpass" in name:
            # a matrix pass runs several ops per dispatch (one per stage): the
            # counters give its matrix-core busy fraction; its algorithmic rate
            # is in the profiled run's own report
            lines.append(f"| `{name}` | {len(d['dur'])} | {dur * 1e3:.3f} | {busy:.3f} | - | - | - |")
            continue
        tflops = 8.0 * 2.0 ** (args.n + k) / dur / 1e12
        done = tflops * (0.75 if "k_dense_3m" in name else 1.0)
        lines.append(f"| `{name}` | {len(d['dur'])} | {dur * 1e3:.3f} | {busy:.3f} | {tflops:.1f} | "
                     f"{tflops * 1e12 / MATRIX_PEAK[rtype]:.3f} | {done:.1f} |")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}")


def circuit_traffic(argv):
    """HBM traffic per launch of the circuit benchmark's kernels (N=32
    complex64): bench_profile.py circuit --fetch D --write D, the counter runs
    of `bench.py --workload circuit --steps 1 --warmup 0`.  FETCH_SIZE and
    WRITE_SIZE are scaled by the copy-kernel factors recorded in
    profiles/gate_sweep_counters_n30.json (same counters, same device);
    writes profiles/circuit_traffic_n32_c64.{md,json}."""
    import bench
    ap = argparse.ArgumentParser(prog="bench_profile.py circuit")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args(argv)
    with open(os.path.join(ROOT, "profiles", "gate_sweep_counters_n30.json")) as f:
        cal = json.load(f)["copy_calibration"]
    f_fetch, f_write = cal["fetch_factor"], cal["write_factor"]
    fetch, write = counters(args.fetch, "FETCH_SIZE"), counters(args.write, "WRITE_SIZE")
    two_s = 2.0 * float(1 << args.n) * 8.0  # read + write of the complex64 state
    kernels = {}
    for sym, vals in fetch.items():
        if sym not in write or not sym.startswith("k_"):
            continue
        fk, wk = statistics.mean(vals), statistics.mean(write[sym])
        b = (fk * f_fetch + wk * f_write) * 1024.0
        kernels[sym] = {"launches": len(vals), "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                        "bytes_per_launch": round(b), "of_read_plus_write": round(b / two_s, 4)}
    with open(os.path.join(args.out, "circuit_traffic_n32_c64.json"), "w") as f:
        json.dump({"source_hash": bench.circuit_source_hash(), "n_qubits": args.n, "dtype": "c64",
                   "copy_calibration": {"fetch_factor": f_fetch, "write_factor": f_write},
                   "read_plus_write_bytes": two_s, "kernels": kernels}, f, indent=1, sort_keys=True)
    lines = ["# Circuit benchmark, N=32 complex64: HBM traffic per kernel launch (rocprofv3 counters)", "",
             "Commands (from the repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```",
             "rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/prof_cfetch -o bench -- python bench.py --workload circuit "
             "--steps 1 --warmup 0",
             "rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/prof_cwrite -o bench -- python bench.py --workload circuit "
             "--steps 1 --warmup 0",
             "python bench_profile.py circuit --fetch gpurun_out/prof_cfetch --write gpurun_out/prof_cwrite",
             "```", "",
             f"Bytes = FETCH_SIZE x {f_fetch:.3f} + WRITE_SIZE x {f_write:.3f} (KiB per dispatch; the factors that turn "
             "the copy kernel's counters into its known bytes, from the gate-sweep counter runs). A pass reads and "
             f"writes the 32 GiB state once: {two_s:.4g} bytes. Kernel source hash: `{bench.circuit_source_hash()}`.", "",
             "| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes / launch | of read + write |",
             "|---|---:|---:|---:|---:|---:|"]
    for sym, k in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"] * kv[1]["launches"]):
        lines.append(f"| `{sym}` | {k['launches']} | {k['fetch_kib']:.0f} | {k['write_kib']:.0f} | "
                     f"{k['bytes_per_launch']:.4g} | {k['of_read_plus_write']:.4f} |")
    with open(os.path.join(args.out, "circuit_traffic_n32_c64.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}/circuit_traffic_n32_c64.md and .json")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "circuit":
        circuit_traffic(sys.argv[2:])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "trace":
        trace_summary(sys.argv[2:])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "mfma":
        mfma_summary(sys.argv[2:])
        return
    import bench
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()

    stats = list(csv.DictReader(open(os.path.join(args.trace, "bench_kernel_stats.csv"))))
    fetch, write = counters(args.fetch, "FETCH_SIZE"), counters(args.write, "WRITE_SIZE")
    copy = "k_copy16"
    copy_bytes = float(1 << (args.n - 1)) * 16.0
    f_fetch = copy_bytes / 1024.0 / statistics.mean(fetch[copy])
    f_write = copy_bytes / 1024.0 / statistics.mean(write[copy])

    import paper_2409_14697_amd as sv
    from svgen import gate_bench_set
    keys = sorted({sv.gate_kernel(args.n, dt, g) for dt in ("c128", "c64") for g in gate_bench_set(args.n, seed=2)})
    sym2key = {bench.kernel_symbol(k): k for k in keys}

    kernels = {}
    for sym, vals in fetch.items():
        if sym not in write or not sym.startswith("k_"):  # this library's kernels only
            continue
        key = sym2key.get(sym, sym)
        fk, wk = statistics.mean(vals), statistics.mean(write[sym])
        kernels[key] = {"symbol": sym, "launches": len(vals), "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                        "bytes_per_launch": round((fk * f_fetch + wk * f_write) * 1024.0)}
    os.makedirs(args.out, exist_ok=True)
    with open(os.path.join(args.out, "gate_sweep_counters_n30.json"), "w") as f:
        json.dump({"source_hash": bench.kernel_source_hash(), "n_qubits": args.n,
                   "copy_calibration": {"fetch_factor": round(f_fetch, 4), "write_factor": round(f_write, 4),
                                        "copy_bytes_each_way": copy_bytes},
                   "kernels": kernels}, f, indent=1, sort_keys=True)

    lines = ["# Gate-sweep benchmark, N=30 (complex128 + complex64): rocprofv3 summary", "",
             "Commands (run from the repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```",
             "rocprofv3 --kernel-trace --stats -f csv -d gpurun_out/prof_trace -o bench -- python bench.py --extras none",
             "rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/prof_fetch -o bench -- python bench.py --steps 1 "
             "--warmup 0 --no-cpu-baseline --copy-ceiling --extras none",
             "rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/prof_write -o bench -- python bench.py --steps 1 "
             "--warmup 0 --no-cpu-baseline --copy-ceiling --extras none",
             "python bench_profile.py --trace gpurun_out/prof_trace --fetch gpurun_out/prof_fetch "
             "--write gpurun_out/prof_write",
             "```", "",
             f"Kernel source hash: `{bench.kernel_source_hash()}`.", "",
             "## Kernel trace (--stats), kernels above 0.5% of GPU time", "",
             "| kernel | identifier | calls | avg ms | total % |", "|---|---|---:|---:|---:|"]
    for r in stats:
        if float(r["Percentage"]) < 0.5:
            continue
        sym = short(r["Name"])
        lines.append(f"| `{sym}` | {sym2key.get(sym, '')} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['Percentage']):.2f} |")
    lines += ["", "## HBM traffic per launch (FETCH_SIZE x %.3f + WRITE_SIZE x %.3f, calibrated on the copy kernel)"
              % (f_fetch, f_write), "",
              "| identifier | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes / launch |", "|---|---:|---:|---:|---:|"]
    for key, k in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"] * kv[1]["launches"]):
        lines.append(f"| {key} | {k['launches']} | {k['fetch_kib']:.0f} | {k['write_kib']:.0f} | "
                     f"{k['bytes_per_launch']:.4g} |")
    with open(os.path.join(args.out, "gate_sweep_n30.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}/gate_sweep_n30.md and gate_sweep_counters_n30.json "
          f"(fetch x{f_fetch:.3f}, write x{f_write:.3f})")


if __name__ == "__main__":
    main()
