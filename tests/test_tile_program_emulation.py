"""The device program of the in-cache tile passes (register stages: 2x2
layers in their forms, register factors, lane items, fixed-point phase items
and their row tables, register permutations), executed by a host model of
the pass kernel (tests/emu/tile_program_emu.cpp) with bounds checks on every
program read, against the oracle.  No GPU: this pins the planner's encoding
and the packer's offsets, which the kernel trusts without checks."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from svgen import (Gate, brickwork_circuit, fused_haar_circuit, gaussian_state_np, haar_unitary, layered_circuit,
                   qaoa_circuit, qft_circuit)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_14697_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "emu", "tile_program_emu.cpp")
BIN = os.path.join(ROOT, "_build", "tile_program_emu")
KIND = {"MATRIX": 0, "H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "T": 6, "RX": 7, "RY": 8, "RZ": 9, "P": 10,
        "CNOT": 11, "CZ": 12, "SWAP": 13, "CPHASE": 14, "RZZ": 15}
TOL = {"c128": 1e-12, "c64": 1e-5}


# SV_SANITIZE=1: the model (and with it the library's planner and packer
# sources) is built with AddressSanitizer and UndefinedBehaviorSanitizer,
# aborting on the first report.
SANITIZE = os.environ.get("SV_SANITIZE", "") not in ("", "0")


def build_model(binary, sanitize):
    srcs = [SRC] + [os.path.join(CSRC, f) for f in ("sv_plan.cpp", "sv_passplan.cpp", "sv_gates.cpp")]
    newest = max(os.path.getmtime(f) for f in srcs + [os.path.join(CSRC, "sv_tile_kernels.h"),
                                                      os.path.join(CSRC, "sv_host.h")])
    if not os.path.exists(binary) or os.path.getmtime(binary) < newest:
        os.makedirs(os.path.dirname(binary), exist_ok=True)
        flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"] if sanitize else ["-O2"]
        cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
               f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"] + flags + srcs + ["-o", binary]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
    return binary


@pytest.fixture(scope="module")
def emu():
    return build_model(BIN + ("_asan" if SANITIZE else ""), SANITIZE)


def run_emu(binary, n, dtype, mode, lds, gates, psi0):
    lines = [f"{n} {dtype} {mode} {lds}"]
    for g in gates:
        k = KIND[g.kind]
        s = f"{k} {len(g.qubits)} {' '.join(str(q) for q in g.qubits)} {float(g.theta or 0.0)!r}"
        if k == 0:
            m = np.asarray(g.matrix, dtype=np.complex128).reshape(-1)
            s += " " + " ".join(f"{float(x.real)!r} {float(x.imag)!r}" for x in m)
        lines.append(s)
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
        for x in psi0:
            f.write(f"{float(x.real)!r} {float(x.imag)!r}\n")
        init = f.name
    try:
        r = subprocess.run([binary], input="\n".join(lines) + "\n", capture_output=True, text=True,
                           env=dict(os.environ, SV_EMU_INIT=init), timeout=300)
    finally:
        os.unlink(init)
    assert r.returncode == 0, r.stderr
    a = np.array([[float(v) for v in line.split()] for line in r.stdout.splitlines()])
    return a[:, 0] + 1j * a[:, 1]


def mixed(n, count, seed):
    from tests.test_gpu_passes import mixed_circuit
    return mixed_circuit(n, count, seed)


def permutations(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(3))
        if k == 0:
            out.append(Gate("X", (int(rng.integers(n)),)))
        else:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append(Gate("CNOT" if k == 1 else "SWAP", (a, b)))
    return out


def dense_pairs(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        r = rng.random()
        if r < 0.3:
            out.append(Gate("MATRIX", (a, b), matrix=haar_unitary(4, rng)))
        elif r < 0.5:
            out.append(Gate("CNOT", (a, b)))
        elif r < 0.7:
            out.append(Gate("RZZ", (a, b), float(rng.uniform(0, 6))))
        else:
            out.append(Gate("RX", (a,), float(rng.uniform(0, 6))))
    return out


def circuits():
    from tests.test_gpu_passes import (diagonal_run_circuit, interleaved_phase_circuit, ladder_circuit,
                                       phase_run_circuit)
    n = 11
    return {
        "layered": (n, lambda: layered_circuit(n, n_gates=250, seed=1)),
        "brickwork": (n, lambda: brickwork_circuit(n, 8, seed=3)),
        "qft": (n, lambda: qft_circuit(n)),
        "qaoa": (n, lambda: qaoa_circuit(n, 2, seed=7)),
        "mixed": (n, lambda: mixed(n, 250, 7)),
        "ladders": (n, lambda: ladder_circuit(n, 1)),
        "phase_runs": (n, lambda: phase_run_circuit(n, 3)),
        "diag_runs": (n, lambda: diagonal_run_circuit(n, 9)),
        "interleaved": (n, lambda: interleaved_phase_circuit(n, 300, 8)),
        "dense_pairs": (n, lambda: dense_pairs(n, 60, 5)),
        "haar": (n, lambda: fused_haar_circuit(n, 5, seed=4, ks=(2, 3))),
        "small": (6, lambda: mixed(6, 150, 6)),
    }


@pytest.mark.parametrize("name", sorted(circuits()))
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tile_program_model_matches_oracle(emu, name, dtype):
    n, make = circuits()[name]
    gates = make()
    psi = gaussian_state_np(n, 5)
    ref = oracle.run(gates, psi0=psi)
    for lds in (0, 6, 9):
        if lds > n:
            continue
        out = run_emu(emu, n, dtype, "pass", lds, gates, psi)
        assert np.max(np.abs(out - ref)) <= TOL[dtype], (name, dtype, lds)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tile_program_model_permutations_exact(emu, dtype):
    """X, CNOT and SWAP only: the register permutations and permutation terms
    move amplitudes without arithmetic, bitwise."""
    n = 11
    gates = permutations(n, 200, 5)
    psi = gaussian_state_np(n, 3)
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    for lds in (0, 5, 8):
        out = run_emu(emu, n, dtype, "pass", lds, gates, psi)
        assert np.array_equal(out, oracle.run(gates, psi0=psi)), lds


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("name", ["brickwork", "grouped"])
def test_matrix_pass_model_matches_oracle(emu, name, dtype):
    """Matrix passes as packed for the kernel (member bits, pool matrices,
    column orders, barrier flags): the host model applies the stages and
    checks that a stage without a barrier keeps every element with its
    wave, against the oracle.  N = 14: two tiles."""
    n = 14
    rng = np.random.default_rng(3)
    if name == "brickwork":
        gates = brickwork_circuit(n, 12, seed=2)
    else:
        gates = []
        pin = 4 if dtype == "c64" else 3
        for _ in range(4):
            pool = list(range(pin)) + [int(x) for x in rng.choice(np.arange(pin, n), 8, replace=False)]
            for _ in range(3):
                k = int(rng.integers(2, 6))
                qs = tuple(int(x) for x in rng.choice(pool, k, replace=False))
                gates.append(Gate("MATRIX", qs, matrix=haar_unitary(1 << k, rng)))
    psi = gaussian_state_np(n, 6)
    out = run_emu(emu, n, dtype, "matrix", 0, gates, psi)
    assert np.max(np.abs(out - oracle.run(gates, psi0=psi))) <= TOL[dtype], (name, dtype)


def test_tile_program_model_under_sanitizers():
    """The planner and packer sources, built with AddressSanitizer and
    UndefinedBehaviorSanitizer into the host model, plan and run a mixed
    circuit, a QAOA level and the QFT without a report."""
    binary = build_model(BIN + "_asan", True)
    n = 10
    for gates in (mixed(n, 200, 3), qaoa_circuit(n, 1, seed=2), qft_circuit(n)):
        psi = gaussian_state_np(n, 2)
        out = run_emu(binary, n, "c64", "pass", 0, gates, psi)
        assert np.max(np.abs(out - oracle.run(gates, psi0=psi))) <= TOL["c64"]
