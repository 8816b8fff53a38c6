"""ctypes binding of libsv.so (include/sv.h).  Argument marshalling only: every
step of the simulation runs in the library's HIP kernels; torch supplies device
memory and the stream.

The library is loaded from this package directory; if it is missing the import
of the binding fails loudly (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_size_t, c_uint, c_uint64, c_void_p
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# SV_LIBRARY names another build of the same library (the sanitizer build of
# build.py); the default is the in-tree libsv.so
LIB_PATH = os.environ.get("SV_LIBRARY") or os.path.join(PKG, "libsv.so")
ROOT = os.path.dirname(PKG)
HEADERS = [os.path.join(ROOT, "include", "sv.h"), os.path.join(ROOT, "include", "sv_util.h")]

SV_OK, SV_ERR_ARG, SV_ERR_QUBIT, SV_ERR_NOMEM, SV_ERR_DEVICE, SV_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SV_C64, SV_C128 = 1, 2
SV_NO_INIT = 1
MODE = {"auto": 0, "sweep": 1, "pass": 2, "matrix": 3}
KIND = {"MATRIX": 0, "H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "T": 6, "RX": 7, "RY": 8, "RZ": 9, "P": 10,
        "CNOT": 11, "CZ": 12, "SWAP": 13, "CPHASE": 14, "RZZ": 15}
MAXQ = 6


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sv error {status}: {msg}")
        self.status = status


class SvGate(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("nq", c_int32), ("q", c_int32 * MAXQ), ("theta", c_double),
                ("m", POINTER(c_double))]


class SvOpts(ctypes.Structure):
    _fields_ = [("max_fuse_qubits", c_int32), ("lds_qubits", c_int32), ("pinned_low_bits", c_int32),
                ("reorder", c_int32), ("fp32_mfma", c_int32), ("renorm_interval", c_int32), ("mode", c_int32),
                ("max_pass_ops", c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          f"(python paper_2409_14697_amd/build.py); there is no fallback")
    # torch ships its own HIP runtime (same soname, libamdhip64.so.7).  Loading
    # torch first makes libsv.so bind to that runtime, so device pointers and
    # streams that torch hands over are valid in the library; loading libsv.so
    # first would bring in a second runtime instance.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    S = c_int  # sv_status
    sig = {
        "sv_default_opts": (S, [POINTER(SvOpts)]),
        "sv_create": (S, [c_int, c_int, c_void_p, c_void_p, c_uint, POINTER(c_void_p)]),
        "sv_destroy": (S, [c_void_p]),
        "sv_state_info": (S, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_void_p)]),
        "sv_set_stream": (S, [c_void_p, c_void_p]),
        "sv_init_basis": (S, [c_void_p, c_uint64]),
        "sv_apply_gate": (S, [c_void_p, POINTER(SvGate)]),
        "sv_fuse": (S, [c_int, c_int, POINTER(SvGate), c_size_t, POINTER(SvOpts), POINTER(c_void_p)]),
        "sv_plan_info": (S, [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]),
        "sv_plan_export": (S, [c_void_p, c_size_t, POINTER(c_int32), POINTER(c_int32), POINTER(c_double),
                               POINTER(c_int32)]),
        "sv_plan_pass_info": (S, [c_void_p, c_size_t, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                  POINTER(c_int32)]),
        "sv_plan_destroy": (S, [c_void_p]),
        "sv_plan_pass_flops": (S, [c_void_p, c_size_t, POINTER(c_double)]),
        "sv_plan_flops": (S, [c_void_p, POINTER(c_double), c_size_t]),
        "sv_plan_pass_ops": (S, [c_void_p, c_size_t, POINTER(c_int32), POINTER(c_int32)]),
        "sv_apply_plan": (S, [c_void_p, c_void_p]),
        "sv_apply_circuit": (S, [c_void_p, POINTER(SvGate), c_size_t, POINTER(SvOpts)]),
        "sv_permute_qubits": (S, [c_void_p, POINTER(c_int32)]),
        "sv_measure_probs": (S, [c_void_p, POINTER(c_int32), c_int, c_void_p]),
        "sv_measure_probs_noalloc": (S, [c_void_p, POINTER(c_int32), c_int, c_void_p]),
        "sv_scale": (S, [c_void_p, c_double]),
        "sv_sync": (S, [c_void_p]),
        "sv_last_error": (c_char_p, []),
        "sv_version": (c_char_p, []),
        "sv_util_copy": (S, [c_void_p, c_void_p, c_size_t, c_void_p]),
        "sv_gate_kernel": (S, [c_int, c_int, POINTER(SvGate), c_char_p, c_size_t]),
        "sv_program_bytes": (S, [c_void_p, POINTER(c_size_t)]),
        "sv_program_create": (S, [c_void_p, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
        "sv_program_info": (S, [c_void_p, POINTER(c_int32), POINTER(c_int), POINTER(c_int32)]),
        "sv_program_destroy": (S, [c_void_p]),
        "sv_batcher_create": (S, [c_void_p, POINTER(c_void_p)]),
        "sv_batcher_run": (S, [c_void_p, c_int, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_int32)]),
        "sv_batcher_probs": (S, [c_void_p, c_void_p, POINTER(c_int32), c_int, c_void_p]),
        "sv_batcher_destroy": (S, [c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols() -> List[str]:
    """Function names declared in include/*.h."""
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def check(status: int) -> None:
    if status != SV_OK:
        raise SvError(status, load_library().sv_last_error().decode())


# ------------------------------------------------------------------ gates
def _kind_code(kind) -> int:
    return KIND[kind] if isinstance(kind, str) else int(kind)


def make_gates(gates: Sequence) -> tuple:
    """Marshal gate objects (attributes kind, qubits, theta, matrix) into a
    ctypes array; returns (array, keepalive)."""
    arr = (SvGate * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        sg = arr[i]
        sg.kind = _kind_code(g.kind)
        qs = tuple(g.qubits)
        sg.nq = len(qs)
        for j in range(MAXQ):
            sg.q[j] = qs[j] if j < len(qs) else -1
        sg.theta = float(getattr(g, "theta", 0.0) or 0.0)
        mat = getattr(g, "matrix", None)
        if mat is not None and sg.kind == KIND["MATRIX"]:
            m = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128)).view(np.float64)
            keep.append(m)
            sg.m = m.ctypes.data_as(POINTER(c_double))
        else:
            sg.m = None
    return arr, keep


def make_opts(opts: Optional[dict]) -> SvOpts:
    o = SvOpts()
    check(load_library().sv_default_opts(byref(o)))
    for k, v in (opts or {}).items():
        if k == "mode" and isinstance(v, str):
            v = MODE[v]
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, int(v))
    return o


# ------------------------------------------------------------------ plans
class Plan:
    """A fused and grouped schedule (host only; sv_fuse)."""

    def __init__(self, n: int, dtype: str, gates: Sequence, opts: Optional[dict] = None):
        lib = load_library()
        arr, keep = make_gates(gates)
        o = make_opts(opts)
        h = c_void_p()
        check(lib.sv_fuse(n, _dt_code(dtype), arr, len(gates), byref(o), byref(h)))
        self._h = h
        self.n, self.dtype = n, dtype

    @classmethod
    def from_array(cls, n: int, dtype: str, marshalled: tuple, n_gates: int, opts: Optional[dict] = None) -> "Plan":
        """Plan from gates already marshalled by make_gates (array, keepalive)."""
        self = cls.__new__(cls)
        arr, _ = marshalled
        o = make_opts(opts)
        h = c_void_p()
        check(load_library().sv_fuse(n, _dt_code(dtype), arr, n_gates, byref(o), byref(h)))
        self._h = h
        self.n, self.dtype = n, dtype
        return self

    @property
    def handle(self):
        return self._h

    def program_bytes(self) -> int:
        """Device bytes of this plan's program (sv_program_bytes)."""
        nb = c_size_t()
        check(load_library().sv_program_bytes(self._h, byref(nb)))
        return nb.value

    def info(self):
        a, b = c_size_t(), c_size_t()
        check(load_library().sv_plan_info(self._h, byref(a), byref(b)))
        return a.value, b.value

    def export(self):
        """List of (qubits, matrix, pass) for every op in execution order."""
        lib = load_library()
        n_ops, _ = self.info()
        out = []
        buf = (c_double * (2 * 64 * 64))()
        for i in range(n_ops):
            nq, ps = c_int32(), c_int32()
            q = (c_int32 * MAXQ)()
            check(lib.sv_plan_export(self._h, i, byref(nq), q, buf, byref(ps)))
            d = 1 << nq.value
            m = np.frombuffer(buf, dtype=np.float64, count=2 * d * d).copy().view(np.complex128).reshape(d, d)
            out.append((tuple(q[j] for j in range(nq.value)), m, ps.value))
        return out

    def passes(self, stages: bool = False):
        """(kind, n_ops, n_local) per pass; with stages=True also n_stages."""
        lib = load_library()
        _, n_passes = self.info()
        out = []
        for i in range(n_passes):
            kind, nops, nloc, nst = c_int32(), c_int32(), c_int32(), c_int32()
            check(lib.sv_plan_pass_info(self._h, i, byref(kind), byref(nops), byref(nloc), byref(nst)))
            out.append((kind.value, nops.value, nloc.value, nst.value) if stages else
                       (kind.value, nops.value, nloc.value))
        return out

    def kernel_ops(self) -> List[Tuple[int, int]]:
        """(kernel ops, fixed-point phase ops among them: ladders and quadratic
        phases) per pass (sv_plan_pass_ops)."""
        lib = load_library()
        _, n_passes = self.info()
        out = []
        a, b = c_int32(), c_int32()
        for i in range(n_passes):
            check(lib.sv_plan_pass_ops(self._h, i, byref(a), byref(b)))
            out.append((a.value, b.value))
        return out

    def pass_flops(self) -> List[float]:
        """Algorithmic real flops per amplitude of every pass (sv_plan_flops,
        one call: the pass query sv_plan_pass_flops per pass gives the same)."""
        lib = load_library()
        _, n_passes = self.info()
        buf = (c_double * max(1, n_passes))()
        check(lib.sv_plan_flops(self._h, buf, n_passes))
        return list(buf[:n_passes])

    def close(self):
        if self._h:
            load_library().sv_plan_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dt_code(dtype) -> int:
    if dtype in ("c128", "complex128", SV_C128):
        return SV_C128
    if dtype in ("c64", "complex64", SV_C64):
        return SV_C64
    import torch
    if dtype == torch.complex128:
        return SV_C128
    if dtype == torch.complex64:
        return SV_C64
    raise ValueError(f"unsupported dtype {dtype}")


# ------------------------------------------------------------------ states
class StateVector:
    """A 2^n state in a torch CUDA tensor, driven through the C ABI."""

    def __init__(self, n: int, dtype="c128", tensor=None, stream=None, init: bool = True):
        import torch
        lib = load_library()
        code = _dt_code(dtype)
        tdt = torch.complex128 if code == SV_C128 else torch.complex64
        if tensor is None:
            tensor = torch.empty(1 << n, dtype=tdt, device="cuda")
        if tensor.dtype != tdt or tensor.numel() != (1 << n) or not tensor.is_cuda or not tensor.is_contiguous():
            raise ValueError("tensor must be a contiguous CUDA tensor of 2^n elements of the state dtype")
        self.tensor = tensor
        self.n = n
        self.dtype = "c128" if code == SV_C128 else "c64"
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        check(lib.sv_create(n, code, c_void_p(tensor.data_ptr()), c_void_p(self.stream.cuda_stream),
                            0 if init else SV_NO_INIT, byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def init_basis(self, index: int = 0):
        check(load_library().sv_init_basis(self._h, index))

    def apply_gate(self, gate):
        arr, keep = make_gates([gate])
        check(load_library().sv_apply_gate(self._h, arr))

    def apply_circuit(self, gates: Sequence, opts: Optional[dict] = None):
        arr, keep = make_gates(gates)
        o = make_opts(opts)
        check(load_library().sv_apply_circuit(self._h, arr, len(gates), byref(o)))

    def apply_plan(self, plan: Plan):
        check(load_library().sv_apply_plan(self._h, plan.handle))

    def permute_qubits(self, dest: Sequence[int]):
        d = (c_int32 * self.n)(*[int(x) for x in dest])
        check(load_library().sv_permute_qubits(self._h, d))

    def measure_probs(self, qubits: Optional[Sequence[int]] = None, out=None, noalloc: bool = False):
        """Marginal probabilities (sv_measure_probs; noalloc=True calls
        sv_measure_probs_noalloc, whose partials live in the library's static
        device array; `out` must then be given by a caller that cannot allocate)."""
        import torch
        qubits = list(range(self.n - 1, -1, -1)) if qubits is None else [int(q) for q in qubits]
        m = len(qubits)
        if out is None:
            out = torch.empty(1 << m, dtype=torch.float64, device=self.tensor.device)
        qa = (c_int32 * max(1, m))(*qubits)
        fn = load_library().sv_measure_probs_noalloc if noalloc else load_library().sv_measure_probs
        check(fn(self._h, qa, m, c_void_p(out.data_ptr())))
        return out

    def norm2(self) -> float:
        out = self.measure_probs([])
        self.sync()
        return float(out.item())

    def scale(self, factor: float):
        check(load_library().sv_scale(self._h, float(factor)))

    def sync(self):
        check(load_library().sv_sync(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load_library().sv_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
class Program:
    """A plan's program (all its passes) resident in device memory (sv_program_*).

    With buffer=None the program's bytes live in a uint8 torch tensor of the
    caching allocator (no hipMalloc once the allocator is warm); the tensor is
    kept alive by this object."""

    def __init__(self, plan: Plan, stream=None, buffer=None):
        import torch
        lib = load_library()
        nb = c_size_t()
        check(lib.sv_program_bytes(plan.handle, byref(nb)))
        self.nbytes = nb.value
        s = stream if stream is not None else torch.cuda.current_stream()
        if buffer is None:
            with torch.cuda.stream(s):  # the caching allocator ties the block to the upload stream
                buffer = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device="cuda")
        self.buffer = buffer
        h = c_void_p()
        check(lib.sv_program_create(plan.handle, c_void_p(buffer.data_ptr()), buffer.numel(),
                                    c_void_p(s.cuda_stream), byref(h)))
        self._h = h
        n, dt, npass = c_int32(), c_int(), c_int32()
        check(lib.sv_program_info(h, byref(n), byref(dt), byref(npass)))
        self.n, self.n_passes = n.value, npass.value
        self.dtype = "c128" if dt.value == SV_C128 else "c64"

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load_library().sv_program_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batcher:
    """One step runs one pass of many states (sv_batcher_*): their tile and
    permutation passes in one kernel launch, matrix, dense and sweep passes as
    launches of their own."""

    def __init__(self, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        check(load_library().sv_batcher_create(c_void_p(self.stream.cuda_stream), byref(h)))
        self._h = h

    def run(self, states: Sequence[StateVector], programs: Sequence[Program], pass_index: Sequence[int]):
        k = len(states)
        if len(programs) != k or len(pass_index) != k:
            raise ValueError("states, programs and pass_index differ in length")
        sa = (c_void_p * max(k, 1))(*[st.handle.value for st in states])
        pa = (c_void_p * max(k, 1))(*[pr.handle.value for pr in programs])
        ia = (c_int32 * max(k, 1))(*[int(i) for i in pass_index])
        check(load_library().sv_batcher_run(self._h, k, sa, pa, ia))

    def probs(self, state: StateVector, qubits: Sequence[int], out):
        qs = [int(q) for q in qubits]
        qa = (c_int32 * max(1, len(qs)))(*qs)
        check(load_library().sv_batcher_probs(self._h, state.handle, qa, len(qs), c_void_p(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "_h", None):
            load_library().sv_batcher_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def util_copy(dst, src, stream=None):
    import torch
    nbytes = src.numel() * src.element_size()
    s = stream if stream is not None else torch.cuda.current_stream()
    check(load_library().sv_util_copy(c_void_p(dst.data_ptr()), c_void_p(src.data_ptr()), nbytes,
                                      c_void_p(s.cuda_stream)))


def gate_kernel(n: int, dtype, gate) -> str:
    """Identifier of the kernel sv_apply_gate launches for `gate` (host only)."""
    arr, keep = make_gates([gate])
    buf = ctypes.create_string_buffer(128)
    check(load_library().sv_gate_kernel(n, _dt_code(dtype), arr, buf, 128))
    return buf.value.decode()


def version() -> str:
    return load_library().sv_version().decode()
