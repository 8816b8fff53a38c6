"""Helpers shared by the GPU parity tests (moving seeded inputs to the device and
results back; no simulator arithmetic)."""
import numpy as np

TOL = {"c128": 1e-12, "c64": 1e-5}


def torch_dtype(dtype):
    import torch
    return torch.complex128 if dtype == "c128" else torch.complex64


def to_device(psi: np.ndarray, dtype: str):
    """Copy a host state to the GPU in the given precision.  Returns the device
    tensor and the complex128 upcast of what the device holds (the oracle's
    input, so the initial rounding to complex64 is not counted as error)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(psi)).to(torch_dtype(dtype)).cuda()
    host = t.cpu().numpy().astype(np.complex128)
    return t, host


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128)


def max_err(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
