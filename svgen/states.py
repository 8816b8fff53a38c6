"""Seeded initial states (inputs only).

Gaussian state: real and imaginary parts i.i.d. N(0, 1) in FP64, divided by
the FP64 2-norm so that the normalisation condition of Sec. II-A holds.
"""
from __future__ import annotations

import numpy as np


def gaussian_state_np(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    dim = 1 << n
    psi = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    return (psi / np.sqrt(np.vdot(psi, psi).real)).astype(np.complex128)


def basis_state_np(n: int, index: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def gaussian_state_torch(n: int, seed: int, dtype, device="cuda"):
    """Large states for the device benchmarks, generated where they live.

    The draw uses torch's seeded generator on the device; the normalisation is
    done in FP64.  Tests that need the same values on the host copy them back
    (sampled) rather than regenerating them."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    t = torch.empty(1 << n, dtype=dtype, device=device)
    torch.view_as_real(t).normal_(generator=g)
    # FP64 norm over the real view, chunked so no FP64 copy of a 16 GiB state is made
    rv = torch.view_as_real(t).reshape(-1)
    acc = torch.zeros((), dtype=torch.float64, device=device)
    step = 1 << 26
    for s in range(0, rv.numel(), step):
        acc += rv[s:s + step].double().pow(2).sum()
    t.mul_((1.0 / acc.sqrt()).to(t.real.dtype))
    return t
