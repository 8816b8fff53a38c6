"""sv_measure_probs_noalloc (reduction partials in the library's static device
array, no allocation) against sv_measure_probs on the same states, through the
C ABI: two calls in a row, the second on a smaller input, in both dtypes and
for marginals that do and do not need reduction partials."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _probs(lib, st, qubits, out, noalloc):
    qa = (ctypes.c_int32 * max(1, len(qubits)))(*qubits)
    fn = lib.sv_measure_probs_noalloc if noalloc else lib.sv_measure_probs
    return fn(st.handle, qa, len(qubits), ctypes.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_probs_matches_allocating_entry(dtype):
    import torch

    import paper_2409_14697_amd as sv
    from paper_2409_14697_amd.binding import load_library
    from svgen import gaussian_state_np

    lib = load_library()
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    # first call: N=22 with a 12-qubit marginal (partials in the static array);
    # second call: a smaller state, N=14, 5-qubit marginal; then the norm
    cases = [(22, [21, 3, 17, 0, 9, 12, 5, 20, 1, 14, 8, 11]), (14, [2, 13, 7, 0, 4]), (14, [])]
    for n, qubits in cases:
        print(f"noalloc probs: dtype={dtype} n={n} m={len(qubits)}", flush=True)
        psi = torch.from_numpy(gaussian_state_np(n, 40 + n)).to(tdt).cuda()
        st = sv.StateVector(n, dtype, tensor=psi, init=False)
        m = len(qubits)
        ref = torch.full((1 << m,), -1.0, dtype=torch.float64, device="cuda")
        got = torch.full((1 << m,), -2.0, dtype=torch.float64, device="cuda")
        assert _probs(lib, st, qubits, ref, noalloc=False) == 0
        assert _probs(lib, st, qubits, got, noalloc=True) == 0
        st.sync()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        # same reduction geometry and order: bitwise equal
        assert np.array_equal(r, g), float(np.max(np.abs(r - g)))
        assert abs(float(g.sum()) - 1.0) < (1e-12 if dtype == "c128" else 1e-5)
        st.close()


def test_noalloc_probs_rejects_bad_arguments():
    import torch

    import paper_2409_14697_amd as sv
    from paper_2409_14697_amd.binding import load_library

    lib = load_library()
    st = sv.StateVector(8, "c128")
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    assert _probs(lib, st, [3, 3], out, noalloc=True) == -2   # SV_ERR_QUBIT: repeated
    assert _probs(lib, st, [8], out, noalloc=True) == -2      # out of range
    qa = (ctypes.c_int32 * 1)(0)
    assert lib.sv_measure_probs_noalloc(st.handle, qa, 1, None) == -1  # null output
    st.close()
