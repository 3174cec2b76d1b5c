"""The allocation-free renormalisation against qsim_renormalize: two calls in a row on one device (the
second on a smaller state), both dtypes, through the C ABI on raw device buffers."""
import ctypes

import numpy as np
import pytest

import qsim_workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0608239_amd as q
    q.lib()
    return q


def _raw_state(psi, dtype):
    import torch
    cd = np.complex128 if dtype == "c128" else np.complex64
    a = np.ascontiguousarray(np.asarray(psi, dtype=cd)).view(np.float64 if dtype == "c128" else np.float32)
    return torch.from_numpy(a.copy()).to("cuda:0")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_renormalize_noalloc_matches_renormalize(q, dtype):
    import torch
    from paper_quant_ph_0608239_amd import _lib
    L = q.lib()
    code = q.dtype_code(dtype)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cd = np.complex128 if dtype == "c128" else np.complex64
    for call, (n, scale) in enumerate([(21, 3.7), (13, 0.25)]):  # the second call on a smaller state
        psi = (wl.gaussian_state(n, 500 + n) * scale).astype(cd)
        # the existing entry point on a library state
        s = q.State(n, dtype)
        s.upload(psi)
        nb_ref = s.renormalize()
        ref = s.download()
        s.close()
        # the allocation-free one on a raw device buffer
        t = _raw_state(psi, dtype)
        nb = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
        rc = L.qsim_renormalize_noalloc(ctypes.c_void_p(t.data_ptr()), n, code, stream, ctypes.c_void_p(nb.data_ptr()))
        assert rc == _lib.OK, L.qsim_last_error()
        torch.cuda.synchronize()
        got = t.cpu().numpy().view(cd)
        print(f"noalloc {dtype} call {call}: n={n} norm before {nb.item()!r} (reference {nb_ref!r})", flush=True)
        assert nb.item() == nb_ref
        assert np.array_equal(got, ref)  # same kernels, same grid: the same bits
        assert abs(np.sum(np.abs(got.astype(np.complex128)) ** 2) - 1.0) < (1e-12 if dtype == "c128" else 1e-5)


def test_renormalize_noalloc_zero_state_and_errors(q):
    import torch
    from paper_quant_ph_0608239_amd import _lib
    L = q.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    t = torch.zeros(2 ** 11, dtype=torch.float64, device="cuda:0")
    nb = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    assert L.qsim_renormalize_noalloc(ctypes.c_void_p(t.data_ptr()), 10, 1, stream, ctypes.c_void_p(nb.data_ptr())) == _lib.OK
    torch.cuda.synchronize()
    assert nb.item() == 0.0 and int(torch.count_nonzero(t)) == 0
    # rejected before anything is launched
    assert L.qsim_renormalize_noalloc(None, 10, 1, stream, None) == _lib.EINVAL
    assert L.qsim_renormalize_noalloc(ctypes.c_void_p(t.data_ptr() + 8), 9, 1, stream, None) == _lib.EINVAL
    assert L.qsim_renormalize_noalloc(ctypes.c_void_p(t.data_ptr()), 0, 1, stream, None) == _lib.EINVAL
    assert L.qsim_renormalize_noalloc(ctypes.c_void_p(t.data_ptr()), 10, 5, stream, None) == _lib.EINVAL
