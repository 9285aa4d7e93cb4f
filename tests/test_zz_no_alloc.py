"""qcheff_propagate_state_noalloc (the entry point that allocates nothing) against
qcheff_propagate in QCHEFF_STATE mode: the same kernels, so the same bits, on two
calls in a row (the second with a smaller input, which must not see the first
call's scratch) and with a trajectory."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")
DEV = "cuda:0"


def _call_noalloc(U, x, traj=None):
    L = q.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = q.C128 if U.dtype == torch.complex128 else q.C64
    r = L.qcheff_propagate_state_noalloc(ctypes.c_void_p(U.data_ptr()), U.shape[0], U.shape[-1], code,
                                         ctypes.c_void_p(x.data_ptr()),
                                         None if traj is None else ctypes.c_void_p(traj.data_ptr()), st)
    assert r == q.OK, L.qcheff_last_error().decode()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_noalloc_matches_propagate_twice(dtype):
    for M, d, seed in ((37, 300, 1), (5, 130, 2)):       # the second call is smaller
        Om = wl.random_skew_hermitian_batch(M, d, 3.0, config_id=1200 + seed)
        U = torch.from_numpy(oracle.expm_skew_hermitian(Om)).to(DEV).to(dtype)
        psi0 = torch.from_numpy(wl.random_state(d, 40 + seed)).to(DEV)
        ref = psi0.clone()
        q.propagate(U, q.STATE, ref)
        x = psi0.clone()
        _call_noalloc(U, x)
        tr_ref = torch.empty((M + 1, d), dtype=torch.complex128, device=DEV)
        q.propagate(U, q.STATE, psi0.clone(), traj=tr_ref)
        tr = torch.empty_like(tr_ref)
        y = psi0.clone()
        _call_noalloc(U, y, traj=tr)
        torch.cuda.synchronize()
        assert torch.equal(x, ref) and torch.equal(y, ref) and torch.equal(tr, tr_ref)
        # and against the oracle's chain of the same (rounded) propagators
        ref_o = oracle.propagate_state(U.cpu().numpy().astype(np.complex128), psi0.cpu().numpy())
        assert np.abs(x.cpu().numpy() - ref_o).max() <= 1e-13 * M * np.sqrt(d)


def test_noalloc_rejects_bad_sizes():
    U = torch.zeros((2, 4, 4), dtype=torch.complex64, device=DEV)
    x = torch.zeros(4, dtype=torch.complex128, device=DEV)
    L = q.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.qcheff_propagate_state_noalloc(ctypes.c_void_p(U.data_ptr()), 2, 20000, q.C64,
                                            ctypes.c_void_p(x.data_ptr()), None, st) == q.EINVAL
    assert L.qcheff_propagate_state_noalloc(ctypes.c_void_p(U.data_ptr()), 2, 4, q.C64, None, None, st) == q.EINVAL
