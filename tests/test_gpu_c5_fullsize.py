"""Four coupled transmons, d = 4096, K = 4, M = 2000, order 2: the three product
precisions (FP64, FP32 MFMA, split-BF16 MFMA; FP64 solve in all) at full size.

Sampled parity: one interval's propagator from each precision against the oracle
(an eigendecomposition of a 4096 x 4096 Hermitian matrix on the host, about half a
minute).  Chains: the state over the first intervals in FP32 and split-BF16
against the FP64 path's state (direction), and every chain's norm (property that
holds at any size).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests.test_gpu_parity import host, say

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")
DEV = "cuda:0"
SAMPLED = 1000          # the interval checked against the oracle
PREFIX = 16             # intervals of the compared chains
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def job():
    w = wl.coupled_transmons()
    assert np.array_equal(w.H0, w.H0.conj().T) and all(np.array_equal(h, h.conj().T) for h in w.Hk)
    H0, Hk = torch.from_numpy(w.H0).to(DEV), torch.from_numpy(w.Hk).to(DEV)
    u = torch.from_numpy(np.ascontiguousarray(w.u)).to(DEV)
    c1, c2 = q.magnus_coeffs(u, w.dt_sample, w.M, w.order)
    return w, H0, Hk, c1, c2


def _expm(w, H0, Hk, c1, c2, idx, prec):
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    ii = torch.tensor(idx, device=DEV)
    om, _ = q.magnus_generators(H0, Hk, c1[ii].contiguous(), c2[ii].contiguous(), w.dt_interval, w.order, dtype)
    U, s = q.expm_batched(om, U=om, skew_hermitian=True, bf16x3=(prec == "bf16x3"), unitary_refine=(prec != "c128"))
    return U, s


def test_c5_sampled_interval_all_precisions(job):
    w, H0, Hk, c1, c2 = job
    say(f"C5 d={w.d}: oracle propagator of interval {SAMPLED}")
    c1h, c2h = c1.cpu().numpy(), c2.cpu().numpy()
    Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1h[SAMPLED:SAMPLED + 1], c2h[SAMPLED:SAMPLED + 1],
                                       w.dt_interval, w.order)
    Uo = oracle.propagator_from_hamiltonian(Hb)[0]
    s_ref = oracle.scaling_exponent(-1j * Hb[0])
    for prec in ("c128", "c64", "bf16x3"):
        say(f"  {prec}")
        U, s = _expm(w, H0, Hk, c1, c2, [SAMPLED], prec)
        torch.cuda.synchronize()
        Ug = host(U[0]).astype(np.complex128)
        inf = abs(float(oracle.propagator_infidelity(Uo, Ug)))
        say(f"  {prec}: s = {int(s[0])}, infidelity {inf:.3e}, unitarity {oracle.unitarity_error(Ug):.3e}")
        if prec == "c128":
            assert int(s[0]) == s_ref
            assert inf <= 1e-12 and np.abs(Ug - Uo).max() <= 1e-10
        else:
            assert inf <= 1e-6 and oracle.unitarity_error(Ug) <= 1e-6
        del U


def test_c5_chain_prefix_all_precisions(job):
    w, H0, Hk, c1, c2 = job
    psi = {}
    smax = 0
    for prec in ("c128", "c64", "bf16x3"):
        say(f"C5 chain of {PREFIX} intervals, {prec}")
        U, s = _expm(w, H0, Hk, c1, c2, list(range(PREFIX)), prec)
        x = torch.from_numpy(w.psi0).to(DEV)
        q.propagate(U, q.STATE, x)
        torch.cuda.synchronize()
        psi[prec] = host(x)
        smax = max(smax, int(s.max()))
        del U
    # the same prefix by the Taylor action on the generators (no propagator formed)
    for prec, dtype in (("action_c128", torch.complex128), ("action_c64", torch.complex64)):
        say(f"C5 chain of {PREFIX} intervals, {prec}")
        ii = torch.arange(PREFIX, device=DEV)
        om, _ = q.magnus_generators(H0, Hk, c1[ii].contiguous(), c2[ii].contiguous(), w.dt_interval, w.order, dtype)
        x = torch.from_numpy(w.psi0).to(DEV)
        q.propagate_action(om, x, skew_hermitian=True)
        torch.cuda.synchronize()
        psi[prec] = host(x)
        del om
    ref = psi["c128"]
    assert oracle.norm_error(ref) <= PREFIX * 1e-13
    assert np.abs(psi["action_c128"] - ref).max() <= PREFIX * 1e-12
    inf = abs(float(oracle.state_infidelity(ref, psi["action_c64"])))
    say(f"  action on complex64 generators vs FP64 path: state infidelity {inf:.3e}")
    assert inf <= 1e-6 and oracle.norm_error(psi["action_c64"]) <= PREFIX * 4 * U32
    for prec in ("c64", "bf16x3"):
        inf = abs(float(oracle.state_infidelity(ref, psi[prec])))
        say(f"  {prec} vs FP64 path: state infidelity {inf:.3e}, norm - 1 = {np.linalg.norm(psi[prec]) - 1:.3e}")
        assert inf <= 1e-6
        assert oracle.norm_error(psi[prec]) <= 1e-6
