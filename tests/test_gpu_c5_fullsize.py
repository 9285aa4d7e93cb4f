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


FULL = {}   # final states of the full-length runs of this module


def test_c5_full_length_action(job):
    # all 2000 intervals by the Taylor action on complex128 and complex64
    # generators (FP64 arithmetic; the truncation of the complex64 chain is held
    # below 2^-24 in all)
    w, H0, Hk, c1, c2 = job
    u = torch.from_numpy(np.ascontiguousarray(w.u)).to(DEV)
    for name, dtype in (("action_c128", torch.complex128), ("action_c64", torch.complex64)):
        say(f"C5 full length ({w.M} intervals), {name}")
        x = q.evolve_state(H0, Hk, u, w.dt_sample, w.M, w.order, torch.from_numpy(w.psi0).to(DEV), dtype=dtype)
        torch.cuda.synchronize()
        FULL[name] = host(x)
        say(f"  |psi_M| - 1 = {np.linalg.norm(FULL[name]) - 1:.3e}")
    assert oracle.norm_error(FULL["action_c128"]) <= 1e-12
    inf = abs(float(oracle.state_infidelity(FULL["action_c128"], FULL["action_c64"])))
    say(f"  action c64 vs c128 over {w.M} intervals: state error {inf:.3e}")
    assert inf <= 1e-6 and oracle.norm_error(FULL["action_c64"]) <= 1e-6


def test_c5_full_length_propagators_c64(job):
    # all 2000 intervals through the propagator path (FP32 products, FP64 solve,
    # refinement to unitarity, complex128 propagators), 32 intervals at a time,
    # against the FP64 action of the same job; det U_n = exp(tr Omega_n) on samples
    w, H0, Hk, c1, c2 = job
    if "action_c128" not in FULL:
        pytest.skip("needs the full-length action run of this module")
    u = torch.from_numpy(np.ascontiguousarray(w.u)).to(DEV)
    say(f"C5 full length ({w.M} intervals), propagators c64")
    x, s = q.evolve_streamed(H0, Hk, u, w.dt_sample, w.M, w.order, torch.from_numpy(w.psi0).to(DEV),
                             dtype=torch.complex64, chunk=32)
    torch.cuda.synchronize()
    psi = host(x)
    inf = abs(float(oracle.state_infidelity(FULL["action_c128"], psi)))
    say(f"  vs FP64 action: state error {inf:.3e}, |psi| - 1 = {np.linalg.norm(psi) - 1:.3e}, "
        f"s in [{int(s.min())}, {int(s.max())}]")
    assert inf <= 1e-6 and oracle.norm_error(psi) <= 1e-6
    for n in (0, 999, 1999):
        ii = torch.tensor([n], device=DEV)
        om, _ = q.magnus_generators(H0, Hk, c1[ii].contiguous(), c2[ii].contiguous(), w.dt_interval, w.order,
                                    torch.complex64)
        U, _ = q.expm_batched(om, skew_hermitian=True, unitary_refine=True, out_c128=True)
        sign, logabs = torch.linalg.slogdet(U[0])
        tr = complex(torch.diagonal(om[0]).to(torch.complex128).sum().cpu())
        ph = float(torch.angle(sign).cpu())
        dph = (ph - tr.imag + np.pi) % (2 * np.pi) - np.pi
        say(f"  interval {n}: log|det U| = {float(logabs):.2e}, arg det U - Im tr Omega = {dph:.2e}")
        # log|det| sums the d radial errors the refinement leaves (about 1e-11 each);
        # the phase sums the d eigenvalue phase errors of the FP32 products: held to
        # 1e-6 per eigenvalue on average
        assert abs(float(logabs)) <= 1e-6 and abs(dph) <= w.d * 1e-6
        del om, U
