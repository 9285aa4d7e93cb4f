"""FP32 products on the BF16 matrix cores (QCHEFF_C64_BF16X3) against the oracle.

Every FP32 operand is split exactly into three BF16 parts and a real product
keeps six of the nine part products; the three dropped ones are below 2^-26 of
|x||y|, under FP32's own rounding, and the part products are exact in the FP32
accumulator.  So the FP32 tolerances hold unchanged.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests.test_gpu_parity import gpu, host, inf_tol, say

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")


@pytest.mark.parametrize("mode", ["general", "skew", "refined"])
@pytest.mark.parametrize("d", [33, 64, 100, 128, 129, 257])
def test_expm_bf16x3_parity(d, mode):
    say(f"expm bf16x3 d={d} {mode}")
    skew, refine = mode != "general", mode == "refined"
    norms = [0.0, 0.01, 1.0, 5.3, 5.4, 11.0, 20.0, 170.0, 1500.0]
    Om = wl.random_skew_hermitian_batch(len(norms), d, norms, config_id=700 + d)
    ref = oracle.expm_skew_hermitian(Om)
    seen = Om.astype(np.complex64).astype(np.complex128)
    s_ref = [oracle.scaling_exponent(x, shift=False) for x in seen]   # FP32 path: no trace reduction
    om = gpu(Om).to(torch.complex64)
    U, s = q.expm_batched(om, skew_hermitian=skew, bf16x3=True, unitary_refine=refine)
    U32, _ = q.expm_batched(om, skew_hermitian=skew, unitary_refine=refine)
    torch.cuda.synchronize()
    assert host(s).tolist() == s_ref
    Ug = host(U).astype(np.complex128)
    inf = np.abs(oracle.propagator_infidelity(ref, Ug))
    say(f"  max infidelity {inf.max():.2e}, unitarity {oracle.unitarity_error(Ug):.2e}")
    assert np.all(inf <= inf_tol(torch.complex64, np.array(s_ref), refined=refine)), inf
    assert oracle.unitarity_error(Ug) <= (1e-6 if refine else 1e-3)
    # next to the FP32-MFMA products of the same inputs
    inf32 = np.abs(oracle.propagator_infidelity(host(U32).astype(np.complex128), Ug))
    assert np.all(inf32 <= 2 * inf_tol(torch.complex64, np.array(s_ref), refined=refine)), inf32


def test_expm_bf16x3_large_and_ragged():
    d = 1030
    say(f"expm bf16x3 d={d}")
    norms = [3.0, 60.0, 900.0]
    Om = wl.random_skew_hermitian_batch(len(norms), d, norms, config_id=731)
    ref = oracle.expm_skew_hermitian(Om)
    for refine in (False, True):
        U, s = q.expm_batched(gpu(Om).to(torch.complex64), skew_hermitian=True, bf16x3=True, unitary_refine=refine)
        torch.cuda.synchronize()
        inf = np.abs(oracle.propagator_infidelity(ref, host(U).astype(np.complex128)))
        assert np.all(inf <= inf_tol(torch.complex64, host(s), refined=refine)), inf


def test_expm_bf16x3_chunks_alias_nonfinite():
    d, B = 45, 7
    Om = wl.random_skew_hermitian_batch(B, d, np.linspace(0.5, 300, B), config_id=78)
    om = gpu(Om).to(torch.complex64)
    U1, s1 = q.expm_batched(om, bf16x3=True)
    U2, s2 = q.expm_batched(om, chunk=3, bf16x3=True)
    om3 = om.clone()
    U3, s3 = q.expm_batched(om3, U=om3, chunk=2, bf16x3=True)
    bad = om.clone()
    bad[2, 3, 4] = float("nan")
    U4, s4 = q.expm_batched(bad, bf16x3=True)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2) and torch.equal(U1, U3) and torch.equal(s1, s2)
    assert int(s4[2]) == -1 and torch.isnan(U4[2]).all()
    assert q.sync_status() == q.ENONFINITE and q.sync_status() == q.OK   # reported once, then cleared
    keep = [0, 1, 3, 4, 5, 6]
    assert torch.equal(U4[keep], U1[keep])


def test_evolve_bf16x3_end_to_end():
    w = wl.random_system(48, 3, 40 * 15, 40, 2, config_id=88, drift_scale=30.0, drive_scale=5.0)
    say("evolve bf16x3, random system d=48 order 2")
    ref = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, 2, psi0=w.psi0)
    dev = "cuda:0"
    out = q.evolve(torch.from_numpy(w.H0).to(dev), torch.from_numpy(w.Hk).to(dev), torch.from_numpy(w.u).to(dev),
                   w.dt_sample, w.M, 2, psi0=torch.from_numpy(w.psi0).to(dev), dtype=torch.complex64, chunk=16,
                   bf16x3=True)
    torch.cuda.synchronize()
    U = host(out["U"]).astype(np.complex128)     # refined to unitarity (the default of evolve)
    assert np.all(np.abs(oracle.propagator_infidelity(ref["U"], U)) <= 1e-6)
    assert abs(oracle.state_infidelity(ref["psi"], host(out["psi"]))) <= 1e-6
    assert oracle.norm_error(host(out["psi"])) <= 1e-6
