"""Full-size parity on the d = 1024 spin chain (10 spins, K = 2, 10^4 samples,
M = 200, second order; the degenerate periodic chain of Sec. 4.3) in the launch
configuration bench.py times for it (`--workload spin_chain_10_d1024`).

d = 1024 fills whole 128 x 128 tiles; the oracle checks every coefficient,
sampled intervals of the propagators, a prefix of the state chain and the norm
of the whole chain, for the FP64, FP32 and split-BF16 products.
"""
import numpy as np
import pytest
import torch

import bench
import oracle
import workloads as wl
from tests.test_gpu_parity import inf_tol, say

pytestmark = pytest.mark.gpu

SAMPLED = [0, 1, 97, 199]
PREFIX = 5
FINAL = {}


@pytest.fixture(scope="module")
def job_and_ref():
    w = wl.spin_chain()
    assert (w.d, w.K, w.M, w.order) == (1024, 2, 200, 2)
    c1o, c2o = oracle.interval_coefficients(w.u, w.dt_sample, w.M, w.order)
    rows = SAMPLED + list(range(PREFIX))
    Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1o[rows], c2o[rows], w.dt_interval, w.order)
    Uo = oracle.propagator_from_hamiltonian(Hb)
    return w, c1o, c2o, Hb, Uo


@pytest.mark.parametrize("dt_name", ["c128", "c64", "bf16x3"])
def test_spin_chain_d1024_full_size(job_and_ref, dt_name):
    w, c1o, c2o, Hb, Uo = job_and_ref
    say(f"spin chain d={w.d} M={w.M} {dt_name}")
    job = bench.Job(w, dt_name, bench.DEFAULT_CHUNK[dt_name])
    job.step()
    torch.cuda.synchronize()
    assert np.abs(job.c1.cpu().numpy() - c1o).max() <= 1e-14 * np.abs(c1o).max()
    assert np.abs(job.c2.cpu().numpy() - c2o).max() <= 1e-13 * np.abs(c2o).max()
    s = job.s.cpu().numpy()
    U = job.omega
    for j, n in enumerate(SAMPLED):
        Ug = U[n].cpu().numpy().astype(np.complex128)
        inf = abs(oracle.propagator_infidelity(Uo[j], Ug))
        unit = np.abs(Ug.conj().T @ Ug - np.eye(w.d)).max()
        say(f"  interval {n}: s={s[n]} infidelity {inf:.3e} max-abs {np.abs(Ug - Uo[j]).max():.3e} "
            f"|U^H U - I| {unit:.2e}")
        assert inf <= inf_tol(job.dtype, s[n])
        assert s[n] == oracle.scaling_exponent(-1j * Hb[j], shift=(dt_name == "c128"))
        if dt_name == "c128":
            assert np.abs(Ug - Uo[j]).max() <= 1e-10
            assert unit <= 1e-12
        else:
            assert unit <= w.d * 2.0 ** s[n] * 2.0 ** -24
    psi = torch.from_numpy(w.psi0).to("cuda:0")
    job.q.propagate(U[:PREFIX].contiguous(), job.q.STATE, psi)
    psi_o = oracle.propagate_state(Uo[len(SAMPLED):], w.psi0)
    sinf = abs(float(oracle.state_infidelity(psi_o, psi.cpu().numpy())))
    say(f"  {PREFIX}-interval chain state infidelity {sinf:.3e}")
    assert sinf <= (1e-12 if dt_name == "c128" else 1e-6)
    norm = float(torch.linalg.vector_norm(job.psi).cpu())
    bound = w.M * 1e-13 if dt_name == "c128" else w.M * 2.0 ** int(s.max()) * 2.0 ** -24
    say(f"  |psi_M| - 1 = {norm - 1:.3e} (bound {bound:.1e})")
    assert abs(norm - 1) <= bound
    FINAL[dt_name] = job.psi.cpu().numpy()


@pytest.mark.parametrize("dt_name", ["c64", "bf16x3"])
def test_spin_chain_d1024_whole_chain_vs_fp64(dt_name):
    # the whole 200-interval chain of an FP32-product path against the FP64 path's
    if not {"c128", dt_name} <= set(FINAL):
        pytest.skip("needs the full-size runs of this module")
    inf = abs(float(oracle.state_infidelity(FINAL["c128"], FINAL[dt_name])))
    say(f"  200-interval chain, {dt_name} vs FP64 path: state infidelity {inf:.3e}")
    assert inf <= 1e-6
