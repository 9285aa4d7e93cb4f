"""Full-size parity: the transmon x resonator job (d = 1000, K = 2, 1e5 samples,
M = 1000, second order) in the launch configuration bench.py times for it
(`--workload transmon10x_resonator100_d1000`).

Checked for the FP64 and FP32 products (FP32 refined to unitarity after its
squarings): every coefficient, sampled generators and propagators against the
oracle (computed here), and the whole 1000-interval chain against the oracle's
stored chain (tests/golden/, see tests/chain_golden.py).
"""
import numpy as np
import pytest
import torch

import bench
import oracle
import workloads as wl
from tests import chain_golden
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu

SAMPLED = [0, 1, 517, 999]


@pytest.fixture(scope="module")
def job_and_ref():
    w = wl.transmon_resonator()
    c1o, c2o = oracle.interval_coefficients(w.u, w.dt_sample, w.M, w.order)
    Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1o[SAMPLED], c2o[SAMPLED], w.dt_interval, w.order)
    Uo = oracle.propagator_from_hamiltonian(Hb)
    return w, c1o, c2o, Hb, Uo, chain_golden.load("transmon10x_resonator100_d1000")


@pytest.mark.parametrize("dt_name", ["c64", "c128"])
def test_transmon_resonator_d1000_full_size(job_and_ref, dt_name):
    w, c1o, c2o, Hb, Uo, gold = job_and_ref
    say(f"full size d={w.d} M={w.M} {dt_name}")
    job = bench.Job(w, dt_name, bench.DEFAULT_CHUNK[dt_name])
    job.step()
    torch.cuda.synchronize()
    fp64 = dt_name == "c128"
    # coefficients, all of them
    assert np.abs(job.c1.cpu().numpy() - c1o).max() <= 1e-15 * np.abs(c1o).max() * 10
    assert np.abs(job.c2.cpu().numpy() - c2o).max() <= 1e-13 * np.abs(c2o).max()
    # propagators of sampled intervals
    s = job.s.cpu().numpy()
    U = job.U
    for j, n in enumerate(SAMPLED):
        Ug = U[n].cpu().numpy().astype(np.complex128)
        inf = abs(oracle.propagator_infidelity(Uo[j], Ug))
        unit = oracle.unitarity_error(Ug)
        say(f"  interval {n}: s={s[n]} infidelity {inf:.3e} max-abs {np.abs(Ug - Uo[j]).max():.3e} "
            f"|U^H U - I| {unit:.2e}")
        assert inf <= (1e-12 if fp64 else 1e-6) and unit <= (1e-12 if fp64 else 1e-6)
        if fp64:
            assert np.abs(Ug - Uo[j]).max() <= 1e-10
        # the FP64 path applies the trace reduction, the FP32 path does not
        assert s[n] == oracle.scaling_exponent(-1j * Hb[j], shift=fp64)
    # generators of the sampled intervals, formed again into a scratch buffer
    idx = torch.tensor(SAMPLED, device="cuda:0")
    om, _ = job.q.magnus_generators(job.H0, job.Hk, job.c1[idx].contiguous(), job.c2[idx].contiguous(),
                                    w.dt_interval, w.order, job.dtype)
    ref = -1j * Hb
    err = np.abs(om.cpu().numpy().astype(np.complex128) - ref).max()
    tol = (1e-13 if fp64 else 1.2e-7) * np.abs(ref).max()
    assert err <= tol, (err, tol)
    chain_golden.check(job, gold, fp64, say)
