"""Full-size parity on the d = 1024 spin chain (10 spins, K = 2, 10^4 samples,
M = 200, second order; the degenerate periodic chain of Sec. 4.3) in the launch
configuration bench.py times for it (its default workload).

d = 1024 fills whole 128 x 128 tiles.  Checked for the FP64, FP32 and split-BF16
products: every coefficient against the oracle, sampled propagators against the
oracle's eigendecomposition (computed here), and the whole 200-interval chain
against the oracle's stored chain (tests/golden/, see tests/chain_golden.py):
the final state, 21 intermediate states, U_n v on 11 intervals and every tr U_n.
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

SAMPLED = [0, 1, 97, 199]
FINAL = {}


@pytest.fixture(scope="module")
def job_and_ref():
    w = wl.spin_chain()
    assert (w.d, w.K, w.M, w.order) == (1024, 2, 200, 2)
    c1o, c2o = oracle.interval_coefficients(w.u, w.dt_sample, w.M, w.order)
    Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1o[SAMPLED], c2o[SAMPLED], w.dt_interval, w.order)
    Uo = oracle.propagator_from_hamiltonian(Hb)
    return w, c1o, c2o, Hb, Uo, chain_golden.load("spin_chain_10_d1024")


@pytest.mark.parametrize("dt_name", ["c128", "c64", "bf16x3"])
def test_spin_chain_d1024_full_size(job_and_ref, dt_name):
    w, c1o, c2o, Hb, Uo, gold = job_and_ref
    say(f"spin chain d={w.d} M={w.M} {dt_name}")
    job = bench.Job(w, dt_name, bench.DEFAULT_CHUNK[dt_name])
    job.step()
    torch.cuda.synchronize()
    assert np.abs(job.c1.cpu().numpy() - c1o).max() <= 1e-14 * np.abs(c1o).max()
    assert np.abs(job.c2.cpu().numpy() - c2o).max() <= 1e-13 * np.abs(c2o).max()
    s = job.s.cpu().numpy()
    U = job.U
    fp64 = dt_name == "c128"
    for j, n in enumerate(SAMPLED):
        Ug = U[n].cpu().numpy().astype(np.complex128)
        inf = abs(oracle.propagator_infidelity(Uo[j], Ug))
        unit = oracle.unitarity_error(Ug)
        say(f"  interval {n}: s={s[n]} infidelity {inf:.3e} max-abs {np.abs(Ug - Uo[j]).max():.3e} "
            f"|U^H U - I| {unit:.2e}")
        assert s[n] == oracle.scaling_exponent(-1j * Hb[j], shift=fp64)
        assert inf <= (1e-12 if fp64 else 1e-6) and unit <= (1e-12 if fp64 else 1e-6)
        if fp64:
            assert np.abs(Ug - Uo[j]).max() <= 1e-10
    FINAL[dt_name] = chain_golden.check(job, gold, fp64, say)
