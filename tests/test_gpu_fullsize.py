"""Full-size parity: the transmon x resonator job (d = 1000, K = 2, 1e5 samples,
M = 1000, second order) in the launch configuration bench.py times.

The oracle cannot afford all 1000 eigendecompositions inside a test, so it
checks every coefficient, sampled intervals of the generators and propagators,
a prefix of the state chain, and properties of the whole chain.
"""
import numpy as np
import pytest
import torch

import bench
import oracle
import workloads as wl
from tests.test_gpu_parity import inf_tol, say

pytestmark = pytest.mark.gpu

SAMPLED = [0, 1, 517, 999]
PREFIX = 6
FINAL = {}      # psi_M of each precision's run, for the comparison of the whole chains


@pytest.fixture(scope="module")
def job_and_ref():
    w = wl.transmon_resonator()
    c1o, c2o = oracle.interval_coefficients(w.u, w.dt_sample, w.M, w.order)
    Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1o[SAMPLED + list(range(PREFIX))],
                                       c2o[SAMPLED + list(range(PREFIX))], w.dt_interval, w.order)
    Uo = oracle.propagator_from_hamiltonian(Hb)
    return w, c1o, c2o, Hb, Uo


@pytest.mark.parametrize("dt_name", ["c64", "c128"])
def test_transmon_resonator_d1000_full_size(job_and_ref, dt_name):
    w, c1o, c2o, Hb, Uo = job_and_ref
    say(f"full size d={w.d} M={w.M} {dt_name}")
    job = bench.Job(w, dt_name, bench.DEFAULT_CHUNK[dt_name])
    job.step()
    torch.cuda.synchronize()
    # coefficients, all of them
    assert np.abs(job.c1.cpu().numpy() - c1o).max() <= 1e-15 * np.abs(c1o).max() * 10
    assert np.abs(job.c2.cpu().numpy() - c2o).max() <= 1e-13 * np.abs(c2o).max()
    # propagators of sampled intervals
    s = job.s.cpu().numpy()
    U = job.omega
    for j, n in enumerate(SAMPLED):
        Ug = U[n].cpu().numpy().astype(np.complex128)
        inf = abs(oracle.propagator_infidelity(Uo[j], Ug))
        say(f"  interval {n}: s={s[n]} infidelity {inf:.3e} max-abs {np.abs(Ug - Uo[j]).max():.3e}")
        assert inf <= inf_tol(job.dtype, s[n])
        if dt_name == "c128":
            assert np.abs(Ug - Uo[j]).max() <= 1e-10
        # the FP64 path applies the trace reduction, the FP32 path does not
        assert s[n] == oracle.scaling_exponent(-1j * Hb[j], shift=(dt_name == "c128"))
    # generators of the sampled intervals, formed again into a scratch buffer
    idx = torch.tensor(SAMPLED, device="cuda:0")
    om, _ = job.q.magnus_generators(job.H0, job.Hk, job.c1[idx].contiguous(), job.c2[idx].contiguous(),
                                    w.dt_interval, w.order, job.dtype)
    ref = -1j * Hb[: len(SAMPLED)]
    err = np.abs(om.cpu().numpy().astype(np.complex128) - ref).max()
    tol = (1e-13 if dt_name == "c128" else 1.2e-7) * np.abs(ref).max()
    assert err <= tol, (err, tol)
    # state chain: prefix against the oracle, the whole chain by its norm
    psi = torch.from_numpy(w.psi0).to("cuda:0")
    job.q.propagate(U[:PREFIX].contiguous(), job.q.STATE, psi)
    psi_o = oracle.propagate_state(Uo[len(SAMPLED):], w.psi0)
    sinf = oracle.state_infidelity(psi_o, psi.cpu().numpy())
    say(f"  {PREFIX}-interval chain state infidelity {sinf:.3e}")
    assert abs(sinf) <= (1e-12 if dt_name == "c128" else 1e-6)
    # The U_n of this job are nearly equal (the drift dominates every interval), so
    # their rounding errors repeat and the norm error of the chain grows linearly
    # in M: at most M * 2^s * u per interval for FP32, M * 1e-13 for FP64.
    norm = float(torch.linalg.vector_norm(job.psi).cpu())
    smax = int(s.max())
    bound = w.M * 1e-13 if dt_name == "c128" else w.M * 2.0 ** smax * 2.0 ** -24
    say(f"  |psi_M| - 1 = {norm - 1:.3e} (bound {bound:.1e})")
    assert abs(norm - 1) <= bound
    FINAL[dt_name] = job.psi.cpu().numpy()


def test_transmon_resonator_d1000_whole_chain_fp32_vs_fp64():
    # The whole 1000-interval chain of the FP32 path against the FP64 path's, whose
    # sampled propagators and prefix match the oracle to 1e-12: the state's
    # direction must hold the FP32 target over the whole job.
    if set(FINAL) != {"c64", "c128"}:
        pytest.skip("needs both full-size runs of this module")
    inf = abs(float(oracle.state_infidelity(FINAL["c128"], FINAL["c64"])))
    say(f"  1000-interval chain, FP32 vs FP64 path: state infidelity {inf:.3e}")
    assert inf <= 1e-6
