"""Batched sweep of uneven dimensions: results equal the one-job path and the oracle,
with the exponentials of all groups in one qcheff_expm_grouped call (the default)
or per group, eagerly and from captured graphs."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")
from paper_2411_09982_amd.sweep import Sweep  # noqa: E402


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_sweep_matches_single_jobs_and_oracle(dtype):
    jobs = wl.sweep_instances(14, M=12, config_id=31, dims=(16, 32, 64))
    say(f"sweep of {len(jobs)} jobs, d = {sorted({j.d for j in jobs})}, {dtype}")
    sw = Sweep(jobs, dtype, chunk=16)
    sw.run()
    got = sw.states()
    dev = "cuda:0"
    for i, j in enumerate(jobs):
        one = q.evolve(torch.from_numpy(j.H0).to(dev), torch.from_numpy(j.Hk).to(dev), torch.from_numpy(j.u).to(dev),
                       j.dt_sample, j.M, j.order, psi0=torch.from_numpy(j.psi0).to(dev), dtype=dtype, chunk=16)
        assert np.abs(one["psi"].cpu().numpy() - got[i]).max() <= 1e-13, i
        ref = oracle.run(j.H0, j.Hk, j.u, j.dt_sample, j.M, j.order, psi0=j.psi0)
        inf = abs(oracle.state_infidelity(ref["psi"], got[i]))
        assert inf <= (1e-12 if dtype == torch.complex128 else 1e-6), (i, j.d, inf)
        # complex64 propagators are refined to unitarity: the norm holds to the target
        nbound = j.M * 1e-13 if dtype == torch.complex128 else 1e-6
        assert oracle.norm_error(got[i]) <= nbound, (i, j.d)


def _states_equal(a, b):
    return all(np.array_equal(a[i], b[i]) for i in a)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_sweep_grouped_matches_per_group_and_oracle(dtype):
    # several groups above the fused small-d limit share every product launch;
    # against each group run alone (the same bits, whatever tile its products
    # take) and against the oracle's chain of every job
    jobs = wl.sweep_instances(9, M=10, config_id=37, dims=(64, 128, 256))
    say(f"grouped sweep of {len(jobs)} jobs, d = {sorted({j.d for j in jobs})}, {dtype}")
    sw = Sweep(jobs, dtype, chunk=8)
    sw.run()
    got = sw.states()
    alone = Sweep(jobs, dtype, chunk=8, grouped=False)
    alone.run()
    ref_alone = alone.states()
    for i, j in enumerate(jobs):
        assert np.array_equal(ref_alone[i], got[i]), i   # the same bits (tile shapes accumulate alike)
        ref = oracle.run(j.H0, j.Hk, j.u, j.dt_sample, j.M, j.order, psi0=j.psi0)
        inf = abs(oracle.state_infidelity(ref["psi"], got[i]))
        assert inf <= (1e-12 if dtype == torch.complex128 else 1e-6), (i, j.d, inf)


@pytest.mark.parametrize("grouped", [True, False])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_sweep_graph_replays_match_eager(dtype, grouped):
    # groups below and above the fused small-d limit; every replay is checked,
    # with eager work and synchronizations between the replays
    jobs = wl.sweep_instances(10, M=8, config_id=41, dims=(16, 64, 128))
    say(f"sweep graph, {len(jobs)} jobs, {dtype}, grouped={grouped}")
    sw = Sweep(jobs, dtype, chunk=8, grouped=grouped)
    sw.run()
    eager = sw.states()
    sw.capture()
    other = torch.from_numpy(wl.random_skew_hermitian_batch(3, 40, 30.0, config_id=5)).to("cuda:0").to(dtype)
    for r in range(3):
        sw.run()
        assert _states_equal(eager, sw.states()), r
        q.expm_batched(other, skew_hermitian=True)     # unrelated eager work between replays
        torch.cuda.synchronize()
    assert sw.replays == 3 * (1 if grouped else len(sw.groups)) and sw.recaptures == 0


@pytest.mark.parametrize("grouped", [True, False])
def test_sweep_graph_recaptures_when_norms_grow(grouped):
    # new controls with larger amplitude (same operators) push the scaling
    # exponent above the captured bound: the sweep runs eagerly and is captured
    # again, and the result equals a fresh eager sweep of the new controls
    dtype = torch.complex64
    jobs = wl.sweep_instances(4, M=8, config_id=43, dims=(64,))
    say(f"sweep graph recapture, grouped={grouped}")
    sw = Sweep(jobs, dtype, chunk=8, grouped=grouped)
    sw.capture()
    bound = (lambda: sw.bound) if grouped else (lambda: sw.groups[0]["bound"])
    b0 = bound()
    # x1024 raises the largest exponent of these jobs from 9 to 11 (oracle)
    for k in range(len(jobs)):
        sw.groups[0]["ops"][k][2].mul_(1024.0)
    for j in jobs:
        j.u = j.u * 1024.0
    sw.run()
    assert sw.recaptures == 1 and bound() > b0
    fresh = Sweep(jobs, dtype, chunk=8, grouped=grouped)
    fresh.run()
    assert _states_equal(fresh.states(), sw.states())
    sw.run()                                           # the new graph holds
    assert sw.recaptures == 1 and _states_equal(fresh.states(), sw.states())
