"""Batched sweep of uneven dimensions: grouped results equal the one-job path and the oracle."""
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
        s_max = int(one["s"].max().cpu())
        tol = 1e-12 if dtype == torch.complex128 else max(1e-6, j.M * 2.0 ** s_max * 2.0 ** -24)
        assert inf <= tol, (i, j.d, inf)
