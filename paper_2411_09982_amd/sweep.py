"""Batched parameter sweeps: many propagation jobs of uneven dimension at once.

Jobs are grouped by Hilbert-space dimension.  Within a group every job's
coefficients and generators are written into one contiguous [jobs * M][d][d]
buffer, all of the group's interval exponentials run as one batched call
(d <= 32: one fused workgroup per matrix; larger d: the MFMA GEMM path in
chunks), and all of the group's state chains advance in one launch
(qcheff_propagate_batched).  Every step is a call of the C ABI.
"""
from __future__ import annotations

import collections
import time

import numpy as np


class Sweep:
    """Device buffers for a list of Workload-like jobs (H0, Hk, u, dt_sample, M, order, psi0)."""

    def __init__(self, jobs, dtype, chunk: int = 256, device: str = "cuda:0"):
        import torch
        import paper_2411_09982_amd as q
        self.q, self.torch = q, torch
        self.dtype = dtype
        code = q.C64 if dtype == torch.complex64 else q.C128
        by_d = collections.defaultdict(list)
        for i, j in enumerate(jobs):
            by_d[j.d].append(i)
        self.jobs = jobs
        self.groups = []
        for d in sorted(by_d):
            idx = by_d[d]
            Ms = {jobs[i].M for i in idx}
            if len(Ms) != 1:
                raise ValueError("jobs of one dimension must share M")
            M = Ms.pop()
            Kmax = max(jobs[i].K for i in idx)
            g = dict(d=d, M=M, idx=idx)
            g["ops"] = [(torch.from_numpy(jobs[i].H0).to(device), torch.from_numpy(jobs[i].Hk).to(device),
                         torch.from_numpy(np.ascontiguousarray(jobs[i].u)).to(device)) for i in idx]
            g["c1"] = [torch.empty((M, jobs[i].K), dtype=torch.float64, device=device) for i in idx]
            g["c2"] = [torch.empty((M, jobs[i].K * (jobs[i].K + 1) // 2), dtype=torch.float64, device=device)
                       if jobs[i].order == 2 else None for i in idx]
            g["omega"] = torch.empty((len(idx) * M, d, d), dtype=dtype, device=device)
            g["psi0"] = torch.from_numpy(np.stack([jobs[i].psi0 for i in idx])).to(device)
            g["psi"] = torch.empty_like(g["psi0"])
            gw = q.workspace_bytes(q.FN_GENERATORS, 1, d, Kmax, 2, q.C128)
            g["gen_ws"] = torch.empty(max(gw, 1), dtype=torch.uint8, device=device)
            nb = min(chunk, len(idx) * M)
            g["exp_ws"] = torch.empty(q.workspace_bytes(q.FN_EXPM, nb, d, 1, 1, code), dtype=torch.uint8,
                                      device=device)
            self.groups.append(g)

    def run(self) -> dict:
        """One pass over every job; returns per-group wall times (s) measured with host clocks."""
        q, torch = self.q, self.torch
        times = {}
        for g in self.groups:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M, d = g["M"], g["d"]
            for k, i in enumerate(g["idx"]):
                j = self.jobs[i]
                H0, Hk, u = g["ops"][k]
                q.magnus_coeffs(u, j.dt_sample, M, j.order, c1=g["c1"][k], c2=g["c2"][k])
                q.magnus_generators(H0, Hk, g["c1"][k], g["c2"][k], j.dt_interval, j.order, self.dtype,
                                    omega=g["omega"][k * M:(k + 1) * M], ws=g["gen_ws"])
            q.expm_batched(g["omega"], U=g["omega"], ws=g["exp_ws"])
            g["psi"].copy_(g["psi0"])
            q.propagate_batched(g["omega"].view(len(g["idx"]), M, d, d), g["psi"])
            torch.cuda.synchronize()
            times[d] = time.perf_counter() - t0
        return times

    def states(self) -> dict:
        """Final state of every job, by job index."""
        out = {}
        for g in self.groups:
            psi = g["psi"].cpu().numpy()
            for k, i in enumerate(g["idx"]):
                out[i] = psi[k]
        return out
