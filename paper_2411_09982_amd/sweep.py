"""Batched parameter sweeps: many propagation jobs of uneven dimension at once.

Jobs are grouped by Hilbert-space dimension.  Within a group every job's
coefficients and generators are written into one contiguous [jobs * M][d][d]
buffer, and all of the group's state chains advance in one launch
(qcheff_propagate_batched).  The exponentials of all groups run in one call of
qcheff_expm_grouped (``grouped=True``, the default): in each round every
product stage is one launch over all groups' tiles (d <= 32 groups
take the fused one-workgroup kernel).  With ``grouped=False`` each group calls
qcheff_expm_batched on its own.  Every step is a call of the C ABI.

``capture()`` records the whole sweep (grouped) or each group's sequence (per
group) into HIP graphs (via torch.cuda.CUDAGraph), after one eager pass has
tuned the GEMM tiles and shown the largest scaling exponent.  The graphs take
the exponentials with a squaring bound (that exponent plus a margin), so
nothing in them waits on the host; ``run()`` then replays them, and a replay
that reports an exponent above its bound (new controls with larger norms) is
redone eagerly and captured again.
"""
from __future__ import annotations

import collections
import time

import numpy as np


class Sweep:
    """Device buffers for a list of Workload-like jobs (H0, Hk, u, dt_sample, M, order, psi0).

    H0 and every H_k must be exactly Hermitian (closed systems): the
    exponentials are taken with the skew-Hermitian structure of the generators.
    """

    def __init__(self, jobs, dtype, chunk: int = 256, device: str = "cuda:0", grouped: bool = True):
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
            # complex64 propagators are refined to unitarity and kept in complex128
            g["U"] = (torch.empty((len(idx) * M, d, d), dtype=torch.complex128, device=device)
                      if dtype == torch.complex64 else g["omega"])
            g["psi0"] = torch.from_numpy(np.stack([jobs[i].psi0 for i in idx])).to(device)
            g["psi"] = torch.empty_like(g["psi0"])
            gw = q.workspace_bytes(q.FN_GENERATORS, 1, d, Kmax, 2, q.C128)
            g["gen_ws"] = torch.empty(max(gw, 1), dtype=torch.uint8, device=device)
            nb = min(chunk, len(idx) * M)
            g["exp_ws"] = None if grouped else torch.empty(q.workspace_bytes(q.FN_EXPM, nb, d, 1, 1, code),
                                                           dtype=torch.uint8, device=device)
            g["s"] = torch.empty(len(idx) * M, dtype=torch.int32, device=device)
            g["graph"] = None
            g["bound"] = None
            self.groups.append(g)
        # complex64 propagators are refined to unitarity after their FP32 squarings
        # (and kept in complex128)
        self.refine = dtype == torch.complex64
        self.margin = 1
        self.replays = 0
        self.recaptures = 0
        self.grouped = grouped
        # one workspace for the grouped exponential: a chunk of each group per round
        self.exp_ws = torch.empty(max(1, q.expm_grouped_ws_bytes(
            [(g["d"], len(g["idx"]) * g["M"]) for g in self.groups], code, chunk)), dtype=torch.uint8,
            device=device) if grouped else None
        self.graph = None
        self.bound = None

    def _generators(self, g) -> None:
        q = self.q
        M = g["M"]
        for k, i in enumerate(g["idx"]):
            j = self.jobs[i]
            H0, Hk, u = g["ops"][k]
            q.magnus_coeffs(u, j.dt_sample, M, j.order, c1=g["c1"][k], c2=g["c2"][k])
            q.magnus_generators(H0, Hk, g["c1"][k], g["c2"][k], j.dt_interval, j.order, self.dtype,
                                omega=g["omega"][k * M:(k + 1) * M], ws=g["gen_ws"])

    def _chains(self, g) -> None:
        M, d = g["M"], g["d"]
        g["psi"].copy_(g["psi0"])
        self.q.propagate_batched(g["U"].view(len(g["idx"]), M, d, d), g["psi"])

    def _enqueue(self, g, bound=None) -> None:
        """One group's whole sequence on the current stream (per-group mode)."""
        self._generators(g)
        self.q.expm_batched(g["omega"], U=g["U"], s_out=g["s"], ws=g["exp_ws"], skew_hermitian=True,
                            squaring_bound=bound, unitary_refine=self.refine, out_c128=self.refine)
        self._chains(g)

    def _enqueue_all(self, bound=None) -> None:
        """The whole sweep on the current stream (grouped mode): every group's
        generators, one grouped exponential, every group's chains."""
        for g in self.groups:
            self._generators(g)
        self.q.expm_grouped([g["omega"] for g in self.groups], Us=[g["U"] for g in self.groups],
                            s_outs=[g["s"] for g in self.groups], ws=self.exp_ws, skew_hermitian=True,
                            squaring_bound=bound, unitary_refine=self.refine, out_c128=self.refine)
        for g in self.groups:
            self._chains(g)

    def _capture_all(self) -> None:
        torch = self.torch
        self.bound = max(int(g["s"].cpu().numpy().max()) for g in self.groups) + self.margin
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()   # default priority
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                self._enqueue_all(self.bound)
        torch.cuda.current_stream().wait_stream(side)
        self.graph = graph

    def _capture(self, g) -> None:
        torch = self.torch
        g["bound"] = int(g["s"].cpu().numpy().max()) + self.margin
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()   # default priority
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                self._enqueue(g, g["bound"])
        torch.cuda.current_stream().wait_stream(side)
        g["graph"] = graph

    def capture(self) -> None:
        """One eager pass, then the graphs (see the module doc)."""
        torch = self.torch
        if self.grouped:
            self._enqueue_all()
            torch.cuda.synchronize()
            self._capture_all()
            torch.cuda.synchronize()
            return
        for g in self.groups:
            self._enqueue(g)
            torch.cuda.synchronize()
            self._capture(g)
        torch.cuda.synchronize()

    def run(self) -> dict:
        """One pass over every job (graph replays once captured); returns wall
        times (s) measured with host clocks: per group, or {"all": t} when grouped."""
        torch = self.torch
        if self.grouped:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if self.graph is None:
                self._enqueue_all()
            else:
                self.graph.replay()
                self.replays += 1
            torch.cuda.synchronize()
            if self.graph is not None and any((g["s"].cpu().numpy() == -2).any() for g in self.groups if g["d"] > 32):
                # an exponent above the bound: redo eagerly, capture with the new maximum
                self._enqueue_all()
                torch.cuda.synchronize()
                self._capture_all()
                self.recaptures += 1
            return {"all": time.perf_counter() - t0}
        times = {}
        for g in self.groups:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if g["graph"] is None:
                self._enqueue(g)
            else:
                g["graph"].replay()
                self.replays += 1
            torch.cuda.synchronize()
            times[g["d"]] = time.perf_counter() - t0
            if g["graph"] is not None and g["d"] > 32 and (g["s"].cpu().numpy() == -2).any():
                # an exponent above the bound: redo eagerly, capture with the new maximum
                self._enqueue(g)
                torch.cuda.synchronize()
                self._capture(g)
                self.recaptures += 1
                times[g["d"]] = time.perf_counter() - t0
        return times

    def states(self) -> dict:
        """Final state of every job, by job index."""
        out = {}
        for g in self.groups:
            psi = g["psi"].cpu().numpy()
            for k, i in enumerate(g["idx"]):
                out[i] = psi[k]
        return out
