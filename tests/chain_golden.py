"""Comparison of a full-size GPU run with the oracle's whole-chain expected values.

The values come from tests/golden/make_chain_goldens.py, which runs the oracle
(complex128, eigendecomposition exponentials) over every interval of the job:
psi_n every M/20 intervals, tr U_n for every interval, and U_n v for a seeded
probe vector v every M/10 intervals.

Gates (the errors of Sec. 4.3, unnormalised):
  FP64 path:        1 - |<psi_ref|psi>|^2 <= 1e-12 for every stored psi_n and for
                    every probe U_n v; |tr U_n - tr U_n,ref| / d <= 1e-12;
  FP32 products:    the same state and probe errors <= 1e-6, with the direction
                    (normalised) error and the norm error | |psi| - 1 | each
                    <= 1e-6 too; the traces are reported, not gated.
"""
import os

import numpy as np
import torch

import oracle

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with np.load(os.path.join(GOLDEN_DIR, f"{name}_chain.npz"), allow_pickle=False) as g:
        return {k: g[k] for k in g.files}


def check(job, gold, fp64, say):
    """job: a bench.Job after step() (U_n in job.U, psi_M in job.psi)."""
    q, w = job.q, job.w
    tol = 1e-12 if fp64 else 1e-6
    U = job.U
    d = w.d
    # every interval's trace
    tr = torch.diagonal(U, dim1=1, dim2=2).to(torch.complex128).sum(dim=1).cpu().numpy()
    dtr = np.abs(tr - gold["trace_U"]).max() / d
    say(f"  max |tr U_n - tr U_n,ref| / d over all {w.M} intervals: {dtr:.3e}")
    if fp64:
        assert dtr <= tol
    # probe vectors: U_n v for sampled intervals
    v = torch.from_numpy(gold["probe"]).to(U.device)
    worst = 0.0
    for j, n in enumerate(gold["probe_at"]):
        x = v.clone()
        q.propagate(U[int(n):int(n) + 1].contiguous(), q.STATE, x)
        inf = abs(float(oracle.state_infidelity(gold["probe_U"][j], x.cpu().numpy())))
        worst = max(worst, inf)
    say(f"  probe U_n v, {len(gold['probe_at'])} intervals: worst state error {worst:.3e}")
    assert worst <= tol
    # the whole chain, and its stored intermediate states
    psi = job.psi.cpu().numpy()
    ref = gold["psi_at"][-1]
    inf = float(oracle.state_infidelity(ref, psi))
    dinf = float(oracle.direction_infidelity(ref, psi))
    nerr = oracle.norm_error(psi)
    say(f"  psi_M after {w.M} intervals: state error {inf:.3e} (direction {dinf:.3e}, |psi| - 1 {nerr:.3e})")
    assert abs(inf) <= tol and abs(dinf) <= tol and nerr <= tol
    traj = torch.empty((w.M + 1, d), dtype=torch.complex128, device=U.device)
    x = torch.from_numpy(w.psi0).to(U.device)
    q.propagate(U, q.STATE, x, traj=traj)
    t = traj[torch.from_numpy(gold["at"]).to(U.device)].cpu().numpy()
    errs = [abs(float(oracle.state_infidelity(a, b))) for a, b in zip(gold["psi_at"], t)]
    say(f"  psi_n at {len(errs)} points: worst state error {max(errs):.3e}")
    assert max(errs) <= tol
    return inf
