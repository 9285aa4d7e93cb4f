"""Continuous batching on the GPU: every job's result is the same alone and in the mix."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")
from paper_2411_09982_amd.serve import Request, Server, max_overlap, path_for, poisson_requests  # noqa: E402

CHUNK = 8


def _make(i, g):
    d = int(g.choice([8, 33, 64, 100]))
    K = int(g.integers(1, 3))
    M = int(g.choice([12, 30]))
    order = int(g.integers(1, 3))
    prec = "c64" if g.random() < 0.5 else "c128"
    w = wl.random_system(d, K, M * 5, M, order, config_id=700 + i, drift_scale=15.0, drive_scale=3.0)
    return Request(i, w.H0, w.Hk, w.u, w.dt_sample, M, order, prec, w.psi0)


def test_mix_equals_alone_and_oracle():
    reqs = poisson_requests(12, 300.0, 11, _make)
    srv = Server(budget_bytes=1, max_slots=3, chunk=CHUNK)
    sizes = sorted(srv.bytes_for(r) for r in reqs)
    srv.adm.budget = int(2.5 * sizes[len(sizes) // 2])      # some jobs must wait for memory
    srv.adm.budget = max(srv.adm.budget, sizes[-1])
    say(f"serving {len(reqs)} jobs, budget {srv.adm.budget} B, sizes {sizes[0]}..{sizes[-1]}")
    res = srv.run(reqs)
    assert sorted(res) == [r.rid for r in reqs]
    say(f"  max jobs in flight {max_overlap(res)}")
    dev = "cuda:0"
    paths = [path_for(r) for r in reqs]
    assert {"action", "propagators"} <= set(paths)                      # both paths served
    for r in reqs:
        dtype = torch.complex64 if r.precision == "c64" else torch.complex128
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        assert res[r.rid].path == path_for(r)
        if path_for(r) == "action":
            psi_alone = q.evolve_state(t(r.H0), t(r.Hk), t(r.u), r.dt_sample, r.M, r.order, t(r.psi0), dtype=dtype,
                                       chunk=CHUNK).cpu().numpy()
        else:
            alone = q.evolve(t(r.H0), t(r.Hk), t(r.u), r.dt_sample, r.M, r.order, psi0=t(r.psi0), dtype=dtype,
                             chunk=CHUNK)
            psi_alone = alone["psi"].cpu().numpy()
        assert np.array_equal(psi_alone, res[r.rid].psi), r.rid        # bit-identical
        ref = oracle.run(r.H0, r.Hk, r.u, r.dt_sample, r.M, r.order, psi0=r.psi0)
        inf = abs(oracle.state_infidelity(ref["psi"], res[r.rid].psi))
        assert inf <= (1e-12 if r.precision == "c128" else 1e-6), (r.rid, inf)
        # FP32 propagators are refined to unitarity; the action keeps FP64
        # arithmetic with the truncation of the whole chain below 2^-24: the norm
        # holds to the target on both paths
        nbound = r.M * 1e-13 if r.precision == "c128" else 1e-6
        assert oracle.norm_error(res[r.rid].psi) <= nbound, r.rid


def test_nonfinite_request_is_marked():
    # a request whose control holds a NaN comes back marked non-finite (its state
    # is NaN), on either path; the requests beside it are unaffected
    reqs = []
    for i, d in enumerate((20, 64, 20, 64)):
        w = wl.random_system(d, 1, 12 * 5, 12, 2, config_id=800 + i, drift_scale=15.0, drive_scale=3.0)
        u = w.u.copy()
        if i >= 2:
            u[0, 7] = float("nan")
        reqs.append(Request(i, w.H0, w.Hk, u, w.dt_sample, 12, 2, "c64", w.psi0))
    say("serving requests with a NaN control")
    res = Server(budget_bytes=1 << 34, max_slots=4, chunk=CHUNK).run(reqs)
    assert {path_for(r) for r in reqs} == {"action", "propagators"}
    for r in reqs:
        bad = r.rid >= 2
        assert res[r.rid].finite == (not bad), r.rid
        assert np.isnan(res[r.rid].psi).all() == bad
    assert q.sync_status() == q.OK        # the server took the flags


def test_large_requests_both_paths():
    # d >= 1024 on both paths in one mix (the propagators forced for two of them):
    # each result equals the job run alone, bit for bit, and the oracle's chain
    g = np.random.default_rng(1024)
    specs = [(1024, "c64", "propagators"), (1024, "c128", "propagators"), (1100, "c64", "action"),
             (1030, "c128", "action")]
    reqs = []
    for i, (d, prec, path) in enumerate(specs):
        w = wl.serving_request_system(d, 6, 2, g)
        reqs.append(Request(i, w.H0, w.Hk, w.u, w.dt_sample, w.M, 2, prec, w.psi0, arrival=0.01 * i, path=path))
    say("serving four requests of d >= 1024 on both paths")
    res = Server(budget_bytes=1 << 36, max_slots=4, chunk=CHUNK).run(reqs)
    dev = "cuda:0"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    for r in reqs:
        dtype = torch.complex64 if r.precision == "c64" else torch.complex128
        if r.path == "action":
            alone = q.evolve_state(t(r.H0), t(r.Hk), t(r.u), r.dt_sample, r.M, r.order, t(r.psi0), dtype=dtype,
                                   chunk=CHUNK).cpu().numpy()
        else:
            alone = q.evolve(t(r.H0), t(r.Hk), t(r.u), r.dt_sample, r.M, r.order, psi0=t(r.psi0), dtype=dtype,
                             chunk=CHUNK)["psi"].cpu().numpy()
        assert res[r.rid].path == r.path
        assert np.array_equal(alone, res[r.rid].psi), r.rid
        ref = oracle.run(r.H0, r.Hk, r.u, r.dt_sample, r.M, r.order, psi0=r.psi0)["psi"]
        inf = abs(oracle.state_infidelity(ref, res[r.rid].psi))
        say(f"  request {r.rid}: d={r.d} {r.precision} {r.path}: state error {inf:.2e}")
        assert inf <= (1e-12 if r.precision == "c128" else 1e-6), (r.rid, inf)
