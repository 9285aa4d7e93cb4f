"""Throughput of the Magnus time-evolution path on one MI355X.

One step = one pass of the whole path over one job, inputs resident in HBM:
  per-interval coefficients -> commutator basis + generators Omega_n ->
  U_n = exp(Omega_n) for all M intervals (Pade scaling and squaring, in chunks) ->
  state chain psi_M = U_M ... U_1 psi_0 (each chunk's chain overlaps the next
  chunk's exponentials on a second stream).
Metric: interval propagators per second (M / step time).

Prints ONE JSON line.  Default workload: the 10-spin chain of Sec. 4.3, d = 1024,
two global controls, 1e4 samples, M = 200 intervals, second order, complex64
products on MFMA with FP64 norm / scaling / Pade solve and an FP64-Gram unitary
refinement of every propagator.  The transmon x resonator job (d = 1000,
M = 1000) runs as a second figure in `extra` (--workload picks the headline job).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--dtype c64|c128|bf16x3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense matrix peaks: FP32, FP64, and BF16 for the split-BF16 products
MFMA_PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6, "bf16x3": 2500.0}
# BF16 MFMA flops executed per algorithmic flop of a split-BF16 product: each real
# product is six BF16 part products
BF16X3_PARTS = 6
GEMM_SOURCE = os.path.join(ROOT, "paper_2411_09982_amd", "csrc", "cgemm.hpp")
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"cgemm_f32_traffic_{workload}.md")


def measured_traffic(workload):
    """HBM bytes per launch of the FP32 GEMM kernel on `workload` from the committed
    rocprofv3 --pmc summary, or None when there is none or the kernel source has
    changed since it was measured."""
    import hashlib
    try:
        text = open(traffic_file(workload)).read()
    except OSError:
        return None
    sha = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("kernel_source_sha256:",
                                                                                         "hbm_bytes_per_launch:")))
    if fields.get("kernel_source_sha256", "").strip() != sha:
        return None
    return float(fields["hbm_bytes_per_launch"])
HBM_PEAK_GBS = 8000.0
DEFAULT_CHUNK = {"c64": 256, "c128": 128, "bf16x3": 256}   # intervals per expm chunk


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spin_chain_10_d1024")
    ap.add_argument("--second-workload", default="transmon10x_resonator100_d1000",
                    help="a second job timed after the headline one and reported in extra ('' for none)")
    ap.add_argument("--no-refine", action="store_true",
                    help="FP32-product tiers without the unitary refinement of the propagators")
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128", "bf16x3"],
                    help="c64: FP32 MFMA products; bf16x3: the same complex64 path with the products on BF16 "
                         "MFMA (three-way split operands); c128: FP64 throughout")
    ap.add_argument("--lanes", type=int, default=1,
                    help="exponential pipelines (streams + host threads) that take the chunks in turn")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--no-fp64-compare", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-intervals", type=int, default=96, help="intervals in the CPU-oracle sample")
    ap.add_argument("--serve", action="store_true",
                    help="serving mode: Poisson request streams through the continuous-batching server; "
                         "prints one JSON line of latency percentiles per rate")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--line-serve-rate", type=float, default=20.0,
                    help="rate of the serving pass reported in the default line's extra (0: none)")
    ap.add_argument("--line-serve-requests", type=int, default=200)
    ap.add_argument("--serve-dmax", type=int, default=2048)
    ap.add_argument("--serve-mmax", type=int, default=1024)
    ap.add_argument("--sweep", action="store_true",
                    help="batched-sweep mode: 512 transmon-chain instances, d in {16..512}, M = 256, order 2; "
                         "prints one JSON line")
    ap.add_argument("--sweep-jobs", type=int, default=512)
    ap.add_argument("--sweep-mode", choices=("both", "grouped", "per-group"), default="both",
                    help="which exponential schedule the sweep mode times (both: per group, then grouped)")
    ap.add_argument("--action", action="store_true",
                    help="state-only mode: the first intervals of the d = 4096 job by the Taylor action vs the "
                         "propagator path; prints one JSON line")
    ap.add_argument("--action-intervals", type=int, default=64)
    ap.add_argument("--c5", action="store_true",
                    help="the d = 4096 job (four coupled transmons, M = 2000) at full length: the Taylor action on "
                         "complex64 and complex128 generators and the streamed propagator path in complex64, "
                         "split-BF16 and complex128; prints one JSON line")
    ap.add_argument("--c5-intervals", type=int, default=0, help="intervals to run (0: all M)")
    ap.add_argument("--npad", action="store_true",
                    help="numerical NPAD on the test matrix a^dag a + (a + a^dag): five consecutive rotations of "
                         "the five smallest couplings, one step of all N/2 disjoint pairs, the largest-coupling "
                         "search; prints one JSON line")
    ap.add_argument("--npad-n", type=int, default=16384)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, three times: under rocprofv3 --pmc its
    FETCH_SIZE and WRITE_SIZE per dispatch are the counters' reading for 1 GiB moved."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=src.numel() * 4, repeats=3)), flush=True)


def build_workload(name):
    import workloads as wl
    if name == "transmon10x_resonator100_d1000":
        return wl.transmon_resonator()
    if name == "spin_chain_10_d1024":
        return wl.spin_chain()
    if name == "transmon_duffing_d8":
        return wl.transmon_duffing()
    raise SystemExit(f"unknown workload {name}")


class Job:
    """Device-resident inputs and preallocated buffers for one workload."""

    def __init__(self, w, dtype_name, chunk, lanes=1, refine=True):
        import torch
        import paper_2411_09982_amd as q
        self.q, self.torch, self.w = q, torch, w
        # the FP32-product tiers refine each propagator to unitarity after its squarings
        self.refine = bool(refine) and dtype_name != "c128"
        dev = "cuda:0"
        self.dtype = torch.complex128 if dtype_name == "c128" else torch.complex64
        self.bf16x3 = dtype_name == "bf16x3"
        code = q.C128 if dtype_name == "c128" else q.C64
        d, K, M = w.d, w.K, w.M
        self.H0 = torch.from_numpy(w.H0).to(dev)
        self.Hk = torch.from_numpy(w.Hk).to(dev)
        self.u = torch.from_numpy(np.ascontiguousarray(w.u)).to(dev)
        self.psi0 = torch.from_numpy(w.psi0).to(dev)
        self.psi = torch.empty_like(self.psi0)
        self.c1 = torch.empty((M, K), dtype=torch.float64, device=dev)
        self.c2 = torch.empty((M, K + K * (K - 1) // 2), dtype=torch.float64, device=dev) if w.order == 2 else None
        self.omega = torch.empty((M, d, d), dtype=self.dtype, device=dev)
        # refined FP32-product propagators are kept in complex128 (no final rounding
        # to complex64); otherwise U overwrites the generators in place
        self.U = torch.empty((M, d, d), dtype=torch.complex128, device=dev) if self.refine else self.omega
        self.s = torch.empty(M, dtype=torch.int32, device=dev)
        gen_ws = q.workspace_bytes(q.FN_GENERATORS, 1, d, K, w.order, q.C128)
        self.gen_ws = torch.empty(max(gen_ws, 1), dtype=torch.uint8, device=dev) if gen_ws else None
        self.chunk = min(chunk, M)
        # `lanes` exponential pipelines, each with its own workspace, HIP stream and
        # host thread, take the chunks in turn, so that one chunk's latency-bound
        # LU kernels overlap another chunk's GEMMs
        self.lanes = max(1, int(lanes))
        ws_bytes = q.workspace_bytes(q.FN_EXPM, self.chunk, d, 1, 1, code)
        self.exp_ws = [torch.empty(ws_bytes, dtype=torch.uint8, device=dev) for _ in range(self.lanes)]
        self.lane_streams = [torch.cuda.Stream() for _ in range(self.lanes)] if self.lanes > 1 else None
        self.prop_ws = torch.empty(q.workspace_bytes(q.FN_PROPAGATE, M, d, 1, q.STATE, q.C128 if self.refine else code),
                                   dtype=torch.uint8, device=dev)
        self.side = torch.cuda.Stream()   # default priority
        if self.lanes > 1:
            import concurrent.futures
            self.pool = concurrent.futures.ThreadPoolExecutor(self.lanes)

    def step(self):
        """The whole path; the state chain of chunk c runs on a side stream while the
        exponentials of chunk c + 1 run on the main one."""
        q, w, torch = self.q, self.w, self.torch
        main = torch.cuda.current_stream()
        q.magnus_coeffs(self.u, w.dt_sample, w.M, w.order, c1=self.c1, c2=self.c2)
        q.magnus_generators(self.H0, self.Hk, self.c1, self.c2, w.dt_interval, w.order, self.dtype,
                            omega=self.omega, ws=self.gen_ws)
        self.psi.copy_(self.psi0)
        if self.lanes == 1:
            for c0 in range(0, w.M, self.chunk):
                c1 = min(w.M, c0 + self.chunk)
                U = self.U[c0:c1]
                q.expm_batched(self.omega[c0:c1], U=U, s_out=self.s[c0:c1], ws=self.exp_ws[0], skew_hermitian=True,
                               bf16x3=self.bf16x3, unitary_refine=self.refine, out_c128=self.refine)
                ev = torch.cuda.Event()
                ev.record(main)
                self.side.wait_event(ev)
                q.propagate(U, q.STATE, self.psi, ws=self.prop_ws, stream=self.side)
            main.wait_stream(self.side)
            return
        ready = torch.cuda.Event()
        ready.record(main)
        chunks = [(c0, min(w.M, c0 + self.chunk)) for c0 in range(0, w.M, self.chunk)]

        def run(idx):
            lane = idx % self.lanes
            st = self.lane_streams[lane]
            c0, c1 = chunks[idx]
            st.wait_event(ready)
            U = self.U[c0:c1]
            q.expm_batched(self.omega[c0:c1], U=U, s_out=self.s[c0:c1], ws=self.exp_ws[lane], skew_hermitian=True,
                           bf16x3=self.bf16x3, unitary_refine=self.refine, out_c128=self.refine, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
            return ev

        # lane l takes chunks l, l + lanes, ...; a lane's next chunk is enqueued
        # after its previous one (same stream), the chain follows chunk order
        futs = {}
        for idx in range(len(chunks)):
            prev = futs.get(idx - self.lanes)
            futs[idx] = self.pool.submit(lambda i=idx, p=prev: (p.result() if p else None, run(i))[1])
        for idx in range(len(chunks)):
            c0, c1 = chunks[idx]
            self.side.wait_event(futs[idx].result())
            q.propagate(self.U[c0:c1], q.STATE, self.psi, ws=self.prop_ws, stream=self.side)
        main.wait_stream(self.side)


def timed(job, steps, warmup, roofline=True):
    torch, q = job.torch, job.q
    for _ in range(warmup):
        job.step()
    torch.cuda.synchronize()
    if roofline:
        q.timing_enable(True)
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        job.step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern = {}
    if roofline:
        kern["f32"] = q.timing_read(q.KERNEL_GEMM_F32)
        kern["f64"] = q.timing_read(q.KERNEL_GEMM_F64)
        kern["bf16x3"] = q.timing_read(q.KERNEL_GEMM_BF16X3)
        q.timing_enable(False)
    return elapsed, times, kern


def flop_count(w, s_hist):
    """Algorithmic flops of one step: (8 (6 + s_n) + 32/3) d^3 per interval for the
    [13/13] Pade products, solve and squarings, plus 16 d^3 per commutator."""
    d = float(w.d)
    n_comm = (w.K + w.K * (w.K - 1) // 2) if w.order == 2 else 0
    return sum((8.0 * (6 + s) + 32.0 / 3.0) * d ** 3 for s in s_hist) + 16.0 * d ** 3 * n_comm


def cpu_baseline(w, n_int):
    """The oracle on the host cores over the first n_int intervals of the same job."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except ImportError:
        cores = os.cpu_count()
    s = w.N // w.M
    u = np.ascontiguousarray(w.u[:, : n_int * s])
    t0 = time.perf_counter()
    c1, c2 = oracle.interval_coefficients(u, w.dt_sample, n_int, w.order)
    Hbar = oracle.effective_hamiltonians(w.H0, w.Hk, c1, c2, w.dt_interval, w.order)
    U = oracle.propagator_from_hamiltonian(Hbar)
    psi = oracle.propagate_state(U, w.psi0)
    el = time.perf_counter() - t0
    return dict(value=n_int / el, unit="interval propagators/s", cores=int(cores), kind="oracle",
                sample=f"first {n_int} of {w.M} intervals of the same job (d={w.d}), coefficients + "
                       f"commutator basis + eigh propagators + state chain, {el:.1f} s"), U, psi


def serving_request(i, g, dmax, mmax):
    """One request of the serving stream: d ~ U{64..dmax}, M ~ U{64..mmax}, order 1 or 2,
    FP32 or FP64, each with probability 1/2; its operators and signals are built when
    the job starts (from a seed drawn here)."""
    import workloads as wl
    from paper_2411_09982_amd.serve import Request
    d = int(g.integers(64, dmax + 1))
    M = int(g.integers(64, mmax + 1))
    order = int(g.integers(1, 3))
    prec = "c64" if g.random() < 0.5 else "c128"
    seed = int(g.integers(0, 2 ** 31))
    spi, t_total = 64, 50.0      # samples per interval, pulse length (ns)

    def build():
        w = wl.serving_request_system(d, M, order, np.random.default_rng(seed), samples_per_interval=spi,
                                      t_total=t_total)
        return w.H0, w.Hk, w.u, w.psi0

    return Request(i, None, None, None, t_total / (spi * M), M, order, prec, None, build=build, dims=(d, 1))


def serve_pass(rate, n, seed, dmax, mmax):
    """One Poisson stream of n requests at `rate` through the continuous-batching
    server (HBM budget 200 GB, 8 jobs in flight); latency percentiles and rates."""
    import torch
    from paper_2411_09982_amd.serve import Server, latency_percentiles, max_overlap, poisson_requests
    reqs = poisson_requests(n, rate, seed, lambda i, g: serving_request(i, g, dmax, mmax))
    srv = Server(budget_bytes=200 << 30, max_slots=8, chunk=64)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    lat = latency_percentiles(res)
    paths = {}
    for r in res.values():
        paths[r.path] = paths.get(r.path, 0) + 1
    out = dict(rate_req_s=rate, requests=n, p50_ms=round(lat["p50_ms"], 1), p99_ms=round(lat["p99_ms"], 1),
               wait_p50_ms=round(lat["wait_p50_ms"], 1), wait_p99_ms=round(lat["wait_p99_ms"], 1),
               service_p50_ms=round(lat["service_p50_ms"], 1), service_p99_ms=round(lat["service_p99_ms"], 1),
               prep_p50_ms=round(lat["prep_p50_ms"], 1), prep_p99_ms=round(lat["prep_p99_ms"], 1),
               completed_req_s=round(n / wall, 2), intervals_s=round(sum(r.M for r in reqs) / wall, 1),
               wall_s=round(wall, 2), paths=paths, max_in_flight=max_overlap(res),
               nonfinite=sum(1 for r in res.values() if not r.finite), d_range=[64, dmax], M_range=[64, mmax])
    del srv, res
    torch.cuda.empty_cache()
    return out


def serve(a):
    """Latency under Poisson arrivals at each rate of --serve-rates, --serve-requests
    requests each (d ~ U{64..2048}, M ~ U{64..1024}, order 1 or 2, FP32 or FP64 per
    request); each request takes the path the server picks for it (propagators or
    the Taylor action on the state).  One JSON line per rate."""
    for rate in [float(x) for x in a.serve_rates.split(",")]:
        out = serve_pass(rate, a.serve_requests, 2411 + int(rate), a.serve_dmax, a.serve_mmax)
        print(json.dumps(dict(metric="serving latency (Magnus propagation requests)", data="synthetic", **out)),
              flush=True)


def sweep(a):
    """Interval propagators/s over a sweep of uneven-dimension jobs (grouped by d)."""
    import torch
    import workloads as wl
    from paper_2411_09982_amd.sweep import Sweep
    jobs = wl.sweep_instances(a.sweep_jobs)
    dtype = torch.complex64 if a.dtype == "c64" else torch.complex128
    n_int = sum(j.M for j in jobs)
    counts = {}
    for j in jobs:
        counts[j.d] = counts.get(j.d, 0) + 1

    def timed_runs(sw, mode):
        for _ in range(max(a.warmup, 0)):
            sw.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per = {}
        for _ in range(a.steps):
            for d, t in sw.run().items():
                per[d] = per.get(d, 0.0) + t
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / a.steps
        print(json.dumps(dict(metric="batched sweep: interval propagators/s", mode=mode, value=round(n_int / el, 1),
                              unit="interval propagators/s", ms_per_step=round(1000 * el, 1), steps=a.steps,
                              jobs=len(jobs), intervals=n_int, dtype=a.dtype, data="synthetic",
                              jobs_per_d={str(k): v for k, v in sorted(counts.items())},
                              ms_per_d={str(k): round(1000 * v / a.steps, 1) for k, v in sorted(per.items())})),
              flush=True)

    # each group's exponentials on their own, then every group's in one grouped
    # call per pass (one persistent launch per product stage, the groups' solves
    # side by side); eagerly and replayed from captured graphs.  The last line
    # (grouped, replayed) is the figure of this mode.
    modes = {"both": (False, True), "grouped": (True,), "per-group": (False,)}[a.sweep_mode]
    for grouped in modes:
        sw = Sweep(jobs, dtype, grouped=grouped)
        name = "grouped" if grouped else "per group"
        timed_runs(sw, f"eager, {name}")
        sw.capture()
        timed_runs(sw, f"hip graph, {name}")
        del sw
        torch.cuda.empty_cache()


def action(a):
    """State-only propagation at d = 4096 (four coupled transmons, K = 4, order 2): the
    first `--action-intervals` intervals by the Taylor action on the generators, against
    the propagator path (expm + chain) of the same intervals."""
    import torch
    import paper_2411_09982_amd as q
    import workloads as wl
    w = wl.coupled_transmons()
    P = a.action_intervals
    dev = "cuda:0"
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    H0, Hk, u, psi0 = t(w.H0), t(w.Hk), t(w.u), t(w.psi0)
    c1, c2 = q.magnus_coeffs(u, w.dt_sample, w.M, w.order)
    c1p, c2p = c1[:P].contiguous(), c2[:P].contiguous()
    out = {}
    for dt_name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        om, gws = q.magnus_generators(H0, Hk, c1p, c2p, w.dt_interval, w.order, dtype)
        ws = torch.empty(q.workspace_bytes(q.FN_ACTION, P, w.d, 1, 1, q.C64 if dt_name == "c64" else q.C128),
                         dtype=torch.uint8, device=dev)
        x = psi0.clone()
        q.propagate_action(om, x, ws=ws, skew_hermitian=True)   # warm-up

        def passes(n):
            for _ in range(n):
                x.copy_(psi0)
                q.magnus_generators(H0, Hk, c1p, c2p, w.dt_interval, w.order, dtype, omega=om, ws=gws,
                                    reuse_basis=True)
                q.propagate_action(om, x, ws=ws, skew_hermitian=True)
            torch.cuda.synchronize()

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        passes(a.steps)                               # the rate, without timing events
        el = (time.perf_counter() - t0) / a.steps
        q.timing_enable(True)                         # one more pass for the term kernel's events
        passes(1)
        k = q.timing_read(q.KERNEL_ACTION)
        q.timing_enable(False)
        out[f"action_{dt_name}"] = dict(intervals_per_s=round(P / el, 2), ms_per_interval=round(1000 * el / P, 3),
                                        products_per_interval=round(k["launches"] / P, 1),
                                        term_kernel_avg_us=round(1000 * k["ms"] / max(k["launches"], 1), 2),
                                        term_kernel_gbs=round(k["bytes"] / max(k["ms"], 1e-9) * 1e-6, 1))
        out[f"psi_action_{dt_name}"] = x.cpu().numpy()
        del om, ws
        torch.cuda.empty_cache()
    # the propagator path of the same intervals (FP32 products, FP64 solve)
    om, _ = q.magnus_generators(H0, Hk, c1p, c2p, w.dt_interval, w.order, torch.complex64)
    ews = torch.empty(q.workspace_bytes(q.FN_EXPM, min(P, 32), w.d, 1, 1, q.C64), dtype=torch.uint8, device=dev)
    pws = torch.empty(q.workspace_bytes(q.FN_PROPAGATE, P, w.d, 1, q.STATE, q.C64), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.magnus_generators(H0, Hk, c1p, c2p, w.dt_interval, w.order, torch.complex64, omega=om)
    q.expm_batched(om, U=om, ws=ews, skew_hermitian=True)
    x = psi0.clone()
    q.propagate(om, q.STATE, x, ws=pws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    psi_full = x.cpu().numpy()
    a64, a32 = out.pop("psi_action_c128"), out.pop("psi_action_c64")
    inf = lambda p, r: float(1 - abs(np.vdot(r, p)) ** 2 / (np.vdot(r, r).real * np.vdot(p, p).real))
    out["propagators_c64"] = dict(intervals_per_s=round(P / el, 2), ms_per_interval=round(1000 * el / P, 3))
    out["speedup_action_c64_vs_propagators"] = round(out["action_c64"]["intervals_per_s"] / (P / el), 2)
    out["state_infidelity_action_c64_vs_action_c128"] = inf(a32, a64)
    out["state_infidelity_propagators_c64_vs_action_c128"] = inf(psi_full, a64)
    print(json.dumps(dict(metric="state-only propagation (Taylor action): intervals/s",
                          config=dict(workload=w.name, d=w.d, K=w.K, M=w.M, order=w.order, intervals_timed=P),
                          data="synthetic", **out)), flush=True)


def c5(a):
    """All intervals of the d = 4096 job (four coupled transmons, K = 4, M = 2000, order 2)
    by each path and precision: intervals/s, the final state's norm error, and each
    state's error (Sec. 4.3, unnormalised, and its direction part) against the
    Taylor action on complex128 generators (FP64 throughout, the closest to exact
    here; the oracle cannot run 2000 eigendecompositions of d = 4096)."""
    import torch
    import paper_2411_09982_amd as q
    import workloads as wl
    w = wl.coupled_transmons()
    M = a.c5_intervals or w.M
    N = w.N // w.M * M
    dev = "cuda:0"
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    H0, Hk, u, psi0 = t(w.H0), t(w.Hk), t(w.u[:, :N]), t(w.psi0)
    last = [time.perf_counter()]

    def progress(n):   # a line every half minute from the streamed runs (each chunk's exponentials wait once)
        if time.perf_counter() - last[0] > 30.0:
            last[0] = time.perf_counter()
            print(f"#   {n} of {M} intervals", file=sys.stderr, flush=True)

    runs = {
        "action_c64": lambda: q.evolve_state(H0, Hk, u, w.dt_sample, M, w.order, psi0, dtype=torch.complex64),
        "action_c128": lambda: q.evolve_state(H0, Hk, u, w.dt_sample, M, w.order, psi0, dtype=torch.complex128),
        "propagators_c64": lambda: q.evolve_streamed(H0, Hk, u, w.dt_sample, M, w.order, psi0,
                                                     dtype=torch.complex64, chunk=32, progress=progress)[0],
        "propagators_bf16x3": lambda: q.evolve_streamed(H0, Hk, u, w.dt_sample, M, w.order, psi0,
                                                        dtype=torch.complex64, chunk=32, bf16x3=True,
                                                        progress=progress)[0],
        "propagators_c128": lambda: q.evolve_streamed(H0, Hk, u, w.dt_sample, M, w.order, psi0,
                                                      dtype=torch.complex128, chunk=16, progress=progress)[0],
    }
    # warm-up: the first chunk of each (tile tuning, code loading)
    uw = t(w.u[:, : w.N // w.M * 16])
    q.evolve_state(H0, Hk, uw, w.dt_sample, 16, w.order, psi0, dtype=torch.complex64)
    for dt, bf in ((torch.complex64, False), (torch.complex64, True), (torch.complex128, False)):
        q.evolve_streamed(H0, Hk, uw, w.dt_sample, 16, w.order, psi0, dtype=dt, chunk=16, bf16x3=bf)
    torch.cuda.synchronize()
    out, psi = {}, {}
    for name, fn in runs.items():
        t0 = time.perf_counter()
        x = fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        psi[name] = x.cpu().numpy()
        out[name] = dict(intervals_per_s=round(M / el, 2), seconds=round(el, 2),
                         norm_minus_1=float(np.linalg.norm(psi[name]) - 1.0))
        print(f"# {name}: {M / el:.1f} intervals/s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    ref = psi["action_c128"]
    for name in runs:
        if name != "action_c128":
            out[name].update({k + "_vs_action_c128": v for k, v in state_errors(ref, psi[name]).items()
                              if k != "norm_minus_1"})
    print(json.dumps(dict(metric="d = 4096 state propagation at full length: intervals/s",
                          config=dict(workload=w.name, d=w.d, K=w.K, M=M, order=w.order), data="synthetic",
                          **out)), flush=True)


def npad_bench(a):
    """Numerical NPAD (Sec. 3.2) on the benchmark matrix of App. B, a^dag a + (a + a^dag)
    truncated to N levels, stored dense in complex128: the time of one NPAD step of five
    consecutive rotations (the five smallest couplings, (0,1) ... (4,5)), of one step
    eliminating all N/2 disjoint pairs (2m, 2m+1) at once (HBM-bound: every entry is
    read and written once by the row pass and once by the column pass), and of the
    largest-coupling search (every entry read once)."""
    import torch
    import paper_2411_09982_amd as q
    N = a.npad_n
    dev = "cuda:0"
    H = torch.zeros((N, N), dtype=torch.complex128, device=dev)
    n = torch.arange(N, device=dev, dtype=torch.float64)
    H.diagonal().copy_(n.to(torch.complex128))
    off = torch.sqrt(n[1:]).to(torch.complex128)
    H.diagonal(1).copy_(off)
    H.diagonal(-1).copy_(off)
    H0 = H.clone()
    ws = torch.empty(q.workspace_bytes(q.FN_NPAD, N // 2, N, 1, 1, q.C128), dtype=torch.uint8, device=dev)
    five = [torch.tensor([[k, k + 1]], dtype=torch.int64, device=dev) for k in range(5)]
    allp = torch.stack([torch.arange(0, N, 2, device=dev), torch.arange(1, N, 2, device=dev)], dim=1).contiguous()
    ij = torch.empty((1, 2), dtype=torch.int64, device=dev)
    mag = torch.empty(1, dtype=torch.float64, device=dev)

    def timed_ms(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def step5():
        for p in five:
            q.npad_eliminate(H, p, ws=ws)

    t5 = timed_ms(step5, 50)
    H.copy_(H0)
    tall = timed_ms(lambda: q.npad_eliminate(H, allp, ws=ws), 10)
    tl = timed_ms(lambda: q.npad_largest(H, ij, mag, ws=ws), 20)
    byt_all = 4.0 * N * N * 16        # two passes, each reading and writing every entry
    byt_l = 1.0 * N * N * 16 / 2      # the upper triangle read once
    ok = q.sync_status() == q.OK
    print(json.dumps(dict(metric="numerical NPAD (Givens-rotation SWT), dense complex128", N=N, data="synthetic",
                          matrix="a^dag a + (a + a^dag)", step_of_5_rotations_ms=round(t5, 4),
                          all_pairs_step_ms=round(tall, 3), all_pairs_rotations_per_s=round(N / 2 / (tall * 1e-3)),
                          all_pairs_hbm_gbs=round(byt_all / (tall * 1e-3) / 1e9, 1),
                          largest_coupling_ms=round(tl, 3),
                          largest_coupling_hbm_gbs=round(byt_l / (tl * 1e-3) / 1e9, 1), status_ok=ok)), flush=True)


def golden_state(workload):
    """psi_M of the oracle's whole chain for `workload` (tests/golden/), or None."""
    path = os.path.join(GOLDEN_DIR, f"{workload}_chain.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as g:
        return g["psi_at"][-1]


def state_errors(ref, psi):
    """The final-state error of Sec. 4.3, 1 - |<ref|psi>|^2 (unnormalised), its
    direction part (norms divided out) and the norm error."""
    ov = abs(np.vdot(ref, psi)) ** 2
    return dict(state_error=float(1.0 - ov),
                direction_error=float(1.0 - ov / (np.vdot(ref, ref).real * np.vdot(psi, psi).real)),
                norm_minus_1=float(np.linalg.norm(psi) - 1.0))


def gemm_rates(kern, steps):
    return dict(
        fp32_gemm=dict(launches=kern["f32"]["launches"], ms_per_step=round(kern["f32"]["ms"] / steps, 2),
                       tflops=round(kern["f32"]["flops"] / max(kern["f32"]["ms"], 1e-9) * 1e-9, 2)),
        fp64_gemm=dict(launches=kern["f64"]["launches"], ms_per_step=round(kern["f64"]["ms"] / steps, 2),
                       tflops=round(kern["f64"]["flops"] / max(kern["f64"]["ms"], 1e-9) * 1e-9, 2)),
        bf16x3_gemm=dict(launches=kern["bf16x3"]["launches"], ms_per_step=round(kern["bf16x3"]["ms"] / steps, 2),
                         algorithmic_tflops=round(kern["bf16x3"]["flops"] / max(kern["bf16x3"]["ms"], 1e-9) * 1e-9,
                                                  2)))


def job_figure(w, dtype_name, steps, warmup, refine=True, roofline=True):
    """Time `steps` steps of one job; its rate, GEMM rates and final-state errors."""
    import torch
    job = Job(w, dtype_name, DEFAULT_CHUNK[dtype_name], refine=refine)
    elapsed, times, kern = timed(job, steps, warmup, roofline=roofline)
    out = dict(value=round(w.M * steps / elapsed, 2), ms_per_step=round(1000 * elapsed / steps, 2))
    if roofline:
        out.update(gemm_rates(kern, steps))
    ref = golden_state(w_name(w))
    if ref is not None:
        out.update(state_errors(ref, job.psi.cpu().numpy()))
    del job
    torch.cuda.empty_cache()
    return out


def w_name(w):
    return {"spin_chain_10": "spin_chain_10_d1024",
            "transmon10x_resonator100": "transmon10x_resonator100_d1000"}.get(w.name, w.name)


def main():
    a = parse()
    if a.action:
        action(a)
        return
    if a.c5:
        c5(a)
        return
    if a.npad:
        npad_bench(a)
        return
    if a.sweep:
        sweep(a)
        return
    if a.copy_calibration:
        copy_calibration()
        return
    if a.serve:
        serve(a)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2411_09982_amd as q
    q.lib()
    w = build_workload(a.workload)
    chunk = a.chunk or DEFAULT_CHUNK[a.dtype]
    refine = not a.no_refine
    job = Job(w, a.dtype, chunk, a.lanes, refine=refine)
    elapsed, times, kern = timed(job, a.steps, a.warmup)
    s_hist = job.s.cpu().numpy().tolist()
    value = w.M * a.steps / elapsed
    ms = 1000.0 * elapsed / a.steps
    fl_step = flop_count(w, s_hist)

    k = kern["f32"] if a.dtype == "c64" else kern["bf16x3"] if a.dtype == "bf16x3" else kern["f64"]
    executed = BF16X3_PARTS if a.dtype == "bf16x3" else 1    # MFMA flops per algorithmic flop
    achieved = executed * k["flops"] / (k["ms"] * 1e-3) / 1e12 if k["ms"] > 0 else 0.0
    peak = MFMA_PEAK_TFLOPS[a.dtype]
    # HBM bytes per launch as counted for this exact job and launch configuration
    traffic = (measured_traffic(a.workload) if a.dtype == "c64" and job.chunk == min(DEFAULT_CHUNK["c64"], w.M)
               and job.lanes == 1 and refine else None)
    roof = dict(bound="mfma", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                frac=round(achieved / peak, 4), traffic=traffic,
                kernel={"c64": "cgemm_kernel<float,...> (Pade products, squarings, unitary refinement)",
                        "bf16x3": "cgemm_bf16x3_planes_kernel (Pade products, squarings, unitary refinement; "
                                  "BF16 MFMA flops executed, 6 per algorithmic flop)",
                        "c128": "cgemm_kernel<double,...> (Pade products, squarings, LU updates)"}[a.dtype],
                launches=k["launches"], avg_launch_ms=round(k["ms"] / max(k["launches"], 1), 4),
                flops_per_launch=executed * k["flops"] / max(k["launches"], 1))
    extra = dict(
        whole_step_tflops=round(fl_step / (ms * 1e-3) / 1e12, 2),
        # the metric's "MFMA %" for a mixed pipeline: each precision's matrix flops
        # over its own peak, summed, over the step time
        mfma_frac_whole_step=round(
            (kern["f32"]["flops"] / (MFMA_PEAK_TFLOPS["c64"] * 1e12)
             + kern["bf16x3"]["flops"] * BF16X3_PARTS / (MFMA_PEAK_TFLOPS["bf16x3"] * 1e12)
             + kern["f64"]["flops"] / (MFMA_PEAK_TFLOPS["c128"] * 1e12)) / (a.steps * ms * 1e-3), 4),
        step_ms_p50=round(1000 * float(np.percentile(times, 50)), 2),
        step_ms_p99=round(1000 * float(np.percentile(times, 99)), 2),
        s_hist={str(v): s_hist.count(v) for v in sorted(set(s_hist))},
        chunk=job.chunk,
        lanes=job.lanes,
        unitary_refine=job.refine,
    )
    extra.update(gemm_rates(kern, a.steps))
    psi_mixed = job.psi.cpu().numpy()
    U_samples = {n: job.U[n].cpu().numpy().astype(np.complex128) for n in (0, w.M // 2, w.M - 1)}
    del job
    torch.cuda.empty_cache()
    ref = golden_state(a.workload)
    if ref is not None:
        # the whole chain against the oracle's (tests/golden/), in Sec. 4.3's error
        extra["final_state_vs_oracle"] = state_errors(ref, psi_mixed)

    if a.dtype in ("c64", "bf16x3") and not a.no_fp64_compare:
        f64 = job_figure(w, "c128", 1, 1, roofline=False)
        f64["mixed_speedup"] = round(value / f64["value"], 3)
        extra["fp64_plain"] = f64
        if refine:
            # the same tier without the unitary refinement: what it costs and buys
            unref = job_figure(w, a.dtype, 2, 1, refine=False, roofline=False)
            extra["fp32_unrefined"] = unref

    if a.second_workload and a.second_workload != a.workload:
        w2 = build_workload(a.second_workload)
        second = dict(workload=w2.name, d=w2.d, M=w2.M, order=w2.order)
        second[a.dtype] = job_figure(w2, a.dtype, 2, 1, refine=refine)
        if a.dtype != "c128":
            second["c128"] = job_figure(w2, "c128", 1, 1, roofline=False)
            second["mixed_speedup"] = round(second[a.dtype]["value"] / second["c128"]["value"], 3)
        extra["second_workload"] = second

    if a.line_serve_rate > 0 and a.line_serve_requests > 0:
        # serving (the metric's p50/p99 latency): one Poisson stream below saturation
        extra["serving"] = serve_pass(a.line_serve_rate, a.line_serve_requests, 2411, a.serve_dmax, a.serve_mmax)

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        cpu, U_or, _ = cpu_baseline(w, a.cpu_intervals)
        # the same oracle with its BLAS / LAPACK pinned to one thread, on a shorter prefix
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                one, _, _ = cpu_baseline(w, max(1, a.cpu_intervals // 12))
            extra["cpu_baseline_1thread"] = dict(value=round(one["value"], 3), unit=one["unit"], cores=1,
                                                 sample=one["sample"])
        except ImportError:
            pass
        # sampled parity of the benchmarked run: U_0 against the oracle's (d^2 form,
        # first order in any radial error, and its direction part), its unitarity
        extra["U0_vs_oracle"] = dict(
            infidelity=float(oracle.propagator_infidelity(U_or[0], U_samples[0])),
            direction_infidelity=float(oracle.propagator_infidelity(U_or[0], U_samples[0], normalized=True)),
            unitarity_error=float(oracle.unitarity_error(U_samples[0])))

    out = dict(
        metric="Magnus interval propagators/s at d=1024 (MFMA %) vs FP64 plain; p50/p99 latency",
        value=round(value, 3), unit="interval propagators/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=round(ms, 2), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={"c64": "c64+f64", "bf16x3": "c64(bf16x3)+f64", "c128": "c128"}[a.dtype],
        data="synthetic",
        config=dict(workload=w.name, d=w.d, K=w.K, N=w.N, M=w.M, order=w.order,
                    precision={"c64": "complex64 MFMA products and squarings, FP64 norm/scaling/Pade solve, "
                                      "FP64-Gram unitary refinement",
                               "bf16x3": "complex64 storage, products and squarings on BF16 MFMA with three-way "
                                         "split operands, FP64 norm/scaling/Pade solve, FP64-Gram unitary "
                                         "refinement",
                               "c128": "complex128 throughout"}[a.dtype]
                    if refine or a.dtype == "c128" else "unrefined " + a.dtype),
        roofline=roof, cpu_baseline=cpu, extra=extra,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
