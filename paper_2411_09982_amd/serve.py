"""Continuous-batching server for Magnus propagation jobs on one GPU.

Requests (H0, H_k, u, dt, M, order, precision, psi0) arrive over time.  A
request is admitted as soon as a slot is free and its device memory fits in the
HBM budget next to the jobs already running; each admitted job runs the whole
path on a stream of its own, so the kernels of different jobs overlap on the
device; its state stays device-resident until it completes.  Admission is
first-come first-served; a job that does not fit waits (it never overtakes an
earlier one).

A request asks for the final state only, so it is served by one of two paths:
"propagators" (coefficients, generators, exponentials, state chain) or "action"
(coefficients, then per chunk of intervals the generators and the truncated
Taylor action on the state, never forming a propagator).  "auto" takes the
propagators for d <= 32, where the fused one-workgroup exponential is cheapest,
and the action above that, where it replaces O(d^3) products per interval by a
few O(d^2) ones.

The admission and accounting logic (`Admission`) is plain host code and is
tested without a GPU; `Server` drives it with worker threads and HIP streams.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    H0: np.ndarray | None     # complex128 [d][d], exactly Hermitian
    Hk: np.ndarray | None     # complex128 [K][d][d], each exactly Hermitian
    u: np.ndarray | None      # float64 [K][N]
    dt_sample: float
    M: int
    order: int
    precision: str            # "c64" or "c128"
    psi0: np.ndarray | None   # complex128 [d]
    arrival: float = 0.0      # seconds, relative to the start of the stream
    path: str = "auto"        # "auto", "propagators" or "action"
    # A request may carry its inputs as a recipe instead: `build()` returns
    # (H0, Hk, u, psi0) and is called when the job starts (so a long stream of
    # large requests does not hold every payload in host memory); `dims` = (d, K)
    # then gives the sizes admission needs before that.
    build: Callable | None = None
    dims: tuple | None = None

    @property
    def d(self) -> int:
        return self.H0.shape[0] if self.H0 is not None else self.dims[0]

    @property
    def K(self) -> int:
        return self.Hk.shape[0] if self.Hk is not None else self.dims[1]

    def inputs(self):
        """(H0, Hk, u, psi0), built from the recipe if the request carries one."""
        if self.H0 is not None:
            return self.H0, self.Hk, self.u, self.psi0
        return self.build()


@dataclasses.dataclass
class Result:
    rid: int
    psi: np.ndarray
    s_max: int                # largest squaring count (propagator path), -1 for the action
    arrival: float
    admitted: float
    done: float
    path: str = "propagators"
    finite: bool = True       # False: a generator norm or a Pade pivot was not finite (the state is NaN)
    prep: float = 0.0         # seconds of the service time spent building the inputs and copying them in

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def job_bytes(d: int, K: int, M: int, order: int, precision: str, chunk: int, ws_fn=None,
              path: str = "propagators") -> int:
    """Device bytes one job holds while it runs: inputs, Omega/U (all M intervals
    for the propagators, one chunk for the action; complex64 propagators are
    refined into a separate complex128 U), workspaces, state."""
    eb = 8 if precision == "c64" else 16
    inputs = (1 + K) * d * d * 16
    omega = (M if path == "propagators" else min(chunk, M)) * d * d * eb
    if path == "propagators" and precision == "c64":
        omega += M * d * d * 16
    coeffs = M * (2 * K + K * (K - 1) // 2) * 8
    ws = ws_fn(d, K, M, order, precision, chunk) if ws_fn else 0
    return inputs + omega + coeffs + ws + 4 * d * 16


def path_for(r: "Request") -> str:
    """The path a request runs ("auto" resolved by its dimension)."""
    if r.path != "auto":
        return r.path
    return "propagators" if r.d <= 32 else "action"


class Admission:
    """FIFO admission under a byte budget and a slot limit (host logic only)."""

    def __init__(self, budget_bytes: int, max_slots: int):
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.in_use = 0
        self.running: dict[int, int] = {}
        self.waiting: collections.deque = collections.deque()

    def offer(self, rid: int, nbytes: int) -> None:
        if nbytes > self.budget:
            raise ValueError(f"request {rid} needs {nbytes} B, more than the whole budget {self.budget} B")
        self.waiting.append((rid, int(nbytes)))

    def admit(self) -> list[int]:
        """Admit waiting requests in arrival order while the head fits."""
        out = []
        while self.waiting and len(self.running) < self.max_slots:
            rid, nb = self.waiting[0]
            if self.in_use + nb > self.budget:
                break
            self.waiting.popleft()
            self.running[rid] = nb
            self.in_use += nb
            out.append(rid)
        return out

    def release(self, rid: int) -> None:
        self.in_use -= self.running.pop(rid)


class Server:
    """Runs requests with continuous batching: worker threads, one HIP stream each."""

    def __init__(self, budget_bytes: int, max_slots: int = 4, chunk: int = 64):
        import torch
        import paper_2411_09982_amd as q
        q.lib()
        self.q, self.torch = q, torch
        self.chunk = chunk
        self.adm = Admission(budget_bytes, max_slots)
        self.lock = threading.Condition()
        self.streams = [torch.cuda.Stream() for _ in range(max_slots)]
        self.free_streams = list(range(max_slots))
        self.requests: dict[int, Request] = {}
        self.results: dict[int, Result] = {}
        self.errors: dict[int, BaseException] = {}
        self.t0 = 0.0

    def _ws_bytes(self, d, K, M, order, precision, chunk, path="propagators"):
        q = self.q
        code = q.C64 if precision == "c64" else q.C128
        gen = q.workspace_bytes(q.FN_GENERATORS, 1, d, K, order, q.C128)
        if path == "action":
            return gen + q.workspace_bytes(q.FN_ACTION, min(chunk, M), d, 1, 1, code)
        return (gen + q.workspace_bytes(q.FN_EXPM, min(chunk, M), d, 1, 1, code)
                + q.workspace_bytes(q.FN_PROPAGATE, M, d, 1, q.STATE, q.C128))

    def bytes_for(self, r: Request) -> int:
        path = path_for(r)
        return job_bytes(r.d, r.K, r.M, r.order, r.precision, self.chunk,
                         lambda *a: self._ws_bytes(*a, path=path), path=path)

    def _run_job(self, r: Request, sidx: int, admitted: float) -> None:
        torch, q = self.torch, self.q
        st = self.streams[sidx]
        try:
            with torch.cuda.stream(st):
                dev = "cuda:0"
                dtype = torch.complex64 if r.precision == "c64" else torch.complex128
                t_in = time.perf_counter()
                H0h, Hkh, uh, psi0h = r.inputs()
                H0 = torch.from_numpy(H0h).to(dev, non_blocking=False)
                Hk = torch.from_numpy(Hkh).to(dev)
                u = torch.from_numpy(np.ascontiguousarray(uh)).to(dev)
                psi = torch.from_numpy(psi0h).to(dev)
                N = uh.shape[1]
                del H0h, Hkh, uh, psi0h
                prep = time.perf_counter() - t_in
                path = path_for(r)
                if path == "action":
                    psi = q.evolve_state(H0, Hk, u, r.dt_sample, r.M, r.order, psi, dtype=dtype, chunk=self.chunk,
                                         stream=st)
                    s_max = -1
                else:
                    c1, c2 = q.magnus_coeffs(u, r.dt_sample, r.M, r.order, stream=st)
                    omega, _ = q.magnus_generators(H0, Hk, c1, c2, r.dt_sample * (N // r.M), r.order, dtype,
                                                   stream=st)
                    # complex64: refined to unitarity and kept in complex128 (as evolve does)
                    fp32 = omega.dtype == torch.complex64
                    U, s = q.expm_batched(omega, U=None if fp32 else omega, chunk=self.chunk, stream=st,
                                          skew_hermitian=True, unitary_refine=fp32, out_c128=fp32)
                    del omega
                    q.propagate(U, q.STATE, psi, stream=st)
                    s_max = int(s.max().cpu())
                psi_h = psi.cpu().numpy()
                st.synchronize()
                # The library's status flags are per device and cannot name the job
                # that raised them; a job's own result says whether it is finite.
                # Taking the flags here keeps them from piling up across jobs.
                q.sync_status(st)
            done = time.perf_counter() - self.t0
            res = Result(r.rid, psi_h, s_max, r.arrival, admitted, done, path,
                         finite=bool(np.isfinite(psi_h).all()), prep=prep)
            with self.lock:
                self.results[r.rid] = res
        except BaseException as e:  # noqa: BLE001 - reported to the caller
            with self.lock:
                self.errors[r.rid] = e
        finally:
            with self.lock:
                self.adm.release(r.rid)
                self.free_streams.append(sidx)
                self.lock.notify_all()

    def _dispatch(self) -> None:
        with self.lock:
            for rid in self.adm.admit():
                sidx = self.free_streams.pop()
                admitted = time.perf_counter() - self.t0
                threading.Thread(target=self._run_job, args=(self.requests[rid], sidx, admitted),
                                 daemon=True).start()

    def run(self, requests: list[Request]) -> dict[int, Result]:
        """Feed requests at their arrival times; return results once all have finished."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        for r in reqs:
            delay = r.arrival - (time.perf_counter() - self.t0)
            if delay > 0:
                time.sleep(delay)
            with self.lock:
                self.requests[r.rid] = r
                self.adm.offer(r.rid, self.bytes_for(r))
            self._dispatch()
        while True:
            with self.lock:
                if len(self.results) + len(self.errors) >= len(reqs):
                    break
                self.lock.wait(timeout=0.05)
            self._dispatch()
        if self.errors:
            rid, e = next(iter(self.errors.items()))
            raise RuntimeError(f"request {rid} failed") from e
        return dict(self.results)


def poisson_requests(n: int, rate: float, seed: int, make: Callable[[int, np.random.Generator], Request]):
    """n requests with exponential inter-arrival times of mean 1/rate."""
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        r = make(i, g)
        r.arrival = float(t[i])
        out.append(r)
    return out


def max_overlap(results: dict[int, Result]) -> int:
    """Largest number of jobs that were running (admitted, not done) at one time."""
    ev = sorted([(r.admitted, 1) for r in results.values()] + [(r.done, -1) for r in results.values()])
    cur = best = 0
    for _, e in ev:
        cur += e
        best = max(best, cur)
    return best


def latency_percentiles(results: dict[int, Result]) -> dict:
    """p50/p99 of the latency (arrival to completion) and of its two parts: the
    wait for admission and the service time (admission to completion); and of the
    part of the service time spent building and copying the inputs."""
    vals = list(results.values())
    lat = np.array([r.latency for r in vals])
    wait = np.array([r.admitted - r.arrival for r in vals])
    svc = np.array([r.done - r.admitted for r in vals])
    prep = np.array([r.prep for r in vals])
    out = dict(n=int(lat.size))
    for name, a in (("", lat), ("wait_", wait), ("service_", svc), ("prep_", prep)):
        out[f"{name}p50_ms"] = float(np.percentile(a, 50) * 1e3)
        out[f"{name}p99_ms"] = float(np.percentile(a, 99) * 1e3)
    return out
