"""Write whole-chain expected values of the two d ~ 1000 jobs from the CPU oracle alone.

Run:  python tests/golden/make_chain_goldens.py [spin_chain_10_d1024] [transmon10x_resonator100_d1000]

For each job (the 10-spin chain of Sec. 4.3: d = 1024, K = 2, 1e4 samples, M = 200,
second order; the transmon x resonator job: d = 1000, K = 2, 1e5 samples, M = 1000,
second order) the oracle runs the stroboscopic chain of Sec. 4.1 over every interval,
a few intervals at a time so that no more than a chunk of propagators is held, and
stores in tests/golden/<job>_chain.npz:

  psi_at    [len(at)][d] complex128  the state psi_n after interval n for n in `at`
                                     (every M/20 intervals, n = 0 is psi_0);
  at        int64 indices n of psi_at;
  trace_U   [M] complex128           tr U_n for every interval;
  probe     [d] complex128           a seeded unit vector v;
  probe_at  int64 intervals n of probe_U;
  probe_U   [len(probe_at)][d]       U_n v for those intervals.

The paper prints no Magnus values for these jobs; the numbers come from the oracle
(complex128, eigendecomposition exponentials) and serve the full-size GPU tests.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

JOBS = {
    "spin_chain_10_d1024": wl.spin_chain,
    "transmon10x_resonator100_d1000": wl.transmon_resonator,
}
CHUNK = 8
PROBE_SEED = 977


def chain_goldens(w, on_chunk=None):
    """Oracle chain of workload w; on_chunk(n0, U) sees every chunk of propagators."""
    M = w.M
    c1, c2 = oracle.interval_coefficients(w.u, w.dt_sample, M, w.order)
    step = max(1, M // 20)
    at = list(range(0, M + 1, step))
    if at[-1] != M:
        at.append(M)
    probe_at = sorted(set(list(range(0, M, max(1, M // 10))) + [M - 1]))
    v = wl.random_state(w.d, PROBE_SEED)
    psi = w.psi0.astype(np.complex128).copy()
    psi_at = [psi.copy()]
    trace_U = np.empty(M, dtype=np.complex128)
    probe_U = []
    t0 = time.time()
    for n0 in range(0, M, CHUNK):
        n1 = min(M, n0 + CHUNK)
        Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1[n0:n1], None if c2 is None else c2[n0:n1],
                                           w.dt_interval, w.order)
        U = oracle.propagator_from_hamiltonian(Hb)
        if on_chunk is not None:
            on_chunk(n0, U)
        for j in range(n1 - n0):
            n = n0 + j
            trace_U[n] = np.trace(U[j])
            if n in probe_at:
                probe_U.append(U[j] @ v)
            psi = oracle.propagate_state(U[j:j + 1], psi)
            if n + 1 in at:
                psi_at.append(psi.copy())
        print(f"  {w.name}: {n1}/{M} intervals, {time.time() - t0:.0f} s", flush=True)
    return dict(psi_at=np.stack(psi_at), at=np.array(at, dtype=np.int64), trace_U=trace_U, probe=v,
                probe_at=np.array(probe_at, dtype=np.int64), probe_U=np.stack(probe_U))


def main(names):
    for name in names:
        w = JOBS[name]()
        g = chain_goldens(w)
        np.savez_compressed(os.path.join(HERE, f"{name}_chain.npz"), **g)


if __name__ == "__main__":
    main(sys.argv[1:] or list(JOBS))
