"""Write the stored expected values under tests/golden/ from the CPU oracle alone.

Run:  python tests/golden/make_golden.py
Fixture: the single-transmon (Duffing, d = 8) job with one Gaussian drive,
1e4 samples, M = 100 first-order intervals (Sec. 4.1, Eqs. magnus-first-order-term
and magnus-first-order-coeff), and the same job at second order.  The paper
prints no Magnus values for a worked example, so these numbers come from the
oracle and pin it against accidental change.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as wl  # noqa: E402


def main():
    out = {}
    for order in (1, 2):
        w = wl.transmon_duffing(order=order)
        r = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, order, psi0=w.psi0, product=True)
        out[f"order{order}"] = dict(
            workload=w.name, d=w.d, K=w.K, N=w.N, M=w.M, dt_sample=w.dt_sample,
            c1_first5=r["c1"][:5, 0].tolist(),
            c2_first5=None if r["c2"] is None else r["c2"][:5, 0].tolist(),
            psi_final_re=r["psi"].real.tolist(), psi_final_im=r["psi"].imag.tolist(),
            P_diag_re=np.diag(r["P"]).real.tolist(), P_diag_im=np.diag(r["P"]).imag.tolist(),
        )
    with open(os.path.join(HERE, "transmon_duffing_d8.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
