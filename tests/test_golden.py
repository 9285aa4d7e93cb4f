"""The oracle reproduces its stored single-transmon fixture (tests/golden/)."""
import json
import os

import numpy as np

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "transmon_duffing_d8.json")


def test_transmon_fixture():
    ref = json.load(open(GOLDEN))
    for order in (1, 2):
        g = ref[f"order{order}"]
        w = wl.transmon_duffing(order=order)
        r = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, order, psi0=w.psi0, product=True)
        np.testing.assert_allclose(r["c1"][:5, 0], g["c1_first5"], rtol=1e-13)
        if order == 2:
            np.testing.assert_allclose(r["c2"][:5, 0], g["c2_first5"], rtol=1e-11, atol=1e-18)
        psi = np.array(g["psi_final_re"]) + 1j * np.array(g["psi_final_im"])
        np.testing.assert_allclose(r["psi"], psi, atol=1e-11)
        assert oracle.state_infidelity(psi, r["psi"]) < 1e-13
