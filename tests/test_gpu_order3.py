"""The third-order Magnus term on the GPU (order 3 of qcheff_magnus_coeffs and
qcheff_magnus_generators) against the oracle (oracle.third_order_coefficients,
oracle.third_order_term, oracle.run(order=3)).

Tolerances: the third-order coefficients within 1e-13 of dt^3 s^3 max|x|^3 (the
running prefix sums of each lane are plain FP64 sums over s samples); generators
as at order 2 (1e-14 d max|Omega| in complex128, 1.2e-7 max|Omega| in complex64);
propagators and states 1e-12 (FP64) and 1e-6 (FP32 products, refined)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests.test_gpu_parity import gpu, host, say

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")


def packed_c3(T):
    """The oracle's T[n,a,b,c] in the library's column order (a, then c >= a, then b;
    a = b = c left out): T_abc + T_cba for a < c, T_aba for a = c."""
    M, K1 = T.shape[0], T.shape[1]
    cols = []
    for a in range(K1):
        for c in range(a, K1):
            for b in range(K1):
                if a == b == c:
                    continue
                cols.append(T[:, a, b, c] + T[:, c, b, a] if a < c else T[:, a, b, a])
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("K,N,M", [(1, 300, 10), (2, 4000, 40), (3, 70, 7), (2, 600, 1), (3, 2560, 5)])
def test_coeffs_order3(K, N, M):
    say(f"coeffs order 3 K={K} N={N} M={M}")
    g = np.random.default_rng(K * 100 + M)
    t = np.linspace(0, 3, N)
    u = np.stack([np.cos(2.3 * t + k) + 0.4 * g.standard_normal(N) for k in range(K)])
    dt = 3.0 / N
    c1, c2 = q.magnus_coeffs(gpu(u), dt, M, 3)
    torch.cuda.synchronize()
    c1o, c2o = oracle.interval_coefficients(u, dt, M, 2)
    T = oracle.third_order_coefficients(u, dt, M)
    P2 = K + K * (K - 1) // 2
    got = host(c2)
    assert got.shape[1] == P2 + (K + 1) * K * (K + 3) // 2
    np.testing.assert_allclose(host(c1), c1o, rtol=0, atol=1e-14 * np.abs(c1o).max())
    np.testing.assert_allclose(got[:, :P2], c2o, rtol=0, atol=1e-13 * np.abs(c2o).max())
    s = N // M
    scale = dt ** 3 * s ** 3 * max(1.0, np.abs(u).max()) ** 3
    err = np.abs(got[:, P2:] - packed_c3(T)).max()
    say(f"  third-order coefficients: max error {err:.2e} (scale {scale:.2e})")
    assert err <= 1e-13 * scale


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d,K", [(5, 1), (33, 2), (130, 3)])
def test_generators_order3(d, K, dtype):
    say(f"generators order 3 d={d} K={K} {dtype}")
    w = wl.random_system(d, K, 12 * 9, 12, 3, config_id=40 + d, drift_scale=10.0, drive_scale=3.0)
    c1o, c2o = oracle.interval_coefficients(w.u, w.dt_sample, w.M, 2)
    T = oracle.third_order_coefficients(w.u, w.dt_sample, w.M)
    Hb = oracle.effective_hamiltonians(w.H0, w.Hk, c1o, c2o, w.dt_interval, 2) + oracle.third_order_term(w.H0, w.Hk, T)
    ref = -1j * 0.5 * (Hb + np.conj(np.swapaxes(Hb, 1, 2)))
    c1, c2 = q.magnus_coeffs(gpu(w.u), w.dt_sample, w.M, 3)
    om, ws = q.magnus_generators(gpu(w.H0), gpu(w.Hk), c1, c2, w.dt_interval, 3, dtype)
    torch.cuda.synchronize()
    err = np.abs(host(om).astype(np.complex128) - ref).max()
    tol = (1e-14 * d if dtype == torch.complex128 else 1.2e-7) * np.abs(ref).max()
    say(f"  max error {err:.2e} (tol {tol:.2e})")
    assert err <= tol
    oh = host(om)
    assert np.abs(oh + np.conj(np.swapaxes(oh, 1, 2))).max() == 0.0      # skew-Hermitian by construction
    # the cached basis (order 2 and 3 parts) serves new signals of the same operators
    u2 = w.u[::-1].copy() * 1.3
    c1b, c2b = q.magnus_coeffs(gpu(u2), w.dt_sample, w.M, 3)
    om2, _ = q.magnus_generators(gpu(w.H0), gpu(w.Hk), c1b, c2b, w.dt_interval, 3, dtype, ws=ws, reuse_basis=True)
    r2 = oracle.run(w.H0, w.Hk, u2, w.dt_sample, w.M, 3, check=False)["Omega"]
    assert np.abs(host(om2).astype(np.complex128) - r2).max() <= 2 * tol * max(1.0, np.abs(r2).max() / np.abs(ref).max())


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_evolve_order3_end_to_end(dtype):
    say(f"evolve order 3, random system d=48 {dtype}")
    w = wl.random_system(48, 2, 40 * 15, 40, 3, config_id=89, drift_scale=30.0, drive_scale=5.0)
    ref = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, 3, psi0=w.psi0)
    out = q.evolve(gpu(w.H0), gpu(w.Hk), gpu(w.u), w.dt_sample, w.M, 3, psi0=gpu(w.psi0), dtype=dtype, chunk=16)
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == torch.complex128 else 1e-6
    inf = np.abs(oracle.propagator_infidelity(ref["U"], host(out["U"]).astype(np.complex128)))
    sinf = abs(oracle.state_infidelity(ref["psi"], host(out["psi"])))
    say(f"  max U_n infidelity {inf.max():.2e}, state error {sinf:.2e}")
    assert np.all(inf <= tol) and sinf <= tol


def test_order3_more_accurate_than_order2():
    # the same job at M intervals against the exact product of the cell
    # propagators (one sample per interval, computed by the oracle): the
    # third-order term cuts the error of the second-order method
    w = wl.random_system(6, 2, 2048, 1, 1, config_id=33, drift_scale=2.0, drive_scale=1.0, t_total=2.0)
    exact = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, 2048, 1, product=True)["P"]
    errs = {}
    for order in (2, 3):
        out = q.evolve(gpu(w.H0), gpu(w.Hk), gpu(w.u), w.dt_sample, 32, order, dtype=torch.complex128, product=True)
        torch.cuda.synchronize()
        errs[order] = np.abs(host(out["P"]) - exact).max()
    say(f"  M = 32: error order 2 {errs[2]:.2e}, order 3 {errs[3]:.2e}")
    assert errs[3] < 0.5 * errs[2]
