"""Pins for the CPU oracle: each check ties it to something other than itself.

Closed forms, library routines (scipy.linalg.expm, scipy.integrate.quad,
scipy.integrate.solve_ivp), exact special cases and invariants.  A plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
product) fails at least one of them; test_oracle_mutations.py plants such
mistakes to show it.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sl
from scipy.special import erf

import oracle
import workloads as wl

SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
SZ = np.array([[1, 0], [0, -1]], dtype=complex)


# ------------------------------------------------------------ coefficients

def test_c1_and_c20_linear_ramp_closed_form():
    # u(t) = alpha + beta (t - mid) sampled at cell midpoints of one interval:
    # integral = alpha*Dt exactly; c20 = -beta dt^3 s (s^2 - 1) / 6 exactly
    for s in (1, 2, 7, 50):
        dt, alpha, beta = 0.013, 0.7, -2.3
        t = (np.arange(s) + 0.5) * dt
        u = (alpha + beta * (t - 0.5 * s * dt))[None]
        c1, c2 = oracle.interval_coefficients(u, dt, 1, 2)
        assert c1[0, 0] == pytest.approx(alpha * s * dt, rel=1e-14, abs=1e-16)
        assert c2[0, 0] == pytest.approx(-beta * dt ** 3 * s * (s * s - 1) / 6.0, rel=1e-12, abs=1e-18)


def _zoh(vals, a, dt):
    """Piecewise-constant function from cell values starting at a."""
    def f(t):
        j = min(max(int(math.floor((t - a) / dt)), 0), len(vals) - 1)
        return vals[j]
    return f


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_second_order_coefficients_against_nested_quadrature():
    # Brute force: nested adaptive quadrature of the double integral of
    # Eq. magnus-avg for a zero-order-hold signal, with breakpoints on the cells.
    g = np.random.default_rng(7)
    K, s, M = 3, 5, 2
    dt = 0.37
    u = g.standard_normal((K, s * M))
    c1, c2 = oracle.interval_coefficients(u, dt, M, 2)
    opts = dict(epsabs=1e-14, epsrel=1e-14, limit=200)
    for n in range(M):
        a, b = n * s * dt, (n + 1) * s * dt
        pts = list(a + dt * np.arange(1, s))
        f = [_zoh(u[k, n * s:(n + 1) * s], a, dt) for k in range(K)]

        def inner(fun, t1):
            if t1 <= a:
                return 0.0
            p = [x for x in pts if x < t1]
            return si.quad(fun, a, t1, points=p or None, **opts)[0]

        for k in range(K):
            ref1 = si.quad(f[k], a, b, points=pts, **opts)[0]
            assert c1[n, k] == pytest.approx(ref1, rel=1e-12, abs=1e-13)
            # int dt1 int_{a}^{t1} dt2 (u(t2) - u(t1))
            ref20 = si.quad(lambda t1: inner(f[k], t1) - (t1 - a) * f[k](t1), a, b,
                            points=pts, **opts)[0]
            assert c2[n, k] == pytest.approx(ref20, rel=1e-10, abs=1e-12)
        for k in range(K):
            for l in range(k + 1, K):
                ref = si.quad(lambda t1: f[k](t1) * inner(f[l], t1) - f[l](t1) * inner(f[k], t1),
                              a, b, points=pts, **opts)[0]
                assert c2[n, oracle.pair_index(k, l, K)] == pytest.approx(ref, rel=1e-10, abs=1e-12)


def test_c2_pair_sinusoid_continuum_limit():
    # u_0 = cos(w t), u_1 = sin(w t) on [0, Dt]: the double integral of
    # sin(w (t2 - t1)) over t2 < t1 is -Dt/w + sin(w Dt)/w^2 (midpoint hold error O(dt^2))
    w, Dt, s = 3.1, 1.7, 4000
    dt = Dt / s
    t = (np.arange(s) + 0.5) * dt
    u = np.stack([np.cos(w * t), np.sin(w * t)])
    _, c2 = oracle.interval_coefficients(u, dt, 1, 2)
    exact = -Dt / w + math.sin(w * Dt) / w ** 2
    assert c2[0, oracle.pair_index(0, 1, 2)] == pytest.approx(exact, rel=1e-6)
    # and [H0, H_k] weights: int (a + b - 2 tau) cos(w tau) d tau on [0, Dt]
    ex0 = (Dt * math.sin(w * Dt) / w) - 2 * ((math.cos(w * Dt) - 1) / w ** 2 + Dt * math.sin(w * Dt) / w)
    assert c2[0, 0] == pytest.approx(ex0, rel=1e-6)


def test_second_order_coefficients_vanish_and_flip():
    g = np.random.default_rng(3)
    K, s, M, dt = 3, 8, 4, 0.1
    const = np.repeat(g.standard_normal((K, M)), s, axis=1)
    _, c2 = oracle.interval_coefficients(const, dt, M, 2)
    assert np.abs(c2).max() < 1e-15
    u = g.standard_normal((K, s * M))
    u[2] = 2.5 * u[0]                                  # proportional pair
    _, c2 = oracle.interval_coefficients(u, dt, M, 2)
    assert np.abs(c2[:, oracle.pair_index(0, 2, K)]).max() < 1e-14
    # reversing the samples inside every interval negates every c2 column
    ur = u.reshape(K, M, s)[:, :, ::-1].reshape(K, M * s)
    _, c2r = oracle.interval_coefficients(ur, dt, M, 2)
    np.testing.assert_allclose(c2r, -c2, rtol=1e-12, atol=1e-15)
    # swapping the controls negates the pair coefficient, keeps c20
    sw = u[[1, 0, 2]]
    _, c2s = oracle.interval_coefficients(sw, dt, M, 2)
    np.testing.assert_allclose(c2s[:, oracle.pair_index(0, 1, K)], -c2[:, oracle.pair_index(0, 1, K)], rtol=1e-12)
    np.testing.assert_allclose(c2s[:, 0], c2[:, 1], rtol=1e-12)


# ------------------------------------------------------------- exponential

@pytest.mark.parametrize("d", [1, 2, 5, 16])
def test_expm_matches_scipy(d):
    g = np.random.default_rng(d)
    for scale in (0.01, 1.0, 30.0):
        Om = -1j * wl.random_hermitian(d, g, scale)
        np.testing.assert_allclose(oracle.expm_skew_hermitian(Om), sl.expm(Om), atol=1e-12 * max(1, scale))


def test_rabi_closed_form():
    # constant H = (D/2) sz + (W/2) sx: U(T) = cos(th) I - i sin(th) (D sz + W sx)/W_R,
    # th = W_R T / 2, W_R = sqrt(D^2 + W^2) (two-level form of Sec. 3.2)
    D, W, T = 0.8, 2.3, 3.7
    N, M = 60, 12
    for order in (1, 2):
        res = oracle.run(0.5 * D * SZ, (0.5 * SX)[None], np.full((1, N), W), T / N, M, order, product=True)
        WR = math.hypot(D, W)
        th = 0.5 * WR * T
        exact = math.cos(th) * np.eye(2) - 1j * math.sin(th) * (D * SZ + W * SX) / WR
        np.testing.assert_allclose(res["P"], exact, atol=1e-13)


def test_commuting_diagonal_closed_form():
    g = np.random.default_rng(11)
    d, K, N, M, dt = 6, 2, 40, 8, 0.05
    e = g.standard_normal(d)
    f = g.standard_normal((K, d))
    u = g.standard_normal((K, N))
    for order in (1, 2):
        res = oracle.run(np.diag(e).astype(complex), np.stack([np.diag(x).astype(complex) for x in f]),
                         u, dt, M, order, product=True)
        phase = e * N * dt + (f * (u.sum(axis=1) * dt)[:, None]).sum(axis=0)
        np.testing.assert_allclose(res["P"], np.diag(np.exp(-1j * phase)), atol=1e-13)
        if order == 2:  # commutators vanish, so H-bar is the first-order term alone
            r1 = oracle.run(np.diag(e).astype(complex), np.stack([np.diag(x).astype(complex) for x in f]),
                            u, dt, M, 1)
            np.testing.assert_allclose(res["Hbar"], r1["Hbar"], atol=1e-15)


def test_rwa_gaussian_closed_form():
    # H_RWA(t) = Om(t)/4 sx (Eq. magnus-rwa-ham) commutes with itself:
    # U = cos(th) I - i sin(th) sx with th = int Om / 4 (erf for a Gaussian)
    Om0, T, sig, N, M = 1.3, 20.0, 3.0, 20000, 50
    t, dt = wl.midpoints(N, T)
    Om = Om0 * np.exp(-((t - T / 2) ** 2) / (2 * sig * sig))
    res = oracle.run(np.zeros((2, 2), complex), (0.25 * SX)[None], Om[None], dt, M, 2, product=True)
    th = 0.25 * Om0 * sig * math.sqrt(math.pi / 2) * 2 * erf(T / (2 * math.sqrt(2) * sig))
    exact = math.cos(th) * np.eye(2) - 1j * math.sin(th) * SX
    np.testing.assert_allclose(res["P"], exact, atol=1e-8)


def test_determinant_and_unitarity():
    w = wl.random_system(7, 2, 400, 20, 2, config_id=41)
    res = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, w.order, psi0=w.psi0, product=True)
    for n in range(w.M):
        assert np.linalg.det(res["U"][n]) == pytest.approx(np.exp(-1j * np.trace(res["Hbar"][n]).real), abs=1e-12)
    assert oracle.unitarity_error(res["U"]) < 1e-13
    assert oracle.unitarity_error(res["P"]) < 1e-12
    assert abs(np.linalg.norm(res["psi"]) - 1) < 1e-13
    np.testing.assert_allclose(res["P"] @ w.psi0, res["psi"], atol=1e-12)


def test_state_infidelity_definition():
    # Sec. 4.3's error 1 - |<psi_ref|psi>|^2 on the vectors as they are: a global
    # phase of a unit vector is no error, a rescaled vector is (1 - 1.7^2), an
    # orthogonal state is 1, two unit vectors at angle a give sin^2 a
    g = np.random.default_rng(3)
    psi = g.standard_normal(6) + 1j * g.standard_normal(6)
    psi /= np.linalg.norm(psi)
    assert abs(oracle.state_infidelity(psi, np.exp(0.4j) * psi)) < 1e-15
    assert oracle.state_infidelity(psi, 1.7 * psi) == pytest.approx(1.0 - 1.7 ** 2, abs=1e-14)
    assert oracle.state_infidelity(psi, (1.0 + 1e-4) * psi) == pytest.approx(-2e-4 - 1e-8, abs=1e-15)
    e0, e1 = np.eye(2)[0].astype(complex), np.eye(2)[1].astype(complex)
    assert oracle.state_infidelity(e0, e1) == pytest.approx(1.0, abs=1e-15)
    a = 0.3
    assert oracle.state_infidelity(e0, math.cos(a) * e0 + 1j * math.sin(a) * e1) == pytest.approx(math.sin(a) ** 2,
                                                                                                   abs=1e-15)
    assert oracle.norm_error(1.25 * psi) == pytest.approx(0.25, abs=1e-15)
    assert oracle.norm_error(psi) < 1e-15


def test_direction_infidelity_of_rays():
    # the direction part alone: a global phase or a rescaling leaves the ray
    # unchanged; orthogonal rays are 1; rays at angle a give sin^2 a at any scale
    g = np.random.default_rng(3)
    psi = g.standard_normal(6) + 1j * g.standard_normal(6)
    psi /= np.linalg.norm(psi)
    assert abs(oracle.direction_infidelity(psi, 1.7 * np.exp(0.4j) * psi)) < 1e-15
    e0, e1 = np.eye(2)[0].astype(complex), np.eye(2)[1].astype(complex)
    assert oracle.direction_infidelity(e0, 3.0 * e1) == pytest.approx(1.0, abs=1e-15)
    a = 0.3
    v = 2.5 * (math.cos(a) * e0 + 1j * math.sin(a) * e1)
    assert oracle.direction_infidelity(e0, v) == pytest.approx(math.sin(a) ** 2, abs=1e-15)


def test_generators_sign():
    # exp(Omega_n) must be the propagator exp(-i H-bar_n) of the interval: for a
    # constant two-level drive the Rabi closed form fixes the sign of Omega = -i H-bar
    D, W, T = 0.8, 2.3, 0.9
    c1, c2 = oracle.interval_coefficients(np.full((1, 10), W), T / 10, 1, 2)
    Om = oracle.generators(0.5 * D * SZ, (0.5 * SX)[None], c1, c2, T, 2)
    WR = math.hypot(D, W)
    th = 0.5 * WR * T
    exact = math.cos(th) * np.eye(2) - 1j * math.sin(th) * (D * SZ + W * SX) / WR
    np.testing.assert_allclose(sl.expm(Om[0]), exact, atol=1e-14)
    np.testing.assert_allclose(Om[0] + Om[0].conj().T, 0.0, atol=1e-15)


def test_normalized_propagator_infidelity():
    # equal to the d^2 form for unitary operands; blind to a rescaling; 1 for
    # trace-orthogonal operators; never negative (Cauchy-Schwarz)
    U = sl.expm(-1j * wl.random_hermitian(5, np.random.default_rng(4)))
    V = sl.expm(-1j * wl.random_hermitian(5, np.random.default_rng(5)))
    assert oracle.propagator_infidelity(U, V, normalized=True) == pytest.approx(oracle.propagator_infidelity(U, V),
                                                                                abs=1e-14)
    assert abs(oracle.propagator_infidelity(U, 1.3 * np.exp(0.2j) * U, normalized=True)) < 1e-15
    assert abs(oracle.propagator_infidelity(U, 1.3 * U)) > 0.5                 # the d^2 form sees the norm
    Z = np.diag([1.0, -1.0]).astype(complex)
    assert oracle.propagator_infidelity(np.eye(2), Z, normalized=True) == pytest.approx(1.0, abs=1e-15)
    g = np.random.default_rng(6)
    A = g.standard_normal((3, 4, 4)) + 1j * g.standard_normal((3, 4, 4))
    B = g.standard_normal((3, 4, 4)) + 1j * g.standard_normal((3, 4, 4))
    assert np.all(oracle.propagator_infidelity(A, B, normalized=True) >= -1e-15)


def test_scaling_exponent_definition():
    th = oracle.THETA13_F64
    g = np.random.default_rng(5)
    for target in [0.1, th, th * 1.0000001, 2 * th, 3 * th, 100.0, 1234.5]:
        Om = wl.random_skew_hermitian_batch(1, 9, target, config_id=int(target * 1000) % 97)[0]
        for shift in (False, True):
            s = oracle.scaling_exponent(Om, shift=shift)
            n1 = oracle.norm1(Om - (oracle.trace_shift(Om) if shift else 0.0) * np.eye(9))
            assert n1 / 2 ** s <= th * (1 + 1e-15)
            if s > 0:
                assert n1 / 2 ** (s - 1) > th
    assert oracle.norm1(np.array([[1, -2j], [3, 0.5]])) == pytest.approx(2.5 + 1.5)
    del g


def test_trace_shift():
    # exp(Omega) = e^mu exp(Omega - mu I) (scipy's expm on both sides); a large
    # multiple of I in the generator costs no squaring once it is split off
    B = wl.random_skew_hermitian_batch(1, 6, 2.0, config_id=9)[0]
    Om = B - 300j * np.eye(6)
    mu = oracle.trace_shift(Om)
    assert mu == pytest.approx(np.trace(B) / 6 - 300j, abs=1e-12)
    np.testing.assert_allclose(sl.expm(Om), np.exp(mu) * sl.expm(Om - mu * np.eye(6)), atol=1e-11)
    assert oracle.scaling_exponent(Om, shift=False) == 6          # ||Om||_1 ~ 302 <= 64 theta_13
    assert oracle.scaling_exponent(Om) == oracle.scaling_exponent(B - oracle.trace_shift(B) * np.eye(6)) == 0
    assert oracle.scaling_exponent(np.full((3, 3), np.nan)) == -1


# -------------------------------------------------------------------- chain

def _fine_product(w):
    P = np.eye(w.d, dtype=complex)
    for j in range(w.N):
        H = w.H0 + np.tensordot(w.u[:, j], w.Hk, axes=1)
        P = sl.expm(-1j * w.dt_sample * H) @ P
    return P


@pytest.mark.parametrize("order", [1, 2])
def test_one_sample_per_interval_is_exact(order):
    # M = N: every interval is one constant cell, so Magnus of any order is exact
    w = wl.random_system(4, 2, 64, 64, order, config_id=9, drift_scale=3.0, drive_scale=2.0, t_total=4.0)
    res = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, order, product=True)
    np.testing.assert_allclose(res["P"], _fine_product(w), atol=1e-12)


def test_against_ode_integration():
    # independent integrator: DOP853 on i dpsi/dt = H(t) psi, cell by cell
    w = wl.random_system(3, 2, 48, 48, 1, config_id=21, drift_scale=2.0, drive_scale=1.5, t_total=3.0)
    psi = w.psi0.copy()
    for j in range(w.N):
        H = w.H0 + np.tensordot(w.u[:, j], w.Hk, axes=1)
        sol = si.solve_ivp(lambda t, y: -1j * (H @ y), (0, w.dt_sample), psi, method="DOP853",
                           rtol=1e-13, atol=1e-14)
        psi = sol.y[:, -1]
    res = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, 1, psi0=w.psi0)
    np.testing.assert_allclose(res["psi"], psi, atol=1e-10)


def test_convergence_orders():
    # error of the M-interval product against the exact fine product falls as
    # M^-2 (first order) and M^-4 (second order)
    N = 2048
    w = wl.random_system(3, 2, N, 1, 1, config_id=33, drift_scale=2.0, drive_scale=1.0, t_total=2.0)
    ref = _fine_product(w)
    for order, slope in ((1, 2.0), (2, 4.0)):
        Ms = [16, 32, 64]
        errs = []
        for M in Ms:
            P = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, M, order, product=True)["P"]
            errs.append(np.abs(P - ref).max())
        slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(Ms) - 1)]
        assert all(abs(x - slope) < 0.25 for x in slopes), (order, errs, slopes)


def test_chain_order_left_multiplication():
    # two non-commuting constant intervals: P = U_2 U_1, not U_1 U_2
    H0 = np.zeros((2, 2), complex)
    Hk = np.stack([SX, SZ])
    u = np.array([[1.0, 0.0], [0.0, 1.0]])
    res = oracle.run(H0, Hk, u, 0.7, 2, 1, product=True)
    exact = sl.expm(-0.7j * SZ) @ sl.expm(-0.7j * SX)
    np.testing.assert_allclose(res["P"], exact, atol=1e-14)
    assert np.abs(res["P"] - sl.expm(-0.7j * SX) @ sl.expm(-0.7j * SZ)).max() > 0.1


def test_input_checks():
    H = np.eye(2, dtype=complex)
    with pytest.raises(ValueError):
        oracle.check_inputs(H, H[None], np.zeros((1, 10)), 3)
    with pytest.raises(ValueError):
        oracle.check_inputs(np.array([[0, 1], [0, 0]], complex), H[None], np.zeros((1, 10)), 5)
    with pytest.raises(ValueError):
        oracle.check_inputs(H, H[None], np.full((1, 10), np.nan), 5)
    oracle.check_inputs(H, H[None], np.zeros((1, 10)), 5)


def test_pade_theta_reproduces_higham_table():
    # Higham (2005), Table 2.3 (u = 2^-53): theta_3 .. theta_13 of the [m/m] approximant
    import oracle.pade_theta as pt
    table = {3: 1.495585217958292e-2, 5: 2.539398330063230e-1, 7: 9.504178996162932e-1,
             9: 2.097847961257068e0, 13: 5.371920351148152e0}
    for m, val in table.items():
        assert pt.theta(m, 2.0 ** -53, n=120) == pytest.approx(val, rel=1e-14)
    assert oracle.THETA13_F64 == table[13]


# --------------------------------------------------------- third-order term

def _bch_cells(H0, Hk, u, dt):
    """A_j = -i (H0 + sum_k u[k, j] H_k) of each cell j and the exact log of the
    product exp(A_s dt) ... exp(A_1 dt) (scipy.linalg.logm)."""
    A = [-1j * (H0 + sum(u[k, j] * Hk[k] for k in range(len(Hk)))) for j in range(u.shape[1])]
    P = np.eye(H0.shape[0], dtype=complex)
    for a in A:
        P = sl.expm(a * dt) @ P
    return A, sl.logm(P)


def _omega3(H0, Hk, u, dt):
    T = oracle.third_order_coefficients(u, dt, 1)
    return -1j * oracle.third_order_term(H0, Hk, T)[0]


def test_third_order_two_cells_is_bch():
    # for two cells the third-order term is the degree-3 part of the
    # Baker-Campbell-Hausdorff series, dt^3/12 ([A2,[A2,A1]] + [A1,[A1,A2]]), exactly
    g = np.random.default_rng(21)
    H0, Hk = wl.random_hermitian(4, g), np.stack([wl.random_hermitian(4, g) for _ in range(2)])
    u = g.standard_normal((2, 2))
    dt = 0.3
    A1, A2 = [-1j * (H0 + u[0, j] * Hk[0] + u[1, j] * Hk[1]) for j in range(2)]
    c = lambda X, Y: X @ Y - Y @ X
    bch3 = dt ** 3 / 12.0 * (c(A2, c(A2, A1)) + c(A1, c(A1, A2)))
    np.testing.assert_allclose(_omega3(H0, Hk, u, dt), bch3, atol=1e-15)


def test_third_order_leaves_fourth_order_residual():
    # over several cells, Omega_1 + Omega_2 + Omega_3 matches log of the exact
    # product up to O(dt^4): halving dt divides the residual by 16
    g = np.random.default_rng(22)
    H0, Hk = wl.random_hermitian(3, g), np.stack([wl.random_hermitian(3, g)])
    u = g.standard_normal((1, 5))
    res = []
    for dt in (0.08, 0.04, 0.02):
        _, L = _bch_cells(H0, Hk, u, dt)
        c1, c2 = oracle.interval_coefficients(u, dt, 1, 2)
        Om12 = oracle.generators(H0, Hk, c1, c2, 5 * dt, 2)[0]
        res.append(np.abs(L - Om12 - _omega3(H0, Hk, u, dt)).max())
    ratios = [res[i] / res[i + 1] for i in range(2)]
    assert all(14.0 < r < 18.0 for r in ratios), (res, ratios)


def test_third_order_coefficients_by_cell_volumes():
    # brute force over cell triples with the simplex volumes 1, 1/2, 1/6
    g = np.random.default_rng(23)
    u = g.standard_normal((2, 5))
    dt = 0.7
    T = oracle.third_order_coefficients(u, dt, 1)[0]
    x = np.vstack([np.ones(5), u])
    for a in range(3):
        for b in range(3):
            for c in range(3):
                tot = 0.0
                for i in range(5):
                    for j in range(i + 1):
                        for k in range(j + 1):
                            vol = 1.0 if i > j > k else (1.0 / 6.0 if i == j == k else 0.5)
                            tot += vol * x[a, i] * x[b, j] * x[c, k]
                assert T[a, b, c] == pytest.approx(dt ** 3 * tot, rel=1e-13, abs=1e-15)


def test_third_order_vanishes_for_constant_signals():
    # a constant H commutes with itself at all times
    g = np.random.default_rng(24)
    H0, Hk = wl.random_hermitian(3, g), np.stack([wl.random_hermitian(3, g)])
    u = np.full((1, 6), 0.8)
    assert np.abs(_omega3(H0, Hk, u, 0.1)).max() < 1e-15


def test_third_order_convergence():
    # with the third-order term the method stays fourth order (its own error is of
    # the size of the fourth-order term) but with a smaller constant than order 2
    N = 2048
    w = wl.random_system(3, 2, N, 1, 1, config_id=33, drift_scale=2.0, drive_scale=1.0, t_total=2.0)
    ref = _fine_product(w)
    errs = {}
    for order in (2, 3):
        errs[order] = [np.abs(oracle.run(w.H0, w.Hk, w.u, w.dt_sample, M, order, product=True)["P"] - ref).max()
                       for M in (16, 32, 64)]
    slopes = [math.log2(errs[3][i] / errs[3][i + 1]) for i in range(2)]
    assert all(abs(x - 4.0) < 0.25 for x in slopes), slopes
    assert all(e3 < 0.5 * e2 for e2, e3 in zip(errs[2], errs[3])), errs
    # one sample per interval: every term beyond the first vanishes, the result is exact
    r = oracle.run(w.H0, w.Hk, w.u[:, :64], w.dt_sample, 64, 3, product=True)
    assert np.abs(r["T"]).max() > 0 and np.abs(oracle.third_order_term(w.H0, w.Hk, r["T"])).max() < 1e-14
