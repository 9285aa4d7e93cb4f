"""GPU parity: every C-ABI entry point against the CPU oracle, element by element.

Tolerances:
  FP64 path (QCHEFF_C128): propagator / state infidelity <= 1e-12 and
      max-abs error <= 1e-10 per U_n (a few hundred roundings of 2^-53 per entry);
  FP32 path (QCHEFF_C64, FP64 norm / scaling / Pade solve) with the unitary
      refinement (skew-Hermitian inputs, QCHEFF_UNITARY_REFINE): infidelity
      <= 1e-6 per U_n and for chained states in the unnormalised error of
      Sec. 4.3;
  FP32 results left unrefined (general inputs, whose exponential need not be
      unitary, or skew-Hermitian ones without the flag): 1e-6 or 4 2^s 2^-24,
      whichever is larger, because every FP32 squaring doubles the radial error
      the FP32 rounding of R leaves (inf_tol below);
  coefficients: within a few ulps of the sum of absolute terms (compensated sums).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")
DEV = "cuda:0"


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


INF_TOL = {torch.complex128: 1e-12, torch.complex64: 1e-6}
U32 = 2.0 ** -24


def inf_tol(dtype, s, refined=True):
    """Per-propagator infidelity bound.  1e-12 (FP64) or 1e-6 (FP32 products,
    refined to unitarity).  Unrefined FP32 results: every squaring doubles the
    deviation of |eigenvalue| from 1 left by the FP32 rounding of R, and that
    radial error enters 1 - |tr(U_ref^dag U)|^2/d^2 at first order, so the bound
    is 1e-6 or 4 * 2^s * u32, whichever is larger."""
    if dtype == torch.complex128 or refined:
        return np.full(np.shape(s), INF_TOL[dtype])
    return np.maximum(INF_TOL[dtype], 4.0 * 2.0 ** np.asarray(s, dtype=float) * U32)


EXPM_MODES = ["general", "skew", "refined", "refined_c128"]


def expm_mode(mode, dtype):
    """expm_batched keywords of a test mode; None where the mode does not apply
    (the FP64 path takes no refinement)."""
    if mode.startswith("refined") and dtype != torch.complex64:
        return None
    return dict(skew_hermitian=mode != "general", unitary_refine=mode.startswith("refined"),
                out_c128=mode == "refined_c128")


# ------------------------------------------------------------ coefficients

def _coeff_bounds(u, dt, M):
    """Sums of absolute terms per coefficient (scale for the rounding bound)."""
    a = np.abs(u)
    ua = oracle.interval_coefficients(a, dt, M, 1)[0]
    K, N = u.shape
    s = N // M
    w = np.abs(s - 1 - 2 * np.arange(s))
    c20 = np.stack([[dt * dt * (w * a[k, n * s:(n + 1) * s]).sum() for k in range(K)] for n in range(M)])
    return ua, c20


@pytest.mark.parametrize("K,N,M,order", [(1, 10_000, 100, 1), (2, 100_000, 1000, 2), (4, 91, 13, 2),
                                         (3, 40, 40, 2), (2, 5000, 1, 2), (1, 7, 7, 1)])
def test_coeffs_parity(K, N, M, order):
    say(f"coeffs K={K} N={N} M={M} order={order}")
    g = np.random.default_rng(K * 1000 + M)
    t = np.linspace(0, 7, N)
    u = np.stack([np.cos(3.1 * t + k) + 0.3 * g.standard_normal(N) for k in range(K)])
    dt = 7.0 / N
    c1o, c2o = oracle.interval_coefficients(u, dt, M, order)
    c1, c2 = q.magnus_coeffs(gpu(u), dt, M, order)
    torch.cuda.synchronize()
    ua, c20a = _coeff_bounds(u, dt, M)
    assert np.all(np.abs(host(c1) - c1o) <= 4e-16 * ua + 1e-300)
    if order == 2:
        c2g = host(c2)
        assert np.all(np.abs(c2g[:, :K] - c2o[:, :K]) <= 4e-16 * c20a + 1e-300)
        # pair terms: products with prefix sums; scale = dt^2 * s * sum|u_k| |u_l| style bound
        s = N // M
        for p in range(K, c2o.shape[1]):
            scale = dt * dt * s * np.max(np.abs(u)) ** 2 * s
            assert np.all(np.abs(c2g[:, p] - c2o[:, p]) <= 1e-14 * scale)


# -------------------------------------------------------------- generators

@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d,K,order", [(1, 1, 2), (7, 2, 2), (33, 3, 2), (130, 2, 1), (130, 2, 2), (200, 4, 2)])
def test_generators_parity(d, K, order, dtype):
    say(f"generators d={d} K={K} order={order} {dtype}")
    w = wl.random_system(d, K, 12 * 5, 12, order, config_id=d + K, drift_scale=20.0, drive_scale=3.0)
    c1, c2 = oracle.interval_coefficients(w.u, w.dt_sample, w.M, order)
    ref = oracle.generators(w.H0, w.Hk, c1, c2, w.dt_interval, order)
    H0, Hk = gpu(w.H0), gpu(w.Hk)
    om, ws = q.magnus_generators(H0, Hk, gpu(c1), gpu(c2) if order == 2 else None, w.dt_interval, order, dtype)
    torch.cuda.synchronize()
    err = np.abs(host(om) - ref).max()
    scale = np.abs(ref).max()
    tol = 1e-14 * scale * d if dtype == torch.complex128 else 1.2e-7 * scale
    assert err <= tol, (err, tol)
    # skew-Hermitian by construction
    om_h = host(om)
    assert np.abs(om_h + np.conj(np.swapaxes(om_h, 1, 2))).max() == 0.0
    if order == 2:
        # same operators, new signals: the cached commutator basis is reused
        u2 = w.u[::-1].copy() * 1.7
        c1b, c2b = oracle.interval_coefficients(u2, w.dt_sample, w.M, order)
        ref2 = oracle.generators(w.H0, w.Hk, c1b, c2b, w.dt_interval, order)
        om2, _ = q.magnus_generators(H0, Hk, gpu(c1b), gpu(c2b), w.dt_interval, order, dtype, ws=ws,
                                     reuse_basis=True)
        torch.cuda.synchronize()
        assert np.abs(host(om2) - ref2).max() <= 2 * tol


def test_generators_parity_long_chunks():
    # d = 730 fills 2048 blocks with one chunk of intervals, and K = 8 (44 coefficients
    # per interval) caps a chunk at 139 intervals: 200 intervals run as 139 + 61
    d, K, M = 730, 8, 200
    say(f"generators d={d} K={K} M={M}")
    w = wl.random_system(d, K, M * 5, M, 2, config_id=7, drift_scale=20.0, drive_scale=3.0)
    c1, c2 = oracle.interval_coefficients(w.u, w.dt_sample, w.M, 2)
    ref = oracle.generators(w.H0, w.Hk, c1, c2, w.dt_interval, 2)
    om, _ = q.magnus_generators(gpu(w.H0), gpu(w.Hk), gpu(c1), gpu(c2), w.dt_interval, 2, torch.complex64)
    torch.cuda.synchronize()
    err = np.abs(host(om) - ref).max()
    assert err <= 1.2e-7 * np.abs(ref).max(), err


# ------------------------------------------------------------- exponential

EXPM_DIMS = [1, 2, 3, 7, 8, 16, 17, 31, 32, 33, 64, 100, 128, 257]


@pytest.mark.parametrize("mode", EXPM_MODES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d", EXPM_DIMS)
def test_expm_parity(d, dtype, mode):
    # skew: the inputs are declared skew-Hermitian, so the Hermitian Pade
    # products are formed by halves and mirrored; refined: the FP32 result is
    # also refined to unitarity after its squarings
    kw = expm_mode(mode, dtype)
    if kw is None:
        pytest.skip("the FP64 path takes no refinement")
    refine = kw["unitary_refine"]
    say(f"expm d={d} {dtype} {mode}")
    q.sync_status()   # flags another test may have left
    norms = [0.0, 0.01, 1.0, 5.3, 5.4, 11.0, 11.5, 20.0, 170.0, 1500.0]   # s = 0 .. 9
    Om = wl.random_skew_hermitian_batch(len(norms), d, norms, config_id=300 + d)
    ref = oracle.expm_skew_hermitian(Om)
    seen = Om.astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else Om
    s_ref = [oracle.scaling_exponent(x, shift=(dtype == torch.complex128)) for x in seen]
    om = gpu(Om).to(dtype)
    U, s = q.expm_batched(om, **kw)
    torch.cuda.synchronize()
    Ug = host(U).astype(np.complex128)
    assert list(host(s)) == s_ref
    inf = np.abs(oracle.propagator_infidelity(ref, Ug))
    say(f"  max infidelity {inf.max():.2e}, unitarity {oracle.unitarity_error(Ug):.2e}")
    assert np.all(inf <= inf_tol(dtype, np.array(s_ref), refined=refine)), inf
    if dtype == torch.complex128:
        assert np.abs(Ug - ref).max() <= 1e-10
        assert oracle.unitarity_error(Ug) <= 1e-12
    elif refine:
        assert oracle.unitarity_error(Ug) <= 1e-6
    else:
        assert oracle.unitarity_error(Ug) <= 1e-3
    assert q.sync_status() == q.OK   # no pivot of a Pade denominator was zero


@pytest.mark.parametrize("mode", EXPM_MODES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d", [1024, 1030])
def test_expm_parity_large(d, dtype, mode):
    # d <= 1024 factors with register-resident panels, d > 1024 through the
    # global-memory panel kernel
    kw = expm_mode(mode, dtype)
    if kw is None:
        pytest.skip("the FP64 path takes no refinement")
    refine = kw["unitary_refine"]
    say(f"expm large d={d} {dtype} {mode}")
    q.sync_status()   # flags another test may have left
    norms = [3.0, 60.0, 900.0]
    Om = wl.random_skew_hermitian_batch(len(norms), d, norms, config_id=400 + d)
    ref = oracle.expm_skew_hermitian(Om)
    seen = Om.astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else Om
    s_ref = [oracle.scaling_exponent(x, shift=(dtype == torch.complex128)) for x in seen]
    U, s = q.expm_batched(gpu(Om).to(dtype), **kw)
    torch.cuda.synchronize()
    Ug = host(U).astype(np.complex128)
    assert list(host(s)) == s_ref
    inf = np.abs(oracle.propagator_infidelity(ref, Ug))
    say(f"  max infidelity {inf.max():.2e}, unitarity {oracle.unitarity_error(Ug):.2e}")
    assert np.all(inf <= inf_tol(dtype, np.array(s_ref), refined=refine)), inf
    if dtype == torch.complex128:
        assert np.abs(Ug - ref).max() <= 1e-10
    elif refine:
        assert oracle.unitarity_error(Ug) <= 1e-6
    assert q.sync_status() == q.OK


@pytest.mark.parametrize("mode", EXPM_MODES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d", [20, 45, 200])
def test_expm_chunked_alias_and_nonfinite(d, dtype, mode):
    # d <= 32 runs the fused one-workgroup kernel, larger d the batched path
    kw = expm_mode(mode, dtype)
    if kw is None:
        pytest.skip("the FP64 path takes no refinement")
    refine = kw["unitary_refine"]
    say(f"expm chunking d={d} {dtype} {mode}")
    B = 7
    Om = wl.random_skew_hermitian_batch(B, d, np.linspace(0.5, 300, B), config_id=77)
    om = gpu(Om).to(dtype)
    U1, s1 = q.expm_batched(om, **kw)                        # one chunk
    U2, s2 = q.expm_batched(om, chunk=3, **kw)               # chunks of 3, 3, 1
    om3 = om.clone()
    U3, s3 = q.expm_batched(om3, U=None if kw.get("out_c128") else om3, chunk=2, **kw)   # in place
    torch.cuda.synchronize()
    assert torch.equal(U1, U2) and torch.equal(U1, U3)
    assert torch.equal(s1, s2) and torch.equal(s1, s3)
    if refine:
        ref = oracle.expm_skew_hermitian(Om)
        inf = np.abs(oracle.propagator_infidelity(ref, host(U1).astype(np.complex128)))
        assert np.all(inf <= 1e-6), inf
    bad = om.clone()
    bad[2, 3, 4] = float("nan")
    U4, s4 = q.expm_batched(bad, **kw)
    torch.cuda.synchronize()
    assert int(s4[2]) == -1 and torch.isnan(U4[2]).all()
    keep = [0, 1, 3, 4, 5, 6]
    assert torch.equal(U4[keep], U1[keep])


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d", [33, 129, 300])
def test_expm_skew_matches_general(d, dtype):
    # the structured products are the general ones up to rounding; with one
    # tile (d = 33 on the FP32 128 tile) and several (129, 300, ragged)
    say(f"expm skew vs general d={d} {dtype}")
    norms = [0.7, 6.0, 45.0, 400.0]
    Om = wl.random_skew_hermitian_batch(len(norms), d, norms, config_id=900 + d)
    om = gpu(Om).to(dtype)
    Ug, sg = q.expm_batched(om)
    Us, ss = q.expm_batched(om, skew_hermitian=True)
    torch.cuda.synchronize()
    assert torch.equal(sg, ss)
    a, b = host(Ug).astype(np.complex128), host(Us).astype(np.complex128)
    inf = np.abs(oracle.propagator_infidelity(a, b))
    assert np.all(inf <= 2 * inf_tol(dtype, host(ss), refined=False)), inf


@pytest.mark.parametrize("dtype,refine,out_c128", [(torch.complex128, False, False), (torch.complex64, False, False),
                                                   (torch.complex64, True, False), (torch.complex64, True, True)])
def test_expm_squaring_bound(dtype, refine, out_c128):
    # a bound at or above every exponent changes no bit; items above a smaller
    # bound come back with s = -2 and NaN, the others unchanged
    d = 70
    norms = [0.5, 20.0, 300.0, 6000.0]       # s = 0, 2, 6, 11
    Om = wl.random_skew_hermitian_batch(len(norms), d, norms, config_id=950)
    om = gpu(Om).to(dtype)
    say(f"expm squaring bound {dtype} refine={refine} out_c128={out_c128}")
    kw = dict(skew_hermitian=True, unitary_refine=refine, out_c128=out_c128)
    U0, s0 = q.expm_batched(om, **kw)
    U1, s1 = q.expm_batched(om, squaring_bound=int(s0.max()), **kw)
    U2, s2 = q.expm_batched(om, squaring_bound=20, **kw)
    U3, s3 = q.expm_batched(om, squaring_bound=5, chunk=3, **kw)
    torch.cuda.synchronize()
    assert host(s0).tolist() == [0, 2, 6, 11]
    assert torch.equal(U0, U1) and torch.equal(U0, U2) and torch.equal(s0, s1) and torch.equal(s0, s2)
    assert host(s3).tolist() == [0, 2, -2, -2]
    assert torch.equal(U3[:2], U0[:2]) and torch.isnan(U3[2:]).all()


@pytest.mark.parametrize("refine", [False, True])
def test_expm_capture_needs_a_bound(refine):
    dtype = torch.complex64
    om = gpu(wl.random_skew_hermitian_batch(2, 50, 10.0, config_id=951)).to(dtype)
    U = torch.empty(om.shape, dtype=torch.complex128 if refine else dtype, device=DEV)
    s = torch.empty(2, dtype=torch.int32, device=DEV)
    ws = torch.empty(q.workspace_bytes(q.FN_EXPM, 2, 50, 1, 1, q.C64), dtype=torch.uint8, device=DEV)
    kw = dict(skew_hermitian=True, unitary_refine=refine, out_c128=refine)
    q.expm_batched(om, U=U, s_out=s, ws=ws, **kw)      # tunes the tile outside capture
    torch.cuda.synchronize()
    ref = U.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            with pytest.raises(q.QcheffError):
                q.expm_batched(om, U=U, s_out=s, ws=ws, **kw)
            q.expm_batched(om, U=U, s_out=s, ws=ws, squaring_bound=8, **kw)
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(3):
        U.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(U, ref)


# -------------------------------------------------------------------- chain

@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("M,d", [(0, 5), (1, 5), (2, 17), (5, 33), (17, 64), (40, 130)])
def test_propagate_parity(M, d, dtype):
    say(f"propagate M={M} d={d} {dtype}")
    Om = wl.random_skew_hermitian_batch(max(M, 1), d, 3.0, config_id=500 + M)[:M]
    Uo = oracle.expm_skew_hermitian(Om) if M else np.zeros((0, d, d), complex)
    Ud = gpu(Uo).to(dtype)
    Uref = host(Ud).astype(np.complex128)       # what the GPU sees (rounded for FP32)
    psi0 = wl.random_state(d, 7)
    psi = gpu(psi0)
    traj = torch.empty((M + 1, d), dtype=torch.complex128, device=DEV)
    q.propagate(Ud, q.STATE, psi, traj=traj)
    P = torch.empty((d, d), dtype=dtype, device=DEV)
    q.propagate(Ud, q.PRODUCT, P)
    torch.cuda.synchronize()
    psi_o, traj_o = oracle.propagate_state(Uref, psi0, trajectory=True)
    tol = 1e-13 * max(M, 1) * math.sqrt(d)
    assert np.abs(host(psi) - psi_o).max() <= tol
    assert np.abs(host(traj) - traj_o).max() <= tol
    P_o = oracle.propagate_product(Uref)
    ptol = tol if dtype == torch.complex128 else 1e-6 * max(M, 1) * math.sqrt(d)
    assert np.abs(host(P).astype(np.complex128) - P_o).max() <= ptol


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d", [1000, 1030, 2100, 4100])
def test_propagate_state_row_widths(d, dtype):
    # the state chain takes 64 to 512 threads per row by the row's 16-byte piece
    # count (complex64 with an odd d: one element per lane); a few intervals at
    # each width, with a ragged last round of pieces, against the oracle's chain
    M = 3
    say(f"propagate state M={M} d={d} {dtype}")
    g = np.random.default_rng(d)
    Uo = (g.standard_normal((M, d, d)) + 1j * g.standard_normal((M, d, d))) / math.sqrt(2 * d)
    Ud = gpu(Uo).to(dtype)
    Uref = host(Ud).astype(np.complex128)
    psi0 = wl.random_state(d, 11)
    psi = gpu(psi0)
    q.propagate(Ud, q.STATE, psi)
    torch.cuda.synchronize()
    psi_o = oracle.propagate_state(Uref, psi0)
    assert np.abs(host(psi) - psi_o).max() <= 1e-13 * M * math.sqrt(d)


# --------------------------------------------------------------- end to end

def _evolve(w, dtype, chunk=None):
    return q.evolve(gpu(w.H0), gpu(w.Hk), gpu(w.u), w.dt_sample, w.M, w.order, psi0=gpu(w.psi0), dtype=dtype,
                    product=True, trajectory=True, chunk=chunk)


@pytest.mark.parametrize("order", [1, 2])
def test_transmon_duffing_d8_end_to_end(order):
    # the single-transmon job (d = 8, 1e4 samples, M = 100), complex128
    say(f"transmon d8 order={order}")
    w = wl.transmon_duffing(order=order)
    ref = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, order, psi0=w.psi0, product=True)
    out = _evolve(w, torch.complex128)
    torch.cuda.synchronize()
    U = host(out["U"])
    assert np.all(oracle.propagator_infidelity(ref["U"], U) <= 1e-12)
    assert np.abs(U - ref["U"]).max() <= 1e-10
    assert oracle.state_infidelity(ref["psi"], host(out["psi"])) <= 1e-12
    assert np.abs(host(out["traj"]) - ref["traj"]).max() <= 1e-10
    assert oracle.propagator_infidelity(ref["P"], host(out["P"])) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_random_system_order2_end_to_end(dtype):
    say(f"random system order 2 {dtype}")
    w = wl.random_system(48, 3, 40 * 15, 40, 2, config_id=88, drift_scale=30.0, drive_scale=5.0)
    ref = oracle.run(w.H0, w.Hk, w.u, w.dt_sample, w.M, 2, psi0=w.psi0, product=True)
    out = _evolve(w, dtype, chunk=16)          # complex64: refined to unitarity
    torch.cuda.synchronize()
    U = host(out["U"]).astype(np.complex128)
    tol = INF_TOL[dtype]
    inf = np.abs(oracle.propagator_infidelity(ref["U"], U))
    psi = host(out["psi"])
    sinf = abs(oracle.state_infidelity(ref["psi"], psi))
    say(f"  max U_n infidelity {inf.max():.2e}, state {sinf:.2e}, |psi| - 1 {oracle.norm_error(psi):.2e}")
    assert np.all(inf <= tol)
    assert sinf <= tol
    assert oracle.norm_error(psi) <= (1e-12 if dtype == torch.complex128 else 1e-6)
    traj = host(out["traj"])
    assert max(abs(oracle.state_infidelity(a, b)) for a, b in zip(ref["traj"], traj)) <= tol
    # The product is formed by a tree of FP32 products (log2 M levels, each
    # rounding to FP32 with FP32 accumulation over d terms): its direction is held
    # to the target and its distance from unitarity to a few roundings per level.
    P = host(out["P"]).astype(np.complex128)
    assert oracle.propagator_infidelity(ref["P"], P, normalized=True) <= tol
    ubound = 1e-12 if dtype == torch.complex128 else math.ceil(math.log2(w.M)) * math.sqrt(w.d) * 4 * U32
    assert oracle.unitarity_error(P) <= ubound


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("B,M,d", [(1, 1, 3), (5, 7, 3), (4, 9, 64), (3, 5, 130)])
def test_propagate_batched_parity(B, M, d, dtype):
    say(f"propagate_batched B={B} M={M} d={d} {dtype}")
    Om = wl.random_skew_hermitian_batch(B * M, d, 2.0, config_id=900 + d)
    Uo = oracle.expm_skew_hermitian(Om).reshape(B, M, d, d)
    Ud = gpu(Uo).to(dtype)
    Uref = host(Ud).astype(np.complex128)
    psi0 = np.stack([wl.random_state(d, 40 + b) for b in range(B)])
    x = gpu(psi0)
    q.propagate_batched(Ud, x)
    torch.cuda.synchronize()
    for b in range(B):
        ref = oracle.propagate_state(Uref[b], psi0[b])
        assert np.abs(host(x)[b] - ref).max() <= 1e-13 * M * math.sqrt(d)


def test_unitary_refine_needs_complex64_skew():
    om = gpu(wl.random_skew_hermitian_batch(2, 40, 3.0, config_id=12))
    with pytest.raises(q.QcheffError) as e:
        q.expm_batched(om, skew_hermitian=True, unitary_refine=True)          # complex128
    assert e.value.status == q.EINVAL
    with pytest.raises(q.QcheffError) as e:
        q.expm_batched(om.to(torch.complex64), unitary_refine=True)           # not declared skew-Hermitian
    assert e.value.status == q.EINVAL
    om32 = om.to(torch.complex64)
    with pytest.raises(q.QcheffError) as e:                                   # FP64 output needs the refinement
        q.expm_batched(om32, skew_hermitian=True, out_c128=True)
    assert e.value.status == q.EINVAL
    with pytest.raises(q.QcheffError) as e:                                   # a complex128 U on omega itself
        q.expm_batched(om32, U=om32, skew_hermitian=True, unitary_refine=True, out_c128=True)
    assert e.value.status == q.EINVAL


def test_sync_status_reports_nonfinite_generators():
    # a NaN generator: the exponential marks it (s = -1, U NaN) and the device
    # status word reports it once; a zero column pivot is reported the same way
    q.sync_status()                                   # clear anything earlier tests left
    for d in (8, 48):
        om = torch.from_numpy(wl.random_skew_hermitian_batch(3, d, 2.0, config_id=d)).to(DEV)
        om[1, 0, 0] = float("nan")
        U, s = q.expm_batched(om, skew_hermitian=True)
        assert s.cpu().tolist()[1] == -1 and torch.isnan(U[1]).all()
        assert q.sync_status() == q.ENONFINITE
        assert q.sync_status() == q.OK
        U, s = q.expm_batched(om[::2].contiguous(), skew_hermitian=True)
        assert q.sync_status() == q.OK
    # the state-only path flags a non-finite generator from the host
    om = torch.from_numpy(wl.random_skew_hermitian_batch(2, 40, 2.0, config_id=3)).to(DEV)
    om[0, 1, 2] = float("inf")
    x = torch.from_numpy(wl.random_state(40, 4)).to(DEV)
    q.propagate_action(om, x)
    assert q.sync_status() == q.ENONFINITE and q.sync_status() == q.OK
