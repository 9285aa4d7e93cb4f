"""Seeded synthetic inputs for the Magnus time-evolution path.

This module only *builds inputs*: drift and control operators (H0, H_k) of the
systems the paper and its benchmarks describe, control signals sampled on a
time grid, initial states, and random matrices for the exponential.  It holds
none of the method's arithmetic (no coefficients, no commutators, no
exponentials).  Both the oracle-side tests and the HIP path consume what it
returns; neither side imports the other.

Conventions
-----------
* hbar = 1; frequencies are angular (rad/ns, written ``2*pi*GHz``), times in ns.
* The drive model is H(t) = H0 + sum_k u_k(t) H_k  (Sec. 4.1, Eq. magnus-generic-ham).
* Control signals are sampled as a zero-order hold: sample i holds on the cell
  [t0 + i*dt, t0 + (i+1)*dt) and is the signal's value at the cell midpoint
  t0 + (i + 1/2)*dt.
* ``u`` is float64 ``[K][N]``; operators are complex128 ``[d][d]`` (row-major).
* Every random draw comes from ``numpy.random.Generator(PCG64(241109982 + id))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

TWO_PI = 2.0 * math.pi
SEED_BASE = 241109982


def rng(config_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(config_id)))


@dataclass
class Workload:
    """One propagation job: H(t) = H0 + sum_k u[k](t) Hk[k] on N samples, M intervals."""
    name: str
    H0: np.ndarray          # complex128 [d][d], Hermitian
    Hk: np.ndarray          # complex128 [K][d][d], Hermitian
    u: np.ndarray           # float64 [K][N], zero-order-hold samples
    dt_sample: float        # cell width (ns)
    M: int                  # number of Magnus intervals, N % M == 0
    order: int              # Magnus order, 1 or 2
    psi0: np.ndarray        # complex128 [d], unit norm
    meta: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return self.H0.shape[0]

    @property
    def K(self) -> int:
        return self.Hk.shape[0]

    @property
    def N(self) -> int:
        return self.u.shape[1]

    @property
    def dt_interval(self) -> float:
        return self.dt_sample * (self.N // self.M)


# ---------------------------------------------------------------- operators

def destroy(n: int) -> np.ndarray:
    """Truncated bosonic lowering operator a on n levels (a|k> = sqrt(k)|k-1>)."""
    a = np.zeros((n, n), dtype=np.complex128)
    for k in range(1, n):
        a[k - 1, k] = math.sqrt(k)
    return a


def duffing(n: int, omega: float, alpha: float) -> np.ndarray:
    """Transmon as a Duffing oscillator: omega*n + (alpha/2)*n*(n-1), diagonal."""
    k = np.arange(n, dtype=np.float64)
    return np.diag(omega * k + 0.5 * alpha * k * (k - 1)).astype(np.complex128)


_SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def site_op(op: np.ndarray, site: int, dims: list[int]) -> np.ndarray:
    """Embed a single-site operator into the tensor product (site 0 is most significant)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for j, dj in enumerate(dims):
        out = np.kron(out, op if j == site else np.eye(dj, dtype=np.complex128))
    return out


def midpoints(n_samples: int, t_total: float, t0: float = 0.0) -> tuple[np.ndarray, float]:
    dt = t_total / n_samples
    return t0 + (np.arange(n_samples, dtype=np.float64) + 0.5) * dt, dt


def gaussian(t: np.ndarray, t_total: float, sigma: float) -> np.ndarray:
    return np.exp(-((t - 0.5 * t_total) ** 2) / (2.0 * sigma * sigma))


def basis_state(d: int, index: int = 0) -> np.ndarray:
    psi = np.zeros(d, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def random_state(d: int, config_id: int) -> np.ndarray:
    g = rng(config_id)
    psi = g.standard_normal(d) + 1j * g.standard_normal(d)
    return psi / np.linalg.norm(psi)


def random_hermitian(d: int, g: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    x = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
    return (scale * 0.5) * (x + x.conj().T)


def random_skew_hermitian_batch(batch: int, d: int, norms1, config_id: int) -> np.ndarray:
    """Batch of random skew-Hermitian matrices; item b is rescaled to 1-norm norms1[b].

    The 1-norm (max column sum of |entries|) is the quantity the scaling step of
    a scaling-and-squaring exponential looks at, so prescribing it sweeps the
    number of squarings.
    """
    g = rng(config_id)
    norms1 = np.broadcast_to(np.asarray(norms1, dtype=np.float64), (batch,))
    out = np.empty((batch, d, d), dtype=np.complex128)
    for b in range(batch):
        h = random_hermitian(d, g)
        w = -1j * h
        n1 = np.abs(w).sum(axis=0).max()
        out[b] = w * (norms1[b] / n1) if n1 > 0 else w
    return out


# ------------------------------------------------------------- workloads

def transmon_duffing(n_samples: int = 10_000, M: int = 100, order: int = 1) -> Workload:
    """Single transmon as a Duffing oscillator (d=8) with one Gaussian drive on a+a^dag.

    omega = 2pi*5 GHz, alpha = -2pi*0.3 GHz, A = 2pi*0.05 GHz, T = 50 ns, sigma = 10 ns,
    carrier at omega.  Default: 1e4 samples, M = 100, first order.
    """
    d = 8
    omega, alpha = TWO_PI * 5.0, -TWO_PI * 0.3
    amp, t_total, sigma = TWO_PI * 0.05, 50.0, 10.0
    a = destroy(d)
    H0 = duffing(d, omega, alpha)
    Hk = (a + a.conj().T)[None]
    t, dt = midpoints(n_samples, t_total)
    u = (amp * gaussian(t, t_total, sigma) * np.cos(omega * t))[None]
    return Workload("transmon_duffing_d8", H0, Hk, np.ascontiguousarray(u), dt, M, order,
                    basis_state(d, 0),
                    dict(omega=omega, alpha=alpha, amp=amp, T=t_total, sigma=sigma))


def transmon_resonator(n_samples: int = 100_000, M: int = 1000, order: int = 2,
                       n_transmon: int = 10, n_resonator: int = 100) -> Workload:
    """Transmon (10 levels) x resonator (100 levels), d = 1000, exchange coupling.

    H0 = H_duffing (x) I + omega_r I (x) a^dag a + g (b (x) a^dag + b^dag (x) a),
    g = 2pi*0.1 GHz, omega_r = 2pi*7 GHz.  Drives: (b + b^dag) (x) I at the transmon
    frequency and I (x) (a + a^dag) at the resonator frequency, Gaussian envelopes
    (T = 50 ns, sigma = 10 ns), amplitudes drawn from U[0.01, 0.1]*2pi GHz.
    Basis index = i_transmon * n_resonator + i_resonator.
    """
    g_rng = rng(2)
    omega_q, alpha, omega_r, gc = TWO_PI * 5.0, -TWO_PI * 0.3, TWO_PI * 7.0, TWO_PI * 0.1
    t_total, sigma = 50.0, 10.0
    dims = [n_transmon, n_resonator]
    b = destroy(n_transmon)
    a = destroy(n_resonator)
    B = site_op(b, 0, dims)
    A = site_op(a, 1, dims)
    H0 = (site_op(duffing(n_transmon, omega_q, alpha), 0, dims)
          + omega_r * (A.conj().T @ A)
          + gc * (B @ A.conj().T + B.conj().T @ A))
    Hk = np.stack([B + B.conj().T, A + A.conj().T])
    amps = TWO_PI * g_rng.uniform(0.01, 0.1, size=2)
    t, dt = midpoints(n_samples, t_total)
    env = gaussian(t, t_total, sigma)
    u = np.stack([amps[0] * env * np.cos(omega_q * t), amps[1] * env * np.cos(omega_r * t)])
    return Workload(f"transmon{n_transmon}x resonator{n_resonator}".replace(" ", "_"),
                    H0, Hk, u, dt, M, order, basis_state(n_transmon * n_resonator, 0),
                    dict(omega_q=omega_q, alpha=alpha, omega_r=omega_r, g=gc, amps=amps.tolist(),
                         T=t_total, sigma=sigma))


def spin_chain(n_spins: int = 10, n_samples: int = 10_000, M: int = 200, order: int = 2,
               config_id: int = 6) -> Workload:
    """Degenerate periodic spin chain of Sec. 4.3 (Eqs. for the drift and control terms).

    H_d = 1/2 sum_j w sz_j - J sum_j sz_j sz_{j+1} - g sum_j sz_j sz_{j+2} (periodic),
    controls H_x = sum_j sx_j, H_y = sum_j sy_j with u_x = A env cos(2 pi f t),
    u_y = A env sin(2 pi f t), f ~ U[0, 10] GHz (seeded), Gaussian env sigma = T/5,
    T = 25 ns.  w = 2pi*5, J = 2pi*0.05, g = 2pi*0.02, A = 2pi*0.05 GHz (the paper
    publishes symbols only; these values are chosen here).  psi0 = |0...0>.
    """
    g_rng = rng(config_id)
    w, J, gnn, amp, t_total = TWO_PI * 5.0, TWO_PI * 0.05, TWO_PI * 0.02, TWO_PI * 0.05, 25.0
    dims = [2] * n_spins
    d = 2 ** n_spins
    # sz is diagonal: build the drift from bit patterns directly
    idx = np.arange(d)
    z = np.empty((n_spins, d))
    for j in range(n_spins):
        z[j] = 1.0 - 2.0 * ((idx >> (n_spins - 1 - j)) & 1)
    diag = 0.5 * w * z.sum(axis=0)
    for j in range(n_spins):
        diag -= J * z[j] * z[(j + 1) % n_spins]
        diag -= gnn * z[j] * z[(j + 2) % n_spins]
    H0 = np.diag(diag).astype(np.complex128)
    Hx = np.zeros((d, d), dtype=np.complex128)
    Hy = np.zeros((d, d), dtype=np.complex128)
    for j in range(n_spins):
        bit = 1 << (n_spins - 1 - j)
        flipped = idx ^ bit
        Hx[flipped, idx] += 1.0
        # sy|0> = i|1>, sy|1> = -i|0>; |0> has the bit clear (sz = +1)
        Hy[flipped, idx] += np.where((idx & bit) == 0, 1j, -1j)
    f = g_rng.uniform(0.0, 10.0)
    t, dt = midpoints(n_samples, t_total)
    env = gaussian(t, t_total, t_total / 5.0)
    u = np.stack([amp * env * np.cos(TWO_PI * f * t), amp * env * np.sin(TWO_PI * f * t)])
    return Workload(f"spin_chain_{n_spins}", H0, np.stack([Hx, Hy]), u, dt, M, order,
                    basis_state(d, 0), dict(w=w, J=J, g=gnn, amp=amp, f=f, T=t_total, dims=dims))


def coupled_transmons(n_transmons: int = 4, levels: int = 8, n_samples: int = 100_000,
                      M: int = 2000, order: int = 2, config_id: int = 5) -> Workload:
    """Chain of Duffing transmons with nearest-neighbour x x coupling (2pi*0.02 GHz).

    omega_j ~ U[4.8, 5.2]*2pi, alpha = -2pi*0.3; one drive per transmon on x_j = b_j + b_j^dag
    with a seeded random phase; T = 50 ns, sigma = 10 ns; psi0 is a seeded random state.
    """
    g_rng = rng(config_id)
    dims = [levels] * n_transmons
    d = levels ** n_transmons
    omegas = TWO_PI * g_rng.uniform(4.8, 5.2, size=n_transmons)
    phases = g_rng.uniform(0.0, TWO_PI, size=n_transmons)
    amps = TWO_PI * g_rng.uniform(0.01, 0.1, size=n_transmons)
    b = destroy(levels)
    x = b + b.conj().T
    H0 = np.zeros((d, d), dtype=np.complex128)
    X = [site_op(x, j, dims) for j in range(n_transmons)]
    for j in range(n_transmons):
        H0 += site_op(duffing(levels, omegas[j], -TWO_PI * 0.3), j, dims)
    for j in range(n_transmons - 1):
        H0 += TWO_PI * 0.02 * (X[j] @ X[j + 1])
    t_total, sigma = 50.0, 10.0
    t, dt = midpoints(n_samples, t_total)
    env = gaussian(t, t_total, sigma)
    u = np.stack([amps[j] * env * np.cos(omegas[j] * t + phases[j]) for j in range(n_transmons)])
    return Workload(f"coupled_transmons_{n_transmons}x{levels}", H0, np.stack(X), u, dt, M, order,
                    random_state(d, 50 + config_id),
                    dict(omegas=omegas.tolist(), phases=phases.tolist(), amps=amps.tolist()))


def random_system(d: int, K: int, n_samples: int, M: int, order: int, config_id: int,
                  drift_scale: float = 1.0, drive_scale: float = 1.0, t_total: float = 10.0) -> Workload:
    """Dense random Hermitian H0, H_k and smooth random multi-tone signals (tests)."""
    g_rng = rng(config_id)
    H0 = random_hermitian(d, g_rng, drift_scale / math.sqrt(d))
    Hk = np.stack([random_hermitian(d, g_rng, drive_scale / math.sqrt(d)) for _ in range(K)])
    t, dt = midpoints(n_samples, t_total)
    u = np.empty((K, n_samples))
    for k in range(K):
        f = g_rng.uniform(0.1, 2.0, size=3)
        ph = g_rng.uniform(0, TWO_PI, size=3)
        a = g_rng.uniform(-1, 1, size=3)
        u[k] = sum(a[i] * np.cos(TWO_PI * f[i] * t + ph[i]) for i in range(3))
    return Workload(f"random_d{d}_K{K}", H0, Hk, u, dt, M, order, random_state(d, 100 + config_id),
                    dict(t_total=t_total))


def serving_request_system(d: int, M: int, order: int, g: np.random.Generator, samples_per_interval: int = 64,
                           t_total: float = 50.0) -> Workload:
    """One request of the serving stream: H0 = diag(2pi U[-1, 1]) + nearest-neighbour
    coupling 2pi*0.02 (tridiagonal), one drive H_1 = (a + a^dag)/sqrt(d) with a
    Gaussian envelope (sigma = T/5) on a carrier drawn from U[0.5, 1.5] GHz,
    amplitude 2pi U[0.01, 0.1] GHz; T = 50 ns, 64 samples per interval."""
    diag = TWO_PI * g.uniform(-1.0, 1.0, size=d)
    H0 = np.diag(diag).astype(np.complex128)
    off = np.full(d - 1, TWO_PI * 0.02)
    H0 += np.diag(off, 1) + np.diag(off, -1)
    a = destroy(d)
    Hk = ((a + a.conj().T) / math.sqrt(d))[None]
    N = M * samples_per_interval
    t, dt = midpoints(N, t_total)
    f = g.uniform(0.5, 1.5)
    amp = TWO_PI * g.uniform(0.01, 0.1)
    u = (amp * gaussian(t, t_total, t_total / 5.0) * np.cos(TWO_PI * f * t))[None]
    psi0 = np.zeros(d, dtype=np.complex128)
    psi0[0] = 1.0
    return Workload(f"serving_d{d}_M{M}", H0, Hk, np.ascontiguousarray(u), dt, M, order, psi0,
                    dict(f=f, amp=amp))


SWEEP_FACTORS = {16: (4, 2), 32: (2, 5), 64: (4, 3), 128: (2, 7), 256: (4, 4), 512: (8, 3)}


def transmon_chain(d: int, g: np.random.Generator, M: int = 256, samples_per_interval: int = 64,
                   order: int = 2, t_total: float = 50.0) -> Workload:
    """One instance of the batched sweep: a chain of Duffing transmons with
    nearest-neighbour exchange, d = levels**sites (16 = 4^2, 32 = 2^5, 64 = 4^3,
    128 = 2^7, 256 = 4^4, 512 = 8^3).  omega_j ~ U[4.5, 5.5]*2pi, alpha_j ~
    U[-0.35, -0.25]*2pi, J ~ U[0.01, 0.02]*2pi GHz; 1-3 drives (b_j + b_j^dag) on
    random sites with Gaussian envelopes (sigma = T/5) at the site frequency,
    random phase, amplitude U[0.01, 0.1]*2pi GHz; T = 50 ns, 64 samples per interval."""
    levels, sites = SWEEP_FACTORS[d]
    dims = [levels] * sites
    b = destroy(levels)
    omegas = TWO_PI * g.uniform(4.5, 5.5, size=sites)
    alphas = TWO_PI * g.uniform(-0.35, -0.25, size=sites)
    J = TWO_PI * g.uniform(0.01, 0.02)
    H0 = np.zeros((d, d), dtype=np.complex128)
    B = [site_op(b, j, dims) for j in range(sites)]
    for j in range(sites):
        H0 += site_op(duffing(levels, omegas[j], alphas[j]), j, dims)
    for j in range(sites - 1):
        X = B[j] @ B[j + 1].conj().T
        H0 += J * (X + X.conj().T)
    K = int(g.integers(1, 4))
    drive_sites = g.choice(sites, size=K, replace=True)
    N = M * samples_per_interval
    t, dt = midpoints(N, t_total)
    env = gaussian(t, t_total, t_total / 5.0)
    Hk = np.stack([B[j] + B[j].conj().T for j in drive_sites])
    u = np.stack([TWO_PI * g.uniform(0.01, 0.1) * env * np.cos(omegas[j] * t + g.uniform(0, TWO_PI))
                  for j in drive_sites])
    return Workload(f"transmon_chain_d{d}", H0, Hk, np.ascontiguousarray(u), dt, M, order, basis_state(d, 0),
                    dict(levels=levels, sites=sites, drive_sites=[int(x) for x in drive_sites]))


def sweep_instances(n: int = 512, M: int = 256, config_id: int = 3, dims=(16, 32, 64, 128, 256, 512)) -> list:
    """The batched sweep: n transmon-chain instances with d drawn uniformly from dims."""
    g = rng(config_id)
    return [transmon_chain(int(g.choice(dims)), g, M=M) for _ in range(n)]


# The bench / parity configurations, by name.
CONFIGS = {
    "transmon_duffing_d8": lambda: transmon_duffing(),
    "transmon10x_resonator100_d1000": lambda: transmon_resonator(),
    "spin_chain_10_d1024": lambda: spin_chain(),
}
