"""Oracle for the Magnus-expansion time-evolution path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or call this module; the product path never does.

A plain, slow, obviously-correct CPU implementation in NumPy complex128 /
float64.  It shares no code with the HIP library and imports nothing from this
repository.  Every function follows the paper (arXiv 2411.09982, Sec. 4.1) step
by step, with no blocking, fusion or reordering:

  coefficients   Eq. magnus-first-order-coeff (first order) and the double
                 integral of Eq. magnus-avg (second order), evaluated exactly for
                 a zero-order-hold signal;
  H-bar_n        Eq. magnus-first-order-term plus the second-order term of
                 Eq. magnus-avg with H(t) of Eq. magnus-generic-ham;
  propagator     U_n = exp(-i H-bar_n), by Hermitian eigendecomposition;
  chain          psi_n = U_n psi_{n-1}, P = U_M ... U_1 (stroboscopic, Sec. 4.1).

Readings of the paper this file takes (the paper is silent or garbled there):
  * sample i of u holds on [t0 + i dt, t0 + (i+1) dt) (zero-order hold), and the
    N samples split into M equal intervals of s = N / M samples;
  * the series is read per interval [t_n, t_n + Delta t] and truncated at order
    1, 2 or 3; the second-order term uses t2 < t1 and the prefactor -i/2; the
    third-order term (Eq. magnus-exp's H-bar^(3), "the pattern of nested
    commutators" the paper leaves unwritten) is the standard one, -(1/6) times the
    triple integral over t3 < t2 < t1 of [H1,[H2,H3]] + [H3,[H2,H1]];
  * U_n = exp(-i H-bar_n) with hbar = 1; the generator is Omega_n = -i H-bar_n;
  * later intervals multiply on the left.

Layout of the second-order coefficient table c2[M][K + K(K-1)/2]:
  columns 0..K-1        c20[n,k] weights the commutator [H0, H_k];
  column  K + p(k,l)    c2[n,(k,l)] weights [H_k, H_l] for k < l, with pairs in
                        row-major order (0,1), (0,2), ..., (0,K-1), (1,2), ...
"""
from __future__ import annotations

import math

import numpy as np

# Higham (2005), "The scaling and squaring method for the matrix exponential
# revisited", Table 2.3: largest 1-norm for which the [13/13] Pade approximant
# reaches double-precision backward error (u = 2^-53).
THETA13_F64 = 5.371920351148152



# ------------------------------------------------------------------ checks

def check_inputs(H0, Hk, u, M, hermitian_tol=1e-12):
    """Validate shapes, finiteness, Hermiticity and N % M == 0; raise ValueError."""
    H0 = np.asarray(H0)
    Hk = np.asarray(Hk)
    u = np.asarray(u)
    if H0.ndim != 2 or H0.shape[0] != H0.shape[1]:
        raise ValueError("H0 must be square")
    d = H0.shape[0]
    if Hk.ndim != 3 or Hk.shape[1:] != (d, d):
        raise ValueError("Hk must be [K][d][d]")
    if u.ndim != 2 or u.shape[0] != Hk.shape[0]:
        raise ValueError("u must be [K][N]")
    if np.iscomplexobj(u) or not np.all(np.isfinite(u)):
        raise ValueError("u must be real and finite")
    N = u.shape[1]
    if M <= 0 or N % M != 0:
        raise ValueError("N must be a positive multiple of M")
    for H in [H0, *Hk]:
        scale = max(np.abs(H).max(), 1e-300)
        if np.abs(H - H.conj().T).max() > hermitian_tol * scale:
            raise ValueError("operators must be Hermitian")


def pair_index(k: int, l: int, K: int) -> int:
    """Column of the (k, l), k < l, commutator coefficient in the c2 table."""
    assert 0 <= k < l < K
    return K + k * K - k * (k + 1) // 2 + (l - k - 1)


# ------------------------------------------------------------ coefficients

def interval_coefficients(u, dt_sample, M, order):
    """Per-interval Magnus coefficients of a zero-order-hold control signal.

    First order (Eq. magnus-first-order-coeff): c1[n,k] is the integral of u_k
    over interval n, i.e. dt * sum of its s samples.

    Second order (Eq. magnus-avg, second line, with H of Eq. magnus-generic-ham):
    the commutator [H(t1), H(t2)] expands into
        sum_k (u_k(t2) - u_k(t1)) [H0, H_k]
      + sum_{k<l} (u_k(t1) u_l(t2) - u_l(t1) u_k(t2)) [H_k, H_l],
    and the double integral over t2 < t1 inside the interval is exact for a
    piecewise-constant signal:
        c20[n,k]   = dt^2 * sum_j (s - 1 - 2 j) u_k[j]
        c2[n,(kl)] = dt^2 * sum_j sum_{i<j} (u_k[j] u_l[i] - u_l[j] u_k[i])
    (j indexes the samples of the interval; same-cell pairs cancel).
    """
    u = np.asarray(u, dtype=np.float64)
    K, N = u.shape
    s = N // M
    dt = float(dt_sample)
    c1 = np.empty((M, K))
    c2 = np.zeros((M, K + K * (K - 1) // 2)) if order == 2 else None
    w = (s - 1 - 2 * np.arange(s)).astype(np.float64)
    for n in range(M):
        seg = u[:, n * s:(n + 1) * s]
        for k in range(K):
            c1[n, k] = dt * math.fsum(seg[k])
        if order == 2:
            for k in range(K):
                c2[n, k] = dt * dt * math.fsum(w * seg[k])
            # exclusive prefix sums P_k[j] = sum_{i<j} u_k[i]
            P = np.zeros_like(seg)
            P[:, 1:] = np.cumsum(seg[:, :-1], axis=1)
            for k in range(K):
                for l in range(k + 1, K):
                    c2[n, pair_index(k, l, K)] = dt * dt * math.fsum(
                        np.concatenate([seg[k] * P[l], -(seg[l] * P[k])]))
    return c1, c2


# -------------------------------------------------------- effective H-bar

def commutator(A, B):
    return A @ B - B @ A


def effective_hamiltonians(H0, Hk, c1, c2, dt_interval, order):
    """H-bar_n for every interval (Eq. magnus-first-order-term; Eq. magnus-avg).

    H-bar_n = Delta t H0 + sum_k c1[n,k] H_k
            - (i/2) (sum_k c20[n,k] [H0,H_k] + sum_{k<l} c2[n,(kl)] [H_k,H_l])   (order 2)
    """
    H0 = np.asarray(H0, dtype=np.complex128)
    Hk = np.asarray(Hk, dtype=np.complex128)
    K, d = Hk.shape[0], H0.shape[0]
    M = c1.shape[0]
    comms = []
    if order == 2:
        comms = [(k, commutator(H0, Hk[k])) for k in range(K)]
        comms += [(pair_index(k, l, K), commutator(Hk[k], Hk[l]))
                  for k in range(K) for l in range(k + 1, K)]
    out = np.empty((M, d, d), dtype=np.complex128)
    for n in range(M):
        H = dt_interval * H0
        for k in range(K):
            H = H + c1[n, k] * Hk[k]
        if order == 2:
            S = np.zeros((d, d), dtype=np.complex128)
            for col, C in comms:
                S = S + c2[n, col] * C
            H = H - 0.5j * S
        out[n] = 0.5 * (H + H.conj().T)
    return out


def generators(H0, Hk, c1, c2, dt_interval, order):
    """Omega_n = -i H-bar_n (skew-Hermitian), so that U_n = exp(Omega_n)."""
    return -1j * effective_hamiltonians(H0, Hk, c1, c2, dt_interval, order)


# ------------------------------------------------------- third-order term

def third_order_coefficients(u, dt_sample, M):
    """T[n, a, b, c] = int_{t3 < t2 < t1 in interval n} x_a(t1) x_b(t2) x_c(t3) for the
    zero-order-hold signals x_0 = 1 (the drift) and x_k = u_{k-1}.

    Cells i (of t1), j (of t2), k (of t3) contribute the volume of the simplex
    t3 < t2 < t1 inside their product, in units of dt^3: 1 for i > j > k, 1/2 for
    i = j > k or i > j = k, 1/6 for i = j = k.  Summed with exclusive prefix sums
    C_c[j] = sum_{k<j} x_c[k], Q[i] = sum_{j<i} x_b[j] C_c[j], R[i] = sum_{j<i} x_b[j] x_c[j]:
        T / dt^3 = sum_i x_a[i] (Q[i] + x_b[i] C_c[i] / 2 + R[i] / 2 + x_b[i] x_c[i] / 6).
    """
    u = np.asarray(u, dtype=np.float64)
    K, N = u.shape
    s = N // M
    dt = float(dt_sample)
    x = np.vstack([np.ones(N), u])
    T = np.empty((M, K + 1, K + 1, K + 1))
    for n in range(M):
        seg = x[:, n * s:(n + 1) * s]
        for a in range(K + 1):
            for b in range(K + 1):
                for c in range(K + 1):
                    Cc = np.concatenate([[0.0], np.cumsum(seg[c])[:-1]])
                    bc = seg[b] * Cc
                    Q = np.concatenate([[0.0], np.cumsum(bc)[:-1]])
                    bb = seg[b] * seg[c]
                    R = np.concatenate([[0.0], np.cumsum(bb)[:-1]])
                    T[n, a, b, c] = dt ** 3 * math.fsum(seg[a] * (Q + 0.5 * bc + 0.5 * R + bb / 6.0))
    return T


def third_order_term(H0, Hk, T):
    """H-bar^(3)_n, the third-order term of Eq. magnus-exp for H(t) of
    Eq. magnus-generic-ham: with A = -i H, Omega_3 = (1/6) int_{t3<t2<t1}
    ([A1, [A2, A3]] + [A3, [A2, A1]]), so
        H-bar^(3)_n = i Omega_3 = -(1/6) sum_{a,b,c} T[n,a,b,c] ([H_a, [H_b, H_c]] + [H_c, [H_b, H_a]])
    with H_0 the drift and H_{k+1} = Hk[k]."""
    H = [np.asarray(H0, dtype=np.complex128)] + [np.asarray(h, dtype=np.complex128) for h in Hk]
    nb = len(H)
    M = T.shape[0]
    d = H[0].shape[0]
    nested = {}
    for a in range(nb):
        for b in range(nb):
            for c in range(nb):
                nested[a, b, c] = (commutator(H[a], commutator(H[b], H[c]))
                                   + commutator(H[c], commutator(H[b], H[a])))
    out = np.zeros((M, d, d), dtype=np.complex128)
    for n in range(M):
        for (a, b, c), C in nested.items():
            out[n] = out[n] - (T[n, a, b, c] / 6.0) * C
    return out


# ------------------------------------------------------------- exponential

def propagator_from_hamiltonian(Hbar):
    """U = exp(-i H-bar) = V diag(exp(-i lambda)) V^dag from eigh of the Hermitian H-bar."""
    Hbar = np.asarray(Hbar, dtype=np.complex128)
    if Hbar.ndim == 2:
        lam, V = np.linalg.eigh(Hbar)
        return (V * np.exp(-1j * lam)) @ V.conj().T
    return np.stack([propagator_from_hamiltonian(h) for h in Hbar])


def expm_skew_hermitian(Omega):
    """exp(Omega) for skew-Hermitian Omega, via eigh of i*Omega (which is Hermitian)."""
    Omega = np.asarray(Omega, dtype=np.complex128)
    H = 1j * Omega
    H = 0.5 * (H + np.conj(np.swapaxes(H, -1, -2)))
    return propagator_from_hamiltonian(H)


def norm1(A):
    """Matrix 1-norm: largest column sum of absolute values."""
    return float(np.abs(np.asarray(A)).sum(axis=-2).max())


def trace_shift(Omega):
    """mu = tr(Omega) / d, the multiple of I that scaling and squaring splits off:
    exp(Omega) = e^mu exp(Omega - mu I), because mu I commutes with Omega."""
    Omega = np.asarray(Omega, dtype=np.complex128)
    return complex(np.trace(Omega)) / Omega.shape[-1]


def scaling_exponent(Omega, theta=THETA13_F64, shift=True):
    """Number of squarings s of the [13/13] scaling-and-squaring method (Higham 2005)
    applied to Omega - mu I (trace reduction, mu = trace_shift(Omega); shift=False
    takes Omega itself): the smallest s >= 0 with ||Omega - mu I||_1 / 2^s <= theta_13
    (that is, max(0, ceil(log2(||.||_1 / theta_13)))), decided by exact float64
    comparisons against theta_13 * 2^s; -1 for a non-finite norm."""
    Omega = np.asarray(Omega, dtype=np.complex128)
    if shift:
        mu = trace_shift(Omega)
        if not (math.isfinite(mu.real) and math.isfinite(mu.imag)):
            return -1
        Omega = Omega - mu * np.eye(Omega.shape[-1])
    nrm = norm1(Omega)
    if not math.isfinite(nrm):
        return -1
    s = 0
    while nrm > math.ldexp(theta, s):
        s += 1
    return s


# -------------------------------------------------------------------- chain

def propagate_state(U, psi0, trajectory=False):
    """Stroboscopic state chain psi_n = U_n psi_{n-1}, n = 1..M."""
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    traj = [psi.copy()]
    for Un in U:
        psi = Un @ psi
        traj.append(psi.copy())
    return (psi, np.stack(traj)) if trajectory else psi


def propagate_product(U):
    """P = U_M ... U_2 U_1 (later intervals on the left)."""
    d = U.shape[-1]
    P = np.eye(d, dtype=np.complex128)
    for Un in U:
        P = Un @ P
    return P


# ------------------------------------------------------------------ metrics

def propagator_infidelity(U_ref, U, normalized=False):
    """1 - |tr(U_ref^dag U)|^2 / d^2 (global-phase insensitive).

    normalized=True divides by tr(U_ref^dag U_ref) tr(U^dag U) instead of d^2:
    equal for unitary operands, and for a finite-precision product whose norm
    has drifted it compares the operator's direction only (like a state's ray);
    its distance from unitarity is judged on its own (unitarity_error).
    """
    U_ref = np.asarray(U_ref, dtype=np.complex128)
    U = np.asarray(U, dtype=np.complex128)
    d = U.shape[-1]
    tr = np.einsum("...ij,...ij->...", U_ref.conj(), U)
    if normalized:
        na = np.einsum("...ij,...ij->...", U_ref.conj(), U_ref).real
        nb = np.einsum("...ij,...ij->...", U.conj(), U).real
        return 1.0 - np.abs(tr) ** 2 / (na * nb)
    return 1.0 - np.abs(tr) ** 2 / (d * d)


def state_infidelity(psi_ref, psi):
    """1 - |<psi_ref|psi>|^2, the final-state error of Sec. 4.3, as written there:
    the overlap of the two vectors as they are, with no normalisation, so that a
    state whose norm has drifted off 1 counts as wrong (the exact evolution is
    unitary).  It is negative when |<psi_ref|psi>| exceeds 1."""
    a, b = np.asarray(psi_ref), np.asarray(psi)
    return 1.0 - abs(np.vdot(a, b)) ** 2


def direction_infidelity(psi_ref, psi):
    """1 - |<psi_ref|psi>|^2 / (<psi_ref|psi_ref> <psi|psi>): the error of the
    state's direction alone (a pure state is a ray); with norm_error it splits the
    state error into its two parts."""
    a, b = np.asarray(psi_ref), np.asarray(psi)
    na, nb = np.vdot(a, a).real, np.vdot(b, b).real
    return 1.0 - abs(np.vdot(a, b)) ** 2 / (na * nb)


def norm_error(psi):
    """| ||psi|| - 1 |: the evolution is unitary, so every exact state has norm 1."""
    return abs(float(np.linalg.norm(np.asarray(psi))) - 1.0)


def unitarity_error(U):
    U = np.asarray(U, dtype=np.complex128)
    d = U.shape[-1]
    G = np.conj(np.swapaxes(U, -1, -2)) @ U
    return float(np.abs(G - np.eye(d)).max())


# --------------------------------------------------------------------- job

def run(H0, Hk, u, dt_sample, M, order, psi0=None, product=False, check=True):
    """The whole path on the CPU: coefficients -> Omega_n -> U_n -> chain.  Order 3
    adds the third-order term (third_order_term) to the second-order H-bar_n."""
    if check:
        check_inputs(H0, Hk, u, M)
    N = np.asarray(u).shape[1]
    dt_interval = dt_sample * (N // M)
    c1, c2 = interval_coefficients(u, dt_sample, M, min(order, 2))
    Hbar = effective_hamiltonians(H0, Hk, c1, c2, dt_interval, min(order, 2))
    T = None
    if order == 3:
        T = third_order_coefficients(u, dt_sample, M)
        Hbar = Hbar + third_order_term(H0, Hk, T)
        Hbar = 0.5 * (Hbar + np.conj(np.swapaxes(Hbar, -1, -2)))
    U = propagator_from_hamiltonian(Hbar)
    out = dict(c1=c1, c2=c2, T=T, Hbar=Hbar, Omega=-1j * Hbar, U=U)
    if psi0 is not None:
        out["psi"], out["traj"] = propagate_state(U, psi0, trajectory=True)
    if product:
        out["P"] = propagate_product(U)
    return out
