"""Pins for the NPAD oracle (oracle/npad.py): each check ties it to something other
than itself -- the two-level closed form of Eq. tls-ham, eigenvalues from
numpy.linalg.eigvalsh, unitary similarity, and the Mott-lobe boundaries of the
Jaynes-Cummings model in closed form (Eq. jc-energies, Eq. mott-lobes-theory,
Sec. 3.3).  test_npad_mutants plants plausible mistakes in copies of the oracle and
checks that these pins catch each."""
import inspect
import math
import types

import numpy as np
import pytest

from oracle import npad


def _herm(d, seed, scale=1.0):
    g = np.random.default_rng(seed)
    X = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
    return scale * 0.5 * (X + X.conj().T)


def test_two_level_closed_form():
    # Eq. tls-ham: eps I + delta sz + g (cos phi sx + sin phi sy) has levels
    # eps +- sqrt(delta^2 + g^2); the rotation keeps their order
    for eps, delta, g, phi in ((0.3, 1.2, 0.7, 0.4), (-1.0, -0.5, 2.0, 2.9), (0.0, 0.0, 1.0, -1.1),
                               (2.0, 3.0, 1e-9, 0.0)):
        H = np.array([[eps + delta, g * np.exp(-1j * phi)], [g * np.exp(1j * phi), eps - delta]])
        Hp = oracle_npad().eliminate(H, [(0, 1)])
        r = math.hypot(delta, g)
        sgn = 1.0 if delta >= 0 else -1.0
        assert abs(Hp[0, 1]) < 1e-15 * (1 + r) and abs(Hp[1, 0]) < 1e-15 * (1 + r)
        assert Hp[0, 0].real == pytest.approx(eps + sgn * r, abs=1e-14)
        assert Hp[1, 1].real == pytest.approx(eps - sgn * r, abs=1e-14)


def test_similarity_invariants():
    # G is unitary, so H -> G H G^dag keeps the spectrum, Hermiticity and the
    # Frobenius norm; the eliminated couplings vanish
    H = _herm(9, 3)
    pairs = [(0, 5), (2, 7), (8, 1)]
    G = oracle_npad().givens_matrix(H, pairs)
    assert np.abs(G @ G.conj().T - np.eye(9)).max() < 1e-15
    Hp = oracle_npad().eliminate(H, pairs)
    np.testing.assert_allclose(np.linalg.eigvalsh(Hp), np.linalg.eigvalsh(H), atol=1e-13)
    assert np.abs(Hp - Hp.conj().T).max() < 1e-14
    assert np.linalg.norm(Hp) == pytest.approx(np.linalg.norm(H), rel=1e-14)
    for i, j in pairs:
        assert abs(Hp[i, j]) < 1e-14 and abs(Hp[j, i]) < 1e-14


def test_disjoint_rotations_commute():
    # rotations in disjoint planes commute: eliminating together equals one after
    # the other
    H = _herm(8, 4)
    both = oracle_npad().eliminate(H, [(1, 4), (6, 2)])
    seq = oracle_npad().eliminate(oracle_npad().eliminate(H, [(1, 4)]), [(6, 2)])
    np.testing.assert_allclose(both, seq, atol=1e-14)
    with pytest.raises(ValueError):
        oracle_npad().eliminate(H, [(1, 4), (4, 2)])


def test_jacobi_convergence_to_eigenvalues():
    # repeated elimination of the largest coupling diagonalises H (Jacobi
    # iteration for Hermitian matrices)
    H = _herm(7, 5)
    Hp = oracle_npad().iterate(H, 300)
    off = Hp - np.diag(np.diag(Hp))
    assert np.abs(off).max() < 1e-10
    np.testing.assert_allclose(np.sort(np.diag(Hp).real), np.linalg.eigvalsh(H), atol=1e-10)


def test_largest_coupling_brute_force():
    H = _herm(11, 6)
    best, arg = -1.0, None
    for i in range(11):
        for j in range(i + 1, 11):
            if abs(H[i, j]) > best:
                best, arg = abs(H[i, j]), (i, j)
    assert oracle_npad().largest_coupling(H) == arg


def jc_site(n_ph, omega, eps, g):
    """Single-site Jaynes-Cummings Hamiltonian (Eq. jch-jc-term) on n_ph photon levels
    times a qubit; basis index 2 * n + q (q = 0 ground, 1 excited)."""
    d = 2 * n_ph
    H = np.zeros((d, d), dtype=np.complex128)
    for n in range(n_ph):
        H[2 * n, 2 * n] = n * omega
        H[2 * n + 1, 2 * n + 1] = n * omega + eps
    for n in range(1, n_ph):          # a^dag sigma^- + sigma^+ a couples |n, g> and |n-1, e>
        H[2 * n, 2 * (n - 1) + 1] = g * math.sqrt(n)
        H[2 * (n - 1) + 1, 2 * n] = g * math.sqrt(n)
    return H


@pytest.mark.parametrize("delta_over_g", [-2.0, -0.3, 0.0, 0.5, 3.0])
def test_mott_lobe_boundaries(delta_over_g):
    # Sec. 3.3: one rotation per polariton-number block (all blocks at once) gives
    # the lower polariton energies E_{n-} exactly; the Mott-lobe boundaries
    # E_{(n+1)-} - E_{n-} = mu obey Eq. mott-lobes-theory
    g, omega = 1.0, 7.0
    eps = omega - delta_over_g * g
    n_ph = 8
    H = jc_site(n_ph, omega, eps, g)
    pairs = [(2 * n, 2 * (n - 1) + 1) for n in range(1, n_ph)]
    Hp = oracle_npad().eliminate(H, pairs)
    E_minus = [min(Hp[2 * n, 2 * n].real, Hp[2 * (n - 1) + 1, 2 * (n - 1) + 1].real) for n in range(1, n_ph)]
    x = delta_over_g / 2.0
    for n in range(1, n_ph - 1):
        mu = E_minus[n] - E_minus[n - 1]               # E_{(n+1)-} - E_{n-}
        theory = omega + g * (math.sqrt(n + x * x) - math.sqrt(n + 1 + x * x))
        assert mu == pytest.approx(theory, abs=1e-12)


# ------------------------------------------------------------------ mutants

MUTANTS = {
    "half_delta_dropped": ("delta = 0.5 * (a - cc)", "delta = (a - cc)"),
    "s_sign": ("s = sgn * g / (2.0 * r * c)", "s = -sgn * g / (2.0 * r * c)"),
    "no_conj": ("G[j, i] = -s * np.conj(e)", "G[j, i] = -s * e"),
    "order_flip": ("sgn = 1.0 if delta >= 0.0 else -1.0", "sgn = 1.0"),
    "adjoint_side": ("return G @ H @ G.conj().T", "return G.conj().T @ H @ G"),
    "cos_from_g": ("cos_t = abs(delta) / r", "cos_t = g / r"),
    "argmax_lower": ("A = np.abs(np.triu(H, 1))", "A = np.abs(np.tril(H, -1))"),
}
_MUT = {}


def oracle_npad():
    return _MUT.get("mod", npad)


@pytest.mark.filterwarnings("ignore")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_npad_mutants(name):
    src = inspect.getsource(npad)
    old, new = MUTANTS[name]
    assert old in src, name
    mod = types.ModuleType(f"npad_mutant_{name}")
    exec(compile(src.replace(old, new), f"<npad mutant {name}>", "exec"), mod.__dict__)
    pins = [test_two_level_closed_form, test_similarity_invariants, test_disjoint_rotations_commute,
            test_jacobi_convergence_to_eigenvalues, test_largest_coupling_brute_force]
    pins += [lambda v=v: test_mott_lobe_boundaries(v) for v in (-2.0, 0.5)]
    caught = 0
    _MUT["mod"] = mod
    try:
        for pin in pins:
            try:
                pin()
            except Exception:
                caught += 1
    finally:
        _MUT.clear()
    assert caught, f"no pin caught mutant {name}"
