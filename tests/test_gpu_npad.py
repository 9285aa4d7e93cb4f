"""Numerical NPAD on the GPU (qcheff_npad_eliminate, qcheff_npad_largest) against the
oracle (oracle/npad.py): element by element at sizes the oracle's dense G H G^dag
finishes in seconds, sampled entries and invariants at d = 8192, and the Mott-lobe
boundaries of Eq. mott-lobes-theory (Sec. 3.3).

Tolerances: complex128, 1e-13 of max|H| per entry (two rotations of at most two
terms touch an entry); complex64, the oracle runs on the complex64-rounded H in
FP64 and the GPU rounds each updated entry once, so 4 2^-24 of max|H|."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import npad as onpad
from tests.test_gpu_parity import say
from tests.test_oracle_npad import jc_site

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")
DEV = "cuda:0"


def _herm(d, seed):
    g = np.random.default_rng(seed)
    X = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
    return 0.5 * (X + X.conj().T)


def _pairs(d, P, seed):
    perm = np.random.default_rng(seed).permutation(d)[: 2 * P]
    return [(int(perm[2 * p]), int(perm[2 * p + 1])) for p in range(P)]


def _tol(dtype, H):
    return (1e-13 if dtype == torch.complex128 else 4 * 2.0 ** -24) * np.abs(H).max()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d,P", [(2, 1), (7, 3), (64, 1), (64, 32), (300, 17), (300, 150), (1030, 63), (1030, 515)])
def test_eliminate_parity(d, P, dtype):
    say(f"npad eliminate d={d} P={P} {dtype}")
    q.sync_status()   # flags another test may have left
    H = _herm(d, d + P)
    Hd = torch.from_numpy(H).to(DEV).to(dtype)
    seen = Hd.cpu().numpy().astype(np.complex128)          # what the GPU sees
    pairs = _pairs(d, P, 7 * d + P)
    ref = onpad.eliminate(seen, pairs)
    q.npad_eliminate(Hd, pairs)
    torch.cuda.synchronize()
    got = Hd.cpu().numpy().astype(np.complex128)
    err = np.abs(got - ref).max()
    say(f"  max error {err:.2e}")
    assert err <= _tol(dtype, seen)
    assert q.sync_status() == q.OK


def test_eliminate_bad_pairs_left_alone():
    # an overlapping pair and an out-of-range one are skipped (and reported); the
    # valid pair of the same call is applied
    d = 40
    H = _herm(d, 3)
    Hd = torch.from_numpy(H).to(DEV)
    q.sync_status()
    q.npad_eliminate(Hd, [(1, 2), (2, 5), (7, 99), (10, 11)])
    torch.cuda.synchronize()
    ref = onpad.eliminate(H, [(10, 11)])
    assert np.abs(Hd.cpu().numpy() - ref).max() <= 1e-13 * np.abs(H).max()
    assert q.sync_status() == q.EINVAL and q.sync_status() == q.OK


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("d", [2, 5, 64, 257, 2000])
def test_largest_coupling(d, dtype):
    H = _herm(d, 11 + d)
    Hd = torch.from_numpy(H).to(DEV).to(dtype)
    seen = Hd.cpu().numpy().astype(np.complex128)
    ij, mag = q.npad_largest(Hd)
    torch.cuda.synchronize()
    i, j = onpad.largest_coupling(seen)
    assert ij.cpu().numpy().tolist() == [[i, j]]
    assert float(mag) == pytest.approx(abs(seen[i, j]), rel=1e-15)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_iterate_matches_oracle(dtype):
    # largest-first elimination, each step's pair found on the device
    d, n = 24, 40
    H = _herm(d, 5)
    Hd = torch.from_numpy(H).to(DEV).to(dtype)
    seen = Hd.cpu().numpy().astype(np.complex128)
    q.npad_iterate(Hd, n)
    torch.cuda.synchronize()
    ref = onpad.iterate(seen, n)
    tol = (1e-12 if dtype == torch.complex128 else 40 * 2.0 ** -24) * np.abs(seen).max()
    assert np.abs(Hd.cpu().numpy().astype(np.complex128) - ref).max() <= tol


@pytest.mark.parametrize("delta_over_g", [-2.0, 0.0, 3.0])
def test_mott_lobes_on_gpu(delta_over_g):
    g, omega, n_ph = 1.0, 7.0, 12
    H = jc_site(n_ph, omega, omega - delta_over_g * g, g)
    Hd = torch.from_numpy(H).to(DEV)
    q.npad_eliminate(Hd, [(2 * n, 2 * (n - 1) + 1) for n in range(1, n_ph)])
    torch.cuda.synchronize()
    D = np.diag(Hd.cpu().numpy()).real
    E = [min(D[2 * n], D[2 * (n - 1) + 1]) for n in range(1, n_ph)]
    x = delta_over_g / 2.0
    for n in range(1, n_ph - 1):
        assert E[n] - E[n - 1] == pytest.approx(omega + g * (math.sqrt(n + x * x) - math.sqrt(n + 1 + x * x)),
                                                abs=1e-12)


def test_eliminate_full_size():
    # d = 8192 (1 GiB of complex128), all 4096 disjoint pairs at once: sampled
    # entries against the oracle's rotation, the eliminated couplings, the
    # Frobenius norm (unitary similarity) and Hermiticity
    d = 8192
    say(f"npad eliminate d={d} P={d // 2}")
    g = np.random.default_rng(8192)
    X = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
    H = 0.5 * (X + X.conj().T)
    del X
    pairs = _pairs(d, d // 2, 8193)
    Hd = torch.from_numpy(H).to(DEV)
    fro = float(torch.linalg.matrix_norm(Hd))
    q.npad_eliminate(Hd, pairs)
    torch.cuda.synchronize()
    assert float(torch.linalg.matrix_norm(Hd)) == pytest.approx(fro, rel=1e-12)
    assert float((Hd - Hd.conj().T).abs().max()) <= 1e-13 * np.abs(H).max()
    P = np.array(pairs)
    vals = Hd[torch.from_numpy(P[:, 0]).to(DEV), torch.from_numpy(P[:, 1]).to(DEV)].abs().max()
    assert float(vals) <= 1e-13 * np.abs(H).max()
    # sampled entries: G has at most two entries per row, so (G H G^dag)_kl needs
    # only the rotations of k and l
    partner = {}
    for i, j in pairs:
        partner[i], partner[j] = j, i
    rs = np.random.default_rng(1)
    got = Hd.cpu().numpy()
    for k, l in zip(rs.integers(0, d, 64), rs.integers(0, d, 64)):
        idx = sorted({k, partner[k], l, partner[l]})
        sub = H[np.ix_(idx, idx)]
        sub_pairs = [(idx.index(a), idx.index(b)) for a, b in pairs if a in idx and b in idx]
        ref = onpad.eliminate(sub, sub_pairs)
        assert abs(got[k, l] - ref[idx.index(k), idx.index(l)]) <= 1e-13 * np.abs(H).max()
