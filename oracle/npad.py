"""Oracle for numerical NPAD (the iterative Schrieffer-Wolff transformation).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or call this module; the product path never does.

Plain NumPy complex128 / float64, written from arXiv 2411.09982, Sec. 3.2: a
Hermitian H is block-diagonalised by Givens rotations, each of which exactly
diagonalises one two-level subspace {i, j} of H without flipping the order of
its two levels; several couplings in disjoint subspaces are eliminated by one
unitary (a product of commuting two-level rotations), H <- G H G^dag.

The two-level rotation (Eq. tls-ham).  Restricted to {i, j},
    H = [[eps + delta, g e^{-i phi}], [g e^{i phi}, eps - delta]],
so delta = (H_ii - H_jj) / 2, g = |H_ij|, e^{-i phi} = H_ij / g.  The Bloch vector
(g cos phi, g sin phi, delta) makes the angle theta = arctan(g / delta) with the z
axis (principal branch, so |theta| < pi/2 and the sign of delta, i.e. the level
order, is kept); rotating it by theta about n = sigma^y cos phi - sigma^x sin phi
onto the z axis is the two-level unitary
    R = [[c, s e^{-i phi}], [-s e^{i phi}, c]],  c = cos(theta/2), s = sin(theta/2),
with R H R^dag = diag(eps + sign(delta) r, eps - sign(delta) r), r = sqrt(delta^2 + g^2).
delta = 0 is read as theta = pi/2 (the level that was first stays the upper one).
The half-angle functions come from cos(theta) = |delta| / r without any
trigonometric call: c = sqrt((1 + cos theta) / 2), s = sign(delta) g / (2 r c).
"""
from __future__ import annotations

import math

import numpy as np


def rotation(H, i, j):
    """(c, s, e^{-i phi}) of the two-level rotation that eliminates H[i, j]."""
    a, b, cc = H[i, i].real, H[i, j], H[j, j].real
    g = abs(b)
    if g == 0.0:
        return 1.0, 0.0, 1.0 + 0.0j
    delta = 0.5 * (a - cc)
    r = math.hypot(delta, g)
    cos_t = abs(delta) / r
    c = math.sqrt(0.5 * (1.0 + cos_t))
    sgn = 1.0 if delta >= 0.0 else -1.0
    s = sgn * g / (2.0 * r * c)
    return c, s, b / g


def givens_matrix(H, pairs):
    """The unitary G that applies the two-level rotation of every (i, j) in `pairs`
    (disjoint index pairs) and is the identity elsewhere."""
    d = H.shape[0]
    G = np.eye(d, dtype=np.complex128)
    seen = set()
    for i, j in pairs:
        if i == j or i in seen or j in seen:
            raise ValueError("pairs must be disjoint and i != j")
        seen.update((i, j))
        c, s, e = rotation(H, i, j)
        G[i, i] = c
        G[i, j] = s * e
        G[j, i] = -s * np.conj(e)
        G[j, j] = c
    return G


def eliminate(H, pairs):
    """G H G^dag for the couplings `pairs` (Sec. 3.2, one NPAD step)."""
    H = np.asarray(H, dtype=np.complex128)
    G = givens_matrix(H, pairs)
    return G @ H @ G.conj().T


def largest_coupling(H):
    """(i, j), i < j, of the largest |H_ij| above the diagonal (the first in row-major
    order among equal magnitudes)."""
    H = np.asarray(H)
    A = np.abs(np.triu(H, 1))
    k = int(np.argmax(A))
    return divmod(k, H.shape[0])


def iterate(H, n):
    """n NPAD steps, each eliminating the largest remaining coupling."""
    H = np.asarray(H, dtype=np.complex128)
    for _ in range(n):
        i, j = largest_coupling(H)
        H = eliminate(H, [(i, j)])
    return H
