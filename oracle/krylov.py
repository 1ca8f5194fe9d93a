"""The Krylov basis and projected matrix by their definition (small m only).

Regular Krylov (paper, Section 3.2, equations (Arn) and (Krylov)): the
columns of V_{m+1} are an orthonormal basis of K_{m+1}(A, v) = span(v, Av,
..., A^m v), nested (span(v_1..v_j) = K_j for every j), and A V_m =
V_{m+1} H with H upper Hessenberg.  Here orthonormality is in the energy
inner product <x, y>_M = x^T M y.  With the sign fixed by h_{j+1,j} > 0
(equivalently a QR factor with positive diagonal) the basis is unique, so it
can be computed directly from the Krylov matrix: V = M^{-1/2} Q where Q R is
the QR factorisation of M^{1/2} [v, Av, ..., A^m v] with diag(R) > 0, and
H = V_{m+1}^T M A V_m.  The Krylov matrix becomes ill-conditioned quickly,
so this is only meaningful for a few steps.
Oracle code: test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .operator import apply_A, material_weights


def krylov_basis(eps, mu, sigma, v, m):
    """(V (n, m+1), H (m+1, m), beta) by QR of the scaled Krylov matrix."""
    w = material_weights(eps, mu)
    sw = np.sqrt(w)
    K = np.empty((v.size, m + 1))
    K[:, 0] = v
    for j in range(m):
        K[:, j + 1] = apply_A(eps, mu, sigma, K[:, j])
    Q, R = np.linalg.qr(sw[:, None] * K)
    sgn = np.sign(np.diag(R))
    Q = Q * sgn[None, :]
    V = Q / sw[:, None]
    AV = np.stack([apply_A(eps, mu, sigma, V[:, j]) for j in range(m)], axis=1)
    H = V.T @ (w[:, None] * AV)
    beta = float(np.sqrt(v @ (w * v)))
    return V, H, beta
