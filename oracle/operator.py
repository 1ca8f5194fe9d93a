"""The semi-discrete 3D Maxwell operator A = M^-1 (S + K).

Paper, Section 2.1: after Yee discretisation the system is y' = -A y +
alpha(t) g with the operator block form diag(M_mu^-1, M_eps^-1) times
[[M_sigma, K], [-K^T, M_sigma]] (equation (ode) and the display after it).
The paper writes the 2D TM case; this is the 3D reading:

* state y = [Hx, Hy, Hz, Ex, Ey, Ez], six N^3 planes in C order [k][j][i];
* C is the discrete curl E -> H on the Yee grid with forward differences,
  C^T the curl H -> E with backward differences; K = [[0, C], [-C^T, 0]];
* every stencil read outside [0, N)^3 is zero (zero ghost), which keeps K
  exactly skew;
* S holds the same per-cell sigma on all six components of a cell, M holds mu
  on the H components and eps on the E components of the cell.

So (A y)_H = (sigma H + C E) / mu and (A y)_E = (sigma E - C^T H) / eps.
Oracle code: test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _fwd(f, axis):
    """g[idx] = f[idx + 1] - f[idx] along ``axis``, with f[N] = 0."""
    g = -f.copy()
    sl_dst = [slice(None)] * 3
    sl_src = [slice(None)] * 3
    sl_dst[axis] = slice(0, -1)
    sl_src[axis] = slice(1, None)
    g[tuple(sl_dst)] += f[tuple(sl_src)]
    return g


def _bwd(f, axis):
    """g[idx] = f[idx] - f[idx - 1] along ``axis``, with f[-1] = 0."""
    g = f.copy()
    sl_dst = [slice(None)] * 3
    sl_src = [slice(None)] * 3
    sl_dst[axis] = slice(1, None)
    sl_src[axis] = slice(0, -1)
    g[tuple(sl_dst)] -= f[tuple(sl_src)]
    return g


# array axes of an [k][j][i] grid
AX_I, AX_J, AX_K = 2, 1, 0


def curl_E(Ex, Ey, Ez):
    """C E: the discrete curl of E, landing on the H positions."""
    cx = _fwd(Ez, AX_J) - _fwd(Ey, AX_K)
    cy = _fwd(Ex, AX_K) - _fwd(Ez, AX_I)
    cz = _fwd(Ey, AX_I) - _fwd(Ex, AX_J)
    return cx, cy, cz


def curl_H(Hx, Hy, Hz):
    """C^T H: the discrete curl of H, landing on the E positions."""
    cx = _bwd(Hz, AX_J) - _bwd(Hy, AX_K)
    cy = _bwd(Hx, AX_K) - _bwd(Hz, AX_I)
    cz = _bwd(Hy, AX_I) - _bwd(Hx, AX_J)
    return cx, cy, cz


def apply_A(eps, mu, sigma, y):
    """w = A y, matrix-free.  ``y`` may be real or complex, length 6 nz ny nx
    (materials of shape (nz, ny, nx); cubes and general boxes alike)."""
    Y = y.reshape((6,) + eps.shape)
    Hx, Hy, Hz, Ex, Ey, Ez = Y
    ce = curl_E(Ex, Ey, Ez)
    ch = curl_H(Hx, Hy, Hz)
    W = np.empty_like(Y)
    for c in range(3):
        W[c] = (sigma * Y[c] + ce[c]) / mu
        W[3 + c] = (sigma * Y[3 + c] - ch[c]) / eps
    return W.reshape(-1)


def diff_1d(N):
    """The N x N forward difference with zero ghost: -1 diagonal, +1 above."""
    return sp.diags([-np.ones(N), np.ones(N - 1)], [0, 1], format="csr")


def curl_matrix(nx, ny=None, nz=None):
    """Sparse C (3 N3 x 3 N3): rows (C E)_x,y,z, columns Ex, Ey, Ez.

    With D_a the 1D forward difference of length a and flattening [k][j][i]
    (i fastest): Dx = I_nz (x) I_ny (x) D_nx, Dy = I_nz (x) D_ny (x) I_nx,
    Dz = D_nz (x) I_ny (x) I_nx and C = [[0, -Dz, Dy], [Dz, 0, -Dx], [-Dy, Dx, 0]].
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    I = lambda a: sp.identity(a, format="csr")
    Dx = sp.kron(I(nz), sp.kron(I(ny), diff_1d(nx)))
    Dy = sp.kron(I(nz), sp.kron(diff_1d(ny), I(nx)))
    Dz = sp.kron(diff_1d(nz), sp.kron(I(ny), I(nx)))
    return sp.bmat([[None, -Dz, Dy], [Dz, None, -Dx], [-Dy, Dx, None]],
                   format="csr")


def assemble_A(eps, mu, sigma):
    """Sparse A = diag(1/m) (diag(sigma_own) + [[0, C], [-C^T, 0]])."""
    nz, ny, nx = eps.shape
    C = curl_matrix(nx, ny, nz)
    K = sp.bmat([[None, C], [-C.T, None]], format="csr")
    s6 = np.tile(sigma.reshape(-1), 6)
    m6 = material_weights(eps, mu)
    return (sp.diags(1.0 / m6) @ (sp.diags(s6) + K)).tocsr()


def material_weights(eps, mu):
    """Diagonal of M: mu on the three H planes, eps on the three E planes."""
    e = eps.reshape(-1)
    m = mu.reshape(-1)
    return np.concatenate([m, m, m, e, e, e])


def m_inner(eps, mu, x, y):
    """The energy inner product <x, y>_M = x^H M y."""
    return np.vdot(x, material_weights(eps, mu) * y)


def m_norm(eps, mu, x):
    return float(np.sqrt(np.real(m_inner(eps, mu, x, x))))
