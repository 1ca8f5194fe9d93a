"""Transmitted power through a z-plane and its gradient w.r.t. per-cell eps.

The paper computes no gradients; this is the reading used by the
differentiation form.  For each angular frequency w the time-harmonic part of
Corollary 3 is Im(e^{i w t} z) with z = (A + i w I)^-1 b.  Its period-averaged
Poynting flux through the plane z = k_f is

    P_w = 1/2 Re sum_{i,j} [ z_Ex conj(Hy_bar) - z_Ey conj(Hx_bar) ]   at k_f,

with H_bar = (z_H[k_f - 1] + z_H[k_f]) / 2 (H sits half a cell above and
below the plane on the Yee grid).  The loss is L = sum_w P_w.

Gradient.  eps enters A only through the E rows: A_E = (S + K)_E / eps, so
dA/d eps_c = -(1/eps_c) e_r e_r^T A summed over the three E rows r of cell c.
Writing dL = Re(a^T dz) (a collects the partial derivatives of L w.r.t. the
entries of z, conjugates included), dz = -(A + i w)^-1 dA z gives

    dL / d eps_c = sum_w sum_{r in E rows of c} Re(lam_r (A z)_r) / eps_c,
    (A + i w)^T lam = a.

The oracle solves the transposed system directly (no structural shortcut).
Oracle code: test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import assemble_A
from .solve import _route, shifted_solve, stationary


def flux(z, N, kf):
    """P = 1/2 Re sum [z_Ex conj(Hy_bar) - z_Ey conj(Hx_bar)] on plane kf."""
    Z = z.reshape(6, N, N, N)
    hx = 0.5 * (Z[0, kf - 1] + Z[0, kf])
    hy = 0.5 * (Z[1, kf - 1] + Z[1, kf])
    ex, ey = Z[3, kf], Z[4, kf]
    return 0.5 * float(np.real(np.sum(ex * np.conj(hy) - ey * np.conj(hx))))


def flux_seed(z, N, kf):
    """a with dP = Re(a^T dz) for the flux P above (complex, length n)."""
    Z = z.reshape(6, N, N, N)
    a = np.zeros_like(Z)
    hx = 0.5 * (Z[0, kf - 1] + Z[0, kf])
    hy = 0.5 * (Z[1, kf - 1] + Z[1, kf])
    a[3, kf] = 0.5 * np.conj(hy)
    a[4, kf] = -0.5 * np.conj(hx)
    for k in (kf - 1, kf):
        a[1, k] += 0.25 * np.conj(Z[3, kf])
        a[0, k] += -0.25 * np.conj(Z[4, kf])
    return a.reshape(-1)


def _adjoint_solve(A, a, omega, method=None):
    """lam = (A + i w I)^-T a on the explicit transpose (no structural
    shortcut), by the same checked library routes as the forward solve."""
    n = A.shape[0]
    At = (A.T.astype(np.complex128) + 1j * omega * sp.identity(n, format="csr")).tocsr()
    return shifted_solve(At, a, _route(n, method))[0]


def loss(eps, mu, sigma, b_cols, omegas, kf, method=None):
    """L = sum_w P_w; returns (L, list of z)."""
    A = assemble_A(eps, mu, sigma)
    N = eps.shape[0]
    zs = [stationary(A, b_cols[:, c], omegas[c], method=method) for c in range(len(omegas))]
    return sum(flux(z, N, kf) for z in zs), zs


def loss_and_grad(eps, mu, sigma, b_cols, omegas, kf, method=None):
    """(L, dL/d eps) with the adjoint formula above; dL/d eps has shape N^3."""
    A = assemble_A(eps, mu, sigma)
    N = eps.shape[0]
    n3 = N ** 3
    L = 0.0
    g = np.zeros(n3)
    for c, w in enumerate(omegas):
        z = stationary(A, b_cols[:, c], w, method=method)
        L += flux(z, N, kf)
        a = flux_seed(z, N, kf)
        lam = _adjoint_solve(A, a, w, method)
        Az = A @ z
        contrib = np.real(lam[3 * n3:] * Az[3 * n3:]).reshape(3, n3).sum(axis=0)
        g += contrib / eps.reshape(-1)
    return L, g.reshape(eps.shape)


def fd_grad(eps, mu, sigma, b_cols, omegas, kf, cells, h=1e-6):
    """Central differences (L(eps + h e_c) - L(eps - h e_c)) / 2h on ``cells`` (i, j, k)."""
    out = []
    for (i, j, k) in cells:
        ep = eps.copy()
        ep[k, j, i] += h
        em = eps.copy()
        em[k, j, i] -= h
        Lp, _ = loss(ep, mu, sigma, b_cols, omegas, kf)
        Lm, _ = loss(em, mu, sigma, b_cols, omegas, kf)
        out.append((Lp - Lm) / (2 * h))
    return np.array(out)
