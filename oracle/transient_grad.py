"""Poynting flux of the field at a finite time T (transient included) and its
gradient with respect to per-cell eps: plain definitions, FP64.

The paper computes no gradients; this is the reading used by the
finite-time form of the differentiation path.  The period-averaged loss of
``grad`` sees only the time-harmonic part of Corollary 3.  Here the loss is
the instantaneous flux of the whole solution at the end time T,

    y_w(T) = Im(e^{i w T} z) - e^{-T A} Im z,   z = (A + i w I)^-1 b,

(equation (split1); the transient is the homogeneous problem (y_homo)),

    F(y) = sum_{i,j} [ Ex Hy_bar - Ey Hx_bar ]   on plane k_f,

with H_bar the mean of the H planes k_f - 1 and k_f (the same staggering as
the time-averaged flux), and L = sum_w F(y_w(T)).

The derivative is taken by forward differentiation of that formula with
library primitives only (no adjoint):

    dA  = -diag(d eps / eps on the E rows) A     (A_E = (S + K)_E / eps)
    dz  = -(A + i w I)^-1 dA z
    dE  = Frechet derivative of the matrix exponential at -T A in the
          direction -T dA (the derivative of e^{-TA})
    dy  = Im(e^{i w T} dz) - dE Im z - e^{-T A} Im dz
    dL  = grad F(y)^T dy

The Frechet derivative comes from scipy's ``expm_frechet`` (dense) or, for a
larger n, from the block identity exp([[X, Y], [0, X]]) = [[e^X, L(X, Y)],
[0, e^X]] applied to (0, v) with ``expm_multiply``.
Oracle code: test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import assemble_A
from .solve import DENSE_MAX, expv, stationary


def flux_real(y, N, kf):
    """F(y) = sum [Ex Hy_bar - Ey Hx_bar] on plane kf for a real field y."""
    Y = np.asarray(y).reshape(6, N, N, N)
    hx = 0.5 * (Y[0, kf - 1] + Y[0, kf])
    hy = 0.5 * (Y[1, kf - 1] + Y[1, kf])
    return float(np.sum(Y[3, kf] * hy - Y[4, kf] * hx))


def flux_real_grad(y, N, kf):
    """dF/dy (a real n-vector) for F above."""
    Y = np.asarray(y).reshape(6, N, N, N)
    g = np.zeros_like(Y)
    g[3, kf] = 0.5 * (Y[1, kf - 1] + Y[1, kf])
    g[4, kf] = -0.5 * (Y[0, kf - 1] + Y[0, kf])
    for k in (kf - 1, kf):
        g[1, k] += 0.5 * Y[3, kf]
        g[0, k] -= 0.5 * Y[4, kf]
    return g.reshape(-1)


def field_at_T(A, b, omega, T):
    """(y(T), z) by Corollary 3."""
    z = stationary(A, b, omega)
    y = np.imag(np.exp(1j * omega * T) * z) - expv(A, T, np.imag(z))
    return y, z


def loss(eps, mu, sigma, b_cols, omegas, kf, T):
    """L = sum_w F(y_w(T))."""
    A = assemble_A(eps, mu, sigma)
    N = eps.shape[0]
    return sum(flux_real(field_at_T(A, b_cols[:, c], w, T)[0], N, kf)
               for c, w in enumerate(omegas))


def _dA(A, eps, d_eps):
    """dA for the permittivity change d_eps (N^3): -(d_eps / eps) on the E rows of A."""
    n3 = eps.size
    d = np.zeros(A.shape[0])
    d[3 * n3:] = np.tile((np.asarray(d_eps) / eps).reshape(-1), 3)
    return -(sp.diags(d) @ A).tocsr()


def expm_derivative(A, dA, T, v, route=None):
    """d/dh e^{-T (A + h dA)} v at h = 0 (the Frechet derivative of the
    exponential at -T A in the direction -T dA, applied to v)."""
    n = A.shape[0]
    if route is None:
        route = "dense" if n <= DENSE_MAX else "sparse"
    if route == "dense":
        L = sla.expm_frechet(-T * A.toarray(), -T * dA.toarray(), compute_expm=False)
        return L @ v
    if route != "sparse":
        raise ValueError(f"unknown route {route!r}")
    B = sp.bmat([[-T * A, -T * dA], [None, -T * A]], format="csr")
    x = np.concatenate([np.zeros(n), np.asarray(v, dtype=np.float64)])
    return spla.expm_multiply(B, x)[:n]


def directional(eps, mu, sigma, b_cols, omegas, kf, T, d_eps, route=None):
    """dL[d_eps] = sum_c d_eps_c dL/d eps_c by the forward formulas above."""
    A = assemble_A(eps, mu, sigma)
    N = eps.shape[0]
    dA = _dA(A, eps, d_eps)
    out = 0.0
    for c, w in enumerate(omegas):
        y, z = field_at_T(A, b_cols[:, c], w, T)
        dz = -stationary(A, dA @ z, w)
        dy = (np.imag(np.exp(1j * w * T) * dz) - expm_derivative(A, dA, T, np.imag(z), route)
              - expv(A, T, np.imag(dz)))
        out += float(flux_real_grad(y, N, kf) @ dy)
    return out


def grad(eps, mu, sigma, b_cols, omegas, kf, T):
    """dL/d eps (shape N^3), one forward derivative per cell, dense (tiny
    grids only): the same formulas as ``directional`` with the factorisation
    of A + i w I and e^{-TA} computed once per frequency."""
    A = assemble_A(eps, mu, sigma)
    n = A.shape[0]
    if n > DENSE_MAX:
        raise ValueError("the per-cell oracle gradient is dense: n <= DENSE_MAX only")
    N = eps.shape[0]
    n3 = eps.size
    Ad = A.toarray()
    E = sla.expm(-T * Ad)
    g = np.zeros(n3)
    for c, w in enumerate(omegas):
        lu = sla.lu_factor(Ad + 1j * w * np.eye(n))
        z = sla.lu_solve(lu, np.asarray(b_cols[:, c], dtype=np.complex128))
        v = np.imag(z)
        y = np.imag(np.exp(1j * w * T) * z) - E @ v
        gF = flux_real_grad(y, N, kf)
        for cell in range(n3):
            rows = [p * n3 + cell for p in (3, 4, 5)]
            dAd = np.zeros_like(Ad)
            dAd[rows] = -Ad[rows] / eps.reshape(-1)[cell]
            dz = -sla.lu_solve(lu, dAd @ z)
            dE = sla.expm_frechet(-T * Ad, -T * dAd, compute_expm=False)
            dy = np.imag(np.exp(1j * w * T) * dz) - dE @ v - E @ np.imag(dz)
            g[cell] += gF @ dy
    return g.reshape(eps.shape)


def fd_grad(eps, mu, sigma, b_cols, omegas, kf, T, cells, h=1e-6):
    """Central differences (L(eps + h e_c) - L(eps - h e_c)) / 2h on ``cells`` (i, j, k)."""
    out = []
    for (i, j, k) in cells:
        ep = eps.copy()
        ep[k, j, i] += h
        em = eps.copy()
        em[k, j, i] -= h
        out.append((loss(ep, mu, sigma, b_cols, omegas, kf, T)
                    - loss(em, mu, sigma, b_cols, omegas, kf, T)) / (2 * h))
    return np.array(out)
