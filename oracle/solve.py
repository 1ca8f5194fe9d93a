"""Solution at time T for sinusoidal sources: plain definitions, FP64.

Problem (paper, Section 2.1, equations (ode), (src), (ic1)): y' = -A y +
Im(e^{i w t}) b with y(0) = 0.  The paper writes sin(2 pi w t) with w a
frequency; here w is the angular frequency and the source is Im(e^{i w t} b),
which for real b is sin(w t) b and for complex b (an oblique incidence phase
ramp) is sin(w t) Re b + cos(w t) Im b.

Corollary 3 (equation (split1)) gives the exact solution as a time-harmonic
part minus a transient, with the minus sign that its proof derives:

    y(T) = Im(e^{i w T} z) - e^{-T A} Im z,    z = (A + i w I)^-1 b.

The oracle evaluates that formula with library linear algebra (dense LU or
sparse LU for z, dense ``expm`` or ``expm_multiply`` (Al-Mohy and Higham,
a method the paper cites) for the exponential action).  Independently of
Corollary 3 it also evaluates the variation-of-constants integral of the
proof, y(T) = int_0^T e^{-(T-s)A} Im(e^{i w s} b) ds, as one exponential of an
augmented matrix (Van Loan's construction): the source's time factor obeys
p' = [[0, w], [-w, 0]] p with p(0) = (0, 1), so (y, p) solves a homogeneous
linear system of size n + 2.
Oracle code: test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import assemble_A

DENSE_MAX = 3072       # n up to which dense matrices are used
SPLU_MAX = 6 * 16 ** 3  # n up to which the sparse LU is used for z


def _route(n, method):
    if method is None:
        return "dense" if n <= DENSE_MAX else ("splu" if n <= SPLU_MAX else "gmres")
    if method not in ("dense", "splu", "gmres"):
        raise ValueError(f"unknown route {method!r}")
    return method


def shifted_solve(As, b, route, rtol=1e-13):
    """x = As^-1 b for a complex sparse As by one library route; returns
    (x, true relative residual |b - As x| / |b|).

    dense: LU of the full matrix; splu: SuperLU plus one step of iterative
    refinement; gmres: restarted GMRES(200) to rtol, then GMRES on the true
    residual once more (iterative refinement).  A GMRES route whose true
    residual misses 100 rtol raises: the oracle never hands back an answer it
    has not checked.
    """
    n = As.shape[0]
    b = np.asarray(b, dtype=np.complex128)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n, dtype=np.complex128), 0.0
    if route == "dense":
        x = np.linalg.solve(As.toarray(), b)
    elif route == "splu":
        lu = spla.splu(As.tocsc())
        x = lu.solve(b)
        x = x + lu.solve(b - As @ x)
    else:
        x, info = spla.gmres(As, b, rtol=rtol, restart=200, maxiter=200)
        dx, info2 = spla.gmres(As, b - As @ x, rtol=rtol, restart=200, maxiter=50)
        x = x + dx
        res = np.linalg.norm(b - As @ x) / bn
        if res > 100 * rtol:
            raise RuntimeError(f"oracle GMRES did not converge: true relative residual "
                               f"{res:.2e} (info {info}, {info2}), target {rtol:.1e}")
        return x, res
    return x, float(np.linalg.norm(b - As @ x) / bn)


def stationary_with_residual(A, b, omega, rtol=1e-13, method=None):
    """(z, true relative residual) with z = (A + i w I)^-1 b, the vector z_stat
    of Corollary 3 (angular w).  ``method`` forces a route (dense, splu,
    gmres); by default dense LU up to n = DENSE_MAX, SuperLU up to SPLU_MAX,
    GMRES above."""
    n = A.shape[0]
    As = (A.astype(np.complex128) + 1j * omega * sp.identity(n, format="csr")).tocsr()
    return shifted_solve(As, b, _route(n, method), rtol)


def stationary(A, b, omega, rtol=1e-13, method=None):
    """z = (A + i w I)^-1 b (the vector z_stat of Corollary 3, angular w)."""
    return stationary_with_residual(A, b, omega, rtol, method)[0]


def expv(A, t, v):
    """e^{-t A} v (the exponential action of equation (y_homo))."""
    n = A.shape[0]
    v = np.asarray(v)
    if t == 0.0:
        return v.copy()
    if n <= DENSE_MAX:
        E = sla.expm(-t * A.toarray())
        return E @ v
    if np.iscomplexobj(v):
        return (spla.expm_multiply(-t * A, v.real)
                + 1j * spla.expm_multiply(-t * A, v.imag))
    return spla.expm_multiply(-t * A, v)


def split_solution(A, b, omega, T, z=None):
    """y(T) by Corollary 3: Im(e^{iwT} z) - e^{-TA} Im z; returns (y, z, y_tilde, y_hat)."""
    if z is None:
        z = stationary(A, b, omega)
    y_tilde = np.imag(np.exp(1j * omega * T) * z)
    y_hat = expv(A, T, np.imag(z))
    return y_tilde - y_hat, z, y_tilde, y_hat


def augmented_matrix(A, b, omega):
    """The (n + 2) x (n + 2) matrix [[-A, Re b, Im b], [0, 0, w], [0, -w, 0]]."""
    n = A.shape[0]
    b = np.asarray(b, dtype=np.complex128)
    B = sp.csr_matrix(np.stack([b.real, b.imag], axis=1)) if n <= DENSE_MAX else \
        sp.csr_matrix(sp.coo_matrix(np.stack([b.real, b.imag], axis=1)))
    Om = sp.csr_matrix(np.array([[0.0, omega], [-omega, 0.0]]))
    return sp.bmat([[-A, B], [None, Om]], format="csr")


def augmented_solution(A, b, omega, T, method=None):
    """y(T) from the variation-of-constants integral, without Corollary 3.

    ``method``: "dense" (expm of the full augmented matrix) or "sparse"
    (expm_multiply); by default dense up to n = DENSE_MAX."""
    n = A.shape[0]
    G = augmented_matrix(A, b, omega)
    e = np.zeros(n + 2)
    e[n + 1] = 1.0
    if method is None:
        method = "dense" if n <= DENSE_MAX else "sparse"
    if method == "dense":
        return (sla.expm(T * G.toarray()) @ e)[:n]
    if method != "sparse":
        raise ValueError(f"unknown route {method!r}")
    return spla.expm_multiply(T * G, e)[:n]


def solve_multifreq(inputs, b_cols, omegas, T):
    """y(T) for every column; ``b_cols`` is (n, ncols) complex, one omega per column."""
    A = assemble_A(inputs.eps, inputs.mu, inputs.sigma)
    out = np.empty((A.shape[0], b_cols.shape[1]))
    for c in range(b_cols.shape[1]):
        out[:, c] = split_solution(A, b_cols[:, c], omegas[c], T)[0]
    return out
