"""Pins of the oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
hand-derived matrix, a closed form, an invariant, or an independent
integration of the ODE.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import solve_ivp

import workloads as wk
from oracle import grad as og
from oracle import operator as op
from oracle import solve as osv


def _medium(N, seed=3, sigma_max=1.0, layer=1, n_spheres=2):
    wl = wk.small(N, seed=seed, n_spheres=n_spheres, layer=layer,
                  sigma_max=sigma_max, radius=(0.8, 1.5))
    return wl, wk.generate(wl)


# --- P1: the single-cell curl, derived by hand from the Yee stencil --------

def test_single_cell_curl_by_hand():
    # One cell, all neighbours outside the grid read as zero: each forward
    # difference f[+1] - f reduces to -f.  (C E)_x = (Ez[j+1]-Ez) - (Ey[k+1]-Ey)
    # = -Ez + Ey, and cyclically.
    C_hand = np.array([[0.0, 1.0, -1.0],
                       [-1.0, 0.0, 1.0],
                       [1.0, -1.0, 0.0]])
    assert np.array_equal(op.curl_matrix(1).toarray(), C_hand)
    one = np.ones((1, 1, 1))
    for col in range(3):
        y = np.zeros(6)
        y[3 + col] = 1.0
        w = op.apply_A(one, one, 0 * one, y)
        assert np.allclose(w[:3], C_hand[:, col], atol=0, rtol=0)
        assert np.allclose(w[3:], 0.0)
    # rank 2 with the node gradient (1, 1, 1) as null space
    assert np.linalg.matrix_rank(C_hand) == 2
    assert np.allclose(C_hand @ np.ones(3), 0)


# --- curl of a gradient and divergence of a curl vanish exactly ------------

def _grad_nodes(phi):
    """Node potential -> E edges: forward differences written out with np.diff."""
    N = phi.shape[0]
    pad = lambda a, ax: np.concatenate([a, np.zeros_like(np.take(a, [0], axis=ax))], axis=ax)
    gx = np.diff(pad(phi, 2), axis=2)
    gy = np.diff(pad(phi, 1), axis=1)
    gz = np.diff(pad(phi, 0), axis=0)
    return gx, gy, gz


def test_curl_of_gradient_is_zero():
    rng = np.random.default_rng(0)
    phi = rng.standard_normal((5, 5, 5))
    gx, gy, gz = _grad_nodes(phi)
    cx, cy, cz = op.curl_E(gx, gy, gz)
    assert max(abs(cx).max(), abs(cy).max(), abs(cz).max()) < 1e-12
    # and the E-side: C^T H is orthogonal to every gradient (G^T C^T = (C G)^T = 0)
    H = rng.standard_normal((3, 5, 5, 5))
    ch = op.curl_H(*H)
    assert abs(sum(np.sum(c * g) for c, g in zip(ch, (gx, gy, gz)))) < 1e-10


def test_divergence_of_curl_is_zero():
    rng = np.random.default_rng(1)
    E = rng.standard_normal((3, 6, 6, 6))
    cx, cy, cz = op.curl_E(*E)
    pad = lambda a, ax: np.concatenate([a, np.zeros_like(np.take(a, [0], axis=ax))], axis=ax)
    div = (np.diff(pad(cx, 2), axis=2) + np.diff(pad(cy, 1), axis=1)
           + np.diff(pad(cz, 0), axis=0))
    assert abs(div).max() < 1e-12


def test_matrix_free_equals_assembled_and_skew():
    wl, inp = _medium(6)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y = wk.random_state(wl.n, 5)
    assert np.allclose(A @ y, op.apply_A(inp.eps, inp.mu, inp.sigma, y), rtol=0, atol=1e-13)
    # K = M (A) - S is exactly skew
    m6 = op.material_weights(inp.eps, inp.mu)
    K = (np.diag(m6) @ A.toarray()) - np.diag(np.tile(inp.sigma.reshape(-1), 6))
    assert np.abs(K + K.T).max() < 1e-14


def test_matrix_free_equals_assembled_on_a_box():
    rng = np.random.default_rng(6)
    shape = (5, 3, 4)   # (nz, ny, nx)
    eps = 1 + 2 * rng.random(shape)
    mu = 1 + rng.random(shape)
    sig = 0.3 * rng.random(shape)
    A = op.assemble_A(eps, mu, sig)
    y = rng.standard_normal(6 * eps.size)
    assert np.allclose(A @ y, op.apply_A(eps, mu, sig, y), rtol=0, atol=1e-13)
    # single-cell-thick box: each axis of length 1 reduces to the hand case
    one = np.ones((1, 1, 1))
    assert np.array_equal(op.curl_matrix(1, 1, 1).toarray(), op.curl_matrix(1).toarray())


# --- P4: separable modes reduce the problem to a 6 x 6 closed form ---------

def _mode(N, q):
    """Separable mode built from numpy's SVD of the 1D forward difference."""
    D = np.diag(-np.ones(N)) + np.diag(np.ones(N - 1), 1)
    U, S, Vt = np.linalg.svd(D)
    prof = []
    s = []
    for d in range(3):
        u, w = U[:, q[d]], Vt[q[d]]
        prof.append((u, w))
        s.append(S[q[d]])
    # along axis d: E_d and the two H components transverse to d take u;
    # the two E components transverse to d and H_d take w
    planes = []
    for comp in range(6):
        field, axis = divmod(comp, 3)   # field 0 = H, 1 = E
        f = []
        for d in range(3):
            use_w = (field == 1 and d != axis) or (field == 0 and d == axis)
            f.append(prof[d][1] if use_w else prof[d][0])
        # array order [k][j][i]: z profile outer, x profile inner
        planes.append(np.einsum("k,j,i->kji", f[2], f[1], f[0]))
    return planes, np.array(s)


def _A6(s, eps, mu, sig):
    X = np.array([[0, -s[2], s[1]], [s[2], 0, -s[0]], [-s[1], s[0], 0]])
    return np.block([[sig / mu * np.eye(3), X / mu], [X / eps, sig / eps * np.eye(3)]])


def test_separable_mode_closed_form():
    N, eps0, mu0, sig0 = 5, 2.0, 1.3, 0.15
    q = (1, 3, 2)
    planes, s = _mode(N, q)
    ones = np.ones((N, N, N))
    amp = np.array([0.3, -1.1, 0.7, 0.9, 0.2, -0.5])
    y = np.concatenate([(a * p).reshape(-1) for a, p in zip(amp, planes)])
    w = op.apply_A(eps0 * ones, mu0 * ones, sig0 * ones, y)
    A6 = _A6(s, eps0, mu0, sig0)
    w6 = A6 @ amp
    expect = np.concatenate([(a * p).reshape(-1) for a, p in zip(w6, planes)])
    assert np.abs(w - expect).max() < 1e-13
    # full solve: the source along the mode; 6x6 closed form by integrating
    # the 6-dim ODE independently
    omega, T = 2 * math.pi * 0.13, 7.0
    beta = np.array([0.0, 0.0, 0.0, 1.0, -0.4, 0.2])
    b = np.concatenate([(a * p).reshape(-1) for a, p in zip(beta, planes)])
    A = op.assemble_A(eps0 * ones, mu0 * ones, sig0 * ones)
    y_or, z, _, _ = osv.split_solution(A, b, omega, T)
    sol = solve_ivp(lambda t, u: -A6 @ u + math.sin(omega * t) * beta, (0, T),
                    np.zeros(6), method="DOP853", rtol=1e-13, atol=1e-15)
    y6 = sol.y[:, -1]
    expect = np.concatenate([(a * p).reshape(-1) for a, p in zip(y6, planes)])
    assert np.abs(y_or - expect).max() < 1e-10 * max(1.0, np.abs(expect).max())
    z6 = np.linalg.solve(A6 + 1j * omega * np.eye(6), beta)
    zexp = np.concatenate([(a * p).reshape(-1) for a, p in zip(z6, planes)])
    assert np.abs(z - zexp).max() < 1e-12


def test_singular_values_closed_form():
    for N in (3, 4, 9):
        D = op.diff_1d(N).toarray()
        s = np.sort(np.linalg.svd(D, compute_uv=False))
        qq = np.arange(1, N + 1)
        f = np.sort(2 * np.sin((2 * qq - 1) * np.pi / (2 * (2 * N + 1))))
        assert np.abs(s - f).max() < 1e-14


# --- P2: Corollary 3 (with its minus sign) against the augmented matrix ----

@pytest.mark.parametrize("theta", [0.0, 0.4])
def test_split_equals_augmented_dense(theta):
    wl, inp = _medium(4, seed=7)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    omega, T = 2 * math.pi * 0.1, 23.0
    b = wk.source_vector(wl, omega, theta)
    y_split = osv.split_solution(A, b, omega, T)[0]
    y_aug = osv.augmented_solution(A, b, omega, T)
    assert np.linalg.norm(y_split - y_aug) <= 1e-12 * np.linalg.norm(y_aug)
    # a plus sign in the split would be far off
    z = osv.stationary(A, b, omega)
    y_plus = np.imag(np.exp(1j * omega * T) * z) + osv.expv(A, T, np.imag(z))
    assert np.linalg.norm(y_plus - y_aug) > 1e-3 * np.linalg.norm(y_aug)


def test_split_equals_direct_integration():
    wl, inp = _medium(3, seed=9)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma).toarray()
    omega, T = 2 * math.pi * 0.1, 15.0
    b = wk.source_vector(wl, omega, 0.0).real
    sol = solve_ivp(lambda t, u: -A @ u + math.sin(omega * t) * b, (0, T),
                    np.zeros(wl.n), method="DOP853", rtol=1e-12, atol=1e-14)
    import scipy.sparse as sp
    y = osv.split_solution(sp.csr_matrix(A), b, omega, T)[0]
    assert np.linalg.norm(y - sol.y[:, -1]) <= 1e-9 * np.linalg.norm(sol.y[:, -1])


def test_sparse_paths_match_dense():
    # N = 9 (n = 4374) takes the sparse LU and expm_multiply routes; compare
    # with dense scipy routines on the same matrix
    wl, inp = _medium(9, seed=2, layer=2, n_spheres=4)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    omega, T = 2 * math.pi * 0.1, 9.0
    b = wk.source_vector(wl, omega, 0.0)
    z = osv.stationary(A, b, omega)
    Ad = A.toarray()
    zd = sla.solve(Ad + 1j * omega * np.eye(wl.n), b)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    v = wk.random_state(wl.n, 3)
    e1 = osv.expv(A, T, v)
    e2 = sla.expm(-T * Ad) @ v
    assert np.linalg.norm(e1 - e2) <= 1e-11 * np.linalg.norm(e2)


# --- P3: invariants -------------------------------------------------------

def test_energy_conserved_without_damping():
    wl, inp = _medium(4, seed=4, sigma_max=0.0)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y0 = wk.random_state(wl.n, 8)
    y = osv.expv(A, 37.0, y0)
    e0 = op.m_norm(inp.eps, inp.mu, y0)
    e1 = op.m_norm(inp.eps, inp.mu, y)
    assert abs(e1 - e0) <= 1e-12 * e0


def test_energy_decays_and_spectrum_in_right_half_plane():
    wl, inp = _medium(4, seed=4, sigma_max=1.0)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y0 = wk.random_state(wl.n, 8)
    norms = [op.m_norm(inp.eps, inp.mu, osv.expv(A, t, y0)) for t in (0.0, 1.0, 3.0, 9.0)]
    assert all(b <= a * (1 + 1e-14) for a, b in zip(norms, norms[1:]))
    lam = np.linalg.eigvals(A.toarray())
    assert lam.real.min() > -1e-10


def test_discrete_divergence_conserved():
    wl, inp = _medium(4, seed=5, sigma_max=0.0)
    N = wl.N
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y0 = wk.random_state(wl.n, 9)
    y = osv.expv(A, 11.0, y0)

    def charges(v):
        V = v.reshape(6, N, N, N)
        # node charge = -(G^T M_eps E), via the adjoint of np.diff gradients
        D = op.diff_1d(N).toarray()
        eE = [inp.eps * V[3 + c] for c in range(3)]
        q = (np.einsum("ai,kja->kji", D, eE[0]) + np.einsum("aj,kai->kji", D, eE[1])
             + np.einsum("ak,aji->kji", D, eE[2]))
        mH = [inp.mu * V[c] for c in range(3)]
        pad = lambda a, ax: np.concatenate([a, np.zeros_like(np.take(a, [0], axis=ax))], axis=ax)
        dm = (np.diff(pad(mH[0], 2), axis=2) + np.diff(pad(mH[1], 1), axis=1)
              + np.diff(pad(mH[2], 0), axis=0))
        return q, dm

    q0, d0 = charges(y0)
    q1, d1 = charges(y)
    assert np.abs(q1 - q0).max() < 1e-11
    assert np.abs(d1 - d0).max() < 1e-11


# --- P6: gradient against brute-force central differences -----------------

def test_flux_seed_directional_derivative():
    rng = np.random.default_rng(2)
    N, kf = 4, 2
    z = rng.standard_normal(6 * N ** 3) + 1j * rng.standard_normal(6 * N ** 3)
    dz = rng.standard_normal(6 * N ** 3) + 1j * rng.standard_normal(6 * N ** 3)
    a = og.flux_seed(z, N, kf)
    h = 1e-6
    fd = (og.flux(z + h * dz, N, kf) - og.flux(z - h * dz, N, kf)) / (2 * h)
    assert abs(fd - np.real(a @ dz)) <= 1e-8 * max(1.0, abs(fd))


def test_adjoint_gradient_matches_fd_every_cell():
    N, kf = 4, 3
    wl = wk.small(N, seed=21, n_spheres=2, layer=1, radius=(0.8, 1.4),
                  omegas=(2 * math.pi * 0.09, 2 * math.pi * 0.11), src_k=1)
    inp = wk.generate(wl)
    b_cols = np.stack([wk.source_vector(wl, w, 0.0) for w in wl.omegas], axis=1)
    L, g = og.loss_and_grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf)
    cells = [(i, j, k) for k in range(N) for j in range(N) for i in range(N)]
    fd = og.fd_grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, cells, h=1e-5)
    gv = np.array([g[k, j, i] for (i, j, k) in cells])
    assert np.linalg.norm(gv - fd) <= 1e-6 * np.linalg.norm(fd)


# --- Krylov basis by definition: properties the definition fixes ----------

def test_krylov_basis_definition_properties():
    from oracle import krylov as okr
    wl, inp = _medium(5, seed=13)
    v = wk.random_state(wl.n, 4)
    m = 5
    V, H, beta = okr.krylov_basis(inp.eps, inp.mu, inp.sigma, v, m)
    w = op.material_weights(inp.eps, inp.mu)
    assert np.abs(V.T @ (w[:, None] * V) - np.eye(m + 1)).max() < 1e-12
    assert np.allclose(V[:, 0] * beta, v, atol=1e-12 * np.abs(v).max())
    # upper Hessenberg with positive subdiagonal
    assert np.abs(np.tril(H, -2)).max() < 1e-10
    assert all(H[j + 1, j] > 0 for j in range(m))
    # Arnoldi relation A V_m = V_{m+1} H
    AV = np.stack([op.apply_A(inp.eps, inp.mu, inp.sigma, V[:, j]) for j in range(m)], axis=1)
    assert np.abs(AV - V @ H).max() < 1e-10
    # energy dissipativity carries to the projection: the symmetric part of
    # H (an orthogonal projection in the energy product) is positive semidefinite
    assert np.linalg.eigvalsh(0.5 * (H[:m] + H[:m].T)).min() > -1e-12


# --- the flux: hand cases and the discrete Poynting balance ----------------

def test_flux_hand_cases_fix_planes_and_signs():
    # 3^3 grid, plane kf = 1: E sits on the plane, H half a cell below (k = 0)
    # and above (k = 1); the flux is the z-component of E x H,
    # 1/2 Re(Ex conj(Hy) - Ey conj(Hx)), with H averaged over the two planes.
    N, kf = 3, 1

    def state(**entries):
        z = np.zeros((6, N, N, N), dtype=np.complex128)
        for name, (k, val) in entries.items():
            z[wk.COMPONENTS.index(name), k, 1, 2] = val
        return z.reshape(-1)

    assert og.flux(state(Ex=(1, 1.0), Hy=(0, 2.0)), N, kf) == pytest.approx(0.5, abs=1e-15)
    assert og.flux(state(Ex=(1, 1.0), Hy=(1, 2.0)), N, kf) == pytest.approx(0.5, abs=1e-15)
    assert og.flux(state(Ey=(1, 1.0), Hx=(1, 2.0)), N, kf) == pytest.approx(-0.5, abs=1e-15)
    assert og.flux(state(Ey=(1, 1.0), Hx=(0, 2.0)), N, kf) == pytest.approx(-0.5, abs=1e-15)
    # the phase enters through Re(E conj(H)): in phase 1/4, in quadrature 0
    assert og.flux(state(Ex=(1, 1j), Hy=(0, 1j)), N, kf) == pytest.approx(0.25, abs=1e-15)
    assert og.flux(state(Ex=(1, 1j), Hy=(0, 1.0)), N, kf) == pytest.approx(0.0, abs=1e-15)
    # fields off the plane, or H two half-cells away, carry no flux here
    assert og.flux(state(Ex=(1, 1.0), Hy=(2, 5.0)), N, kf) == 0.0
    assert og.flux(state(Ex=(0, 1.0), Hy=(0, 5.0)), N, kf) == 0.0
    assert og.flux(state(Ez=(1, 1.0), Hx=(1, 5.0), Hy=(0, 3.0)), N, kf) == 0.0


def _dissipation_above(z, sigma, N, kf):
    """Power absorbed above the two staggered cuts that straddle plane kf.

    Cut a (between H at kf - 1/2 and E at kf) leaves every component of the
    cells k >= kf above it; cut b (between E, Hz at kf and Ez, Hx, Hy at
    kf + 1/2) leaves the cells k > kf and the Ez, Hx, Hy of layer kf above it.
    With S = diag(sigma) on all six components, the real part of
    z^H (S + K + i w M) z restricted to a region with no source is
    sum sigma |z|^2 plus the K-coupling across the cut, i.e. the inflow."""
    Z = z.reshape(6, N, N, N)
    mag = np.abs(Z) ** 2
    above_a = np.sum(sigma[kf:] * mag[:, kf:].sum(axis=0))
    above_b = np.sum(sigma[kf + 1:] * mag[:, kf + 1:].sum(axis=0))
    above_b += np.sum(sigma[kf] * (mag[0, kf] + mag[1, kf] + mag[5, kf]))
    return above_a, above_b


@pytest.mark.parametrize("theta", [0.0, 0.4])
def test_flux_equals_dissipated_power_above_plane(theta):
    # Discrete Poynting theorem: for (A + i w) z = b with b zero above a cut,
    # Re of z^H M (A + i w) z over the components above the cut is zero
    # (K restricted to them is real skew, i w M is imaginary), so the flux
    # through the cut equals the absorbed power sum sigma |z|^2 above it.
    # The flux through plane kf with H averaged over kf - 1/2 and kf + 1/2 is
    # the mean of the inflows through cuts a and b, each twice its power.
    N, kf = 6, 3
    wl = wk.small(N, seed=5, n_spheres=3, layer=2, radius=(0.8, 1.5), src_k=1)
    inp = wk.generate(wl)
    mu = 1.0 + np.random.default_rng(4).uniform(0.0, 1.0, size=inp.eps.shape)
    A = op.assemble_A(inp.eps, mu, inp.sigma)
    omega = 2 * math.pi * 0.1
    b = wk.source_vector(wl, omega, theta)
    z = osv.stationary(A, b, omega)
    pa, pb = _dissipation_above(z, inp.sigma, N, kf)
    P = og.flux(z, N, kf)
    assert pa > 0 and pb > 0
    assert abs(P - 0.25 * (pa + pb)) <= 1e-12 * P

    # plausible mistakes in the flux fail the balance: H averaged over the
    # planes kf, kf + 1, or the Ey Hx term with the wrong sign
    Z = z.reshape(6, N, N, N)

    def flux_variant(h_lo, h_hi, sign):
        hx = 0.5 * (Z[0, h_lo] + Z[0, h_hi])
        hy = 0.5 * (Z[1, h_lo] + Z[1, h_hi])
        return 0.5 * float(np.real(np.sum(Z[3, kf] * np.conj(hy) + sign * Z[4, kf] * np.conj(hx))))

    assert flux_variant(kf - 1, kf, -1) == pytest.approx(P, rel=1e-14)
    for wrong in (flux_variant(kf, kf + 1, -1), flux_variant(kf - 1, kf, +1)):
        assert abs(wrong - 0.25 * (pa + pb)) > 1e-3 * P


# --- the sparse and iterative oracle routes against independent ones ------

@pytest.mark.parametrize("theta", [0.0, 0.4])
def test_augmented_sparse_route_matches_split(theta):
    # n = 4374 > DENSE_MAX: the augmented matrix goes through expm_multiply
    # (the route of the stored full-size expected values), the split through
    # SuperLU and expm_multiply of A alone (both pinned to dense routines)
    wl, inp = _medium(9, seed=2, n_spheres=4)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    omega, T = 2 * math.pi * 0.1, 9.0
    b = wk.source_vector(wl, omega, theta)
    assert A.shape[0] > osv.DENSE_MAX
    y_aug = osv.augmented_solution(A, b, omega, T)
    y_split = osv.split_solution(A, b, omega, T)[0]
    assert np.linalg.norm(y_aug - y_split) <= 1e-12 * np.linalg.norm(y_split)


def test_gmres_routes_match_sparse_lu():
    # the GMRES branches (forward and explicit-transpose adjoint) against
    # SuperLU on the same systems, with their true residuals reported
    wl, inp = _medium(9, seed=2, n_spheres=4)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    omega = 2 * math.pi * 0.1
    b = wk.source_vector(wl, omega, 0.3)
    z_lu, r_lu = osv.stationary_with_residual(A, b, omega, method="splu")
    z_gm, r_gm = osv.stationary_with_residual(A, b, omega, method="gmres")
    assert r_lu < 1e-14 and r_gm < 1e-12
    assert np.linalg.norm(z_gm - z_lu) <= 1e-12 * np.linalg.norm(z_lu)
    a = og.flux_seed(z_lu, wl.N, 5)
    lam_lu = og._adjoint_solve(A, a, omega, "splu")
    lam_gm = og._adjoint_solve(A, a, omega, "gmres")
    At = A.T.toarray() + 1j * omega * np.eye(wl.n)
    assert np.linalg.norm(At @ lam_lu - a) <= 1e-13 * np.linalg.norm(a)
    assert np.linalg.norm(lam_gm - lam_lu) <= 1e-12 * np.linalg.norm(lam_lu)


def test_gmres_route_raises_when_target_is_missed():
    wl, inp = _medium(2, seed=2, n_spheres=1)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    import scipy.sparse as sp
    As = (A.astype(np.complex128) + 0.3j * sp.identity(wl.n)).tocsr()
    b = wk.random_state(wl.n, 1).astype(np.complex128)
    x, res = osv.shifted_solve(As, b, "gmres", rtol=1e-13)
    assert res < 1e-12
    with pytest.raises(RuntimeError, match="did not converge"):
        osv.shifted_solve(As, b, "gmres", rtol=1e-30)


# --- the flux at a finite time T and its forward-mode gradient -------------

def _tflux_case(N, kf, omegas, seed=21):
    wl = wk.small(N, seed=seed, n_spheres=1, layer=1, radius=(0.8, 1.4), omegas=omegas, src_k=0)
    inp = wk.generate(wl)
    b_cols = np.stack([wk.source_vector(wl, w, 0.0) for w in wl.omegas], axis=1)
    return wl, inp, b_cols


def test_instantaneous_flux_hand_cases():
    # 3^3 grid, plane kf = 1: the z-component of E x H for a real field,
    # Ex Hy - Ey Hx, with H averaged over the planes below (k = 0) and above
    # (k = 1) the E plane
    from oracle import transient_grad as tg
    N, kf = 3, 1

    def state(**entries):
        y = np.zeros((6, N, N, N))
        for name, (k, val) in entries.items():
            y[wk.COMPONENTS.index(name), k, 2, 0] = val
        return y.reshape(-1)

    assert tg.flux_real(state(Ex=(1, 1.0), Hy=(0, 2.0)), N, kf) == pytest.approx(1.0, abs=1e-15)
    assert tg.flux_real(state(Ex=(1, 3.0), Hy=(1, 2.0)), N, kf) == pytest.approx(3.0, abs=1e-15)
    assert tg.flux_real(state(Ey=(1, 1.0), Hx=(1, 2.0)), N, kf) == pytest.approx(-1.0, abs=1e-15)
    assert tg.flux_real(state(Ey=(1, -1.0), Hx=(0, 4.0)), N, kf) == pytest.approx(2.0, abs=1e-15)
    assert tg.flux_real(state(Ex=(1, 1.0), Hy=(2, 5.0)), N, kf) == 0.0
    assert tg.flux_real(state(Ez=(1, 1.0), Hx=(1, 5.0), Hy=(0, 3.0)), N, kf) == 0.0


def test_instantaneous_flux_averages_to_the_harmonic_flux():
    # over one period the instantaneous flux of Im(e^{i w t} z) averages to
    # the period-averaged flux 1/2 Re(Ex conj(Hy) - Ey conj(Hx)) (the flux is
    # quadratic, so four equispaced phases average it exactly)
    from oracle import transient_grad as tg
    rng = np.random.default_rng(8)
    N, kf, w = 4, 2, 0.7
    z = rng.standard_normal(6 * N ** 3) + 1j * rng.standard_normal(6 * N ** 3)
    per = 2 * math.pi / w
    avg = np.mean([tg.flux_real(np.imag(np.exp(1j * w * j * per / 4) * z), N, kf) for j in range(4)])
    assert avg == pytest.approx(og.flux(z, N, kf), rel=1e-13)
    # and its derivative is the one central differences give (F is quadratic)
    y = rng.standard_normal(6 * N ** 3)
    d = rng.standard_normal(6 * N ** 3)
    fd = (tg.flux_real(y + d, N, kf) - tg.flux_real(y - d, N, kf)) / 2
    assert tg.flux_real_grad(y, N, kf) @ d == pytest.approx(fd, rel=1e-12)


def test_expm_derivative_routes_against_differences():
    # the block identity route (expm_multiply on a 2n system) and scipy's
    # dense Frechet derivative against central differences of e^{-T(A + h dA)} v
    from oracle import transient_grad as tg
    wl, inp = _medium(4, seed=6)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    d_eps = np.random.default_rng(2).standard_normal(inp.eps.shape)
    dA = tg._dA(A, inp.eps, d_eps)
    v = wk.random_state(wl.n, 5)
    T, h = 6.0, 1e-5
    fd = (osv.expv(A + h * dA, T, v) - osv.expv(A - h * dA, T, v)) / (2 * h)
    dense = tg.expm_derivative(A, dA, T, v, "dense")
    sparse = tg.expm_derivative(A, dA, T, v, "sparse")
    assert np.linalg.norm(dense - fd) <= 1e-8 * np.linalg.norm(fd)
    assert np.linalg.norm(sparse - dense) <= 1e-11 * np.linalg.norm(dense)
    # the perturbation changes only the E rows: a change of the H rows'
    # weights (mu) is not what d eps means
    assert np.abs(dA[: 3 * inp.eps.size].toarray()).max() == 0.0


def test_transient_flux_gradient_matches_fd_every_cell():
    from oracle import transient_grad as tg
    N, kf, T = 3, 2, 7.0
    wl, inp, b_cols = _tflux_case(N, kf, (2 * math.pi * 0.1,))
    g = tg.grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, T)
    cells = [(i, j, k) for k in range(N) for j in range(N) for i in range(N)]
    fd = tg.fd_grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, T, cells, h=1e-5)
    gv = np.array([g[k, j, i] for (i, j, k) in cells])
    assert np.linalg.norm(gv - fd) <= 1e-7 * np.linalg.norm(fd)
    # the transient matters here: dropping it changes the gradient
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y, z = tg.field_at_T(A, b_cols[:, 0], wl.omegas[0], T)
    assert np.linalg.norm(osv.expv(A, T, np.imag(z))) > 0.1 * np.linalg.norm(y)


def test_transient_flux_directional_derivative_routes():
    # per-cell gradient, dense and block-identity directional derivatives on
    # two frequencies agree, and all vanish at T = 0 (y(0) = 0)
    from oracle import transient_grad as tg
    N, kf, T = 3, 1, 5.0
    wl, inp, b_cols = _tflux_case(N, kf, (2 * math.pi * 0.09, 2 * math.pi * 0.11), seed=4)
    g = tg.grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, T)
    d = np.random.default_rng(3).standard_normal(inp.eps.shape)
    dd = tg.directional(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, T, d, "dense")
    ds = tg.directional(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, T, d, "sparse")
    assert dd == pytest.approx(float((g * d).sum()), rel=1e-11)
    assert ds == pytest.approx(dd, rel=1e-11)
    assert tg.loss(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, 0.0) == pytest.approx(0.0, abs=1e-15)
    assert tg.directional(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, 0.0, d) == \
        pytest.approx(0.0, abs=1e-14)
