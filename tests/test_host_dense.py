"""Host-side small dense routines of the library (built with g++, no GPU)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("dense") / "libdense_shim.so"
    srcs = [os.path.join(ROOT, "tests", "native", "dense_shim.cpp"),
            os.path.join(ROOT, "paper_1707_00023_amd", "csrc", "kry_dense.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out)] + srcs,
                   check=True)
    L = ctypes.CDLL(str(out))
    L.t_choose_step.restype = ctypes.c_double
    L.t_choose_step_block.restype = ctypes.c_double
    return L


def P(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@pytest.mark.parametrize("m,scale", [(1, 0.3), (5, 0.01), (12, 1.0), (30, 25.0), (64, 400.0)])
def test_expm_matches_scipy(lib, m, scale):
    rng = np.random.default_rng(m)
    A = scale * rng.standard_normal((m, m)) / np.sqrt(m)
    E = np.zeros((m, m), order="F")
    Af = np.asfortranarray(A)
    lib.t_expm(m, P(Af), P(E))
    ref = sla.expm(A)
    assert np.abs(E - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_expm_skew_is_orthogonal(lib):
    rng = np.random.default_rng(3)
    S = rng.standard_normal((20, 20))
    S = 30.0 * (S - S.T)
    E = np.zeros((20, 20), order="F")
    lib.t_expm(20, P(np.asfortranarray(S)), P(E))
    assert np.abs(E.T @ E - np.eye(20)).max() < 1e-11


def _hess(rng, N, cplx=True):
    M = rng.standard_normal((N, N)) + (1j * rng.standard_normal((N, N)) if cplx else 0)
    return np.triu(M, -1).astype(np.complex128)


def test_hess_solve_and_bordered_matrix(lib):
    rng = np.random.default_rng(4)
    for N in (1, 2, 7, 33):
        M = _hess(rng, N)
        M[:, -1] = rng.standard_normal(N)   # dense last column (bordered form)
        b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        y = np.zeros(N, np.complex128)
        assert lib.t_hess_solve(N, P(np.asfortranarray(M)), P(b), P(y)) == 1
        assert np.abs(M @ y - b).max() <= 1e-11 * np.abs(b).max() * np.linalg.cond(M)


def test_hess_shift_and_dense_solve(lib):
    rng = np.random.default_rng(5)
    m = 17
    H = np.triu(rng.standard_normal((m + 1, m)), -1)
    Hf = np.asfortranarray(H)
    b = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    y = np.zeros(m, np.complex128)
    assert lib.t_hess_shift_solve(m, P(Hf), m + 1, ctypes.c_double(0.0), ctypes.c_double(0.7),
                                  P(b), P(y)) == 1
    ref = np.linalg.solve(H[:m] + 0.7j * np.eye(m), b)
    assert np.abs(y - ref).max() <= 1e-10 * np.abs(ref).max()
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    y2 = np.zeros(m, np.complex128)
    assert lib.t_dense_solve(m, P(np.asfortranarray(A)), P(b), P(y2)) == 1
    assert np.abs(y2 - np.linalg.solve(A, b)).max() <= 1e-10 * np.abs(y2).max()


def test_best_real_direction_is_optimal(lib):
    rng = np.random.default_rng(6)
    for n in (2, 5, 40):
        q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        w = np.zeros(n)
        lib.t_best_real_direction(n, P(q), P(w))
        assert abs(np.linalg.norm(w) - 1) < 1e-14
        best = abs(np.vdot(q, w))
        # brute force over the plane spanned by Re q, Im q
        Q, _ = np.linalg.qr(np.stack([q.real, q.imag], 1))
        ang = np.linspace(0, np.pi, 20001)
        cand = np.abs(np.stack([np.cos(ang), np.sin(ang)], 1) @ (Q.T @ q.conj()))
        assert best >= cand.max() * (1 - 1e-8)
        assert best >= np.linalg.norm(q) / np.sqrt(2) * (1 - 1e-14)


def test_choose_step_respects_residual_rate(lib):
    rng = np.random.default_rng(7)
    m = 12
    S = rng.standard_normal((m, m))
    H = np.triu(0.5 * (S - S.T) + 0.05 * np.eye(m), -1)
    Hbar = np.zeros((m + 1, m))
    Hbar[:m] = H
    hnext, beta, rate = 0.8, 2.0, 1e-6
    u = np.zeros(m)
    err = ctypes.c_double()
    tau = lib.t_choose_step(m, P(np.asfortranarray(Hbar)), m + 1, ctypes.c_double(hnext),
                            ctypes.c_double(beta), ctypes.c_double(5.0), ctypes.c_double(rate),
                            16, P(u), ctypes.byref(err))
    assert 0 < tau <= 5.0
    ref = beta * sla.expm(-tau * H)[:, 0]
    assert np.abs(u - ref).max() <= 1e-12 * beta
    ts = np.linspace(0, tau, 200)
    rho = [abs(hnext * (beta * sla.expm(-t * H)[:, 0])[-1]) for t in ts]
    assert max(rho) <= 1.05 * rate


def test_cholqr_factor_full_rank_and_deficient(lib):
    rng = np.random.default_rng(8)
    n, p = 200, 9
    w = 1 + rng.random(n)
    W = rng.standard_normal((n, p))
    W[:, 4] = W[:, 1] - 2 * W[:, 7]          # exact dependence -> rank 8
    W[:, 2] *= 1e-4                           # small but independent: kept
    G = W.T @ (w[:, None] * W)
    Cm = np.zeros((p, p))
    Rf = np.zeros((p, p))
    # a Gram-based factorisation resolves directions only to ~sqrt(eps): the
    # exact dependence is detected with a 1e-6 threshold
    r = lib.t_cholqr_factor(p, P(np.ascontiguousarray(G)), ctypes.c_double(1e-6), P(Cm), P(Rf))
    assert r == 8
    V = W @ Cm
    Gv = V.T @ (w[:, None] * V)
    expect = np.zeros((p, p))
    expect[:r, :r] = np.eye(r)
    assert np.abs(Gv - expect).max() < 1e-9
    assert np.abs(V @ Rf - W).max() < 1e-6 * np.abs(W).max()
    assert np.abs((V @ Rf - W)[:, 2]).max() < 1e-9 * np.abs(W[:, 2]).max()
    assert np.all(Rf[r:] == 0)


def test_block_shift_lsq_matches_numpy(lib):
    rng = np.random.default_rng(9)
    q, m = 4, 5
    K = q * m
    Hb = np.zeros((K + q, K))
    for j in range(m):
        Hb[: (j + 2) * q, j * q:(j + 1) * q] = rng.standard_normal(((j + 2) * q, q))
    bw = 2 * q - 1
    s = 0.37j
    g = np.zeros(K + q, np.complex128)
    g[:q] = rng.standard_normal(q) + 1j * rng.standard_normal(q)
    y = np.zeros(K, np.complex128)
    res = np.zeros(K + q, np.complex128)
    lib.t_block_shift_lsq(K, q, bw, P(np.asfortranarray(Hb)), K + q, ctypes.c_double(s.real),
                          ctypes.c_double(s.imag), P(g), P(y), P(res))
    Ms = Hb.astype(np.complex128)
    Ms[:K] += s * np.eye(K)
    yref = np.linalg.lstsq(Ms, g, rcond=None)[0]
    assert np.abs(y - yref).max() <= 1e-10 * np.abs(yref).max()
    assert np.abs(res - (g - Ms @ y)).max() <= 1e-12 * np.abs(g).max()


def test_choose_step_block_bounds_every_column(lib):
    rng = np.random.default_rng(10)
    q, m, g = 3, 4, 3
    K = q * m
    S = rng.standard_normal((K, K))
    H = 0.5 * (S - S.T) + 0.05 * np.eye(K)
    Hb = np.zeros((K + q, K))
    Hb[:K] = H
    Hb[K:, K - q:] = 0.4 * rng.standard_normal((q, q))
    U0 = np.zeros((K, g))
    U0[:q] = rng.standard_normal((q, g))
    rate = np.array([1e-5, 2e-5, 5e-6])
    U = np.zeros((K, g), order="F")
    err = np.zeros(g)
    tau, trial = 0.0, 3.0
    for _ in range(20):
        if tau > 0.0:
            break
        tau = lib.t_choose_step_block(K, q, g, P(np.asfortranarray(Hb)), K + q,
                                      P(np.asfortranarray(U0)), ctypes.c_double(trial), P(rate),
                                      16, P(U), P(err))
        trial /= 16
    assert tau < 3.0
    assert 0 < tau <= 3.0
    ref = sla.expm(-tau * H) @ U0
    assert np.abs(U - ref).max() <= 1e-12 * np.abs(U0).max()
    for t in np.linspace(0, tau, 100):
        Ut = sla.expm(-t * H) @ U0
        rho = np.linalg.norm(Hb[K:, K - q:] @ Ut[K - q:], axis=0)
        assert np.all(rho <= 1.05 * rate)


def test_qr_pivoted_resolves_to_rounding(lib):
    rng = np.random.default_rng(11)
    m, q = 60, 7
    S = rng.standard_normal((m, q))
    S[:, 3] = S[:, 0] + 1e-11 * rng.standard_normal(m)   # independent at 1e-11
    S[:, 5] = 2 * S[:, 1] - S[:, 4]                       # exactly dependent
    Q = np.zeros((m, q), order="F")
    Rf = np.zeros((q, q))
    r = lib.t_qr_pivoted(m, q, P(np.asfortranarray(S)), ctypes.c_double(1e-14), P(Q), P(Rf))
    assert r == 6
    assert np.abs(Q[:, :r].T @ Q[:, :r] - np.eye(r)).max() < 1e-14
    assert np.abs(Q @ Rf - S).max() < 1e-13 * np.abs(S).max()


# ------------------------------------------------------------ s-step Arnoldi --

def _dissipative(rng, n):
    """A = M^{-1}(S + K): K skew, S >= 0 diagonal, M > 0 diagonal."""
    K = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.08)
    K = K - K.T
    S = np.diag(0.3 * rng.random(n) * (rng.random(n) < 0.3))
    w = 1.0 + 2.0 * rng.random(n)
    return (S + K) / w[:, None], w


def _arnoldi_mgs2(A, w, v0, m):
    n = v0.size
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = v0 / np.sqrt(v0 @ (w * v0))
    for j in range(m):
        x = A @ V[:, j]
        for _ in range(2):
            for i in range(j + 1):
                h = V[:, i] @ (w * x)
                x = x - h * V[:, i]
                H[i, j] += h
        H[j + 1, j] = np.sqrt(x @ (w * x))
        V[:, j + 1] = x / H[j + 1, j]
    return V, H


def _pass_pip(lib, Vb, w, S, thr, use_ref):
    """One Gram-Schmidt pass as the library runs it: P = [V, S]^T M S in one
    product, the projected Gram matrix by Pythagoras, Cholesky, and the
    update [V, S] K = (S - V C) R^{-1} in one product."""
    M, ss = Vb.shape[1], S.shape[1]
    X = np.hstack([Vb, S])
    Pm = np.ascontiguousarray(X.T @ (w[:, None] * S))
    G = np.zeros((ss, ss))
    ref = np.zeros(ss)
    lib.t_proj_gram(M, ss, P(Pm), P(G), P(ref))
    C = np.ascontiguousarray(Pm[:M])
    R = np.zeros((ss, ss))
    r = ref if use_ref else np.ones(ss)
    assert lib.t_chol_upper(ss, P(G), P(r), ctypes.c_double(thr), P(R)) == 1
    Ri = np.zeros((ss, ss))
    lib.t_inv_upper(ss, P(R), P(Ri))
    K = np.zeros((M + ss, ss))
    lib.t_stack_coef(M, ss, P(C), P(Ri), P(K))
    return X @ K, C, R


def _arnoldi_sstep(lib, A, w, v0, m, s, rho, pip=False, c=0.0):
    """The s-step cycle with the library's host algebra; the tall-skinny
    products (done on the GPU by the library) are plain numpy here."""
    n = v0.size
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m), order="F")
    V[:, 0] = v0 / np.sqrt(v0 @ (w * v0))
    j0 = 0
    while j0 < m:
        ss = min(s, m - j0)
        M = j0 + 1
        T = np.zeros((n, ss + 1))
        T[:, 0] = V[:, j0]
        T[:, 1] = (A @ T[:, 0] - c * T[:, 0]) / rho
        for k in range(1, ss):
            T[:, k + 1] = 2 * (A @ T[:, k] - c * T[:, k]) / rho + T[:, k - 1]
        Sb = T[:, 1:].copy()
        Vb = V[:, :M]
        if pip:
            Tb, C1, R1 = _pass_pip(lib, Vb, w, Sb, 1e-10, True)
            Q, C2, R2 = _pass_pip(lib, Vb, w, Tb, 1e-8, False)
            V[:, M:M + ss] = Q
            lib.t_sstep_hessenberg(j0, ss, ctypes.c_double(rho), ctypes.c_double(c), P(C1), P(C2),
                                   P(R1), P(R2), P(H), m + 1)
            j0 += ss
            continue
        C1 = np.ascontiguousarray(Vb.T @ (w[:, None] * Sb))
        Sb -= Vb @ C1
        G = np.ascontiguousarray(Sb.T @ (w[:, None] * Sb))
        ref = np.diag(G) + (C1 ** 2).sum(axis=0)
        R1 = np.zeros((ss, ss))
        assert lib.t_chol_upper(ss, P(G), P(ref), ctypes.c_double(1e-10), P(R1)) == 1
        Ri = np.zeros((ss, ss))
        lib.t_inv_upper(ss, P(R1), P(Ri))
        Tb = Sb @ Ri
        C2 = np.ascontiguousarray(Vb.T @ (w[:, None] * Tb))
        Tb -= Vb @ C2
        G = np.ascontiguousarray(Tb.T @ (w[:, None] * Tb))
        R2 = np.zeros((ss, ss))
        assert lib.t_chol_upper(ss, P(G), P(np.ones(ss)), ctypes.c_double(1e-8), P(R2)) == 1
        lib.t_inv_upper(ss, P(R2), P(Ri))
        V[:, M:M + ss] = Tb @ Ri
        lib.t_sstep_hessenberg(j0, ss, ctypes.c_double(rho), ctypes.c_double(c), P(C1), P(C2), P(R1),
                               P(R2), P(H), m + 1)
        j0 += ss
    return V, H


@pytest.mark.parametrize("m,s,pip,shift", [(24, 8, False, False), (23, 5, False, False),
                                           (16, 16, False, False), (9, 2, False, False),
                                           (24, 8, True, False), (23, 5, True, True),
                                           (16, 16, True, True)])
def test_sstep_arnoldi_host_algebra(lib, m, s, pip, shift):
    rng = np.random.default_rng(40 + m + s)
    n = 300
    A, w = _dissipative(rng, n)
    lam = np.linalg.eigvals(A)
    rho = float(np.abs(lam.imag).max())
    c = 0.5 * float(lam.real.max()) if shift else 0.0
    v0 = rng.standard_normal(n)
    V, H = _arnoldi_sstep(lib, A, w, v0, m, s, rho, pip, c)
    # Arnoldi relation, M-orthonormality, Hessenberg form with h_{j+1,j} > 0
    assert np.abs(A @ V[:, :m] - V @ H).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(V.T @ (w[:, None] * V) - np.eye(m + 1)).max() <= 1e-12
    assert np.all(np.tril(H, -2) == 0.0)
    assert np.all(np.diag(H, -1) > 0.0)
    # the Arnoldi factorisation is unique: same H as one-step Gram-Schmidt
    Vr, Hr = _arnoldi_mgs2(A, w, v0, m)
    assert np.abs(H - Hr).max() <= 1e-9 * np.abs(Hr).max()
    assert np.abs(V - Vr).max() <= 1e-9 * np.abs(Vr).max()


def test_chol_upper_flags_dependent_column(lib):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((50, 4))
    X[:, 2] = X[:, 0] - 0.5 * X[:, 1] + 1e-13 * rng.standard_normal(50)
    G = np.ascontiguousarray(X.T @ X)
    R = np.zeros((4, 4))
    assert lib.t_chol_upper(4, P(G), P(np.diag(G).copy()), ctypes.c_double(1e-10), P(R)) == 0
    Y = rng.standard_normal((50, 4))
    G = np.ascontiguousarray(Y.T @ Y)
    assert lib.t_chol_upper(4, P(G), P(np.diag(G).copy()), ctypes.c_double(1e-10), P(R)) == 1
    assert np.abs(R.T @ R - G).max() <= 1e-12 * np.abs(G).max()
    Ri = np.zeros((4, 4))
    lib.t_inv_upper(4, P(R), P(Ri))
    assert np.abs(Ri @ R - np.eye(4)).max() <= 1e-12


def test_stack_coef_products(lib):
    # [V, S] K == (S - V C) F, for triangular (stack_coef) and general F
    rng = np.random.default_rng(11)
    n, M, s = 40, 7, 5
    V, S = rng.standard_normal((n, M)), rng.standard_normal((n, s))
    C = np.ascontiguousarray(rng.standard_normal((M, s)))
    Fu = np.ascontiguousarray(np.triu(rng.standard_normal((s, s))))
    Fg = np.ascontiguousarray(rng.standard_normal((s, s)))
    K = np.zeros((M + s, s))
    lib.t_stack_coef(M, s, P(C), P(Fu), P(K))
    assert np.abs(np.hstack([V, S]) @ K - (S - V @ C) @ Fu).max() <= 1e-12
    lib.t_stack_coef_full(M, s, P(C), P(Fg), P(K))
    assert np.abs(np.hstack([V, S]) @ K - (S - V @ C) @ Fg).max() <= 1e-12


@pytest.mark.parametrize("m,seed", [(1, 0), (2, 1), (5, 2), (30, 3), (64, 4)])
def test_hess_eigvals_matches_numpy(lib, m, seed):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((m, m)), -1)
    Hf = np.asfortranarray(H)
    re, im = np.zeros(m), np.zeros(m)
    assert lib.t_hess_eigvals(m, P(Hf), m, P(re), P(im)) == 1
    got = np.sort_complex(re + 1j * im)
    ref = np.sort_complex(np.linalg.eigvals(H))
    assert np.abs(got - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


def test_hess_eigvals_of_arnoldi_matrix(lib):
    # Ritz values of a dissipative operator's Arnoldi matrix: conjugate pairs
    # and Re >= 0 (the energy-product field of values)
    rng = np.random.default_rng(9)
    A, w = _dissipative(rng, 300)
    V, H = _arnoldi_mgs2(A, w, rng.standard_normal(300), 40)
    Hm = np.asfortranarray(H[:40])
    re, im = np.zeros(40), np.zeros(40)
    assert lib.t_hess_eigvals(40, P(Hm), 40, P(re), P(im)) == 1
    got = np.sort_complex(re + 1j * im)
    ref = np.sort_complex(np.linalg.eigvals(H[:40]))
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    assert re.min() >= -1e-10


def test_leja_steps_pairs_and_cut(lib):
    re = np.array([0.1, 0.1, 0.3, 0.05, 0.05, 0.2])
    im = np.array([2.0, -2.0, 0.0, -1.0, 1.0, 0.0])
    for s in (1, 2, 3, 4, 6):
        al, q = np.zeros(s), np.zeros(s)
        k = lib.t_leja_steps(6, P(re), P(im), s, ctypes.c_double(3.0), P(al), P(q))
        assert k == s
        # second step of a pair carries beta^2 / scale, first steps none
        for i in range(k):
            if q[i] != 0.0:
                assert i > 0 and q[i - 1] == 0.0 and al[i] == al[i - 1]
                assert q[i] in (4.0 / 3.0, 1.0 / 3.0)
    # the first shift is the largest in modulus (the pair at +-2i)
    al, q = np.zeros(2), np.zeros(2)
    lib.t_leja_steps(6, P(re), P(im), 2, ctypes.c_double(3.0), P(al), P(q))
    assert al[0] == 0.1 and q[1] == pytest.approx(4.0 / 3.0)
    # a pair cut by the block end is replaced by its real part
    al, q = np.zeros(1), np.zeros(1)
    lib.t_leja_steps(6, P(re), P(im), 1, ctypes.c_double(3.0), P(al), P(q))
    assert al[0] == 0.1 and q[0] == 0.0


def _arnoldi_sstep_newton(lib, A, w, v0, m, s, alpha, q, scale):
    """s-step cycle with a Newton basis t_{k+1} = (A t_k - alpha_k t_k +
    q_k t_{k-1}) / scale and the library's host algebra (Pythagorean
    passes, general basis-change matrix)."""
    n = v0.size
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m), order="F")
    V[:, 0] = v0 / np.sqrt(v0 @ (w * v0))
    j0 = 0
    while j0 < m:
        ss = min(s, m - j0)
        M = j0 + 1
        T = np.zeros((n, ss + 1))
        T[:, 0] = V[:, j0]
        Tm = np.zeros((ss + 1, ss))
        for k in range(ss):
            prev = T[:, k - 1] if k > 0 else 0.0
            qk = q[k] if k > 0 else 0.0
            T[:, k + 1] = (A @ T[:, k] - alpha[k] * T[:, k] + qk * prev) / scale
            Tm[k + 1, k] = scale
            Tm[k, k] = alpha[k]
            if k > 0:
                Tm[k - 1, k] = -qk
        Tb, C1, R1 = _pass_pip(lib, V[:, :M], w, T[:, 1:].copy(), 1e-10, True)
        Q, C2, R2 = _pass_pip(lib, V[:, :M], w, Tb, 1e-8, False)
        V[:, M:M + ss] = Q
        lib.t_sstep_hessenberg_tm(j0, ss, P(np.ascontiguousarray(Tm)), P(C1), P(C2), P(R1), P(R2),
                                  P(H), m + 1)
        j0 += ss
    return V, H


@pytest.mark.parametrize("m,s", [(24, 8), (30, 16), (24, 24)])
def test_sstep_newton_basis_host_algebra(lib, m, s):
    rng = np.random.default_rng(70 + m + s)
    n = 300
    A, w = _dissipative(rng, n)
    v0 = rng.standard_normal(n)
    # shifts: Ritz values of a first cycle, in Leja order
    _, H1 = _arnoldi_mgs2(A, w, rng.standard_normal(n), s)
    re, im = np.zeros(s), np.zeros(s)
    assert lib.t_hess_eigvals(s, P(np.asfortranarray(H1[:s])), s, P(re), P(im)) == 1
    scale = float(np.abs(np.linalg.eigvals(A)).max())
    al, q = np.zeros(s), np.zeros(s)
    assert lib.t_leja_steps(s, P(re), P(im), s, ctypes.c_double(scale), P(al), P(q)) == s
    V, H = _arnoldi_sstep_newton(lib, A, w, v0, m, s, al, q, scale)
    assert np.abs(A @ V[:, :m] - V @ H).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(V.T @ (w[:, None] * V) - np.eye(m + 1)).max() <= 1e-12
    Vr, Hr = _arnoldi_mgs2(A, w, v0, m)
    assert np.abs(H - Hr).max() <= 1e-9 * np.abs(Hr).max()


def _groups_valid(w, gid, ng, max_size, band):
    """Each group is a run of consecutive values, within its size and band
    limits, and no group could have taken the next value (greedy)."""
    order = np.argsort(w, kind="stable")
    ids = gid[order]
    assert ids[0] == 0 and np.all(np.diff(ids) >= 0) and np.all(np.diff(ids) <= 1)
    assert ids[-1] == ng - 1
    for g in range(ng):
        mem = np.sort(w[gid == g])
        assert 1 <= mem.size <= max_size
        assert mem[-1] - mem[0] <= band * 0.5 * (mem[0] + mem[-1]) + 1e-15
        nxt = np.sort(w)[np.searchsorted(np.sort(w), mem[-1], side="right"):]
        if nxt.size:  # the next value would break a limit
            lo, hi = mem[0], nxt[0]
            assert mem.size == max_size or hi - lo > band * 0.5 * (lo + hi)


def test_group_shifts(lib):
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib.t_group_shifts.restype = ctypes.c_int
    # 16 frequencies over 2 pi [0.08, 0.12]: four groups of neighbours
    w = 2 * np.pi * np.linspace(0.08, 0.12, 16)
    gid = np.zeros(16, dtype=np.int32)
    ng = lib.t_group_shifts(16, P(w), 16, ctypes.c_double(0.1), P(gid))
    assert ng == 4
    _groups_valid(w, gid, ng, 16, 0.1)
    assert list(gid[:4]) == [0] * 4 and list(gid[4:8]) == [1] * 4
    # a narrow band in one group; the size limit splits it
    w = 2 * np.pi * np.linspace(0.1, 0.101, 40)
    gid = np.zeros(40, dtype=np.int32)
    ng = lib.t_group_shifts(40, P(w), 16, ctypes.c_double(0.1), P(gid))
    assert ng == 3 and list(np.bincount(gid)) == [16, 16, 8]
    # unsorted input, a zero shift and a single shift
    rng = np.random.default_rng(5)
    for n in (1, 7, 33):
        w = np.concatenate([[0.0], rng.uniform(0.0, 2.0, n - 1)]) if n > 1 else np.array([0.7])
        rng.shuffle(w)
        gid = np.zeros(n, dtype=np.int32)
        ng = lib.t_group_shifts(n, P(w), 5, ctypes.c_double(0.1), P(gid))
        _groups_valid(w, gid, ng, 5, 0.1)


# --- the projected problem of the residual-restarted inhomogeneous method --

def test_gauss_legendre_rule(lib):
    for q in (1, 4, 8, 13):
        x, w = np.zeros(q), np.zeros(q)
        lib.t_gauss_legendre01(q, P(x), P(w))
        xr, wr = np.polynomial.legendre.leggauss(q)
        assert np.abs(x - 0.5 * (xr + 1)).max() < 1e-15
        assert np.abs(w - 0.5 * wr).max() < 1e-15


def _stable_hessenberg(m, seed):
    # an Arnoldi matrix of a dissipative operator (skew plus small positive
    # diagonal), the kind of H the restarted method projects on
    rng = np.random.default_rng(seed)
    n = 4 * m
    S = rng.standard_normal((n, n))
    A = (S - S.T) / np.sqrt(n) * 3.0 + np.diag(rng.uniform(0.0, 0.3, n))
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    v = rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        x = A @ V[:, j]
        for _ in range(2):
            h = V[:, :j + 1].T @ x
            x -= V[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(x)
        V[:, j + 1] = x / H[j + 1, j]
    return H


@pytest.mark.parametrize("m,q,dt", [(12, 8, 0.1), (40, 8, 0.12)])
def test_rst_march_matches_exact_projected_solution(lib, m, q, dt):
    # u' = -H u + beta f(t) e_1 with f = sin(w t) (column 0) and cos(w t)
    # (column 1), sampled at the Gauss nodes of each step: u(T) and the new
    # residual source -h e_m^T u(t) against the exact solution from one
    # exponential of the augmented matrix [[-H, beta e1, 0], [0, 0, w],
    # [0, -w, 0]] (the source as the output of a rotation)
    Hb = _stable_hessenberg(m, 3)
    H = np.asfortranarray(Hb[:m, :m])
    h = Hb[m, m - 1]
    om, beta, nt = 0.7, 1.3, 50
    x, w = np.zeros(q), np.zeros(q)
    lib.t_gauss_legendre01(q, P(x), P(w))
    t = (np.arange(nt)[:, None] * dt + dt * x[None, :]).reshape(-1)
    fin = np.ascontiguousarray(np.stack([np.sin(om * t), np.cos(om * t)]))
    fout = np.zeros_like(fin)
    uT = np.zeros((2, m))
    resint = np.zeros(2)
    lib.t_rst_march(m, P(H), m, q, ctypes.c_double(dt), P(x), P(w), nt, 2, ctypes.c_double(beta),
                    ctypes.c_double(h), P(fin), P(fout), P(uT), P(resint))
    G = np.zeros((m + 2, m + 2))
    G[:m, :m] = -H
    G[0, m] = beta
    G[m, m + 1] = om
    G[m + 1, m] = -om
    T = nt * dt
    for c, p0 in ((0, [0.0, 1.0]), (1, [1.0, 0.0])):  # (sin, cos) and (cos, -sin) outputs
        xi0 = np.concatenate([np.zeros(m), p0])
        uex = (sla.expm(T * G) @ xi0)[:m]
        assert np.linalg.norm(uT[c] - uex) <= 1e-11 * np.linalg.norm(uex)
        for k in (0, 7, len(t) // 2, len(t) - 1):
            ut = (sla.expm(t[k] * G) @ xi0)[:m]
            assert abs(fout[c, k] + h * ut[-1]) <= 1e-11 * max(1.0, abs(h * ut[-1]))
    # the residual integral is the Gauss rule of |fout| over [0, T]
    assert np.allclose(resint, (np.abs(fout).reshape(2, nt, q) * (dt * w)).sum(axis=(1, 2)), rtol=1e-13)
