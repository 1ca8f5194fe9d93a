"""GPU path (through the C ABI) against the FP64 CPU oracle.

Floating-point parity targets: the operator to rounding (1e-14 relative
FP64, 1e-6 FP32); the Arnoldi basis and projected matrix to 1e-11 for the
first steps (the Krylov matrix conditioning grows after that); exponential
actions, shifted solves and full solutions to 1e-8 relative 2-norm (FP64
path), 1e-5 (FP32 storage).
"""
import json
import math
import os
import time

import numpy as np
import pytest

import workloads as wk
from oracle import krylov as okr
from oracle import operator as op
from oracle import solve as osv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kry():
    import paper_1707_00023_amd as kry
    return kry


def _dev():
    return torch.device("cuda:0")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=_dev())


def _solver(eps, mu=None, sigma=None, **kw):
    kry = _kry()
    return kry.Solver(_t(eps), None if mu is None else _t(mu),
                      None if sigma is None else _t(sigma), kry.Options(**kw))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _box(shape, seed, with_mu=True):
    rng = np.random.default_rng(seed)
    eps = 1 + 2 * rng.random(shape)
    mu = 1 + 0.5 * rng.random(shape) if with_mu else None
    sig = 0.4 * rng.random(shape)
    return eps, mu, sig


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


# --------------------------------------------------------------- operator --

@pytest.mark.parametrize("shape,with_mu", [((9, 5, 7), True), ((9, 5, 7), False),
                                           ((1, 1, 1), True), ((16, 16, 16), False)])
def test_apply_matches_oracle(shape, with_mu):
    _announce(f"apply {shape} mu={with_mu}")
    eps, mu, sig = _box(shape, 3, with_mu)
    s = _solver(eps, mu, sig)
    mu_or = mu if mu is not None else np.ones(shape)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, 6 * eps.size))
    w = s.apply(_t(v)).cpu().numpy()
    for c in range(3):
        ref = op.apply_A(eps, mu_or, sig, v[c])
        assert np.abs(w[c] - ref).max() <= 1e-14 * np.abs(ref).max()
    w32 = s.apply_f32(_t(v.astype(np.float32))).cpu().numpy()
    ref = op.apply_A(eps, mu_or, sig, v[0].astype(np.float32).astype(np.float64))
    assert np.abs(w32[0] - ref).max() <= 2e-6 * np.abs(ref).max()


def test_apply_large_ragged_grid():
    # 131 x 129 x 130 cells: the multi-cell-per-thread launch with a ragged tail
    shape = (130, 129, 131)
    _announce(f"apply {shape}")
    eps, _, sig = _box(shape, 5, with_mu=False)
    s = _solver(eps, None, sig)
    v = np.random.default_rng(2).standard_normal(6 * eps.size)
    w = s.apply(_t(v)).cpu().numpy()[0]
    ref = op.apply_A(eps, np.ones(shape), sig, v)
    assert np.abs(w - ref).max() <= 1e-14 * np.abs(ref).max()


def test_apply_at_c2_materials():
    wl = wk.C2
    _announce("apply c2 materials 128^3")
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma)
    v = wk.random_state(wl.n, 7)
    w = s.apply(_t(v)).cpu().numpy()[0]
    ref = op.apply_A(inp.eps, inp.mu, inp.sigma, v)
    assert np.abs(w - ref).max() <= 1e-14 * np.abs(ref).max()


# ---------------------------------------------------------------- Arnoldi --

@pytest.mark.parametrize("orth,s_step", [("delayed", 0), ("cgs2", 0), ("delayed", 4)])
def test_arnoldi_matches_definition_first_steps(orth, s_step):
    _announce(f"arnoldi vs definition ({orth}, s_step {s_step})")
    eps, mu, sig = _box((6, 6, 6), 8)
    s = _solver(eps, mu, sig, krylov_dim=8, orth=orth, s_step=s_step)
    v = np.random.default_rng(3).standard_normal(6 * eps.size)
    m = 5
    V, H, beta, steps = s.arnoldi(_t(v), m)
    Vo, Ho, bo = okr.krylov_basis(eps, mu, sig, v, m)
    assert steps == m
    assert abs(beta - bo) <= 1e-13 * bo
    assert np.abs(H - Ho).max() <= 1e-11 * np.abs(Ho).max()
    assert np.abs(V.cpu().numpy() - Vo.T).max() <= 1e-11 * np.abs(Vo).max()


@pytest.mark.parametrize("m,orth,s_step", [(30, "delayed", 0), (64, "delayed", 0), (64, "cgs2", 0),
                                          (64, "delayed", 8), (30, "delayed", 7),
                                          (32, "delayed", 16), (64, "delayed", 32),
                                          (48, "delayed", 64), (64, "delayed", 24)])
def test_arnoldi_relation_and_orthogonality(m, orth, s_step):
    _announce(f"arnoldi relation m={m} {orth} s_step {s_step}")
    wl = wk.small(12, seed=4, n_spheres=5)
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=m, orth=orth, s_step=s_step)
    v = wk.random_state(wl.n, 9)
    V, H, beta, steps = s.arnoldi(_t(v), m)
    V = V.cpu().numpy().T
    w = op.material_weights(inp.eps, inp.mu)
    G = V.T @ (w[:, None] * V)
    # an s-step block is accepted after one Gram-Schmidt pass when its loss
    # of orthogonality, of order u cond(R1)^2, is below 1e-11
    assert np.abs(G - np.eye(m + 1)).max() <= (1e-10 if s_step > 1 else 1e-12)
    AV = np.stack([op.apply_A(inp.eps, inp.mu, inp.sigma, V[:, j]) for j in range(m)], axis=1)
    R = AV - V @ H
    assert np.abs(R).max() <= 1e-12 * np.abs(AV).max()
    assert np.abs(np.tril(H, -2)).max() == 0.0
    # Lemma 1 (homogeneous case): residual of y_m(t) = V_m u(t), u = beta e^{-tH} e_1
    import scipy.linalg as sla
    t = 1.7
    u = beta * sla.expm(-t * H[:m])[:, 0]
    ym = V[:, :m] @ u
    dym = -V[:, :m] @ (H[:m] @ u)
    r = -dym - op.apply_A(inp.eps, inp.mu, inp.sigma, ym)
    est = H[m, m - 1] * abs(u[-1])
    assert abs(math.sqrt(r @ (w * r)) - est) <= 1e-10 * max(est, 1e-300) + 1e-13 * beta


@pytest.mark.parametrize("shape,with_mu,storage", [((67, 13, 23), True, "f64"), ((64, 8, 16), False, "f64"),
                                                   ((130, 5, 37), False, "f32")])
def test_zmarch_stencil_equals_cell_parallel(shape, with_mu, storage):
    # the z-marching form of the s-step basis stencil (4, 8 and 16 planes per
    # workgroup; ragged tiles in x, y and z) computes the same expressions in
    # the same order as the cell-parallel one: the s-step Arnoldi bases and H
    # agree bitwise
    _announce(f"z-march stencil {shape} mu={with_mu} {storage}")
    eps, mu, sig = _box(shape, 21, with_mu)
    v = np.random.default_rng(5).standard_normal(6 * eps.size)
    ref = None
    for zm in (0, 4, 8, 16):
        s = _solver(eps, mu, sig, krylov_dim=32, s_step=16, storage=storage)
        s.set_tune(zm_stencil=zm)
        V, H, beta, steps = s.arnoldi(_t(v), 32)
        s.close()
        if ref is None:
            ref = (V.cpu().numpy(), H)
            # and the basis is a Krylov basis of the oracle operator (the
            # s-step Hessenberg algebra carries the block's conditioning:
            # 1e-11 on these random boxes)
            Vn = ref[0].astype(np.float64).T
            mu_or = mu if mu is not None else np.ones(shape)
            AV = np.stack([op.apply_A(eps, mu_or, sig, Vn[:, j]) for j in range(steps)], axis=1)
            tol = 1e-11 if storage == "f64" else 2e-6
            assert np.abs(AV - Vn @ H[:, :steps]).max() <= tol * np.abs(AV).max()
        else:
            assert np.array_equal(V.cpu().numpy(), ref[0]) and np.array_equal(H, ref[1])


@pytest.mark.parametrize("N,m,s_step", [(20, 64, 16), (16, 30, 8), (12, 48, 16)])
def test_device_block_finish_matches_host(N, m, s_step):
    # the s-step cycle with each block's Gram-Schmidt factors, checks and
    # coefficients on the device (one synchronisation per cycle) against the
    # host form of the same cycle: bases and H to rounding, and a solve
    _announce(f"device block finish {N}^3 m={m} s={s_step}")
    wl = wk.small(N, seed=N, n_spheres=6, layer=2)
    inp = wk.generate(wl)
    eps, sig = inp.eps, inp.sigma
    shape = eps.shape
    v = np.random.default_rng(8).standard_normal(6 * eps.size)
    out = {}
    for hb in (True, False):
        s = _solver(eps, None, sig, krylov_dim=m, s_step=s_step, host_blocks=hb, tol=1e-10)
        V, H, beta, steps = s.arnoldi(_t(v), m)
        b = np.zeros(6 * eps.size, dtype=np.complex128)
        b[3 * eps.size: 4 * eps.size] = np.random.default_rng(9).standard_normal(eps.size)
        y = s.solve_multifreq([0.6, 0.65], _t(b[None, :]), 12.0).cpu().numpy()
        out[hb] = (V.cpu().numpy(), H, beta, steps, y, s.last_stats)
        s.close()
    Vh, Hh, bh, sh, yh, sth = out[True]
    Vd, Hd, bd, sd, yd, std_ = out[False]
    assert sh == sd == m and abs(bh - bd) <= 1e-14 * bh
    # both are M-orthonormal Krylov bases with the Arnoldi relation; the two
    # forms round the small factors differently, and an s-step block passes
    # the difference on amplified by its condition (up to 1e6 by the guard),
    # so the bases themselves agree to 1e-6 here, the solves to 1e-9
    w = op.material_weights(eps, np.ones(shape))
    for V, H in ((Vh, Hh), (Vd, Hd)):
        Vn = V.T
        assert np.abs(Vn.T @ (w[:, None] * Vn) - np.eye(m + 1)).max() <= 1e-10
        AV = np.stack([op.apply_A(eps, np.ones(shape), sig, Vn[:, j]) for j in range(m)], axis=1)
        assert np.abs(AV - Vn @ H).max() <= 1e-11 * np.abs(AV).max()
    assert np.abs(Vd - Vh).max() <= 1e-6 * np.abs(Vh).max()
    assert np.abs(Hd - Hh).max() <= 1e-6 * np.abs(Hh).max()
    assert _rel(yd, yh) <= 1e-9


@pytest.mark.parametrize("m,s_step", [(32, 16), (30, 8), (64, 32)])
def test_sstep_arnoldi_fp32_storage(m, s_step):
    # FP32 storage: the Chebyshev block and both Gram-Schmidt passes are
    # FP64, only the orthonormal result is rounded to FP32, so the relation
    # and the orthogonality hold to FP32 rounding
    _announce(f"s-step arnoldi fp32 storage m={m} s={s_step}")
    wl = wk.small(12, seed=4, n_spheres=5)
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=m, storage="f32", s_step=s_step)
    v = wk.random_state(wl.n, 9)
    V, H, beta, steps = s.arnoldi(_t(v), m)
    assert steps == m
    V = V.cpu().numpy().astype(np.float64).T
    w = op.material_weights(inp.eps, inp.mu)
    G = V.T @ (w[:, None] * V)
    assert np.abs(G - np.eye(m + 1)).max() <= 2e-6
    AV = np.stack([op.apply_A(inp.eps, inp.mu, inp.sigma, V[:, j]) for j in range(m)], axis=1)
    assert np.abs(AV - V @ H).max() <= 2e-6 * np.abs(AV).max()
    Vo, Ho, bo = okr.krylov_basis(inp.eps, inp.mu, inp.sigma, v, 5)
    assert np.abs(H[:6, :5] - Ho).max() <= 1e-5 * np.abs(Ho).max()


def test_delayed_equals_classical_twice():
    _announce("arnoldi delayed vs cgs2")
    wl = wk.C1
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0).real
    out = {}
    for orth in ("delayed", "cgs2"):
        s = _solver(inp.eps, None, inp.sigma, krylov_dim=40, orth=orth)
        V, H, beta, steps = s.arnoldi(_t(b), 40)
        out[orth] = (V.cpu().numpy(), H, beta, steps)
    Vd, Hd, bd, sd = out["delayed"]
    Vc, Hc, bc, sc = out["cgs2"]
    assert sd == sc == 40
    assert abs(bd - bc) <= 1e-14 * bc
    assert np.abs(Hd - Hc).max() <= 1e-11 * np.abs(Hc).max()
    assert np.abs(Vd - Vc).max() <= 1e-10 * np.abs(Vc).max()


@pytest.mark.parametrize("orth,s_step", [("delayed", 0), ("cgs2", 0), ("delayed", 8)])
def test_arnoldi_happy_breakdown_on_separable_mode(orth, s_step):
    _announce(f"arnoldi breakdown ({orth}, s_step {s_step})")
    N = 6
    ones = np.ones((N, N, N))
    D = np.diag(-np.ones(N)) + np.diag(np.ones(N - 1), 1)
    U, S, Vt = np.linalg.svd(D)
    qx, qy, qz = 1, 2, 4
    # Ex mode: u along x, w along y and z
    ex = np.einsum("k,j,i->kji", Vt[qz], Vt[qy], U[:, qx])
    v = np.zeros((6, N, N, N))
    v[3] = ex
    s = _solver(2.0 * ones, None, 0.1 * ones, krylov_dim=20, orth=orth, s_step=s_step)
    V, H, beta, steps = s.arnoldi(_t(v.reshape(-1)), 20)
    assert 1 <= steps <= 6
    Vn = V.cpu().numpy()
    assert np.all(np.isfinite(Vn)) and np.all(np.isfinite(H))


# ------------------------------------------------------------ exponential --

@pytest.mark.parametrize("N,t,s_step", [(8, 13.0, 0), (12, 40.0, 0), (12, 40.0, 8)])
def test_expv_matches_oracle(N, t, s_step):
    _announce(f"expv N={N} t={t} s_step {s_step}")
    wl = wk.small(N, seed=N, n_spheres=4)
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-10, s_step=s_step)
    rng = np.random.default_rng(5)
    v = rng.standard_normal((2, wl.n))
    y = s.expv(t, _t(v)).cpu().numpy()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for c in range(2):
        assert _rel(y[c], osv.expv(A, t, v[c])) <= 1e-9


# ------------------------------------------------------- stationary part --

@pytest.mark.parametrize("s_step,n_omega", [(0, 3), (8, 3), (8, 10), (16, 16)])
def test_stationary_multishift_matches_oracle(s_step, n_omega):
    # the band is split into groups of neighbouring shifts, each group
    # sharing one Krylov space per cycle
    _announce(f"stationary multishift s_step {s_step} n_omega {n_omega}")
    wl = wk.small(8, seed=2, n_spheres=4, layer=2)
    inp = wk.generate(wl)
    om = list(2 * math.pi * np.linspace(0.08, 0.12, n_omega))
    b = wk.source_vector(wl, om[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-11, s_step=s_step)
    z = s.stationary(om, _t(b[None, :])).cpu().numpy()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for k, w in enumerate(om):
        assert _rel(z[k], osv.stationary(A, b, w)) <= 1e-9


def test_stationary_complex_source_per_omega():
    _announce("stationary complex per-omega")
    wl = wk.small(8, seed=3, n_spheres=4, layer=2)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.09, 2 * math.pi * 0.11]
    th = 0.35
    B = np.stack([wk.source_vector(wl, w, th) for w in om])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=24, tol=1e-11)
    z = s.stationary(om, _t(B), b_per_omega=True).cpu().numpy()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for k, w in enumerate(om):
        assert _rel(z[k], osv.stationary(A, B[k], w)) <= 1e-9


# ----------------------------------------------------------- full solves --

@pytest.mark.parametrize("s_step", [0, 8])
def test_solve_c1_matches_oracle(s_step):
    wl = wk.C1
    _announce(f"solve c1 16^3 s_step {s_step}")
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol, s_step=s_step)
    y = s.solve_multifreq(wl.omegas, _t(b[None, :]), wl.T).cpu().numpy()[0]
    st = s.last_stats
    assert st["converged"] == 1
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y_or = osv.split_solution(A, b, wl.omegas[0], wl.T)[0]
    assert _rel(y, y_or) <= 1e-8


def test_solve_multi_source_multi_omega():
    _announce("solve multi source")
    wl = wk.small(9, seed=6, n_spheres=5, layer=2, T=60.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.085, 2 * math.pi * 0.115]
    srcs = np.stack([wk.source_vector(wl, om[0], 0.0), wk.source_vector(wl, om[0], 0.3)])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-9)
    y = s.solve_multifreq(om, _t(srcs), wl.T).cpu().numpy()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for k, w in enumerate(om):
        for si in range(2):
            ref = osv.augmented_solution(A, srcs[si], w, wl.T)
            assert _rel(y[k * 2 + si], ref) <= 1e-8


@pytest.mark.parametrize("s_step", [0, 8])
def test_solve_fp32_storage(s_step):
    _announce(f"solve fp32 storage s_step {s_step}")
    wl = wk.small(12, seed=7, n_spheres=6, layer=2, T=80.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.1]
    b = wk.source_vector(wl, om[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-6, storage="f32", s_step=s_step)
    y = s.solve_multifreq(om, _t(b[None, :]), wl.T).cpu().numpy()[0]
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y_or = osv.split_solution(A, b, om[0], wl.T)[0]
    assert _rel(y, y_or) <= 1e-5


@pytest.mark.parametrize("mode", ["omega_continuation"])
def test_batched_multifreq_modes_match_oracle(mode):
    # per-frequency oblique sources at nine neighbouring frequencies and two
    # angles.  omega_continuation starts each shifted solve from the
    # extrapolation of the earlier frequencies' solutions: the plain fields
    # with fewer operator applications; a zero source column stays zero.
    _announce(f"batched multi-frequency: {mode}")
    wl = wk.small(10, seed=31, n_spheres=5, layer=2, T=50.0)
    inp = wk.generate(wl)
    om = list(2 * math.pi * np.linspace(0.09, 0.11, 9))
    th = [0.2, 0.45]
    B = np.stack([wk.source_vector(wl, w, t) for w in om for t in th])
    B[3] = 0.0
    out = {}
    for on in (False, True):
        s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-9, **{mode: on})
        out[on] = (s.solve_multifreq(om, _t(B), wl.T, b_per_omega=True).cpu().numpy(),
                   s.last_stats)
        s.close()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for on in (False, True):
        y = out[on][0]
        assert np.all(y[3] == 0.0)
        for col in range(len(B)):
            if col == 3:
                continue
            k, t = divmod(col, len(th))
            ref = osv.augmented_solution(A, B[col], om[k], wl.T)
            assert _rel(y[col], ref) <= 1e-8, (on, col)
        assert out[on][1]["converged"] == 1
    assert out[True][1]["matvecs_stationary"] < out[False][1]["matvecs_stationary"]
    _announce(f"matvecs plain {out[False][1]['matvecs_stationary']} "
              f"{mode} {out[True][1]['matvecs_stationary']}")


# ------------------------------------------------------------ edge cases --

def test_zero_source_zero_time_and_errors():
    _announce("edge cases")
    kry = _kry()
    wl = wk.small(5, seed=8, n_spheres=2, layer=1)
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=10, tol=1e-10)
    zero = np.zeros((1, wl.n), dtype=np.complex128)
    y = s.solve_multifreq([0.6], _t(zero), 30.0).cpu().numpy()
    assert np.all(y == 0.0)
    b = wk.source_vector(wl, 0.6, 0.0)
    y0 = s.solve_multifreq([0.6], _t(b[None, :]), 0.0).cpu().numpy()
    assert np.abs(y0).max() <= 1e-10 * np.abs(b).max()
    bad = inp.eps.copy()
    bad[0, 0, 0] = 0.0
    with pytest.raises(kry.KryError, match="EINVAL"):
        _solver(bad, None, inp.sigma)
    nan = inp.sigma.copy()
    nan[1, 1, 1] = float("nan")
    with pytest.raises(kry.KryError, match="EINVAL"):
        _solver(inp.eps, None, nan)
    with pytest.raises(kry.KryError, match="EINVAL"):
        s.solve_multifreq([-1.0], _t(b[None, :]), 1.0)


def test_bitwise_reproducible():
    _announce("determinism")
    wl = wk.small(10, seed=9, n_spheres=4, layer=2, T=30.0)
    inp = wk.generate(wl)
    b = wk.source_vector(wl, 0.6, 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=20, tol=1e-9)
    y1 = s.solve_multifreq([0.6], _t(b[None, :]), wl.T).cpu().numpy()
    y2 = s.solve_multifreq([0.6], _t(b[None, :]), wl.T).cpu().numpy()
    assert np.array_equal(y1, y2)


# ------------------------------------------------------ full-size c2 run --

GOLD_C2 = os.path.join(ROOT, "tests", "golden", "c2_yT_samples.json")


@pytest.mark.skipif(not os.path.exists(GOLD_C2), reason="c2 oracle samples not generated")
def test_solve_c2_against_oracle_samples():
    wl = wk.C2
    _announce("solve c2 128^3 (full size)")
    gold = json.load(open(GOLD_C2))
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol)
    t0 = time.time()
    y = s.solve_multifreq(wl.omegas, _t(b[None, :]), wl.T).cpu().numpy()[0]
    _announce(f"c2 solve {time.time() - t0:.2f}s stats={s.last_stats}")
    col = gold["columns"][0]
    idx = np.asarray(gold["indices"])
    ref = np.asarray(col["values"])
    nrm = col["norm2"]
    assert np.linalg.norm(y[idx] - ref) <= 1e-8 * np.linalg.norm(ref)
    assert abs(np.linalg.norm(y) - nrm) <= 1e-8 * nrm
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_golden import projection_vector
    for k, p in enumerate(col["projections"]):
        assert abs(projection_vector(wl.n, k) @ y - p) <= 4e-8 * nrm


GOLD_C3 = os.path.join(ROOT, "tests", "golden", "c3_yT_samples.json")


@pytest.mark.skipif(not os.path.exists(GOLD_C3), reason="c3 oracle samples not generated")
def test_batched_c3_against_oracle_samples():
    """Batched form at 96^3: four (omega, angle) columns of the 256-column
    block, each with its own complex phase-ramp source, solved together in
    one block Krylov space and compared with oracle samples."""
    wl = wk.C3
    _announce("batched solve c3 96^3, 4 golden columns, block width 8")
    gold = json.load(open(GOLD_C3))
    inp = wk.generate(wl)
    cols = gold["columns"]
    om = [wl.omegas[c["omega_index"]] for c in cols]
    B = np.stack([wk.source_vector(wl, wl.omegas[c["omega_index"]],
                                   float(inp.thetas[c["theta_index"]])) for c in cols])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol,
                block_width=8, block_steps=16)
    t0 = time.time()
    y = s.solve_multifreq(om, _t(B), wl.T, b_per_omega=True).cpu().numpy()
    _announce(f"c3 batched solve {time.time() - t0:.2f}s stats={s.last_stats}")
    idx = np.asarray(gold["indices"])
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_golden import projection_vector
    P = [projection_vector(wl.n, k) for k in range(len(cols[0]["projections"]))]
    for k, col in enumerate(cols):
        assert abs(col["omega"] - om[k]) <= 1e-15 * om[k]
        ref = np.asarray(col["values"])
        nrm = col["norm2"]
        assert np.linalg.norm(y[k, idx] - ref) <= 1e-8 * np.linalg.norm(ref)
        assert abs(np.linalg.norm(y[k]) - nrm) <= 1e-8 * nrm
        for p, pr in zip(P, col["projections"]):
            assert abs(p @ y[k] - pr) <= 4e-8 * nrm


def _check_c2_samples(y, label):
    gold = json.load(open(GOLD_C2))
    col = gold["columns"][0]
    idx = np.asarray(gold["indices"])
    ref = np.asarray(col["values"])
    nrm = col["norm2"]
    err = float(np.linalg.norm(y[idx] - ref) / np.linalg.norm(ref))
    _announce(f"{label}: sampled rel err {err:.2e}")
    assert err <= 1e-8
    assert abs(np.linalg.norm(y) - nrm) <= 1e-8 * nrm
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_golden import projection_vector
    for k, p in enumerate(col["projections"]):
        assert abs(projection_vector(y.size, k) @ y - p) <= 4e-8 * nrm


@pytest.mark.parametrize("method", ["restarted", "split2"])
def test_other_methods_c2_against_oracle_samples(method):
    # the 128^3 workload (T = 500, tol 1e-8) by the residual-restarted method
    # and by source splitting (5 periods per subinterval), no shifted solve
    wl = wk.C2
    _announce(f"c2 128^3 (full size) by {method}")
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol)
    t0 = time.time()
    if method == "restarted":
        y = s.solve_restarted(wl.omegas, b, wl.T)
    else:
        y = s.solve_split2(wl.omegas, b, wl.T, periods=5)
    y = y.cpu().numpy()[0]
    _announce(f"c2 {method} {time.time() - t0:.2f}s stats={s.last_stats}")
    s.close()
    _check_c2_samples(y, f"c2 {method}")


def test_c2_three_routes_agree_on_the_whole_field():
    # the 128^3 workload by the split (Corollary 3), the residual-restarted
    # method and source splitting: three routes that share no step beyond
    # the operator and Arnoldi kernels; each is pinned to the stored oracle
    # samples elsewhere, here their whole 12.6M-entry fields agree
    wl = wk.C2
    _announce("c2 128^3: split, restarted and source splitting on the whole field")
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol)
    y1 = s.solve_multifreq(wl.omegas, b, wl.T)[0]
    y2 = s.solve_restarted(wl.omegas, b, wl.T)[0]
    y3 = s.solve_split2(wl.omegas, b, wl.T, periods=5)[0]
    s.close()
    n1 = float(torch.linalg.norm(y1))
    d12 = float(torch.linalg.norm(y1 - y2)) / n1
    d13 = float(torch.linalg.norm(y1 - y3)) / n1
    _announce(f"c2 whole field: split vs restarted {d12:.2e}, split vs source splitting {d13:.2e}")
    # each route stops at relative error tol = 1e-8, so two of them differ by
    # at most twice that
    assert d12 <= 2e-8 and d13 <= 2e-8


def test_sstep_basis_orthogonality_at_full_size():
    # s-step Arnoldi (s = 16, one Gram-Schmidt pass where the block's
    # condition estimate allows) on the 128^3 medium from its plane source,
    # m = 64: the basis is M-orthonormal to 1e-10 and satisfies the Arnoldi
    # relation at full size, where the skipped second passes happen
    wl = wk.C2
    _announce("s-step basis orthogonality at 128^3")
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=64, tol=1e-8, s_step=16)
    v = _t(wk.source_vector(wl, wl.omegas[0], 0.0).real)
    V, H, beta, steps = s.arnoldi(v, 64)
    assert steps == 64
    w = _t(op.material_weights(inp.eps, inp.mu))
    G = (V * w) @ V.T
    orth = float((G - torch.eye(65, dtype=G.dtype, device=G.device)).abs().max())
    AV = s.apply(V[:64].contiguous())
    Ht = torch.as_tensor(H, device=V.device)
    rel = float(torch.linalg.norm(AV - Ht.T @ V) / torch.linalg.norm(AV))
    s.close()
    _announce(f"128^3 s-step basis: max |V^T M V - I| {orth:.2e}, Arnoldi relation {rel:.2e}")
    assert orth <= 1e-10 and rel <= 1e-12


@pytest.mark.skipif(not os.path.exists(GOLD_C3), reason="c3 oracle samples not generated")
def test_batched_c3_all_columns_restarted_against_oracle_samples():
    """The batched workload as configured: all 256 columns (32 frequencies x
    8 angles, one oblique source each) solved together by the restarted
    method through one compressed basis of the sources; the 4 columns with
    stored oracle samples compared."""
    wl = wk.C3
    _announce("batched c3 96^3, all 256 columns, restarted method")
    gold = json.load(open(GOLD_C3))
    inp = wk.generate(wl)
    nth = len(inp.thetas)
    B = np.stack([wk.source_vector(wl, w, float(t)) for w in wl.omegas for t in inp.thetas])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol)
    t0 = time.time()
    y = s.solve_restarted(list(wl.omegas), _t(B), wl.T, b_per_omega=True)
    _announce(f"c3 all columns {time.time() - t0:.2f}s stats={s.last_stats}")
    s.close()
    idx = np.asarray(gold["indices"])
    for col in gold["columns"]:
        yk = y[col["omega_index"] * nth + col["theta_index"]].cpu().numpy()
        ref = np.asarray(col["values"])
        assert np.linalg.norm(yk[idx] - ref) <= 1e-8 * np.linalg.norm(ref)
        assert abs(np.linalg.norm(yk) - col["norm2"]) <= 1e-8 * col["norm2"]


# ---------------------------------------------------------- differentiation --

@pytest.mark.parametrize("cont", [False, True])
def test_grad_matches_oracle_adjoint_and_fd(cont):
    # cont: the adjoint solves start from the extrapolation of the earlier
    # frequencies' adjoint solutions
    _announce(f"gradient vs oracle (omega continuation {cont})")
    from oracle import grad as og
    N, kf = 7, 5
    wl = wk.small(N, seed=22, n_spheres=3, layer=1, radius=(0.8, 1.6),
                  omegas=(2 * math.pi * 0.09, 2 * math.pi * 0.1, 2 * math.pi * 0.11), src_k=1)
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-12, omega_continuation=cont)
    L, g = s.grad(wl.omegas, _t(b[None, :]), kf)
    g = g.cpu().numpy()
    b_cols = np.stack([b] * len(wl.omegas), axis=1)
    Lo, go = og.loss_and_grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf)
    assert abs(L - Lo) <= 1e-10 * abs(Lo)
    assert np.linalg.norm(g - go) <= 1e-8 * np.linalg.norm(go)
    cells = [(1, 2, 3), (3, 3, 2), (5, 1, 4), (2, 5, 3)]
    fd = og.fd_grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, kf, cells, h=1e-5)
    gv = np.array([g[k, j, i] for (i, j, k) in cells])
    assert np.linalg.norm(gv - fd) <= 1e-6 * np.linalg.norm(fd)


def test_grad_per_omega_sources_and_autograd():
    _announce("gradient per-omega + autograd")
    from oracle import grad as og
    kry = _kry()
    N, kf = 6, 4
    om = (2 * math.pi * 0.1, 2 * math.pi * 0.105)
    wl = wk.small(N, seed=23, n_spheres=2, layer=1, radius=(0.8, 1.4), omegas=om, src_k=1)
    inp = wk.generate(wl)
    B = np.stack([wk.source_vector(wl, w, 0.3) for w in om])
    eps_t = _t(inp.eps).requires_grad_(True)
    L = kry.flux_loss(eps_t, _t(inp.sigma), _t(B), om, kf,
                      kry.Options(krylov_dim=30, tol=1e-12), b_per_omega=True)
    L.backward()
    Lo, go = og.loss_and_grad(inp.eps, inp.mu, inp.sigma, B.T.copy(), om, kf)
    assert abs(L.item() - Lo) <= 1e-10 * abs(Lo)
    g = eps_t.grad.cpu().numpy()
    assert np.linalg.norm(g - go) <= 1e-8 * np.linalg.norm(go)


def test_grad_16cube_full_vector_against_oracle():
    # the whole gradient vector (4096 cells, 16 workgroups per plane sweep)
    # and the loss for two frequencies against the oracle's SuperLU forward
    # and explicit-transpose adjoint solves (tests/golden/grad16_oracle.json,
    # written by tests/golden/make_golden.py grad16)
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_golden import grad16_workload
    with open(os.path.join(ROOT, "tests", "golden", "grad16_oracle.json")) as f:
        ref = json.load(f)
    wl = grad16_workload()
    _announce("gradient 16^3, two frequencies, full vector vs oracle")
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    assert list(wl.omegas) == ref["omegas"] and wl.flux_plane == ref["plane_k"]
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=1e-12)
    L, g = s.grad(wl.omegas, _t(b[None, :]), wl.flux_plane)
    s.close()
    go = np.asarray(ref["grad"])
    assert abs(L - ref["loss"]) <= 1e-10 * abs(ref["loss"])
    assert _rel(g.cpu().numpy().reshape(-1), go) <= 1e-8


def _flux_increment(z, d, N, kf):
    """P(z + d) - P(z) for the period-averaged flux 1/2 Re sum [Ex conj(Hy_bar)
    - Ey conj(Hx_bar)] through plane kf (H_bar the mean of the H planes kf-1
    and kf), from its cross terms: the flux is a real quadratic form in z, so
    the increment needs no difference of two large fluxes.  z, d: complex
    device tensors of length 6 N^3."""
    Z = z.view(6, N, N, N)
    D = d.view(6, N, N, N)

    def hbar(V, c):
        return 0.5 * (V[c, kf - 1] + V[c, kf])

    def pair(E, H):
        return torch.sum(E[3, kf] * torch.conj(hbar(H, 1)) - E[4, kf] * torch.conj(hbar(H, 0)))

    return 0.5 * float(torch.real(pair(D, Z) + pair(Z, D) + pair(D, D)))


def test_grad_c4_full_size_against_difference_solves():
    # 64^3, 8 frequencies, flux plane 58, 20 seeded cells, central
    # differences with step h = 1e-6.  Each difference L(eps +- h e_c) - L(eps)
    # comes from one exact difference solve per frequency: with A+- the
    # operator of the perturbed medium, z+- = z + d+- where
    # (A+- + i w) d+- = -(A+- - A) z, and -(A+- - A) z is non-zero only on the
    # three E edges of cell c, where it is (1 - eps / (eps +- h)) (A z)_e.  The flux
    # increment then follows from z and d+- directly, so the central
    # difference carries no cancellation between two full solves and its
    # error is the solve tolerance, not eps_mach L / (h |g|).
    wl = wk.C4
    h = 1e-6
    N = wl.N
    kf = wl.flux_plane
    _announce(f"gradient c4 64^3 (full size), difference solves, h = {h:g}")
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=1e-12)
    t0 = time.time()
    L, g = s.grad(wl.omegas, b, kf)
    _announce(f"c4 grad {time.time() - t0:.1f}s L={L:.6e} stats={s.last_stats}")
    g = g.cpu().numpy()
    z = s.stationary(wl.omegas, b)  # (8, n) complex
    # the flux written out here agrees with the library's loss
    Lz = sum(_flux_increment(torch.zeros_like(z[k]), z[k], N, kf) for k in range(len(wl.omegas)))
    assert abs(Lz - L) <= 1e-10 * abs(L)
    Az = torch.complex(s.apply(z.real.contiguous()), s.apply(z.imag.contiguous()))
    s.close()
    n3 = N ** 3
    gv = np.array([g[k, j, i] for (i, j, k) in inp.fd_cells])
    fd = []
    t0 = time.time()
    for n_done, (i, j, k) in enumerate(inp.fd_cells):
        cell = (k * N + j) * N + i
        e0 = float(inp.eps[k, j, i])
        dP = []
        for sgn in (1.0, -1.0):
            e = inp.eps.copy()
            e[k, j, i] += sgn * h
            rhs = torch.zeros_like(z)
            for comp in (3, 4, 5):
                idx = comp * n3 + cell
                rhs[:, idx] = (1.0 - e0 / float(e[k, j, i])) * Az[:, idx]
            sp = _solver(e, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=1e-12)
            d = sp.stationary(wl.omegas, rhs, b_per_omega=True)
            sp.close()
            dP.append(sum(_flux_increment(z[q], d[q], N, kf) for q in range(len(wl.omegas))))
        fd.append((dP[0] - dP[1]) / (2 * h))
        if n_done % 5 == 4:
            _announce(f"c4 fd: {n_done + 1} of {len(inp.fd_cells)} cells, {time.time() - t0:.0f}s")
    fd = np.array(fd)
    err = float(np.linalg.norm(gv - fd) / np.linalg.norm(fd))
    per_cell = np.abs(gv - fd) / np.abs(fd)
    _announce(f"c4 fd h={h:g}: rel err {err:.3e}, worst cell {per_cell.max():.3e}")
    assert err <= 1e-5


# --------------------------------------------------- per-column records --

def test_column_stats_and_norm_series():
    # per-column records of a split solve: three frequencies of one source.
    # The transient's |y_hat(t)|_M decays (A is dissipative in the energy
    # norm), starts at |Im z|_M and ends at |e^{-TA} Im z|_M (oracle); the
    # per-column operator applications add up to the call's totals
    kry = _kry()
    wl = wk.small(10, seed=12, n_spheres=4, layer=2, radius=(0.8, 1.5), src_k=1, T=30.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.09, 2 * math.pi * 0.1, 2 * math.pi * 0.11]
    b = wk.source_vector(wl, om[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-10)
    s.solve_multifreq(om, _t(b[None, :]), wl.T)
    tot = s.last_stats
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    w = op.material_weights(inp.eps, inp.mu)
    mv = 0
    for k, omega in enumerate(om):
        cs = s.column_stats(k)
        t, nrm, ms = s.norm_series(k)
        mv += cs["matvecs_transient"]
        assert cs["omega"] == omega and cs["source"] == 0 and cs["converged"] == 1
        assert cs["matvecs_stationary"] == tot["matvecs_stationary"]  # one group
        assert cs["residual"] <= 0.1 * 1e-10
        assert cs["series_len"] == len(t) == cs["steps_transient"] + 1
        z = osv.stationary(A, b, omega)
        yh = osv.expv(A, wl.T, np.imag(z))
        assert t[0] == 0.0 and t[-1] == wl.T and np.all(np.diff(t) > 0)
        assert abs(nrm[0] - math.sqrt(np.imag(z) @ (w * np.imag(z)))) <= 1e-9 * nrm[0]
        assert abs(nrm[-1] - math.sqrt(yh @ (w * yh))) <= 1e-9 * nrm[0]
        assert np.all(np.diff(nrm) <= 1e-10 * nrm[0])
        assert np.all(ms[:-1] > 0) and ms[-1] == 0.0
    assert mv == tot["matvecs_transient"]
    with pytest.raises(kry.KryError):
        s.column_stats(3)
    s.close()


# ------------------------------------- flux at a finite time T (NEXT-3) --

def _tgrad_ref():
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_golden import tgrad_direction, tgrad_workloads
    with open(os.path.join(ROOT, "tests", "golden", "tgrad_oracle.json")) as f:
        ref = json.load(f)
    return ref, tgrad_workloads(), tgrad_direction


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, "tests", "golden", "tgrad_oracle.json")),
                    reason="finite-time gradient oracle values not generated")
def test_grad_transient_5cube_full_vector_against_oracle():
    # the whole gradient (125 cells, two frequencies, T = 12) of the flux of
    # the field at time T against the oracle's per-cell forward derivatives
    # (dense LU and the Frechet derivative of expm), and the loss
    ref, (w5, _, T, _), _ = _tgrad_ref()
    r = ref["small"]
    _announce(f"finite-time flux gradient 5^3 vs oracle, T = {T}")
    inp = wk.generate(w5)
    b = wk.source_vector(w5, w5.omegas[0], 0.0)
    assert list(w5.omegas) == r["omegas"] and w5.flux_plane == r["plane_k"] and T == ref["T"]
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=w5.krylov_dim, tol=1e-12)
    L, g = s.grad_transient(w5.omegas, _t(b[None, :]), w5.flux_plane, T)
    st = s.last_stats
    s.close()
    go = np.asarray(r["grad"])
    err = _rel(g.cpu().numpy().reshape(-1), go)
    _announce(f"5^3: loss {L:.10e} (oracle {r['loss']:.10e}), gradient rel err {err:.2e}, stats {st}")
    assert abs(L - r["loss"]) <= 1e-9 * abs(r["loss"])
    assert err <= 1e-8


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, "tests", "golden", "tgrad_oracle.json")),
                    reason="finite-time gradient oracle values not generated")
def test_grad_transient_15cube_directional_against_oracle():
    # 15^3 (3375 cells: 14 workgroups, a ragged last one): the loss and the
    # gradient along three seeded random permittivity changes against the
    # oracle's forward derivatives (SuperLU, expm_multiply, 2n block identity)
    ref, (_, w15, T, ndir), direction = _tgrad_ref()
    r = ref["medium"]
    _announce(f"finite-time flux gradient 15^3, directional vs oracle, T = {T}")
    inp = wk.generate(w15)
    b = wk.source_vector(w15, w15.omegas[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=w15.krylov_dim, tol=1e-12)
    L, g = s.grad_transient(w15.omegas, _t(b[None, :]), w15.flux_plane, T)
    s.close()
    g = g.cpu().numpy()
    assert abs(L - r["loss"]) <= 1e-9 * abs(r["loss"])
    gnorm = np.linalg.norm(g)
    for k in range(ndir):
        d = direction(w15.N, k)
        dd = float((g * d).sum())
        _announce(f"15^3 direction {k}: {dd:.10e} (oracle {r['directional'][k]:.10e})")
        assert abs(dd - r["directional"][k]) <= 1e-8 * gnorm * np.linalg.norm(d)


def _flux_real(y, N, kf):
    """Instantaneous flux sum [Ex Hy_bar - Ey Hx_bar] of a real device field
    through plane kf (H_bar the mean of the H planes kf - 1 and kf)."""
    Y = y.view(6, N, N, N)
    hx = 0.5 * (Y[0, kf - 1] + Y[0, kf])
    hy = 0.5 * (Y[1, kf - 1] + Y[1, kf])
    return float(torch.sum(Y[3, kf] * hy - Y[4, kf] * hx))


def test_grad_transient_full_size_directional_differences():
    # the 64^3 medium of the gradient workload, two of its frequencies,
    # T = 60: the adjoint gradient along two random permittivity changes
    # against central differences of the loss.  Two independent shifted
    # solves differ by far more than their residual target (the systems are
    # ill-conditioned near the cavity's resonances), so the perturbed z come
    # from exact difference solves, z+- = z + d+- with (A+- + i w) d+- =
    # -(A+- - A) z, which is (1 - eps / (eps +- h d)) (A z) on the E edges;
    # the transients e^{-T A+-} Im z+- are computed on the perturbed media,
    # and the flux of y+-(T) follows.  The loss still carries ~1e-9 of
    # noise (the flux is a small sum of large plane products, and each
    # transient's error is independent), which steps of 1e-5 turn into
    # 2e-5 of the derivative whatever the transients' tolerance; so steps of
    # 5e-4 and 1e-3 are taken and combined by Richardson extrapolation,
    # (4 D(h) - D(2h)) / 3, which removes the O(h^2) truncation
    wl = wk.C4
    N, kf, T, h = wl.N, wl.flux_plane, 60.0, 5e-4
    om = list(wl.omegas[::4])
    n3 = N ** 3
    _announce(f"finite-time flux gradient 64^3, T = {T}, directional central differences")
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=1e-13)
    t0 = time.time()
    L, g = s.grad_transient(om, b, kf, T)
    _announce(f"64^3 finite-time gradient {time.time() - t0:.1f}s L={L:.6e} stats={s.last_stats}")
    g = g.cpu().numpy()
    z = s.stationary(om, b)  # (2, n) complex
    Az = torch.complex(s.apply(z.real.contiguous()), s.apply(z.imag.contiguous()))

    def loss_of(zz, solver):
        tot = 0.0
        for q, w in enumerate(om):
            yh = solver.expv(T, zz[q].imag.contiguous())[0]
            y = torch.imag(np.exp(1j * w * T) * zz[q]) - yh
            tot += _flux_real(y, N, kf)
        return tot

    # the flux written out here agrees with the library's loss
    L0 = loss_of(z, s)
    _announce(f"64^3 loss written out {L0:.12e}, library {L:.12e}")
    # z here and inside the library come from two independent solves, which
    # differ by more than their residual target near the resonances (above);
    # the two losses have been seen 5e-11 to 3e-10 apart, with the loss's
    # own noise near 1e-9
    assert abs(L0 - L) <= 2e-9 * abs(L)
    s.close()
    rng = np.random.default_rng(77)
    eps_t = _t(inp.eps.reshape(-1))
    def loss_perturbed(e):
        fac = 1.0 - eps_t / _t(e.reshape(-1))
        rhs = torch.zeros_like(z)
        for comp in (3, 4, 5):
            rhs[:, comp * n3:(comp + 1) * n3] = fac * Az[:, comp * n3:(comp + 1) * n3]
        sp = _solver(e, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=1e-13)
        dz = sp.stationary(om, rhs, b_per_omega=True)
        out = loss_of(z + dz, sp)
        sp.close()
        return out

    for k in range(2):
        d = rng.standard_normal(inp.eps.shape)
        D = [(loss_perturbed(inp.eps + a * h * d) - loss_perturbed(inp.eps - a * h * d)) / (2 * a * h)
             for a in (1, 2)]
        fd = (4 * D[0] - D[1]) / 3
        dd = float((g * d).sum())
        _announce(f"64^3 direction {k}: adjoint {dd:.10e}, differences h {D[0]:.10e}, 2h {D[1]:.10e}, "
                  f"extrapolated {fd:.10e}")
        assert abs(dd - fd) <= 1e-5 * abs(fd)


def test_grad_transient_edges_and_autograd():
    kry = _kry()
    wl = wk.small(8, seed=31, n_spheres=3, layer=2, radius=(0.8, 1.5), src_k=1)
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-12)
    # T = 0: y(0) = 0, so the loss and its gradient vanish
    L0, g0 = s.grad_transient(wl.omegas, b, 5, 0.0)
    assert L0 == 0.0 and float(g0.abs().max()) == 0.0
    with pytest.raises(kry.KryError):
        s.grad_transient(wl.omegas, b, 5, -1.0)
    with pytest.raises(kry.KryError):
        s.grad_transient(wl.omegas, b, 0, 5.0)
    L, g = s.grad_transient(wl.omegas, b, 5, 9.0)
    s.close()
    # through torch.autograd: the backward hands the adjoint gradient back
    eps = _t(inp.eps).requires_grad_(True)
    out = kry.flux_loss_at(eps, _t(inp.sigma), b, wl.omegas, 5, 9.0,
                           kry.Options(krylov_dim=30, tol=1e-12))
    out.backward()
    assert abs(float(out) - L) <= 1e-13 * abs(L)
    assert float((eps.grad - g).abs().max()) <= 1e-12 * float(g.abs().max())


# ------------------------------------------------ transient continuation --

@pytest.mark.parametrize("per_omega", [False, True])
def test_transient_continuation_matches_oracle(per_omega):
    # six neighbouring frequencies (a scan): each column's transient after
    # the first is continued from the previous column's (equation (4diff));
    # every column against the oracle's augmented-matrix route at 1e-8, and
    # fewer transient operator applications than the plain transients
    _announce(f"transient continuation (per-omega sources {per_omega})")
    wl = wk.small(12, seed=34, n_spheres=5, layer=2, T=90.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * f for f in np.linspace(0.095, 0.105, 6)]
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    if per_omega:
        B = np.stack([wk.source_vector(wl, w, 0.25) for w in om])
        refs = [osv.augmented_solution(A, B[k], w, wl.T) for k, w in enumerate(om)]
    else:
        B = wk.source_vector(wl, om[0], 0.0)[None, :]
        refs = [osv.augmented_solution(A, B[0], w, wl.T) for w in om]
    mv = {}
    for tc in (False, True):
        s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-10, transient_continuation=tc)
        y = s.solve_multifreq(om, _t(B), wl.T, b_per_omega=per_omega).cpu().numpy()
        mv[tc] = s.last_stats["matvecs_transient"]
        assert s.last_stats["converged"] == 1
        s.close()
        for k in range(len(om)):
            assert _rel(y[k], refs[k]) <= 1e-8
    _announce(f"transient operator applications: plain {mv[False]}, continued {mv[True]}")
    assert mv[True] < mv[False]


def test_continuation_with_coincident_frequencies():
    # per-column sources with a frequency that repeats along one chain: the
    # extrapolation in omega needs distinct nodes, so such a column starts
    # from zero; every column stays finite and matches the oracle
    _announce("continuation with coincident frequencies")
    wl = wk.small(8, seed=37, n_spheres=3, layer=2, T=40.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.1, 2 * math.pi * 0.1, 2 * math.pi * 0.104, 2 * math.pi * 0.104]
    B = np.stack([wk.source_vector(wl, w, 0.1 * k) for k, w in enumerate(om)])
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-10, omega_continuation=True,
                transient_continuation=True)
    y = s.solve_multifreq(om, _t(B), wl.T, b_per_omega=True).cpu().numpy()
    s.close()
    assert np.isfinite(y).all()
    for k, w in enumerate(om):
        assert _rel(y[k], osv.augmented_solution(A, B[k], w, wl.T)) <= 1e-8


# ------------------------------------------ restarted inhomogeneous Krylov --

@pytest.mark.parametrize("m", [30, 64, 80])
def test_restarted_inhomogeneous_c1_matches_oracle(m):
    # m <= 64: projected problems marched on the GPU; m = 80: on the host
    # c1 (16^3, T = 200, tol 1e-10) by the residual-restarted method, with no
    # shifted solve, against the oracle's split solution (SuperLU and
    # expm_multiply)
    wl = wk.C1
    _announce(f"restarted inhomogeneous Krylov c1, m = {m}")
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=m, tol=wl.tol)
    y = s.solve_restarted(wl.omegas, _t(b[None, :]), wl.T).cpu().numpy()[0]
    st = s.last_stats
    _announce(f"restarted c1 m={m}: {st['steps_transient']} restarts, {st['matvecs_transient']} "
              f"operator applications, {st['ms_total']:.0f} ms, error estimate {st['max_err_estimate']:.2e}")
    s.close()
    assert st["converged"] == 1 and st["max_err_estimate"] <= 0.5 * wl.tol
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    y_or = osv.split_solution(A, b, wl.omegas[0], wl.T)[0]
    assert _rel(y, y_or) <= 1e-8


def test_restarted_inhomogeneous_shared_and_per_omega_sources():
    # 10^3, three frequencies, T = 60: a complex source shared by all of them
    # (one sequence of bases per real part serves every frequency) and
    # per-frequency oblique sources, against the oracle's augmented-matrix
    # route per column
    _announce("restarted inhomogeneous Krylov, several frequencies and sources")
    wl = wk.small(10, seed=33, n_spheres=4, layer=2, T=60.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * f for f in (0.09, 0.1, 0.115)]
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=40, tol=1e-10)
    srcs = [wk.source_vector(wl, om[0], 0.35), wk.source_vector(wl, om[1], 0.0)]
    y = s.solve_restarted(om, _t(np.stack(srcs)), wl.T).cpu().numpy()
    st = s.last_stats
    assert st["converged"] == 1
    for k, w in enumerate(om):
        for si, bs in enumerate(srcs):
            ref = osv.augmented_solution(A, bs, w, wl.T)
            assert _rel(y[k * len(srcs) + si], ref) <= 1e-8
    B = np.stack([wk.source_vector(wl, w, 0.2) for w in om])
    y = s.solve_restarted(om, _t(B), wl.T, b_per_omega=True).cpu().numpy()
    for k, w in enumerate(om):
        assert _rel(y[k], osv.augmented_solution(A, B[k], w, wl.T)) <= 1e-8
    # a restart cap returns the current approximation with KRY_ENOCONV
    s.close()
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=10, tol=1e-10, max_restarts=2)
    kry = _kry()
    with pytest.raises(kry.NotConverged):
        s.solve_restarted(om, _t(np.stack(srcs)), wl.T)
    y = s.solve_restarted(om, _t(np.stack(srcs)), wl.T, allow_noconv=True)
    assert torch.isfinite(y).all() and s.last_stats["max_err_estimate"] > 1e-10
    s.close()


def test_restarted_per_column_sources_share_a_compressed_basis():
    # 5 frequencies x 3 oblique angles, one source per column (the batched
    # recipe at 10^3): the sources are spanned by a few real vectors, each of
    # which drives one time function per column, so a handful of sequences
    # of bases serve all 15 columns; every column against the oracle, and
    # fewer restarts than two sequences per column
    _announce("restarted method, per-column sources through a compressed basis")
    wl = wk.small(10, seed=36, n_spheres=4, layer=2, T=50.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * f for f in np.linspace(0.09, 0.11, 5)]
    th = [0.0, 0.2, 0.45]
    B = np.stack([wk.source_vector(wl, w, t) for w in om for t in th])
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=40, tol=1e-10)
    y = s.solve_restarted(om, _t(B), wl.T, b_per_omega=True).cpu().numpy()
    st = s.last_stats
    assert st["converged"] == 1
    for k, w in enumerate(om):
        for i in range(len(th)):
            col = k * len(th) + i
            assert _rel(y[col], osv.augmented_solution(A, B[col], w, wl.T)) <= 1e-8
    restarts_shared = st["steps_transient"]
    one = 0
    for col in (0, 7, 14):  # columns solved alone: two sequences each (Re and Im)
        s.solve_restarted([om[col // 3]], _t(B[col:col + 1]), wl.T, b_per_omega=True)
        one += s.last_stats["steps_transient"]
    s.close()
    _announce(f"restarts: 15 columns together {restarts_shared}, 3 columns alone {one}")
    assert restarts_shared < 5 * one


@pytest.mark.parametrize("storage,tol,bound", [("f64", 1e-10, 1e-8), ("f32", 2e-6, 1e-5)])
def test_restarted_many_columns_matrix_core_combination(storage, tol, bound):
    # 10 frequencies x 7 angles (70 columns: two full groups of 32 outputs
    # and a ragged third; 6^3 gives 1296 entries, a partial last block of
    # 32): the restarted method's basis combination for many time functions
    # runs on the matrix cores, with FP64 or FP32 storage; every column
    # against the oracle (dense route at 6^3)
    _announce(f"restarted method, 70 columns, matrix-core combination, {storage}")
    wl = wk.small(6, seed=37, n_spheres=2, layer=1, T=40.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * f for f in np.linspace(0.09, 0.11, 10)]
    th = [0.0, 0.1, 0.2, 0.3, 0.35, 0.4, 0.5]
    B = np.stack([wk.source_vector(wl, w, t) for w in om for t in th])
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=40, tol=tol, storage=storage)
    y = s.solve_restarted(om, _t(B), wl.T, b_per_omega=True).cpu().numpy()
    assert s.last_stats["converged"] == 1
    s.close()
    worst = 0.0
    for k, w in enumerate(om):
        for i in range(len(th)):
            col = k * len(th) + i
            worst = max(worst, _rel(y[col], osv.augmented_solution(A, B[col], w, wl.T)))
    _announce(f"70 columns ({storage}): worst relative error {worst:.2e}")
    assert worst <= bound


# ------------------------------------------------------- source splitting --

@pytest.mark.parametrize("T,periods", [(60.0, 1), (65.0, 2)])
def test_source_splitting_matches_oracle(T, periods):
    # equation (split2): y(k dT) = e^{-dT A} y((k-1) dT) + w2(dT) over
    # subintervals of whole periods, w2 from the restarted method on one
    # window, plus a remainder window where T is not a whole number of
    # subintervals (both frequencies at T = 65, the second one at T = 60);
    # a complex shared source, every column against the oracle's
    # augmented-matrix route
    _announce(f"source splitting T={T} periods={periods}")
    wl = wk.small(10, seed=35, n_spheres=4, layer=2)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.1, 2 * math.pi * 0.113]
    b = wk.source_vector(wl, om[0], 0.3)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=40, tol=1e-10)
    y = s.solve_split2(om, _t(b[None, :]), T, periods=periods).cpu().numpy()
    st = s.last_stats
    s.close()
    assert st["converged"] == 1
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for k, w in enumerate(om):
        assert _rel(y[k], osv.augmented_solution(A, b, w, T)) <= 1e-8


# ------------------------------------------------------------ error paths --

def test_noconv_returns_best_estimate_and_true_residual():
    # a restart cap: KRY_ENOCONV raises NotConverged (stats attached) unless
    # the caller allows it; then the outputs are the finite best estimate and
    # the stats report the residual of the returned z
    kry = _kry()
    _announce("KRY_ENOCONV contract")
    wl = wk.small(12, seed=31, n_spheres=3, layer=2, T=30.0)
    inp = wk.generate(wl)
    om = wl.omegas[0]
    b = wk.source_vector(wl, om, 0.2)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=12, tol=1e-10, max_restarts=2)
    with pytest.raises(kry.NotConverged) as ei:
        s.solve_multifreq([om], _t(b[None, :]), wl.T)
    assert ei.value.stats is not None and ei.value.stats["converged"] == 0
    z = s.stationary([om], _t(b[None, :]), allow_noconv=True)[0].cpu().numpy()
    st = s.last_stats
    assert st["converged"] == 0 and np.isfinite(z).all()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    w = op.material_weights(inp.eps, inp.mu)
    r = b - (A @ z + 1j * om * z)
    true_res = math.sqrt(np.real(np.vdot(r, w * r)) / np.real(np.vdot(b, w * b)))
    assert true_res > 1e-10 * 0.05
    assert true_res <= st["max_residual"] * (1 + 1e-6)
    y = s.solve_multifreq([om], _t(b[None, :]), wl.T, allow_noconv=True)
    assert torch.isfinite(y).all()
    s.close()


def test_max_residual_bounds_true_residual_in_a_wide_shift_group():
    # 16 shifts over 2 pi [0.08, 0.12] in shared real Krylov sequences: the
    # reported max_residual is the largest true residual b - (A + i w) z of
    # the returned fields (checked against the oracle's operator)
    _announce("max_residual vs true residuals, 16 shifts")
    wl = wk.small(12, seed=32, n_spheres=4, layer=2)
    inp = wk.generate(wl)
    om = [2 * math.pi * f for f in np.linspace(0.08, 0.12, 16)]
    b = wk.source_vector(wl, om[0], 0.0)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=30, tol=1e-9)
    z = s.stationary(om, _t(b[None, :])).cpu().numpy()
    st = s.last_stats
    s.close()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    w = op.material_weights(inp.eps, inp.mu)
    bn = math.sqrt(np.real(np.vdot(b, w * b)))
    worst = 0.0
    for k, wk_ in enumerate(om):
        r = b - (A @ z[k] + 1j * wk_ * z[k])
        worst = max(worst, math.sqrt(np.real(np.vdot(r, w * r))) / bn)
    assert st["converged"] == 1
    assert worst <= st["max_residual"] * (1 + 1e-6) + 1e-13
    assert st["max_residual"] <= 2e-9


def test_enomem_for_a_basis_beyond_device_memory():
    # 256^3 with krylov_dim 1000 asks for about 820 GB of basis: the
    # allocation fails cleanly with KRY_ENOMEM and the device stays usable
    kry = _kry()
    _announce("KRY_ENOMEM contract")
    N = 256
    eps = torch.ones((N, N, N), dtype=torch.float64, device=_dev())
    s = kry.Solver(eps, None, None, kry.Options(krylov_dim=1000, tol=1e-8))
    v = torch.zeros((1, s.n), dtype=torch.float64, device=_dev())
    v[0, 3 * N ** 3 + 5] = 1.0
    with pytest.raises(kry.KryError) as ei:
        s.expv(1.0, v)
    assert ei.value.code == kry.KRY_ENOMEM
    s.close()
    del v, eps
    wl = wk.small(6, seed=3)
    inp = wk.generate(wl)
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=10)
    x = wk.random_state(wl.n, 2)
    w = s.apply(_t(x[None, :])).cpu().numpy()[0]
    assert _rel(w, op.apply_A(inp.eps, inp.mu, inp.sigma, x)) <= 1e-14
    s.close()


# -------------------------------------------------------------- block form --

@pytest.mark.parametrize("shape,p,mb", [((12, 12, 12), 4, 6), ((11, 9, 13), 20, 3),
                                        ((16, 16, 16), 32, 2)])
def test_block_arnoldi_relation_and_orthogonality(shape, p, mb):
    _announce(f"block arnoldi {shape} p={p} mb={mb}")
    eps, mu, sig = _box(shape, 12)
    s = _solver(eps, mu, sig, krylov_dim=30)
    n = 6 * eps.size
    V0 = np.random.default_rng(4).standard_normal((p, n))
    V, H, steps = s.block_arnoldi(_t(V0), mb)
    assert steps == mb
    V = V.cpu().numpy().T                     # n x (mb+1) p
    w = op.material_weights(eps, mu)
    G = V.T @ (w[:, None] * V)
    assert np.abs(G - np.eye((mb + 1) * p)).max() <= 1e-12
    AV = np.stack([op.apply_A(eps, mu, sig, V[:, j]) for j in range(mb * p)], axis=1)
    assert np.abs(AV - V @ H).max() <= 1e-12 * np.abs(AV).max()
    for j in range(mb):                       # block upper Hessenberg
        assert np.abs(H[(j + 2) * p:, j * p:(j + 1) * p]).max(initial=0.0) == 0.0
    # the first block spans the start block
    P0 = V[:, :p] @ (V[:, :p].T @ (w[:, None] * V0.T))
    assert np.abs(P0 - V0.T).max() <= 1e-12 * np.abs(V0).max()


def test_block_arnoldi_deficient_start_block():
    _announce("block arnoldi deficient")
    eps, mu, sig = _box((8, 8, 8), 13, with_mu=False)
    s = _solver(eps, None, sig, krylov_dim=30)
    n = 6 * eps.size
    rng = np.random.default_rng(5)
    V0 = rng.standard_normal((4, n))
    V0[2] = 2.0 * V0[0] - V0[1]
    V, H, steps = s.block_arnoldi(_t(V0), 4)
    V = V.cpu().numpy().T
    w = op.material_weights(eps, np.ones_like(eps))
    G = V.T @ (w[:, None] * V)
    d = np.diag(G)
    zero = d < 0.5
    # the dependence is either dropped (zero column) or kept as an extra
    # orthonormal direction; the nonzero columns stay orthonormal either way
    assert np.abs(G[~zero][:, ~zero] - np.eye((~zero).sum())).max() <= 1e-12
    AV = np.stack([op.apply_A(eps, np.ones_like(eps), sig, V[:, j]) for j in range(4 * 4)], axis=1)
    assert np.abs(AV - V @ H).max() <= 1e-12 * np.abs(AV).max()
    P0 = V[:, :4] @ (V[:, :4].T @ (w[:, None] * V0.T))
    assert np.abs(P0 - V0.T).max() <= 1e-10 * np.abs(V0).max()


def test_block_stationary_per_column_shifts():
    _announce("block stationary")
    wl = wk.small(8, seed=14, n_spheres=4, layer=2)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.08, 2 * math.pi * 0.1, 2 * math.pi * 0.12]
    th = [0.1, 0.3, 0.45]
    B = np.stack([wk.source_vector(wl, w, t) for w, t in zip(om, th)])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=48, tol=1e-11, block_width=6)
    z = s.stationary(om, _t(B), b_per_omega=True).cpu().numpy()
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for k, w in enumerate(om):
        assert _rel(z[k], osv.stationary(A, B[k], w)) <= 1e-9


@pytest.mark.parametrize("bw,bst", [(4, 0), (8, 0), (4, 24), (8, 16)])
def test_block_solve_matches_oracle(bw, bst):
    _announce(f"block solve bw={bw} block transient steps={bst}")
    wl = wk.small(9, seed=15, n_spheres=5, layer=2, T=50.0)
    inp = wk.generate(wl)
    om = [2 * math.pi * 0.09, 2 * math.pi * 0.11]
    th = [0.2, 0.4]
    cols = [(w, t) for w in om for t in th]
    B = np.stack([wk.source_vector(wl, w, t) for (w, t) in cols])
    s = _solver(inp.eps, None, inp.sigma, krylov_dim=48, tol=1e-9, block_width=bw,
                block_steps_transient=bst)
    y = s.solve_multifreq(om, _t(B), wl.T, b_per_omega=True).cpu().numpy()
    assert s.last_stats["converged"] == 1
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    for c, (w, t) in enumerate(cols):
        ref = osv.augmented_solution(A, B[c], w, wl.T)
        assert _rel(y[c], ref) <= 1e-8


# ------------------------------------------------------------- HIP graphs --

def test_graph_replay_matches_eager_bitwise():
    # every restart cycle replays the captured graph; the eager run between
    # the graph runs exercises interleaving with ordinary launches
    _announce("graph replay vs eager")
    wl = wk.C1
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    eager = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol)
    graph = _solver(inp.eps, None, inp.sigma, krylov_dim=wl.krylov_dim, tol=wl.tol, use_graph=True)
    t0 = time.time()
    y_e = eager.solve_multifreq(wl.omegas, b, wl.T).cpu().numpy()
    t_e = time.time() - t0
    outs = []
    for rep in range(2):
        t0 = time.time()
        outs.append(graph.solve_multifreq(wl.omegas, b, wl.T).cpu().numpy())
        t_g = time.time() - t0
        eager.solve_multifreq(wl.omegas, b, wl.T)
    _announce(f"c1 eager {t_e:.3f}s graph {t_g:.3f}s cycles {graph.last_stats['cycles_stationary']}")
    for y in outs:
        assert np.array_equal(y, y_e)
    v = wk.random_state(wl.n, 3)
    V1, H1, b1, s1 = eager.arnoldi(_t(v), 20)
    V2, H2, b2, s2 = graph.arnoldi(_t(v), 20)
    assert np.array_equal(H1, H2) and np.array_equal(V1.cpu().numpy(), V2.cpu().numpy())


def test_sstep_cycle_graph_replay_matches_eager_bitwise():
    # the s-step cycle with the device block finish, captured once per basis
    # steps (a Chebyshev cycle, then the Newton cycles of each call) and
    # replayed for every restart cycle: two solves (each recaptures for its
    # own Newton steps) with an eager solve between them, and an Arnoldi
    # call, all bitwise equal to the eager runs
    _announce("s-step cycle graph replay vs eager")
    wl = wk.small(32, seed=3, n_spheres=20, layer=3, T=30.0, krylov_dim=64, tol=1e-9)
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    om = [wl.omegas[0], 1.1 * wl.omegas[0]]
    eager = _solver(inp.eps, None, inp.sigma, krylov_dim=64, tol=1e-9, s_step=16)
    graph = _solver(inp.eps, None, inp.sigma, krylov_dim=64, tol=1e-9, s_step=16, use_graph=True)
    y_e = eager.solve_multifreq(om, b, wl.T).cpu().numpy()
    outs = []
    for rep in range(2):
        outs.append(graph.solve_multifreq(om, b, wl.T).cpu().numpy())
        eager.solve_multifreq(om, b, wl.T)
    _announce(f"32^3 s-step graph: cycles {graph.last_stats['cycles_stationary']}, "
              f"steps {graph.last_stats['steps_transient']}")
    assert graph.last_stats["cycles_stationary"] > 3
    for y in outs:
        assert np.array_equal(y, y_e)
    v = wk.random_state(wl.n, 3)
    V1, H1, b1, s1 = eager.arnoldi(_t(v), 64)
    V2, H2, b2, s2 = graph.arnoldi(_t(v), 64)
    assert np.array_equal(H1, H2) and np.array_equal(V1.cpu().numpy(), V2.cpu().numpy())
    eager.close()
    graph.close()


# --------------------------------------------------------------- autotuner --

def test_autotune_choice_and_results(tmp_path):
    _announce("autotune")
    wl = wk.small(40, seed=16, n_spheres=30, layer=4, T=40.0, krylov_dim=32, tol=1e-9)
    inp = wk.generate(wl)
    b = _t(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :])
    s0 = _solver(inp.eps, None, inp.sigma, krylov_dim=32, tol=1e-9)
    y0 = s0.solve_multifreq(wl.omegas, b, wl.T).cpu().numpy()
    s1 = _solver(inp.eps, None, inp.sigma, krylov_dim=32, tol=1e-9)
    cache = str(tmp_path / "tune.json")
    t = s1.autotune(cache=cache)
    _announce(f"autotune {t}")
    assert t["cpt_stencil"] in (1, 2, 4) and t["cpt_update"] in (1, 2, 4)
    assert all(x > 0 for x in t["us_stencil"] + t["us_update"] + t["us_dots"])
    y1 = s1.solve_multifreq(wl.omegas, b, wl.T).cpu().numpy()
    assert _rel(y1, y0) <= 1e-10
    s2 = _solver(inp.eps, None, inp.sigma, krylov_dim=32, tol=1e-9)
    t2 = s2.autotune(cache=cache)
    assert t2["cached"] and t2["cpt_update"] == t["cpt_update"]
    # the s-step block size: one timed restart cycle per candidate, the
    # fastest applied; the solve with it agrees with the default one
    s3 = _solver(inp.eps, None, inp.sigma, krylov_dim=32, tol=1e-9)
    cache_s = str(tmp_path / "tune_s.json")
    t3 = s3.autotune(cache=cache_s, s_candidates=(0, 8, 16, 32))
    _announce(f"autotune with s: {t3}")
    assert t3["s_step"] in (0, 8, 16, 32) and all(x > 0 for x in t3["us_cycle"])
    y3 = s3.solve_multifreq(wl.omegas, b, wl.T).cpu().numpy()
    assert _rel(y3, y0) <= 1e-8
    s4 = _solver(inp.eps, None, inp.sigma, krylov_dim=32, tol=1e-9)
    t4 = s4.autotune(cache=cache_s, s_candidates=(0, 8, 16, 32))
    assert t4["cached"] and t4["s_step"] == t3["s_step"]
