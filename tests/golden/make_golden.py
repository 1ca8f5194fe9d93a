"""Write sampled oracle results for the large workloads (calls only the oracle).

The full-size workloads are too large for the oracle to finish inside a test,
so this script runs it once and stores what a test can compare against:
the 2-norm of y(T), its values at seeded random indices, and its projections
on seeded random vectors.  y(T) is evaluated by the variation-of-constants
route (one exponential action of the augmented matrix), which needs no
shifted solve and does not use Corollary 3.

    python tests/golden/make_golden.py c2        # ~1 h on one CPU core
    python tests/golden/make_golden.py c3        # 4 of the 256 columns
    python tests/golden/make_golden.py grad16    # 16^3 flux gradient, ~1 min
    python tests/golden/make_golden.py tgrad     # flux at time T: 5^3 gradient, 15^3 directions

grad16 stores the oracle's whole gradient vector dL/d eps (4096 cells) and
the loss for GRAD16, a 16^3 medium with two frequencies: both shifted solves
and both explicit-transpose adjoint solves by SuperLU (n = 24576).

tgrad stores, for the flux of the whole field at a finite time T (transient
included), the oracle's per-cell gradient on a 5^3 medium (forward
derivatives with dense LU and scipy's Frechet derivative of expm) and, on a
15^3 medium, the loss and three directional derivatives along seeded random
permittivity changes (SuperLU solves, expm_multiply for the exponential and
for its Frechet derivative through the 2n block identity).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wk  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import solve as osv  # noqa: E402

N_SAMPLES = 4096
N_PROJ = 4
SAMPLE_SEED = 20170630
# columns (omega index, theta index) evaluated for the batched workload
SUBSETS = {"c3": [(0, 0), (15, 3), (31, 7), (16, 5)]}


def grad16_workload():
    """16^3, two frequencies, flux plane 12 (outside the 2-cell layer at
    14..15), Ex source at k = 3, 24 random spheres; one shared source."""
    return wk.small(16, seed=41, n_spheres=24, layer=2, radius=(1.0, 2.0),
                    omegas=(2 * np.pi * 0.09, 2 * np.pi * 0.11), src_k=3,
                    flux_plane=12, tol=1e-12, krylov_dim=40)


def make_grad16():
    from oracle import grad as og
    wl = grad16_workload()
    inp = wk.generate(wl)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    b_cols = np.stack([b] * len(wl.omegas), axis=1)
    t0 = time.time()
    L, g = og.loss_and_grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, wl.flux_plane)
    dt = time.time() - t0
    out = {"workload": wl.name, "N": wl.N, "omegas": list(wl.omegas), "plane_k": wl.flux_plane,
           "route": "SuperLU shifted and explicit-transpose adjoint solves",
           "loss": float(L), "grad": g.reshape(-1).tolist(), "oracle_seconds": dt}
    with open(os.path.join(HERE, "grad16_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"grad16 L={L:.12e} |g|={np.linalg.norm(g):.6e} {dt:.1f}s", flush=True)


def tgrad_workloads():
    """(small, medium, T, directions): the 5^3 and 15^3 media of the
    finite-time flux gradient, two frequencies, one shared Ex source."""
    om = (2 * np.pi * 0.09, 2 * np.pi * 0.11)
    w5 = wk.small(5, seed=52, n_spheres=2, layer=1, radius=(0.8, 1.4), omegas=om, src_k=1,
                  flux_plane=3, tol=1e-12, krylov_dim=30)
    w15 = wk.small(15, seed=53, n_spheres=12, layer=2, radius=(1.0, 2.0), omegas=om, src_k=3,
                   flux_plane=11, tol=1e-12, krylov_dim=40)
    return w5, w15, 12.0, 3


def tgrad_direction(N, k):
    return np.random.default_rng(SAMPLE_SEED + 100 + k).standard_normal((N, N, N))


def make_tgrad():
    from oracle import transient_grad as tg
    w5, w15, T, ndir = tgrad_workloads()
    out = {"T": T}
    for tag, wl in (("small", w5), ("medium", w15)):
        inp = wk.generate(wl)
        b = wk.source_vector(wl, wl.omegas[0], 0.0)
        b_cols = np.stack([b] * len(wl.omegas), axis=1)
        t0 = time.time()
        L = tg.loss(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, wl.flux_plane, T)
        rec = {"workload": wl.name, "N": wl.N, "omegas": list(wl.omegas), "plane_k": wl.flux_plane,
               "loss": float(L)}
        if tag == "small":
            g = tg.grad(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, wl.flux_plane, T)
            rec["grad"] = g.reshape(-1).tolist()
            rec["route"] = "dense LU and expm_frechet, one forward derivative per cell"
        else:
            rec["directional"] = [
                tg.directional(inp.eps, inp.mu, inp.sigma, b_cols, wl.omegas, wl.flux_plane, T,
                               tgrad_direction(wl.N, k)) for k in range(ndir)]
            rec["route"] = "SuperLU, expm_multiply and the 2n block identity"
        rec["oracle_seconds"] = time.time() - t0
        out[tag] = rec
        print(f"tgrad {tag} L={L:.12e} {rec['oracle_seconds']:.1f}s", flush=True)
    with open(os.path.join(HERE, "tgrad_oracle.json"), "w") as f:
        json.dump(out, f)


def sample_spec(n):
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(n, size=min(N_SAMPLES, n), replace=False))
    return idx


def projection_vector(n, k):
    return np.random.default_rng(SAMPLE_SEED + 1 + k).standard_normal(n)


def main(cfg_name: str):
    wl = wk.CONFIGS[cfg_name]
    inp = wk.generate(wl)
    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    out = {"workload": wl.name, "n": wl.n, "T": wl.T, "columns": [],
           "route": "augmented-matrix exponential action (expm_multiply)"}
    idx = sample_spec(wl.n)
    out["indices"] = idx.tolist()
    cols = SUBSETS.get(cfg_name, [(wi, ti) for wi in range(len(wl.omegas))
                                   for ti in range(len(inp.thetas))])
    for wi, ti in cols:
        omega, theta = wl.omegas[wi], float(inp.thetas[ti])
        b = wk.source_vector(wl, omega, float(theta))
        t0 = time.time()
        y = osv.augmented_solution(A, b, omega, wl.T)
        dt = time.time() - t0
        col = {"omega_index": wi, "theta_index": ti, "omega": omega,
               "theta": float(theta), "norm2": float(np.linalg.norm(y)),
               "values": y[idx].tolist(),
               "projections": [float(projection_vector(wl.n, k) @ y)
                               for k in range(N_PROJ)],
               "oracle_seconds": dt}
        out["columns"].append(col)
        print(f"{cfg_name} col ({wi},{ti}) |y|={col['norm2']:.6e} {dt:.1f}s", flush=True)
    with open(os.path.join(HERE, f"{cfg_name}_yT_samples.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    if sys.argv[1] == "grad16":
        make_grad16()
    elif sys.argv[1] == "tgrad":
        make_tgrad()
    else:
        main(sys.argv[1])
