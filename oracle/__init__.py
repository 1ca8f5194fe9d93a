"""Oracle: a plain, slow, FP64 CPU implementation of the solver's hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute this package: it exists so that the tests, the smoke check
and the benchmark's CPU-baseline leg have an independent answer to compare
the HIP path against.  It shares no code with the HIP path; the only module
both sides use is ``workloads`` (seeded input generation, no arithmetic of the
method).

What it computes, following the paper (arXiv 1707.00023):

* ``operator``  -- the semi-discrete Maxwell operator A = M^-1 (S + K) of the
  ODE system y' = -A y + alpha(t) g (Section 2.1, equation (ode) and the block
  form of A-hat after it), written matrix-free and assembled as a sparse
  matrix from Kronecker products.
* ``solve``     -- the solution at time T by the time-harmonic / transient
  split of Corollary 3 (equation (split1)): y(T) = Im(e^{i w T} z) -
  e^{-T A} Im z with z = (A + i w I)^-1 b; plus an independent route via the
  variation-of-constants integral written as one exponential of an augmented
  matrix, and the plain exponential action e^{-tA} v of equation (y_homo).
* ``grad``      -- the period-averaged Poynting flux of the time-harmonic
  field through a z-plane and its exact gradient with respect to per-cell
  permittivity (the paper is silent on gradients; the reading is documented
  in the design notes), plus brute-force central differences.
* ``transient_grad`` -- the instantaneous flux of the whole solution at a
  finite time T (time-harmonic part minus the transient of equation
  (y_homo)) and its gradient w.r.t. per-cell permittivity by forward
  differentiation (library solves and the Frechet derivative of the matrix
  exponential), plus central differences.

Readings of the paper where it is silent or 2D-only (3D Yee staggering,
zero-ghost boundary, damping scaling sigma/eps, angular omega, minus sign of
the split) are listed in the design notes and restated in each docstring.
"""
from . import operator, solve, grad, krylov, transient_grad  # noqa: F401
