// Small dense FP64 kernels of the projected problems, run on the host.
//
// All matrices are column-major, leading dimension = rows.
#pragma once
#include <complex>
#include <vector>

namespace kry {

using cplx = std::complex<double>;

// E = expm(A) for an m x m matrix: scaling and squaring with the diagonal
// [13/13] Pade approximant (Higham, SIAM J. Matrix Anal. Appl. 26, 2005).
void expm(int m, const double* A, double* E);

// Solve (H + s I) y = rhs for an m x m upper-Hessenberg H and complex shift
// s, by Gaussian elimination with partial pivoting between adjacent rows
// (Hessenberg structure: O(m^2)).  H has leading dimension ldh.
// Returns false if a pivot is exactly zero (singular projected system).
bool hess_shift_solve(int m, const double* H, int ldh, cplx s, const cplx* rhs, cplx* y);

// Solve M y = rhs for an N x N complex upper-Hessenberg matrix M (dense,
// column-major, leading dimension N; entries below the first subdiagonal
// are ignored).  Adjacent-row partial pivoting, O(N^2).
bool hess_solve(int N, const cplx* M, const cplx* rhs, cplx* y);

// Solve A y = rhs for a general N x N complex matrix (partial pivoting).
bool dense_solve(int N, const cplx* A, const cplx* rhs, cplx* y);

// Real unit direction w in span{Re q, Im q} maximising |q^H w|: the top
// eigenvector of Re(q) Re(q)^T + Im(q) Im(q)^T.  Length n.
void best_real_direction(int n, const cplx* q, double* w);

// Step control of the restarted exponential: for the projected problem
// u' = -H u, u(0) = beta e_1, with residual norm rho(s) = hnext |e_m^T u(s)|
// (Lemma 1, homogeneous case), find the largest tau in (0, tau_try] among
// K equispaced candidates such that rho stays below `rate` on [0, tau]
// (so that the integral of the residual over the step is <= rate * tau).
// On success returns tau and writes u(tau) into u (length m).  If even the
// first candidate fails, returns 0 and the caller shrinks tau_try.
double choose_step(int m, const double* H, int ldh, double hnext, double beta,
                   double tau_try, double rate, int K, double* u, double* err_out);

}  // namespace kry
