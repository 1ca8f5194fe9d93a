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

// Rank-revealing Cholesky QR factor of a block W with Gram matrix
// G = W^T M W (p x p, symmetric).  Columns are first scaled to unit
// norm; diagonal pivoting; a direction whose remaining norm is below thr
// relative to
// its own column is dropped (rank r <= p).  The threshold is clamped below
// at 1e-10.  Outputs (p x p, row-major):
//   Cm: V = W Cm has M-orthonormal columns 0..r-1 and zero columns r..p-1,
//   Rf: W ~= V Rf (rows r..p-1 zero), exact for the kept directions.
// Returns r.
int cholqr_factor(int p, const double* G, double thr, double* Cm, double* Rf);

// Householder QR with column pivoting of a real m x q matrix S (column-
// major): S ~= Q Rf with Q (m x q column-major; columns r.. zero) having
// orthonormal columns and Rf (q x q row-major; rows r.. zero), rank r set
// by |R_kk| > thr * (largest column norm).  Returns r.
int qr_pivoted(int m, int q, const double* S, double thr, double* Q, double* Rf);

// Least squares for one column of a block shifted system:
// y = argmin | g - (Hbar + s Ibar) y |_2 with Hbar (K + q) x K real,
// column-major with leading dimension ldh, zero below row k + bw of column
// k; Ibar = [I_K; 0].  Banded complex Householder QR.  res receives
// g - (Hbar + s Ibar) y (length K + q).  Directions with a vanishing
// diagonal of R (zero basis columns) get y = 0.
void block_shift_lsq(int K, int q, int bw, const double* H, int ldh, cplx s, const cplx* g, cplx* y,
                     cplx* res);

// Block step control for U(s) = e^{-s H} U0 (H K x K column-major, ldh;
// U0 K x g column-major): the residual of column c is
// |B U(s)[K-q:K, c]|_2 with B = Hbar[K:K+q, K-q:K] (Lemma 1 for a block).
// Finds the largest of Ks equispaced candidates in (0, tau_try] with every
// column's residual below rate[c] up to it; writes U(tau) into U (K x g)
// and the per-column error bounds into err.  Returns tau or 0.
double choose_step_block(int K, int q, int g, const double* H, int ldh, const double* U0,
                         double tau_try, const double* rate, int Ks, double* U, double* err);

// Upper Cholesky factor R (p x p row-major, R^T R = G) of a symmetric
// Gram matrix G (row-major).  Returns false when a pivot is not above
// thr^2 ref[k] (ref[k]: squared norm of column k before any projection,
// so a dependent direction is caught relative to its own size) or is not
// finite.
bool chol_upper(int p, const double* G, const double* ref, double thr, double* R);

// X = R^{-1} for an upper-triangular p x p matrix R (both row-major).
void inv_upper(int p, const double* R, double* X);

// Hessenberg columns j0..j0+s-1 of an s-step Arnoldi block.  The block
// [t_0..t_s] with t_0 = v_j0 obeys A [t_0..t_{s-1}] = rho [t_0..t_s] Tm +
// c [t_0..t_{s-1}] (Chebyshev basis on the segment c + [-i rho, i rho]:
// Tm[1][0] = 1, Tm[k+1][k] = 1/2, Tm[k-1][k] = -1/2).  Two projection passes gave t_k = V C1 + u_k,
// u = q1 R1, q1 = V C2 + Q R2 (V = v_0..v_j0; C1, C2 (j0+1) x s row-major;
// R1, R2 s x s upper row-major), so [t_1..t_s] = V (C1 + C2 R1) + Q R2 R1.
// With [t_0..t_s] = V_ext Rhat this writes
//   H[:, j0:j0+s] = (rho Rhat Tm + c Rhat[:, :s] - [H[:j0+1, :j0] Rtop; 0]) Rs^{-1}
// into H (column-major, leading dimension ldh >= j0 + s + 1; columns < j0
// already filled).  Entries below the first subdiagonal are left zero.
void sstep_hessenberg(int j0, int s, double rho, double c, const double* C1, const double* C2,
                      const double* R1, const double* R2, double* H, int ldh);

// The same for a general basis-change matrix: A [t_0..t_{s-1}] =
// [t_0..t_s] Tm with Tm ((s+1) x s, row-major) upper Hessenberg with a
// nonzero subdiagonal (Chebyshev, Newton, ... recurrences).
void sstep_hessenberg_tm(int j0, int s, const double* Tm, const double* C1, const double* C2,
                         const double* R1, const double* R2, double* H, int ldh);

// Eigenvalues (re[k], im[k], k < m) of an m x m upper-Hessenberg matrix H
// (column-major, leading dimension ldh; entries below the subdiagonal are
// ignored) by the implicitly shifted double-shift QR iteration (Francis).
// Returns false if an eigenvalue does not converge in 60 m sweeps.
bool hess_eigvals(int m, const double* H, int ldh, double* re, double* im);

// Newton-basis steps from shifts theta_k (Ritz values): picks at most s
// shifts in Leja order (each new shift maximises the product of its
// distances to the ones already taken; a complex shift is taken with its
// conjugate right after it) and writes, per step k < s, the recurrence
// t_{k+1} = (A t_k - alpha_k t_k + q_k t_{k-1}) / scale as alpha[k] and
// q[k] (q_k = beta^2 / scale on the second step of a conjugate pair
// alpha +- i beta, else 0).  A pair that would be cut by the block end is
// replaced by its real part.  Returns the number of shifts used (s).
int leja_steps(int nr, const double* re, const double* im, int s, double scale, double* alpha,
               double* q);

// Groups of neighbouring shifts, one shared Krylov sequence each: the n
// shifts w are taken in increasing order, and a group is closed when the
// next shift would make it larger than max_size or its spread (highest
// minus lowest) larger than rel_band times the mean of those two.  Writes
// group[k], the 0-based group of shift k (groups numbered in increasing
// order of their shifts); returns the number of groups.
int group_shifts(int n, const double* w, int max_size, double rel_band, int* group);

// Projected Gram matrix of an s-column block S against an M-orthonormal
// basis V from one product P = [V, S]^T M S ((M + s) x s, row-major):
// G = S^T M S - C^T C with C = P[:M] (s x s, row-major) and ref[k] =
// (S^T M S)_kk, the squared column norms before projection.
void proj_gram(int M, int s, const double* P, double* G, double* ref);

// Coefficients K ((M + s) x s, row-major) with [V, S] K = (S - V C) Rinv:
// rows k < M are -(C Rinv)[k], rows M + a are Rinv[a] (C: M x s, Rinv:
// s x s upper, both row-major).
void stack_coef(int M, int s, const double* C, const double* Rinv, double* K);

// As stack_coef for a general (not triangular) s x s factor F:
// [V, S] K = (S - V C) F.
void stack_coef_full(int M, int s, const double* C, const double* F, double* K);

}  // namespace kry

namespace kry {

// Gauss-Legendre rule with q points on [0, 1]: nodes x (increasing) and
// weights w (summing to 1), by Newton's method on the Legendre polynomial.
void gauss_legendre01(int q, double* x, double* w);

// Propagators of the projected problem u' = -H u + f(t) e_1 (H m x m) over
// one time step of length dt, for a source f known at the q nodes dt x_i
// of the step (interpolated by the degree q-1 polynomial through them):
//   u(dt)        = E u(0) + W f,            E = e^{-dt H},  W  m x q,
//   e_m^T u(s_i) = El[i] u(0) + Wl[i] f,    El q x m,       Wl q x q,
// with s_i = dt x_i.  The polynomial part is exact: the integrals of
// e^{-(tau-s)H} e_1 against the monomials (s/dt)^r come from one
// exponential of the augmented matrix [[-H, e_1 e_1^T], [0, J]] (J the
// q x q shift) per node, and the Lagrange weights from the inverse of the
// Vandermonde matrix of the nodes.  All row-major except E, W
// (column-major).
struct RstProp {
  int m = 0, q = 0;
  double dt = 0.0;
  std::vector<double> E, W, El, Wl;
};
void rst_prepare(int m, const double* H, int ldh, int q, double dt, const double* x, RstProp* P);

// March ncol projected problems u_c' = -H u_c + beta f_c(t) e_1, u_c(0) = 0,
// over nt steps of P.dt: f_c is given by its samples fin[c][j q + i] at
// t = j dt + dt x_i; writes the samples of the new residual source
// fout[c][j q + i] = -hnext e_m^T u_c(t) at the same times, u_c(nt dt)
// into uT (m x ncol column-major), and the integral of |fout| over the
// interval (Gauss rule with weights dt w_i) into resint[c].
void rst_march(const RstProp& P, int nt, int ncol, double beta, double hnext, const double* w,
               const double* const* fin, double* const* fout, double* uT, double* resint);

}  // namespace kry
