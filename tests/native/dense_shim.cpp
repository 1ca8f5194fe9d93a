// Test-only C wrappers around the host small-dense routines of libkry.
#include <algorithm>
#include <complex>
#include <vector>

#include "../../paper_1707_00023_amd/csrc/kry_dense.h"

using kry::cplx;

extern "C" {

void t_expm(int m, const double* A, double* E) { kry::expm(m, A, E); }

int t_hess_solve(int N, const double* Mri, const double* rhs_ri, double* y_ri) {
  return kry::hess_solve(N, reinterpret_cast<const cplx*>(Mri), reinterpret_cast<const cplx*>(rhs_ri),
                         reinterpret_cast<cplx*>(y_ri));
}

int t_dense_solve(int N, const double* Ari, const double* rhs_ri, double* y_ri) {
  return kry::dense_solve(N, reinterpret_cast<const cplx*>(Ari), reinterpret_cast<const cplx*>(rhs_ri),
                          reinterpret_cast<cplx*>(y_ri));
}

int t_hess_shift_solve(int m, const double* H, int ldh, double sr, double si, const double* rhs_ri,
                       double* y_ri) {
  return kry::hess_shift_solve(m, H, ldh, cplx(sr, si), reinterpret_cast<const cplx*>(rhs_ri),
                               reinterpret_cast<cplx*>(y_ri));
}

void t_best_real_direction(int n, const double* q_ri, double* w) {
  kry::best_real_direction(n, reinterpret_cast<const cplx*>(q_ri), w);
}

double t_choose_step(int m, const double* H, int ldh, double hnext, double beta, double tau_try,
                     double rate, int K, double* u, double* err) {
  return kry::choose_step(m, H, ldh, hnext, beta, tau_try, rate, K, u, err);
}

int t_cholqr_factor(int p, const double* G, double thr, double* Cm, double* Rf) {
  return kry::cholqr_factor(p, G, thr, Cm, Rf);
}

void t_block_shift_lsq(int K, int q, int bw, const double* H, int ldh, double sr, double si,
                       const double* g_ri, double* y_ri, double* res_ri) {
  kry::block_shift_lsq(K, q, bw, H, ldh, cplx(sr, si), reinterpret_cast<const cplx*>(g_ri),
                       reinterpret_cast<cplx*>(y_ri), reinterpret_cast<cplx*>(res_ri));
}

int t_qr_pivoted(int m, int q, const double* S, double thr, double* Q, double* Rf) {
  return kry::qr_pivoted(m, q, S, thr, Q, Rf);
}

int t_chol_upper(int p, const double* G, const double* ref, double thr, double* R) {
  return kry::chol_upper(p, G, ref, thr, R) ? 1 : 0;
}

void t_inv_upper(int p, const double* R, double* X) { kry::inv_upper(p, R, X); }

void t_sstep_hessenberg(int j0, int s, double rho, double c, const double* C1, const double* C2,
                        const double* R1, const double* R2, double* H, int ldh) {
  kry::sstep_hessenberg(j0, s, rho, c, C1, C2, R1, R2, H, ldh);
}

void t_proj_gram(int M, int s, const double* P, double* G, double* ref) { kry::proj_gram(M, s, P, G, ref); }

void t_stack_coef(int M, int s, const double* C, const double* Rinv, double* K) {
  kry::stack_coef(M, s, C, Rinv, K);
}

void t_stack_coef_full(int M, int s, const double* C, const double* F, double* K) {
  kry::stack_coef_full(M, s, C, F, K);
}

void t_sstep_hessenberg_tm(int j0, int s, const double* Tm, const double* C1, const double* C2,
                           const double* R1, const double* R2, double* H, int ldh) {
  kry::sstep_hessenberg_tm(j0, s, Tm, C1, C2, R1, R2, H, ldh);
}

int t_hess_eigvals(int m, const double* H, int ldh, double* re, double* im) {
  return kry::hess_eigvals(m, H, ldh, re, im) ? 1 : 0;
}

int t_group_shifts(int n, const double* w, int max_size, double rel_band, int* group) {
  return kry::group_shifts(n, w, max_size, rel_band, group);
}

int t_leja_steps(int nr, const double* re, const double* im, int s, double scale, double* alpha,
                 double* q) {
  return kry::leja_steps(nr, re, im, s, scale, alpha, q);
}

double t_choose_step_block(int K, int q, int g, const double* H, int ldh, const double* U0,
                           double tau_try, const double* rate, int Ks, double* U, double* err) {
  return kry::choose_step_block(K, q, g, H, ldh, U0, tau_try, rate, Ks, U, err);
}

void t_gauss_legendre01(int q, double* x, double* w) { kry::gauss_legendre01(q, x, w); }

void t_rst_prepare(int m, const double* H, int ldh, int q, double dt, const double* x, double* E,
                   double* W, double* El, double* Wl) {
  kry::RstProp P;
  kry::rst_prepare(m, H, ldh, q, dt, x, &P);
  std::copy(P.E.begin(), P.E.end(), E);
  std::copy(P.W.begin(), P.W.end(), W);
  std::copy(P.El.begin(), P.El.end(), El);
  std::copy(P.Wl.begin(), P.Wl.end(), Wl);
}

// fin, fout: ncol x (nt q) row-major
void t_rst_march(int m, const double* H, int ldh, int q, double dt, const double* x, const double* w,
                 int nt, int ncol, double beta, double hnext, const double* fin, double* fout, double* uT,
                 double* resint) {
  kry::RstProp P;
  kry::rst_prepare(m, H, ldh, q, dt, x, &P);
  std::vector<const double*> fi(ncol);
  std::vector<double*> fo(ncol);
  for (int c = 0; c < ncol; ++c) {
    fi[c] = fin + (size_t)c * nt * q;
    fo[c] = fout + (size_t)c * nt * q;
  }
  kry::rst_march(P, nt, ncol, beta, hnext, w, fi.data(), fo.data(), uT, resint);
}
}  // extern "C"
