// Test-only C wrappers around the host small-dense routines of libkry.
#include <complex>

#include "../../paper_1707_00023_amd/csrc/kry_dense.h"

extern "C" {
void t_expm(int m, const double* A, double* E) { kry::expm(m, A, E); }
int t_hess_solve(int N, const double* Mri, const double* rhs_ri, double* y_ri) {
  return kry::hess_solve(N, reinterpret_cast<const kry::cplx*>(Mri),
                         reinterpret_cast<const kry::cplx*>(rhs_ri),
                         reinterpret_cast<kry::cplx*>(y_ri));
}
int t_dense_solve(int N, const double* Ari, const double* rhs_ri, double* y_ri) {
  return kry::dense_solve(N, reinterpret_cast<const kry::cplx*>(Ari),
                          reinterpret_cast<const kry::cplx*>(rhs_ri),
                          reinterpret_cast<kry::cplx*>(y_ri));
}
int t_hess_shift_solve(int m, const double* H, int ldh, double sr, double si,
                       const double* rhs_ri, double* y_ri) {
  return kry::hess_shift_solve(m, H, ldh, kry::cplx(sr, si),
                               reinterpret_cast<const kry::cplx*>(rhs_ri),
                               reinterpret_cast<kry::cplx*>(y_ri));
}
void t_best_real_direction(int n, const double* q_ri, double* w) {
  kry::best_real_direction(n, reinterpret_cast<const kry::cplx*>(q_ri), w);
}
double t_choose_step(int m, const double* H, int ldh, double hnext, double beta, double tau_try,
                     double rate, int K, double* u, double* err) {
  return kry::choose_step(m, H, ldh, hnext, beta, tau_try, rate, K, u, err);
}
}
