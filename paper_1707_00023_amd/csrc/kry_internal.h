// Internal interface between the C-ABI driver and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kry {

enum Storage : int { F64 = 0, F32 = 1 };

struct DevGrid {
  int nx, ny, nz;
  long long N3;  // cells
  // cells per thread (1, 2 or 4) of the operator kernels, the basis-update
  // kernels and the dot-product kernels (chosen by heuristic or autotuner)
  int cpt_s = 1, cpt_u = 1, cpt_d = 1;
  // planes per workgroup of the z-marching basis stencil (4, 8 or 16; 0:
  // the cell-parallel one with cpt_s cells per thread)
  int zm_s = 0;
};

// Per-cell material data derived at context creation (all FP64, N3 each).
struct DevMats {
  const double* inv_eps;  // 1 / eps
  const double* sigma;    // sigma (sigma/mu when mu is given)
  const double* inv_mu;   // 1 / mu, or nullptr when mu == 1
  const double* eps;      // eps: energy weight of the E planes
  const double* mu;       // mu: energy weight of the H planes, or nullptr
};

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kChunk = 16;       // basis vectors per dot-product chunk
constexpr int kMaxCoef = 1026;   // max coefficients staged by an update (m <= 1024)

// Default cells per thread for a grid, and the workgroups of a
// cell-parallel launch with `cpt` cells per thread.
int cells_per_thread(long long N3);
int cell_blocks(long long N3, int cpt);

// w = A v (single column).  If V != nullptr also writes per-workgroup
// partial sums of <w, V_i>_M for i < cnt and |w|_M^2 (slot cnt) into
// partials[blk * (cnt + 1) + q].
hipError_t launch_stencil(Storage st, const void* v, void* w, const void* V, long long ldv,
                          int cnt, const DevGrid& g, const DevMats& m, double* partials,
                          hipStream_t s);

// out = alpha A v + gamma v + beta prev (prev may be null); out must not
// alias v.
hipError_t launch_stencil_axpby(Storage st, const void* v, const void* prev, void* out, double alpha,
                                double gamma, double beta, const DevGrid& g, const DevMats& m,
                                hipStream_t s);

// Pass A of a delayed-reorthogonalisation Arnoldi step: x = A u and partial
// sums of [<x,V_i>_M (cnt), <u,V_i>_M (cnt), |u|_M^2, <u,x>_M] per workgroup
// (stride 2 cnt + 2).
hipError_t launch_stencil_lag(Storage st, const void* u, void* x, const void* V, long long ldv,
                              int cnt, const DevGrid& g, const DevMats& m, double* partials,
                              hipStream_t s);

// Pass B: vnew = u co[2cnt] - sum co[i] V_i, unext = x co[2cnt] -
// co[2cnt+1] u - sum co[cnt+i] V_i (unext may alias u).
hipError_t launch_lag_update(Storage st, const void* u, const void* x, const void* V, long long ldv,
                             int cnt, const double* co, void* vnew, void* unext, const DevGrid& g,
                             hipStream_t s);

// Small step between the passes of Arnoldi step j (see the kernel).
hipError_t launch_lag_fin(const double* red, int j, double* H, int ldh, double* co, double* scal,
                          hipStream_t s);

// Completes the last column of a cycle from red = [<u_m, V_i>_M (m), |u_m|_M^2].
hipError_t launch_lag_final(const double* red, int m, double* H, int ldh, double* scal,
                            hipStream_t s);

// Partial sums of <x, V_i>_M (i < cnt) and |x|_M^2 (slot cnt).
hipError_t launch_dots(Storage st, const void* x, const void* V, long long ldv, int cnt,
                       const DevGrid& g, const DevMats& m, double* partials, hipStream_t s);

// out = (w - sum_i coef[i] V_i) * (*scale or 1); out may alias w.
hipError_t launch_update(Storage st, const void* w, const void* V, long long ldv, int cnt,
                         const double* coef, const double* scale, void* out,
                         const DevGrid& g, hipStream_t s);

// out[q] = sum_p partials[p * stride + q] for q < cnt, fixed order.  With
// skip != nullptr the launch does nothing when *skip (device) is non-zero
// (likewise for launch_gram and launch_gemm_nn in their N <= 32 forms).
hipError_t launch_reduce(const double* partials, int nparts, int stride, int cnt, double* out,
                         hipStream_t s, const int* skip = nullptr);

// scal[1] = sqrt(red[0]), scal[0] = 1/scal[1] (0 if scal[1] == 0).
hipError_t launch_fin_start(const double* red, double* scal, hipStream_t s);

// Arnoldi column j after two Gram-Schmidt passes: H[:, j] = red1 + red2,
// H[j+1, j] = nu = sqrt(|w1|^2 - |red2|^2) (0 on breakdown), scal[0] = 1/nu.
hipError_t launch_fin_step(const double* red1, const double* red2, int j, double* H, int ldh,
                           double* scal, hipStream_t s);

// out = x * (*scale).
hipError_t launch_scale(Storage st, const void* x, const double* scale, void* out, long long n,
                        hipStream_t s);

// out_c (= or +=) sum_{i<m} V_i Y[i + c*m] for c < ncol; column c goes to
// out + colmap[c] * ldo (colmap may be nullptr: identity).  With out_last,
// the last column goes there instead, assigned (never accumulated); it may
// be one of the V_i, and then ncol must be at most 8.
hipError_t launch_combine(Storage st, const void* V, long long ldv, int m, const double* Y,
                          int ncol, void* out, long long ldo, const int* colmap, int accumulate,
                          const DevGrid& g, hipStream_t s, void* out_last = nullptr);

// Conversions between caller FP64 buffers and storage-type vectors.
// r = b - (A + i w)(zre + i zim) from azr = A zre, azi = A zim (b, r complex
// interleaved FP64).
hipError_t launch_shift_residual(Storage st, const double* b, const void* zre, const void* zim,
                                 const void* azr, const void* azi, double w, double* r, long long n,
                                 hipStream_t s);
hipError_t launch_load_complex(Storage st, const double* b, int part, void* out, long long n,
                               hipStream_t s);
hipError_t launch_load_real(Storage st, const double* src, void* out, long long n, hipStream_t s);
hipError_t launch_store_real(Storage st, const void* src, double* out, long long n, hipStream_t s);
hipError_t launch_store_complex(Storage st, const void* re, const void* im, double* out,
                                long long n, hipStream_t s);

// out = sn * re + cs * im - yhat  (yhat may be nullptr): Im(e^{iwT} z) - y_hat(T).
hipError_t launch_assemble(Storage st, const void* re, const void* im, const void* yhat,
                           double sn, double cs, double* out, long long n, hipStream_t s);

// p[0:n] = v (a kernel, so that it can sit in a captured graph).
hipError_t launch_fill(double* p, double v, long long n, hipStream_t s);

// w_c = A v_c for ncols columns at stride ld (columns of a block).
hipError_t launch_stencil_cols(Storage st, const void* v, void* w, long long ld, int ncols,
                               const DevGrid& g, const DevMats& m, hipStream_t s);

// Block kernels on FP64 matrix cores (kry_block.hip).
// partials[split][M x N] = X[:, :M]^T diag(w) Y[:, :N] over element splits.
// With X2 != nullptr, X is two segments: columns k < M1 at X + k ld and
// columns k >= M1 at X2 + (k - M1) ld.
int gram_splits(long long n, int M, int N);
// st2 (-1: st) is the element type of X2 and Y; a type other than st is
// supported for st = F32, st2 = F64 with Y = X2 and N = M - M1 <= 16.
hipError_t launch_gram(Storage st, const void* X, int M, const void* Y, int N, long long ld,
                       const double* w, long long n, double* partials, int nsplit, hipStream_t s,
                       const void* X2 = nullptr, int M1 = 0, int st2 = -1, const int* skip = nullptr);
// Out[:, :N] = (accumulate ? Out : 0) + alpha X[:, :M] C (C row-major M x N);
// X in one or two segments as for launch_gram.  Out must not overlap X,
// except for N <= 16 with M <= 256 and N <= 32 with M <= 128 (the
// column-owning kernel), where Out may be rows of X or X2 of the same
// element type (in place).
// st2, sto (-1: st): element types of X2 and Out; mixed types (st = F32
// with F64 in X2 and/or Out) for N <= 16, M <= 256 only.
hipError_t launch_gemm_nn(Storage st, const void* X, int M, const double* C, int N, void* Out,
                          long long ld, long long n, double alpha, int accumulate, hipStream_t s,
                          const void* X2 = nullptr, int M1 = 0, int st2 = -1, int sto = -1,
                          const int* skip = nullptr);
// Device finish of one Gram-Schmidt pass of an s-step block (kry_sstep.hip;
// one workgroup): from P = [V, S]^T M S ((M + s) x s row-major, reduced) it
// forms the projected Gram matrix, its Cholesky factor R, the coefficients
// K ((M + s) x s row-major) of the update [V, S] K = (S - V C) R^{-1}, and
// stores C, R (and on pass 1 the squared column norms of S) in `stash` for
// the Hessenberg algebra on the host; flags[0..3] = pass-1 factor valid,
// pass 1 final (the second pass is skipped: flags[1] is the skip flag of the
// pass-2 launches), pass-2 factor valid, basis too ill-conditioned.  A
// failed factor leaves K = [0; I] (S unchanged) and the host redoes the
// cycle.  s <= 16, M + s <= 256.
int sstep_stash_doubles(int M, int s);
hipError_t launch_sstep_fin(int pass, int M, int s, const double* P, double* K, double* stash,
                            int* flags, double one_pass_max, double one_pass_left, double cond_max,
                            hipStream_t st);
// Energy weight of every entry (mu on H planes, eps on E planes).
hipError_t launch_weights(const double* eps, const double* mu, double* w, long long N3,
                          hipStream_t s);

// Flux of z = zre + i zim through plane kf (per-block partials, *nblocks
// of them) and, if rhs != nullptr, the adjoint right-hand side P M^-1 dP/dz
// written into the complex interleaved rhs (zero elsewhere beforehand).
hipError_t launch_flux_seed(Storage st, const void* zre, const void* zim, int kf, const DevGrid& g,
                            const DevMats& m, double* partials, double* rhs, int* nblocks,
                            hipStream_t s);

// g[c] -= sum_{E planes} Re(x (b - i w z)) (the adjoint gradient term).
hipError_t launch_grad_acc(Storage st, const void* zre, const void* zim, const void* xre,
                           const void* xim, const double* b, double w, double* g, long long N3,
                           hipStream_t s);

// Projected problems of the residual-restarted inhomogeneous method
// (kry_rst.hip): for each of ncol time functions a (stored as column
// c = cmap[a], or a when cmap is null), march u' = -H u + beta f_c(t) e_1,
// u(0) = 0, over nt steps of length dt with the step propagators E (m x m),
// W (m x q) (column-major), El (q x m), Wl (q x q) (row-major) and the
// sampled sources fin[c ldf + j q + i]; writes the next residual source
// samples fout (same layout), u(nt dt) into uT[a m + .] and the Gauss-rule
// integral of |fout_c| (node weights gw, times dt) into resint[a].  All
// device pointers.  m <= rst_march_max_m(), q = 8, ldf >= nt q.
// Source compression for the restarted method (kry_rst.hip): mask[e] = 1
// where any of ncols complex interleaved columns of b (stride 2n doubles) is
// non-zero; C (nr x 2 ncols, column-major) = the energy-scaled real and
// imaginary parts sqrt(w) b at the rows idx; out_j (stride ld, zero
// elsewhere beforehand) = Q[:, j] / sqrt(w) scattered back to the rows idx.
hipError_t launch_nonzero_rows(const double* b, int ncols, long long n, unsigned char* mask, hipStream_t s);
hipError_t launch_gather_rows(const double* b, int ncols, long long n, const int* idx, int nr, const double* w,
                              double* C, hipStream_t s);
hipError_t launch_scatter_basis(Storage st, const double* Q, int nr, int r, const int* idx, const double* w,
                                void* out, long long ld, hipStream_t s);
// p[0:n] = pseudo-random values in [-1/2, 1/2) from a hash of the index.
hipError_t launch_fill_hash(void* p, Storage st, long long n, unsigned seed, hipStream_t s);
// Squared energy norms of the columns cols[0..ncol) of Z (stride ldz):
// partials[b * ncol + y] for the col_norm_blocks(N3) workgroups b, to be
// summed with launch_reduce(partials, col_norm_blocks(N3), ncol, ncol, out)
// (kry_rst.hip).  mu may be null (mu = 1).
int col_norm_blocks(long long N3);
hipError_t launch_col_norms(Storage st, const void* Z, long long ldz, const int* cols, int ncol, long long N3,
                            const double* eps, const double* mu, double* partials, hipStream_t s);
// The sampled time functions of the restarted method (kry_rst.hip):
// F[k ldf + j q + i] = ca_k sin(w_k t) + cb_k cos(w_k t), t = (j + gx[i]) dt,
// cw[3 k .. 3 k + 2] = (w_k, ca_k, cb_k); gx (q), cw device.
hipError_t launch_rst_samples(int nc, int nt, int q, double dt, const double* gx, const double* cw, double* F,
                              long long ldf, hipStream_t s);
int rst_march_max_m();
// Parallel-in-time form: with 1 <= L < nt, EL = E^L (m x m column-major,
// device) and `work` of rst_march_work(m, nt, ncol, L) doubles (device),
// the steps are scanned in chunks of L (local march, carry of the chunk
// starts with EL, final march); otherwise one sequential march.
long long rst_march_work(int m, int nt, int ncol, int L);
hipError_t launch_rst_march(int m, int q, int nt, int ncol, const double* E, const double* W,
                            const double* El, const double* Wl, const double* gw, double beta,
                            double hnext, double dt, const int* cmap, const double* fin, double* fout,
                            long long ldf, double* uT, double* resint, hipStream_t s, int L = 0,
                            const double* EL = nullptr, double* work = nullptr);

// out_{cmap[j]} += sum_{k < m} V_k Y[k + j m] for j < ncol (cmap may be
// nullptr: identity) on the matrix cores, the basis read once per 32
// outputs (kry_combine.hip).  Out columns must be distinct and not in V.
hipError_t launch_combine_mfma(Storage st, const void* V, long long ldv, int m, const double* Y, int ncol,
                               void* out, long long ldo, const int* cmap, long long n, hipStream_t s);

// Gradient of the flux at a finite time T (kry_adjoint.hip).
// F = sum over plane kf of Ex Hy_bar - Ey Hx_bar for the real FP64 field y
// (per-workgroup partial sums, *nblk of them) and, if r0 != nullptr, the
// adjoint start vector r0 = P M^-1 dF/dy at its six entries per plane cell
// (r0 zero elsewhere beforehand; storage type).
hipError_t launch_flux_inst(Storage st, const double* y, int kf, const DevGrid& g, const DevMats& m,
                            double* partials, void* r0, int* nblk, hipStream_t s);
// rhs = sn r0 + i (rT - cs r0) (complex interleaved FP64).
hipError_t launch_adj_rhs(Storage st, const void* r0, const void* rT, double sn, double cs, double* rhs,
                          long long n, hipStream_t s);
// g[c] += sum over the E rows p of cell c of sum_{i < nv, j < nw}
// V_i[p] C[i][j] W_j[p], C row-major with row stride frechet_cols();
// nw <= frechet_cols().  V, W: storage type, stride ld.
int frechet_cols();
hipError_t launch_frechet_acc(Storage st, const void* V, int nv, const void* W, int nw, const double* C,
                              long long ld, long long N3, double* g, hipStream_t s);

}  // namespace kry
