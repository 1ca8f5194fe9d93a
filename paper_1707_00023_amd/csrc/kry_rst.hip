// Projected problems of the residual-restarted inhomogeneous Krylov method
// on the GPU: the march of u' = -H u + beta f(t) e_1 over the sampled time
// grid for many time functions at once (one wave per time function).
//
// Per time step j (length dt, q Gauss nodes), with a = beta f at the step's
// nodes and the step propagators of the restart (computed on the host from
// H: E = e^{-dt H}, W the weights of the node samples, El / Wl the same for
// e_m^T u at the nodes):
//   fout[j q + i] = -hnext (El[i] u + Wl[i] a)      (the next residual source)
//   u            <- E u + W a.
// Lane r owns row r of u and keeps row r of E and W in registers; u and a
// live in LDS, double-buffered, so one barrier per step suffices.
#include "kry_internal.h"

namespace kry {

namespace {

constexpr int kRstM = 64;  // largest projected dimension of the GPU march
constexpr int kRstQ = 8;   // nodes per time step

__global__ __launch_bounds__(64) void k_rst_march(int m, int nt, const double* __restrict__ E,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ El,
                                                  const double* __restrict__ Wl,
                                                  const double* __restrict__ gw, double beta,
                                                  double hnext, double dt, const int* __restrict__ cmap,
                                                  const double* __restrict__ fin,
                                                  double* __restrict__ fout, long long ldf,
                                                  double* __restrict__ uT, double* __restrict__ resint) {
  __shared__ double su[2][kRstM];
  __shared__ double sa[2][kRstQ];
  __shared__ double sEl[kRstM][kRstQ];  // El transposed: [k][node]
  __shared__ double sWl[kRstQ][kRstQ];
  const int r = threadIdx.x;
  const int col = cmap ? cmap[blockIdx.x] : (int)blockIdx.x;
  const double* fi = fin + (long long)col * ldf;
  double* fo = fout + (long long)col * ldf;
  double er[kRstM], wr[kRstQ];
#pragma unroll
  for (int k = 0; k < kRstM; ++k) er[k] = (r < m && k < m) ? E[r + (long long)k * m] : 0.0;
#pragma unroll
  for (int l = 0; l < kRstQ; ++l) wr[l] = r < m ? W[r + (long long)l * m] : 0.0;
  for (int k = 0; k < m; ++k)
    if (r < kRstQ) sEl[k][r] = El[(long long)r * m + k];
  if (r < kRstQ)
#pragma unroll
    for (int l = 0; l < kRstQ; ++l) sWl[r][l] = Wl[r * kRstQ + l];
  su[0][r] = 0.0;
  if (r < kRstQ) sa[0][r] = nt > 0 ? beta * fi[r] : 0.0;
  const double wnode = r < kRstQ ? gw[r] : 0.0;
  double racc = 0.0;
  __syncthreads();
  for (int j = 0; j < nt; ++j) {
    const int cur = j & 1, nxt = cur ^ 1;
    // next step's source samples into the other buffer
    if (r < kRstQ) sa[nxt][r] = (j + 1 < nt) ? beta * fi[(long long)(j + 1) * kRstQ + r] : 0.0;
    const double* u = su[cur];
    const double* a = sa[cur];
    if (r < kRstQ) {
      double v = 0.0;
      for (int k = 0; k < m; ++k) v += sEl[k][r] * u[k];
#pragma unroll
      for (int l = 0; l < kRstQ; ++l) v += sWl[r][l] * a[l];
      const double f = -hnext * v;
      fo[(long long)j * kRstQ + r] = f;
      racc += wnode * fabs(f);
    }
    double un = 0.0;
#pragma unroll
    for (int k = 0; k < kRstM; ++k) un += er[k] * u[k];
#pragma unroll
    for (int l = 0; l < kRstQ; ++l) un += wr[l] * a[l];
    su[nxt][r] = r < m ? un : 0.0;
    __syncthreads();
  }
  if (r < m) uT[(long long)blockIdx.x * m + r] = su[nt & 1][r];
  // integral of |fout|: the q node lanes' sums (Gauss weights times dt)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) racc += __shfl_xor(racc, off, 64);
  if (r == 0) resint[blockIdx.x] = dt * racc;
}

// mask[e] = 1 where any of the ncols complex interleaved columns of b
// (stride 2 n doubles) is non-zero at entry e.
__global__ __launch_bounds__(256) void k_nonzero_rows(const double* __restrict__ b, int ncols, long long n,
                                                      unsigned char* __restrict__ mask) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  unsigned char nz = 0;
  for (int c = 0; c < ncols && !nz; ++c) {
    const double* bc = b + (long long)c * 2 * n + 2 * e;
    nz = (bc[0] != 0.0 || bc[1] != 0.0);
  }
  mask[e] = nz;
}

// C[i + (2 c + p) nr] = sqrt(w[idx[i]]) * (p ? Im : Re) b_c[idx[i]]
__global__ __launch_bounds__(256) void k_gather_rows(const double* __restrict__ b, int ncols, long long n,
                                                     const int* __restrict__ idx, int nr,
                                                     const double* __restrict__ w, double* __restrict__ C) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nr) return;
  const long long e = idx[i];
  const double sw = sqrt(w[e]);
  for (int c = 0; c < ncols; ++c) {
    const double* bc = b + (long long)c * 2 * n + 2 * e;
    C[i + (long long)(2 * c) * nr] = sw * bc[0];
    C[i + (long long)(2 * c + 1) * nr] = sw * bc[1];
  }
}

// out_j[idx[i]] = Q[i + j nr] / sqrt(w[idx[i]]) for j < r (out_j at stride
// ld, zero elsewhere beforehand).
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_basis(const double* __restrict__ Q, int nr, int r,
                                                       const int* __restrict__ idx,
                                                       const double* __restrict__ w, T* __restrict__ out,
                                                       long long ld) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nr) return;
  const long long e = idx[i];
  const double isw = 1.0 / sqrt(w[e]);
  for (int j = 0; j < r; ++j) out[(long long)j * ld + e] = T(Q[i + (long long)j * nr] * isw);
}

}  // namespace

hipError_t launch_nonzero_rows(const double* b, int ncols, long long n, unsigned char* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_nonzero_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, ncols, n, mask);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double* b, int ncols, long long n, const int* idx, int nr, const double* w,
                              double* C, hipStream_t s) {
  if (nr < 1) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, b, ncols, n, idx, nr, w,
                     C);
  return hipGetLastError();
}

hipError_t launch_scatter_basis(Storage st, const double* Q, int nr, int r, const int* idx, const double* w,
                                void* out, long long ld, hipStream_t s) {
  if (nr < 1 || r < 1) return hipSuccess;
  const dim3 grid((unsigned)((nr + 255) / 256));
  if (st == F64)
    hipLaunchKernelGGL(k_scatter_basis<double>, grid, dim3(256), 0, s, Q, nr, r, idx, w, (double*)out, ld);
  else
    hipLaunchKernelGGL(k_scatter_basis<float>, grid, dim3(256), 0, s, Q, nr, r, idx, w, (float*)out, ld);
  return hipGetLastError();
}

int rst_march_max_m() { return kRstM; }

hipError_t launch_rst_march(int m, int q, int nt, int ncol, const double* E, const double* W,
                            const double* El, const double* Wl, const double* gw, double beta,
                            double hnext, double dt, const int* cmap, const double* fin, double* fout,
                            long long ldf, double* uT, double* resint, hipStream_t s) {
  if (m < 1 || m > kRstM || q != kRstQ || ncol < 1 || nt < 1 || ldf < (long long)nt * q)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rst_march, dim3(ncol), dim3(64), 0, s, m, nt, E, W, El, Wl, gw, beta, hnext, dt,
                     cmap, fin, fout, ldf, uT, resint);
  return hipGetLastError();
}

}  // namespace kry
