// Projected problems of the residual-restarted inhomogeneous Krylov method
// on the GPU: the march of u' = -H u + beta f(t) e_1 over the sampled time
// grid for many time functions at once.
//
// Per time step j (length dt, q Gauss nodes), with a = beta f at the step's
// nodes and the step propagators of the restart (computed on the host from
// H: E = e^{-dt H}, W the weights of the node samples, El / Wl the same for
// e_m^T u at the nodes):
//   fout[j q + i] = -hnext (El[i] u + Wl[i] a)      (the next residual source)
//   u            <- E u + W a.
// The recurrence is linear in u, so it is scanned in parallel over time:
// the steps are cut into P chunks of L steps; every chunk is first marched
// from u = 0 (its own contribution v_p), one wave per (chunk, time function);
// then one wave per time function carries the chunk starts,
// u_{p+1} = E^L u_p + v_p, with E^L = e^{-L dt H} from the host; then every
// chunk is marched again from its start, writing the residual samples.
// The chain of dependent steps is L + P + L long instead of P L.
// Lane r owns u_r and keeps row r of E and W in registers; u and a reach
// the other lanes by lane broadcasts.  The residual samples El u take 8
// values of El per lane, El[r mod 8][8 (r div 8) + kk] for kk < 8: each lane
// gathers its 8 entries of u by lane shuffles, and the 8 lane groups are
// summed by three xor shuffles (a full row of El per lane would double the
// registers and leave one wave per SIMD).
#include "kry_internal.h"

namespace kry {

namespace {

constexpr int kRstM = 64;  // largest projected dimension of the GPU march
constexpr int kRstQ = 8;   // nodes per time step

// Value of lane `lane` of v, in every lane (lane must be wave-uniform).
__device__ __forceinline__ double bcast(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// One wave per (chunk p = blockIdx.x, time function a = blockIdx.y): the
// steps [p L, min(nt, (p + 1) L)) from u = u0[a P + p] (zero if u0 is null).
// OUT: also write the residual samples of those steps and the chunk's share
// of the integral of |fout| into rpart[a P + p].  The end state goes to
// uend[a P + p] (if given) and, for the last chunk, to uT[a].  Four partial
// sums per dot break the chain of dependent FMAs.
template <bool OUT>
__global__ __launch_bounds__(64) void k_rst_march(int m, int nt, int L, const double* __restrict__ E,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ El,
                                                  const double* __restrict__ Wl,
                                                  const double* __restrict__ gw, double beta,
                                                  double hnext, double dt, const int* __restrict__ cmap,
                                                  const double* __restrict__ fin,
                                                  double* __restrict__ fout, long long ldf,
                                                  const double* __restrict__ u0, double* __restrict__ uend,
                                                  double* __restrict__ uT, double* __restrict__ rpart) {
  const int r = threadIdx.x;
  const int p = blockIdx.x, P = gridDim.x;
  const int a = blockIdx.y;
  const int col = cmap ? cmap[a] : a;
  const long long slot = (long long)a * P + p;
  const double* fi = fin + (long long)col * ldf;
  double* fo = OUT ? fout + (long long)col * ldf : nullptr;
  const int j0 = p * L;
  const int j1 = min(nt, j0 + L);
  static_assert(kRstM == 8 * kRstQ, "the residual-sample layout takes 8 lane groups of q lanes");
  double er[kRstM], el[kRstQ], wr[kRstQ], wl[kRstQ];
  const int gbase = (r / kRstQ) * 8;  // first u entry of this lane's group
#pragma unroll
  for (int k = 0; k < kRstM; ++k) er[k] = (r < m && k < m) ? E[r + (long long)k * m] : 0.0;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    el[kk] = (OUT && gbase + kk < m) ? El[(long long)(r % kRstQ) * m + gbase + kk] : 0.0;
#pragma unroll
  for (int l = 0; l < kRstQ; ++l) {
    wr[l] = r < m ? W[r + (long long)l * m] : 0.0;
    wl[l] = (OUT && r < kRstQ) ? Wl[r * kRstQ + l] : 0.0;
  }
  const double wnode = r < kRstQ ? gw[r] : 0.0;
  double u = (u0 && r < m) ? u0[slot * m + r] : 0.0;
  double anext = (r < kRstQ && j0 < j1) ? beta * fi[(long long)j0 * kRstQ + r] : 0.0;
  double racc = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double acur = anext;
    if (r < kRstQ && j + 1 < j1) anext = beta * fi[(long long)(j + 1) * kRstQ + r];
    double av[kRstQ];
#pragma unroll
    for (int l = 0; l < kRstQ; ++l) av[l] = bcast(acur, l);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, t = 0.0;
    if (OUT) {  // El u: this lane's 8 terms, then the sum over the 8 lane groups
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) t += el[kk] * __shfl(u, gbase + kk, 64);
      t += __shfl_xor(t, 8, 64);
      t += __shfl_xor(t, 16, 64);
      t += __shfl_xor(t, 32, 64);
    }
#pragma unroll
    for (int k = 0; k < kRstM; k += 4) {
      s0 += er[k] * bcast(u, k);
      s1 += er[k + 1] * bcast(u, k + 1);
      s2 += er[k + 2] * bcast(u, k + 2);
      s3 += er[k + 3] * bcast(u, k + 3);
    }
    double sa = 0.0, ta = 0.0;
#pragma unroll
    for (int l = 0; l < kRstQ; ++l) {
      sa += wr[l] * av[l];
      if (OUT) ta += wl[l] * av[l];
    }
    if (OUT && r < kRstQ) {
      const double f = -hnext * (t + ta);
      fo[(long long)j * kRstQ + r] = f;
      racc += wnode * fabs(f);
    }
    u = r < m ? ((s0 + s1) + (s2 + s3)) + sa : 0.0;
  }
  if (uend && r < m) uend[slot * m + r] = u;
  if (uT && p == P - 1 && r < m) uT[(long long)a * m + r] = u;
  if (OUT) {
    // the q node lanes' sums (Gauss weights times dt)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) racc += __shfl_xor(racc, off, 64);
    if (r == 0) rpart[slot] = dt * racc;
  }
}

// One wave per time function: chunk starts u_0 = 0, u_{p+1} = EL u_p + v_p
// (EL = E^L, column-major m x m), written to ustart[a P + p].
__global__ __launch_bounds__(64) void k_rst_carry(int m, int P, const double* __restrict__ EL,
                                                  const double* __restrict__ v, double* __restrict__ ustart) {
  const int r = threadIdx.x;
  const int a = blockIdx.x;
  double er[kRstM];
#pragma unroll
  for (int k = 0; k < kRstM; ++k) er[k] = (r < m && k < m) ? EL[r + (long long)k * m] : 0.0;
  double u = 0.0;
  for (int p = 0; p < P; ++p) {
    const long long slot = (long long)a * P + p;
    if (r < m) ustart[slot * m + r] = u;
    const double vp = r < m ? v[slot * m + r] : 0.0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int k = 0; k < kRstM; k += 4) {
      s0 += er[k] * bcast(u, k);
      s1 += er[k + 1] * bcast(u, k + 1);
      s2 += er[k + 2] * bcast(u, k + 2);
      s3 += er[k + 3] * bcast(u, k + 3);
    }
    u = r < m ? ((s0 + s1) + (s2 + s3)) + vp : 0.0;
  }
}

// resint[a] = sum_p rpart[a P + p], in chunk order.
__global__ __launch_bounds__(64) void k_rst_sum(int ncol, int P, const double* __restrict__ rpart,
                                                double* __restrict__ resint) {
  const int a = blockIdx.x * 64 + threadIdx.x;
  if (a >= ncol) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += rpart[(long long)a * P + p];
  resint[a] = s;
}

}  // namespace

namespace {

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

namespace {

// Pseudo-random values in [-1/2, 1/2) from an integer hash of the index (a
// fixed, reproducible vector for timing runs).
template <typename T>
__global__ __launch_bounds__(256) void k_fill_hash(T* __restrict__ p, long long n, unsigned seed) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  unsigned h = (unsigned)i * 2654435761u ^ seed;
  h ^= h >> 16;
  h *= 2246822519u;
  h ^= h >> 13;
  h *= 3266489917u;
  h ^= h >> 16;
  p[i] = T((double)h * (1.0 / 4294967296.0) - 0.5);
}


// Squared energy norms of many columns in one launch: partials[b ncol + y]
// = sum over the cells of workgroup b of sum_p w_p x_p^2, x = column
// cols[y] of Z (w: mu on the H planes, eps on the E planes; per cell the
// products and sums of the single-column dot kernel).  grid (ceil(N3 /
// 256), ncol), one cell per thread.
template <typename T, bool HAS_MU>
__global__ __launch_bounds__(256) void k_col_norms(const T* __restrict__ Z, long long ldz,
                                                   const int* __restrict__ cols, int ncol, long long N3,
                                                   const double* __restrict__ eps, const double* __restrict__ mu,
                                                   double* __restrict__ partials) {
  __shared__ double part[4];
  const int y = blockIdx.y;
  const T* x = Z + (long long)cols[y] * ldz;
  const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (c < N3) {
    const double we = eps[c];
    const double wh = HAS_MU ? mu[c] : 1.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double xv = (double)x[p * N3 + c];
      const double xm = (p < 3 ? wh : we) * xv;
      s += xm * xv;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[(long long)blockIdx.x * ncol + y] = (part[0] + part[1]) + (part[2] + part[3]);
}


// Sampled time functions of the restarted method: F[k ldf + j q + i] =
// ca_k sin(w_k t) + cb_k cos(w_k t) at t = (j + gx[i]) dt, for nc functions
// (cw = w, ca, cb of function k at 3 k), nt steps and q nodes per step.
__global__ __launch_bounds__(256) void k_rst_samples(int nc, int nt, int q, double dt, const double* __restrict__ gx,
                                                     const double* __restrict__ cw, double* __restrict__ F,
                                                     long long ldf) {
  const long long per = (long long)nt * q;
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= per * nc) return;
  const int k = (int)(idx / per);
  const long long r = idx - (long long)k * per;
  const int j = (int)(r / q), i = (int)(r - (long long)j * q);
  const double t = (j + gx[i]) * dt;
  const double w = cw[3 * k], ca = cw[3 * k + 1], cb = cw[3 * k + 2];
  F[(long long)k * ldf + r] = ca * sin(w * t) + cb * cos(w * t);
}

}  // namespace

hipError_t launch_fill_hash(void* p, Storage st, long long n, unsigned seed, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256));
  if (st == F64)
    hipLaunchKernelGGL(k_fill_hash<double>, grid, dim3(256), 0, s, (double*)p, n, seed);
  else
    hipLaunchKernelGGL(k_fill_hash<float>, grid, dim3(256), 0, s, (float*)p, n, seed);
  return hipGetLastError();
}

int col_norm_blocks(long long N3) { return (int)((N3 + 255) / 256); }

hipError_t launch_col_norms(Storage st, const void* Z, long long ldz, const int* cols, int ncol, long long N3,
                            const double* eps, const double* mu, double* partials, hipStream_t s) {
  if (ncol <= 0 || N3 <= 0) return hipSuccess;
  if (ncol > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)col_norm_blocks(N3), (unsigned)ncol);
  if (st == F64) {
    if (mu)
      hipLaunchKernelGGL((k_col_norms<double, true>), grid, dim3(256), 0, s, (const double*)Z, ldz, cols, ncol, N3,
                         eps, mu, partials);
    else
      hipLaunchKernelGGL((k_col_norms<double, false>), grid, dim3(256), 0, s, (const double*)Z, ldz, cols, ncol,
                         N3, eps, mu, partials);
  } else {
    if (mu)
      hipLaunchKernelGGL((k_col_norms<float, true>), grid, dim3(256), 0, s, (const float*)Z, ldz, cols, ncol, N3,
                         eps, mu, partials);
    else
      hipLaunchKernelGGL((k_col_norms<float, false>), grid, dim3(256), 0, s, (const float*)Z, ldz, cols, ncol, N3,
                         eps, mu, partials);
  }
  return hipGetLastError();
}

hipError_t launch_rst_samples(int nc, int nt, int q, double dt, const double* gx, const double* cw, double* F,
                              long long ldf, hipStream_t s) {
  if (nc <= 0 || nt <= 0 || q <= 0) return hipSuccess;
  if (ldf < (long long)nt * q) return hipErrorInvalidValue;
  const long long total = (long long)nc * nt * q;
  hipLaunchKernelGGL(k_rst_samples, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, nc, nt, q, dt, gx, cw, F,
                     ldf);
  return hipGetLastError();
}

int rst_march_max_m() { return kRstM; }

long long rst_march_work(int m, int nt, int ncol, int L) {
  if (L < 1 || L >= nt) return 0;
  const long long P = (nt + L - 1) / L;
  return 2LL * ncol * P * m + (long long)ncol * P;
}

hipError_t launch_rst_march(int m, int q, int nt, int ncol, const double* E, const double* W,
                            const double* El, const double* Wl, const double* gw, double beta,
                            double hnext, double dt, const int* cmap, const double* fin, double* fout,
                            long long ldf, double* uT, double* resint, hipStream_t s, int L,
                            const double* EL, double* work) {
  if (m < 1 || m > kRstM || q != kRstQ || ncol < 1 || nt < 1 || ldf < (long long)nt * q)
    return hipErrorInvalidValue;
  if (L < 1 || L >= nt || !EL || !work) {  // one chunk
    hipLaunchKernelGGL(k_rst_march<true>, dim3(1, ncol), dim3(64), 0, s, m, nt, nt, E, W, El, Wl, gw, beta,
                       hnext, dt, cmap, fin, fout, ldf, nullptr, nullptr, uT, resint);
    return hipGetLastError();
  }
  const int P = (nt + L - 1) / L;
  double* v = work;
  double* ustart = v + (long long)ncol * P * m;
  double* rpart = ustart + (long long)ncol * P * m;
  hipLaunchKernelGGL(k_rst_march<false>, dim3(P, ncol), dim3(64), 0, s, m, nt, L, E, W, El, Wl, gw, beta,
                     hnext, dt, cmap, fin, nullptr, ldf, nullptr, v, nullptr, nullptr);
  hipLaunchKernelGGL(k_rst_carry, dim3(ncol), dim3(64), 0, s, m, P, EL, v, ustart);
  hipLaunchKernelGGL(k_rst_march<true>, dim3(P, ncol), dim3(64), 0, s, m, nt, L, E, W, El, Wl, gw, beta,
                     hnext, dt, cmap, fin, fout, ldf, ustart, nullptr, uT, rpart);
  hipLaunchKernelGGL(k_rst_sum, dim3((ncol + 63) / 64), dim3(64), 0, s, ncol, P, rpart, resint);
  return hipGetLastError();
}

}  // namespace kry
