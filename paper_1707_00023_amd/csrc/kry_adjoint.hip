// Kernels of the gradient of the flux at a finite time T (the transient of
// equation (y_homo) included): the instantaneous flux of a real field and
// its adjoint seed, the right-hand side of the adjoint shifted solve, and
// the accumulation of the Frechet-derivative term of e^{-TA} from two
// Krylov bases (one of the forward transient, one of the adjoint one).
#include "kry_internal.h"

namespace kry {

namespace {

// Sum of v over the workgroup (kBlock threads) into *dst by thread 0.
__device__ __forceinline__ void wg_sum_store(double v, double* dst) {
  __shared__ double part[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) s += part[k];
    *dst = s;
  }
}

// One thread per (i, j) of plane kf: F = Ex Hy_bar - Ey Hx_bar with H_bar
// the mean of the H planes kf - 1 and kf, and the adjoint start vector
// r0 = P M^-1 dF/dy (P = +1 on H rows, -1 on E rows), written at the six
// entries F depends on (every other entry of r0 is zero beforehand):
//   dF/dEx = Hy_bar, dF/dEy = -Hx_bar, dF/dHy[kf-1, kf] = Ex / 2,
//   dF/dHx[kf-1, kf] = -Ey / 2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flux_inst(const double* __restrict__ y, int kf, DevGrid g,
                                                      DevMats mt, double* __restrict__ partials,
                                                      T* __restrict__ r0) {
  const long long N2 = (long long)g.nx * g.ny;
  const long long N3 = g.N3;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  double f = 0.0;
  if (t < N2) {
    const long long c1 = (long long)kf * N2 + t;
    const long long c0 = c1 - N2;
    const double hx = 0.5 * (y[c0] + y[c1]);
    const double hy = 0.5 * (y[N3 + c0] + y[N3 + c1]);
    const double ex = y[3 * N3 + c1], ey = y[4 * N3 + c1];
    f = ex * hy - ey * hx;
    if (r0) {
      const double ie = mt.inv_eps[c1];
      const double im0 = mt.inv_mu ? mt.inv_mu[c0] : 1.0;
      const double im1 = mt.inv_mu ? mt.inv_mu[c1] : 1.0;
      r0[3 * N3 + c1] = (T)(-hy * ie);
      r0[4 * N3 + c1] = (T)(hx * ie);
      r0[N3 + c0] = (T)(0.5 * ex * im0);
      r0[N3 + c1] = (T)(0.5 * ex * im1);
      r0[c0] = (T)(-0.5 * ey * im0);
      r0[c1] = (T)(-0.5 * ey * im1);
    }
  }
  wg_sum_store(f, partials + blockIdx.x);
}

// rhs = sn r0 + i (rT - cs r0), complex interleaved FP64.
template <typename T>
__global__ void k_adj_rhs(const T* __restrict__ r0, const T* __restrict__ rT, double sn, double cs,
                          double* __restrict__ rhs, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const double a = (double)r0[e];
  rhs[2 * e] = sn * a;
  rhs[2 * e + 1] = (double)rT[e] - cs * a;
}

constexpr int kFW = 64;  // columns of W (and of C) per launch

// g[c] += sum_{p in Ex, Ey, Ez} sum_{i < nv} V_i[p, c] sum_{j < nw} C[i][j] W_j[p, c]
// (C row-major with row stride kFW).  One thread per cell; the thread keeps
// its 64 W entries of the current component in registers and walks the rows
// of C, which are the same for every thread (scalar loads).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_frechet_acc(const T* __restrict__ V, int nv,
                                                        const T* __restrict__ W, int nw,
                                                        const double* __restrict__ C, long long ld,
                                                        long long N3, double* __restrict__ g) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= N3) return;
  double acc = 0.0;
  for (int p = 3; p < 6; ++p) {
    const long long e = p * N3 + c;
    double w[kFW];
#pragma unroll
    for (int j = 0; j < kFW; ++j) w[j] = j < nw ? (double)W[(long long)j * ld + e] : 0.0;
    for (int i = 0; i < nv; ++i) {
      const double* Ci = C + (long long)i * kFW;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
      for (int j = 0; j < kFW; j += 4) {
        t0 += Ci[j] * w[j];
        t1 += Ci[j + 1] * w[j + 1];
        t2 += Ci[j + 2] * w[j + 2];
        t3 += Ci[j + 3] * w[j + 3];
      }
      acc += (double)V[(long long)i * ld + e] * ((t0 + t1) + (t2 + t3));
    }
  }
  g[c] += acc;
}

inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int frechet_cols() { return kFW; }

hipError_t launch_flux_inst(Storage st, const double* y, int kf, const DevGrid& g, const DevMats& m,
                            double* partials, void* r0, int* nblk, hipStream_t s) {
  const long long N2 = (long long)g.nx * g.ny;
  const unsigned nb = nblocks(N2);
  *nblk = (int)nb;
  if (st == F64)
    hipLaunchKernelGGL(k_flux_inst<double>, dim3(nb), dim3(kBlock), 0, s, y, kf, g, m, partials,
                       (double*)r0);
  else
    hipLaunchKernelGGL(k_flux_inst<float>, dim3(nb), dim3(kBlock), 0, s, y, kf, g, m, partials,
                       (float*)r0);
  return hipGetLastError();
}

hipError_t launch_adj_rhs(Storage st, const void* r0, const void* rT, double sn, double cs, double* rhs,
                          long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (st == F64)
    hipLaunchKernelGGL(k_adj_rhs<double>, dim3(nblocks(n)), dim3(kBlock), 0, s, (const double*)r0,
                       (const double*)rT, sn, cs, rhs, n);
  else
    hipLaunchKernelGGL(k_adj_rhs<float>, dim3(nblocks(n)), dim3(kBlock), 0, s, (const float*)r0,
                       (const float*)rT, sn, cs, rhs, n);
  return hipGetLastError();
}

hipError_t launch_frechet_acc(Storage st, const void* V, int nv, const void* W, int nw, const double* C,
                              long long ld, long long N3, double* g, hipStream_t s) {
  if (nv <= 0 || nw <= 0 || N3 <= 0) return hipSuccess;
  if (nw > kFW) return hipErrorInvalidValue;
  if (st == F64)
    hipLaunchKernelGGL(k_frechet_acc<double>, dim3(nblocks(N3)), dim3(kBlock), 0, s, (const double*)V, nv,
                       (const double*)W, nw, C, ld, N3, g);
  else
    hipLaunchKernelGGL(k_frechet_acc<float>, dim3(nblocks(N3)), dim3(kBlock), 0, s, (const float*)V, nv,
                       (const float*)W, nw, C, ld, N3, g);
  return hipGetLastError();
}

}  // namespace kry
