// Block (multi-column) kernels for gfx950: tall-skinny Gram and update
// products of block Gram-Schmidt on FP64 matrix cores.
//
// A block of vectors is a set of columns in the usual layout (each column a
// contiguous n-vector, stride ld), so the reduction dimension of V^T W is the
// contiguous one.  Both products use v_mfma_f64_16x16x4f64 (D[16x16] +=
// A[16x4] B[4x16] in FP64).  Operand lane layout of that instruction: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the result holds
// D[4 r + l / 16][l % 16] in its r-th FP64 register (r = 0..3).
#include "kry_internal.h"

namespace kry {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// partials[split][M x N] = X[:, 0:M]^T diag(w) Y[:, 0:N] over the elements
// [split * kchunk, (split + 1) * kchunk).  Workgroup = 4 waves = a 32 x 32
// output tile (one 16 x 16 tile per wave); grid (nsplit, ceil(M/32),
// ceil(N/32)).  Out-of-range rows, columns and elements contribute zeros.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_tn(const T* __restrict__ X, int M,
                                                 const T* __restrict__ Y, int N, long long ld,
                                                 const double* __restrict__ w, long long n,
                                                 long long kchunk, double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32 + (wave >> 1) * 16;
  const int n0 = blockIdx.z * 32 + (wave & 1) * 16;
  const int i = lane & 15, kk = lane >> 4;
  const long long e_begin = (long long)blockIdx.x * kchunk;
  const long long e_end = min(n, e_begin + kchunk);
  const bool arow = m0 + i < M, bcol = n0 + i < N;
  const T* xc = X + (long long)(arow ? m0 + i : 0) * ld;
  const T* yc = Y + (long long)(bcol ? n0 + i : 0) * ld;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (long long e0 = e_begin; e0 < e_end; e0 += 4) {
    const long long e = e0 + kk;
    const bool ok = e < e_end;
    const double a = (arow && ok) ? (double)xc[e] : 0.0;
    const double b = (bcol && ok) ? w[e] * (double)yc[e] : 0.0;
    acc = mfma16(a, b, acc);
  }
  double* out = partials + (long long)blockIdx.x * M * N;
  const int col = n0 + i;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + 4 * r + kk;
    if (row < M && col < N) out[(long long)row * N + col] = acc[r];
  }
}

// Out[:, j] = (accumulate ? Out[:, j] : 0) + alpha sum_k X[:, k] C[k][j] for
// j < N (C row-major M x N, FP64).  Each wave computes 16 elements x 64
// columns (four 16 x 16 tiles of Out^T = C^T X^T): A = C^T (from C), B =
// X^T (16 consecutive elements per k: coalesced).  grid (ceil(n / 64),
// ceil(N / 64)).  Out may not overlap X.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nn(const T* __restrict__ X, int M,
                                                 const double* __restrict__ C, int N,
                                                 T* __restrict__ Out, long long ld, long long n,
                                                 double alpha, int accumulate) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e0 = ((long long)blockIdx.x * 4 + wave) * 16;
  const int jbase = blockIdx.y * 64;
  const int i = lane & 15, kk = lane >> 4;
  const long long e = e0 + i;
  const bool eok = e < n;
  v4d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < M; k0 += 4) {
    const int k = k0 + kk;
    const bool kok = k < M;
    const double b = (kok && eok) ? (double)X[(long long)k * ld + e] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = jbase + t * 16 + i;
      const double a = (kok && j < N) ? C[(long long)k * N + j] : 0.0;
      acc[t] = mfma16(a, b, acc[t]);
    }
  }
  if (!eok) return;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = jbase + t * 16 + 4 * r + kk;
      if (j < N) {
        T* o = Out + (long long)j * ld + e;
        const double prev = accumulate ? (double)*o : 0.0;
        *o = T(prev + alpha * acc[t][r]);
      }
    }
  }
}

// Energy weights per entry: mu on the three H planes, eps on the E planes.
__global__ void k_weights(const double* __restrict__ eps, const double* __restrict__ mu,
                          double* __restrict__ w, long long N3) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= N3) return;
  const double e = eps[c], m = mu ? mu[c] : 1.0;
  for (int p = 0; p < 3; ++p) w[p * N3 + c] = m;
  for (int p = 3; p < 6; ++p) w[p * N3 + c] = e;
}

}  // namespace

int gram_splits(long long n, int M, int N) {
  const int tiles = ((M + 31) / 32) * ((N + 31) / 32);
  long long s = 2048 / tiles;
  if (s < 1) s = 1;
  const long long maxs = (n + 255) / 256;
  if (s > maxs) s = maxs;
  return (int)s;
}

hipError_t launch_gram(Storage st, const void* X, int M, const void* Y, int N, long long ld,
                       const double* w, long long n, double* partials, int nsplit, hipStream_t s) {
  long long kchunk = (n + nsplit - 1) / nsplit;
  kchunk = (kchunk + 3) / 4 * 4;
  const dim3 grid(nsplit, (M + 31) / 32, (N + 31) / 32);
  if (st == F64)
    hipLaunchKernelGGL(k_gram_tn<double>, grid, dim3(256), 0, s, (const double*)X, M,
                       (const double*)Y, N, ld, w, n, kchunk, partials);
  else
    hipLaunchKernelGGL(k_gram_tn<float>, grid, dim3(256), 0, s, (const float*)X, M,
                       (const float*)Y, N, ld, w, n, kchunk, partials);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(Storage st, const void* X, int M, const double* C, int N, void* Out,
                          long long ld, long long n, double alpha, int accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 63) / 64), (N + 63) / 64);
  if (st == F64)
    hipLaunchKernelGGL(k_gemm_nn<double>, grid, dim3(256), 0, s, (const double*)X, M, C, N,
                       (double*)Out, ld, n, alpha, accumulate);
  else
    hipLaunchKernelGGL(k_gemm_nn<float>, grid, dim3(256), 0, s, (const float*)X, M, C, N,
                       (float*)Out, ld, n, alpha, accumulate);
  return hipGetLastError();
}

hipError_t launch_weights(const double* eps, const double* mu, double* w, long long N3,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_weights, dim3((unsigned)((N3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     eps, mu, w, N3);
  return hipGetLastError();
}

}  // namespace kry
