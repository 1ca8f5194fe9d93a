// Basis combination for many outputs on FP64 matrix cores: out_{cmap[j]} +=
// sum_{k < m} V_k Y[k + j m] for j < ncol (Y column-major m x ncol, m <= 80).
// This is a tall-skinny product V Y: a wave computes 16-entry x 32-column
// tiles with v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] =
// Y[k][j] and B[l / 16][l % 16] = V_k[e]; the result holds output column
// 4 r + l / 16 of a 16-column tile, entry l % 16, in its r-th register), so
// the basis is read once per 32 outputs where the vector-ALU combination
// reads it once per 8.  For the restarted method's batched form, where one
// basis serves hundreds of time functions.  The outputs' read-modify-write
// is most of the traffic (2 ncol vectors against m), so the kernel is built
// around it: the old output values of a tile are loaded before its MFMAs,
// their latency hidden behind the dense work, and 32 columns per wave (not
// 64) leave registers for three waves per SIMD (measured at 96^3, m = 64,
// 256 outputs: 6.2 ms against 10.6 ms for 64 columns per wave without the
// early loads).
#include "kry_internal.h"

namespace kry {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// One wave owns 32 output columns (two 16-column tiles) and keeps their
// coefficients, the MFMA A operands for every k, in registers (loaded once);
// it then streams tpw 16-entry tiles of the basis through them, the four
// waves of a workgroup on 64 consecutive entries at a time.  Workgroup b
// covers entry block eb and column group cg with b = ((eb / 8) ncg + cg) 8 +
// eb mod 8: the column groups of an entry block run on one XCD at nearby
// dispatch times, so its basis entries come from HBM once.
// MC: 16-row chunks of k (m <= 16 MC).
template <typename T, int MC>
__global__ __launch_bounds__(256) void k_combine_mfma(const T* __restrict__ V, long long ldv, int m,
                                                      const double* __restrict__ Y, int ncol, T* __restrict__ out,
                                                      long long ldo, const int* __restrict__ cmap, long long n,
                                                      int tpw, int ncg, long long neb) {
  constexpr int NT = 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long bt = blockIdx.x >> 3;
  const int cg = (int)(bt % ncg);
  const long long eb = (bt / ncg) * 8 + (blockIdx.x & 7);
  if (eb >= neb) return;
  const int jbase = cg * 16 * NT;
  const int i = lane & 15, kk = lane >> 4;
  double a[MC][4][NT];
#pragma unroll
  for (int c = 0; c < MC; ++c)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int k = 16 * c + 4 * u + kk, j = jbase + t * 16 + i;
        a[c][u][t] = (k < m && j < ncol) ? Y[k + (long long)j * m] : 0.0;
      }
  T* op[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = jbase + t * 16 + 4 * r + kk;
      op[t][r] = j < ncol ? out + (long long)(cmap ? cmap[j] : j) * ldo : nullptr;
    }
  const long long tile0 = eb * 4 * tpw + wave;
  for (int tt = 0; tt < tpw; ++tt) {
    const long long e0 = (tile0 + 4LL * tt) * 16;
    if (e0 >= n) break;
    const long long e = e0 + i;
    const bool eok = e < n;
    double prev[NT][4];  // the old outputs, loaded first
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) prev[t][r] = (op[t][r] && eok) ? (double)op[t][r][e] : 0.0;
    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      double b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 16 * c + 4 * u + kk;
        b[u] = (k < m && eok) ? (double)V[(long long)k * ldv + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][u][t], b[u], acc[t], 0, 0, 0);
    }
    if (eok) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (op[t][r]) op[t][r][e] = T(prev[t][r] + acc[t][r]);
    }
  }
}

}  // namespace

hipError_t launch_combine_mfma(Storage st, const void* V, long long ldv, int m, const double* Y, int ncol,
                               void* out, long long ldo, const int* cmap, long long n, hipStream_t s) {
  if (m <= 0 || ncol <= 0 || n <= 0) return hipSuccess;
  if (m > 80) return hipErrorInvalidValue;
  constexpr int TPW = 16;  // 16-entry tiles per wave
  const long long tiles = (n + 15) / 16;
  const long long neb = (tiles + 4 * TPW - 1) / (4 * TPW);  // entry blocks of 4 TPW tiles
  const int ncg = (ncol + 31) / 32;                         // column groups of 32
  const dim3 grid((unsigned)((neb + 7) / 8 * 8 * ncg));
  const int mc = (m + 15) / 16;
#define KRY_CMF(MC)                                                                                        \
  if (st == F64)                                                                                          \
    hipLaunchKernelGGL((k_combine_mfma<double, MC>), grid, dim3(256), 0, s, (const double*)V, ldv, m, Y, ncol, \
                       (double*)out, ldo, cmap, n, TPW, ncg, neb);                                                  \
  else                                                                                                    \
    hipLaunchKernelGGL((k_combine_mfma<float, MC>), grid, dim3(256), 0, s, (const float*)V, ldv, m, Y, ncol,  \
                       (float*)out, ldo, cmap, n, TPW, ncg, neb);
  switch (mc) {
    case 1: KRY_CMF(1) break;
    case 2: KRY_CMF(2) break;
    case 3: KRY_CMF(3) break;
    case 4: KRY_CMF(4) break;
    default: KRY_CMF(5) break;
  }
#undef KRY_CMF
  return hipGetLastError();
}

}  // namespace kry
