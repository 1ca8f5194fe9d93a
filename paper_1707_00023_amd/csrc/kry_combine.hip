// Basis combination for many outputs on FP64 matrix cores: out_{cmap[j]} +=
// sum_{k < m} V_k Y[k + j m] for j < ncol (Y column-major m x ncol, m <= 80).
// This is a tall-skinny product V Y: a wave computes 32-entry x 32-column
// tiles with v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] =
// Y[k][j] and B[l / 16][l % 16] = V_k[e]; the result holds output column
// 4 r + l / 16 of a 16-column tile, entry l % 16, in its r-th register), so
// the basis is read once per 32 outputs where the vector-ALU combination
// reads it once per 8.  For the restarted method's batched form, where one
// basis serves hundreds of time functions.  The outputs' read-modify-write
// is most of the traffic (2 ncol vectors against m), so the kernel is built
// around it: the old output values of a tile are loaded before its MFMAs,
// their latency hidden behind the dense work, and the read-modify-write
// goes through LDS, so that each load and store instruction covers 4
// columns x 32 entries (256 bytes in FP64) instead of the 16 entries of
// the MFMA result layout, with non-temporal loads and stores.  Measured at
// 96^3, m = 64, 256 outputs, in isolation: 5.5 ms per launch with the
// coefficients in LDS, 5.9 ms with them in registers, 6.0 ms with ordinary
// accesses, 6.5 ms with the read-modify-write in the result layout and
// 10.6 ms for 64 columns per wave without the early loads.
#include "kry_internal.h"

namespace kry {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
// vector types for the non-temporal load and store builtins
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));

constexpr int kOutStride = 34;  // LDS row stride (doubles) of a column's 32 entries

// One wave owns 32 output columns (two 16-column tiles); their coefficients,
// the MFMA A operands for every k, sit in LDS for the workgroup (read per
// MFMA: in registers they took 64 VGPRs and left two waves per SIMD, in LDS
// three, 9% faster); the wave streams tpw blocks of 32 entries of the basis
// through them, the
// four waves of a workgroup on 128 consecutive entries at a time.  Per block
// the old outputs are read first in the read-modify-write layout (load
// instruction q: lane l takes column 4 q + l / 16, entries 2 (l % 16) and
// 2 (l % 16) + 1), the MFMA results go through the wave's LDS slot
// [32 columns][32 entries] into the same layout, and the sums are stored.
// A wave's LDS traffic stays in its own slot and in its own program order.
// Workgroup b covers entry block eb and column group cg with b = ((eb / 8)
// ncg + cg) 8 + eb mod 8: the column groups of an entry block run on one
// XCD at nearby dispatch times, so its basis entries come from HBM once.
// MC: 16-row chunks of k (m <= 16 MC).
template <typename T, int MC>
__global__ __launch_bounds__(256, 3) void k_combine_mfma(const T* __restrict__ V, long long ldv, int m,
                                                      const double* __restrict__ Y, int ncol, T* __restrict__ out,
                                                      long long ldo, const int* __restrict__ cmap, long long n,
                                                      int tpw, int ncg, long long neb) {
  __shared__ double slots[4][32 * kOutStride];
  __shared__ double ya[16 * MC][32];  // ya[k][jj] = Y[k][jbase + jj]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long bt = blockIdx.x >> 3;
  const int cg = (int)(bt % ncg);
  const long long eb = (bt / ncg) * 8 + (blockIdx.x & 7);
  if (eb >= neb) return;
  const int jbase = cg * 32;
  const int i = lane & 15, kk = lane >> 4;
  double* slot = slots[wave];
  for (int t = threadIdx.x; t < 16 * MC * 32; t += 256) {
    const int k = t / 32, j = jbase + t % 32;
    ya[k][t % 32] = (k < m && j < ncol) ? Y[k + (long long)j * m] : 0.0;
  }
  __syncthreads();
  T* op[8];  // output column of lane l in read-modify-write instruction q
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int j = jbase + 4 * q + kk;
    op[q] = j < ncol ? out + (long long)(cmap ? cmap[j] : j) * ldo : nullptr;
  }
  const long long base = eb * 128LL * tpw;
  for (int tt = 0; tt < tpw; ++tt) {
    const long long e0 = base + (4LL * tt + wave) * 32;
    if (e0 >= n) break;
    const bool full = e0 + 32 <= n;
    double pv[8][2];  // the old outputs, loaded first
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      pv[q][0] = pv[q][1] = 0.0;
      if (op[q] && full) {  // (non-temporal: the outputs are not reused from the caches)
        if constexpr (sizeof(T) == 8) {
          const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(op[q] + e0 + 2 * i));
          pv[q][0] = v.x;
          pv[q][1] = v.y;
        } else {
          const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(op[q] + e0 + 2 * i));
          pv[q][0] = v.x;
          pv[q][1] = v.y;
        }
      }
    }
    v4d acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[x][t] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      double b[2][4];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const long long e = e0 + 16 * x + i;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = 16 * c + 4 * u + kk;
          b[x][u] = (k < m && e < n) ? (double)V[(long long)k * ldv + e] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 16 * c + 4 * u + kk;
        const double a0 = ya[k][i], a1 = ya[k][16 + i];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          acc[x][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b[x][u], acc[x][0], 0, 0, 0);
          acc[x][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b[x][u], acc[x][1], 0, 0, 0);
        }
      }
    }
    // acc[x][t][r]: column 16 t + 4 r + kk, entry 16 x + i
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) slot[(16 * t + 4 * r + kk) * kOutStride + 16 * x + i] = acc[x][t][r];
    if (full) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (!op[q]) continue;
        const double2 d = *reinterpret_cast<const double2*>(slot + (4 * q + kk) * kOutStride + 2 * i);
        if constexpr (sizeof(T) == 8) {
          nt_d2 r;
          r.x = pv[q][0] + d.x;
          r.y = pv[q][1] + d.y;
          __builtin_nontemporal_store(r, reinterpret_cast<nt_d2*>(op[q] + e0 + 2 * i));
        } else {
          nt_f2 r;
          r.x = T(pv[q][0] + d.x);
          r.y = T(pv[q][1] + d.y);
          __builtin_nontemporal_store(r, reinterpret_cast<nt_f2*>(op[q] + e0 + 2 * i));
        }
      }
    } else {  // the last, partial block of entries
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (!op[q]) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const long long e = e0 + 2 * i + h;
          if (e < n) op[q][e] = T((double)op[q][e] + slot[(4 * q + kk) * kOutStride + 2 * i + h]);
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_combine_mfma(Storage st, const void* V, long long ldv, int m, const double* Y, int ncol,
                               void* out, long long ldo, const int* cmap, long long n, hipStream_t s) {
  if (m <= 0 || ncol <= 0 || n <= 0) return hipSuccess;
  if (m > 80) return hipErrorInvalidValue;
  constexpr int TPW = 8;  // 32-entry blocks per wave
  const long long blocks = (n + 127) / 128;                  // 128 entries: one step of a workgroup
  const long long neb = (blocks + TPW - 1) / TPW;            // entry blocks of TPW steps
  const int ncg = (ncol + 31) / 32;                          // column groups of 32
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
