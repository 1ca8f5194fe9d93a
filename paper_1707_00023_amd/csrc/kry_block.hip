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

// Load four consecutive entries e..e+3 (e a multiple of 4, base 32-byte
// aligned) as FP64, masking entries at or beyond `end`.
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ p, long long e, long long end,
                                      double (&v)[4]) {
  if (e + 3 < end) {
    if constexpr (sizeof(T) == 8) {
      const double2 a = *reinterpret_cast<const double2*>(p + e);
      const double2 b = *reinterpret_cast<const double2*>(p + e + 2);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
      const float4 a = *reinterpret_cast<const float4*>(p + e);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (e + t < end) ? (double)p[e + t] : 0.0;
  }
}

// partials[split][M x N] = X[:, 0:M]^T diag(w) Y[:, 0:N] over the elements
// [split * kchunk, (split + 1) * kchunk) (kchunk a multiple of 16).  Each
// wave owns 16 rows (columns of X) and NT 16-column tiles of Y; per
// 16-element chunk lane (i, kk) reads entries e0 + 4 kk .. e0 + 4 kk + 3 of
// its X column and of the NT Y columns with 32-byte loads and feeds them to
// four MFMAs, the t-th taking entry e0 + 4 kk + t as its k = kk slot (a
// permutation of the reduction order).  grid (nsplit, ceil(M / 64),
// ceil(N / (16 NT))).  Out-of-range rows, columns and entries add zeros.
// X is given in two segments: columns k < M1 at X + k ld, columns k >= M1
// at X2 + (k - M1) ld (a basis and a block stored apart).
template <typename T, int NT>
__global__ __launch_bounds__(256) void k_gram_tn(const T* __restrict__ X, int M1,
                                                 const T* __restrict__ X2, int M,
                                                 const T* __restrict__ Y, int N, long long ld,
                                                 const double* __restrict__ w, long long n,
                                                 long long kchunk, double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + wave * 16;
  const int nbase = blockIdx.z * 16 * NT;
  const int i = lane & 15, kk = lane >> 4;
  const long long e_begin = (long long)blockIdx.x * kchunk;
  const long long e_end = min(n, e_begin + kchunk);
  const bool arow = m0 + i < M;
  const int xr = arow ? m0 + i : 0;
  const T* xc = xr < M1 ? X + (long long)xr * ld : X2 + (long long)(xr - M1) * ld;
  bool bcol[NT];
  const T* yc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    bcol[t] = nbase + t * 16 + i < N;
    yc[t] = Y + (long long)(bcol[t] ? nbase + t * 16 + i : 0) * ld;
  }
  v4d acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  if (m0 < M) {
    for (long long e0 = e_begin; e0 < e_end; e0 += 16) {
      const long long eb = e0 + 4 * kk;
      double xa[4], ww[4], yb[NT][4];
      if (arow) load4(xc, eb, e_end, xa);
      else xa[0] = xa[1] = xa[2] = xa[3] = 0.0;
      load4(w, eb, e_end, ww);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (bcol[t]) load4(yc[t], eb, e_end, yb[t]);
        else yb[t][0] = yb[t][1] = yb[t][2] = yb[t][3] = 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma16(xa[u], ww[u] * yb[t][u], acc[t]);
    }
  }
  double* out = partials + (long long)blockIdx.x * M * N;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = nbase + t * 16 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + 4 * r + kk;
      if (row < M && col < N) out[(long long)row * N + col] = acc[t][r];
    }
  }
}

// Tall-skinny Gram product for N <= 16 NT (NT = 1, 2): partials[4 bx +
// wave][M x N] = X[:, rows]^T diag(w) Y over the elements the wave visits.
// Workgroup bx owns [bx kchunk, (bx + 1) kchunk); its four waves take
// interleaved 16-element slices of it, and each wave accumulates all MT
// 16-row tiles of its row block (r0 = 16 MT blockIdx.y) against the NT
// 16-column tiles of Y, so every X, Y and w entry is loaded once.  Lane
// (i, kk) reads entries e0 + 4 kk .. e0 + 4 kk + 3 of column i of each tile
// with 32-byte loads; the u-th of four MFMAs per tile pair takes entry
// e0 + 4 kk + u as its k = kk slot.  Out-of-range rows, columns and entries
// add zeros.  X in two segments as in k_gram_tn.  grid (nsplit / 4,
// ceil(M / (16 MT))).
// YSEG: Y is the second segment of X itself (Y = X2, N = M - M1, one row
// block).  Row tiles 0..NT-1 then hold Y and the later tiles the first
// segment, so the Y operand is data already in registers (Y is read once,
// not twice); output rows are mapped back to the [X; X2] order.
// T2: element type of the second segment (and of Y); a second segment of
// another type than the first is supported in the YSEG layout only.
template <typename T, typename T2, int MT, int NT, bool YSEG>
__global__ __launch_bounds__(256) void k_gram_tall(const T* __restrict__ X, int M1,
                                                   const T2* __restrict__ X2, int M,
                                                   const T2* __restrict__ Y, int N, long long ld,
                                                   const double* __restrict__ w, long long n,
                                                   long long kchunk, double* __restrict__ partials,
                                                   const int* __restrict__ skip) {
  static_assert(!YSEG || MT > NT, "YSEG keeps Y in the first NT row tiles");
  if (skip && *skip) return;  // (uniform: the whole grid skips)
  static_assert(YSEG || sizeof(T) == sizeof(T2), "mixed element types need the YSEG layout");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int r0 = blockIdx.y * 16 * MT;
  const long long e_begin = (long long)blockIdx.x * kchunk;
  const long long e_end = min(n, e_begin + kchunk);
  constexpr int YT = YSEG ? NT : 0;  // row tiles holding the second segment
  bool arow[MT];
  const T* xc[MT];
  const T2* x2c[NT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int r = r0 + 16 * t + i;
    xc[t] = X;
    if (YSEG) {  // virtual rows: [0, 16 NT) second segment, then the first
      if (t < YT) {
        arow[t] = r < N;
        x2c[t] = X2 + (long long)(arow[t] ? r : 0) * ld;
      } else {
        arow[t] = r - 16 * YT < M1;
        xc[t] = X + (long long)(arow[t] ? r - 16 * YT : 0) * ld;
      }
    } else {
      arow[t] = r < M;
      const int rr = arow[t] ? r : 0;
      xc[t] = rr < M1 ? X + (long long)rr * ld
                      : reinterpret_cast<const T*>(X2) + (long long)(rr - M1) * ld;
    }
  }
  bool bcol[NT];
  const T2* yc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    bcol[q] = 16 * q + i < N;
    yc[q] = Y + (long long)(bcol[q] ? 16 * q + i : 0) * ld;
  }
  v4d acc[MT][NT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int q = 0; q < NT; ++q) acc[t][q] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (long long e0 = e_begin + 16 * wave; e0 < e_end; e0 += 64) {
    const long long eb = e0 + 4 * kk;
    double xa[MT][4], ww[4], yb[NT][4];
    load4(w, eb, e_end, ww);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (!arow[t]) xa[t][0] = xa[t][1] = xa[t][2] = xa[t][3] = 0.0;
      else if (YSEG && t < YT) load4(x2c[t < YT ? t : 0], eb, e_end, xa[t]);
      else load4(xc[t], eb, e_end, xa[t]);
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (YSEG) {
#pragma unroll
        for (int u = 0; u < 4; ++u) yb[q][u] = xa[q][u];
      } else if (bcol[q]) {
        load4(yc[q], eb, e_end, yb[q]);
      } else {
        yb[q][0] = yb[q][1] = yb[q][2] = yb[q][3] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const double b = ww[u] * yb[q][u];
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t][q] = mfma16(xa[t][u], b, acc[t][q]);
      }
  }
  double* out = partials + ((long long)blockIdx.x * 4 + wave) * M * N;
#pragma unroll
  for (int t = 0; t < MT; ++t) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int col = 16 * q + i;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int vr = r0 + 16 * t + 4 * r + kk;
        int row = vr;
        if (YSEG)
          row = vr < 16 * YT ? (vr < N ? M1 + vr : M) : (vr - 16 * YT < M1 ? vr - 16 * YT : M);
        if (row < M && col < N) out[(long long)row * N + col] = acc[t][q][r];
      }
    }
  }
}

// The Gram product of an s-step block in FP64 (the layout of k_gram_tall
// with YSEG, N <= 16): partials[4 bx + wave][M x N] = [X; X2]^T diag(w) X2
// over the elements the wave visits, with the loads regrouped through LDS.
// In the MFMA operand layout every load instruction touches 16 columns at
// 64 bytes each, and such narrow runs hold a plain read near 3.4-5.7 TB/s
// on gfx950 where runs of 256 bytes or more reach 6.1-6.3 TB/s.  So per
// step of 32 entries a wave loads each 16-column tile with four
// instructions of 4 columns x 256 bytes (lane l: column 4 q + l / 16,
// entries 2 (l % 16) and 2 (l % 16) + 1), writes the tile to its own LDS
// slot [16][kLdsStride] and reads it back in the operand layout (lane
// (i, kk): column i, entries 8 kk .. 8 kk + 7; the k = kk slot of the h-th
// MFMA takes entry 8 kk + h).  The row stride 34 puts the 16-byte accesses
// of eight consecutive lanes on distinct banks, on the write and the read
// side.  A wave's LDS traffic stays in its own slot and in its own program
// order, so no barrier is needed.  Tile 0 holds X2 (also the Y operand),
// tiles 1.. the first segment; inactive columns read column 0 of their
// segment (their rows and columns of the product are never stored).  The
// waves of a workgroup take interleaved steps of its chunk (kchunk a
// multiple of 128); a last partial step loads directly with masks.
// T: element type of the first segment (FP32 storage keeps the block X2 in
// FP64: its loads are then 8 bytes per lane, 4 columns x 128 bytes, and the
// values enter the LDS tile as FP64).  grid (nsplit / 4).
constexpr int kLdsStride = 34;
constexpr int kStepLdsMaxTiles = 6;  // basis of up to 80 columns before the block
template <typename T, int MT>
__global__ __launch_bounds__(256) void k_gram_step_lds(const T* __restrict__ X, int M1,
                                                       const double* __restrict__ X2, int N, long long ld,
                                                       const double* __restrict__ w, long long n,
                                                       long long kchunk, double* __restrict__ partials,
                                                       const int* __restrict__ skip) {
  if (skip && *skip) return;  // (uniform: the whole grid skips)
  __shared__ double tiles[4][16 * kLdsStride];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = lane & 15, kk = lane >> 4;
  double* slot = tiles[wave];
  const long long e_begin = (long long)blockIdx.x * kchunk;
  const long long e_end = min(n, e_begin + kchunk);
  // column read by lane l in load instruction q of tile t: 4 q + l / 16
  const double* lc2[4];
  const T* lc[MT > 1 ? MT - 1 : 1][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = 4 * q + kk;
    lc2[q] = X2 + (long long)(c < N ? c : 0) * ld;
#pragma unroll
    for (int t = 1; t < MT; ++t) {
      const int r = 16 * (t - 1) + c;
      lc[t - 1][q] = X + (long long)(r < M1 ? r : 0) * ld;
    }
  }
  v4d acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  const long long es = e_begin + 32 * wave;
  const long long nfull = e_end - es >= 32 ? (e_end - es - 32) / 128 + 1 : 0;
  for (long long p = 0; p < nfull; ++p) {
    const long long e0 = es + 128 * p;
    double2 g[MT][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) g[0][q] = *reinterpret_cast<const double2*>(lc2[q] + e0 + 2 * i);
#pragma unroll
    for (int t = 1; t < MT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (sizeof(T) == 8) {
          g[t][q] = *reinterpret_cast<const double2*>(lc[t - 1][q] + e0 + 2 * i);
        } else {
          const float2 f = *reinterpret_cast<const float2*>(lc[t - 1][q] + e0 + 2 * i);
          g[t][q] = make_double2((double)f.x, (double)f.y);
        }
      }
    double ww[8], yb[8];
    {
      const double4 a = *reinterpret_cast<const double4*>(w + e0 + 8 * kk);
      const double4 b = *reinterpret_cast<const double4*>(w + e0 + 8 * kk + 4);
      ww[0] = a.x; ww[1] = a.y; ww[2] = a.z; ww[3] = a.w;
      ww[4] = b.x; ww[5] = b.y; ww[6] = b.z; ww[7] = b.w;
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<double2*>(slot + (4 * q + kk) * kLdsStride + 2 * i) = g[t][q];
      double xa[8];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const double2 v = *reinterpret_cast<const double2*>(slot + i * kLdsStride + 8 * kk + 2 * h);
        xa[2 * h] = v.x;
        xa[2 * h + 1] = v.y;
      }
      if (t == 0) {
#pragma unroll
        for (int h = 0; h < 8; ++h) yb[h] = ww[h] * xa[h];
      }
#pragma unroll
      for (int h = 0; h < 8; ++h) acc[t] = mfma16(xa[h], yb[h], acc[t]);
    }
  }
  for (long long e0 = es + 128 * nfull; e0 < e_end; e0 += 128) {  // a partial step
    const long long eb = e0 + 8 * kk;
    double ww[8], yb[8];
    load4(w, eb, e_end, *reinterpret_cast<double(*)[4]>(ww));
    load4(w, eb + 4, e_end, *reinterpret_cast<double(*)[4]>(ww + 4));
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      double xa[8];
      if (t == 0) {
        const double* col = X2 + (long long)(i < N ? i : 0) * ld;
        load4(col, eb, e_end, *reinterpret_cast<double(*)[4]>(xa));
        load4(col, eb + 4, e_end, *reinterpret_cast<double(*)[4]>(xa + 4));
      } else {
        const T* col = X + (long long)(16 * (t - 1) + i < M1 ? 16 * (t - 1) + i : 0) * ld;
        load4(col, eb, e_end, *reinterpret_cast<double(*)[4]>(xa));
        load4(col, eb + 4, e_end, *reinterpret_cast<double(*)[4]>(xa + 4));
      }
      if (t == 0) {
#pragma unroll
        for (int h = 0; h < 8; ++h) yb[h] = ww[h] * xa[h];
      }
#pragma unroll
      for (int h = 0; h < 8; ++h) acc[t] = mfma16(xa[h], yb[h], acc[t]);
    }
  }
  const int M = M1 + N;
  double* out = partials + ((long long)blockIdx.x * 4 + wave) * M * N;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vr = 4 * r + kk;
      const int row = t == 0 ? (vr < N ? M1 + vr : M) : (16 * (t - 1) + vr < M1 ? 16 * (t - 1) + vr : M);
      if (row < M && i < N) out[(long long)row * N + i] = acc[t][r];
    }
}

// Out[:, j] = (accumulate ? Out[:, j] : 0) + alpha sum_k X[:, k] C[k][j] for
// j < N (C row-major M x N, FP64).  Each wave computes 16 entries x 16 NT
// columns (NT tiles of Out^T = C^T X^T): A = C^T (from C), B = X^T (16
// consecutive entries per k: coalesced).  Per iteration a lane loads four
// basis entries (k = k0 + 4u + kk, u = 0..3) before the 4 NT MFMAs, so
// four independent loads are in flight.  grid (ceil(n / 64),
// ceil(N / (16 NT))).  Out may not overlap X.  X in two segments as in
// k_gram_tn (columns k >= M1 at X2 + (k - M1) ld).
template <typename T, int NT>
__global__ __launch_bounds__(256) void k_gemm_nn(const T* __restrict__ X, int M1,
                                                 const T* __restrict__ X2, int M,
                                                 const double* __restrict__ C, int N,
                                                 T* __restrict__ Out, long long ld, long long n,
                                                 double alpha, int accumulate) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e0 = ((long long)blockIdx.x * 4 + wave) * 16;
  const int jbase = blockIdx.y * 16 * NT;
  const int i = lane & 15, kk = lane >> 4;
  const long long e = e0 + i;
  const bool eok = e < n;
  v4d acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < M; k0 += 16) {
    double b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + kk;
      const T* xk = k < M1 ? X + (long long)k * ld : X2 + (long long)(k - M1) * ld;
      b[u] = (k < M && eok) ? (double)xk[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + kk;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int j = jbase + t * 16 + i;
        const double a = (k < M && j < N) ? C[(long long)k * N + j] : 0.0;
        acc[t] = mfma16(a, b[u], acc[t]);
      }
    }
  }
  if (!eok) return;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
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

// Update for N <= 16 output columns on the vector ALUs: Out[:, j] =
// (accumulate ? Out[:, j] : 0) + alpha sum_k X[:, k] C[k][j].  A thread owns
// EPT entries (stride 256, consecutive threads consecutive entries, so
// every column access is coalesced) and all N outputs of each; the
// coefficients sit in LDS and are read as broadcasts.  The dense part is
// 2 N M flops per entry, far below the FP64 vector rate at the bandwidth
// this kernel moves, so the matrix cores gain nothing here.  X in two
// segments as in k_gram_tn.  A thread reads its entries of every input row
// before it writes any output, and no other thread touches those entries,
// so Out may be rows of X or X2 themselves (an in-place update; no
// __restrict__ on them for that reason).
// T2: element type of the second segment; TO: of Out.  NO (16 or 32): the
// largest N, the width of the coefficient rows in LDS and of a thread's
// accumulators.
template <typename T, typename T2, typename TO, int EPT, int NO>
__global__ __launch_bounds__(256) void k_gemm_cols(const T* X, int M1, const T2* X2, int M,
                                                   const double* __restrict__ C, int N,
                                                   TO* Out, long long ld, long long n,
                                                   double alpha, int accumulate,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;  // (uniform: the whole grid skips)
  extern __shared__ double sC[];  // M x NO
  for (int t = threadIdx.x; t < M * NO; t += 256) {
    const int k = t / NO, j = t % NO;
    sC[t] = j < N ? C[(long long)k * N + j] : 0.0;
  }
  __syncthreads();
  const long long base = (long long)blockIdx.x * 256 * EPT + threadIdx.x;
  double acc[EPT][NO];
  bool ok[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    ok[q] = base + 256LL * q < n;
#pragma unroll
    for (int j = 0; j < NO; ++j) acc[q][j] = 0.0;
  }
  // one row k of a segment: acc += x_k C[k][:].  Every load and store of
  // the sweep is marked non-temporal (nothing is reused from the caches):
  // measured at 128^3, 5.3-5.8 TB/s against 5.1-5.2 with ordinary accesses
  // (either hint alone gains nothing)
  auto row_update = [&](const auto* xk, int k) {
    double x[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) x[q] = ok[q] ? (double)__builtin_nontemporal_load(xk + base + 256LL * q) : 0.0;
    const double2* row = reinterpret_cast<const double2*>(sC + NO * k);
#pragma unroll
    for (int j2 = 0; j2 < NO / 2; ++j2) {
      const double2 cc = row[j2];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        acc[q][2 * j2] += x[q] * cc.x;
        acc[q][2 * j2 + 1] += x[q] * cc.y;
      }
    }
  };
  // the two segments in loops of their own (no branch in the loop body)
#pragma unroll 2
  for (int k = 0; k < M1; ++k) row_update(X + (long long)k * ld, k);
#pragma unroll 2
  for (int k = M1; k < M; ++k) row_update(X2 + (long long)(k - M1) * ld, k);
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    if (!ok[q]) continue;
    const long long e = base + 256LL * q;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      if (j < N) {
        TO* o = Out + (long long)j * ld + e;
        const double prev = accumulate ? (double)__builtin_nontemporal_load(o) : 0.0;
        __builtin_nontemporal_store(TO(prev + alpha * acc[q][j]), o);
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

// Rows of X per workgroup of k_gram_tall (16 MT) for M rows.
static int tall_mt(int M) {
  const int tiles = (M + 15) / 16;
  return tiles <= 8 ? tiles : 8;
}

int gram_splits(long long n, int M, int N) {
  const long long maxs = (n + 255) / 256;
  if (N <= 32) {
    // k_gram_tall: four partials per workgroup, about 1024 workgroups
    const int mt = tall_mt(M);
    const int rowblk = (M + 16 * mt - 1) / (16 * mt);
    long long wg = 1024 / rowblk;
    if (wg > maxs) wg = maxs;
    if (wg < 1) wg = 1;
    return (int)(4 * wg);
  }
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  long long s = 2048 / tiles;
  if (s < 1) s = 1;
  if (s > maxs) s = maxs;
  return (int)s;
}

hipError_t launch_gram(Storage st, const void* X, int M, const void* Y, int N, long long ld,
                       const double* w, long long n, double* partials, int nsplit, hipStream_t s,
                       const void* X2, int M1, int st2_, const int* skip) {
  const Storage st2 = st2_ < 0 ? st : (Storage)st2_;
  if (!X2) {  // one segment
    M1 = M;
    X2 = X;
    if (st2 != st) return hipErrorInvalidValue;
  }
  if (N <= 32) {
    const int wg = nsplit / 4;
    long long kchunk = (n + wg - 1) / wg;
    kchunk = (kchunk + 63) / 64 * 64;
    const int nt = (N + 15) / 16;
    // Y is the second segment of X: one row block with Y in the first nt
    // row tiles
    const bool yseg = Y == X2 && N == M - M1 && M1 + 16 * nt <= 128;
    if (st2 != st && !(yseg && st == F32 && st2 == F64)) return hipErrorInvalidValue;
    const int mt = yseg ? nt + (M1 + 15) / 16 : tall_mt(M);
    if (yseg && mt > 8) return hipErrorInvalidValue;
    if (yseg && nt == 1 && st2 == F64 && mt <= kStepLdsMaxTiles) {
      // the s-step block (FP64; the basis FP64 or FP32): loads regrouped
      // through LDS
      long long kc = (n + wg - 1) / wg;
      kc = (kc + 127) / 128 * 128;
#define KRY_STEP_LDS(MT)                                                                                  \
  if (st == F64)                                                                                          \
    hipLaunchKernelGGL((k_gram_step_lds<double, MT>), dim3(wg), dim3(256), 0, s, (const double*)X, M1,   \
                       (const double*)X2, N, ld, w, n, kc, partials, skip);                              \
  else                                                                                                    \
    hipLaunchKernelGGL((k_gram_step_lds<float, MT>), dim3(wg), dim3(256), 0, s, (const float*)X, M1,     \
                       (const double*)X2, N, ld, w, n, kc, partials, skip);
      switch (mt) {
        case 1: KRY_STEP_LDS(1) break;
        case 2: KRY_STEP_LDS(2) break;
        case 3: KRY_STEP_LDS(3) break;
        case 4: KRY_STEP_LDS(4) break;
        case 5: KRY_STEP_LDS(5) break;
        default: KRY_STEP_LDS(6) break;
      }
#undef KRY_STEP_LDS
      return hipGetLastError();
    }
    const dim3 grid(wg, yseg ? 1 : (M + 16 * mt - 1) / (16 * mt));
#define KRY_TALL_(T, T2, MT, NT, YS)                                                              \
  hipLaunchKernelGGL((k_gram_tall<T, T2, MT, NT, YS>), grid, dim3(256), 0, s, (const T*)X, M1,     \
                     (const T2*)X2, M, (const T2*)Y, N, ld, w, n, kchunk, partials, skip);
#define KRY_TALL_NT(MT, NT)                             \
  if (yseg) {                                           \
    if constexpr (MT > NT) {                            \
      if (st == F64) {                                  \
        KRY_TALL_(double, double, MT, NT, true)         \
      } else if (st2 == F64) {                          \
        KRY_TALL_(float, double, MT, NT, true)          \
      } else {                                          \
        KRY_TALL_(float, float, MT, NT, true)           \
      }                                                 \
    }                                                   \
  } else if (st == F64) {                               \
    KRY_TALL_(double, double, MT, NT, false)            \
  } else {                                              \
    KRY_TALL_(float, float, MT, NT, false)              \
  }
#define KRY_TALL(MT)                \
  if (nt == 1) {                    \
    KRY_TALL_NT(MT, 1)              \
  } else {                          \
    KRY_TALL_NT(MT, 2)              \
  }
    switch (mt) {
      case 1: KRY_TALL(1) break;
      case 2: KRY_TALL(2) break;
      case 3: KRY_TALL(3) break;
      case 4: KRY_TALL(4) break;
      case 5: KRY_TALL(5) break;
      case 6: KRY_TALL(6) break;
      case 7: KRY_TALL(7) break;
      default: KRY_TALL(8) break;
    }
#undef KRY_TALL
#undef KRY_TALL_NT
#undef KRY_TALL_
    return hipGetLastError();
  }
  if (st2 != st || skip) return hipErrorInvalidValue;  // (no skip flag in the wide form)
  long long kchunk = (n + nsplit - 1) / nsplit;
  kchunk = (kchunk + 15) / 16 * 16;
  const int nt = N >= 64 ? 4 : (N + 15) / 16;
  const dim3 grid(nsplit, (M + 63) / 64, (N + 16 * nt - 1) / (16 * nt));
#define KRY_GRAM(NT)                                                                        \
  if (st == F64)                                                                           \
    hipLaunchKernelGGL((k_gram_tn<double, NT>), grid, dim3(256), 0, s, (const double*)X, M1, \
                       (const double*)X2, M, (const double*)Y, N, ld, w, n, kchunk, partials); \
  else                                                                                     \
    hipLaunchKernelGGL((k_gram_tn<float, NT>), grid, dim3(256), 0, s, (const float*)X, M1,   \
                       (const float*)X2, M, (const float*)Y, N, ld, w, n, kchunk, partials);
  switch (nt) {
    case 1: KRY_GRAM(1) break;
    case 2: KRY_GRAM(2) break;
    case 3: KRY_GRAM(3) break;
    default: KRY_GRAM(4) break;
  }
#undef KRY_GRAM
  return hipGetLastError();
}

hipError_t launch_gemm_nn(Storage st, const void* X, int M, const double* C, int N, void* Out,
                          long long ld, long long n, double alpha, int accumulate, hipStream_t s,
                          const void* X2, int M1, int st2_, int sto_, const int* skip) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const Storage st2 = st2_ < 0 ? st : (Storage)st2_;
  const Storage sto = sto_ < 0 ? st : (Storage)sto_;
  if (!X2) {
    M1 = M;
    X2 = X;
    if (st2 != st) return hipErrorInvalidValue;
  }
  const bool mixed = st2 != st || sto != st;
  if ((N <= 16 && M <= 256) || (N <= 32 && M <= 128)) {
    // N <= 16: two entries per thread, 16 accumulators each; N <= 32: one
    // entry per thread, 32 accumulators
    const bool wide = N > 16;
    const int ept = wide ? 1 : 2;
    const dim3 grid((unsigned)((n + 256 * ept - 1) / (256 * ept)));
    const size_t lds = sizeof(double) * (wide ? 32 : 16) * (size_t)M;
#define KRY_GCOLS_(T, T2, TO, EPT, NO)                                                             \
  hipLaunchKernelGGL((k_gemm_cols<T, T2, TO, EPT, NO>), grid, dim3(256), lds, s, (const T*)X, M1,   \
                     (const T2*)X2, M, C, N, (TO*)Out, ld, n, alpha, accumulate, skip);
#define KRY_GCOLS(T, T2, TO)         \
  if (wide) {                        \
    KRY_GCOLS_(T, T2, TO, 1, 32)     \
  } else {                           \
    KRY_GCOLS_(T, T2, TO, 2, 16)     \
  }
    if (st == F64 && st2 == F64 && sto == F64) {
      KRY_GCOLS(double, double, double)
    } else if (st == F32 && st2 == F32 && sto == F32) {
      KRY_GCOLS(float, float, float)
    } else if (st == F32 && st2 == F64 && sto == F64) {
      KRY_GCOLS(float, double, double)
    } else if (st == F32 && st2 == F64 && sto == F32) {
      KRY_GCOLS(float, double, float)
    } else if (st == F32 && st2 == F32 && sto == F64) {
      KRY_GCOLS(float, float, double)
    } else {
      return hipErrorInvalidValue;
    }
#undef KRY_GCOLS
#undef KRY_GCOLS_
    return hipGetLastError();
  }
  if (mixed || skip) return hipErrorInvalidValue;  // (no skip flag in the wide form)
  const int nt = N >= 64 ? 4 : (N + 15) / 16;
  const dim3 grid((unsigned)((n + 63) / 64), (N + 16 * nt - 1) / (16 * nt));
#define KRY_GEMM(NT)                                                                          \
  if (st == F64)                                                                             \
    hipLaunchKernelGGL((k_gemm_nn<double, NT>), grid, dim3(256), 0, s, (const double*)X, M1,  \
                       (const double*)X2, M, C, N, (double*)Out, ld, n, alpha, accumulate);   \
  else                                                                                       \
    hipLaunchKernelGGL((k_gemm_nn<float, NT>), grid, dim3(256), 0, s, (const float*)X, M1,    \
                       (const float*)X2, M, C, N, (float*)Out, ld, n, alpha, accumulate);
  switch (nt) {
    case 1: KRY_GEMM(1) break;
    case 2: KRY_GEMM(2) break;
    case 3: KRY_GEMM(3) break;
    default: KRY_GEMM(4) break;
  }
#undef KRY_GEMM
  return hipGetLastError();
}

hipError_t launch_weights(const double* eps, const double* mu, double* w, long long N3,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_weights, dim3((unsigned)((N3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     eps, mu, w, N3);
  return hipGetLastError();
}

}  // namespace kry
