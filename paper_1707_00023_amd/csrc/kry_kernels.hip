// HIP kernels for gfx950 (CDNA4): Yee operator, Arnoldi Gram-Schmidt in the
// energy inner product, basis combinations and conversions.
//
// Every streaming kernel is cell-parallel: a thread owns whole cells and
// touches the six planes [Hx, Hy, Hz, Ex, Ey, Ez] of each, so plane offsets
// are p * N3 and no 64-bit division is needed; consecutive threads own
// consecutive cells, so every plane access is coalesced.  Reductions are
// two-stage (per-workgroup partial sums, then a fixed-order sum), so the
// results are bitwise reproducible run to run.
#include "kry_internal.h"

namespace kry {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum CH per-thread values over the workgroup; thread q < valid stores the
// q-th total to dst[q].
template <int CH>
__device__ __forceinline__ void block_sum_store(const double (&acc)[CH], int valid, double* dst) {
  __shared__ double sh[CH][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) sh[q][wid] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < valid) {
    const int q = threadIdx.x;
    dst[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
  }
  __syncthreads();
}

// As block_sum_store for 2*CH values: totals q < valid go to dstA[q],
// totals CH + q (q < valid) to dstB[q].
template <int CH>
__device__ __forceinline__ void block_sum_store_split(const double (&acc)[2 * CH], int valid,
                                                      double* dstA, double* dstB) {
  __shared__ double sh[2 * CH][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 2 * CH; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) sh[q][wid] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * CH && (t % CH) < valid) {
    const double v = (sh[t][0] + sh[t][1]) + (sh[t][2] + sh[t][3]);
    if (t < CH) dstA[t] = v;
    else dstB[t - CH] = v;
  }
  __syncthreads();
}

// Logical block index with consecutive logical blocks kept on one XCD: the
// dispatcher places block b on XCD (b mod 8), so remap b -> (b mod 8) *
// (nblk / 8) + b / 8 over the largest multiple of 8, keeping neighbouring
// z-slabs of the stencil in the same L2.
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int full = nblk & ~7;
  if (b >= full) return b;
  const int per = full >> 3;
  return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Yee operator at one cell:
//   (A y)_H = sigma/mu H + (C E)/mu,   (A y)_E = (sigma E - C^T H)/eps
//   (C E)x = dEz/dy - dEy/dz with forward differences (zero beyond the last
//   cell), (C^T H)x = dHz/dy - dHy/dz with backward differences (zero before
//   the first cell), and cyclically.
// o receives the six outputs, ctr the six input values at the cell itself.
// Arithmetic is in the storage type T (FP32 storage computes the stencil in
// FP32).
template <typename T, bool HAS_MU>
__device__ __forceinline__ void yee_cell(const T* __restrict__ v, long long c, const DevGrid& g,
                                         const DevMats& mt, T (&o)[6], T (&ctr)[6]) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N3 = g.N3;
  const long long sy = nx, sz = (long long)nx * ny;
  const T* Hx = v;
  const T* Hy = v + N3;
  const T* Hz = v + 2 * N3;
  const T* Ex = v + 3 * N3;
  const T* Ey = v + 4 * N3;
  const T* Ez = v + 5 * N3;
  const int ci = (int)c;
  const int i = ci % nx;
  const int t = ci / nx;
  const int j = t % ny;
  const int k = t / ny;
  const T z0 = T(0);
  const T ex = Ex[c], ey = Ey[c], ez = Ez[c];
  const T ex_j = (j + 1 < ny) ? Ex[c + sy] : z0;
  const T ex_k = (k + 1 < nz) ? Ex[c + sz] : z0;
  const T ey_i = (i + 1 < nx) ? Ey[c + 1] : z0;
  const T ey_k = (k + 1 < nz) ? Ey[c + sz] : z0;
  const T ez_i = (i + 1 < nx) ? Ez[c + 1] : z0;
  const T ez_j = (j + 1 < ny) ? Ez[c + sy] : z0;
  const T cex = (ez_j - ez) - (ey_k - ey);
  const T cey = (ex_k - ex) - (ez_i - ez);
  const T cez = (ey_i - ey) - (ex_j - ex);
  const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
  const T hx_j = (j > 0) ? Hx[c - sy] : z0;
  const T hx_k = (k > 0) ? Hx[c - sz] : z0;
  const T hy_i = (i > 0) ? Hy[c - 1] : z0;
  const T hy_k = (k > 0) ? Hy[c - sz] : z0;
  const T hz_i = (i > 0) ? Hz[c - 1] : z0;
  const T hz_j = (j > 0) ? Hz[c - sy] : z0;
  const T chx = (hz - hz_j) - (hy - hy_k);
  const T chy = (hx - hx_k) - (hz - hz_i);
  const T chz = (hy - hy_i) - (hx - hx_j);
  const T ie = T(mt.inv_eps[c]);
  const T sg = T(mt.sigma[c]);
  if (HAS_MU) {
    const T im = T(mt.inv_mu[c]);
    const T se = T(mt.sigma[c] * mt.mu[c]);
    o[0] = sg * hx + im * cex;
    o[1] = sg * hy + im * cey;
    o[2] = sg * hz + im * cez;
    o[3] = ie * (se * ex - chx);
    o[4] = ie * (se * ey - chy);
    o[5] = ie * (se * ez - chz);
  } else {
    o[0] = sg * hx + cex;
    o[1] = sg * hy + cey;
    o[2] = sg * hz + cez;
    o[3] = ie * (sg * ex - chx);
    o[4] = ie * (sg * ey - chy);
    o[5] = ie * (sg * ez - chz);
  }
  ctr[0] = hx; ctr[1] = hy; ctr[2] = hz;
  ctr[3] = ex; ctr[4] = ey; ctr[5] = ez;
}

// w = A v, optionally fused with the first classical Gram-Schmidt dot pass:
// partial sums of <w, V_i>_M for i < cnt and |w|_M^2 (slot cnt).
template <typename T, bool HAS_MU, int CPT, bool DOTS>
__global__ __launch_bounds__(kBlock) void k_stencil(const T* __restrict__ v, T* __restrict__ w,
                                                    const T* __restrict__ V, long long ldv, int cnt,
                                                    DevGrid g, DevMats mt,
                                                    double* __restrict__ partials) {
  const long long N3 = g.N3;
  if (!DOTS) {  // grid.y indexes columns at stride ldv
    v += (long long)blockIdx.y * ldv;
    w += (long long)blockIdx.y * ldv;
  }
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  double wm[CPT][6];  // weight * output, for the dots
  long long cellq[CPT];
  bool okq[CPT];
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const long long c = ((long long)lb * CPT + q) * kBlock + threadIdx.x;
    okq[q] = c < N3;
    cellq[q] = okq[q] ? c : 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) wm[q][p] = 0.0;
    if (!okq[q]) continue;
    T o[6], ctr[6];
    yee_cell<T, HAS_MU>(v, c, g, mt, o, ctr);
#pragma unroll
    for (int p = 0; p < 6; ++p) w[p * N3 + c] = o[p];
    if (DOTS) {
      const double we = mt.eps[c];
      const double wh = HAS_MU ? mt.mu[c] : 1.0;
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const double ov = (double)o[p];
        wm[q][p] = (p < 3 ? wh : we) * ov;
        nrm += wm[q][p] * ov;
      }
    }
  }
  if (!DOTS) return;
  for (int i0 = 0; i0 < cnt; i0 += kChunk) {
    double acc[kChunk];
#pragma unroll
    for (int r = 0; r < kChunk; ++r) acc[r] = 0.0;
#pragma unroll
    for (int r = 0; r < kChunk; ++r) {
      if (i0 + r < cnt) {
        const T* vi = V + (long long)(i0 + r) * ldv;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          if (!okq[q]) continue;
#pragma unroll
          for (int p = 0; p < 6; ++p) acc[r] += wm[q][p] * (double)vi[p * N3 + cellq[q]];
        }
      }
    }
    const int valid = min(kChunk, cnt - i0);
    block_sum_store<kChunk>(acc, valid, partials + (long long)lb * (cnt + 1) + i0);
  }
  const double a1[1] = {nrm};
  block_sum_store<1>(a1, 1, partials + (long long)lb * (cnt + 1) + cnt);
}

// One step of a three-term polynomial basis: out = alpha A v + gamma v +
// beta prev (prev may be null: beta is then ignored).  The operator is
// evaluated in the storage type, the combination in FP64.
template <typename T, bool HAS_MU, int CPT>
__global__ __launch_bounds__(kBlock) void k_stencil_axpby(const T* __restrict__ v,
                                                          const T* __restrict__ prev,
                                                          T* __restrict__ out, double alpha,
                                                          double gamma, double beta, DevGrid g,
                                                          DevMats mt) {
  const long long N3 = g.N3;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const long long c = ((long long)lb * CPT + q) * kBlock + threadIdx.x;
    if (c >= N3) continue;
    T o[6], ctr[6];
    yee_cell<T, HAS_MU>(v, c, g, mt, o, ctr);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      double r = alpha * (double)o[p] + gamma * (double)ctr[p];
      if (prev) r += beta * (double)__builtin_nontemporal_load(prev + p * N3 + c);
      __builtin_nontemporal_store(T(r), out + p * N3 + c);
    }
  }
}

// The same step by z-marching columns of cells: a workgroup owns a 64 x 4
// tile of (i, j) (one wave per row of 64 consecutive i: coalesced loads)
// and KZ consecutive planes; each thread walks its (i, j) column up the
// planes and keeps the z-neighbours in registers (H at k - 1 is the last
// plane's own H, E at k + 1 becomes the next plane's own E), so v is read
// once per plane plus one halo plane (Hx, Hy below, Ex, Ey above) per
// chunk.  The x and y neighbours are read from the same or the adjacent
// rows of the tile (cache hits).  No barriers: threads outside the grid
// return at once.
template <typename T, bool HAS_MU, int KZ>
__global__ __launch_bounds__(kBlock) void k_stencil_axpby_zm(const T* __restrict__ v,
                                                             const T* __restrict__ prev,
                                                             T* __restrict__ out, double alpha,
                                                             double gamma, double beta, DevGrid g,
                                                             DevMats mt, int tiles_x, int tiles_y) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int tx = lb % tiles_x;
  const int rest = lb / tiles_x;
  const int ty = rest % tiles_y;
  const int kc = rest / tiles_y;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int i = tx * 64 + (threadIdx.x & 63);
  const int j = ty * 4 + (threadIdx.x >> 6);
  if (i >= nx || j >= ny) return;
  const int k0 = kc * KZ;
  const int k1 = min(nz, k0 + KZ);
  const long long N3 = g.N3;
  const long long sy = nx, sz = (long long)nx * ny;
  const T* Hx = v;
  const T* Hy = v + N3;
  const T* Hz = v + 2 * N3;
  const T* Ex = v + 3 * N3;
  const T* Ey = v + 4 * N3;
  const T* Ez = v + 5 * N3;
  const T z0 = T(0);
  long long c = (long long)k0 * sz + (long long)j * nx + i;
  T hxm = k0 > 0 ? Hx[c - sz] : z0;  // H at k - 1
  T hym = k0 > 0 ? Hy[c - sz] : z0;
  T ex = Ex[c], ey = Ey[c];           // E at k
  for (int k = k0; k < k1; ++k, c += sz) {
    const T ez = Ez[c];
    const T exk = (k + 1 < nz) ? Ex[c + sz] : z0;
    const T eyk = (k + 1 < nz) ? Ey[c + sz] : z0;
    const T ex_j = (j + 1 < ny) ? Ex[c + sy] : z0;
    const T ey_i = (i + 1 < nx) ? Ey[c + 1] : z0;
    const T ez_i = (i + 1 < nx) ? Ez[c + 1] : z0;
    const T ez_j = (j + 1 < ny) ? Ez[c + sy] : z0;
    const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
    const T hx_j = (j > 0) ? Hx[c - sy] : z0;
    const T hy_i = (i > 0) ? Hy[c - 1] : z0;
    const T hz_i = (i > 0) ? Hz[c - 1] : z0;
    const T hz_j = (j > 0) ? Hz[c - sy] : z0;
    const T cex = (ez_j - ez) - (eyk - ey);
    const T cey = (exk - ex) - (ez_i - ez);
    const T cez = (ey_i - ey) - (ex_j - ex);
    const T chx = (hz - hz_j) - (hy - hym);
    const T chy = (hx - hxm) - (hz - hz_i);
    const T chz = (hy - hy_i) - (hx - hx_j);
    const T ie = T(mt.inv_eps[c]);
    const T sg = T(mt.sigma[c]);
    T o[6];
    if (HAS_MU) {
      const T im = T(mt.inv_mu[c]);
      const T se = T(mt.sigma[c] * mt.mu[c]);
      o[0] = sg * hx + im * cex;
      o[1] = sg * hy + im * cey;
      o[2] = sg * hz + im * cez;
      o[3] = ie * (se * ex - chx);
      o[4] = ie * (se * ey - chy);
      o[5] = ie * (se * ez - chz);
    } else {
      o[0] = sg * hx + cex;
      o[1] = sg * hy + cey;
      o[2] = sg * hz + cez;
      o[3] = ie * (sg * ex - chx);
      o[4] = ie * (sg * ey - chy);
      o[5] = ie * (sg * ez - chz);
    }
    const T ctr[6] = {hx, hy, hz, ex, ey, ez};
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      double r = alpha * (double)o[p] + gamma * (double)ctr[p];
      if (prev) r += beta * (double)__builtin_nontemporal_load(prev + p * N3 + c);
      __builtin_nontemporal_store(T(r), out + p * N3 + c);
    }
    hxm = hx;
    hym = hy;
    ex = exk;
    ey = eyk;
  }
}

// Pass A of a delayed-reorthogonalisation Arnoldi step.  For the candidate
// u (orthogonalised once against V_0..cnt-1, neither reorthogonalised nor
// normalised): x = A u, and in the same sweep the partial sums of
// a_i = <x, V_i>_M, b_i = <u, V_i>_M (i < cnt), alpha = |u|_M^2 and
// beta = <u, x>_M, stored at partials[blk * (2 cnt + 2) + {i, cnt + i,
// 2 cnt, 2 cnt + 1}].
template <typename T, bool HAS_MU, int CPT, int CH>
__global__ __launch_bounds__(kBlock) void k_stencil_lag(const T* __restrict__ u, T* __restrict__ x,
                                                        const T* __restrict__ V, long long ldv,
                                                        int cnt, DevGrid g, DevMats mt,
                                                        double* __restrict__ partials) {
  const long long N3 = g.N3;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const long long stride = 2 * cnt + 2;
  double xm[CPT][6];  // weight * x
  double um[CPT][6];  // weight * u
  long long cellq[CPT];
  bool okq[CPT];
  double alpha = 0.0, beta = 0.0;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const long long c = ((long long)lb * CPT + q) * kBlock + threadIdx.x;
    okq[q] = c < N3;
    cellq[q] = okq[q] ? c : 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) xm[q][p] = um[q][p] = 0.0;
    if (!okq[q]) continue;
    T o[6], ctr[6];
    yee_cell<T, HAS_MU>(u, c, g, mt, o, ctr);
#pragma unroll
    for (int p = 0; p < 6; ++p) x[p * N3 + c] = o[p];
    const double we = mt.eps[c];
    const double wh = HAS_MU ? mt.mu[c] : 1.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double w8 = p < 3 ? wh : we;
      const double ov = (double)o[p], uu = (double)ctr[p];
      xm[q][p] = w8 * ov;
      um[q][p] = w8 * uu;
      alpha += um[q][p] * uu;
      beta += um[q][p] * ov;
    }
  }
  double* dst = partials + (long long)lb * stride;
  for (int i0 = 0; i0 < cnt; i0 += CH) {
    double acc[2 * CH];
#pragma unroll
    for (int r = 0; r < 2 * CH; ++r) acc[r] = 0.0;
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      if (i0 + r < cnt) {
        const T* vi = V + (long long)(i0 + r) * ldv;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          if (!okq[q]) continue;
#pragma unroll
          for (int p = 0; p < 6; ++p) {
            const double vv = (double)vi[p * N3 + cellq[q]];
            acc[r] += xm[q][p] * vv;
            acc[CH + r] += um[q][p] * vv;
          }
        }
      }
    }
    block_sum_store_split<CH>(acc, min(CH, cnt - i0), dst + i0, dst + cnt + i0);
  }
  const double a2[2] = {alpha, beta};
  block_sum_store<2>(a2, 2, dst + 2 * cnt);
}

// Pass B of a delayed-reorthogonalisation Arnoldi step, one sweep over
// V_0..cnt-1: v_new = u * co[2cnt] - sum_i co[i] V_i (the reorthogonalised,
// normalised u) and u_next = x * co[2cnt] - co[2cnt+1] u - sum_i co[cnt+i]
// V_i (the next candidate).  u_next may alias u (read before written).
template <typename T, int CPT>
__global__ __launch_bounds__(kBlock) void k_lag_update(const T* u, const T* __restrict__ x,
                                                       const T* __restrict__ V, long long ldv,
                                                       int cnt, const double* __restrict__ co,
                                                       T* vnew, T* unext,
                                                       long long N3) {
  __shared__ double sb[kMaxCoef];
  __shared__ double sd[kMaxCoef];
  for (int t = threadIdx.x; t < cnt; t += kBlock) {
    sb[t] = co[t];
    sd[t] = co[cnt + t];
  }
  __syncthreads();
  const double inv_nu = co[2 * cnt];
  const double kappa = co[2 * cnt + 1];
  double av[CPT][6], au[CPT][6];
  long long cellq[CPT];
  bool okq[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const long long c = ((long long)blockIdx.x * CPT + q) * kBlock + threadIdx.x;
    okq[q] = c < N3;
    cellq[q] = okq[q] ? c : 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double uu = okq[q] ? (double)u[p * N3 + c] : 0.0;
      const double xx = okq[q] ? (double)x[p * N3 + c] : 0.0;
      av[q][p] = uu * inv_nu;
      au[q][p] = xx * inv_nu - kappa * uu;
    }
  }
  for (int i = 0; i < cnt; ++i) {
    const double b = sb[i], d = sd[i];
    const T* vi = V + (long long)i * ldv;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      if (!okq[q]) continue;
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const double vv = (double)vi[p * N3 + cellq[q]];
        av[q][p] -= b * vv;
        au[q][p] -= d * vv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    if (!okq[q]) continue;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      vnew[p * N3 + cellq[q]] = T(av[q][p]);
      unext[p * N3 + cellq[q]] = T(au[q][p]);
    }
  }
}

// Small step between pass A and pass B of step j (one workgroup).  With
// red = [a (j), b (j), alpha, beta] from pass A and H the Hessenberg matrix
// (leading dimension ldh) holding columns < j:
//   nu = sqrt(alpha - |b|^2): norm of u after its second projection;
//   H[:j, j-1] += b, H[j, j-1] = nu (column j-1 completed; for j = 0, nu is
//   the start-vector norm, kept in scal[1]);
//   c = Hbar_{j-1} b (length j+1), so A v_j = (x - V_j c) / nu by the Arnoldi
//   relation A V_{j-1} = V_j Hbar_{j-1};
//   h1_i = (a_i - c_i) / nu (i < j), h1_j = (beta - a.b - nu c_j) / nu^2:
//   the first projection of A v_j, stored as H[:j+1, j];
//   co = [b / nu, d, 1 / nu, kappa] for pass B, with kappa = (c_j/nu + h1_j)/nu
//   and d_i = c_i / nu + h1_i - kappa b_i.
// A vanishing nu (relative to the column it completes) is an exact
// invariant subspace: nu and every coefficient are set to zero.
__global__ __launch_bounds__(kBlock) void k_lag_fin(const double* __restrict__ red, int j,
                                                    double* __restrict__ H, int ldh,
                                                    double* __restrict__ co,
                                                    double* __restrict__ scal) {
  __shared__ double sc[kMaxCoef + 1];
  __shared__ double s_nu[1], s_ab[1], s_hj[1];
  const double* a = red;
  const double* b = red + j;
  const double alpha = red[2 * j], beta = red[2 * j + 1];
  double bb = 0.0, ab = 0.0, col = 0.0;
  for (int i = threadIdx.x; i < j; i += kBlock) {
    bb += b[i] * b[i];
    ab += a[i] * b[i];
    const double hv = H[i + (long long)(j - 1) * ldh];
    col += hv * hv;
  }
  __shared__ double t3[3];
  {
    const double v3[3] = {bb, ab, col};
    block_sum_store<3>(v3, 3, t3);
  }
  if (threadIdx.x == 0) {
    const double nu2 = alpha - t3[0];
    double nu = sqrt(fmax(nu2, 0.0));
    const double scale = sqrt(fmax(t3[2] + alpha, 0.0));
    if (!(nu > 1e-12 * scale)) nu = 0.0;
    s_nu[0] = nu;
    s_ab[0] = t3[1];
    if (j == 0) scal[1] = nu;
    else H[j + (long long)(j - 1) * ldh] = nu;
  }
  __syncthreads();
  const double nu = s_nu[0];
  // complete column j-1 and form c = Hbar_{j-1} b (needs the updated column)
  for (int i = threadIdx.x; i < j; i += kBlock) H[i + (long long)(j - 1) * ldh] += b[i];
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += kBlock) {
    double acc = 0.0;
    for (int l = (i > 0 ? i - 1 : 0); l < j; ++l) acc += H[i + (long long)l * ldh] * b[l];
    sc[i] = acc;
  }
  __syncthreads();
  if (nu == 0.0) {
    for (int i = threadIdx.x; i < 2 * j + 2; i += kBlock) co[i] = 0.0;
    for (int i = threadIdx.x; i <= j; i += kBlock) H[i + (long long)j * ldh] = 0.0;
    return;
  }
  const double inv = 1.0 / nu;
  if (threadIdx.x == 0) {
    const double hj = (beta - s_ab[0] - nu * sc[j]) * inv * inv;
    s_hj[0] = hj;
    H[j + (long long)j * ldh] = hj;
    co[2 * j] = inv;
    co[2 * j + 1] = (sc[j] * inv + hj) * inv;
  }
  __syncthreads();
  const double kappa = (sc[j] * inv + s_hj[0]) * inv;
  for (int i = threadIdx.x; i < j; i += kBlock) {
    const double h1 = (a[i] - sc[i]) * inv;
    H[i + (long long)j * ldh] = h1;
    co[i] = b[i] * inv;
    co[j + i] = sc[i] * inv + h1 - kappa * b[i];
  }
}

// End of a cycle: complete the last column from red = [b (m), alpha] (the
// dots of the last candidate u_m with V_0..m-1): H[:m, m-1] += b,
// H[m, m-1] = nu, scal[0] = 1/nu (0 on an invariant subspace).
__global__ __launch_bounds__(kBlock) void k_lag_final(const double* __restrict__ red, int m,
                                                      double* __restrict__ H, int ldh,
                                                      double* __restrict__ scal) {
  double bb = 0.0, col = 0.0;
  for (int i = threadIdx.x; i < m; i += kBlock) {
    bb += red[i] * red[i];
    const double hv = H[i + (long long)(m - 1) * ldh];
    col += hv * hv;
  }
  __shared__ double t2[2];
  const double v2[2] = {bb, col};
  block_sum_store<2>(v2, 2, t2);
  __shared__ double s_nu[1];
  if (threadIdx.x == 0) {
    const double alpha = red[m];
    double nu = sqrt(fmax(alpha - t2[0], 0.0));
    if (!(nu > 1e-12 * sqrt(fmax(t2[1] + alpha, 0.0)))) nu = 0.0;
    H[m + (long long)(m - 1) * ldh] = nu;
    scal[0] = nu > 0.0 ? 1.0 / nu : 0.0;
    s_nu[0] = nu;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += kBlock) H[i + (long long)(m - 1) * ldh] += red[i];
}

// Partial sums of <x, V_i>_M and |x|_M^2.
template <typename T, bool HAS_MU, int CPT>
__global__ __launch_bounds__(kBlock) void k_dots(const T* __restrict__ x, const T* __restrict__ V,
                                                 long long ldv, int cnt, DevGrid g, DevMats mt,
                                                 double* __restrict__ partials) {
  const long long N3 = g.N3;
  double xm[CPT][6];
  long long cellq[CPT];
  bool okq[CPT];
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const long long c = ((long long)blockIdx.x * CPT + q) * kBlock + threadIdx.x;
    okq[q] = c < N3;
    cellq[q] = okq[q] ? c : 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) xm[q][p] = 0.0;
    if (!okq[q]) continue;
    const double we = mt.eps[c];
    const double wh = HAS_MU ? mt.mu[c] : 1.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double xv = (double)x[p * N3 + c];
      xm[q][p] = (p < 3 ? wh : we) * xv;
      nrm += xm[q][p] * xv;
    }
  }
  for (int i0 = 0; i0 < cnt; i0 += kChunk) {
    double acc[kChunk];
#pragma unroll
    for (int r = 0; r < kChunk; ++r) acc[r] = 0.0;
#pragma unroll
    for (int r = 0; r < kChunk; ++r) {
      if (i0 + r < cnt) {
        const T* vi = V + (long long)(i0 + r) * ldv;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          if (!okq[q]) continue;
#pragma unroll
          for (int p = 0; p < 6; ++p) acc[r] += xm[q][p] * (double)vi[p * N3 + cellq[q]];
        }
      }
    }
    const int valid = min(kChunk, cnt - i0);
    block_sum_store<kChunk>(acc, valid, partials + (long long)blockIdx.x * (cnt + 1) + i0);
  }
  const double a1[1] = {nrm};
  block_sum_store<1>(a1, 1, partials + (long long)blockIdx.x * (cnt + 1) + cnt);
}

// out = (w - sum_i coef[i] V_i) * scale; out may alias w (each element is
// read before it is written by the same thread).
template <typename T, int CPT>
__global__ __launch_bounds__(kBlock) void k_update(const T* w, const T* __restrict__ V,
                                                   long long ldv, int cnt,
                                                   const double* __restrict__ coef,
                                                   const double* __restrict__ scale, T* out,
                                                   long long N3) {
  __shared__ double sc[kMaxCoef];
  for (int t = threadIdx.x; t < cnt; t += kBlock) sc[t] = coef[t];
  __syncthreads();
  const double s = scale ? *scale : 1.0;
  double acc[CPT][6];
  long long cellq[CPT];
  bool okq[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const long long c = ((long long)blockIdx.x * CPT + q) * kBlock + threadIdx.x;
    okq[q] = c < N3;
    cellq[q] = okq[q] ? c : 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) acc[q][p] = okq[q] ? (double)w[p * N3 + c] : 0.0;
  }
  for (int i = 0; i < cnt; ++i) {
    const double h = sc[i];
    const T* vi = V + (long long)i * ldv;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      if (!okq[q]) continue;
#pragma unroll
      for (int p = 0; p < 6; ++p) acc[q][p] -= h * (double)vi[p * N3 + cellq[q]];
    }
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    if (!okq[q]) continue;
#pragma unroll
    for (int p = 0; p < 6; ++p) out[p * N3 + cellq[q]] = T(acc[q][p] * s);
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ partials, int nparts,
                                                   int stride, double* __restrict__ out,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;  // (uniform: the whole grid skips)
  const int q = blockIdx.x;
  double acc = 0.0;
  for (int p = threadIdx.x; p < nparts; p += kBlock) acc += partials[(long long)p * stride + q];
  const double a1[1] = {acc};
  block_sum_store<1>(a1, 1, out + q);
}

__global__ void k_fin_start(const double* __restrict__ red, double* __restrict__ scal) {
  if (threadIdx.x == 0) {
    const double b = sqrt(fmax(red[0], 0.0));
    scal[1] = b;
    scal[0] = b > 0.0 ? 1.0 / b : 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_fin_step(const double* __restrict__ red1,
                                                     const double* __restrict__ red2, int j,
                                                     double* __restrict__ H, int ldh,
                                                     double* __restrict__ scal) {
  double ss = 0.0;
  for (int i = threadIdx.x; i <= j; i += kBlock) {
    H[i + (long long)j * ldh] = red1[i] + red2[i];
    ss += red2[i] * red2[i];
  }
  __shared__ double tot[1];
  const double a1[1] = {ss};
  block_sum_store<1>(a1, 1, tot);
  if (threadIdx.x == 0) {
    const double wnorm = sqrt(fmax(red1[j + 1], 0.0));  // |A v_j|_M before projection
    const double nu2 = red2[j + 1] - tot[0];
    double nu = sqrt(fmax(nu2, 0.0));
    if (!(nu > 1e-12 * wnorm)) nu = 0.0;  // exact invariant subspace (or A v_j = 0)
    H[j + 1 + (long long)j * ldh] = nu;
    scal[0] = nu > 0.0 ? 1.0 / nu : 0.0;
  }
}

template <typename T>
__global__ void k_scale(const T* __restrict__ x, const double* __restrict__ s, T* out, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) out[e] = T((double)x[e] * (*s));
}

// out_c (=|+=) sum_{i<m} V_i Y[i + c*m]; columns processed CC at a time.
// With out_last != null the last column (c = ncol - 1) is written to
// out_last instead, never accumulated; out_last may be one of the V_i (a
// thread reads every V_i at its entries before writing them), so then all
// columns must be in one workgroup row (ncol <= CC).
// A thread owns EP consecutive entries of the flat vector (one in FP64, two
// in FP32: every row access is one 512-byte run per wave), and every load
// and store is non-temporal (nothing of the sweep is reused from the
// caches).  The entry count is even and every column starts 64 entries
// aligned, so the FP32 pairs are aligned.  Measured at 128^3, m = 65, on its own: 1.14 ms
// for 3 outputs (6.2 TB/s) against 1.44 ms when a thread owned the six
// components of a cell (six runs per row 2 MB apart, ordinary accesses),
// 1.73 against 2.22 ms for 16 outputs.
// Block b covers entry chunk i and column chunk k with b = ((i / 8) ncc + k)
// 8 + i mod 8: every column chunk of an entry chunk runs on the XCD that the
// dispatcher assigns to b mod 8 = i mod 8, at nearby dispatch times, so the
// basis entries of the chunk come from HBM once and from that XCD's L2 for
// the other column chunks.
typedef float vf2 __attribute__((ext_vector_type(2)));  // FP32 pair for the non-temporal builtins

template <typename T, int CC>
__global__ __launch_bounds__(kBlock) void k_combine(const T* V, long long ldv, int m,
                                                    const double* __restrict__ Y, int ncol,
                                                    T* out, long long ldo,
                                                    const int* __restrict__ colmap, int accumulate,
                                                    T* out_last, long long n, int ncc, long long gx) {
  extern __shared__ double sY[];  // m * CC
  const long long bt = blockIdx.x >> 3;
  const int kchunk = (int)(bt % ncc);
  const long long ichunk = (bt / ncc) * 8 + (blockIdx.x & 7);
  if (ichunk >= gx) return;
  const int c0 = kchunk * CC;
  const int nc = min(CC, ncol - c0);
  for (int t = threadIdx.x; t < m * CC; t += kBlock) {
    const int i = t / CC, cc = t % CC;
    sY[t] = (cc < nc) ? Y[i + (long long)(c0 + cc) * m] : 0.0;
  }
  __syncthreads();
  constexpr int EP = sizeof(T) == 4 ? 2 : 1;
  const long long e = (ichunk * kBlock + threadIdx.x) * EP;
  if (e >= n) return;
  double acc[EP][CC];
#pragma unroll
  for (int q = 0; q < EP; ++q)
#pragma unroll
    for (int cc = 0; cc < CC; ++cc) acc[q][cc] = 0.0;
#pragma unroll 2
  for (int i = 0; i < m; ++i) {
    double v[EP];
    if constexpr (EP == 2) {
      const vf2 x = __builtin_nontemporal_load(reinterpret_cast<const vf2*>(V + (long long)i * ldv + e));
      v[0] = x.x;
      v[1] = x.y;
    } else {
      v[0] = (double)__builtin_nontemporal_load(V + (long long)i * ldv + e);
    }
#pragma unroll
    for (int cc = 0; cc < CC; ++cc) {
      const double y = sY[i * CC + cc];
#pragma unroll
      for (int q = 0; q < EP; ++q) acc[q][cc] += v[q] * y;
    }
  }
#pragma unroll
  for (int cc = 0; cc < CC; ++cc) {
    if (cc >= nc) break;
    const bool last = out_last && c0 + cc == ncol - 1;
    const int col = last ? 0 : (colmap ? colmap[c0 + cc] : (c0 + cc));
    T* o = (last ? out_last : out + (long long)col * ldo) + e;
    const bool acc_on = !last && accumulate;
    if constexpr (EP == 2) {
      vf2 r;
      if (acc_on) {
        const vf2 prev = __builtin_nontemporal_load(reinterpret_cast<const vf2*>(o));
        r.x = T((double)prev.x + acc[0][cc]);
        r.y = T((double)prev.y + acc[1][cc]);
      } else {
        r.x = T(acc[0][cc]);
        r.y = T(acc[1][cc]);
      }
      __builtin_nontemporal_store(r, reinterpret_cast<vf2*>(o));
    } else {
      const double prev = acc_on ? (double)__builtin_nontemporal_load(o) : 0.0;
      __builtin_nontemporal_store(T(prev + acc[0][cc]), o);
    }
  }
}

template <typename T>
__global__ void k_load_complex(const double* __restrict__ b, int part, T* __restrict__ out,
                               long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) out[e] = T(b[2 * e + part]);
}

template <typename T>
__global__ void k_load_real(const double* __restrict__ src, T* __restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) out[e] = T(src[e]);
}

template <typename T>
__global__ void k_store_real(const T* __restrict__ src, double* __restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) out[e] = (double)src[e];
}

template <typename T>
__global__ void k_store_complex(const T* __restrict__ re, const T* __restrict__ im,
                                double* __restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) {
    out[2 * e] = (double)re[e];
    out[2 * e + 1] = (double)im[e];
  }
}

template <typename T>
__global__ void k_assemble(const T* __restrict__ re, const T* __restrict__ im,
                           const T* __restrict__ yhat, double sn, double cs,
                           double* __restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) {
    double v = sn * (double)re[e] + cs * (double)im[e];
    if (yhat) v -= (double)yhat[e];
    out[e] = v;
  }
}

// Residual of a complex shifted system for a trial z = zre + i zim:
// r = b - (A + i w) z, with azr = A zre and azi = A zim already applied;
// b and r complex interleaved (FP64).
template <typename T>
__global__ void k_shift_residual(const double* __restrict__ b, const T* __restrict__ zre,
                                 const T* __restrict__ zim, const T* __restrict__ azr,
                                 const T* __restrict__ azi, double w, double* __restrict__ r,
                                 long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) {
    r[2 * e] = b[2 * e] - ((double)azr[e] - w * (double)zim[e]);
    r[2 * e + 1] = b[2 * e + 1] - ((double)azi[e] + w * (double)zre[e]);
  }
}

// Period-averaged Poynting flux of the time-harmonic field z = zre + i zim
// through the plane z = kf, and the adjoint right-hand side.  One thread per
// (i, j) column of the plane:
//   Hbar = (z_H[kf-1] + z_H[kf]) / 2,
//   P += 1/2 Re(z_Ex conj(Hbar_y) - z_Ey conj(Hbar_x))   (block partials),
// and with a = dP/dz (dP = Re(a^T dz)):
//   a_Ex = conj(Hbar_y)/2, a_Ey = -conj(Hbar_x)/2,
//   a_Hy[kf-1] = a_Hy[kf] = conj(z_Ex)/4, a_Hx[kf-1] = a_Hx[kf] = -conj(z_Ey)/4,
// the adjoint system (A^T + i w) lam = a is solved as (A + i w) x = P M^-1 a
// (A^T = M P A P M^-1 with P = diag(I_H, -I_E)), so rhs = P M^-1 a is
// written (complex interleaved) at those entries; rhs must be zero elsewhere.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flux_seed(const T* __restrict__ zre,
                                                      const T* __restrict__ zim, int kf,
                                                      DevGrid g, DevMats mt,
                                                      double* __restrict__ partials,
                                                      double* __restrict__ rhs) {
  const long long N2 = (long long)g.nx * g.ny;
  const long long N3 = g.N3;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  double p = 0.0;
  if (t < N2) {
    const long long c1 = (long long)kf * N2 + t;  // cell at kf
    const long long c0 = c1 - N2;                 // cell at kf - 1
    auto Z = [&](int comp, long long c, double& re, double& im) {
      re = (double)zre[comp * N3 + c];
      im = (double)zim[comp * N3 + c];
    };
    double hx0r, hx0i, hx1r, hx1i, hy0r, hy0i, hy1r, hy1i, exr, exi, eyr, eyi;
    Z(0, c0, hx0r, hx0i);
    Z(0, c1, hx1r, hx1i);
    Z(1, c0, hy0r, hy0i);
    Z(1, c1, hy1r, hy1i);
    Z(3, c1, exr, exi);
    Z(4, c1, eyr, eyi);
    const double hxr = 0.5 * (hx0r + hx1r), hxi = 0.5 * (hx0i + hx1i);
    const double hyr = 0.5 * (hy0r + hy1r), hyi = 0.5 * (hy0i + hy1i);
    // Re(u conj(v)) = ur vr + ui vi
    p = 0.5 * ((exr * hyr + exi * hyi) - (eyr * hxr + eyi * hxi));
    if (rhs) {
      const double ie = mt.inv_eps[c1];
      const double im0 = mt.inv_mu ? mt.inv_mu[c0] : 1.0;
      const double im1 = mt.inv_mu ? mt.inv_mu[c1] : 1.0;
      // E rows: -a_E / eps
      rhs[2 * (3 * N3 + c1)] = -0.5 * hyr * ie;
      rhs[2 * (3 * N3 + c1) + 1] = 0.5 * hyi * ie;
      rhs[2 * (4 * N3 + c1)] = 0.5 * hxr * ie;
      rhs[2 * (4 * N3 + c1) + 1] = -0.5 * hxi * ie;
      // H rows: a_H / mu
      rhs[2 * (1 * N3 + c0)] = 0.25 * exr * im0;
      rhs[2 * (1 * N3 + c0) + 1] = -0.25 * exi * im0;
      rhs[2 * (1 * N3 + c1)] = 0.25 * exr * im1;
      rhs[2 * (1 * N3 + c1) + 1] = -0.25 * exi * im1;
      rhs[2 * (0 * N3 + c0)] = -0.25 * eyr * im0;
      rhs[2 * (0 * N3 + c0) + 1] = 0.25 * eyi * im0;
      rhs[2 * (0 * N3 + c1)] = -0.25 * eyr * im1;
      rhs[2 * (0 * N3 + c1) + 1] = 0.25 * eyi * im1;
    }
  }
  const double a1[1] = {p};
  block_sum_store<1>(a1, 1, partials + blockIdx.x);
}

// Gradient of the flux w.r.t. per-cell eps for one frequency, accumulated:
// dL/d eps_c += sum_{E rows r of c} Re(lam_r (A z)_r) / eps_c with
// lam = M P x (so lam_E = -eps x_E) and A z = b - i w z (the shifted
// equation), i.e. g_c -= sum_{p in Ex,Ey,Ez} Re(x_p (b_p - i w z_p)).
template <typename T>
__global__ void k_grad_acc(const T* __restrict__ zre, const T* __restrict__ zim,
                           const T* __restrict__ xre, const T* __restrict__ xim,
                           const double* __restrict__ b, double w, double* __restrict__ g,
                           long long N3) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= N3) return;
  double acc = 0.0;
#pragma unroll
  for (int p = 3; p < 6; ++p) {
    const long long e = p * N3 + c;
    const double azr = b[2 * e] + w * (double)zim[e];
    const double azi = b[2 * e + 1] - w * (double)zre[e];
    acc += (double)xre[e] * azr - (double)xim[e] * azi;
  }
  g[c] -= acc;
}

__global__ void k_fill(double* __restrict__ p, double v, long long n) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) p[e] = v;
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int cells_per_thread(long long N3) { return N3 >= (long long)kBlock * 4 * 1024 ? 4 : 1; }
int cell_blocks(long long N3, int cpt) {
  const long long per = (long long)kBlock * cpt;
  return (int)((N3 + per - 1) / per);
}

// dispatch a kernel template over cells per thread (1, 2, 4)
#define KRY_CPT_SWITCH(cpt, X) \
  switch (cpt) {               \
    case 4: X(4) break;        \
    case 2: X(2) break;        \
    default: X(1) break;       \
  }

template <typename T>
static hipError_t stencil_t(const void* v, void* w, const void* V, long long ldv, int cnt,
                            const DevGrid& g, const DevMats& m, double* partials, hipStream_t s) {
  const int cpt = g.cpt_s;
  const dim3 grid(cell_blocks(g.N3, cpt)), blk(kBlock);
  const T* vv = (const T*)v;
  T* ww = (T*)w;
  const T* VV = (const T*)V;
  const bool dots = V != nullptr;
  const bool mu = m.inv_mu != nullptr;
#define KRY_STENCIL(C)                                                                           \
  if (mu) {                                                                                      \
    if (dots) hipLaunchKernelGGL((k_stencil<T, true, C, true>), grid, blk, 0, s, vv, ww, VV, ldv, cnt, g, m, partials); \
    else hipLaunchKernelGGL((k_stencil<T, true, C, false>), grid, blk, 0, s, vv, ww, VV, ldv, cnt, g, m, partials);     \
  } else {                                                                                       \
    if (dots) hipLaunchKernelGGL((k_stencil<T, false, C, true>), grid, blk, 0, s, vv, ww, VV, ldv, cnt, g, m, partials); \
    else hipLaunchKernelGGL((k_stencil<T, false, C, false>), grid, blk, 0, s, vv, ww, VV, ldv, cnt, g, m, partials);     \
  }
  KRY_CPT_SWITCH(cpt, KRY_STENCIL)
#undef KRY_STENCIL
  return hipGetLastError();
}

template <typename T>
static hipError_t stencil_cols_t(const void* v, void* w, long long ld, int ncols, const DevGrid& g,
                                 const DevMats& m, hipStream_t s) {
  const int cpt = g.cpt_s;
  const dim3 grid(cell_blocks(g.N3, cpt), ncols), blk(kBlock);
  const T* vv = (const T*)v;
  T* ww = (T*)w;
  const bool mu = m.inv_mu != nullptr;
#define KRY_SCOLS(C)                                                                                   \
  if (mu) hipLaunchKernelGGL((k_stencil<T, true, C, false>), grid, blk, 0, s, vv, ww, nullptr, ld, 0, g, m, nullptr); \
  else hipLaunchKernelGGL((k_stencil<T, false, C, false>), grid, blk, 0, s, vv, ww, nullptr, ld, 0, g, m, nullptr);
  KRY_CPT_SWITCH(cpt, KRY_SCOLS)
#undef KRY_SCOLS
  return hipGetLastError();
}

hipError_t launch_stencil_cols(Storage st, const void* v, void* w, long long ld, int ncols,
                               const DevGrid& g, const DevMats& m, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  return st == F64 ? stencil_cols_t<double>(v, w, ld, ncols, g, m, s)
                   : stencil_cols_t<float>(v, w, ld, ncols, g, m, s);
}

template <typename T>
static hipError_t stencil_axpby_t(const void* v, const void* prev, void* out, double alpha,
                                  double gamma, double beta, const DevGrid& g, const DevMats& m,
                                  hipStream_t s) {
  if (g.zm_s > 0) {  // z-marching columns, g.zm_s planes per workgroup
    const int tiles_x = (g.nx + 63) / 64, tiles_y = (g.ny + 3) / 4;
    const int kz = g.zm_s >= 16 ? 16 : (g.zm_s >= 8 ? 8 : 4);
    const dim3 grid((unsigned)(tiles_x * tiles_y * ((g.nz + kz - 1) / kz))), blk(kBlock);
    const T* vv = (const T*)v;
    const T* pp = (const T*)prev;
    T* oo = (T*)out;
    const bool mu = m.inv_mu != nullptr;
#define KRY_SZM(KZ)                                                                                      \
  if (mu) hipLaunchKernelGGL((k_stencil_axpby_zm<T, true, KZ>), grid, blk, 0, s, vv, pp, oo, alpha, gamma, \
                             beta, g, m, tiles_x, tiles_y);                                             \
  else hipLaunchKernelGGL((k_stencil_axpby_zm<T, false, KZ>), grid, blk, 0, s, vv, pp, oo, alpha, gamma,   \
                          beta, g, m, tiles_x, tiles_y);
    if (kz == 16) { KRY_SZM(16) } else if (kz == 8) { KRY_SZM(8) } else { KRY_SZM(4) }
#undef KRY_SZM
    return hipGetLastError();
  }
  const int cpt = g.cpt_s;
  const dim3 grid(cell_blocks(g.N3, cpt)), blk(kBlock);
  const T* vv = (const T*)v;
  const T* pp = (const T*)prev;
  T* oo = (T*)out;
  const bool mu = m.inv_mu != nullptr;
#define KRY_SAXPBY(C)                                                                            \
  if (mu) hipLaunchKernelGGL((k_stencil_axpby<T, true, C>), grid, blk, 0, s, vv, pp, oo, alpha, gamma, beta, g, m); \
  else hipLaunchKernelGGL((k_stencil_axpby<T, false, C>), grid, blk, 0, s, vv, pp, oo, alpha, gamma, beta, g, m);
  KRY_CPT_SWITCH(cpt, KRY_SAXPBY)
#undef KRY_SAXPBY
  return hipGetLastError();
}

hipError_t launch_stencil_axpby(Storage st, const void* v, const void* prev, void* out, double alpha,
                                double gamma, double beta, const DevGrid& g, const DevMats& m,
                                hipStream_t s) {
  return st == F64 ? stencil_axpby_t<double>(v, prev, out, alpha, gamma, beta, g, m, s)
                   : stencil_axpby_t<float>(v, prev, out, alpha, gamma, beta, g, m, s);
}

hipError_t launch_stencil(Storage st, const void* v, void* w, const void* V, long long ldv, int cnt,
                          const DevGrid& g, const DevMats& m, double* partials, hipStream_t s) {
  return st == F64 ? stencil_t<double>(v, w, V, ldv, cnt, g, m, partials, s)
                   : stencil_t<float>(v, w, V, ldv, cnt, g, m, partials, s);
}

template <typename T>
static hipError_t stencil_lag_t(const void* u, void* x, const void* V, long long ldv, int cnt,
                                const DevGrid& g, const DevMats& m, double* partials, hipStream_t s) {
  const int cpt = g.cpt_s;
  const dim3 grid(cell_blocks(g.N3, cpt)), blk(kBlock);
  const T* uu = (const T*)u;
  T* xx = (T*)x;
  const T* VV = (const T*)V;
  const bool mu = m.inv_mu != nullptr;
  constexpr int CH = 8;
#define KRY_SLAG(C)                                                                                     \
  if (mu) hipLaunchKernelGGL((k_stencil_lag<T, true, C, CH>), grid, blk, 0, s, uu, xx, VV, ldv, cnt, g, m, partials); \
  else hipLaunchKernelGGL((k_stencil_lag<T, false, C, CH>), grid, blk, 0, s, uu, xx, VV, ldv, cnt, g, m, partials);
  KRY_CPT_SWITCH(cpt, KRY_SLAG)
#undef KRY_SLAG
  return hipGetLastError();
}

hipError_t launch_stencil_lag(Storage st, const void* u, void* x, const void* V, long long ldv, int cnt,
                              const DevGrid& g, const DevMats& m, double* partials, hipStream_t s) {
  return st == F64 ? stencil_lag_t<double>(u, x, V, ldv, cnt, g, m, partials, s)
                   : stencil_lag_t<float>(u, x, V, ldv, cnt, g, m, partials, s);
}

template <typename T>
static hipError_t lag_update_t(const void* u, const void* x, const void* V, long long ldv, int cnt,
                               const double* co, void* vnew, void* unext, const DevGrid& g,
                               hipStream_t s) {
  if (cnt > kMaxCoef) return hipErrorInvalidValue;
  const int cpt = g.cpt_u;
  const dim3 grid(cell_blocks(g.N3, cpt)), blk(kBlock);
#define KRY_LUPD(C)                                                                                \
  hipLaunchKernelGGL((k_lag_update<T, C>), grid, blk, 0, s, (const T*)u, (const T*)x, (const T*)V, \
                     ldv, cnt, co, (T*)vnew, (T*)unext, g.N3);
  KRY_CPT_SWITCH(cpt, KRY_LUPD)
#undef KRY_LUPD
  return hipGetLastError();
}

hipError_t launch_lag_update(Storage st, const void* u, const void* x, const void* V, long long ldv,
                             int cnt, const double* co, void* vnew, void* unext, const DevGrid& g,
                             hipStream_t s) {
  return st == F64 ? lag_update_t<double>(u, x, V, ldv, cnt, co, vnew, unext, g, s)
                   : lag_update_t<float>(u, x, V, ldv, cnt, co, vnew, unext, g, s);
}

hipError_t launch_lag_fin(const double* red, int j, double* H, int ldh, double* co, double* scal,
                          hipStream_t s) {
  if (j + 1 > kMaxCoef) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lag_fin, dim3(1), dim3(kBlock), 0, s, red, j, H, ldh, co, scal);
  return hipGetLastError();
}

hipError_t launch_lag_final(const double* red, int m, double* H, int ldh, double* scal,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_lag_final, dim3(1), dim3(kBlock), 0, s, red, m, H, ldh, scal);
  return hipGetLastError();
}

template <typename T>
static hipError_t dots_t(const void* x, const void* V, long long ldv, int cnt, const DevGrid& g,
                         const DevMats& m, double* partials, hipStream_t s) {
  const int cpt = g.cpt_d;
  const dim3 grid(cell_blocks(g.N3, cpt)), blk(kBlock);
  const bool mu = m.inv_mu != nullptr;
  const T* xx = (const T*)x;
  const T* VV = (const T*)V;
#define KRY_DOTS(C)                                                                                   \
  if (mu) hipLaunchKernelGGL((k_dots<T, true, C>), grid, blk, 0, s, xx, VV, ldv, cnt, g, m, partials); \
  else hipLaunchKernelGGL((k_dots<T, false, C>), grid, blk, 0, s, xx, VV, ldv, cnt, g, m, partials);
  KRY_CPT_SWITCH(cpt, KRY_DOTS)
#undef KRY_DOTS
  return hipGetLastError();
}

hipError_t launch_dots(Storage st, const void* x, const void* V, long long ldv, int cnt,
                       const DevGrid& g, const DevMats& m, double* partials, hipStream_t s) {
  return st == F64 ? dots_t<double>(x, V, ldv, cnt, g, m, partials, s)
                   : dots_t<float>(x, V, ldv, cnt, g, m, partials, s);
}

template <typename T>
static hipError_t update_t(const void* w, const void* V, long long ldv, int cnt, const double* coef,
                           const double* scale, void* out, const DevGrid& g, hipStream_t s) {
  if (cnt > kMaxCoef) return hipErrorInvalidValue;
  const int cpt = g.cpt_u;
  const dim3 grid(cell_blocks(g.N3, cpt)), blk(kBlock);
#define KRY_UPD(C)                                                                                  \
  hipLaunchKernelGGL((k_update<T, C>), grid, blk, 0, s, (const T*)w, (const T*)V, ldv, cnt, coef,   \
                     scale, (T*)out, g.N3);
  KRY_CPT_SWITCH(cpt, KRY_UPD)
#undef KRY_UPD
  return hipGetLastError();
}

hipError_t launch_update(Storage st, const void* w, const void* V, long long ldv, int cnt,
                         const double* coef, const double* scale, void* out, const DevGrid& g,
                         hipStream_t s) {
  return st == F64 ? update_t<double>(w, V, ldv, cnt, coef, scale, out, g, s)
                   : update_t<float>(w, V, ldv, cnt, coef, scale, out, g, s);
}

hipError_t launch_reduce(const double* partials, int nparts, int stride, int cnt, double* out,
                         hipStream_t s, const int* skip) {
  hipLaunchKernelGGL(k_reduce, dim3(cnt), dim3(kBlock), 0, s, partials, nparts, stride, out, skip);
  return hipGetLastError();
}

hipError_t launch_fin_start(const double* red, double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(64), 0, s, red, scal);
  return hipGetLastError();
}

hipError_t launch_fin_step(const double* red1, const double* red2, int j, double* H, int ldh,
                           double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_step, dim3(1), dim3(kBlock), 0, s, red1, red2, j, H, ldh, scal);
  return hipGetLastError();
}

hipError_t launch_scale(Storage st, const void* x, const double* scale, void* out, long long n,
                        hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_scale<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s, (const double*)x,
                       scale, (double*)out, n);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s, (const float*)x,
                       scale, (float*)out, n);
  return hipGetLastError();
}

template <typename T>
static hipError_t combine_t(const void* V, long long ldv, int m, const double* Y, int ncol, void* out,
                            long long ldo, const int* colmap, int accumulate, void* out_last,
                            const DevGrid& g, hipStream_t s) {
  if (m <= 0 || ncol <= 0) return hipSuccess;
  // columns per workgroup: 1, 4, 8 or chunks of CMAX.  FP64: chunks of 16
  // (8 waves per SIMD; at 128^3, m = 65, 16 outputs took 1.73 ms against
  // 2.42 ms in two chunks of 8).  FP32 (two entries per thread): chunks of
  // 8 (at 256^3, m = 49, 16 outputs took 8.9 ms against 10.8 ms in one
  // chunk of 16, whose 32 accumulators leave 5 waves per SIMD)
  constexpr int CMAX = sizeof(T) == 4 ? 8 : 16;
  constexpr int EPT = sizeof(T) == 4 ? 2 : 1;  // entries per thread
  if (out_last && ncol > CMAX) return hipErrorInvalidValue;
  const long long n = 6 * g.N3;
  const long long gx = (n + kBlock * EPT - 1) / (kBlock * EPT);  // workgroups per column chunk
  const long long g8 = (gx + 7) / 8 * 8;
#define KRY_COMB(CCW)                                                                                     \
  {                                                                                                       \
    const int ncc = (ncol + (CCW) - 1) / (CCW);                                                           \
    const size_t shm = sizeof(double) * (size_t)m * (CCW);                                                \
    hipLaunchKernelGGL((k_combine<T, CCW>), dim3((unsigned)(g8 * ncc)), dim3(kBlock), shm, s, (const T*)V, \
                       ldv, m, Y, ncol, (T*)out, ldo, colmap, accumulate, (T*)out_last, n, ncc, gx);      \
  }
  if (ncol == 1)
    KRY_COMB(1)
  else if (ncol <= 4)
    KRY_COMB(4)
  else if (ncol <= 8)
    KRY_COMB(8)
  else
    KRY_COMB(CMAX)
#undef KRY_COMB
  return hipGetLastError();
}

hipError_t launch_combine(Storage st, const void* V, long long ldv, int m, const double* Y, int ncol,
                          void* out, long long ldo, const int* colmap, int accumulate,
                          const DevGrid& g, hipStream_t s, void* out_last) {
  return st == F64 ? combine_t<double>(V, ldv, m, Y, ncol, out, ldo, colmap, accumulate, out_last, g, s)
                   : combine_t<float>(V, ldv, m, Y, ncol, out, ldo, colmap, accumulate, out_last, g, s);
}

hipError_t launch_shift_residual(Storage st, const double* b, const void* zre, const void* zim,
                                 const void* azr, const void* azi, double w, double* r, long long n,
                                 hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_shift_residual<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s, b,
                       (const double*)zre, (const double*)zim, (const double*)azr,
                       (const double*)azi, w, r, n);
  else
    hipLaunchKernelGGL(k_shift_residual<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s, b,
                       (const float*)zre, (const float*)zim, (const float*)azr, (const float*)azi, w,
                       r, n);
  return hipGetLastError();
}

hipError_t launch_load_complex(Storage st, const double* b, int part, void* out, long long n,
                               hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_load_complex<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s, b, part,
                       (double*)out, n);
  else
    hipLaunchKernelGGL(k_load_complex<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s, b, part,
                       (float*)out, n);
  return hipGetLastError();
}

hipError_t launch_load_real(Storage st, const double* src, void* out, long long n, hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_load_real<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s, src,
                       (double*)out, n);
  else
    hipLaunchKernelGGL(k_load_real<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s, src,
                       (float*)out, n);
  return hipGetLastError();
}

hipError_t launch_store_real(Storage st, const void* src, double* out, long long n, hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_store_real<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                       (const double*)src, out, n);
  else
    hipLaunchKernelGGL(k_store_real<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                       (const float*)src, out, n);
  return hipGetLastError();
}

hipError_t launch_store_complex(Storage st, const void* re, const void* im, double* out,
                                long long n, hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_store_complex<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                       (const double*)re, (const double*)im, out, n);
  else
    hipLaunchKernelGGL(k_store_complex<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                       (const float*)re, (const float*)im, out, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_flux_seed(Storage st, const void* zre, const void* zim, int kf, const DevGrid& g,
                            const DevMats& m, double* partials, double* rhs, int* nblocks,
                            hipStream_t s) {
  const long long N2 = (long long)g.nx * g.ny;
  const unsigned nb = blocks_for(N2);
  *nblocks = (int)nb;
  if (st == F64)
    hipLaunchKernelGGL(k_flux_seed<double>, dim3(nb), dim3(kBlock), 0, s, (const double*)zre,
                       (const double*)zim, kf, g, m, partials, rhs);
  else
    hipLaunchKernelGGL(k_flux_seed<float>, dim3(nb), dim3(kBlock), 0, s, (const float*)zre,
                       (const float*)zim, kf, g, m, partials, rhs);
  return hipGetLastError();
}

hipError_t launch_grad_acc(Storage st, const void* zre, const void* zim, const void* xre,
                           const void* xim, const double* b, double w, double* g, long long N3,
                           hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_grad_acc<double>, dim3(blocks_for(N3)), dim3(kBlock), 0, s,
                       (const double*)zre, (const double*)zim, (const double*)xre,
                       (const double*)xim, b, w, g, N3);
  else
    hipLaunchKernelGGL(k_grad_acc<float>, dim3(blocks_for(N3)), dim3(kBlock), 0, s,
                       (const float*)zre, (const float*)zim, (const float*)xre,
                       (const float*)xim, b, w, g, N3);
  return hipGetLastError();
}

hipError_t launch_assemble(Storage st, const void* re, const void* im, const void* yhat, double sn,
                           double cs, double* out, long long n, hipStream_t s) {
  if (st == F64)
    hipLaunchKernelGGL(k_assemble<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                       (const double*)re, (const double*)im, (const double*)yhat, sn, cs, out, n);
  else
    hipLaunchKernelGGL(k_assemble<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                       (const float*)re, (const float*)im, (const float*)yhat, sn, cs, out, n);
  return hipGetLastError();
}

}  // namespace kry
