// Device finish of one Gram-Schmidt pass of an s-step Arnoldi block, so
// that a whole restart cycle runs without a host round trip per block.
//
// Pass p of block classical Gram-Schmidt on the block S (s columns) against
// the M-orthonormal basis V (M columns) has the Gram product
// P = [V, S]^T M S: C = P[:M] = V^T M S, and the projected Gram matrix
// G = S^T M S - C^T C (Pythagoras).  With the Cholesky factor R of G
// (R^T R = G, R upper) the pass's result is (S - V C) R^{-1}, one update
// [V, S] K with K = [-C R^{-1}; R^{-1}].  A pivot at or below thr^2 ref_k
// (ref: the squared column norms of S on pass 1, 1 on pass 2) marks a
// dependent block.  Pass 1 is final when the column-scaled condition
// estimate |R D|_F |(R D)^{-1}|_F (D = diag(1 / |S_k|)) is at most
// one_pass_max and every column keeps at least one_pass_left of its squared
// norm after the projection (G is a difference: a block mostly inside the
// basis loses digits there); after pass 2 the product R2 R1 must stay below
// cond_max.
// One workgroup of 256 threads; s <= 16 and M + s <= 256.
#include "kry_internal.h"

namespace kry {

namespace {

constexpr int kSS = 16;  // largest block size of the device finish

__global__ __launch_bounds__(256) void k_sstep_fin(int pass, int M, int s, const double* __restrict__ P,
                                                   double* __restrict__ K, double* __restrict__ stash,
                                                   int* __restrict__ flags, double one_pass_max,
                                                   double one_pass_left, double cond_max) {
  if (pass == 2 && flags[1]) return;  // final after pass 1 (uniform)
  __shared__ double G[kSS * kSS], R[kSS * kSS], Ri[kSS * kSS], ref[kSS], part1[256], part2[256];
  __shared__ double Ps[256 * kSS];  // P staged once, read many times
  __shared__ int ok;
  const int t = threadIdx.x;
  for (int e = t; e < (M + s) * s; e += 256) Ps[e] = P[e];
  __syncthreads();
  // stash layout: C1 (M s), R1 (s s), |S_k|^2 (s), R1^{-1} (s s), C2 (M s), R2 (s s)
  double* C1 = stash;
  double* R1 = C1 + (long long)M * s;
  double* nrm = R1 + s * s;
  double* Ri1 = nrm + s;
  double* C2 = Ri1 + s * s;
  double* R2 = C2 + (long long)M * s;
  double* Cst = pass == 1 ? C1 : C2;
  double* Rst = pass == 1 ? R1 : R2;
  if (t < s * s) {
    const int a = t / s, b = t % s;
    double g = Ps[(M + a) * s + b];
    for (int k = 0; k < M; ++k) g -= Ps[k * s + a] * Ps[k * s + b];
    G[a * kSS + b] = g;
  }
  if (t < s) ref[t] = pass == 1 ? Ps[(M + t) * s + t] : 1.0;
  for (int e = t; e < M * s; e += 256) Cst[e] = Ps[e];
  if (t == 0) ok = 1;
  __syncthreads();
  if (pass == 1 && t < s) nrm[t] = ref[t];
  // Cholesky by rows (row k from the rows above it, the order of the host
  // factorisation); every thread reads the same pivot, so the exit on a
  // dependent block is uniform
  const double thr = pass == 1 ? 1e-10 : 1e-8;
  __shared__ double row[kSS];
  for (int k = 0; k < s; ++k) {
    if (t >= k && t < s) {
      double v = G[k * kSS + t];
      for (int l = 0; l < k; ++l) v -= R[l * kSS + k] * R[l * kSS + t];
      row[t] = v;
    }
    __syncthreads();
    const double piv = row[k];
    if (!(piv > thr * thr * ref[k]) || !isfinite(piv)) {
      if (t == 0) ok = 0;
      break;
    }
    const double rkk = sqrt(piv);
    if (t < s) R[k * kSS + t] = t < k ? 0.0 : (t == k ? rkk : row[t] / rkk);
    __syncthreads();
  }
  __syncthreads();
  const bool good = ok != 0;
  // R^{-1}, one column per thread
  if (good && t < s) {
    const int j = t;
    Ri[j * kSS + j] = 1.0 / R[j * kSS + j];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int l = i + 1; l <= j; ++l) acc += R[i * kSS + l] * Ri[l * kSS + j];
      Ri[i * kSS + j] = -acc / R[i * kSS + i];
    }
    for (int i = j + 1; i < s; ++i) Ri[i * kSS + j] = 0.0;
  }
  __syncthreads();
  // column-scaled condition estimate: of R1 (pass 1) or of R2 R1 (pass 2)
  part1[t] = 0.0;
  part2[t] = 0.0;
  if (good && t < s * s) {
    const int a = t / s, k = t % s;
    if (a <= k) {
      double r = 0.0, ri = 0.0;
      if (pass == 1) {
        r = R[a * kSS + k];
        ri = Ri[a * kSS + k];
      } else {
        for (int l = a; l <= k; ++l) {
          r += R[a * kSS + l] * R1[l * s + k];
          ri += Ri1[a * s + l] * Ri[l * kSS + k];
        }
      }
      part1[t] = r * r / fmax(nrm[k], 1e-300);
      part2[t] = nrm[a] * ri * ri;
    }
  }
  __syncthreads();
  // stash R (and R^{-1} on pass 1), the coefficients K
  if (t < s * s) {
    const int a = t / s, b = t % s;
    Rst[a * s + b] = good ? (a <= b ? R[a * kSS + b] : 0.0) : 0.0;
    if (pass == 1) Ri1[a * s + b] = good ? Ri[a * kSS + b] : 0.0;
  }
  for (int e = t; e < (M + s) * s; e += 256) {
    const int k = e / s, b = e % s;
    double v;
    if (!good) {
      v = (k >= M && k - M == b) ? 1.0 : 0.0;
    } else if (k < M) {
      double acc = 0.0;
      for (int l = 0; l <= b; ++l) acc += Ps[k * s + l] * Ri[l * kSS + b];
      v = -acc;
    } else {
      v = Ri[(k - M) * kSS + b];
    }
    K[e] = v;
  }
  // the two Frobenius sums: a tree over the 256 partial values
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      part1[t] += part1[t + h];
      part2[t] += part2[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double f1 = part1[0], f2 = part2[0];
    const double est = sqrt(f1 * f2);
    double left = 1.0;
    for (int k = 0; k < s; ++k) left = fmin(left, G[k * kSS + k] / fmax(ref[k], 1e-300));
    if (pass == 1) {
      flags[0] = good ? 1 : 0;
      // (a failed block skips pass 2)
      flags[1] = good ? (est <= one_pass_max && left >= one_pass_left ? 1 : 0) : 1;
      flags[2] = 1;
      flags[3] = 0;
    } else {
      flags[2] = good ? 1 : 0;
      flags[3] = good ? (est <= cond_max ? 0 : 1) : 0;
    }
  }
}

}  // namespace

int sstep_stash_doubles(int M, int s) { return 2 * M * s + 3 * s * s + s; }

hipError_t launch_sstep_fin(int pass, int M, int s, const double* P, double* K, double* stash, int* flags,
                            double one_pass_max, double one_pass_left, double cond_max, hipStream_t st) {
  if ((pass != 1 && pass != 2) || s < 1 || s > kSS || M < 1 || M + s > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sstep_fin, dim3(1), dim3(256), 0, st, pass, M, s, P, K, stash, flags, one_pass_max,
                     one_pass_left, cond_max);
  return hipGetLastError();
}

}  // namespace kry
