// C-ABI driver: context, workspaces, Arnoldi cycles, restarted multi-shift
// shifted solves, time-restarted exponential, split assembly.
#include "../../include/kry.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "kry_dense.h"
#include "kry_internal.h"

using kry::cplx;

struct kry_ctx {
  kry::DevGrid g{};
  long long n = 0;    // 6 N3
  long long ldv = 0;  // padded vector stride (elements)
  kry::Storage st = kry::F64;
  size_t esz = 8;
  kry_opts opts{};
  hipStream_t stream = nullptr;

  double* d_mat = nullptr;  // one allocation holding the derived material arrays
  kry::DevMats mats{};

  // Krylov workspace: slots 0..mcap hold the basis, slot mcap+1 the work vector.
  int mcap = 0;
  int vextra = 0;  // work slots after the basis in the allocation
  void* V = nullptr;
  double* partials = nullptr;
  double* d_red1 = nullptr;
  double* d_red2 = nullptr;
  double* d_scal = nullptr;
  double* d_co = nullptr;  // pass-B coefficients of the delayed scheme
  double* d_H = nullptr;
  double* d_Y = nullptr;
  int* d_colmap = nullptr;
  // column-norm workspace: partials (cn_cap doubles) and column indices
  double* d_cnp = nullptr;
  size_t cn_cap = 0;
  int* d_cnc = nullptr;
  int cnc_cap = 0;
  int ycap = 0;   // columns of d_Y
  int yrows = 0;  // rows of d_Y
  double* h_H = nullptr;     // pinned (mcap+1) x mcap
  double* h_scal = nullptr;  // pinned, 4 doubles
  // half-width of the imaginary segment [-i rho, i rho] holding the
  // spectrum of the curl part of A (bound 2 sqrt(3) / sqrt(min eps min mu))
  double rho = 0.0;
  // s-step block size in use (opts.s_step, halved whenever a block's basis
  // is too ill-conditioned for the Hessenberg algebra)
  int s_eff = 0;
  // Newton-basis shifts for the next s-step cycle: Ritz values of the last
  // cycle's H in Leja order (alpha, q per step; none before the first cycle
  // of a call, which uses the Chebyshev basis)
  std::vector<double> sh_alpha, sh_q;

  void* Z = nullptr;  // 2 * zcap columns (Re, Im per solution column)
  int zcap = 0;
  // omega continuation: earlier solutions per source (2 vectors each) and
  // the residual of an extrapolated start (complex interleaved FP64)
  void* Zh = nullptr;
  int zh_cap = 0;
  // transient continuation: per source, Im z of the chain's last column and
  // its y_hat(T) (2 vectors each, storage type)
  void* TC = nullptr;
  int tc_cap = 0;
  // FP64 work block of the s-step Arnoldi under FP32 storage
  double* SB = nullptr;
  int sb_cap = 0;
  double* d_r = nullptr;

  // block (batched) form: basis slots, energy weights, Gram partials
  void* BV = nullptr;
  int bslots = 0;
  double* d_w = nullptr;       // energy weight per entry (n)
  double* d_gp = nullptr;      // Gram partials
  size_t gp_cap = 0;
  double* d_bc = nullptr;      // reduced Gram / coefficient matrices
  size_t bc_cap = 0;
  // device finish of the s-step blocks: update coefficients, per-block
  // stash of the Gram-Schmidt factors, per-block flags
  double* d_K = nullptr;
  double* d_stash = nullptr;
  size_t stash_cap = 0;
  int* d_flags = nullptr;
  int flags_cap = 0;

  // captured Arnoldi cycles (one per cycle length), replayed on `stream`
  hipStream_t cstream = nullptr;  // private capture stream (default priority)
  std::map<int, hipGraphExec_t> graphs;
  // the captured s-step cycle (device block finish) and what it was
  // captured for (Krylov dimension, block size, basis steps)
  hipGraphExec_t sstep_graph = nullptr;
  std::vector<double> sstep_key;

  // optional per-kernel-class timing with HIP events
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  double k_ms[KRY_K_CLASSES] = {};
  long long k_launch[KRY_K_CLASSES] = {};
  double k_bytes[KRY_K_CLASSES] = {};
  double k_flops[KRY_K_CLASSES] = {};
  // every launch of a class (timed or not) and its algorithmic bytes, and
  // the count of timing opportunities (one in opts.timing is timed)
  long long k_launch_all[KRY_K_CLASSES] = {};
  double k_bytes_all[KRY_K_CLASSES] = {};
  long long t_count = 0;

  // per-column record of the last kry_solve_multifreq call (single-vector path)
  struct ColRecord {
    kry_col_stats s{};
    std::vector<double> t, norm, ms;  // |y_hat(t)|_M series
  };
  std::vector<ColRecord> cols;
  // true relative residual of each Z pair after its last check (NaN: none)
  std::vector<double> zres;
  // operator applications and status of the last shifted-solve group
  long long grp_mv = 0;
  int grp_status = 0;

  std::string err;
};

namespace {

std::string g_create_err;

int fail(kry_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_create_err = msg;
  return code;
}

#define KRY_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(c, KRY_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

template <typename F>
struct Defer {
  F f;
  ~Defer() { f(); }
};

hipEvent_t take_event(kry_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Record the start event of a timed launch (no-op unless timing is on; with
// opts.timing = N > 1 only one launch in N is timed).
hipEvent_t tbeg(kry_ctx* c) {
  if (c->opts.timing <= 0) return nullptr;
  if (c->opts.timing > 1 && (c->t_count++ % c->opts.timing) != 0) return nullptr;
  hipEvent_t a = take_event(c);
  if (a) hipEventRecord(a, c->stream);
  return a;
}

void tend(kry_ctx* c, hipEvent_t a, int cls, double bytes, double flops = 0.0) {
  if (c->opts.timing <= 0) return;
  c->k_launch_all[cls] += 1;
  c->k_bytes_all[cls] += bytes;
  if (!a) return;
  hipEvent_t b = take_event(c);
  if (!b) return;
  hipEventRecord(b, c->stream);
  c->pending.push_back({cls, a, b, bytes, flops});
}

// Fold completed event pairs into the per-class totals (after a stream sync).
void tresolve(kry_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->k_ms[p.cls] += ms;
      c->k_launch[p.cls] += 1;
      c->k_bytes[p.cls] += p.bytes;
      c->k_flops[p.cls] += p.flops;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

// Start of a solver call: per-kernel timing cleared, and the s-step block
// size back at the requested one (a halving after an ill-conditioned block
// lasts for one call, so results do not depend on earlier calls).
void treset(kry_ctx* c) {
  c->s_eff = c->opts.s_step > 1 ? c->opts.s_step : 0;
  c->sh_alpha.clear();
  c->sh_q.clear();
  for (int k = 0; k < KRY_K_CLASSES; ++k) {
    c->k_ms[k] = c->k_bytes[k] = c->k_flops[k] = c->k_bytes_all[k] = 0.0;
    c->k_launch[k] = c->k_launch_all[k] = 0;
  }
  c->t_count = 0;
}

void texport(kry_ctx* c, kry_stats* st) {
  if (!st) return;
  tresolve(c);
  for (int k = 0; k < KRY_K_CLASSES; ++k) {
    st->kernel_ms[k] = c->k_ms[k];
    st->kernel_launches[k] = c->k_launch[k];
    st->kernel_bytes[k] = c->k_bytes[k];
    st->kernel_flops[k] = c->k_flops[k];
    st->kernel_launches_all[k] = c->k_launch_all[k];
    st->kernel_bytes_all[k] = c->k_bytes_all[k];
  }
}

// Algorithmic bytes: every vector entry read or written once; materials once
// per cell (inv_eps, sigma, plus the eps weight of the dots; mu adds two).
double vbytes(kry_ctx* c) { return 6.0 * c->g.N3 * c->esz; }
double mbytes(kry_ctx* c, bool stencil) {
  const double per = stencil ? (c->mats.inv_mu ? 40.0 : 24.0) : (c->mats.inv_mu ? 16.0 : 8.0);
  return per * c->g.N3;
}

void* slot(kry_ctx* c, int i) { return (char*)c->V + (size_t)i * c->ldv * c->esz; }
void* zcol(kry_ctx* c, int col) { return (char*)c->Z + (size_t)col * c->ldv * c->esz; }

void drop_graphs(kry_ctx* c) {
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  if (c->sstep_graph) hipGraphExecDestroy(c->sstep_graph);
  c->sstep_graph = nullptr;
  c->sstep_key.clear();
}

int ensure_basis(kry_ctx* c, int m) {
  const int need_extra = c->st == kry::F64 ? std::max(2, std::min(c->opts.s_step, std::max(m, c->mcap))) : 2;
  if (m <= c->mcap && c->V && need_extra <= c->vextra) return KRY_OK;
  m = std::max(m, c->mcap);
  drop_graphs(c);
  if (m + 2 > kry::kMaxCoef) return fail(c, KRY_ENOMEM, "krylov_dim too large");
  hipFree(c->V);
  hipFree(c->partials);
  hipFree(c->d_red1);
  hipFree(c->d_red2);
  hipFree(c->d_co);
  hipFree(c->d_H);
  hipHostFree(c->h_H);
  c->V = nullptr;
  c->partials = nullptr;
  c->d_red1 = c->d_red2 = c->d_co = c->d_H = c->h_H = nullptr;
  c->mcap = 0;
  // slots 0..m: basis; m+1: candidate / work vector; m+2: operator output
  // (an s-step block uses slots m+1..m+s as its work block)
  const int extra = c->st == kry::F64 ? std::max(2, std::min(c->opts.s_step, m)) : 2;
  c->vextra = 0;
  const size_t vbytes = (size_t)(m + 1 + extra) * c->ldv * c->esz;
  if (hipMalloc(&c->V, vbytes) != hipSuccess) {
    c->V = nullptr;
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate Krylov basis of " + std::to_string(vbytes) + " bytes");
  }
  const size_t nparts = (size_t)kry::cell_blocks(c->g.N3, 1);  // the most workgroups
  KRY_HIP(hipMalloc(&c->partials, sizeof(double) * nparts * (size_t)(2 * m + 4)));
  KRY_HIP(hipMalloc(&c->d_red1, sizeof(double) * (2 * m + 4)));
  KRY_HIP(hipMalloc(&c->d_red2, sizeof(double) * (2 * m + 4)));
  KRY_HIP(hipMalloc(&c->d_co, sizeof(double) * (2 * m + 4)));
  KRY_HIP(hipMalloc(&c->d_H, sizeof(double) * (size_t)(m + 1) * m));
  KRY_HIP(hipHostMalloc(&c->h_H, sizeof(double) * (size_t)(m + 1) * m, hipHostMallocDefault));
  c->mcap = m;
  c->vextra = extra;
  return KRY_OK;
}

int ensure_y(kry_ctx* c, int m, int ncol) {
  if (c->d_Y && ncol <= c->ycap && m <= c->yrows) return KRY_OK;
  hipFree(c->d_Y);
  hipFree(c->d_colmap);
  c->d_Y = nullptr;
  c->d_colmap = nullptr;
  const int cap = std::max(ncol, 8);
  KRY_HIP(hipMalloc(&c->d_Y, sizeof(double) * (size_t)std::max(m, 1) * cap));
  KRY_HIP(hipMalloc(&c->d_colmap, sizeof(int) * cap));
  c->ycap = cap;
  c->yrows = std::max(m, 1);
  return KRY_OK;
}

int ensure_z(kry_ctx* c, int ncols) {
  if (c->Z && ncols <= c->zcap) return KRY_OK;
  hipFree(c->Z);
  c->Z = nullptr;
  c->zcap = 0;
  const size_t bytes = (size_t)2 * ncols * c->ldv * c->esz;
  if (hipMalloc(&c->Z, bytes) != hipSuccess) {
    c->Z = nullptr;
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate solution workspace of " + std::to_string(bytes) + " bytes");
  }
  c->zcap = ncols;
  return KRY_OK;
}

// |x|_M^2 and <x, y_i>_M for i < cnt (y_i = slots of a contiguous array with
// stride ldv), returned on the host (synchronises the stream).
int host_dots(kry_ctx* c, const void* x, const void* Y, int cnt, std::vector<double>& out) {
  const int nparts = kry::cell_blocks(c->g.N3, c->g.cpt_d);
  KRY_HIP(kry::launch_dots(c->st, x, Y, c->ldv, cnt, c->g, c->mats, c->partials, c->stream));
  KRY_HIP(kry::launch_reduce(c->partials, nparts, cnt + 1, cnt + 1, c->d_red1, c->stream));
  out.assign(cnt + 1, 0.0);
  KRY_HIP(hipMemcpyAsync(out.data(), c->d_red1, sizeof(double) * (cnt + 1), hipMemcpyDeviceToHost,
                         c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  return KRY_OK;
}

// Arnoldi in the energy inner product (regular Krylov, equation (Arn)):
// the start vector sits unnormalised in slot 0; on return slots 0..m hold
// V_{m+1}, h_H holds H ((m+1) x m, column-major), *beta = |start|_M and
// *m_eff the steps before an exact invariant subspace (h_{j+1,j} = 0).
// Each step: w = A v_j fused with the dots of pass 1, then
// w -= V h1, dots of pass 2 (classical Gram-Schmidt twice), then
// v_{j+1} = (w - V h2) / nu.
int arnoldi_cgs2(kry_ctx* c, int m, double* beta, int* m_eff) {
  const int np_s = kry::cell_blocks(c->g.N3, c->g.cpt_s);
  const int nparts = kry::cell_blocks(c->g.N3, c->g.cpt_d);
  hipStream_t s = c->stream;
  const long long ldv = c->ldv;
  KRY_HIP(hipMemsetAsync(c->d_H, 0, sizeof(double) * (size_t)(m + 1) * m, s));
  // normalise the start vector
  KRY_HIP(kry::launch_dots(c->st, slot(c, 0), nullptr, ldv, 0, c->g, c->mats, c->partials, s));
  KRY_HIP(kry::launch_reduce(c->partials, nparts, 1, 1, c->d_red1, s));
  KRY_HIP(kry::launch_fin_start(c->d_red1, c->d_scal + 2, s));  // scal[2] = 1/beta, scal[3] = beta
  KRY_HIP(kry::launch_scale(c->st, slot(c, 0), c->d_scal + 2, slot(c, 0), c->n, s));
  void* W = slot(c, c->mcap + 1);
  for (int j = 0; j < m; ++j) {
    const int cnt = j + 1;
    const double vb = vbytes(c);
    hipEvent_t e = tbeg(c);
    KRY_HIP(kry::launch_stencil(c->st, slot(c, j), W, c->V, ldv, cnt, c->g, c->mats, c->partials, s));
    tend(c, e, KRY_K_STENCIL, vb * (cnt + 2) + mbytes(c, true));
    KRY_HIP(kry::launch_reduce(c->partials, np_s, cnt + 1, cnt + 1, c->d_red1, s));
    e = tbeg(c);
    KRY_HIP(kry::launch_update(c->st, W, c->V, ldv, cnt, c->d_red1, nullptr, W, c->g, s));
    tend(c, e, KRY_K_UPDATE, vb * (cnt + 2));
    e = tbeg(c);
    KRY_HIP(kry::launch_dots(c->st, W, c->V, ldv, cnt, c->g, c->mats, c->partials, s));
    tend(c, e, KRY_K_DOTS, vb * (cnt + 1) + mbytes(c, false));
    KRY_HIP(kry::launch_reduce(c->partials, nparts, cnt + 1, cnt + 1, c->d_red2, s));
    KRY_HIP(kry::launch_fin_step(c->d_red1, c->d_red2, j, c->d_H, m + 1, c->d_scal, s));
    e = tbeg(c);
    KRY_HIP(kry::launch_update(c->st, W, c->V, ldv, cnt, c->d_red2, c->d_scal, slot(c, j + 1), c->g, s));
    tend(c, e, KRY_K_UPDATE, vb * (cnt + 2));
  }
  KRY_HIP(hipMemcpyAsync(c->h_H, c->d_H, sizeof(double) * (size_t)(m + 1) * m, hipMemcpyDeviceToHost, s));
  KRY_HIP(hipMemcpyAsync(c->h_scal, c->d_scal, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
  KRY_HIP(hipStreamSynchronize(s));
  tresolve(c);
  *beta = c->h_scal[3];
  int me = m;
  for (int j = 0; j < m; ++j) {
    if (c->h_H[j + 1 + (size_t)j * (m + 1)] == 0.0) { me = j + 1; break; }
  }
  if (*beta == 0.0) me = 0;
  *m_eff = me;
  return KRY_OK;
}

// Arnoldi with the second Gram-Schmidt projection delayed by one step (two
// sweeps over the basis per step instead of four).  Step j applies A to
// the candidate u_j (projected once, not yet reorthogonalised or
// normalised): pass A computes x = A u_j with <x, v_i>, <u_j, v_i>, |u_j|^2
// and <u_j, x>; the small step (k_lag_fin) completes column j-1 (second
// projection of u_j and its norm), rebuilds A v_j from x through the
// Arnoldi relation A V_{j-1} = V_j Hbar_{j-1}, and its first projection;
// pass B sweeps the basis once to write v_j and the next candidate u_{j+1}.
// After m steps the last candidate is reorthogonalised and normalised.
// Same contract as arnoldi_cgs2 (start vector unnormalised in slot 0).
// Enqueue one delayed-reorthogonalisation Arnoldi cycle on stream s (no
// host synchronisation inside, so the whole cycle can be captured).
int enqueue_arnoldi_lag(kry_ctx* c, int m, hipStream_t s, bool timed) {
  const int np_s = kry::cell_blocks(c->g.N3, c->g.cpt_s);
  const int nparts = kry::cell_blocks(c->g.N3, c->g.cpt_d);
  const long long ldv = c->ldv;
  const int ldh = m + 1;
  KRY_HIP(kry::launch_fill(c->d_H, 0.0, (long long)(m + 1) * m, s));
  void* U = slot(c, c->mcap + 1);
  void* X = slot(c, c->mcap + 2);
  const double vb = vbytes(c);
  for (int j = 0; j < m; ++j) {
    const int cnt = j;
    void* uj = (j == 0) ? slot(c, 0) : U;
    hipEvent_t e = timed ? tbeg(c) : nullptr;
    KRY_HIP(kry::launch_stencil_lag(c->st, uj, X, c->V, ldv, cnt, c->g, c->mats, c->partials, s));
    tend(c, e, KRY_K_STENCIL, vb * (cnt + 2) + mbytes(c, true));
    KRY_HIP(kry::launch_reduce(c->partials, np_s, 2 * cnt + 2, 2 * cnt + 2, c->d_red1, s));
    KRY_HIP(kry::launch_lag_fin(c->d_red1, j, c->d_H, ldh, c->d_co, c->d_scal, s));
    e = timed ? tbeg(c) : nullptr;
    KRY_HIP(kry::launch_lag_update(c->st, uj, X, c->V, ldv, cnt, c->d_co, slot(c, j), U, c->g, s));
    tend(c, e, KRY_K_UPDATE, vb * (cnt + 4));
  }
  // last candidate: second projection and normalisation -> v_m
  hipEvent_t e = timed ? tbeg(c) : nullptr;
  KRY_HIP(kry::launch_dots(c->st, U, c->V, ldv, m, c->g, c->mats, c->partials, s));
  tend(c, e, KRY_K_DOTS, vb * (m + 1) + mbytes(c, false));
  KRY_HIP(kry::launch_reduce(c->partials, nparts, m + 1, m + 1, c->d_red1, s));
  KRY_HIP(kry::launch_lag_final(c->d_red1, m, c->d_H, ldh, c->d_scal, s));
  e = timed ? tbeg(c) : nullptr;
  KRY_HIP(kry::launch_update(c->st, U, c->V, ldv, m, c->d_red1, c->d_scal, slot(c, m), c->g, s));
  tend(c, e, KRY_K_UPDATE, vb * (m + 2));
  return KRY_OK;
}

// The cycle as a HIP graph: captured once per cycle length on the private
// stream, then replayed on the solver's stream.
int launch_arnoldi_graph(kry_ctx* c, int m) {
  auto it = c->graphs.find(m);
  if (it == c->graphs.end()) {
    if (!c->cstream) KRY_HIP(hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    KRY_HIP(hipStreamBeginCapture(c->cstream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_arnoldi_lag(c, m, c->cstream, false);
    const hipError_t ec = hipStreamEndCapture(c->cstream, &graph);
    if (rc) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    KRY_HIP(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    KRY_HIP(ei);
    it = c->graphs.emplace(m, exec).first;
  }
  KRY_HIP(hipGraphLaunch(it->second, c->stream));
  return KRY_OK;
}

// Arnoldi with the second Gram-Schmidt projection delayed by one step (two
// sweeps over the basis per step instead of four).  Step j applies A to
// the candidate u_j (projected once, not yet reorthogonalised or
// normalised): pass A computes x = A u_j with <x, v_i>, <u_j, v_i>, |u_j|^2
// and <u_j, x>; the small step (k_lag_fin) completes column j-1 (second
// projection of u_j and its norm), rebuilds A v_j from x through the
// Arnoldi relation A V_{j-1} = V_j Hbar_{j-1}, and its first projection;
// pass B sweeps the basis once to write v_j and the next candidate u_{j+1}.
// After m steps the last candidate is reorthogonalised and normalised.
// Same contract as arnoldi_cgs2 (start vector unnormalised in slot 0).
int arnoldi_lag(kry_ctx* c, int m, double* beta, int* m_eff) {
  hipStream_t s = c->stream;
  const int ldh = m + 1;
  int rc = (c->opts.use_graph && !c->opts.timing) ? launch_arnoldi_graph(c, m)
                                                   : enqueue_arnoldi_lag(c, m, s, true);
  if (rc) return rc;
  KRY_HIP(hipMemcpyAsync(c->h_H, c->d_H, sizeof(double) * (size_t)(m + 1) * m, hipMemcpyDeviceToHost, s));
  KRY_HIP(hipMemcpyAsync(c->h_scal, c->d_scal, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
  KRY_HIP(hipStreamSynchronize(s));
  tresolve(c);
  *beta = c->h_scal[1];
  int me = m;
  for (int j = 0; j < m; ++j) {
    if (c->h_H[j + 1 + (size_t)j * ldh] == 0.0) { me = j + 1; break; }
  }
  if (*beta == 0.0) me = 0;
  *m_eff = me;
  return KRY_OK;
}

int arnoldi_ca(kry_ctx* c, int m, double* beta, int* m_eff);

int arnoldi(kry_ctx* c, int m, double* beta, int* m_eff) {
  if (c->s_eff > 1) return arnoldi_ca(c, m, beta, m_eff);
  return c->opts.orth == 1 ? arnoldi_cgs2(c, m, beta, m_eff) : arnoldi_lag(c, m, beta, m_eff);
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Restarted multi-shift solve of (A + i w_k I) z_k = coef_k * s for all k
// at once, with s (real) in slot 0.  All shifts share one real Krylov
// sequence (a Krylov space is shift invariant); a restart must then leave
// every shift's residual on one common real vector.  FOM does that with
// v_{m+1} (Lemma 1 with a constant source: the residual is a multiple of
// v_{m+1}, the collinearity behind Corollaries 1 and 2), but restarted FOM
// can diverge on these indefinite systems.  Here the common direction is
// instead chosen per cycle as the real unit vector w in span(V_{m+1}) that
// minimises the residual of the worst shift (the "seed"): with q the left
// null vector of the seed's (m+1) x m projected matrix, the residual for a
// restart direction w is |q^H g| |w| / |q^H w|, maximised over real w by
// the top eigenvector of Re q Re q^T + Im q Im q^T (within sqrt 2 of the
// unconstrained GMRES minimum).  Every shift then solves the bordered
// Hessenberg system [Hbar_k, -w] [y_k; rho_k] = coef_k beta e_1, so its new
// residual is -rho_k V_{m+1} w.
// Z columns zre_k = 2 * zcol_k, zim_k = 2 * zcol_k + 1 accumulate V_m y_k.
// zscale (optional, per shift) multiplies the solution added to Z.  Many
// shifts whose Z columns are contiguous update Z with one tall-skinny
// product (the basis is read once, not once per group of columns).
int block_gemm(kry_ctx* c, const void* X, int M, const std::vector<double>& C, int N, void* Out,
               double alpha, int accumulate, const void* X2, int M1, int st1, int st2, int sto);

// A shift whose residual grows 100-fold above its best (the collinear
// restart can do that to shifts far from the seed) is dropped and listed in
// *diverged (its Z columns then hold garbage); the caller solves it again.
int multishift(kry_ctx* c, const std::vector<double>& omegas, std::vector<cplx> coef,
               const std::vector<int>& zcolk, double bnorm, double tol, kry_stats* st,
               double* max_res, const std::vector<double>* zscale = nullptr,
               std::vector<int>* diverged = nullptr) {
  const int nw = (int)omegas.size();
  std::vector<double> best(nw, std::numeric_limits<double>::infinity());  // smallest residual so far
  bool contiguous = 2 * nw > 16;
  for (int k = 1; k < nw && contiguous; ++k) contiguous = zcolk[k] == zcolk[0] + k;
  std::vector<double> Cz;
  const int m = c->opts.krylov_dim;
  int rc = ensure_basis(c, m);
  if (rc) return rc;
  rc = ensure_y(c, m + 1, 2 * nw + 1);
  if (rc) return rc;
  std::vector<char> active(nw, 1);
  std::vector<double> Yh((size_t)(m + 1) * (2 * nw + 1));
  std::vector<int> cmap(2 * nw);
  const int maxcyc = c->opts.max_restarts > 0 ? c->opts.max_restarts : 100000;
  double worst = 0.0;
  const int M1 = m + 1;
  std::vector<cplx> Mb((size_t)M1 * M1), g(M1), sol(M1), q(M1), Hs((size_t)m * m), rhs(m);
  std::vector<double> wt(M1);
  for (int cyc = 0; cyc < maxcyc; ++cyc) {
    double beta = 0.0;
    int me = 0;
    rc = arnoldi(c, m, &beta, &me);
    if (rc) return rc;
    if (st) { st->matvecs_stationary += m; st->cycles_stationary += 1; }
    if (me == 0) {  // zero start vector: nothing left to solve
      worst = 0.0;
      break;
    }
    const int ldh = m + 1;
    const double* H = c->h_H;
    const bool exact = me < m;  // invariant subspace: projected solve is exact
    if (!exact) {
      // seed: the active shift with the largest residual
      int k0 = -1;
      for (int k = 0; k < nw; ++k)
        if (active[k] && (k0 < 0 || std::abs(coef[k]) > std::abs(coef[k0]))) k0 = k;
      // left null vector of the seed's Hbar: (H + i w I)^H q[:m] = -h e_m, q[m] = 1
      const double hnext = H[m + (size_t)(m - 1) * ldh];
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          // (H + i w I)^H entry (i, j) = conj(H(j, i) + i w delta_ij)
          cplx v = (j <= i + 1) ? cplx(H[j + (size_t)i * ldh], 0.0) : cplx(0.0);
          if (i == j) v += cplx(0.0, omegas[k0]);
          Hs[i + (size_t)j * m] = std::conj(v);
        }
      std::fill(rhs.begin(), rhs.end(), cplx(0.0));
      rhs[m - 1] = -hnext;
      bool okq = kry::dense_solve(m, Hs.data(), rhs.data(), q.data());
      q[m] = 1.0;
      if (okq) {
        kry::best_real_direction(M1, q.data(), wt.data());
      } else {  // singular seed projection: fall back to the FOM direction
        std::fill(wt.begin(), wt.end(), 0.0);
        wt[m] = 1.0;
      }
    }
    int ncol = 0;
    worst = 0.0;
    for (int k = 0; k < nw; ++k) {
      if (!active[k]) continue;
      cplx rho = 0.0;
      if (exact) {
        std::fill(rhs.begin(), rhs.end(), cplx(0.0));
        rhs[0] = coef[k] * beta;
        if (!kry::hess_shift_solve(me, H, ldh, cplx(0.0, omegas[k]), rhs.data(), sol.data()))
          return fail(c, KRY_ENOCONV, "singular projected shifted system");
      } else {
        // bordered upper-Hessenberg system [Hbar + i w Ibar, -wt]
        for (int j = 0; j < m; ++j)
          for (int i = 0; i < M1; ++i) {
            cplx v = (i <= j + 1) ? cplx(H[i + (size_t)j * ldh], 0.0) : cplx(0.0);
            if (i == j) v += cplx(0.0, omegas[k]);
            Mb[i + (size_t)j * M1] = v;
          }
        for (int i = 0; i < M1; ++i) Mb[i + (size_t)m * M1] = -wt[i];
        std::fill(g.begin(), g.end(), cplx(0.0));
        g[0] = coef[k] * beta;
        if (!kry::hess_solve(M1, Mb.data(), g.data(), sol.data()))
          return fail(c, KRY_ENOCONV, "singular projected shifted system");
        rho = sol[m];
      }
      const double zs = zscale ? (*zscale)[k] : 1.0;
      for (int i = 0; i < me; ++i) {
        Yh[i + (size_t)(2 * ncol) * me] = zs * sol[i].real();
        Yh[i + (size_t)(2 * ncol + 1) * me] = zs * sol[i].imag();
      }
      cmap[2 * ncol] = 2 * zcolk[k];
      cmap[2 * ncol + 1] = 2 * zcolk[k] + 1;
      ++ncol;
      coef[k] = exact ? cplx(0.0) : -rho;  // new residual: coef_k * (V_{m+1} w), |V w|_M = 1
      const double res = std::abs(coef[k]) / bnorm;
      if (diverged && nw > 1 && (!std::isfinite(res) || res > 1e2 * best[k])) {
        active[k] = 0;
        coef[k] = 0.0;
        diverged->push_back(k);
        continue;
      }
      best[k] = std::min(best[k], res);
      worst = std::max(worst, res);
      if (res <= tol) active[k] = 0;
    }
    bool any_active = false;
    for (int k = 0; k < nw; ++k) any_active |= active[k] != 0;
    const bool restart = !exact && any_active && cyc + 1 < maxcyc;
    // the Z update and the next start vector s = V_{m+1} w in one sweep of
    // the basis (s overwrites slot 0: each cell is read before it is written)
    const bool fused = restart && !contiguous && 2 * ncol + 1 <= 8;
    if (fused) {
      std::vector<double> Yf((size_t)M1 * (2 * ncol + 1), 0.0);
      for (int col = 0; col < 2 * ncol; ++col)
        for (int i = 0; i < me; ++i) Yf[i + (size_t)col * M1] = Yh[i + (size_t)col * me];
      for (int i = 0; i < M1; ++i) Yf[i + (size_t)(2 * ncol) * M1] = wt[i];
      KRY_HIP(hipMemcpyAsync(c->d_Y, Yf.data(), sizeof(double) * Yf.size(), hipMemcpyHostToDevice,
                             c->stream));
      if (ncol > 0)
        KRY_HIP(hipMemcpyAsync(c->d_colmap, cmap.data(), sizeof(int) * 2 * ncol, hipMemcpyHostToDevice,
                               c->stream));
      hipEvent_t e = tbeg(c);
      KRY_HIP(kry::launch_combine(c->st, c->V, c->ldv, M1, c->d_Y, 2 * ncol + 1, c->Z, c->ldv,
                                  c->d_colmap, 1, c->g, c->stream, slot(c, 0)));
      tend(c, e, KRY_K_COMBINE, vbytes(c) * (M1 + 4.0 * ncol + 1.0));
      KRY_HIP(hipStreamSynchronize(c->stream));  // Yf is a local array
    } else if (ncol > 0 && contiguous) {
      // Z[:, 2 zcolk[0] ..] += V_me Cz, Cz (me x 2 nw, row-major; zero for
      // shifts already converged)
      Cz.assign((size_t)me * 2 * nw, 0.0);
      for (int a = 0; a < ncol; ++a) {
        const int zc = cmap[2 * a] - 2 * zcolk[0];
        for (int i = 0; i < me; ++i) {
          Cz[(size_t)i * 2 * nw + zc] = Yh[i + (size_t)(2 * a) * me];
          Cz[(size_t)i * 2 * nw + zc + 1] = Yh[i + (size_t)(2 * a + 1) * me];
        }
      }
      rc = block_gemm(c, c->V, me, Cz, 2 * nw, zcol(c, 2 * zcolk[0]), 1.0, 1, nullptr, 0, -1, -1, -1);
      if (rc) return rc;
    } else if (ncol > 0) {
      KRY_HIP(hipMemcpyAsync(c->d_Y, Yh.data(), sizeof(double) * (size_t)me * 2 * ncol,
                             hipMemcpyHostToDevice, c->stream));
      KRY_HIP(hipMemcpyAsync(c->d_colmap, cmap.data(), sizeof(int) * 2 * ncol, hipMemcpyHostToDevice,
                             c->stream));
      hipEvent_t e = tbeg(c);
      KRY_HIP(kry::launch_combine(c->st, c->V, c->ldv, me, c->d_Y, 2 * ncol, c->Z, c->ldv,
                                  c->d_colmap, 1, c->g, c->stream));
      tend(c, e, KRY_K_COMBINE, vbytes(c) * (me + 4.0 * ncol));
    }
    if (c->opts.verbose && (cyc + 1) % 20 == 0)
      std::fprintf(stderr, "[kry] shifted solve cycle %d: largest relative residual %.3e\n", cyc + 1, worst);
    if (fused) continue;  // slot 0 already holds the next start vector
    bool any = false;
    for (int k = 0; k < nw; ++k) any |= active[k] != 0;
    if (!any || exact) {
      KRY_HIP(hipStreamSynchronize(c->stream));
      break;
    }
    if (cyc + 1 == maxcyc) {
      KRY_HIP(hipStreamSynchronize(c->stream));
      *max_res = std::max(*max_res, worst);
      return KRY_ENOCONV;
    }
    // next start vector s = V_{m+1} w (overwrites slot 0 after the Z update read it)
    double* Yw = c->d_Y + (size_t)me * 2 * ncol;
    KRY_HIP(hipMemcpyAsync(Yw, wt.data(), sizeof(double) * M1, hipMemcpyHostToDevice, c->stream));
    hipEvent_t e = tbeg(c);
    KRY_HIP(kry::launch_combine(c->st, c->V, c->ldv, M1, Yw, 1, slot(c, 0), c->ldv, nullptr, 0,
                                c->g, c->stream));
    tend(c, e, KRY_K_COMBINE, vbytes(c) * (M1 + 1.0));
    // the host arrays are reused next cycle: wait for the copies
    KRY_HIP(hipStreamSynchronize(c->stream));
  }
  *max_res = std::max(*max_res, worst);
  return KRY_OK;
}

// e^{-T A} x for the vector in slot 0, by restarts in time; the result is
// left in slot 0.  Each step picks tau so that the Lemma 1 residual
// h_{m+1,m} |e_m^T u(s)| stays below rate = abstol / T on [0, tau]: the
// error of the step is then at most rate * tau in the energy norm (A is
// dissipative in that norm, so e^{-sA} does not amplify it), and the total
// stays below abstol.  Once |y_hat(t)|_M <= drop the remainder is dropped
// (e^{-(T-t)A} cannot increase it).
// With `tr`, every step's start vector is kept (checkpoint) with its start
// time, length and basis size, for a later pass that regenerates the step's
// Krylov basis from it (the gradient through the exponential).
struct ExpvTrace {
  void* ck = nullptr;  // device: checkpoint j at ck + j ldv (storage type)
  int cap = 0;
  bool keep_ck = true;  // false: record the norm series only
  std::vector<double> t0, tau, hnorm;  // per accepted step; hnorm = |H|_1 of its basis
  // every restart: its start time, |y_hat|_M there and its wall time (ms)
  std::vector<double> s_t, s_beta, s_ms;
  ExpvTrace() = default;
  ExpvTrace(const ExpvTrace&) = delete;
  ExpvTrace& operator=(const ExpvTrace&) = delete;
  ~ExpvTrace() { hipFree(ck); }
  int steps() const { return (int)t0.size(); }
  void clear() { t0.clear(), tau.clear(), hnorm.clear(), s_t.clear(), s_beta.clear(), s_ms.clear(); }
};

void* trace_ck(kry_ctx* c, const ExpvTrace* tr, int j) {
  return (char*)tr->ck + (size_t)j * c->ldv * c->esz;
}

// Copy slot 0 into checkpoint tr->steps(), growing the buffer as needed.
int trace_push(kry_ctx* c, ExpvTrace* tr) {
  const int j = tr->steps();
  if (j >= tr->cap) {
    const int cap = std::max(8, 2 * tr->cap);
    void* nb = nullptr;
    if (hipMalloc(&nb, (size_t)cap * c->ldv * c->esz) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate checkpoints of the exponential");
    }
    if (j > 0)
      KRY_HIP(hipMemcpyAsync(nb, tr->ck, (size_t)j * c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
    KRY_HIP(hipStreamSynchronize(c->stream));
    hipFree(tr->ck);
    tr->ck = nb;
    tr->cap = cap;
  }
  KRY_HIP(hipMemcpyAsync(trace_ck(c, tr, j), slot(c, 0), c->ldv * c->esz, hipMemcpyDeviceToDevice,
                         c->stream));
  return KRY_OK;
}

int expv_slot0(kry_ctx* c, double T, double abstol, double drop, kry_stats* st, double* err_est,
               ExpvTrace* tr = nullptr) {
  const int m = c->opts.krylov_dim;
  int rc = ensure_basis(c, m);
  if (rc) return rc;
  rc = ensure_y(c, m, 1);
  if (rc) return rc;
  const int ldh = m + 1;
  double t = 0.0;
  double tau_try = T;
  double err = 0.0;
  const double rate = abstol / std::max(T, 1e-300);
  const int maxsteps = c->opts.max_restarts > 0 ? c->opts.max_restarts : 100000;
  std::vector<double> u(m), Hc((size_t)m * m);
  int steps = 0;
  while (t < T) {
    if (steps >= maxsteps) { *err_est = err; return KRY_ENOCONV; }
    const double tstep = tr ? now_ms() : 0.0;
    if (tr && tr->keep_ck) {
      rc = trace_push(c, tr);
      if (rc) return rc;
    }
    double beta = 0.0;
    int me = 0;
    rc = arnoldi(c, m, &beta, &me);
    if (rc) return rc;
    ++steps;
    if (tr) {
      tr->s_t.push_back(t);
      tr->s_beta.push_back(beta);
      tr->s_ms.push_back(0.0);
    }
    if (st) { st->matvecs_transient += m; st->steps_transient += 1; }
    if (me == 0) {  // y_hat(t) = 0
      if (tr) tr->s_ms.back() = now_ms() - tstep;
      break;
    }
    if (beta <= drop) {  // remainder below the drop threshold
      KRY_HIP(hipMemsetAsync(slot(c, 0), 0, c->ldv * c->esz, c->stream));
      err += beta;
      if (tr) tr->s_ms.back() = now_ms() - tstep;
      break;
    }
    const double tmax = T - t;
    double tau = 0.0;
    double step_err = 0.0;
    if (me < m) {
      // exact invariant subspace: the projected exponential is exact
      for (int j = 0; j < me; ++j)
        for (int i = 0; i < me; ++i) Hc[i + (size_t)j * me] = -tmax * c->h_H[i + (size_t)j * ldh];
      std::vector<double> E((size_t)me * me);
      kry::expm(me, Hc.data(), E.data());
      for (int i = 0; i < me; ++i) u[i] = beta * E[i];
      tau = tmax;
    } else {
      const double hnext = c->h_H[m + (size_t)(m - 1) * ldh];
      double trial = std::min(tau_try, tmax);
      for (int attempt = 0; attempt < 60 && tau == 0.0; ++attempt) {
        tau = kry::choose_step(m, c->h_H, ldh, hnext, beta, trial, rate, 16, u.data(), &step_err);
        if (tau == 0.0) trial /= 16.0;
      }
      if (tau == 0.0) return fail(c, KRY_ENOCONV, "time step underflow in the restarted exponential");
      tau_try = (tau >= trial * (1.0 - 1e-12)) ? 2.0 * trial : 1.25 * tau;
      if (t + tau > T * (1.0 - 1e-15)) tau = tmax;
    }
    err += step_err;
    if (tr) {
      double hn = 0.0;
      for (int j = 0; j < me; ++j) {
        double col = 0.0;
        for (int i = 0; i <= std::min(j + 1, me - 1); ++i) col += std::abs(c->h_H[i + (size_t)j * ldh]);
        hn = std::max(hn, col);
      }
      tr->t0.push_back(t);
      tr->tau.push_back(tau);
      tr->hnorm.push_back(hn);
    }
    if (c->opts.verbose && steps % 20 == 0)
      std::fprintf(stderr, "[kry] exponential step %d: t = %.4g of %.4g\n", steps, t + tau, T);
    KRY_HIP(hipMemcpyAsync(c->d_Y, u.data(), sizeof(double) * me, hipMemcpyHostToDevice, c->stream));
    hipEvent_t e = tbeg(c);
    KRY_HIP(kry::launch_combine(c->st, c->V, c->ldv, me, c->d_Y, 1, slot(c, 0), c->ldv, nullptr, 0,
                                c->g, c->stream));
    tend(c, e, KRY_K_COMBINE, vbytes(c) * (me + 1.0));
    KRY_HIP(hipStreamSynchronize(c->stream));
    t += tau;
    if (tr) tr->s_ms.back() = now_ms() - tstep;
  }
  *err_est = err;
  return KRY_OK;
}

bool finite_all(const std::vector<double>& a) {
  for (double v : a)
    if (!std::isfinite(v)) return false;
  return true;
}

}  // namespace

namespace {

void api_destroy(kry_ctx* c);
int scratch_on_current_device(double** out, std::string* err);

int api_create(const kry_grid* grid, const double* eps, const double* mu, const double* sigma,
               const kry_opts* opts, kry_ctx** out) {
  kry_ctx* c = nullptr;
  if (!grid || !eps || !opts || !out) return fail(nullptr, KRY_EINVAL, "null argument");
  *out = nullptr;
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->boundary != 0)
    return fail(nullptr, KRY_EINVAL, "invalid grid");
  const long long N3 = (long long)grid->nx * grid->ny * grid->nz;
  if (N3 > (1LL << 30) / 6) return fail(nullptr, KRY_EINVAL, "grid too large");
  if (opts->storage != 0 && opts->storage != 1) return fail(nullptr, KRY_EINVAL, "invalid storage");
  if (opts->krylov_dim < 1 || opts->krylov_dim + 2 > kry::kMaxCoef)
    return fail(nullptr, KRY_EINVAL, "krylov_dim out of range");
  if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) return fail(nullptr, KRY_EINVAL, "invalid tol");
  if (opts->inner_product != 0) return fail(nullptr, KRY_EINVAL, "only the energy inner product is supported");
  if (opts->orth != 0 && opts->orth != 1) return fail(nullptr, KRY_EINVAL, "invalid orth");
  if (opts->block_width < 0 || opts->block_width > 256)
    return fail(nullptr, KRY_EINVAL, "block_width out of range");
  if (opts->block_steps < 0 || opts->block_steps > 512 || opts->block_steps_transient < 0 ||
      opts->block_steps_transient > 512)
    return fail(nullptr, KRY_EINVAL, "block steps out of range");
  std::vector<double> he(N3), hm, hs(N3, 0.0);
  if (hipMemcpy(he.data(), eps, sizeof(double) * N3, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(nullptr, KRY_EINVAL, "eps is not a readable device array");
  if (mu) {
    hm.resize(N3);
    if (hipMemcpy(hm.data(), mu, sizeof(double) * N3, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(nullptr, KRY_EINVAL, "mu is not a readable device array");
  }
  if (sigma && hipMemcpy(hs.data(), sigma, sizeof(double) * N3, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(nullptr, KRY_EINVAL, "sigma is not a readable device array");
  if (!finite_all(he) || !finite_all(hm) || !finite_all(hs))
    return fail(nullptr, KRY_EINVAL, "non-finite material value");
  double min_e = he[0], min_m = mu ? hm[0] : 1.0;
  for (long long i = 0; i < N3; ++i) {
    if (!(he[i] > 0.0)) return fail(nullptr, KRY_EINVAL, "eps must be > 0");
    if (mu && !(hm[i] > 0.0)) return fail(nullptr, KRY_EINVAL, "mu must be > 0");
    if (hs[i] < 0.0) return fail(nullptr, KRY_EINVAL, "sigma must be >= 0");
    min_e = std::min(min_e, he[i]);
    if (mu) min_m = std::min(min_m, hm[i]);
  }
  if (opts->s_step < 0 || opts->s_step > 64) return fail(nullptr, KRY_EINVAL, "s_step out of range");
  if (opts->host_blocks != 0 && opts->host_blocks != 1) return fail(nullptr, KRY_EINVAL, "invalid host_blocks");
  c = new (std::nothrow) kry_ctx();
  if (!c) return fail(nullptr, KRY_ENOMEM, "host allocation failed");
  c->g.nx = grid->nx;
  c->g.ny = grid->ny;
  c->g.nz = grid->nz;
  c->g.N3 = N3;
  c->g.cpt_s = c->g.cpt_u = c->g.cpt_d = kry::cells_per_thread(N3);
  c->n = 6 * N3;
  c->ldv = (c->n + 63) / 64 * 64;
  c->st = opts->storage == 1 ? kry::F32 : kry::F64;
  c->esz = opts->storage == 1 ? 4 : 8;
  c->opts = *opts;
  c->stream = (hipStream_t)opts->stream;
  // |curl| <= 2 sqrt(3) on the unit grid (each component is a difference of
  // two unit differences), scaled by the smallest eps and mu
  c->rho = 2.0 * std::sqrt(3.0) / std::sqrt(min_e * min_m);
  c->s_eff = opts->s_step > 1 ? opts->s_step : 0;

  // derived arrays: inv_eps, sigma (or sigma/mu), eps, [inv_mu, mu]
  const int narr = mu ? 5 : 3;
  std::vector<double> host((size_t)narr * N3);
  for (long long i = 0; i < N3; ++i) {
    host[i] = 1.0 / he[i];
    host[N3 + i] = mu ? hs[i] / hm[i] : hs[i];
    host[2 * N3 + i] = he[i];
    if (mu) {
      host[3 * N3 + i] = 1.0 / hm[i];
      host[4 * N3 + i] = hm[i];
    }
  }
  if (hipMalloc(&c->d_mat, sizeof(double) * host.size()) != hipSuccess) {
    delete c;
    return fail(nullptr, KRY_ENOMEM, "cannot allocate material arrays");
  }
  if (hipMemcpy(c->d_mat, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMalloc(&c->d_scal, sizeof(double) * 4) != hipSuccess ||
      hipHostMalloc(&c->h_scal, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess) {
    api_destroy(c);
    return fail(nullptr, KRY_EHIP, "device setup failed");
  }
  c->mats.inv_eps = c->d_mat;
  c->mats.sigma = c->d_mat + N3;
  c->mats.eps = c->d_mat + 2 * N3;
  c->mats.inv_mu = mu ? c->d_mat + 3 * N3 : nullptr;
  c->mats.mu = mu ? c->d_mat + 4 * N3 : nullptr;
  {
    // set-up of the allocation-free Arnoldi: the address of this device's
    // `scratch` (a failure here is reported by that entry point itself)
    double* scr = nullptr;
    std::string err;
    (void)scratch_on_current_device(&scr, &err);
  }
  *out = c;
  return KRY_OK;
}

void api_destroy(kry_ctx* c) {
  if (!c) return;
  hipFree(c->d_mat);
  hipFree(c->V);
  hipFree(c->partials);
  hipFree(c->d_red1);
  hipFree(c->d_red2);
  hipFree(c->d_scal);
  hipFree(c->d_co);
  hipFree(c->d_H);
  hipFree(c->d_Y);
  hipFree(c->d_colmap);
  hipFree(c->d_cnp);
  hipFree(c->d_cnc);
  hipFree(c->Z);
  hipFree(c->Zh);
  hipFree(c->TC);
  hipFree(c->d_r);
  hipFree(c->SB);
  hipFree(c->BV);
  hipFree(c->d_w);
  hipFree(c->d_gp);
  hipFree(c->d_bc);
  hipFree(c->d_K);
  hipFree(c->d_stash);
  hipFree(c->d_flags);
  drop_graphs(c);
  if (c->cstream) hipStreamDestroy(c->cstream);
  for (auto& p : c->pending) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  if (c->h_H) hipHostFree(c->h_H);
  if (c->h_scal) hipHostFree(c->h_scal);
  delete c;
}

const char* api_last_error(const kry_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int64_t api_size(const kry_ctx* c) { return c ? c->n : 0; }

int api_apply(kry_ctx* c, const double* v, double* w, int32_t ncols) {
  if (!c || !v || !w || ncols < 0) return fail(c, KRY_EINVAL, "invalid argument");
  for (int k = 0; k < ncols; ++k)
    KRY_HIP(kry::launch_stencil(kry::F64, v + (size_t)k * c->n, w + (size_t)k * c->n, nullptr, 0, 0,
                                c->g, c->mats, nullptr, c->stream));
  return KRY_OK;
}

int api_apply_f32(kry_ctx* c, const float* v, float* w, int32_t ncols) {
  if (!c || !v || !w || ncols < 0) return fail(c, KRY_EINVAL, "invalid argument");
  for (int k = 0; k < ncols; ++k)
    KRY_HIP(kry::launch_stencil(kry::F32, v + (size_t)k * c->n, w + (size_t)k * c->n, nullptr, 0, 0,
                                c->g, c->mats, nullptr, c->stream));
  return KRY_OK;
}

int api_arnoldi(kry_ctx* c, const double* v, int32_t m, void* V_out, double* H_out, double* beta_out) {
  if (!c || !v || !V_out || !H_out || !beta_out) return fail(c, KRY_EINVAL, "null argument");
  treset(c);
  if (m < 1 || m + 2 > kry::kMaxCoef) return fail(c, KRY_EINVAL, "invalid m");
  int rc = ensure_basis(c, std::max(m, c->opts.krylov_dim));
  if (rc) return rc;
  KRY_HIP(kry::launch_load_real(c->st, v, slot(c, 0), c->n, c->stream));
  double beta = 0.0;
  int me = 0;
  rc = arnoldi(c, m, &beta, &me);
  if (rc) return rc;
  std::memcpy(H_out, c->h_H, sizeof(double) * (size_t)(m + 1) * m);
  *beta_out = beta;
  for (int j = 0; j <= m; ++j)
    KRY_HIP(hipMemcpyAsync((char*)V_out + (size_t)j * c->n * c->esz, slot(c, j), c->n * c->esz,
                           hipMemcpyDeviceToDevice, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  return me;
}

int api_expv(kry_ctx* c, double t, const double* v, double* y, int32_t ncols, kry_stats* st) {
  if (!c || !v || !y || ncols < 0) return fail(c, KRY_EINVAL, "invalid argument");
  if (!(t >= 0.0) || !std::isfinite(t)) return fail(c, KRY_EINVAL, "invalid time");
  if (st) std::memset(st, 0, sizeof(*st));
  treset(c);
  const double t0 = now_ms();
  int rc = ensure_basis(c, c->opts.krylov_dim);
  if (rc) return rc;
  int status = KRY_OK;
  double worst = 0.0;
  for (int k = 0; k < ncols; ++k) {
    KRY_HIP(kry::launch_load_real(c->st, v + (size_t)k * c->n, slot(c, 0), c->n, c->stream));
    std::vector<double> d;
    rc = host_dots(c, slot(c, 0), nullptr, 0, d);
    if (rc) return rc;
    const double vn = std::sqrt(std::max(d[0], 0.0));
    double err = 0.0;
    if (t > 0.0 && vn > 0.0) {
      rc = expv_slot0(c, t, 0.5 * c->opts.tol * vn, 0.25 * c->opts.tol * vn, st, &err);
      if (rc == KRY_ENOCONV) status = KRY_ENOCONV;
      else if (rc) return rc;
    }
    worst = std::max(worst, vn > 0.0 ? err / vn : 0.0);
    KRY_HIP(kry::launch_store_real(c->st, slot(c, 0), y + (size_t)k * c->n, c->n, c->stream));
  }
  KRY_HIP(hipStreamSynchronize(c->stream));
  if (st) {
    st->max_err_estimate = worst;
    st->ms_transient = st->ms_total = now_ms() - t0;
    st->converged = status == KRY_OK;
    texport(c, st);
  }
  return status;
}

}  // namespace

namespace {

// Shifted solves for a group of columns sharing one complex source (slot
// data from b_col): z_k = (A + i w_k)^{-1} b for the listed shifts, stored
// in Z columns 2*zcolk[k] (Re) and 2*zcolk[k]+1 (Im).
int refine_shift(kry_ctx* c, const double* bcol, double w, int zk, int spare, double tol_rel,
                 double bn, kry_stats* st, double* max_res, bool correct);
int cnorm(kry_ctx* c, const double* x, double* out);

// spare >= 0: a free Z pair; once every shift reports convergence, its
// true residual b - (A + i w) z is checked, and corrected once where it
// misses the target (the residual of a shift that is not the restart seed
// is carried as a coefficient of the shared start vector, and rounding can
// open a gap between the two).  b_col must not be c->d_r when spare >= 0.
int stationary_group(kry_ctx* c, const double* b_col, const std::vector<double>& omegas,
                     const std::vector<int>& zcolk, double tol_rel, kry_stats* st, double* max_res,
                     double* bnorm_out, int spare = -1) {
  const int nw = (int)omegas.size();
  if ((int)c->zres.size() < c->zcap) c->zres.resize(c->zcap, NAN);
  for (int k = 0; k < nw; ++k) {
    KRY_HIP(hipMemsetAsync(zcol(c, 2 * zcolk[k]), 0, 2 * c->ldv * c->esz, c->stream));
    if (zcolk[k] < (int)c->zres.size()) c->zres[zcolk[k]] = NAN;
  }
  // norms of Re b and Im b
  std::vector<double> d;
  KRY_HIP(kry::launch_load_complex(c->st, b_col, 1, slot(c, 0), c->n, c->stream));
  int rc = host_dots(c, slot(c, 0), nullptr, 0, d);
  if (rc) return rc;
  const double nim2 = d[0];
  KRY_HIP(kry::launch_load_complex(c->st, b_col, 0, slot(c, 0), c->n, c->stream));
  rc = host_dots(c, slot(c, 0), nullptr, 0, d);
  if (rc) return rc;
  const double nre2 = d[0];
  const double bnorm = std::sqrt(nre2 + nim2);
  *bnorm_out = bnorm;
  if (bnorm == 0.0) return KRY_OK;
  int status = KRY_OK;
  const double tol_part = tol_rel / ((nre2 > 0 && nim2 > 0) ? std::sqrt(2.0) : 1.0);
  // shifts in groups of neighbours: at most 16, spanning at most a tenth of
  // their mean frequency (one restart direction has to serve every shift
  // of a group, which a wide band of shifts defeats)
  std::vector<int> gid(nw);
  const int ng = kry::group_shifts(nw, omegas.data(), 16, 0.1, gid.data());
  std::vector<std::vector<int>> groups(ng);
  for (int k = 0; k < nw; ++k) groups[gid[k]].push_back(k);
  std::vector<int> redo;
  auto solve = [&](const std::vector<int>& idx, bool single) -> int {
    std::vector<double> om;
    std::vector<int> zc;
    for (int k : idx) {
      om.push_back(omegas[k]);
      zc.push_back(zcolk[k]);
    }
    std::vector<int> div;
    for (int part = 0; part < 2; ++part) {
      if ((part == 0 ? nre2 : nim2) <= 0.0) continue;
      KRY_HIP(kry::launch_load_complex(c->st, b_col, part, slot(c, 0), c->n, c->stream));
      const cplx cf = part == 0 ? cplx(1.0, 0.0) : cplx(0.0, 1.0);
      const int r = multishift(c, om, std::vector<cplx>(om.size(), cf), zc, bnorm, tol_part, st,
                               max_res, nullptr, single ? nullptr : &div);
      if (r == KRY_ENOCONV) status = r;
      else if (r) return r;
    }
    for (int i : div)
      if (std::find(redo.begin(), redo.end(), idx[i]) == redo.end()) redo.push_back(idx[i]);
    return KRY_OK;
  };
  for (const auto& g : groups) {
    rc = solve(g, false);
    if (rc) return rc;
  }
  // shifts dropped by a group: again on their own, from zero
  for (int k : redo) {
    if (c->opts.verbose)
      std::fprintf(stderr, "[kry] shift omega = %.6f solved again on its own\n", omegas[k]);
    KRY_HIP(hipMemsetAsync(zcol(c, 2 * zcolk[k]), 0, 2 * c->ldv * c->esz, c->stream));
    rc = solve(std::vector<int>{k}, true);
    if (rc) return rc;
  }
  if (spare >= 0) {
    // every shift's true residual goes into the statistics; shifts of a
    // group that reported convergence are corrected where it misses
    const bool correct = status == KRY_OK;
    for (int k = 0; k < nw; ++k) {
      rc = refine_shift(c, b_col, omegas[k], zcolk[k], spare, tol_rel, bnorm, st, max_res, correct);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
    }
  }
  return status;
}

// True residual r = b - (A + i w) z_k, |r|_M / |b|_M folded into *max_res.
// With `correct`, where |r|_M misses the acceptance level: solve
// (A + i w) d = r into the spare pair, z_k += d, and take the true residual
// again (the statistics then hold the residual of the returned z, never an
// estimate); KRY_ENOCONV if it still misses.  The acceptance level is
// 2 tol_rel |b|_M, but never below what the storage type can represent:
// rounding z (and A z) to the storage precision u alone moves the residual
// by up to u (|A z|_M + w |z|_M), so the level is at least 8 times that
// (it matters for FP32 storage at tight tolerances).
// *floor receives that rounding level.
int true_residual(kry_ctx* c, const double* bcol, double w, int zk, kry_stats* st, double* rn,
                  double* floor) {
  KRY_HIP(kry::launch_stencil_cols(c->st, zcol(c, 2 * zk), slot(c, 1), c->ldv, 2, c->g, c->mats, c->stream));
  KRY_HIP(kry::launch_shift_residual(c->st, bcol, zcol(c, 2 * zk), zcol(c, 2 * zk + 1), slot(c, 1), slot(c, 2),
                                     w, c->d_r, c->n, c->stream));
  if (st) st->matvecs_stationary += 2;
  int rc = cnorm(c, c->d_r, rn);
  if (rc) return rc;
  double az2 = 0.0, z2 = 0.0;
  std::vector<double> d;
  for (int part = 0; part < 2; ++part) {
    rc = host_dots(c, slot(c, 1 + part), nullptr, 0, d);
    if (rc) return rc;
    az2 += d[0];
    rc = host_dots(c, zcol(c, 2 * zk + part), nullptr, 0, d);
    if (rc) return rc;
    z2 += d[0];
  }
  const double u = c->st == kry::F32 ? 0x1p-24 : 0x1p-53;
  *floor = u * (std::sqrt(std::max(az2, 0.0)) + w * std::sqrt(std::max(z2, 0.0)));
  return KRY_OK;
}

int refine_shift(kry_ctx* c, const double* bcol, double w, int zk, int spare, double tol_rel,
                 double bn, kry_stats* st, double* max_res, bool correct) {
  if (!c->d_r) {  // the residual vector (complex, n entries)
    if (hipMalloc(&c->d_r, sizeof(double) * 2 * c->n) != hipSuccess) {
      c->d_r = nullptr;
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate the residual vector");
    }
  }
  if (!(bn > 0.0)) return KRY_OK;
  double rn = 0.0, fl = 0.0;
  int rc = true_residual(c, bcol, w, zk, st, &rn, &fl);
  if (rc) return rc;
  if (!std::isfinite(rn) || !std::isfinite(fl)) {
    *max_res = INFINITY;
    return fail(c, KRY_ENOCONV, "non-finite shifted solution");
  }
  const double accept = std::max(2.0 * tol_rel * bn, 8.0 * fl);
  if (zk < (int)c->zres.size()) c->zres[zk] = rn / bn;
  if (!correct || !(rn > accept)) {
    *max_res = std::max(*max_res, rn / bn);
    return KRY_OK;
  }
  if (c->opts.verbose)
    std::fprintf(stderr, "[kry] shift omega = %.6f: true relative residual %.3e, corrected\n", w, rn / bn);
  double lr = 0.0, rn2 = 0.0;
  const int status = stationary_group(c, c->d_r, std::vector<double>{w}, std::vector<int>{spare},
                                      tol_rel * bn / rn, st, &lr, &rn2, -1);
  if (status && status != KRY_ENOCONV) return status;
  const double I2[4] = {1.0, 0.0, 0.0, 1.0};
  KRY_HIP(hipMemcpyAsync(c->d_Y, I2, sizeof(I2), hipMemcpyHostToDevice, c->stream));
  KRY_HIP(kry::launch_combine(c->st, zcol(c, 2 * spare), c->ldv, 2, c->d_Y, 2, zcol(c, 2 * zk), c->ldv, nullptr,
                              1, c->g, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  rc = true_residual(c, bcol, w, zk, st, &rn, &fl);
  if (rc) return rc;
  if (zk < (int)c->zres.size()) c->zres[zk] = rn / bn;
  *max_res = std::max(*max_res, std::isfinite(rn) ? rn / bn : INFINITY);
  if (!std::isfinite(rn)) return fail(c, KRY_ENOCONV, "non-finite shifted solution");
  if (c->opts.verbose)
    std::fprintf(stderr, "[kry] shift omega = %.6f: true relative residual %.3e after the correction\n", w,
                 rn / bn);
  return rn > std::max(2.0 * tol_rel * bn, 8.0 * fl) ? KRY_ENOCONV : KRY_OK;
}

// |x|_M for a complex interleaved FP64 device vector x (slot 0 as staging).
int cnorm(kry_ctx* c, const double* x, double* out) {
  double s2 = 0.0;
  std::vector<double> d;
  for (int part = 0; part < 2; ++part) {
    KRY_HIP(kry::launch_load_complex(c->st, x, part, slot(c, 0), c->n, c->stream));
    int rc = host_dots(c, slot(c, 0), nullptr, 0, d);
    if (rc) return rc;
    s2 += d[0];
  }
  *out = std::sqrt(std::max(s2, 0.0));
  return KRY_OK;
}

void* zhist(kry_ctx* c, int i) { return (char*)c->Zh + (size_t)i * c->ldv * c->esz; }

int ensure_cont(kry_ctx* c, int nvec) {
  if (!c->Zh || nvec > c->zh_cap) {
    hipFree(c->Zh);
    c->Zh = nullptr;
    c->zh_cap = 0;
    const size_t bytes = (size_t)nvec * c->ldv * c->esz;
    if (hipMalloc(&c->Zh, bytes) != hipSuccess) {
      c->Zh = nullptr;
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate continuation workspace of " + std::to_string(bytes) + " bytes");
    }
    c->zh_cap = nvec;
  }
  if (!c->d_r) KRY_HIP(hipMalloc(&c->d_r, sizeof(double) * 2 * c->n));
  return KRY_OK;
}

// Shifted solve of one column with a start from earlier frequencies: z0 =
// sum_a L_a z(omega_a) (Lagrange extrapolation in omega from the q stored
// solutions hist_a at omegas om_a), r = b - (A + i w) z0, then
// (A + i w) d = r to the residual target tol_s |b|_M, z = z0 + d in Z
// pair zk (columns 2 zk, 2 zk + 1); Z pair zs is scratch.  *bnorm receives
// |b|_M, *res the final relative residual.
int stationary_from(kry_ctx* c, const double* bcol, double w, const std::vector<double>& om_a,
                    const std::vector<int>& hist_a, double tol_s, kry_stats* st, double* res,
                    double* bnorm, int zk = 0, int zs = 1) {
  const int q = (int)om_a.size();
  // z0 into Z columns 2, 3
  std::vector<double> Y((size_t)4 * q, 0.0);  // (2q) x 2, column-major; inputs ordered as hist slots
  // the history vectors of one source are contiguous: inputs 2 h, 2 h + 1
  int hmin = hist_a[0];
  for (int a = 0; a < q; ++a) hmin = std::min(hmin, hist_a[a]);
  int hmax = hmin;
  for (int a = 0; a < q; ++a) hmax = std::max(hmax, hist_a[a]);
  const int m = 2 * (hmax - hmin + 1);
  Y.assign((size_t)2 * m, 0.0);
  for (int a = 0; a < q; ++a) {
    double L = 1.0;
    for (int b2 = 0; b2 < q; ++b2)
      if (b2 != a) L *= (w - om_a[b2]) / (om_a[a] - om_a[b2]);
    const int i = 2 * (hist_a[a] - hmin);
    Y[i] = L;              // Re z0 from Re z_a
    Y[(i + 1) + m] = L;    // Im z0 from Im z_a
  }
  int rc = ensure_y(c, m, 2);
  if (rc) return rc;
  KRY_HIP(hipMemcpyAsync(c->d_Y, Y.data(), sizeof(double) * 2 * m, hipMemcpyHostToDevice, c->stream));
  KRY_HIP(kry::launch_combine(c->st, zhist(c, 2 * hmin), c->ldv, m, c->d_Y, 2, zcol(c, 2 * zs), c->ldv,
                              nullptr, 0, c->g, c->stream));
  // r = b - (A + i w) z0 (A z0 staged in basis slots 1, 2)
  KRY_HIP(kry::launch_stencil_cols(c->st, zcol(c, 2 * zs), slot(c, 1), c->ldv, 2, c->g, c->mats, c->stream));
  KRY_HIP(kry::launch_shift_residual(c->st, bcol, zcol(c, 2 * zs), zcol(c, 2 * zs + 1), slot(c, 1), slot(c, 2), w,
                                     c->d_r, c->n, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));  // Y is reused below
  if (st) st->matvecs_stationary += 2;
  double bn = 0.0, rn = 0.0;
  rc = cnorm(c, bcol, &bn);
  if (rc) return rc;
  rc = cnorm(c, c->d_r, &rn);
  if (rc) return rc;
  *bnorm = bn;
  *res = bn > 0.0 ? rn / bn : 0.0;
  if (bn == 0.0) {
    KRY_HIP(hipMemsetAsync(zcol(c, 2 * zk), 0, 2 * c->ldv * c->esz, c->stream));
    *res = 0.0;
    return KRY_OK;
  }
  if (!(rn > tol_s * bn)) {  // the extrapolation already meets the target
    KRY_HIP(hipMemcpyAsync(zcol(c, 2 * zk), zcol(c, 2 * zs), 2 * c->ldv * c->esz, hipMemcpyDeviceToDevice,
                           c->stream));
    return KRY_OK;
  }
  double lr = 0.0, rn2 = 0.0;
  const int status = stationary_group(c, c->d_r, std::vector<double>{w}, std::vector<int>{zk},
                                      tol_s * bn / rn, st, &lr, &rn2, -1);
  if (status && status != KRY_ENOCONV) return status;
  *res = lr * rn / bn;
  // z = z0 + d
  const double I2[4] = {1.0, 0.0, 0.0, 1.0};
  KRY_HIP(hipMemcpyAsync(c->d_Y, I2, sizeof(I2), hipMemcpyHostToDevice, c->stream));
  KRY_HIP(kry::launch_combine(c->st, zcol(c, 2 * zs), c->ldv, 2, c->d_Y, 2, zcol(c, 2 * zk), c->ldv, nullptr, 1,
                              c->g, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  return status;
}

int check_multifreq_args(kry_ctx* c, const double* omegas, int n_omega, int n_src, const double* b) {
  if (!c) return KRY_EINVAL;
  if (!omegas || !b || n_omega < 1 || n_src < 1) return fail(c, KRY_EINVAL, "invalid argument");
  for (int k = 0; k < n_omega; ++k)
    if (!std::isfinite(omegas[k]) || omegas[k] < 0.0) return fail(c, KRY_EINVAL, "invalid omega");
  return KRY_OK;
}

// Runs the shifted solves for every output column; calls `each(col, omega)`
// once the Z columns of a group are ready.  Groups: one per source when the
// sources are shared by all omegas, one per column otherwise.
template <typename F>
int for_each_group(kry_ctx* c, const double* omegas, int n_omega, int n_src, const double* b,
                   int b_per_omega, double tol_s, kry_stats* st, double* max_res, F each) {
  int status = KRY_OK;
  {
    int rc0 = ensure_basis(c, c->opts.krylov_dim);
    if (rc0) return rc0;
  }
  if (!b_per_omega) {
    int rc = ensure_z(c, n_omega + 1);  // pair n_omega: refinement scratch
    if (rc) return rc;
    std::vector<double> om(omegas, omegas + n_omega);
    std::vector<int> zc(n_omega);
    for (int k = 0; k < n_omega; ++k) zc[k] = k;
    for (int s = 0; s < n_src; ++s) {
      double bn = 0.0;
      const long long mv0 = st ? st->matvecs_stationary : 0;
      rc = stationary_group(c, b + (size_t)s * 2 * c->n, om, zc, tol_s, st, max_res, &bn, n_omega);
      c->grp_mv = (st ? st->matvecs_stationary : 0) - mv0;
      c->grp_status = rc;
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      for (int k = 0; k < n_omega; ++k) {
        rc = each(k * n_src + s, omegas[k], k, bn);
        if (rc == KRY_ENOCONV) status = rc;
        else if (rc) return rc;
      }
    }
  } else {
    // per-frequency sources; with omega continuation, up to kQ earlier
    // solutions of each source are kept (ring of kQ vector pairs)
    constexpr int kQ = 3;
    const bool cont = c->opts.omega_continuation && n_omega > 1;
    int rc = ensure_z(c, 2);  // pair 0: z; pair 1: continuation start, refinement scratch
    if (rc) return rc;
    if (cont) {
      rc = ensure_cont(c, 2 * kQ * n_src);
      if (rc) return rc;
    }
    for (int k = 0; k < n_omega; ++k) {
      for (int s = 0; s < n_src; ++s) {
        const int col = k * n_src + s;
        const double* bcol = b + (size_t)col * 2 * c->n;
        double bn = 0.0;
        int q = cont ? std::min(k, kQ) : 0;
        // extrapolation nodes must be distinct frequencies
        for (int a = k - q; a < k && q > 0; ++a)
          for (int b2 = a + 1; b2 <= k; ++b2)
            if (std::abs(omegas[a] - omegas[b2]) <= 1e-12 * std::max(std::abs(omegas[b2]), 1.0)) q = 0;
        const long long mv0 = st ? st->matvecs_stationary : 0;
        if (q == 0) {
          rc = stationary_group(c, bcol, std::vector<double>{omegas[k]}, std::vector<int>{0}, tol_s,
                                st, max_res, &bn, 1);
        } else {
          std::vector<double> om_a;
          std::vector<int> hist_a;
          for (int kk = k - q; kk < k; ++kk) {
            om_a.push_back(omegas[kk]);
            hist_a.push_back(s * kQ + kk % kQ);
          }
          double res = 0.0;
          rc = stationary_from(c, bcol, omegas[k], om_a, hist_a, tol_s, st, &res, &bn);
          *max_res = std::max(*max_res, res);
          if (rc == KRY_OK || rc == KRY_ENOCONV) {
            const int r2 = refine_shift(c, bcol, omegas[k], 0, 1, tol_s, bn, st, max_res, rc == KRY_OK);
            if (r2 != KRY_OK) rc = r2;
          }
        }
        c->grp_mv = (st ? st->matvecs_stationary : 0) - mv0;
        c->grp_status = rc;
        if (rc == KRY_ENOCONV) status = rc;
        else if (rc) return rc;
        rc = each(col, omegas[k], 0, bn);
        if (rc == KRY_ENOCONV) status = rc;
        else if (rc) return rc;
        if (cont)  // keep z (Z columns 0, 1) for the next frequencies
          KRY_HIP(hipMemcpyAsync(zhist(c, 2 * (s * kQ + k % kQ)), zcol(c, 0), 2 * c->ldv * c->esz,
                                 hipMemcpyDeviceToDevice, c->stream));
      }
    }
  }
  return status;
}

}  // namespace


// ---------------------------------------------------------------------------
// Block (batched) form.  Several columns share one real block Krylov space
// K(A, [X]) (Corollaries 1 and 2: the space does not depend on the time
// factor of the source; a Krylov space is also shift invariant, so columns
// with different omega can share it).  Block Gram-Schmidt runs as
// tall-skinny FP64 matrix-core products (V^T M W and W - V C), with
// rank-revealing Cholesky QR (twice) for each new block.

namespace {

void* bslot(kry_ctx* c, int i) { return (char*)c->BV + (size_t)i * c->ldv * c->esz; }

int ensure_sblock(kry_ctx* c, int nvec) {
  if (c->SB && nvec <= c->sb_cap) return KRY_OK;
  hipFree(c->SB);
  c->SB = nullptr;
  c->sb_cap = 0;
  const size_t bytes = (size_t)nvec * c->ldv * sizeof(double);
  if (hipMalloc(&c->SB, bytes) != hipSuccess) {
    c->SB = nullptr;
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate s-step block of " + std::to_string(bytes) + " bytes");
  }
  c->sb_cap = nvec;
  return KRY_OK;
}

int ensure_weights(kry_ctx* c) {
  if (!c->d_w) {
    KRY_HIP(hipMalloc(&c->d_w, sizeof(double) * c->ldv));
    KRY_HIP(kry::launch_weights(c->mats.eps, c->mats.mu, c->d_w, c->g.N3, c->stream));
  }
  return KRY_OK;
}

int ensure_block(kry_ctx* c, int slots) {
  int rc = ensure_weights(c);
  if (rc) return rc;
  if (slots > c->bslots || !c->BV) {
    hipFree(c->BV);
    c->BV = nullptr;
    c->bslots = 0;
    const size_t bytes = (size_t)slots * c->ldv * c->esz;
    if (hipMalloc(&c->BV, bytes) != hipSuccess) {
      c->BV = nullptr;
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate block basis of " + std::to_string(bytes) + " bytes");
    }
    c->bslots = slots;
  }
  return KRY_OK;
}

int ensure_gp(kry_ctx* c, size_t doubles, size_t bc) {
  if (doubles > c->gp_cap || bc > c->bc_cap) drop_graphs(c);  // captured launches hold the old buffers
  if (doubles > c->gp_cap) {
    hipFree(c->d_gp);
    c->d_gp = nullptr;
    KRY_HIP(hipMalloc(&c->d_gp, sizeof(double) * doubles));
    c->gp_cap = doubles;
  }
  if (bc > c->bc_cap) {
    hipFree(c->d_bc);
    c->d_bc = nullptr;
    KRY_HIP(hipMalloc(&c->d_bc, sizeof(double) * bc));
    c->bc_cap = bc;
  }
  return KRY_OK;
}

// C (M x N, row-major, host) = X^T M Y for block columns X[:M], Y[:N]
// (device pointers to the first column; stride ldv).  Synchronises.
// With X2 != nullptr, X is two segments (columns k >= M1 at X2).
// Bytes of one vector of storage type st (-1: the context's).
double vbytes_of(kry_ctx* c, int st) {
  const int t = st < 0 ? (int)c->st : st;
  return 6.0 * c->g.N3 * (t == kry::F64 ? 8.0 : 4.0);
}

// st1: element type of X's first segment, st2 of X2 and Y (-1: the
// context's storage type).
int block_gram_host(kry_ctx* c, const void* X, int M, const void* Y, int N, std::vector<double>& C,
                    const void* X2 = nullptr, int M1 = 0, int st1 = -1, int st2 = -1) {
  const int ns = kry::gram_splits(c->n, M, N);
  int rc = ensure_gp(c, (size_t)ns * M * N, (size_t)M * N);
  if (rc) return rc;
  const kry::Storage s1 = st1 < 0 ? c->st : (kry::Storage)st1;
  hipEvent_t e = tbeg(c);
  KRY_HIP(kry::launch_gram(s1, X, M, Y, N, c->ldv, c->d_w, c->n, c->d_gp, ns, c->stream, X2, M1, st2));
  // algorithmic bytes: every distinct column once (Y may be part of X)
  const bool y_in_x = (X2 && Y == X2 && N == M - M1) || (!X2 && Y == X && N <= M);
  const int seg1 = X2 ? M1 : M;
  const double xb = vbytes_of(c, s1) * seg1 + vbytes_of(c, st2 < 0 ? s1 : st2) * (M - seg1);
  tend(c, e, KRY_K_GRAM, xb + (y_in_x ? 0.0 : vbytes_of(c, st2 < 0 ? s1 : st2) * N) + 8.0 * c->n,
       2.0 * c->n * M * N);
  KRY_HIP(kry::launch_reduce(c->d_gp, ns, M * N, M * N, c->d_bc, c->stream));
  C.resize((size_t)M * N);
  KRY_HIP(hipMemcpyAsync(C.data(), c->d_bc, sizeof(double) * M * N, hipMemcpyDeviceToHost, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  return KRY_OK;
}

// Out[:N] (=|+=) alpha X[:M] C with C (M x N row-major) from the host.
// X in one or two segments as for block_gram_host.
// st1, st2, sto: element types of X's first segment, of X2 and of Out (-1:
// the context's storage type).
int block_gemm(kry_ctx* c, const void* X, int M, const std::vector<double>& C, int N, void* Out,
               double alpha, int accumulate, const void* X2 = nullptr, int M1 = 0, int st1 = -1,
               int st2 = -1, int sto = -1) {
  int rc = ensure_gp(c, 0, (size_t)M * N);
  if (rc) return rc;
  const kry::Storage s1 = st1 < 0 ? c->st : (kry::Storage)st1;
  KRY_HIP(hipMemcpyAsync(c->d_bc, C.data(), sizeof(double) * M * N, hipMemcpyHostToDevice, c->stream));
  hipEvent_t e = tbeg(c);
  KRY_HIP(kry::launch_gemm_nn(s1, X, M, c->d_bc, N, Out, c->ldv, c->n, alpha, accumulate, c->stream,
                              X2, M1, st2, sto));
  const int seg1 = X2 ? M1 : M;
  const double xb = vbytes_of(c, s1) * seg1 + vbytes_of(c, st2 < 0 ? s1 : st2) * (M - seg1);
  tend(c, e, KRY_K_GEMM, xb + vbytes_of(c, sto < 0 ? s1 : sto) * (accumulate ? 2.0 : 1.0) * N,
       2.0 * c->n * M * N);
  // the host array may be reused by the caller right after
  KRY_HIP(hipStreamSynchronize(c->stream));
  return KRY_OK;
}

// s-step Arnoldi (same contract as arnoldi_cgs2: start vector unnormalised
// in slot 0; slots 0..m and h_H hold V_{m+1} and Hbar on return).  Each
// block of s steps first applies the operator s times to build a Chebyshev
// basis on the segment c + [-i rho, i rho] (rho bounds the imaginary extent
// of the curl part; the centre c is 0, see below): t_0 = v_j0,
// t_1 = (A - c) t_0 / rho, t_{k+1} = 2 (A - c) t_k / rho + t_{k-1}, so that
// A [t_0..t_{s-1}] = rho [t_0..t_s] Tm + c [t_0..t_{s-1}] with Tm[1][0] = 1,
// Tm[k+1][k] = 1/2, Tm[k-1][k] = -1/2.  The block is then orthogonalised
// against V_0..j0 by block classical Gram-Schmidt twice with a Cholesky QR
// per pass, all as tall-skinny products on the matrix cores: each pass is
// one Gram product [V, S]^T M S (the projected Gram matrix follows by
// Pythagoras) and one update (S - V C) R^{-1}, so a block of s steps costs
// two sweeps over the basis instead of two per step.  With
// [t_0..t_s] = V_ext Rhat (Rhat from the projection coefficients and the
// Cholesky factors), the new Hessenberg columns are exact algebra:
//   Hbar[:, j0:j0+s] = (rho Rhat Tm + c Rhat[:, :s] - [Hbar_{j0} Rtop; 0]) Rs^{-1},
// where Rtop and Rs are the rows of Rhat[:, :s] for V_0..j0-1 and for
// v_j0..v_{j0+s-1}.  A block whose projected Gram matrix loses rank (an
// invariant subspace, or too ill-conditioned a basis) sends the cycle to
// the delayed Arnoldi from the same normalised start vector.
const std::vector<double>& stack_coef(int M, int s, const std::vector<double>& C,
                                      const std::vector<double>& Rinv, std::vector<double>& K) {
  K.resize((size_t)(M + s) * s);
  kry::stack_coef(M, s, C.data(), Rinv.data(), K.data());
  return K;
}

int arnoldi_ca_host(kry_ctx* c, int m, double* beta, int* m_eff) {
  const int s = c->s_eff;
  // largest accepted condition estimate |R|_F |R^-1|_F of a block's
  // triangular factor: rounding of the stored block reaches Hbar amplified
  // by it, and the block is always FP64 (1e-16 * 1e6)
  const double cond_max = 1e6;
  // one pass (the Gram matrix of the projected block by Pythagoras) leaves
  // a loss of orthogonality of order u * cond(R1)^2; the second pass is
  // skipped when the column-scaled estimate of cond(R1) puts that below
  // 1e-11 (u = 1.1e-16)
  const double one_pass_max = 300.0;
  // ... and when no column lost all but 1e-6 of its squared norm to the
  // projection (the Pythagorean Gram matrix keeps ~10 digits there)
  const double one_pass_left = 1e-6;
  const int ldh = m + 1;
  hipStream_t st = c->stream;
  int rc = ensure_weights(c);
  if (rc) return rc;
  // the work block: FP64 storage keeps it in the basis slots (S right after
  // v_j0, Tb after the basis); FP32 storage keeps an FP64 copy of v_j0, S
  // and Tb apart, and only the final orthonormal block is rounded to FP32
  const bool wide = c->st == kry::F32;
  if (wide && m > 112) {  // the mixed-type Gram product keeps [V, S] in one row block
    double b1 = 0.0;
    const int r = arnoldi_lag(c, m, &b1, m_eff);
    *beta = b1;
    return r;
  }
  if (wide) {
    rc = ensure_sblock(c, 2 * s + 1);
    if (rc) return rc;
  }
  const int f64 = (int)kry::F64;
  std::vector<double> d;
  rc = host_dots(c, slot(c, 0), nullptr, 0, d);
  if (rc) return rc;
  double* H = c->h_H;
  std::fill(H, H + (size_t)(m + 1) * m, 0.0);
  const double b0 = std::sqrt(std::max(d[0], 0.0));
  if (!(b0 > 0.0)) {
    *beta = 0.0;
    *m_eff = 0;
    return KRY_OK;
  }
  // v_0 = start / b0 (d_red1[0] still holds |start|^2)
  KRY_HIP(kry::launch_fin_start(c->d_red1, c->d_scal + 2, st));
  KRY_HIP(kry::launch_scale(c->st, slot(c, 0), c->d_scal + 2, slot(c, 0), c->n, st));
  // basis recurrence t_{k+1} = (A t_k - alpha_k t_k + q_k t_{k-1}) / sig_k:
  // Newton steps on the Leja-ordered Ritz values of the previous cycle when
  // there are s of them, else the Chebyshev basis on [-i rho, i rho]
  // (centre 0: the damping is confined to the absorbing layer, so most of
  // a field's spectral weight sits at Re = 0)
  const double rho = c->rho;
  const bool newton = (int)c->sh_alpha.size() >= s;
  // block size of this cycle: the Chebyshev basis (before any Ritz values)
  // is kept to blocks of at most 16, the Newton basis takes s
  const int bs = newton ? s : std::min(s, 16);
  std::vector<double> al(bs, 0.0), qq(bs, 0.0), sg(bs, 0.0);
  for (int k = 0; k < bs; ++k) {
    if (newton) {
      al[k] = c->sh_alpha[k];
      qq[k] = c->sh_q[k];
      sg[k] = rho;
    } else {  // t_1 = A t_0 / rho, t_{k+1} = 2 A t_k / rho + t_{k-1}
      sg[k] = k == 0 ? rho : 0.5 * rho;
      qq[k] = k == 0 ? 0.0 : 0.5 * rho;
    }
  }
  auto sb = [&](int i) { return (void*)((char*)c->SB + (size_t)i * c->ldv * sizeof(double)); };
  void* Tb0 = wide ? sb(s + 1) : slot(c, c->mcap + 1);
  const double mb_axpby = mbytes(c, true) - 8.0 * c->g.N3;
  const double vb64 = vbytes_of(c, f64);
  std::vector<double> C1, C2, G, P, R1, R2, Ri, ref, K;
  for (int j0 = 0; j0 < m; j0 += bs) {
    const int ss = std::min(bs, m - j0);
    const int M = j0 + 1;
    // the update kernel for these shapes reads all its entries of every
    // input row before writing them, so FP64 storage can update S in place
    const bool inplace = !wide && ((ss <= 16 && M + ss <= 256) || (ss <= 32 && M + ss <= 128));
    // t_0 (FP64), then the basis block t_1..t_ss into S
    void* t0 = slot(c, j0);
    void* S = slot(c, j0 + 1);
    if (wide) {
      KRY_HIP(kry::launch_store_real(c->st, slot(c, j0), (double*)sb(0), c->n, st));
      t0 = sb(0);
      S = sb(1);
    }
    auto tk = [&](int k) { return k == 0 ? t0 : (void*)((char*)S + (size_t)(k - 1) * c->ldv * 8); };
    std::vector<double> Tm((size_t)(ss + 1) * ss, 0.0);  // A t_k = [t_0..t_ss] Tm[:, k]
    for (int k = 0; k < ss; ++k) {
      const bool prev = k > 0 && qq[k] != 0.0;
      hipEvent_t e = tbeg(c);
      KRY_HIP(kry::launch_stencil_axpby(kry::F64, tk(k), prev ? tk(k - 1) : nullptr, tk(k + 1),
                                        1.0 / sg[k], -al[k] / sg[k], prev ? qq[k] / sg[k] : 0.0,
                                        c->g, c->mats, st));
      tend(c, e, KRY_K_STENCIL, vb64 * (prev ? 3.0 : 2.0) + mb_axpby);
      Tm[(size_t)(k + 1) * ss + k] = sg[k];
      Tm[(size_t)k * ss + k] = al[k];
      if (prev) Tm[(size_t)(k - 1) * ss + k] = -qq[k];
    }
    R1.resize((size_t)ss * ss);
    R2.resize((size_t)ss * ss);
    Ri.resize((size_t)ss * ss);
    // pass 1: one Gram product [V, S]^T M S gives C1 = V^T M S and S^T M S,
    // so the projected Gram matrix is S^T M S - C1^T C1 (Pythagoras; V is
    // M-orthonormal); then Tb = (S - V C1) R1^{-1} in one product
    rc = block_gram_host(c, slot(c, 0), M + ss, S, ss, P, S, M, -1, f64);
    if (rc) return rc;
    C1.assign(P.begin(), P.begin() + (size_t)M * ss);
    G.resize((size_t)ss * ss);
    ref.resize(ss);
    kry::proj_gram(M, ss, P.data(), G.data(), ref.data());
    const std::vector<double> nrm2 = ref;  // squared column norms of S
    // column-scaled condition estimate |R|_F |R^-1|_F of an upper factor
    auto cond_est = [&](const std::vector<double>& R) {
      std::vector<double> Rs((size_t)ss * ss, 0.0), RI((size_t)ss * ss);
      for (int a = 0; a < ss; ++a)
        for (int k = a; k < ss; ++k)
          Rs[(size_t)a * ss + k] = R[(size_t)a * ss + k] / std::sqrt(std::max(nrm2[k], 1e-300));
      kry::inv_upper(ss, Rs.data(), RI.data());
      double f1 = 0.0, f2 = 0.0;
      for (size_t i = 0; i < Rs.size(); ++i) f1 += Rs[i] * Rs[i], f2 += RI[i] * RI[i];
      return std::sqrt(f1 * f2);
    };
    // the smallest share of a column's squared norm left after the
    // projection: the projected Gram matrix comes from a difference, so a
    // block mostly inside the basis (a nearly invariant space) loses digits
    // there, and one pass is not enough however well conditioned R1 is
    double left = 1.0;
    for (int k = 0; k < ss; ++k) left = std::min(left, G[(size_t)k * ss + k] / std::max(nrm2[k], 1e-300));
    bool ok = kry::chol_upper(ss, G.data(), ref.data(), 1e-10, R1.data());
    // a well-conditioned block is final after one pass: written straight
    // into the basis slots in the storage type
    const bool one = ok && (inplace || wide) && left >= one_pass_left && cond_est(R1) <= one_pass_max;
    void* Tb = inplace ? S : Tb0;
    if (ok) {
      kry::inv_upper(ss, R1.data(), Ri.data());
      rc = block_gemm(c, slot(c, 0), M + ss, stack_coef(M, ss, C1, Ri, K), ss,
                      one ? slot(c, j0 + 1) : Tb, 1.0, 0, S, M, -1, f64, one ? -1 : f64);
      if (rc) return rc;
    } else {
      // cancellation in the projected Gram matrix: project explicitly
      rc = block_gemm(c, slot(c, 0), M, C1, ss, S, -1.0, 1, nullptr, 0, -1, -1, f64);
      if (rc) return rc;
      rc = block_gram_host(c, S, ss, S, ss, G, nullptr, 0, f64, f64);
      if (rc) return rc;
      ok = kry::chol_upper(ss, G.data(), ref.data(), 1e-10, R1.data());
      if (ok) {
        kry::inv_upper(ss, R1.data(), Ri.data());
        rc = block_gemm(c, S, ss, Ri, ss, Tb, 1.0, 0, nullptr, 0, f64, f64, f64);
        if (rc) return rc;
      }
    }
    if (ok && one) {
      C2.assign((size_t)M * ss, 0.0);
      std::fill(R2.begin(), R2.end(), 0.0);
      for (int a = 0; a < ss; ++a) R2[(size_t)a * ss + a] = 1.0;
    } else if (ok) {
      // pass 2, the same on Tb
      rc = block_gram_host(c, slot(c, 0), M + ss, Tb, ss, P, Tb, M, -1, f64);
      if (rc) return rc;
      C2.assign(P.begin(), P.begin() + (size_t)M * ss);
      G.resize((size_t)ss * ss);
      ref.resize(ss);
      kry::proj_gram(M, ss, P.data(), G.data(), ref.data());
      std::fill(ref.begin(), ref.end(), 1.0);
      ok = kry::chol_upper(ss, G.data(), ref.data(), 1e-8, R2.data());
    }
    bool illc = false;
    if (ok && !one) {  // condition estimate of R = R2 R1 with unit columns of S
      std::vector<double> R((size_t)ss * ss, 0.0);
      for (int a = 0; a < ss; ++a)
        for (int k = a; k < ss; ++k) {
          double v = 0.0;
          for (int l = a; l <= k; ++l) v += R2[(size_t)a * ss + l] * R1[(size_t)l * ss + k];
          R[(size_t)a * ss + k] = v;
        }
      illc = !(cond_est(R) <= cond_max);
    }
    if (!ok || illc) {
      // dependent or ill-conditioned block: redo the cycle with one step per
      // sweep; an ill-conditioned basis also halves s from here on
      if (illc) {
        c->s_eff = bs / 2 >= 2 ? bs / 2 : 0;
        if (c->opts.verbose)
          std::fprintf(stderr, "[kry] s-step basis ill-conditioned at s = %d: s = %d from now on\n", bs,
                       c->s_eff);
      }
      double b1 = 0.0;
      rc = arnoldi_lag(c, m, &b1, m_eff);
      *beta = b0 * b1;
      return rc;
    }
    // Q = (Tb - V C2) R2^{-1} into the basis slots j0+1..j0+ss (storage type)
    if (!one) {
      kry::inv_upper(ss, R2.data(), Ri.data());
      rc = block_gemm(c, slot(c, 0), M + ss, stack_coef(M, ss, C2, Ri, K), ss, slot(c, j0 + 1), 1.0, 0,
                      Tb, M, -1, f64, -1);
      if (rc) return rc;
    }
    kry::sstep_hessenberg_tm(j0, ss, Tm.data(), C1.data(), C2.data(), R1.data(), R2.data(), H, ldh);
  }
  tresolve(c);
  *beta = b0;
  *m_eff = m;
  // shifts for the later cycles of this call: Ritz values of the first
  // cycle's H in Leja order (they only steer the basis' conditioning, so
  // one estimate of the spectrum serves the whole call)
  if (!newton) {
    std::vector<double> re(m), im(m);
    c->sh_alpha.assign(s, 0.0);
    c->sh_q.assign(s, 0.0);
    if (!kry::hess_eigvals(m, H, ldh, re.data(), im.data()) ||
        kry::leja_steps(m, re.data(), im.data(), s, rho, c->sh_alpha.data(), c->sh_q.data()) < s) {
      c->sh_alpha.clear();
      c->sh_q.clear();
    }
  }
  return KRY_OK;
}

// The s-step cycle with every block finished on the device: the Gram
// product, its reduction, the Cholesky factor, the condition checks and the
// update coefficients (launch_sstep_fin), then the update, per pass; the
// second pass's launches skip themselves (a device flag) when the first
// pass was final.  The host waits once, at the end of the cycle, for the
// blocks' factors and flags, and forms H with the same algebra as the host
// path.  Any block that the host path would not take as is (a dependent or
// too ill-conditioned block) sets *redo: the caller then runs the cycle on
// the host path from the normalised start vector (slot 0).  FP64 storage,
// blocks of at most 16 steps, M + s <= 256.
bool dev_cycle_ok(kry_ctx* c, int m) {
  const int s = c->s_eff;
  return c->st == kry::F64 && s > 1 && s <= 16 && m + 1 <= 256 && !c->opts.host_blocks;
}

// The launches of one device s-step cycle on `st` (from the normalisation
// of the start vector to the last block's update); `timed`: record the
// kernel-class events (never inside a graph capture).
struct SstepPlan {
  int m = 0, bs = 0, nblk = 0;
  std::vector<double> al, qq, sg;
  std::vector<size_t> off;
  size_t tot = 0;
};

int enqueue_sstep_dev(kry_ctx* c, const SstepPlan& P, hipStream_t st, bool timed) {
  const double cond_max = 1e6, one_pass_max = 300.0, one_pass_left = 1e-6;
  const int m = P.m, bs = P.bs;
  KRY_HIP(kry::launch_fin_start(c->d_red1, c->d_scal + 2, st));
  KRY_HIP(kry::launch_scale(c->st, slot(c, 0), c->d_scal + 2, slot(c, 0), c->n, st));
  const double mb_axpby = mbytes(c, true) - 8.0 * c->g.N3;
  const double vb = vbytes(c);
  for (int j0 = 0, b = 0; j0 < m; j0 += bs, ++b) {
    const int ss = std::min(bs, m - j0);
    const int M = j0 + 1;
    void* S = slot(c, j0 + 1);
    auto tk = [&](int k) { return slot(c, j0 + k); };
    for (int k = 0; k < ss; ++k) {
      const bool prev = k > 0 && P.qq[k] != 0.0;
      hipEvent_t e = timed ? tbeg(c) : nullptr;
      KRY_HIP(kry::launch_stencil_axpby(kry::F64, tk(k), prev ? tk(k - 1) : nullptr, tk(k + 1), 1.0 / P.sg[k],
                                        -P.al[k] / P.sg[k], prev ? P.qq[k] / P.sg[k] : 0.0, c->g, c->mats, st));
      if (timed) tend(c, e, KRY_K_STENCIL, vb * (prev ? 3.0 : 2.0) + mb_axpby);
    }
    const int ns = kry::gram_splits(c->n, M + ss, ss);
    double* stash = c->d_stash + P.off[b];
    int* flags = c->d_flags + 4 * b;
    const double gram_bytes = vb * (M + ss) + 8.0 * c->n;
    const double gemm_bytes = vb * (M + ss) + vb * ss;
    for (int pass = 1; pass <= 2; ++pass) {
      const int* skip = pass == 2 ? flags + 1 : nullptr;
      // the second pass's launches are timed only when they are known to run
      hipEvent_t e = (timed && pass == 1) ? tbeg(c) : nullptr;
      KRY_HIP(kry::launch_gram(kry::F64, slot(c, 0), M + ss, S, ss, c->ldv, c->d_w, c->n, c->d_gp, ns, st, S, M,
                               -1, skip));
      if (timed && pass == 1) tend(c, e, KRY_K_GRAM, gram_bytes, 2.0 * c->n * (M + ss) * ss);
      KRY_HIP(kry::launch_reduce(c->d_gp, ns, (M + ss) * ss, (M + ss) * ss, c->d_bc, st, skip));
      KRY_HIP(kry::launch_sstep_fin(pass, M, ss, c->d_bc, c->d_K, stash, flags, one_pass_max, one_pass_left,
                                    cond_max, st));
      e = (timed && pass == 1) ? tbeg(c) : nullptr;
      KRY_HIP(kry::launch_gemm_nn(kry::F64, slot(c, 0), M + ss, c->d_K, ss, S, c->ldv, c->n, 1.0, 0, st, S, M,
                                  -1, -1, skip));
      if (timed && pass == 1) tend(c, e, KRY_K_GEMM, gemm_bytes, 2.0 * c->n * (M + ss) * ss);
    }
  }
  return KRY_OK;
}

int arnoldi_ca_dev(kry_ctx* c, int m, double* beta, int* m_eff, bool* redo) {
  *redo = false;
  const int s = c->s_eff;
  const int ldh = m + 1;
  hipStream_t st = c->stream;
  int rc = ensure_weights(c);
  if (rc) return rc;
  std::vector<double> d;
  rc = host_dots(c, slot(c, 0), nullptr, 0, d);
  if (rc) return rc;
  double* H = c->h_H;
  std::fill(H, H + (size_t)(m + 1) * m, 0.0);
  const double b0 = std::sqrt(std::max(d[0], 0.0));
  if (!(b0 > 0.0)) {
    *beta = 0.0;
    *m_eff = 0;
    return KRY_OK;
  }
  const double rho = c->rho;
  const bool newton = (int)c->sh_alpha.size() >= s;
  SstepPlan P;
  P.m = m;
  P.bs = newton ? s : std::min(s, 16);
  const int bs = P.bs;
  P.al.assign(bs, 0.0);
  P.qq.assign(bs, 0.0);
  P.sg.assign(bs, 0.0);
  for (int k = 0; k < bs; ++k) {
    if (newton) {
      P.al[k] = c->sh_alpha[k];
      P.qq[k] = c->sh_q[k];
      P.sg[k] = rho;
    } else {
      P.sg[k] = k == 0 ? rho : 0.5 * rho;
      P.qq[k] = k == 0 ? 0.0 : 0.5 * rho;
    }
  }
  // per-block stash offsets, workspace
  size_t gp = 0, bc = 0;
  std::vector<std::vector<double>> Tms;
  for (int j0 = 0; j0 < m; j0 += bs, ++P.nblk) {
    const int ss = std::min(bs, m - j0), M = j0 + 1;
    P.off.push_back(P.tot);
    P.tot += (size_t)kry::sstep_stash_doubles(M, ss);
    gp = std::max(gp, (size_t)kry::gram_splits(c->n, M + ss, ss) * (M + ss) * ss);
    bc = std::max(bc, (size_t)(M + ss) * ss);
    // A [t_0..t_{ss-1}] = [t_0..t_ss] Tm of the block's recurrence
    std::vector<double> Tm((size_t)(ss + 1) * ss, 0.0);
    for (int k = 0; k < ss; ++k) {
      const bool prev = k > 0 && P.qq[k] != 0.0;
      Tm[(size_t)(k + 1) * ss + k] = P.sg[k];
      Tm[(size_t)k * ss + k] = P.al[k];
      if (prev) Tm[(size_t)(k - 1) * ss + k] = -P.qq[k];
    }
    Tms.push_back(std::move(Tm));
  }
  const int nblk = P.nblk;
  rc = ensure_gp(c, gp, bc);
  if (rc) return rc;
  if (!c->d_K) KRY_HIP(hipMalloc(&c->d_K, sizeof(double) * 256 * 16));
  if (P.tot > c->stash_cap) {
    drop_graphs(c);
    hipFree(c->d_stash);
    c->d_stash = nullptr;
    KRY_HIP(hipMalloc(&c->d_stash, sizeof(double) * P.tot));
    c->stash_cap = P.tot;
  }
  if (4 * nblk > c->flags_cap) {
    drop_graphs(c);
    hipFree(c->d_flags);
    c->d_flags = nullptr;
    KRY_HIP(hipMalloc(&c->d_flags, sizeof(int) * 4 * nblk));
    c->flags_cap = 4 * nblk;
  }
  if (c->opts.use_graph && c->opts.timing <= 0) {
    // one captured cycle per (m, block size, basis steps), replayed on the
    // solver's stream for the cycles of a call that share its steps
    std::vector<double> key = {(double)m, (double)bs, rho};
    key.insert(key.end(), P.al.begin(), P.al.end());
    key.insert(key.end(), P.qq.begin(), P.qq.end());
    key.insert(key.end(), P.sg.begin(), P.sg.end());
    if (!c->sstep_graph || key != c->sstep_key) {
      if (c->sstep_graph) hipGraphExecDestroy(c->sstep_graph);
      c->sstep_graph = nullptr;
      c->sstep_key.clear();
      if (!c->cstream) KRY_HIP(hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      KRY_HIP(hipStreamBeginCapture(c->cstream, hipStreamCaptureModeThreadLocal));
      const int rc2 = enqueue_sstep_dev(c, P, c->cstream, false);
      const hipError_t ec = hipStreamEndCapture(c->cstream, &graph);
      if (rc2) {
        if (graph) hipGraphDestroy(graph);
        return rc2;
      }
      KRY_HIP(ec);
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      KRY_HIP(ei);
      c->sstep_graph = exec;
      c->sstep_key = key;
    }
    KRY_HIP(hipGraphLaunch(c->sstep_graph, st));
  } else {
    rc = enqueue_sstep_dev(c, P, st, true);
    if (rc) return rc;
  }
  const double vb = vbytes(c);
  std::vector<double> hs(P.tot);
  std::vector<int> hf(4 * nblk);
  KRY_HIP(hipMemcpyAsync(hs.data(), c->d_stash, sizeof(double) * P.tot, hipMemcpyDeviceToHost, st));
  KRY_HIP(hipMemcpyAsync(hf.data(), c->d_flags, sizeof(int) * 4 * nblk, hipMemcpyDeviceToHost, st));
  KRY_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < nblk; ++b) {
    const int* f = hf.data() + 4 * b;
    if (!f[0] || (!f[1] && (!f[2] || f[3]))) {
      tresolve(c);
      *beta = b0;
      *redo = true;
      return KRY_OK;
    }
  }
  for (int j0 = 0, b = 0; j0 < m; j0 += bs, ++b) {
    const int ss = std::min(bs, m - j0), M = j0 + 1;
    const double* C1 = hs.data() + P.off[b];
    const double* R1 = C1 + (size_t)M * ss;
    const double* C2 = R1 + (size_t)ss * ss + ss + (size_t)ss * ss;
    const double* R2 = C2 + (size_t)M * ss;
    std::vector<double> C2h, R2h;
    if (hf[4 * b + 1]) {  // final after one pass
      C2h.assign((size_t)M * ss, 0.0);
      R2h.assign((size_t)ss * ss, 0.0);
      for (int a = 0; a < ss; ++a) R2h[(size_t)a * ss + a] = 1.0;
      C2 = C2h.data();
      R2 = R2h.data();
    } else if (c->opts.timing > 0) {  // its second pass ran: count its launches
      c->k_launch_all[KRY_K_GRAM] += 1;
      c->k_bytes_all[KRY_K_GRAM] += vb * (M + ss) + 8.0 * c->n;
      c->k_launch_all[KRY_K_GEMM] += 1;
      c->k_bytes_all[KRY_K_GEMM] += vb * (M + 2.0 * ss);
    }
    kry::sstep_hessenberg_tm(j0, ss, Tms[b].data(), C1, C2, R1, R2, H, ldh);
  }
  tresolve(c);
  *beta = b0;
  *m_eff = m;
  if (!newton) {
    std::vector<double> re(m), im(m);
    c->sh_alpha.assign(s, 0.0);
    c->sh_q.assign(s, 0.0);
    if (!kry::hess_eigvals(m, H, ldh, re.data(), im.data()) ||
        kry::leja_steps(m, re.data(), im.data(), s, rho, c->sh_alpha.data(), c->sh_q.data()) < s) {
      c->sh_alpha.clear();
      c->sh_q.clear();
    }
  }
  return KRY_OK;
}

int arnoldi_ca(kry_ctx* c, int m, double* beta, int* m_eff) {
  if (dev_cycle_ok(c, m)) {
    bool redo = false;
    int rc = arnoldi_ca_dev(c, m, beta, m_eff, &redo);
    if (rc || !redo) return rc;
    // a block the host path treats apart: the cycle again on the host path
    // from the normalised start vector
    const double b0 = *beta;
    double b1 = 0.0;
    rc = arnoldi_ca_host(c, m, &b1, m_eff);
    *beta = b0 * b1;
    return rc;
  }
  return arnoldi_ca_host(c, m, beta, m_eff);
}

// Rank-revealing Cholesky QR, twice: Out[:p] = M-orthonormal basis of W[:p]
// (zero columns for dropped directions), W ~= Out Rf.  W and Out must not
// overlap; T2 is scratch (p columns).
int block_cholqr2(kry_ctx* c, void* W, int p, void* T2, void* Out, std::vector<double>& Rf, int* rank) {
  std::vector<double> G, Cm((size_t)p * p), R1((size_t)p * p), Cm2((size_t)p * p), R2((size_t)p * p);
  int rc = block_gram_host(c, W, p, W, p, G);
  if (rc) return rc;
  const int r1 = kry::cholqr_factor(p, G.data(), 1e-10, Cm.data(), R1.data());
  rc = block_gemm(c, W, p, Cm, p, T2, 1.0, 0);
  if (rc) return rc;
  rc = block_gram_host(c, T2, p, T2, p, G);
  if (rc) return rc;
  const int r2 = kry::cholqr_factor(p, G.data(), 1e-10, Cm2.data(), R2.data());
  rc = block_gemm(c, T2, p, Cm2, p, Out, 1.0, 0);
  if (rc) return rc;
  Rf.assign((size_t)p * p, 0.0);
  for (int a = 0; a < p; ++a)
    for (int b = 0; b < p; ++b) {
      double acc = 0.0;
      for (int k = 0; k < p; ++k) acc += R2[(size_t)a * p + k] * R1[(size_t)k * p + b];
      Rf[(size_t)a * p + b] = acc;
    }
  *rank = std::min(r1, r2);
  return KRY_OK;
}

// Block Arnoldi (block classical Gram-Schmidt twice, each pass one Gram
// product [V, W]^T M W with the projected Gram matrix by Pythagoras, a
// rank-revealing Cholesky QR, and one update (W - V C) Cm): start block
// V_0 already orthonormal in slots [0, p); fills slots up to (mb+1) p and
// Hb ((mb+1) p x mb p, column-major).  Stops early (*mb_eff) when a new
// block is entirely dependent (an invariant block Krylov space).  Work
// slots: W at ws, T2 at ws + p.
int block_arnoldi(kry_ctx* c, int p, int mb, int ws, std::vector<double>& Hb, int* mb_eff,
                  kry_stats* st, bool transient) {
  const int ldh = (mb + 1) * p;
  Hb.assign((size_t)ldh * mb * p, 0.0);
  void* W = bslot(c, ws);
  void* T2 = bslot(c, ws + p);
  std::vector<double> P1, P2, C1, C2, G((size_t)p * p), ref(p), Cm1((size_t)p * p), Rf1((size_t)p * p),
      Cm2((size_t)p * p), Rf2((size_t)p * p), K;
  *mb_eff = mb;
  for (int j = 0; j < mb; ++j) {
    hipEvent_t e = tbeg(c);
    KRY_HIP(kry::launch_stencil_cols(c->st, bslot(c, j * p), W, c->ldv, p, c->g, c->mats, c->stream));
    tend(c, e, KRY_K_STENCIL, vbytes(c) * 2.0 * p + mbytes(c, true) - 8.0 * c->g.N3);
    if (st) (transient ? st->matvecs_transient : st->matvecs_stationary) += p;
    const int M = (j + 1) * p;
    // pass 1: [V, W]^T M W in one product, projected Gram by Pythagoras,
    // rank-revealing Cholesky QR, T2 = (W - V C1) Cm1 in one product
    int rc = block_gram_host(c, bslot(c, 0), M + p, W, p, P1, W, M);
    if (rc) return rc;
    C1.assign(P1.begin(), P1.begin() + (size_t)M * p);
    kry::proj_gram(M, p, P1.data(), G.data(), ref.data());
    bool cancel = false;  // projected norms lost to rounding: project explicitly
    for (int k = 0; k < p; ++k) cancel |= !(G[(size_t)k * p + k] > 1e-12 * ref[k]) && ref[k] > 0.0;
    int r1;
    if (!cancel) {
      r1 = kry::cholqr_factor(p, G.data(), 1e-10, Cm1.data(), Rf1.data());
      K.resize((size_t)(M + p) * p);
      kry::stack_coef_full(M, p, C1.data(), Cm1.data(), K.data());
      rc = block_gemm(c, bslot(c, 0), M + p, K, p, T2, 1.0, 0, W, M);
      if (rc) return rc;
    } else {
      rc = block_gemm(c, bslot(c, 0), M, C1, p, W, -1.0, 1);
      if (rc) return rc;
      rc = block_gram_host(c, W, p, W, p, G);
      if (rc) return rc;
      r1 = kry::cholqr_factor(p, G.data(), 1e-10, Cm1.data(), Rf1.data());
      rc = block_gemm(c, W, p, Cm1, p, T2, 1.0, 0);
      if (rc) return rc;
    }
    // pass 2 on T2 (nearly orthogonal to V: no cancellation), result Q in
    // the next basis block
    rc = block_gram_host(c, bslot(c, 0), M + p, T2, p, P2, T2, M);
    if (rc) return rc;
    C2.assign(P2.begin(), P2.begin() + (size_t)M * p);
    kry::proj_gram(M, p, P2.data(), G.data(), ref.data());
    const int r2 = kry::cholqr_factor(p, G.data(), 1e-10, Cm2.data(), Rf2.data());
    K.resize((size_t)(M + p) * p);
    kry::stack_coef_full(M, p, C2.data(), Cm2.data(), K.data());
    rc = block_gemm(c, bslot(c, 0), M + p, K, p, bslot(c, (j + 1) * p), 1.0, 0, T2, M);
    if (rc) return rc;
    // W = V (C1 + C2 Rf1) + Q (Rf2 Rf1)
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < p; ++b) {
        double v = C1[(size_t)a * p + b];
        for (int l = 0; l < p; ++l) v += C2[(size_t)a * p + l] * Rf1[(size_t)l * p + b];
        Hb[a + (size_t)(j * p + b) * ldh] = v;
      }
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        double v = 0.0;
        for (int l = 0; l < p; ++l) v += Rf2[(size_t)a * p + l] * Rf1[(size_t)l * p + b];
        Hb[(j + 1) * p + a + (size_t)(j * p + b) * ldh] = v;
      }
    if (std::min(r1, r2) == 0) {  // the block space is invariant: stop here
      *mb_eff = j + 1;
      break;
    }
  }
  return KRY_OK;
}

// Stationary part for a group of g complex columns (b_k, w_k): block GMRES
// with one shift per column in the shared real block space.  Each cycle
// minimises every column's residual over its own shifted projection; the
// next start block spans the real and imaginary parts of the residual
// coefficient vectors of the unconverged columns.  Those coefficients are
// known exactly on the host in the orthonormal basis, so the restart block
// is orthonormalised there (pivoted Householder QR) and the restart is
// exact.  z_k accumulates in Z columns 2k (Re), 2k+1 (Im).
int block_stationary(kry_ctx* c, const std::vector<const double*>& bcols, const std::vector<double>& om,
                     double tol, kry_stats* st, double* max_res, std::vector<double>& bnorm) {
  const int g = (int)bcols.size();
  const int pmax = 2 * g;
  const int mb = c->opts.block_steps > 0 ? c->opts.block_steps : std::max(2, c->opts.krylov_dim / pmax);
  const int ws = (mb + 1) * pmax;  // work slots: W, T2, start block
  int rc = ensure_block(c, ws + 3 * pmax);
  if (rc) return rc;
  rc = ensure_z(c, g);
  if (rc) return rc;
  for (int k = 0; k < g; ++k) KRY_HIP(hipMemsetAsync(zcol(c, 2 * k), 0, 2 * c->ldv * c->esz, c->stream));
  void* X = bslot(c, ws + 2 * pmax);
  for (int k = 0; k < g; ++k) {
    KRY_HIP(kry::launch_load_complex(c->st, bcols[k], 0, bslot(c, ws + 2 * pmax + 2 * k), c->n, c->stream));
    KRY_HIP(kry::launch_load_complex(c->st, bcols[k], 1, bslot(c, ws + 2 * pmax + 2 * k + 1), c->n, c->stream));
  }
  std::vector<double> G;
  rc = block_gram_host(c, X, pmax, X, pmax, G);
  if (rc) return rc;
  bnorm.assign(g, 0.0);
  std::vector<char> active(g, 1);
  for (int k = 0; k < g; ++k) {
    bnorm[k] = std::sqrt(G[(size_t)(2 * k) * pmax + 2 * k] + G[(size_t)(2 * k + 1) * pmax + 2 * k + 1]);
    if (bnorm[k] == 0.0) active[k] = 0;
  }
  // first start block: V_0 R = [Re b_k, Im b_k]
  std::vector<double> Rf;
  int rank = 0;
  rc = block_cholqr2(c, X, pmax, bslot(c, ws + pmax), bslot(c, 0), Rf, &rank);
  if (rc) return rc;
  int p = pmax;
  // gk[k]: column k's residual in the current start block V_0 (length p)
  std::vector<std::vector<cplx>> gk(g, std::vector<cplx>(p, 0.0));
  for (int k = 0; k < g; ++k)
    for (int a = 0; a < p; ++a)
      gk[k][a] = cplx(Rf[(size_t)a * p + 2 * k], Rf[(size_t)a * p + 2 * k + 1]);
  const int maxcyc = c->opts.max_restarts > 0 ? c->opts.max_restarts : 100000;
  std::vector<double> Hb;
  double worst = 0.0;
  for (int cyc = 0; cyc < maxcyc; ++cyc) {
    int nact = 0;
    for (int k = 0; k < g; ++k) nact += active[k];
    if (nact == 0) break;
    int mbe = 0;
    rc = block_arnoldi(c, p, mb, ws, Hb, &mbe, st, false);
    if (rc) return rc;
    if (st) st->cycles_stationary += 1;
    const int ldh = (mb + 1) * p;
    const int K = mbe * p;
    const int R = K + p;
    std::vector<double> Yz((size_t)K * 2 * g, 0.0);  // row-major K x 2g
    std::vector<std::vector<cplx>> res(g);
    worst = 0.0;
    for (int k = 0; k < g; ++k) {
      if (!active[k]) continue;
      std::vector<cplx> rhs(R, 0.0), y(K), r(R);
      for (int a = 0; a < p; ++a) rhs[a] = gk[k][a];
      kry::block_shift_lsq(K, p, 2 * p - 1, Hb.data(), ldh, cplx(0.0, om[k]), rhs.data(), y.data(), r.data());
      for (int i = 0; i < K; ++i) {
        Yz[(size_t)i * 2 * g + 2 * k] = y[i].real();
        Yz[(size_t)i * 2 * g + 2 * k + 1] = y[i].imag();
      }
      double rn = 0.0;
      for (auto& v : r) rn += std::norm(v);
      rn = std::sqrt(rn) / bnorm[k];
      worst = std::max(worst, rn);
      res[k] = r;
      if (rn <= tol) active[k] = 0;
    }
    rc = block_gemm(c, bslot(c, 0), K, Yz, 2 * g, zcol(c, 0), 1.0, 1);
    if (rc) return rc;
    if (c->opts.verbose && (cyc + 1) % 20 == 0)
      std::fprintf(stderr, "[kry] block shifted solve cycle %d: largest relative residual %.3e\n", cyc + 1, worst);
    nact = 0;
    for (int k = 0; k < g; ++k) nact += active[k];
    if (nact == 0) break;
    if (cyc + 1 == maxcyc) {
      *max_res = std::max(*max_res, worst);
      return KRY_ENOCONV;
    }
    // next start block: orthonormal basis of the real and imaginary parts of
    // the active residual coefficients, S = Q Rq on the host, V_0 = V_R Q
    const int q = 2 * nact;
    std::vector<double> Sm((size_t)R * q, 0.0);  // column-major R x q
    std::vector<int> idx;
    for (int k = 0; k < g; ++k) {
      if (!active[k]) continue;
      const int a = (int)idx.size();
      idx.push_back(k);
      for (int i = 0; i < R; ++i) {
        Sm[i + (size_t)(2 * a) * R] = res[k][i].real();
        Sm[i + (size_t)(2 * a + 1) * R] = res[k][i].imag();
      }
    }
    std::vector<double> Q((size_t)R * q), Rq((size_t)q * q);
    kry::qr_pivoted(R, q, Sm.data(), 1e-15, Q.data(), Rq.data());
    std::vector<double> Qr((size_t)R * q);  // row-major for the product kernel
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < q; ++j) Qr[(size_t)i * q + j] = Q[i + (size_t)j * R];
    rc = block_gemm(c, bslot(c, 0), R, Qr, q, X, 1.0, 0);
    if (rc) return rc;
    KRY_HIP(hipMemcpyAsync(bslot(c, 0), X, (size_t)q * c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
    p = q;
    for (int a = 0; a < nact; ++a) {
      const int k = idx[a];
      gk[k].assign(p, 0.0);
      for (int b = 0; b < p; ++b) gk[k][b] = cplx(Rq[(size_t)b * q + 2 * a], Rq[(size_t)b * q + 2 * a + 1]);
    }
  }
  *max_res = std::max(*max_res, worst);
  return KRY_OK;
}

int transient_steps(kry_ctx* c) {
  return c->opts.block_steps_transient > 0 ? c->opts.block_steps_transient : 32;
}

struct ExpvTrace;
int expv_slot0(kry_ctx* c, double T, double abstol, double drop, kry_stats* st, double* err_est,
               ExpvTrace* tr);

// Transients for a group of g columns: X (slots at xs, g columns) holds
// Im z_k; e^{-T A} X by restarts in time with block Arnoldi, left in X.
// rate[k] is the residual rate of column k (its error budget / T).  The
// first start block is orthonormalised on the device (Cholesky QR twice);
// later ones are X = V_K U with U known on the host, so V_0 = V_K Q from a
// host QR of U, exactly.
int block_transient(kry_ctx* c, int xs, int g, double T, const std::vector<double>& rate,
                    kry_stats* st, std::vector<double>& err) {
  const int p = g;
  const int mb = transient_steps(c);
  const int ws = (mb + 1) * p;
  int rc = ensure_block(c, std::max(ws + 2 * p, xs + g));
  if (rc) return rc;
  if (xs < ws + 2 * p) return fail(c, KRY_EINVAL, "block transient slot overlap");
  void* X = bslot(c, xs);
  err.assign(g, 0.0);
  double t = 0.0, tau_try = T;
  std::vector<double> Hb, R0, U, e;
  int rank = 0;
  rc = block_cholqr2(c, X, p, bslot(c, ws), bslot(c, 0), R0, &rank);
  if (rc) return rc;
  if (rank == 0) return KRY_OK;  // every transient is zero
  const int maxsteps = c->opts.max_restarts > 0 ? c->opts.max_restarts : 100000;
  int steps = 0;
  while (true) {
    if (steps >= maxsteps) return KRY_ENOCONV;
    int mbe = 0;
    rc = block_arnoldi(c, p, mb, ws, Hb, &mbe, st, true);
    if (rc) return rc;
    ++steps;
    if (st) st->steps_transient += 1;
    const int ldh = (mb + 1) * p;
    const int K = mbe * p;
    std::vector<double> U0((size_t)K * g, 0.0);  // column-major K x g
    for (int a = 0; a < p; ++a)
      for (int k = 0; k < g; ++k) U0[a + (size_t)k * K] = R0[(size_t)a * p + k];
    const double tmax = T - t;
    double tau = 0.0;
    U.assign((size_t)K * g, 0.0);
    e.assign(g, 0.0);
    if (mbe < mb) {  // invariant block space: exact projected exponential
      std::vector<double> Hm((size_t)K * K), E((size_t)K * K);
      for (int j = 0; j < K; ++j)
        for (int i = 0; i < K; ++i) Hm[i + (size_t)j * K] = -tmax * Hb[i + (size_t)j * ldh];
      kry::expm(K, Hm.data(), E.data());
      for (int k = 0; k < g; ++k)
        for (int i = 0; i < K; ++i) {
          double acc = 0.0;
          for (int l = 0; l < K; ++l) acc += E[i + (size_t)l * K] * U0[l + (size_t)k * K];
          U[i + (size_t)k * K] = acc;
        }
      tau = tmax;
    } else {
      double trial = std::min(tau_try, tmax);
      for (int attempt = 0; attempt < 60 && tau == 0.0; ++attempt) {
        tau = kry::choose_step_block(K, p, g, Hb.data(), ldh, U0.data(), trial, rate.data(), 16,
                                     U.data(), e.data());
        if (tau == 0.0) trial /= 16.0;
      }
      if (tau == 0.0) return fail(c, KRY_ENOCONV, "time step underflow in the block exponential");
      tau_try = (tau >= trial * (1.0 - 1e-12)) ? 2.0 * trial : 1.25 * tau;
      if (t + tau > T * (1.0 - 1e-15)) tau = tmax;
    }
    for (int k = 0; k < g; ++k) err[k] += e[k];
    t += tau;
    if (t >= T) {
      // X = V_K U
      std::vector<double> Ur((size_t)K * g);
      for (int i = 0; i < K; ++i)
        for (int k = 0; k < g; ++k) Ur[(size_t)i * g + k] = U[i + (size_t)k * K];
      return block_gemm(c, bslot(c, 0), K, Ur, g, X, 1.0, 0);
    }
    // next start block from U = Q R0 (host), V_0 = V_K Q
    std::vector<double> Q((size_t)K * g), Rq((size_t)g * g);
    const int r = kry::qr_pivoted(K, g, U.data(), 1e-15, Q.data(), Rq.data());
    if (r == 0) {  // the transients vanished exactly
      KRY_HIP(hipMemsetAsync(X, 0, (size_t)g * c->ldv * c->esz, c->stream));
      return KRY_OK;
    }
    std::vector<double> Qr((size_t)K * g);
    for (int i = 0; i < K; ++i)
      for (int k = 0; k < g; ++k) Qr[(size_t)i * g + k] = Q[i + (size_t)k * K];
    rc = block_gemm(c, bslot(c, 0), K, Qr, g, X, 1.0, 0);
    if (rc) return rc;
    KRY_HIP(hipMemcpyAsync(bslot(c, 0), X, (size_t)g * c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
    R0 = Rq;
  }
}

// Batched solve: columns in groups of block_width/2 complex columns.
int solve_blocked(kry_ctx* c, const double* omegas, int n_omega, int n_src, const double* b,
                  int b_per_omega, double T, double* yT, kry_stats* st, double* max_res,
                  double* max_err, double* t_trans) {
  const int ncols = n_omega * n_src;
  const int g = std::max(1, c->opts.block_width / 2);
  const double tol = c->opts.tol;
  int status = KRY_OK;
  for (int c0 = 0; c0 < ncols; c0 += g) {
    const int gg = std::min(g, ncols - c0);
    std::vector<const double*> bc(gg);
    std::vector<double> om(gg);
    for (int k = 0; k < gg; ++k) {
      const int col = c0 + k;
      const int w = col / n_src, s = col % n_src;
      bc[k] = b + (size_t)(b_per_omega ? col : s) * 2 * c->n;
      om[k] = omegas[w];
    }
    std::vector<double> bnorm;
    int rc = block_stationary(c, bc, om, 0.05 * tol, st, max_res, bnorm);
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
    const double t1 = now_ms();
    // |Im(e^{iwT} z_k)|_M for the budgets
    std::vector<double> Gz;
    rc = block_gram_host(c, zcol(c, 0), 2 * gg, zcol(c, 0), 2 * gg, Gz);
    if (rc) return rc;
    std::vector<double> rate(gg), ynorm(gg);
    for (int k = 0; k < gg; ++k) {
      const double sn = std::sin(om[k] * T), cs = std::cos(om[k] * T);
      const int P = 2 * gg;
      const double rr = Gz[(size_t)(2 * k) * P + 2 * k], ii = Gz[(size_t)(2 * k + 1) * P + 2 * k + 1];
      const double ri = Gz[(size_t)(2 * k) * P + 2 * k + 1];
      ynorm[k] = std::sqrt(std::max(sn * sn * rr + cs * cs * ii + 2 * sn * cs * ri, 0.0));
      rate[k] = 0.15 * tol * std::max(ynorm[k], 1e-300) / std::max(T, 1e-300);
    }
    if (c->opts.block_steps_transient <= 0) {
      // transients one column at a time with the single-vector exponential
      // (a long basis lets it take far larger time steps than a short block)
      for (int k = 0; k < gg; ++k) {
        const double sn = std::sin(om[k] * T), cs = std::cos(om[k] * T);
        KRY_HIP(hipMemcpyAsync(slot(c, 0), zcol(c, 2 * k + 1), c->ldv * c->esz,
                               hipMemcpyDeviceToDevice, c->stream));
        double err = 0.0;
        if (T > 0.0) {
          const double sc = std::max(ynorm[k], 1e-300);
          rc = expv_slot0(c, T, 0.15 * tol * sc, 0.15 * tol * sc, st, &err);
          if (rc == KRY_ENOCONV) status = rc;
          else if (rc) return rc;
        }
        *max_err = std::max(*max_err, err / std::max(ynorm[k], 1e-300));
        KRY_HIP(kry::launch_assemble(c->st, zcol(c, 2 * k), zcol(c, 2 * k + 1), slot(c, 0), sn, cs,
                                     yT + (size_t)(c0 + k) * c->n, c->n, c->stream));
      }
    } else {
      // transient block: X = Im z_k, in slots after the transient workspace
      const int mbt = transient_steps(c);
      const int xs = (mbt + 1) * gg + 2 * gg;
      rc = ensure_block(c, xs + gg);
      if (rc) return rc;
      for (int k = 0; k < gg; ++k)
        KRY_HIP(hipMemcpyAsync(bslot(c, xs + k), zcol(c, 2 * k + 1), c->ldv * c->esz,
                               hipMemcpyDeviceToDevice, c->stream));
      std::vector<double> err;
      if (T > 0.0) {
        rc = block_transient(c, xs, gg, T, rate, st, err);
        if (rc == KRY_ENOCONV) status = rc;
        else if (rc) return rc;
      } else {
        err.assign(gg, 0.0);
      }
      for (int k = 0; k < gg; ++k) {
        const double sn = std::sin(om[k] * T), cs = std::cos(om[k] * T);
        *max_err = std::max(*max_err, err[k] / std::max(ynorm[k], 1e-300));
        KRY_HIP(kry::launch_assemble(c->st, zcol(c, 2 * k), zcol(c, 2 * k + 1), bslot(c, xs + k), sn,
                                     cs, yT + (size_t)(c0 + k) * c->n, c->n, c->stream));
      }
    }
    KRY_HIP(hipStreamSynchronize(c->stream));
    *t_trans += now_ms() - t1;
  }
  return status;
}

}  // namespace

namespace {

int api_stationary(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src, const double* b,
                   int32_t b_per_omega, double* z, kry_stats* st) {
  int rc = check_multifreq_args(c, omegas, n_omega, n_src, b);
  if (rc) return rc;
  if (!z) return fail(c, KRY_EINVAL, "null output");
  if (st) std::memset(st, 0, sizeof(*st));
  treset(c);
  const double t0 = now_ms();
  double max_res = 0.0;
  if (c->opts.block_width > 1) {
    const int ncols = n_omega * n_src;
    const int g = std::max(1, c->opts.block_width / 2);
    int status = KRY_OK;
    rc = ensure_basis(c, c->opts.krylov_dim);
    if (rc) return rc;
    for (int c0 = 0; c0 < ncols; c0 += g) {
      const int gg = std::min(g, ncols - c0);
      std::vector<const double*> bc(gg);
      std::vector<double> om(gg), bn;
      for (int k = 0; k < gg; ++k) {
        const int col = c0 + k;
        bc[k] = b + (size_t)(b_per_omega ? col : col % n_src) * 2 * c->n;
        om[k] = omegas[col / n_src];
      }
      rc = block_stationary(c, bc, om, c->opts.tol, st, &max_res, bn);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      for (int k = 0; k < gg; ++k)
        KRY_HIP(kry::launch_store_complex(c->st, zcol(c, 2 * k), zcol(c, 2 * k + 1),
                                          z + (size_t)(c0 + k) * 2 * c->n, c->n, c->stream));
    }
    KRY_HIP(hipStreamSynchronize(c->stream));
    if (st) {
      st->max_residual = max_res;
      st->ms_stationary = st->ms_total = now_ms() - t0;
      st->converged = status == KRY_OK;
      texport(c, st);
    }
    return status;
  }
  rc = for_each_group(c, omegas, n_omega, n_src, b, b_per_omega, c->opts.tol, st, &max_res,
                      [&](int col, double, int zk, double) -> int {
                        KRY_HIP(kry::launch_store_complex(c->st, zcol(c, 2 * zk), zcol(c, 2 * zk + 1),
                                                          z + (size_t)col * 2 * c->n, c->n, c->stream));
                        return KRY_OK;
                      });
  if (rc && rc != KRY_ENOCONV) return rc;
  KRY_HIP(hipStreamSynchronize(c->stream));
  if (st) {
    st->max_residual = max_res;
    st->ms_stationary = st->ms_total = now_ms() - t0;
    st->converged = rc == KRY_OK;
    texport(c, st);
  }
  return rc;
}

int api_solve_multifreq(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src,
                        const double* b, int32_t b_per_omega, double T, double* yT, kry_stats* st) {
  int rc = check_multifreq_args(c, omegas, n_omega, n_src, b);
  if (rc) return rc;
  if (!yT) return fail(c, KRY_EINVAL, "null output");
  if (!(T >= 0.0) || !std::isfinite(T)) return fail(c, KRY_EINVAL, "invalid T");
  kry_stats st_local;
  if (!st) st = &st_local;  // the per-column records need the counters
  std::memset(st, 0, sizeof(*st));
  treset(c);
  c->cols.clear();
  const double t0 = now_ms();
  double max_res = 0.0, max_err = 0.0;
  double t_trans = 0.0;
  // error budget (relative to |y(T)|_M): shifted residual 0.05 tol,
  // transient steps 0.15 tol, dropped remainder 0.15 tol
  const double tol = c->opts.tol;
  if (c->opts.block_width > 1) {
    rc = ensure_basis(c, c->opts.krylov_dim);
    if (rc) return rc;
    rc = solve_blocked(c, omegas, n_omega, n_src, b, b_per_omega, T, yT, st, &max_res, &max_err,
                       &t_trans);
    if (rc && rc != KRY_ENOCONV) return rc;
    KRY_HIP(hipStreamSynchronize(c->stream));
    if (st) {
      st->max_residual = max_res;
      st->max_err_estimate = max_err;
      st->ms_total = now_ms() - t0;
      st->ms_transient = t_trans;
      st->ms_stationary = st->ms_total - t_trans;
      st->converged = rc == KRY_OK;
      texport(c, st);
    }
    return rc;
  }
  // transient continuation (equation (4diff)): per source, a chain whose
  // last column left Im z and y_hat(T) in TC and an accumulated error
  // estimate acc (absolute, energy norm)
  const bool tcont = c->opts.transient_continuation != 0 && T > 0.0;
  std::vector<double> chain_acc(n_src, -1.0);  // < 0: no chain yet
  if (tcont && (!c->TC || c->tc_cap < 2 * n_src)) {
    hipFree(c->TC);
    c->TC = nullptr;
    c->tc_cap = 0;
    const size_t bytes = (size_t)2 * n_src * c->ldv * c->esz;
    if (hipMalloc(&c->TC, bytes) != hipSuccess) {
      c->TC = nullptr;
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate transient continuation workspace");
    }
    c->tc_cap = 2 * n_src;
  }
  auto tcv = [&](int i) { return (void*)((char*)c->TC + (size_t)i * c->ldv * c->esz); };
  c->cols.assign((size_t)n_omega * n_src, kry_ctx::ColRecord{});
  ExpvTrace tr;  // the norm series of each column's transient
  tr.keep_ck = false;
  rc = for_each_group(
      c, omegas, n_omega, n_src, b, b_per_omega, 0.05 * tol, st, &max_res,
      [&](int col, double w, int zk, double bnorm) -> int {
        const double t1 = now_ms();
        const double sn = std::sin(w * T), cs = std::cos(w * T);
        void* zre = zcol(c, 2 * zk);
        void* zim = zcol(c, 2 * zk + 1);
        double* out = yT + (size_t)col * c->n;
        const int src = col % n_src;
        kry_col_stats& rec = c->cols[col].s;
        rec.omega = w;
        rec.source = src;
        rec.matvecs_stationary = c->grp_mv;
        rec.residual = zk < (int)c->zres.size() ? c->zres[zk] : NAN;
        rec.converged = c->grp_status == KRY_OK;
        const long long mvt0 = st->matvecs_transient, sst0 = st->steps_transient;
        tr.clear();
        if (bnorm == 0.0) {
          KRY_HIP(hipMemsetAsync(out, 0, sizeof(double) * c->n, c->stream));
          if (tcont) chain_acc[src] = -1.0;
          return KRY_OK;
        }
        // |Im(e^{iwT} z)|_M from <re,re>, <re,im>, <im,im>
        std::vector<double> d1, d2;
        int r = host_dots(c, zre, zre, 2, d1);  // <re,re>, <re,im>, |re|^2
        if (r) return r;
        const double nre = d1[2], xri = d1[1];
        r = host_dots(c, zim, nullptr, 0, d2);
        if (r) return r;
        const double nim = d2[0];
        const double yt2 = sn * sn * nre + cs * cs * nim + 2.0 * sn * cs * xri;
        const double ynorm = std::sqrt(std::max(yt2, 0.0));
        const double scale = std::max(ynorm, 1e-300);
        double err = 0.0;
        int status = KRY_OK;
        const double budget = 0.3 * tol * scale;  // steps + dropped remainder
        if (tcont && chain_acc[src] >= 0.0 && budget - chain_acc[src] >= 0.25 * budget) {
          // w(0) = Im z - Im z_prev, y_hat(T) = y_hat_prev(T) + e^{-TA} w(0)
          const double room = budget - chain_acc[src];
          const double Ym[2] = {-1.0, 1.0};
          KRY_HIP(hipMemcpyAsync(slot(c, 0), zim, c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
          KRY_HIP(hipMemcpyAsync(c->d_Y, Ym, sizeof(Ym), hipMemcpyHostToDevice, c->stream));
          KRY_HIP(kry::launch_combine(c->st, tcv(2 * src), c->ldv, 1, c->d_Y, 1, slot(c, 0), c->ldv, nullptr, 1,
                                      c->g, c->stream));
          r = expv_slot0(c, T, 0.25 * room, 0.25 * room, st, &err, &tr);
          if (r == KRY_ENOCONV) status = r;
          else if (r) return r;
          // (the exponential used d_Y for its own coefficients: upload +1 again)
          KRY_HIP(hipMemcpyAsync(c->d_Y, Ym + 1, sizeof(double), hipMemcpyHostToDevice, c->stream));
          KRY_HIP(kry::launch_combine(c->st, tcv(2 * src + 1), c->ldv, 1, c->d_Y, 1, slot(c, 0), c->ldv,
                                      nullptr, 1, c->g, c->stream));
          err += chain_acc[src];
        } else {
          // transient: y_hat(0) = Im z (a new chain when continuing)
          KRY_HIP(hipMemcpyAsync(slot(c, 0), zim, c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
          if (T > 0.0) {
            const double part = tcont ? 0.25 * budget : 0.5 * budget;
            r = expv_slot0(c, T, part, part, st, &err, &tr);
            if (r == KRY_ENOCONV) status = r;
            else if (r) return r;
          }
        }
        if (tcont) {  // this column closes the chain: keep Im z and y_hat(T)
          chain_acc[src] = err;
          KRY_HIP(hipMemcpyAsync(tcv(2 * src), zim, c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
          KRY_HIP(hipMemcpyAsync(tcv(2 * src + 1), slot(c, 0), c->ldv * c->esz, hipMemcpyDeviceToDevice,
                                 c->stream));
        }
        max_err = std::max(max_err, err / scale);
        // the series' last sample: |y_hat(T)|_M of the returned transient
        std::vector<double> dn;
        r = host_dots(c, slot(c, 0), nullptr, 0, dn);
        if (r) return r;
        KRY_HIP(kry::launch_assemble(c->st, zre, zim, slot(c, 0), sn, cs, out, c->n, c->stream));
        KRY_HIP(hipStreamSynchronize(c->stream));
        auto& cr = c->cols[col];
        cr.t = tr.s_t;
        cr.norm = tr.s_beta;
        cr.ms = tr.s_ms;
        cr.t.push_back(T);
        cr.norm.push_back(std::sqrt(std::max(dn[0], 0.0)));
        cr.ms.push_back(0.0);
        rec.matvecs_transient = st->matvecs_transient - mvt0;
        rec.steps_transient = st->steps_transient - sst0;
        rec.err_estimate = err / scale;
        rec.harmonic_norm = ynorm;
        rec.converged = rec.converged && status == KRY_OK;
        rec.series_len = (int32_t)cr.t.size();
        rec.ms_transient = now_ms() - t1;
        t_trans += now_ms() - t1;
        return status;
      });
  if (rc && rc != KRY_ENOCONV) return rc;
  KRY_HIP(hipStreamSynchronize(c->stream));
  if (st) {
    st->max_residual = max_res;
    st->max_err_estimate = max_err;
    st->ms_total = now_ms() - t0;
    st->ms_transient = t_trans;
    st->ms_stationary = st->ms_total - t_trans;
    st->converged = rc == KRY_OK;
    texport(c, st);
  }
  return rc;
}

}  // namespace

namespace {

int api_grad(kry_ctx* c, const double* omegas, int32_t n_omega, const double* b,
             int32_t b_per_omega, int32_t plane_k, double* loss, double* dL_deps, kry_stats* st) {
  int rc = check_multifreq_args(c, omegas, n_omega, 1, b);
  if (rc) return rc;
  if (!loss) return fail(c, KRY_EINVAL, "null output");
  if (plane_k < 1 || plane_k > c->g.nz - 1) return fail(c, KRY_EINVAL, "plane_k out of range");
  if (st) std::memset(st, 0, sizeof(*st));
  treset(c);
  const double t0 = now_ms();
  rc = ensure_basis(c, c->opts.krylov_dim);
  if (rc) return rc;
  // Z pairs: forward solutions 0..n_omega-1, the adjoint solution n_omega,
  // and with omega continuation a scratch pair n_omega + 1 (allocated now:
  // growing Z later would drop the forward solutions)
  constexpr int kQ = 3;
  const bool cont = c->opts.omega_continuation && n_omega > 1 && dL_deps;
  rc = ensure_z(c, n_omega + (cont ? 2 : 1));
  if (rc) return rc;
  if (cont) {
    rc = ensure_cont(c, 2 * kQ);
    if (rc) return rc;
  }
  const long long n = c->n, N3 = c->g.N3;
  double* rhs = nullptr;
  double* fpart = nullptr;
  const long long N2 = (long long)c->g.nx * c->g.ny;
  const int nfb = (int)((N2 + kry::kBlock - 1) / kry::kBlock);
  if (hipMalloc(&rhs, sizeof(double) * 2 * n) != hipSuccess ||
      hipMalloc(&fpart, sizeof(double) * nfb) != hipSuccess) {
    hipFree(rhs);
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate adjoint workspace");
  }
  Defer<std::function<void()>> free_ws{[&]() {
    hipFree(rhs);
    hipFree(fpart);
  }};
  int status = KRY_OK;
  double max_res = 0.0;
  const double tol = c->opts.tol;
  std::vector<double> om(omegas, omegas + n_omega);
  // forward: z_w in Z columns 0..n_omega-1
  if (!b_per_omega) {
    std::vector<int> zc(n_omega);
    for (int k = 0; k < n_omega; ++k) zc[k] = k;
    double bn = 0.0;
    rc = stationary_group(c, b, om, zc, tol, st, &max_res, &bn, n_omega);  // pair n_omega: scratch
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
  } else {
    for (int k = 0; k < n_omega; ++k) {
      double bn = 0.0;
      rc = stationary_group(c, b + (size_t)k * 2 * n, std::vector<double>{om[k]},
                            std::vector<int>{k}, tol, st, &max_res, &bn);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
    }
  }
  if (dL_deps) KRY_HIP(hipMemsetAsync(dL_deps, 0, sizeof(double) * N3, c->stream));
  double L = 0.0;
  std::vector<double> hp(nfb);
  for (int k = 0; k < n_omega; ++k) {
    void* zre = zcol(c, 2 * k);
    void* zim = zcol(c, 2 * k + 1);
    KRY_HIP(hipMemsetAsync(rhs, 0, sizeof(double) * 2 * n, c->stream));
    int nb = 0;
    KRY_HIP(kry::launch_flux_seed(c->st, zre, zim, plane_k, c->g, c->mats, fpart, rhs, &nb, c->stream));
    KRY_HIP(hipMemcpyAsync(hp.data(), fpart, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
    KRY_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < nb; ++i) L += hp[i];
    if (!dL_deps) continue;  // loss only
    // adjoint: (A + i w) x = P M^-1 a, x in Z column n_omega
    double bn = 0.0;
    const int q = cont ? std::min(k, kQ) : 0;
    if (q == 0) {
      rc = stationary_group(c, rhs, std::vector<double>{om[k]}, std::vector<int>{n_omega}, tol, st,
                            &max_res, &bn);
    } else {
      std::vector<double> om_a;
      std::vector<int> hist_a;
      for (int kk = k - q; kk < k; ++kk) {
        om_a.push_back(om[kk]);
        hist_a.push_back(kk % kQ);
      }
      double res = 0.0;
      rc = stationary_from(c, rhs, om[k], om_a, hist_a, tol, st, &res, &bn, n_omega, n_omega + 1);
      max_res = std::max(max_res, res);
    }
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
    if (cont)
      KRY_HIP(hipMemcpyAsync(zhist(c, 2 * (k % kQ)), zcol(c, 2 * n_omega), 2 * c->ldv * c->esz,
                             hipMemcpyDeviceToDevice, c->stream));
    const double* bk = b_per_omega ? b + (size_t)k * 2 * n : b;
    KRY_HIP(kry::launch_grad_acc(c->st, zre, zim, zcol(c, 2 * n_omega), zcol(c, 2 * n_omega + 1), bk,
                                 om[k], dL_deps, N3, c->stream));
  }
  KRY_HIP(hipStreamSynchronize(c->stream));
  *loss = L;
  if (st) {
    st->max_residual = max_res;
    st->ms_stationary = st->ms_total = now_ms() - t0;
    st->converged = status == KRY_OK;
    texport(c, st);
  }
  return status;
}

// ---------------------------------------------------------------------------
// Gradient of the flux at a finite time T, the transient included.
//
// L = sum_w F(y_w(T)), F the instantaneous Poynting flux of the real field
// y_w(T) = Im(e^{iwT} z) - x(T) through plane k_f (Corollary 3, with
// x(s) = e^{-sA} Im z the transient of equation (y_homo)).  With
// g = dF/dy(T) and r0 = P M^-1 g (P = +1 on H rows, -1 on E rows), the
// identity A^T = M P A P M^-1 gives e^{-tA^T} g = M P r(t) with
// r(t) = e^{-tA} r0, so the adjoint transient runs on A itself, and
//   dL/d eps_c = sum_E Im(lam (A z)) / eps_c              (through z)
//              + sum_E int_0^T r(T - s) (A x(s)) ds        (through e^{-TA})
// with (A^T + i w) lam = e^{iwT} g - M P r(T), solved as the forward
// system (A + i w) x = sin(wT) r0 + i (r(T) - cos(wT) r0), lam = -i M P x.
// The second term is the Frechet derivative of the exponential.  Both
// transients run by restarts in time with their start vectors kept; the
// integral is taken over every interval where one forward step (basis V,
// x(s) = V u(s), A x(s) = V Hbar u(s)) and one backward step (basis W,
// r(T - s) = W w(T - s)) overlap, each basis regenerated once from its
// checkpoint: it is sum_ij V_i C_ij W_j per entry with C = Hbar int u w^T ds,
// a small matrix integrated on the host by Gauss-Legendre panels fine
// enough for the bases' norms.

// One regenerated basis and the propagators of the panel grid's node gaps.
struct GapBasis {
  int me = 0;  // Arnoldi steps (0: the start vector was zero)
  int nv = 0;  // basis vectors in A V_me = V_nv Hbar (me + 1, or me on an invariant subspace)
  double beta = 0.0;
  std::vector<double> H;               // me x me, column-major
  std::vector<double> Hb;              // nv x me, column-major
  std::vector<std::vector<double>> D;  // e^{-gap_g H} per distinct gap
};

int regen_basis(kry_ctx* c, const ExpvTrace* tr, int j, void* dst, const std::vector<double>& gaps,
                GapBasis* b, kry_stats* st) {
  const int m = c->opts.krylov_dim;
  const int ldh = m + 1;
  KRY_HIP(hipMemcpyAsync(slot(c, 0), trace_ck(c, tr, j), c->ldv * c->esz, hipMemcpyDeviceToDevice,
                         c->stream));
  double beta = 0.0;
  int me = 0;
  int rc = arnoldi(c, m, &beta, &me);
  if (rc) return rc;
  if (st) st->matvecs_transient += me;
  b->me = me;
  b->beta = beta;
  b->nv = me == m ? m + 1 : me;
  if (me == 0) return KRY_OK;
  KRY_HIP(hipMemcpyAsync(dst, slot(c, 0), (size_t)b->nv * c->ldv * c->esz, hipMemcpyDeviceToDevice,
                         c->stream));
  b->H.assign((size_t)me * me, 0.0);
  b->Hb.assign((size_t)b->nv * me, 0.0);
  for (int q = 0; q < me; ++q)
    for (int i = 0; i < b->nv; ++i) {
      const double h = c->h_H[i + (size_t)q * ldh];
      b->Hb[i + (size_t)q * b->nv] = h;
      if (i < me) b->H[i + (size_t)q * me] = h;
    }
  b->D.assign(gaps.size(), {});
  std::vector<double> X((size_t)me * me);
  for (size_t g = 0; g < gaps.size(); ++g) {
    for (size_t i = 0; i < X.size(); ++i) X[i] = -gaps[g] * b->H[i];
    b->D[g].resize((size_t)me * me);
    kry::expm(me, X.data(), b->D[g].data());
  }
  KRY_HIP(hipStreamSynchronize(c->stream));
  return KRY_OK;
}

// beta e^{-h H} e_1 (length me).
std::vector<double> exp_e1(const GapBasis& b, double h) {
  const int me = b.me;
  std::vector<double> X((size_t)me * me), E((size_t)me * me), u(me);
  for (size_t i = 0; i < X.size(); ++i) X[i] = -h * b.H[i];
  kry::expm(me, X.data(), E.data());
  for (int i = 0; i < me; ++i) u[i] = b.beta * E[i];
  return u;
}

void matvec(int me, const std::vector<double>& D, const std::vector<double>& x, std::vector<double>& y) {
  y.assign(me, 0.0);
  for (int q = 0; q < me; ++q) {
    const double xq = x[q];
    const double* col = D.data() + (size_t)q * me;
    for (int i = 0; i < me; ++i) y[i] += col[i] * xq;
  }
}

// The Frechet term over [0, T] from the two traces; V and W: device buffers
// of m + 1 vectors each, dC: (m + 1) x frechet_cols() doubles.
int frechet_term(kry_ctx* c, double T, const ExpvTrace& trf, const ExpvTrace& trb, void* Vb, void* Wb,
                 double* dC, double* g, kry_stats* st) {
  const int Kf = trf.steps(), Kb = trb.steps();
  if (Kf == 0 || Kb == 0 || !(T > 0.0)) return KRY_OK;
  // forward steps cover s in [t_k, t_k + tau_k); backward steps sigma in
  // (sigma_l, sigma_l + tau_l], i.e. s in [T - sigma_l - tau_l, T - sigma_l)
  const double fend = trf.t0[Kf - 1] + trf.tau[Kf - 1];
  const double bend = trb.t0[Kb - 1] + trb.tau[Kb - 1];
  const double lo = std::max(0.0, T - bend), hi = std::min(T, fend);
  if (!(hi > lo)) return KRY_OK;
  // panel grid: 8-point Gauss-Legendre panels of width delta, with delta
  // times the sum of the two bases' norms at most 2.5 (the integrand's
  // frequencies are sums of eigenvalues of the two projected matrices)
  constexpr int Q = 8;
  double hmax_f = 0.0, hmax_b = 0.0;
  for (double h : trf.hnorm) hmax_f = std::max(hmax_f, h);
  for (double h : trb.hnorm) hmax_b = std::max(hmax_b, h);
  const double den = std::max(hmax_f + hmax_b, 1e-300);
  const long long P = std::max(1LL, (long long)std::ceil(T * den / 2.5));
  if (P > (1LL << 26)) return fail(c, KRY_EINVAL, "time horizon too long for the gradient's panel grid");
  const double delta = T / (double)P;
  double xq[Q], wq[Q];
  kry::gauss_legendre01(Q, xq, wq);
  auto node = [&](long long id) { return ((double)(id / Q) + xq[id % Q]) * delta; };
  auto first_at_or_after = [&](double a) {
    long long id = std::max(0LL, (long long)std::floor(a / delta) - 1) * Q;
    while (id < P * Q && node(id) < a) ++id;
    return id;
  };
  // distinct gaps between consecutive nodes: within a panel (x_{q+1} - x_q)
  // delta, and across panels (1 - x_{Q-1} + x_0) delta; gap index of the
  // step from node id to id + 1 is gidx[id % Q]
  std::vector<double> gaps;
  int gidx[Q];
  for (int q = 0; q < Q; ++q) {
    const double gv = q < Q - 1 ? (xq[q + 1] - xq[q]) * delta : (1.0 - xq[Q - 1] + xq[0]) * delta;
    int found = -1;
    for (size_t k = 0; k < gaps.size(); ++k)
      if (std::abs(gaps[k] - gv) <= 1e-13 * delta) found = (int)k;
    if (found < 0) {
      found = (int)gaps.size();
      gaps.push_back(gv);
    }
    gidx[q] = found;
  }
  // breakpoints of the overlap
  std::vector<double> bp = {lo, hi};
  for (int k = 0; k < Kf; ++k)
    if (trf.t0[k] > lo && trf.t0[k] < hi) bp.push_back(trf.t0[k]);
  for (int l = 0; l < Kb; ++l) {
    const double sb = T - trb.t0[l];
    if (sb > lo && sb < hi) bp.push_back(sb);
  }
  std::sort(bp.begin(), bp.end());
  const int fcols = kry::frechet_cols();
  const int m = c->opts.krylov_dim;
  GapBasis bf, bb;
  int kcur = -1, lcur = -1;
  long long fid = 0;  // node at which uf is evaluated
  std::vector<double> uf, tmp;
  long long wlo = 0;  // first node id held in wn
  std::vector<std::vector<double>> wn;
  std::vector<double> S, C, Cc((size_t)(m + 1) * fcols);
  for (size_t ib = 0; ib + 1 < bp.size(); ++ib) {
    const double a = bp[ib], b = bp[ib + 1];
    if (!(b - a > 1e-14 * T)) continue;
    const double mid = 0.5 * (a + b);
    // forward step containing mid; backward step whose s-range contains mid
    int k = (int)(std::upper_bound(trf.t0.begin(), trf.t0.end(), mid) - trf.t0.begin()) - 1;
    if (k < 0 || mid >= trf.t0[k] + trf.tau[k]) continue;
    int l = -1;
    for (int q = 0; q < Kb; ++q)
      if (T - trb.t0[q] - trb.tau[q] <= mid && mid < T - trb.t0[q]) { l = q; break; }
    if (l < 0) continue;
    if (k != kcur) {
      int rc = regen_basis(c, &trf, k, Vb, gaps, &bf, st);
      if (rc) return rc;
      kcur = k;
      fid = first_at_or_after(trf.t0[k]);
      if (bf.me > 0 && fid < P * Q) uf = exp_e1(bf, node(fid) - trf.t0[k]);
    }
    if (l != lcur) {
      int rc = regen_basis(c, &trb, l, Wb, gaps, &bb, st);
      if (rc) return rc;
      lcur = l;
      wn.clear();
      if (bb.me > 0) {
        // nodes of s in [top - tau_l, top), padded by a rounding margin (the
        // breakpoints are T - sigma_l, computed apart)
        const double top = T - trb.t0[l];  // sigma = sigma_l
        const double pad = 1e-12 * T;
        const long long idb = first_at_or_after(std::max(0.0, top - trb.tau[l] - pad));
        const long long idt = first_at_or_after(top + pad) - 1;
        if (idt >= idb) {
          wlo = idb;
          wn.assign((size_t)(idt - idb + 1), {});
          wn.back() = exp_e1(bb, top - node(idt));
          for (long long id = idt - 1; id >= idb; --id)
            matvec(bb.me, bb.D[gidx[id % Q]], wn[(size_t)(id + 1 - wlo)], wn[(size_t)(id - wlo)]);
        }
      }
    }
    if (bf.me == 0 || bb.me == 0 || wn.empty()) continue;
    const long long id0 = first_at_or_after(a), id1 = first_at_or_after(b);
    if (id1 <= id0) continue;
    // S = sum over the nodes of weight * u w^T (me_f x me_b, column-major)
    S.assign((size_t)bf.me * bb.me, 0.0);
    while (fid < id0) {  // the overlap may begin inside the forward step
      matvec(bf.me, bf.D[gidx[fid % Q]], uf, tmp);
      uf.swap(tmp);
      ++fid;
    }
    for (long long id = id0; id < id1; ++id) {
      if (id < wlo || id - wlo >= (long long)wn.size()) return fail(c, KRY_EINVAL, "node outside the adjoint step");
      const std::vector<double>& wv = wn[(size_t)(id - wlo)];
      const double wt = wq[id % Q] * delta;
      for (int j = 0; j < bb.me; ++j) {
        const double wj = wt * wv[j];
        double* Sj = S.data() + (size_t)j * bf.me;
        for (int i = 0; i < bf.me; ++i) Sj[i] += uf[i] * wj;
      }
      matvec(bf.me, bf.D[gidx[id % Q]], uf, tmp);
      uf.swap(tmp);
      ++fid;
    }
    // C = Hbar S (nv_f x me_b), then the device accumulation per chunk of
    // 64 columns of W
    C.assign((size_t)bf.nv * bb.me, 0.0);
    for (int j = 0; j < bb.me; ++j)
      for (int q = 0; q < bf.me; ++q) {
        const double sq = S[q + (size_t)j * bf.me];
        if (sq == 0.0) continue;
        const double* hc = bf.Hb.data() + (size_t)q * bf.nv;
        double* cj = C.data() + (size_t)j * bf.nv;
        for (int i = 0; i < bf.nv; ++i) cj[i] += hc[i] * sq;
      }
    for (int j0 = 0; j0 < bb.me; j0 += fcols) {
      const int nw = std::min(fcols, bb.me - j0);
      std::fill(Cc.begin(), Cc.end(), 0.0);
      for (int i = 0; i < bf.nv; ++i)
        for (int jj = 0; jj < nw; ++jj) Cc[(size_t)i * fcols + jj] = C[i + (size_t)(j0 + jj) * bf.nv];
      KRY_HIP(hipMemcpyAsync(dC, Cc.data(), sizeof(double) * (size_t)bf.nv * fcols, hipMemcpyHostToDevice,
                             c->stream));
      KRY_HIP(kry::launch_frechet_acc(c->st, Vb, bf.nv, (char*)Wb + (size_t)j0 * c->ldv * c->esz, nw, dC,
                                      c->ldv, c->g.N3, g, c->stream));
      KRY_HIP(hipStreamSynchronize(c->stream));  // Cc is reused
    }
  }
  return KRY_OK;
}

int api_grad_transient(kry_ctx* c, const double* omegas, int32_t n_omega, const double* b,
                       int32_t b_per_omega, int32_t plane_k, double T, double* loss, double* dL_deps,
                       kry_stats* st) {
  int rc = check_multifreq_args(c, omegas, n_omega, 1, b);
  if (rc) return rc;
  if (!loss) return fail(c, KRY_EINVAL, "null output");
  if (plane_k < 1 || plane_k > c->g.nz - 1) return fail(c, KRY_EINVAL, "plane_k out of range");
  if (!(T >= 0.0) || !std::isfinite(T)) return fail(c, KRY_EINVAL, "invalid T");
  if (st) std::memset(st, 0, sizeof(*st));
  treset(c);
  const double t0 = now_ms();
  const int m = c->opts.krylov_dim;
  rc = ensure_basis(c, m);
  if (rc) return rc;
  // Z pairs: forward solutions 0..n_omega-1, the adjoint solution n_omega,
  // refinement scratch n_omega + 1 (and n_omega for the forward group)
  rc = ensure_z(c, n_omega + 2);
  if (rc) return rc;
  const long long n = c->n, N3 = c->g.N3;
  const long long N2 = (long long)c->g.nx * c->g.ny;
  const int nfb = (int)((N2 + kry::kBlock - 1) / kry::kBlock);
  const size_t vb = c->ldv * c->esz;
  double* rhs = nullptr;   // adjoint right-hand side, complex interleaved
  double* ybuf = nullptr;  // y(T), FP64
  double* fpart = nullptr;
  double* dC = nullptr;
  void* work = nullptr;    // r0, r(T), then the two regenerated bases
  const int fcols = kry::frechet_cols();
  const bool grad = dL_deps != nullptr;
  const int wvecs = grad ? 2 + 2 * (m + 1) : 0;
  if (hipMalloc(&ybuf, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&fpart, sizeof(double) * nfb) != hipSuccess ||
      (grad && (hipMalloc(&rhs, sizeof(double) * 2 * n) != hipSuccess ||
                hipMalloc(&dC, sizeof(double) * (size_t)(m + 1) * fcols) != hipSuccess ||
                hipMalloc(&work, (size_t)wvecs * vb) != hipSuccess))) {
    hipFree(ybuf), hipFree(fpart), hipFree(rhs), hipFree(dC), hipFree(work);
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate the gradient workspace");
  }
  Defer<std::function<void()>> free_ws{[&]() {
    hipFree(ybuf), hipFree(fpart), hipFree(rhs), hipFree(dC), hipFree(work);
  }};
  auto wv = [&](int i) { return (void*)((char*)work + (size_t)i * vb); };
  int status = KRY_OK;
  double max_res = 0.0, max_err = 0.0;
  const double tol = c->opts.tol;
  std::vector<double> om(omegas, omegas + n_omega);
  if (!b_per_omega) {
    std::vector<int> zc(n_omega);
    for (int k = 0; k < n_omega; ++k) zc[k] = k;
    double bn = 0.0;
    rc = stationary_group(c, b, om, zc, tol, st, &max_res, &bn, n_omega);
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
  } else {
    for (int k = 0; k < n_omega; ++k) {
      double bn = 0.0;
      rc = stationary_group(c, b + (size_t)k * 2 * n, std::vector<double>{om[k]}, std::vector<int>{k}, tol,
                            st, &max_res, &bn, n_omega);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
    }
  }
  const double t_stat = now_ms();
  if (grad) KRY_HIP(hipMemsetAsync(dL_deps, 0, sizeof(double) * N3, c->stream));
  double L = 0.0;
  std::vector<double> hp(nfb), d;
  ExpvTrace trf, trb;
  for (int k = 0; k < n_omega; ++k) {
    const double w = om[k];
    const double sn = std::sin(w * T), cs = std::cos(w * T);
    void* zre = zcol(c, 2 * k);
    void* zim = zcol(c, 2 * k + 1);
    // forward transient x(s) = e^{-sA} Im z, start vectors kept
    rc = host_dots(c, zim, nullptr, 0, d);
    if (rc) return rc;
    const double vn = std::sqrt(std::max(d[0], 0.0));
    KRY_HIP(hipMemcpyAsync(slot(c, 0), zim, vb, hipMemcpyDeviceToDevice, c->stream));
    trf.clear();
    double err = 0.0;
    if (vn > 0.0 && T > 0.0) {
      rc = expv_slot0(c, T, 0.5 * tol * vn, 0.25 * tol * vn, st, &err, grad ? &trf : nullptr);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      max_err = std::max(max_err, err / vn);
    }
    // y(T) = Im(e^{iwT} z) - x(T), its flux and the adjoint start r0
    KRY_HIP(kry::launch_assemble(c->st, zre, zim, slot(c, 0), sn, cs, ybuf, n, c->stream));
    if (grad) KRY_HIP(hipMemsetAsync(wv(0), 0, vb, c->stream));
    int nb = 0;
    KRY_HIP(kry::launch_flux_inst(c->st, ybuf, plane_k, c->g, c->mats, fpart, grad ? wv(0) : nullptr, &nb,
                                  c->stream));
    KRY_HIP(hipMemcpyAsync(hp.data(), fpart, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
    KRY_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < nb; ++i) L += hp[i];
    if (!grad) continue;
    rc = host_dots(c, wv(0), nullptr, 0, d);
    if (rc) return rc;
    const double rn = std::sqrt(std::max(d[0], 0.0));
    if (!(rn > 0.0)) continue;  // F does not depend on y here: no gradient from this frequency
    // backward transient r(sigma) = e^{-sigma A} r0, start vectors kept
    KRY_HIP(hipMemcpyAsync(slot(c, 0), wv(0), vb, hipMemcpyDeviceToDevice, c->stream));
    trb.clear();
    if (T > 0.0) {
      double err2 = 0.0;
      rc = expv_slot0(c, T, 0.5 * tol * rn, 0.25 * tol * rn, st, &err2, &trb);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      max_err = std::max(max_err, err2 / rn);
    }
    KRY_HIP(hipMemcpyAsync(wv(1), slot(c, 0), vb, hipMemcpyDeviceToDevice, c->stream));
    // adjoint shifted solve and the terms through z
    KRY_HIP(kry::launch_adj_rhs(c->st, wv(0), wv(1), sn, cs, rhs, n, c->stream));
    double bn = 0.0;
    rc = stationary_group(c, rhs, std::vector<double>{w}, std::vector<int>{n_omega}, tol, st, &max_res, &bn,
                          n_omega + 1);
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
    const double* bk = b_per_omega ? b + (size_t)k * 2 * n : b;
    KRY_HIP(kry::launch_grad_acc(c->st, zre, zim, zcol(c, 2 * n_omega), zcol(c, 2 * n_omega + 1), bk, w,
                                 dL_deps, N3, c->stream));
    // the term through e^{-TA}
    rc = frechet_term(c, T, trf, trb, wv(2), wv(2 + m + 1), dC, dL_deps, st);
    if (rc) return rc;
  }
  KRY_HIP(hipStreamSynchronize(c->stream));
  *loss = L;
  if (st) {
    st->max_residual = max_res;
    st->max_err_estimate = max_err;
    st->ms_total = now_ms() - t0;
    st->ms_stationary = t_stat - t0;
    st->ms_transient = st->ms_total - st->ms_stationary;
    st->converged = status == KRY_OK;
    texport(c, st);
  }
  return status;
}

}  // namespace

namespace {

int api_block_arnoldi(kry_ctx* c, const double* V0, int32_t p, int32_t mb, void* V_out,
                      double* H_out) {
  if (!c || !V0 || !V_out || !H_out) return fail(c, KRY_EINVAL, "null argument");
  if (p < 1 || p > 128 || mb < 1 || (mb + 1) * p > 4096) return fail(c, KRY_EINVAL, "invalid p or mb");
  const int ws = (mb + 1) * p;
  int rc = ensure_block(c, ws + 3 * p);
  if (rc) return rc;
  void* X = bslot(c, ws + 2 * p);
  for (int k = 0; k < p; ++k)
    KRY_HIP(kry::launch_load_real(c->st, V0 + (size_t)k * c->n, bslot(c, ws + 2 * p + k), c->n, c->stream));
  std::vector<double> Rf, Hb;
  int rank = 0;
  rc = block_cholqr2(c, X, p, bslot(c, ws + p), bslot(c, 0), Rf, &rank);
  if (rc) return rc;
  int mbe = 0;
  rc = block_arnoldi(c, p, mb, ws, Hb, &mbe, nullptr, false);
  if (rc) return rc;
  std::memcpy(H_out, Hb.data(), sizeof(double) * Hb.size());
  for (int j = 0; j < (mb + 1) * p; ++j)
    KRY_HIP(hipMemcpyAsync((char*)V_out + (size_t)j * c->n * c->esz, bslot(c, j), c->n * c->esz,
                           hipMemcpyDeviceToDevice, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  return mbe;
}

}  // namespace

namespace {

int api_set_tune(kry_ctx* c, const kry_tune* t) {
  if (!c || !t) return fail(c, KRY_EINVAL, "null argument");
  auto ok = [](int v) { return v == 1 || v == 2 || v == 4; };
  if (!ok(t->cpt_stencil) || !ok(t->cpt_update) || !ok(t->cpt_dots))
    return fail(c, KRY_EINVAL, "cells per thread must be 1, 2 or 4");
  if (!(t->zm_stencil == 0 || t->zm_stencil == 4 || t->zm_stencil == 8 || t->zm_stencil == 16))
    return fail(c, KRY_EINVAL, "z-marching planes must be 0, 4, 8 or 16");
  c->g.cpt_s = t->cpt_stencil;
  c->g.cpt_u = t->cpt_update;
  c->g.cpt_d = t->cpt_dots;
  c->g.zm_s = t->zm_stencil;
  drop_graphs(c);  // captured launches carry the old shapes
  return KRY_OK;
}

int api_autotune(kry_ctx* c, int32_t cnt, kry_tune* out) {
  if (!c || !out) return fail(c, KRY_EINVAL, "null argument");
  const int m = c->opts.krylov_dim;
  if (cnt <= 0) cnt = std::max(1, m / 2);
  if (cnt > m) return fail(c, KRY_EINVAL, "cnt exceeds krylov_dim");
  int rc = ensure_basis(c, m);
  if (rc) return rc;
  KRY_HIP(hipMemsetAsync(c->V, 0, (size_t)(c->mcap + 3) * c->ldv * c->esz, c->stream));
  KRY_HIP(kry::launch_fill(c->d_co, 0.0, 2 * m + 4, c->stream));
  hipEvent_t e0, e1;
  KRY_HIP(hipEventCreate(&e0));
  KRY_HIP(hipEventCreate(&e1));
  Defer<std::function<void()>> free_ev{[&]() {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }};
  const kry::DevGrid saved = c->g;
  void* U = slot(c, c->mcap + 1);
  void* X = slot(c, c->mcap + 2);
  // the s-step Arnoldi builds its basis blocks with the FP64 stencil on an
  // FP64 work block under either storage type (FP32 storage with m > 112
  // runs one step per sweep, in the storage type)
  const bool ca_f64 = c->opts.s_step > 1 && !(c->st == kry::F32 && m > 112);
  void *U64 = U, *P64 = slot(c, cnt), *X64 = X;
  if (ca_f64 && c->st == kry::F32) {
    rc = ensure_sblock(c, 3);
    if (rc) return rc;
    KRY_HIP(hipMemsetAsync(c->SB, 0, (size_t)3 * c->ldv * sizeof(double), c->stream));
    U64 = c->SB;
    P64 = c->SB + c->ldv;
    X64 = c->SB + 2 * c->ldv;
  }
  const int cpts[3] = {1, 2, 4};
  auto time_us = [&](auto&& launch) -> double {
    double best = 1e300;
    for (int rep = 0; rep < 4; ++rep) {  // first launch warms up
      hipEventRecord(e0, c->stream);
      if (launch() != hipSuccess) return -1.0;
      hipEventRecord(e1, c->stream);
      hipEventSynchronize(e1);
      float ms = 0.0f;
      hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, (double)ms * 1e3);
    }
    return best;
  };
  for (int k = 0; k < 3; ++k) {
    c->g.cpt_s = c->g.cpt_u = c->g.cpt_d = cpts[k];
    // the operator kernel the solver runs: the s-step basis stencil, or the
    // stencil fused with the Gram-Schmidt dots of the one-step Arnoldi
    out->us_stencil[k] = time_us([&]() {
      if (ca_f64)
        return kry::launch_stencil_axpby(kry::F64, U64, P64, X64, 2.0 / c->rho, 0.0, 1.0, c->g, c->mats,
                                         c->stream);
      return kry::launch_stencil_lag(c->st, U, X, c->V, c->ldv, cnt, c->g, c->mats, c->partials, c->stream);
    });
    out->us_update[k] = time_us([&]() {
      return kry::launch_lag_update(c->st, U, X, c->V, c->ldv, cnt, c->d_co, slot(c, cnt), U, c->g, c->stream);
    });
    out->us_dots[k] = time_us([&]() {
      return kry::launch_dots(c->st, U, c->V, c->ldv, cnt, c->g, c->mats, c->partials, c->stream);
    });
    if (out->us_stencil[k] < 0 || out->us_update[k] < 0 || out->us_dots[k] < 0) {
      c->g = saved;
      return fail(c, KRY_EHIP, "autotune launch failed");
    }
  }
  auto pick = [&](const double* us) {
    int b = 0;
    for (int k = 1; k < 3; ++k)
      if (us[k] < us[b]) b = k;
    return cpts[b];
  };
  // the stencil keeps one cell per thread unless another shape is faster by
  // more than kStencilMargin: one launch timed in isolation varies by 1-2%,
  // and one cell per thread fetches the least from HBM (on the 128^3 medium
  // 1.01 of its algorithmic bytes, against 1.06 with two cells per thread
  // and 1.04 for the z-marching form)
  constexpr double kStencilMargin = 0.03;
  {
    int b = 0;
    for (int k = 1; k < 3; ++k)
      if (out->us_stencil[k] < out->us_stencil[b] && out->us_stencil[k] < (1.0 - kStencilMargin) * out->us_stencil[0])
        b = k;
    out->cpt_stencil = cpts[b];
  }
  out->cpt_update = pick(out->us_update);
  out->cpt_dots = pick(out->us_dots);
  // the z-marching form of the s-step basis stencil, 4, 8 and 16 planes
  // per workgroup, against the best cell-parallel shape
  out->zm_stencil = 0;
  out->pad_ = 0;
  for (int k = 0; k < 3; ++k) out->us_stencil_zm[k] = 0.0;
  if (ca_f64) {
    const int zms[3] = {4, 8, 16};
    double best = (1.0 - kStencilMargin) * out->us_stencil[out->cpt_stencil == 1 ? 0 : out->cpt_stencil == 2 ? 1 : 2];
    c->g.cpt_s = out->cpt_stencil;
    for (int k = 0; k < 3; ++k) {
      c->g.zm_s = zms[k];
      out->us_stencil_zm[k] = time_us([&]() {
        return kry::launch_stencil_axpby(kry::F64, U64, P64, X64, 2.0 / c->rho, 0.0, 1.0, c->g, c->mats,
                                         c->stream);
      });
      if (out->us_stencil_zm[k] < 0) {
        c->g = saved;
        return fail(c, KRY_EHIP, "autotune launch failed");
      }
      if (out->us_stencil_zm[k] < best) {
        best = out->us_stencil_zm[k];
        out->zm_stencil = zms[k];
      }
    }
  }
  c->g = saved;
  KRY_HIP(hipStreamSynchronize(c->stream));
  return api_set_tune(c, out);
}

}  // namespace

// ---------------------------------------------------------------------------
// Residual-restarted Krylov method for the inhomogeneous problem (Section 3,
// restarting in Krylov dimension: equation (rst), Corollary 2 and the
// algorithm of Fig. alg:rst, regular Krylov variant).  For a real source
// vector g driven by a time function alpha(t), m Arnoldi steps from g give
// V_{m+1}, H; the projected problem u' = -H_m u + alpha(t) beta e_1 (equation
// (corr2)) is solved on [0, T] for every time function that drives g; the
// update y(T) += V_m u(T) follows (equation (upd1)); the residual is
// alpha_hat(t) v_{m+1} with alpha_hat = -h_{m+1,m} e_m^T u(t) (Lemma 1), so
// the next restart starts from g = v_{m+1} with the source alpha_hat, the
// same vector for every time function (Corollary 2: the bases are shared by
// all frequencies of one source).  Each alpha_hat is sampled and stored on
// [0, T] (step (2b) of the algorithm) at the Gauss nodes of a uniform time
// grid, fine enough that the polynomial through a step's nodes represents
// it to rounding; a time function stops once the integral of its residual
// norm over [0, T], which bounds the error of y(T) in the energy norm (A is
// dissipative in it), is below its share of tol |y(T)|_M (step (2c)).
// A complex source b contributes Im(e^{i w t} b) = sin(w t) Re b +
// cos(w t) Im b: two real parts, each with its own sequence of bases.

constexpr int kRstNodes = 8;  // Gauss nodes per time step of the sampled sources

// Run fn(c) for c in [0, n) on up to `threads` host threads.
template <typename F>
void parallel_columns(int n, F&& fn) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nth = std::min(n, std::min(hw, 16));
  if (nth <= 1) {
    for (int k = 0; k < n; ++k) fn(k);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&, t]() {
      for (int k = t; k < n; k += nth) fn(k);
    });
  for (auto& th : pool) th.join();
}

struct RstColumn {
  int out;       // output column (Z column of the accumulated y(T))
  double w;      // angular frequency
  double ca, cb; // time function ca sin(w t) + cb cos(w t)
  double share;  // fraction of the column's error budget given to this part
  bool active = true;
  double resint = 0.0;
  double ynorm = 0.0;  // |y(T)|_M of the output column at the last check
};

// |Z column|_M for every listed column, with one synchronisation.
int zcol_norms(kry_ctx* c, const std::vector<int>& zc, std::vector<double>& out) {
  const int nz = (int)zc.size();
  out.assign(nz, 0.0);
  if (nz == 0) return KRY_OK;
  // all columns in one launch, one reduction: partials and the index list
  // in a workspace kept on the context (grown on demand; the reduction's
  // results follow the partials)
  const int nblk = kry::col_norm_blocks(c->g.N3);
  const size_t need = (size_t)(nblk + 1) * nz;
  if (need > c->cn_cap) {
    hipFree(c->d_cnp);
    c->d_cnp = nullptr;
    c->cn_cap = 0;
    if (hipMalloc(&c->d_cnp, sizeof(double) * need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate column norm workspace");
    }
    c->cn_cap = need;
  }
  if (nz > c->cnc_cap) {
    hipFree(c->d_cnc);
    c->d_cnc = nullptr;
    c->cnc_cap = 0;
    if (hipMalloc(&c->d_cnc, sizeof(int) * (size_t)nz) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate column norm workspace");
    }
    c->cnc_cap = nz;
  }
  double* red = c->d_cnp + (size_t)nblk * nz;
  KRY_HIP(hipMemcpyAsync(c->d_cnc, zc.data(), sizeof(int) * nz, hipMemcpyHostToDevice, c->stream));
  KRY_HIP(kry::launch_col_norms(c->st, c->Z, c->ldv, c->d_cnc, nz, c->g.N3, c->mats.eps, c->mats.mu, c->d_cnp,
                                c->stream));
  KRY_HIP(kry::launch_reduce(c->d_cnp, nblk, nz, nz, red, c->stream));
  KRY_HIP(hipMemcpyAsync(out.data(), red, sizeof(double) * nz, hipMemcpyDeviceToHost, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  for (auto& v : out) v = std::sqrt(std::max(v, 0.0));
  return KRY_OK;
}

// One real source part in slot 0 (unnormalised) and the time functions that
// drive it; y(T) accumulates into the Z columns of `cols`.  The sampled
// sources of every time function live in two device buffers (current and
// next restart); the projected problems are marched on the GPU, one wave per
// time function (on the host for Krylov dimensions above 64).
int rst_part(kry_ctx* c, std::vector<RstColumn>& cols, double T, int nt, const std::vector<double>& gx,
             const std::vector<double>& gw, kry_stats* st, double* max_err) {
  const int m = c->opts.krylov_dim;
  const int q = kRstNodes;
  const double dt = T / nt;
  const int ldh = m + 1;
  const int nc = (int)cols.size();
  const bool gpu = m <= kry::rst_march_max_m();
  const size_t ldf = (size_t)nt * q;
  // the sampled time functions: computed on the device for the GPU march
  // (nc nt q samples, two trigonometric evaluations each), on the host for
  // the host march
  auto sample_host = [&](std::vector<double>& f0) {
    f0.assign((size_t)nc * ldf, 0.0);
    for (int k = 0; k < nc; ++k)
      for (int j = 0; j < nt; ++j)
        for (int i = 0; i < q; ++i) {
          const double t = (j + gx[i]) * dt;
          f0[(size_t)k * ldf + (size_t)j * q + i] =
              cols[k].ca * std::sin(cols[k].w * t) + cols[k].cb * std::cos(cols[k].w * t);
        }
  };
  // device buffers: samples (2 nc ldf), packed propagators E, W, El, Wl,
  // the Gauss weights and E^L, u(T) per time function, residual integrals,
  // index map, and the chunk states of the parallel-in-time march (chunks of
  // L steps, L ~ sqrt(nt / 2): a chain of about 2 L + nt / L dependent steps)
  const int Lc = std::max(16, (int)std::ceil(std::sqrt(nt / 2.0)));
  const bool chunked = gpu && Lc < nt;
  const size_t npk = 2 * (size_t)m * m + 2 * (size_t)m * q + (size_t)q * q + q;
  const long long nwork = chunked ? kry::rst_march_work(m, nt, nc, Lc) : 0;
  double *dF = nullptr, *dP = nullptr, *dU = nullptr, *dR = nullptr, *dWk = nullptr, *dSw = nullptr;
  int* dMap = nullptr;
  // pinned host staging of each restart's small transfers (propagators,
  // residual integrals, active list, output map), so they queue behind the
  // march and the combination without a host round trip in between; reused
  // after the restart's stream synchronisation
  void* hpin = nullptr;
  Defer<std::function<void()>> free_bufs{[&]() {
    hipFree(dF);
    hipFree(dP);
    hipFree(dU);
    hipFree(dR);
    hipFree(dMap);
    hipFree(dWk);
    hipFree(dSw);
    if (hpin) hipHostFree(hpin);
  }};
  if (hipHostMalloc(&hpin, sizeof(double) * (npk + nc) + sizeof(int) * 2 * (size_t)nc, hipHostMallocDefault) !=
      hipSuccess) {
    hpin = nullptr;
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate the restarted method's pinned staging");
  }
  double* h_pk = (double*)hpin;
  double* h_rs = h_pk + npk;
  int* h_act = (int*)(h_rs + nc);
  int* h_cmap = h_act + nc;
  std::vector<double> hF[2];
  std::vector<double> sw;  // nodes and (w, ca, cb) per time function; kept until the function returns
  if (gpu) {
    if (hipMalloc(&dF, sizeof(double) * 2 * nc * ldf) != hipSuccess || hipMalloc(&dP, sizeof(double) * npk) != hipSuccess ||
        hipMalloc(&dU, sizeof(double) * (size_t)m * nc) != hipSuccess || hipMalloc(&dR, sizeof(double) * nc) != hipSuccess ||
        hipMalloc(&dMap, sizeof(int) * nc) != hipSuccess ||
        hipMalloc(&dSw, sizeof(double) * ((size_t)q + 3 * (size_t)nc)) != hipSuccess ||
        (nwork > 0 && hipMalloc(&dWk, sizeof(double) * nwork) != hipSuccess)) {
      (void)hipGetLastError();
      return fail(c, KRY_ENOMEM, "cannot allocate the sampled sources of the restarted method");
    }
    sw.assign((size_t)q + 3 * (size_t)nc, 0.0);
    std::copy(gx.begin(), gx.end(), sw.begin());
    for (int k = 0; k < nc; ++k) {
      sw[q + 3 * (size_t)k] = cols[k].w;
      sw[q + 3 * (size_t)k + 1] = cols[k].ca;
      sw[q + 3 * (size_t)k + 2] = cols[k].cb;
    }
    KRY_HIP(hipMemcpyAsync(dSw, sw.data(), sizeof(double) * sw.size(), hipMemcpyHostToDevice, c->stream));
    KRY_HIP(kry::launch_rst_samples(nc, nt, q, dt, dSw, dSw + q, dF, (long long)ldf, c->stream));
  } else {
    sample_host(hF[0]);
    hF[1].assign(hF[0].size(), 0.0);
  }
  const int maxcyc = c->opts.max_restarts > 0 ? c->opts.max_restarts : 100000;
  int rc = ensure_y(c, m + 1, nc);
  if (rc) return rc;
  kry::RstProp P;
  std::vector<int> act, cmap;
  std::vector<double> uT, Yh, rs;
  int cur = 0;
  int status = KRY_ENOCONV;
  for (int cyc = 0; cyc < maxcyc; ++cyc) {
    double beta = 0.0;
    int me = 0;
    rc = arnoldi(c, m, &beta, &me);
    if (rc) return rc;
    if (st) { st->matvecs_transient += m; st->steps_transient += 1; }
    if (me == 0) {  // the source vector vanished: nothing left
      status = KRY_OK;
      break;
    }
    const double hnext = me < m ? 0.0 : c->h_H[m + (size_t)(m - 1) * ldh];
    // E^L = e^{-L dt H} for the carry between chunks of the GPU march, on a
    // second host thread while the step propagators are formed (the two
    // dense computations are independent; joined on every path below)
    std::vector<double> Xel, Eel;
    std::thread th_el;
    Defer<std::function<void()>> join_el{[&]() {
      if (th_el.joinable()) th_el.join();
    }};
    if (gpu && chunked) {
      Xel.resize((size_t)me * me);
      Eel.resize((size_t)me * me);
      for (int jj = 0; jj < me; ++jj)
        for (int ii = 0; ii < me; ++ii) Xel[ii + (size_t)jj * me] = -(double)Lc * dt * c->h_H[ii + (size_t)jj * ldh];
      th_el = std::thread([&]() { kry::expm(me, Xel.data(), Eel.data()); });
    }
    kry::rst_prepare(me, c->h_H, ldh, q, dt, gx.data(), &P);
    act.clear();
    for (int k = 0; k < nc; ++k)
      if (cols[k].active) act.push_back(k);
    const int na = (int)act.size();
    cmap.assign(na, 0);
    for (int a = 0; a < na; ++a) cmap[a] = cols[act[a]].out;
    rs.assign(na, 0.0);
    const double* Ydev = c->d_Y;
    if (gpu) {
      double* p = h_pk;
      std::copy(P.E.begin(), P.E.end(), p);
      std::copy(P.W.begin(), P.W.end(), p + (size_t)me * me);
      std::copy(P.El.begin(), P.El.end(), p + (size_t)me * me + (size_t)me * q);
      std::copy(P.Wl.begin(), P.Wl.end(), p + (size_t)me * me + 2 * (size_t)me * q);
      std::copy(gw.begin(), gw.end(), p + (size_t)me * me + 2 * (size_t)me * q + (size_t)q * q);
      double* pEL = p + (size_t)me * me + 2 * (size_t)me * q + (size_t)q * q + q;
      if (chunked) {  // E^L from the second thread
        th_el.join();
        std::copy(Eel.begin(), Eel.end(), pEL);
      }
      const double* dE = dP;
      const double* dW = dP + (size_t)me * me;
      const double* dEl = dW + (size_t)me * q;
      const double* dWl = dEl + (size_t)q * me;
      const double* dgw = dWl + (size_t)q * q;
      const double* dEL = dgw + q;
      std::copy(act.begin(), act.end(), h_act);
      KRY_HIP(hipMemcpyAsync(dP, h_pk, sizeof(double) * npk, hipMemcpyHostToDevice, c->stream));
      KRY_HIP(hipMemcpyAsync(dMap, h_act, sizeof(int) * na, hipMemcpyHostToDevice, c->stream));
      KRY_HIP(kry::launch_rst_march(me, q, nt, na, dE, dW, dEl, dWl, dgw, beta, hnext, dt, dMap,
                                    dF + (size_t)cur * nc * ldf, dF + (size_t)(cur ^ 1) * nc * ldf, (long long)ldf,
                                    dU, dR, c->stream, chunked ? Lc : 0, chunked ? dEL : nullptr, dWk));
      KRY_HIP(hipMemcpyAsync(h_rs, dR, sizeof(double) * na, hipMemcpyDeviceToHost, c->stream));
      Ydev = dU;
    } else {
      uT.assign((size_t)me * na, 0.0);
      parallel_columns(na, [&](int a) {
        const double* fi = hF[cur].data() + (size_t)act[a] * ldf;
        double* fo = hF[cur ^ 1].data() + (size_t)act[a] * ldf;
        kry::rst_march(P, nt, 1, beta, hnext, gw.data(), &fi, &fo, &uT[(size_t)a * me], &rs[a]);
      });
      KRY_HIP(hipMemcpyAsync(c->d_Y, uT.data(), sizeof(double) * uT.size(), hipMemcpyHostToDevice, c->stream));
    }
    // y(T) += V_m u(T) for every active time function, one sweep of the basis
    std::copy(cmap.begin(), cmap.end(), h_cmap);
    KRY_HIP(hipMemcpyAsync(c->d_colmap, h_cmap, sizeof(int) * na, hipMemcpyHostToDevice, c->stream));
    hipEvent_t e = tbeg(c);
    if (na >= 32 && me <= 80)  // many outputs: on the matrix cores, the basis read once per 32 outputs
      KRY_HIP(kry::launch_combine_mfma(c->st, c->V, c->ldv, me, Ydev, na, c->Z, c->ldv, c->d_colmap, c->n,
                                       c->stream));
    else
      KRY_HIP(kry::launch_combine(c->st, c->V, c->ldv, me, Ydev, na, c->Z, c->ldv, c->d_colmap, 1, c->g,
                                  c->stream));
    tend(c, e, KRY_K_COMBINE, vbytes(c) * (me + 2.0 * na));
    // residual integral against the column's share of tol |y(T)|_M.  The
    // output norms (a sweep over every active column) are refreshed only
    // when some residual integral is within 16 times of its threshold at
    // the last norms (or none are known yet); until then no time function
    // can stop.
    bool any = false;
    KRY_HIP(hipStreamSynchronize(c->stream));  // rs is on the host now
    if (gpu) std::copy(h_rs, h_rs + na, rs.begin());
    bool near = false;
    for (int a = 0; a < na; ++a) {
      const RstColumn& cl = cols[act[a]];
      near |= !(cl.ynorm > 0.0) || rs[a] <= 16.0 * cl.share * c->opts.tol * cl.ynorm;
    }
    std::vector<double> yns;
    if (near || me < m) {
      rc = zcol_norms(c, cmap, yns);
      if (rc) return rc;
    }
    for (int a = 0; a < na; ++a)
      if (!std::isfinite(rs[a])) {
        *max_err = INFINITY;
        return fail(c, KRY_ENOCONV, "non-finite residual in the restarted inhomogeneous Krylov method");
      }
    for (int a = 0; a < na; ++a) {
      RstColumn& cl = cols[act[a]];
      cl.resint = rs[a];
      if (!yns.empty()) cl.ynorm = yns[a];
      const double yn = cl.ynorm;
      const double rel = yn > 0.0 ? cl.resint / yn : (cl.resint > 0.0 ? INFINITY : 0.0);
      if (cl.resint <= cl.share * c->opts.tol * yn || me < m) {
        cl.active = false;
        *max_err = std::max(*max_err, rel);
      } else {
        any = true;
      }
    }
    cur ^= 1;
    if (c->opts.verbose && (cyc + 1) % 5 == 0)
      std::fprintf(stderr, "[kry] restarted inhomogeneous Krylov: restart %d, %d time functions active\n",
                   cyc + 1, (int)std::count_if(cols.begin(), cols.end(), [](const RstColumn& x) { return x.active; }));
    if (!any) {
      status = KRY_OK;
      break;
    }
    // next start vector g = v_{m+1} (energy norm 1)
    KRY_HIP(hipMemcpyAsync(slot(c, 0), slot(c, m), c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
  }
  if (status == KRY_ENOCONV) {
    std::vector<int> zc;
    std::vector<double> yns;
    for (auto& cl : cols)
      if (cl.active) zc.push_back(cl.out);
    rc = zcol_norms(c, zc, yns);
    if (rc) return rc;
    int a = 0;
    for (auto& cl : cols) {
      if (!cl.active) continue;
      const double yn = yns[a++];
      *max_err = std::max(*max_err, yn > 0.0 ? cl.resint / yn : INFINITY);
    }
    fail(c, KRY_ENOCONV, "restart limit reached in the restarted inhomogeneous Krylov method");
  }
  return status;
}

// Zero-start solution over [0, Tw] of y' = -A y + Im(e^{i w t} b) for one
// complex source column by the restarted method, into Z column zout; each
// real part stops at tol_rel / 2 (per part) of its |y(Tw)|_M.  *rel_err
// receives the largest residual integral relative to |y(Tw)|_M.
int rst_window(kry_ctx* c, const double* bcol, double w, double Tw, int zout, double tol_rel,
               kry_stats* st, double* rel_err) {
  KRY_HIP(hipMemsetAsync(zcol(c, zout), 0, c->ldv * c->esz, c->stream));
  *rel_err = 0.0;
  if (!(Tw > 0.0)) return KRY_OK;
  const int nt = std::max(1, (int)std::ceil(Tw * (c->rho + w) / 0.5));
  std::vector<double> gx(kRstNodes), gw(kRstNodes);
  kry::gauss_legendre01(kRstNodes, gx.data(), gw.data());
  double nrm2[2] = {0.0, 0.0};
  for (int part = 0; part < 2; ++part) {
    KRY_HIP(kry::launch_load_complex(c->st, bcol, part, slot(c, 0), c->n, c->stream));
    std::vector<double> d;
    int rc = host_dots(c, slot(c, 0), nullptr, 0, d);
    if (rc) return rc;
    nrm2[part] = d[0];
  }
  const int parts = (nrm2[0] > 0.0) + (nrm2[1] > 0.0);
  int status = KRY_OK;
  for (int part = 0; part < 2; ++part) {
    if (!(nrm2[part] > 0.0)) continue;
    std::vector<RstColumn> cols{RstColumn{zout, w, part == 0 ? 1.0 : 0.0, part == 0 ? 0.0 : 1.0,
                                          0.5 / parts * tol_rel / c->opts.tol}};
    KRY_HIP(kry::launch_load_complex(c->st, bcol, part, slot(c, 0), c->n, c->stream));
    const int rc = rst_part(c, cols, Tw, nt, gx, gw, st, rel_err);
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
  }
  return status;
}

// Source splitting (equation (split2)): for a subinterval length dT that is
// a whole number of periods of the source, the zero-start solution w2 over
// [0, dT] is the same on every subinterval, so with y_0 = 0
//   y(k dT) = e^{-dT A} y((k-1) dT) + w2(dT),   k = 1..N,  N = floor(T / dT),
// and a remainder r = T - N dT takes y(T) = e^{-r A} y(N dT) + w2(r) (the
// source restarts in phase at N dT).  w2 comes from the restarted method on
// the short window (no shifted solve); the homogeneous steps are the
// time-restarted exponential.  Error budget (energy norm, A dissipative, so
// e^{-tA} does not amplify): the error of w2 enters N times, so w2 is
// solved to tol / (4 N) of its norm; each of the N - 1 steps gets
// tol |y| / (4 N); the remainder's pieces tol / 4 each.
int api_solve_split2(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src, const double* b,
                     int32_t b_per_omega, double T, int32_t periods, double* yT, kry_stats* st) {
  int rc = check_multifreq_args(c, omegas, n_omega, n_src, b);
  if (rc) return rc;
  if (!yT) return fail(c, KRY_EINVAL, "null output");
  if (!(T >= 0.0) || !std::isfinite(T)) return fail(c, KRY_EINVAL, "invalid T");
  if (periods < 1) return fail(c, KRY_EINVAL, "periods per subinterval must be >= 1");
  for (int k = 0; k < n_omega; ++k)
    if (!(omegas[k] > 0.0)) return fail(c, KRY_EINVAL, "source splitting needs w > 0 (a period)");
  if (st) std::memset(st, 0, sizeof(*st));
  treset(c);
  const double t0 = now_ms();
  const int m = c->opts.krylov_dim;
  rc = ensure_basis(c, m);
  if (rc) return rc;
  rc = ensure_z(c, 2);  // Z columns: 0 = w2(dT), 1 = saved y(N dT), 2 = w2(r)
  if (rc) return rc;
  rc = ensure_y(c, m + 1, 1);
  if (rc) return rc;
  const double tol = c->opts.tol;
  const double one = 1.0;
  int status = KRY_OK;
  double max_err = 0.0;
  const int ncols = n_omega * n_src;
  auto add_z = [&](int zc) -> int {  // slot 0 += Z column zc
    KRY_HIP(hipMemcpyAsync(c->d_Y, &one, sizeof(double), hipMemcpyHostToDevice, c->stream));
    KRY_HIP(kry::launch_combine(c->st, zcol(c, zc), c->ldv, 1, c->d_Y, 1, slot(c, 0), c->ldv, nullptr, 1, c->g,
                                c->stream));
    KRY_HIP(hipStreamSynchronize(c->stream));
    return KRY_OK;
  };
  auto mnorm = [&](const void* x, double* out) -> int {
    std::vector<double> d;
    const int r = host_dots(c, x, nullptr, 0, d);
    *out = std::sqrt(std::max(d.empty() ? 0.0 : d[0], 0.0));
    return r;
  };
  for (int col = 0; col < ncols; ++col) {
    const double w = omegas[col / n_src];
    const double* bcol = b + (size_t)(b_per_omega ? col : col % n_src) * 2 * c->n;
    const double period = 2.0 * M_PI / w;
    const double dT = periods * period;
    int N = (int)std::floor(T / dT * (1.0 + 1e-13));
    double r = T - N * dT;
    if (r < 1e-12 * std::max(T, 1.0)) r = 0.0;
    double err_abs = 0.0;
    KRY_HIP(hipMemsetAsync(slot(c, 0), 0, c->ldv * c->esz, c->stream));
    if (N >= 1) {
      double rel_w2 = 0.0, nw2 = 0.0;
      rc = rst_window(c, bcol, w, dT, 0, tol / (4.0 * N), st, &rel_w2);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      rc = mnorm(zcol(c, 0), &nw2);
      if (rc) return rc;
      err_abs += N * rel_w2 * nw2;
      KRY_HIP(hipMemcpyAsync(slot(c, 0), zcol(c, 0), c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
      for (int k = 2; k <= N; ++k) {
        double yn = 0.0, e = 0.0;
        rc = mnorm(slot(c, 0), &yn);
        if (rc) return rc;
        if (yn > 0.0) {
          const double a = tol * yn / (4.0 * N);
          rc = expv_slot0(c, dT, 0.5 * a, 0.5 * a, st, &e);
          if (rc == KRY_ENOCONV) status = rc;
          else if (rc) return rc;
          err_abs += e;
        }
        rc = add_z(0);
        if (rc) return rc;
        if (c->opts.verbose && k % 10 == 0)
          std::fprintf(stderr, "[kry] source splitting: subinterval %d of %d\n", k, N);
      }
    }
    if (r > 0.0) {
      KRY_HIP(hipMemcpyAsync(zcol(c, 1), slot(c, 0), c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
      double rel_r = 0.0, nwr = 0.0;
      rc = rst_window(c, bcol, w, r, 2, 0.25 * tol, st, &rel_r);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      rc = mnorm(zcol(c, 2), &nwr);
      if (rc) return rc;
      err_abs += rel_r * nwr;
      KRY_HIP(hipMemcpyAsync(slot(c, 0), zcol(c, 1), c->ldv * c->esz, hipMemcpyDeviceToDevice, c->stream));
      double yn = 0.0, e = 0.0;
      rc = mnorm(slot(c, 0), &yn);
      if (rc) return rc;
      if (yn > 0.0) {
        rc = expv_slot0(c, r, 0.125 * tol * yn, 0.125 * tol * yn, st, &e);
        if (rc == KRY_ENOCONV) status = rc;
        else if (rc) return rc;
        err_abs += e;
      }
      rc = add_z(2);
      if (rc) return rc;
    }
    double yT_norm = 0.0;
    rc = mnorm(slot(c, 0), &yT_norm);
    if (rc) return rc;
    max_err = std::max(max_err, yT_norm > 0.0 ? err_abs / yT_norm : 0.0);
    KRY_HIP(kry::launch_store_real(c->st, slot(c, 0), yT + (size_t)col * c->n, c->n, c->stream));
  }
  KRY_HIP(hipStreamSynchronize(c->stream));
  if (st) {
    st->max_err_estimate = max_err;
    st->ms_total = st->ms_transient = now_ms() - t0;
    st->converged = status == KRY_OK;
    texport(c, st);
  }
  return status;
}

// Per-column sources b_c (b_per_omega): a real basis {s_j} of the span of
// all Re b_c, Im b_c in the energy inner product, by a pivoted Householder
// QR of their non-zero rows scaled by sqrt(M) (truncated where the pivot
// falls below 1e-4 tol of the largest column), so that b_c = sum_j
// (x_cj + i y_cj) s_j and the source of column c is sum_j [x_cj sin(w_c t) +
// y_cj cos(w_c t)] s_j.  Each s_j then drives one time function per column,
// and its sequence of bases serves all of them (Corollary 2): r sequences
// instead of two per column.  Column c's error budget is split evenly over
// the s_j it uses.  *used = 0 (and nothing solved) when the sources are not
// compressible: too many non-zero rows for the host factorisation, or a
// rank above 3/4 of the two real parts per column.
int rst_compressed(kry_ctx* c, const double* omegas, int n_omega, int n_src, const double* b, double T, int nt,
                   const std::vector<double>& gx, const std::vector<double>& gw, kry_stats* st, double* max_err,
                   int* used) {
  *used = 0;
  const int ncols = n_omega * n_src;
  const long long n = c->n;
  int rc = ensure_weights(c);
  if (rc) return rc;
  unsigned char* dmask = nullptr;
  int* didx = nullptr;
  double* dC = nullptr;
  void* SRC = nullptr;
  Defer<std::function<void()>> fr{[&]() {
    hipFree(dmask);
    hipFree(didx);
    hipFree(dC);
    hipFree(SRC);
  }};
  if (hipMalloc(&dmask, (size_t)n) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate the source row mask");
  }
  KRY_HIP(kry::launch_nonzero_rows(b, ncols, n, dmask, c->stream));
  std::vector<unsigned char> mask((size_t)n);
  KRY_HIP(hipMemcpyAsync(mask.data(), dmask, (size_t)n, hipMemcpyDeviceToHost, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  std::vector<int> idx;
  for (long long e = 0; e < n; ++e)
    if (mask[e]) idx.push_back((int)e);
  const int nr = (int)idx.size();
  const int q = 2 * ncols;
  if (nr == 0 || (double)nr * q > (double)(1 << 26)) return KRY_OK;  // empty, or above 512 MB
  if (hipMalloc(&didx, sizeof(int) * nr) != hipSuccess || hipMalloc(&dC, sizeof(double) * (size_t)nr * q) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate the source compression workspace");
  }
  KRY_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int) * nr, hipMemcpyHostToDevice, c->stream));
  KRY_HIP(kry::launch_gather_rows(b, ncols, n, didx, nr, c->d_w, dC, c->stream));
  std::vector<double> C((size_t)nr * q), Q((size_t)nr * q), Rf((size_t)q * q);
  KRY_HIP(hipMemcpyAsync(C.data(), dC, sizeof(double) * C.size(), hipMemcpyDeviceToHost, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  const int r = kry::qr_pivoted(nr, q, C.data(), 1e-4 * c->opts.tol, Q.data(), Rf.data());
  if (r < 1 || 4 * r > 3 * q) return KRY_OK;
  if (c->opts.verbose)
    std::fprintf(stderr, "[kry] %d per-column sources share %d real source vectors (%d non-zero rows)\n", ncols, r,
                 nr);
  // the basis vectors s_j, in the storage type
  const size_t vb = (size_t)c->ldv * c->esz;
  if (hipMalloc(&SRC, vb * r) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, KRY_ENOMEM, "cannot allocate the compressed sources");
  }
  KRY_HIP(hipMemsetAsync(SRC, 0, vb * r, c->stream));
  KRY_HIP(hipMemcpyAsync(dC, Q.data(), sizeof(double) * (size_t)nr * r, hipMemcpyHostToDevice, c->stream));
  KRY_HIP(kry::launch_scatter_basis(c->st, dC, nr, r, didx, c->d_w, SRC, c->ldv, c->stream));
  // sequences used per column (non-zero coefficients)
  std::vector<int> uses(ncols, 0);
  for (int j = 0; j < r; ++j)
    for (int k = 0; k < ncols; ++k)
      if (Rf[(size_t)j * q + 2 * k] != 0.0 || Rf[(size_t)j * q + 2 * k + 1] != 0.0) ++uses[k];
  int status = KRY_OK;
  for (int j = 0; j < r; ++j) {
    std::vector<RstColumn> cols;
    for (int k = 0; k < ncols; ++k) {
      const double x = Rf[(size_t)j * q + 2 * k], y = Rf[(size_t)j * q + 2 * k + 1];
      if (x == 0.0 && y == 0.0) continue;
      cols.push_back(RstColumn{k, omegas[k / n_src], x, y, 0.5 / std::max(uses[k], 1)});
    }
    if (cols.empty()) continue;
    KRY_HIP(hipMemcpyAsync(slot(c, 0), (char*)SRC + vb * j, vb, hipMemcpyDeviceToDevice, c->stream));
    rc = rst_part(c, cols, T, nt, gx, gw, st, max_err);
    if (rc == KRY_ENOCONV) status = rc;
    else if (rc) return rc;
    if (c->opts.verbose)
      std::fprintf(stderr, "[kry] compressed source %d of %d done\n", j + 1, r);
  }
  *used = 1;
  return status;
}

int api_solve_restarted(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src, const double* b,
                        int32_t b_per_omega, double T, double* yT, kry_stats* st) {
  int rc = check_multifreq_args(c, omegas, n_omega, n_src, b);
  if (rc) return rc;
  if (!yT) return fail(c, KRY_EINVAL, "null output");
  if (!(T >= 0.0) || !std::isfinite(T)) return fail(c, KRY_EINVAL, "invalid T");
  if (st) std::memset(st, 0, sizeof(*st));
  treset(c);
  const double t0 = now_ms();
  const int m = c->opts.krylov_dim;
  rc = ensure_basis(c, m);
  if (rc) return rc;
  const int ncols = n_omega * n_src;
  rc = ensure_z(c, (ncols + 1) / 2);
  if (rc) return rc;
  for (int k = 0; k < ncols; ++k) KRY_HIP(hipMemsetAsync(zcol(c, k), 0, c->ldv * c->esz, c->stream));
  int status = KRY_OK;
  double max_err = 0.0;
  if (T > 0.0) {
    // time grid: the projected matrices and the sources carry frequencies
    // up to rho (the curl part's imaginary extent) plus the largest w; a
    // step of 0.5 / that bandwidth makes the degree-7 interpolant through 8
    // Gauss nodes exact to about 1e-12 relative
    double wmax = 0.0;
    for (int k = 0; k < n_omega; ++k) wmax = std::max(wmax, omegas[k]);
    const int nt = std::max(1, (int)std::ceil(T * (c->rho + wmax) / 0.5));
    std::vector<double> gx(kRstNodes), gw(kRstNodes);
    kry::gauss_legendre01(kRstNodes, gx.data(), gw.data());
    // per-column sources: try one real basis of all of them (the sequences
    // of bases then serve every column, Corollary 2)
    bool done = false;
    if (b_per_omega && ncols >= 2) {
      int used = 0;
      rc = rst_compressed(c, omegas, n_omega, n_src, b, T, nt, gx, gw, st, &max_err, &used);
      if (rc == KRY_ENOCONV) status = rc;
      else if (rc) return rc;
      done = used != 0;
    }
    // one group of time functions per (source, part)
    const int ngroups = done ? 0 : (b_per_omega ? ncols : n_src);
    for (int gi = 0; gi < ngroups; ++gi) {
      const double* bcol = b + (size_t)gi * 2 * c->n;
      double nrm2[2] = {0.0, 0.0};
      for (int part = 0; part < 2; ++part) {
        KRY_HIP(kry::launch_load_complex(c->st, bcol, part, slot(c, 0), c->n, c->stream));
        std::vector<double> d;
        rc = host_dots(c, slot(c, 0), nullptr, 0, d);
        if (rc) return rc;
        nrm2[part] = d[0];
      }
      const int parts = (nrm2[0] > 0.0) + (nrm2[1] > 0.0);
      for (int part = 0; part < 2; ++part) {
        if (!(nrm2[part] > 0.0)) continue;
        const double ca = part == 0 ? 1.0 : 0.0, cb = part == 0 ? 0.0 : 1.0;
        std::vector<RstColumn> cols;
        if (b_per_omega) {
          cols.push_back(RstColumn{gi, omegas[gi / n_src], ca, cb, 0.5 / parts});
        } else {
          for (int k = 0; k < n_omega; ++k)
            cols.push_back(RstColumn{k * n_src + gi, omegas[k], ca, cb, 0.5 / parts});
        }
        KRY_HIP(kry::launch_load_complex(c->st, bcol, part, slot(c, 0), c->n, c->stream));
        rc = rst_part(c, cols, T, nt, gx, gw, st, &max_err);
        if (rc == KRY_ENOCONV) status = rc;
        else if (rc) return rc;
      }
    }
  }
  for (int k = 0; k < ncols; ++k)
    KRY_HIP(kry::launch_store_real(c->st, zcol(c, k), yT + (size_t)k * c->n, c->n, c->stream));
  KRY_HIP(hipStreamSynchronize(c->stream));
  if (st) {
    st->max_err_estimate = max_err;
    st->ms_total = st->ms_transient = now_ms() - t0;
    st->converged = status == KRY_OK;
    texport(c, st);
  }
  return status;
}

// ---------------------------------------------------------------------------
// Arnoldi that allocates nothing, for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its per-workgroup partial sums, reduction buffers,
// normalisation scalars and Hessenberg matrix live in `scratch`, one
// fixed-size array per device, which holds them until the process ends.
// Every call on a device shares that device's array (its contents are
// those of the last call), so calls that overlap on one device race.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch;  // device ordinal -> that device's `scratch`

// The address of `scratch` on the current device (looked up once per
// device).  In host code the array's name only stands in for the symbol:
// kernels and copies get this address, never the name.
int scratch_on_current_device(double** out, std::string* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return KRY_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    *out = it->second;
    return KRY_OK;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return KRY_EHIP;
  }
  g_scratch[dev] = static_cast<double*>(p);
  *out = static_cast<double*>(p);
  return KRY_OK;
}

// m steps of Arnoldi (classical Gram-Schmidt twice, one operator
// application per step, equation (Arn)) from v, written straight into the
// caller's V_out (column j at offset j n, context storage type): column
// j + 1 serves as the work vector of step j, so nothing beyond the inputs,
// outputs and `scratch` is touched.
int api_arnoldi_noalloc(kry_ctx* c, const double* v, int32_t m, void* V_out, double* H_out,
                        double* beta_out) {
  if (!c || !v || !V_out || !H_out || !beta_out) return fail(c, KRY_EINVAL, "null argument");
  if (m < 1 || m + 2 > kry::kMaxCoef) return fail(c, KRY_EINVAL, "invalid m");
  double* scr = nullptr;
  std::string err;
  int rc = scratch_on_current_device(&scr, &err);
  if (rc) return fail(c, rc, err);
  const long long n = c->n;
  const int np_s = kry::cell_blocks(c->g.N3, c->g.cpt_s);
  const int np_d = kry::cell_blocks(c->g.N3, c->g.cpt_d);
  auto up = [](size_t x) { return (x + 31) / 32 * 32; };  // 256-byte pieces
  const size_t n_part = up((size_t)std::max(np_s, np_d) * (size_t)(m + 1));
  const size_t n_red = up((size_t)m + 2);
  const size_t n_h = (size_t)(m + 1) * m;
  const size_t need = n_part + 2 * n_red + 32 + up(n_h);
  if (need > kScratchDoubles)
    return fail(c, KRY_EINVAL,
                "grid and m need " + std::to_string(need * sizeof(double)) +
                    " bytes of scratch; the allocation-free Arnoldi has " +
                    std::to_string(kScratchBytes));
  double* partials = scr;
  double* red1 = partials + n_part;
  double* red2 = red1 + n_red;
  double* scal = red2 + n_red;  // scal[0] = 1/nu, scal[2] = 1/beta, scal[3] = beta
  double* H = scal + 32;
  hipStream_t s = c->stream;
  char* V = static_cast<char*>(V_out);
  auto col = [&](int j) { return (void*)(V + (size_t)j * n * c->esz); };
  // H starts at zero (a fill kernel, not a memset: callers may capture this)
  KRY_HIP(kry::launch_fill(H, 0.0, (long long)n_h, s));
  KRY_HIP(kry::launch_load_real(c->st, v, col(0), n, s));
  KRY_HIP(kry::launch_dots(c->st, col(0), nullptr, n, 0, c->g, c->mats, partials, s));
  KRY_HIP(kry::launch_reduce(partials, np_d, 1, 1, red1, s));
  KRY_HIP(kry::launch_fin_start(red1, scal + 2, s));
  KRY_HIP(kry::launch_scale(c->st, col(0), scal + 2, col(0), n, s));
  for (int j = 0; j < m; ++j) {
    const int cnt = j + 1;
    void* W = col(j + 1);
    KRY_HIP(kry::launch_stencil(c->st, col(j), W, V, n, cnt, c->g, c->mats, partials, s));
    KRY_HIP(kry::launch_reduce(partials, np_s, cnt + 1, cnt + 1, red1, s));
    KRY_HIP(kry::launch_update(c->st, W, V, n, cnt, red1, nullptr, W, c->g, s));
    KRY_HIP(kry::launch_dots(c->st, W, V, n, cnt, c->g, c->mats, partials, s));
    KRY_HIP(kry::launch_reduce(partials, np_d, cnt + 1, cnt + 1, red2, s));
    KRY_HIP(kry::launch_fin_step(red1, red2, j, H, m + 1, scal, s));
    KRY_HIP(kry::launch_update(c->st, W, V, n, cnt, red2, scal, W, c->g, s));
  }
  double sc[4] = {0.0, 0.0, 0.0, 0.0};
  KRY_HIP(hipMemcpyAsync(H_out, H, sizeof(double) * n_h, hipMemcpyDeviceToHost, s));
  KRY_HIP(hipMemcpyAsync(sc, scal, sizeof(sc), hipMemcpyDeviceToHost, s));
  KRY_HIP(hipStreamSynchronize(s));
  *beta_out = sc[3];
  if (sc[3] == 0.0) return 0;
  for (int j = 0; j < m; ++j)
    if (H_out[j + 1 + (size_t)j * (m + 1)] == 0.0) return j + 1;
  return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// s-step block size by measurement: one restart cycle of krylov_dim steps,
// the cycle every solver here runs, from a fixed pseudo-random start vector,
// per candidate s.  A warm-up cycle sets the Newton shifts (Ritz values of
// the first cycle, as in a solve) and the best of three further cycles is
// kept; a candidate whose basis blocks trip the conditioning guard pays for
// its fallback in its own time.
namespace {

int api_autotune_sstep(kry_ctx* c, const int32_t* cand, int32_t ncand, int32_t* best, double* us) {
  if (!c || !cand || !best || !us || ncand < 1 || ncand > 16) return fail(c, KRY_EINVAL, "invalid argument");
  for (int i = 0; i < ncand; ++i)
    if (cand[i] < 0 || cand[i] > 64) return fail(c, KRY_EINVAL, "s candidates must be in 0..64");
  const int m = c->opts.krylov_dim;
  const int32_t saved = c->opts.s_step;
  int bi = -1;
  for (int i = 0; i < ncand; ++i) {
    c->opts.s_step = cand[i];
    int rc = ensure_basis(c, m);
    if (rc) {
      c->opts.s_step = saved;
      return rc;
    }
    treset(c);
    double t_best = 1e300;
    for (int rep = 0; rep < 4; ++rep) {
      KRY_HIP(kry::launch_fill_hash(slot(c, 0), c->st, c->n, 20170630u, c->stream));
      const double t0 = now_ms();
      double beta = 0.0;
      int me = 0;
      rc = arnoldi(c, m, &beta, &me);
      if (rc) {
        c->opts.s_step = saved;
        return rc;
      }
      KRY_HIP(hipStreamSynchronize(c->stream));
      if (rep > 0) t_best = std::min(t_best, now_ms() - t0);
    }
    us[i] = 1e3 * t_best;
    if (bi < 0 || us[i] < us[bi]) bi = i;
  }
  c->opts.s_step = cand[bi];
  treset(c);
  *best = cand[bi];
  return KRY_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported entry points.  Every body runs inside `guarded`, so no C++
// exception (a host allocation failure in a std::vector, std::string or
// std::map, or any other) crosses the C interface: it becomes KRY_ENOMEM or
// KRY_EINVAL with a message in kry_last_error.
namespace {

void note(kry_ctx* c, const char* msg) noexcept {
  try {
    if (c) c->err = msg; else g_create_err = msg;
  } catch (...) {
  }
}

template <typename F>
int guarded(kry_ctx* c, F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    note(c, "host allocation failed");
    return KRY_ENOMEM;
  } catch (const std::exception& e) {
    note(c, e.what());
    return KRY_EINVAL;
  } catch (...) {
    note(c, "unexpected host exception");
    return KRY_EINVAL;
  }
}

}  // namespace

extern "C" {

int kry_create(const kry_grid* grid, const double* eps, const double* mu, const double* sigma,
               const kry_opts* opts, kry_ctx** out) {
  return guarded(nullptr, [&] { return api_create(grid, eps, mu, sigma, opts, out); });
}

void kry_destroy(kry_ctx* c) {
  try {
    api_destroy(c);
  } catch (...) {
  }
}

const char* kry_last_error(const kry_ctx* c) { return api_last_error(c); }

int kry_column_stats(const kry_ctx* c, int32_t col, kry_col_stats* out) {
  if (!c || !out) return KRY_EINVAL;
  if (col < 0 || col >= (int32_t)c->cols.size()) return KRY_EINVAL;
  *out = c->cols[col].s;
  return KRY_OK;
}

int kry_norm_series(const kry_ctx* c, int32_t col, double* t, double* norm, double* ms, int32_t cap) {
  if (!c || cap < 0) return KRY_EINVAL;
  if (col < 0 || col >= (int32_t)c->cols.size()) return KRY_EINVAL;
  const auto& r = c->cols[col];
  const int len = (int)r.t.size();
  for (int k = 0; k < std::min(cap, len); ++k) {
    if (t) t[k] = r.t[k];
    if (norm) norm[k] = r.norm[k];
    if (ms) ms[k] = r.ms[k];
  }
  return len;
}

int64_t kry_size(const kry_ctx* c) { return api_size(c); }

int kry_apply(kry_ctx* c, const double* v, double* w, int32_t ncols) {
  return guarded(c, [&] { return api_apply(c, v, w, ncols); });
}

int kry_apply_f32(kry_ctx* c, const float* v, float* w, int32_t ncols) {
  return guarded(c, [&] { return api_apply_f32(c, v, w, ncols); });
}

int kry_arnoldi(kry_ctx* c, const double* v, int32_t m, void* V_out, double* H_out, double* beta_out) {
  return guarded(c, [&] { return api_arnoldi(c, v, m, V_out, H_out, beta_out); });
}

int kry_expv(kry_ctx* c, double t, const double* v, double* y, int32_t ncols, kry_stats* st) {
  return guarded(c, [&] { return api_expv(c, t, v, y, ncols, st); });
}

int kry_stationary(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src, const double* b,
                   int32_t b_per_omega, double* z, kry_stats* st) {
  return guarded(c, [&] { return api_stationary(c, omegas, n_omega, n_src, b, b_per_omega, z, st); });
}

int kry_solve_multifreq(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src,
                        const double* b, int32_t b_per_omega, double T, double* yT, kry_stats* st) {
  return guarded(c, [&] {
    return api_solve_multifreq(c, omegas, n_omega, n_src, b, b_per_omega, T, yT, st);
  });
}

int kry_solve_restarted(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src,
                        const double* b, int32_t b_per_omega, double T, double* yT, kry_stats* st) {
  return guarded(c, [&] {
    return api_solve_restarted(c, omegas, n_omega, n_src, b, b_per_omega, T, yT, st);
  });
}

int kry_solve_split2(kry_ctx* c, const double* omegas, int32_t n_omega, int32_t n_src, const double* b,
                     int32_t b_per_omega, double T, int32_t periods, double* yT, kry_stats* st) {
  return guarded(c, [&] {
    return api_solve_split2(c, omegas, n_omega, n_src, b, b_per_omega, T, periods, yT, st);
  });
}

int kry_grad(kry_ctx* c, const double* omegas, int32_t n_omega, const double* b,
             int32_t b_per_omega, int32_t plane_k, double* loss, double* dL_deps, kry_stats* st) {
  return guarded(c, [&] {
    return api_grad(c, omegas, n_omega, b, b_per_omega, plane_k, loss, dL_deps, st);
  });
}

int kry_grad_transient(kry_ctx* c, const double* omegas, int32_t n_omega, const double* b,
                       int32_t b_per_omega, int32_t plane_k, double T, double* loss, double* dL_deps,
                       kry_stats* st) {
  return guarded(c, [&] {
    return api_grad_transient(c, omegas, n_omega, b, b_per_omega, plane_k, T, loss, dL_deps, st);
  });
}

int kry_arnoldi_noalloc(kry_ctx* c, const double* v, int32_t m, void* V_out, double* H_out,
                        double* beta_out) {
  return guarded(c, [&] { return api_arnoldi_noalloc(c, v, m, V_out, H_out, beta_out); });
}

int kry_block_arnoldi(kry_ctx* c, const double* V0, int32_t p, int32_t mb, void* V_out,
                      double* H_out) {
  return guarded(c, [&] { return api_block_arnoldi(c, V0, p, mb, V_out, H_out); });
}

int kry_set_tune(kry_ctx* c, const kry_tune* t) {
  return guarded(c, [&] { return api_set_tune(c, t); });
}

int kry_autotune_sstep(kry_ctx* c, const int32_t* cand, int32_t ncand, int32_t* best, double* us) {
  return guarded(c, [&] { return api_autotune_sstep(c, cand, ncand, best, us); });
}

int kry_autotune(kry_ctx* c, int32_t cnt, kry_tune* out) {
  return guarded(c, [&] { return api_autotune(c, cnt, out); });
}

}  // extern "C"
