/*
 * kry.h -- C ABI of the exponential-Krylov multi-frequency Maxwell solver.
 *
 * The library computes, for the semi-discrete Maxwell system
 *
 *     y'(t) = -A y(t) + Im(e^{i w t}) b,   y(0) = 0,               (1)
 *
 * (the ODE of the paper's Section 2.1, equation (ode), with the sinusoidal
 * source of equation (src) written for an angular frequency w), the field
 * y(T) through the time-harmonic / transient split of Corollary 3,
 * equation (split1):
 *
 *     y(T) = Im(e^{i w T} z) - e^{-T A} Im z,   z = (A + i w I)^{-1} b.
 *
 * A = M^{-1} (S + K) is the 3D Yee operator: K = [[0, C], [-C^T, 0]] with C
 * the discrete curl E -> H, S the per-cell conductivity on all six
 * components, M = diag(mu on H, eps on E) (the block form of the operator
 * after equation (ode)).  All Krylov bases are built by Arnoldi in the
 * energy inner product <x, y>_M = x^T M y, in which A is dissipative.
 *
 * Layout.  A state vector has n = 6 * nx * ny * nz entries: six planes
 * [Hx, Hy, Hz, Ex, Ey, Ez], each an nz x ny x nx array in C order (x
 * fastest).  Cell (i, j, k) owns Ex(i+1/2, j, k), Ey(i, j+1/2, k),
 * Ez(i, j, k+1/2), Hx(i, j+1/2, k+1/2), Hy(i+1/2, j, k+1/2),
 * Hz(i+1/2, j+1/2, k).  Stencil reads outside the grid are zero.
 * Several vectors ("columns") are stored one after another, column c at
 * offset c * n (c * 2n doubles for complex, interleaved re/im).
 *
 * Memory and streams.  Every pointer documented as "device" is a device
 * pointer owned by the caller; the library never frees it.  The context
 * owns its workspaces (Krylov basis, reduction buffers).  All work is
 * enqueued on the stream given in kry_opts; calls that return host data
 * (H matrices, statistics) synchronise that stream before returning.
 * A context is not thread-safe.
 *
 * Errors.  Every int-returning function returns 0 on success or one of the
 * negative KRY_E* codes; kry_last_error() then describes the failure.
 * No C++ exception crosses this interface: a host allocation failure
 * inside the library returns KRY_ENOMEM, any other host exception
 * KRY_EINVAL.
 */
#ifndef KRY_H
#define KRY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KRY_OK 0
#define KRY_EINVAL (-1)  /* invalid argument: sizes, NaN/Inf, eps <= 0, ... */
#define KRY_ENOMEM (-2)  /* device allocation failed or size out of range     */
#define KRY_EHIP (-3)    /* a HIP runtime call failed (message kept)          */
#define KRY_ENOCONV (-4) /* restart limit reached; outputs hold best estimate */

typedef struct kry_ctx kry_ctx;

typedef struct {
  int32_t nx, ny, nz; /* cells per axis, each >= 1                       */
  int32_t boundary;   /* 0: zero ghost values outside the grid (only mode) */
} kry_grid;

typedef struct {
  int32_t storage;      /* 0: FP64 fields and bases; 1: FP32 storage with
                           FP32 stencil, FP64 dots/norms/small dense       */
  int32_t krylov_dim;   /* Arnoldi steps per restart cycle m, 1..1024      */
  int32_t max_restarts; /* cap on restart cycles per solve (0: 100000)     */
  double tol;           /* relative accuracy target of each output column  */
  int32_t block_width;  /* batched form: 0 or 1 = one column at a time; B > 1
                           = columns processed in groups of B/2 sharing one
                           block Krylov space (2 real columns per complex
                           source), block Gram-Schmidt on matrix cores     */
  int32_t use_graph;    /* 1: each single-vector Arnoldi cycle is captured
                           once as a HIP graph and replayed (removes the
                           launch cost of small grids); ignored when
                           timing = 1                                     */
  int32_t inner_product;/* 0: energy inner product (the only mode)         */
  void* stream;         /* hipStream_t; NULL = the null stream             */
  int32_t timing;       /* 1: time every launch of the main kernel classes
                           with HIP events on the stream (about 4% of a
                           128^3 solve in host overhead); N > 1: time one
                           launch in N (counted over all classes in launch
                           order) and count every launch; 0: off.  Results
                           in kry_stats.kernel_*                           */
  int32_t block_steps;  /* batched form: block Arnoldi steps per restart of
                           the shifted solves (0: max(2, krylov_dim / p)) */
  int32_t block_steps_transient; /* batched form: 0 = transients one
                           column at a time (single-vector exponential);
                           k > 0 = block exponential, k block steps per
                           restart in time                                */
  int32_t verbose;      /* 1: one progress line on stderr per 20 restart
                           cycles / time steps (long solves)              */
  int32_t orth;         /* Gram-Schmidt: 0 = classical twice with the second
                           projection delayed by one step (two basis sweeps
                           per step, default); 1 = classical twice, both
                           projections in the step (four sweeps)          */
  int32_t s_step;       /* 0 or 1: one operator application per
                           Gram-Schmidt step (as chosen by orth); s in
                           2..64: s-step Arnoldi, s operator applications
                           build a basis block (Chebyshev in a call's first
                           restart cycle, then Newton steps on that cycle's
                           Ritz values in Leja order) that is
                           orthogonalised as one tall-skinny block (two
                           basis sweeps per pass; a second pass only where
                           the first leaves a loss of orthogonality of
                           order u cond^2 above 1e-11).  The block is FP64
                           also with FP32 storage (only the orthonormal
                           result is rounded to FP32; FP32 storage with
                           krylov_dim > 112 runs one step per sweep).  A
                           block whose triangular factor has a condition
                           estimate above 1e6 is redone one step per sweep
                           and halves s for the rest of the call          */
  int32_t omega_continuation; /* 1 (per-frequency sources only): each
                           column's shifted solve starts from the
                           extrapolation, in omega, of the same source's
                           solutions at up to three earlier frequencies of
                           the call, and only the correction is solved    */
  int32_t transient_continuation; /* 1: the transient of each column after
                           the first of a source is continued from the
                           previous column of that source (equation
                           (4diff), steps 4-6 of Fig. alg:spl1):
                           y_hat_next(T) = y_hat(T) + e^{-TA} (Im z_next -
                           Im z), each column's accumulated error estimate
                           kept within its own budget (a column starts a
                           new chain otherwise)                           */
  int32_t host_blocks;  /* s-step Arnoldi with FP64 storage: 0 = each block's
                           Gram-Schmidt factors, checks and coefficients on
                           the device, one host synchronisation per restart
                           cycle (blocks the host would treat apart send
                           the cycle to the host form); 1 = the host form,
                           one synchronisation per Gram-Schmidt pass       */
} kry_opts;

/* Kernel classes reported by the per-kernel timing. */
#define KRY_K_STENCIL 0 /* operator applications (fused with the first
                           Gram-Schmidt dots in the one-step Arnoldi; the
                           polynomial-basis stencil in the s-step one)    */
#define KRY_K_UPDATE 1  /* one-step Arnoldi: w -= V h (multi-vector update) */
#define KRY_K_DOTS 2    /* one-step Arnoldi: second Gram-Schmidt dot pass  */
#define KRY_K_COMBINE 3 /* basis combinations V Y                          */
#define KRY_K_GRAM 4    /* block form: Gram products V^T M W (matrix cores) */
#define KRY_K_GEMM 5    /* block form: updates W -= V C (matrix cores)      */
#define KRY_K_CLASSES 6

typedef struct {
  int64_t matvecs_stationary; /* operator applications, shifted solves     */
  int64_t matvecs_transient;  /* operator applications, exponential part   */
  int64_t cycles_stationary;  /* restart cycles of the shifted solves      */
  int64_t steps_transient;    /* restarts in time of the exponential part  */
  double max_residual;        /* largest final relative shifted residual   */
  double max_err_estimate;    /* largest transient error bound / |y|_M     */
  double ms_stationary;       /* wall time of the phases (host clock)      */
  double ms_transient;
  double ms_total;
  int32_t converged;          /* 1 if every column met its target          */
  /* filled when kry_opts.timing >= 1 (else zero), per kernel class:
     summed HIP-event durations, launches, algorithmic bytes (each
     vector read or written once, materials once per cell) and
     algorithmic FP64 flops of the matrix-core products (2 per
     multiply-add; zero for the streaming classes)                     */
  double kernel_ms[KRY_K_CLASSES];
  int64_t kernel_launches[KRY_K_CLASSES];
  double kernel_bytes[KRY_K_CLASSES];
  double kernel_flops[KRY_K_CLASSES];
  /* every launch of the class and its algorithmic bytes (the fields above
     cover the timed launches: all of them with timing = 1, one in N with
     timing = N)                                                        */
  int64_t kernel_launches_all[KRY_K_CLASSES];
  double kernel_bytes_all[KRY_K_CLASSES];
} kry_stats;

/* Per-column record of the last kry_solve_multifreq call on a context (the
 * single-vector path; other calls leave no records).  The metrics the paper
 * reports per run (residuals, restarts in time, the decay of |y_hat(t)|
 * that makes the split pay, Fig. `normy`), per output column. */
typedef struct {
  double omega;
  int32_t source;              /* source index; column = omega index * n_src + source */
  int32_t converged;           /* 1 if the column's shifted solve and transient met their targets */
  int64_t matvecs_stationary;  /* of the column's shifted-solve group (shared by its columns) */
  int64_t matvecs_transient;   /* this column's transient */
  int64_t steps_transient;     /* this column's restarts in time */
  double residual;             /* true relative shifted residual |b - (A + i w) z|_M / |b|_M of
                                  the returned z; NaN where the path does not compute it */
  double err_estimate;         /* transient error bound / |Im(e^{iwT} z)|_M */
  double harmonic_norm;        /* |Im(e^{iwT} z)|_M (time-harmonic part at T) */
  double ms_transient;         /* wall time of this column's transient and assembly */
  int32_t series_len;          /* samples in the column's |y_hat(t)| series */
  int32_t pad_;
} kry_col_stats;

/* Create a context for the grid and per-cell materials: the operator
 * A = M^{-1} (S + K) of the semi-discrete Maxwell system (Section 2.1,
 * equation (ode) and the block form of the operator after it: M holds the
 * permittivity and permeability, S the conductivity, K the curl pair; here
 * the 3D Yee curl with the same per-cell sigma on all six components).
 * eps, mu, sigma: device arrays of nx*ny*nz doubles (C order, x fastest).
 * mu may be NULL (mu = 1 everywhere), sigma may be NULL (sigma = 0).
 * eps > 0, mu > 0, sigma >= 0 and all finite, else KRY_EINVAL.
 * The arrays are copied into the context; the caller may free them after.
 * opts is copied.  On success *out holds the new context. */
int kry_create(const kry_grid* grid, const double* eps, const double* mu,
               const double* sigma, const kry_opts* opts, kry_ctx** out);

/* Free the context and all of its device memory. NULL is allowed. */
void kry_destroy(kry_ctx* ctx);

/* Message of the last failure on this context (or of the last failed
 * kry_create when ctx is NULL).  Valid until the next call on ctx. */
const char* kry_last_error(const kry_ctx* ctx);

/* Problem size n = 6 nx ny nz. */
int64_t kry_size(const kry_ctx* ctx);

/* w = A v for ncols columns (operator of equation (ode)); v, w device,
 * FP64, n x ncols.  v and w must not overlap. */
int kry_apply(kry_ctx* ctx, const double* v, double* w, int32_t ncols);

/* As kry_apply with FP32 vectors and FP32 arithmetic (the stencil of the
 * FP32-storage form). */
int kry_apply_f32(kry_ctx* ctx, const float* v, float* w, int32_t ncols);

/* m steps of Arnoldi in the energy inner product from the start vector v
 * (device, FP64, length n): V_{m+1} with V^T M V = I and the (m+1) x m
 * upper-Hessenberg H with A V_m = V_{m+1} H (equation (Arn), regular
 * Krylov, with v_1 = v / |v|_M as in equation (Krylov)).
 * V_out: device, (m+1) x n in the context's storage type (double or
 * float), column j at offset j*n.  H_out: host, (m+1) x m doubles,
 * column-major.  beta_out: host, |v|_M.  Returns the number of steps taken
 * (< m on an exact invariant subspace, h_{j+1,j} = 0), or a KRY_E* code. */
int kry_arnoldi(kry_ctx* ctx, const double* v, int32_t m, void* V_out,
                double* H_out, double* beta_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Arnoldi relation as kry_arnoldi, computed with classical Gram-Schmidt
 * twice and one operator application per step, without allocating
 * anything.  The basis is built in place in V_out (device, (m+1) x n in the
 * context's storage type, column j at offset j*n; column j+1 is the work
 * vector of step j), and every other intermediate (partial sums,
 * reductions, H) lives in a fixed 32 MiB array per device that the library
 * holds until the process ends.  H_out (host, (m+1) x m column-major) and
 * beta_out (host) as for kry_arnoldi; the call synchronises the context's
 * stream and returns the steps taken or a KRY_E* code.  Sizes whose partial
 * sums and H do not fit in the 32 MiB (about 8 (m+1) nx ny nz / 256 bytes
 * for the partials) give KRY_EINVAL.  All calls on one device share that
 * array, so calls that overlap on one device (several streams or threads)
 * race: the caller serialises them. */
int kry_arnoldi_noalloc(kry_ctx* ctx, const double* v, int32_t m, void* V_out, double* H_out,
                        double* beta_out);

/* Block Arnoldi: mb block steps from the start block V0 (device, FP64, p
 * columns of length n), the block form of equation (Arn) with p columns per
 * block.  Block Gram-Schmidt in the energy inner product runs on FP64
 * matrix cores (V^T M W and W - V C products), each new block is
 * orthonormalised by rank-revealing Cholesky QR twice (dependent directions
 * become zero columns).  V_out: device, (mb+1)*p columns of length n in the
 * context's storage type (block 0 = orthonormalised V0).  H_out: host,
 * ((mb+1) p) x (mb p) doubles, column-major, with A V_{mb} = V_{mb+1} H.
 * Returns the number of block steps taken (< mb if the block space became
 * invariant) or a KRY_E* code.  1 <= p <= 128. */
int kry_block_arnoldi(kry_ctx* ctx, const double* V0, int32_t p, int32_t mb, void* V_out,
                      double* H_out);

/* y = e^{-t A} v for ncols columns (equation (y_homo)), by restarts in time
 * with the residual of Lemma 1 (g = 0) bounding the error of each step.
 * v, y: device FP64, n x ncols (may alias). Target: |err|_M <= tol |v|_M. */
int kry_expv(kry_ctx* ctx, double t, const double* v, double* y,
             int32_t ncols, kry_stats* stats);

/* y(T) of problem (1) for every (w, source) pair, by Corollary 3.
 * omegas: host, n_omega angular frequencies (w >= 0).
 * b: device, complex interleaved (re, im) FP64 sources.  If b_per_omega is
 *    0, b holds n_src columns shared by every w; otherwise n_omega*n_src
 *    columns, column (w, s) at index w*n_src + s.
 * yT: device FP64, n x (n_omega*n_src), column (w, s) at w*n_src + s.
 * The shifted systems of the w that share a source are solved in real
 * Krylov sequences shared by groups of neighbouring w (at most 16, spanning
 * at most a tenth of their mean; restarted multi-shift method with the
 * residuals kept collinear across a group, cf. Corollaries 1 and 2); a
 * shift that diverges in its group is solved again alone, and every shift's
 * true residual is checked and corrected once where it misses the target.
 * The transients are then integrated per column.  stats: host, may be
 * NULL. */
int kry_solve_multifreq(kry_ctx* ctx, const double* omegas, int32_t n_omega,
                        int32_t n_src, const double* b, int32_t b_per_omega,
                        double T, double* yT, kry_stats* stats);

/* y(T) of problem (1) for every (w, source) pair by the residual-restarted
 * Krylov method for the inhomogeneous problem (Section 3, restarting in
 * Krylov dimension: equation (rst), Corollary 2 and the algorithm of
 * Fig. alg:rst, regular Krylov variant), with no shifted solve: each real
 * source part (Re b driven by sin(w t), Im b by cos(w t)) gets one sequence
 * of krylov_dim-step Arnoldi bases, shared by every w that drives it (the
 * bases do not depend on the time function, Corollary 2); per w the
 * projected problem (equation (corr2)) is solved on [0, T] with its source
 * sampled on a fine time grid, y(T) += V_m u(T), and the next restart
 * starts from v_{m+1} with the sampled residual function
 * -h_{m+1,m} e_m^T u(t) as its source (Lemma 1).  A w stops once the
 * integral over [0, T] of its residual norm, which bounds the energy-norm
 * error of y(T), is below tol/2 |y(T)|_M.  Arguments as for
 * kry_solve_multifreq; stats: matvecs_transient and steps_transient count
 * the operator applications and restarts, max_err_estimate the largest
 * residual integral relative to |y(T)|_M.  KRY_ENOCONV after max_restarts
 * restarts (outputs hold the current approximation). */
int kry_solve_restarted(kry_ctx* ctx, const double* omegas, int32_t n_omega, int32_t n_src,
                        const double* b, int32_t b_per_omega, double T, double* yT,
                        kry_stats* stats);

/* y(T) of problem (1) for every (w, source) pair by splitting off the
 * source term (equation (split2)): with a subinterval dT of `periods`
 * periods 2 pi / w of the source, the zero-start solution w2 over [0, dT]
 * is the same on every subinterval, so y(k dT) = e^{-dT A} y((k-1) dT) +
 * w2(dT) for k = 1..floor(T / dT), and a remainder r takes y(T) =
 * e^{-r A} y + w2(r).  w2 comes from the restarted method of
 * kry_solve_restarted on the window (no shifted solve), the steps from the
 * time-restarted exponential of kry_expv.  Each column is solved on its
 * own.  Arguments as for kry_solve_multifreq; every w must be > 0
 * (KRY_EINVAL otherwise); periods >= 1. */
int kry_solve_split2(kry_ctx* ctx, const double* omegas, int32_t n_omega, int32_t n_src,
                     const double* b, int32_t b_per_omega, double T, int32_t periods, double* yT,
                     kry_stats* stats);

/* Time-harmonic fields only: z_w = (A + i w I)^{-1} b for every column, the
 * vector z_stat of Corollary 3.  Same argument conventions as
 * kry_solve_multifreq; z: device, complex interleaved FP64,
 * n x (n_omega*n_src).  Target: shifted residual <= tol |b|_M. */
int kry_stationary(kry_ctx* ctx, const double* omegas, int32_t n_omega,
                   int32_t n_src, const double* b, int32_t b_per_omega,
                   double* z, kry_stats* stats);

/* Launch shapes of the streaming kernels: cells per thread (1, 2 or 4) of
 * the operator kernels (stencil), of the basis-update kernels and of the
 * dot-product kernels, with the timings (microseconds, best of several
 * launches, index 0/1/2 for 1/2/4 cells per thread) that chose them. */
typedef struct {
  int32_t cpt_stencil, cpt_update, cpt_dots;
  double us_stencil[3], us_update[3], us_dots[3];
  /* the s-step basis stencil: planes per workgroup of its z-marching form
     (4, 8 or 16), or 0 for the cell-parallel form with cpt_stencil cells
     per thread; us_stencil_zm: its times at 4, 8 and 16 planes (0 where
     not timed)                                                          */
  int32_t zm_stencil;
  int32_t pad_;
  double us_stencil_zm[3];
} kry_tune;

/* Time the operator kernel the solver runs (the s-step basis stencil when
 * opts.s_step > 1, which is the FP64 stencil on the FP64 work block under
 * either storage type, in its cell-parallel and its z-marching forms, else
 * the stencil fused with the first Gram-Schmidt dots), and the update and
 * dot kernels of one one-step Arnoldi step with
 * `cnt` basis vectors (0: krylov_dim / 2), for every launch shape on this
 * context's grid and workspace; apply the fastest per kernel class, and
 * report the choice and timings in *out (host).  Overwrites the context's
 * Krylov workspace (no solve may be in progress on the stream). */
int kry_autotune(kry_ctx* ctx, int32_t cnt, kry_tune* out);

/* Choose the s-step block size (opts.s_step) by measurement: one restart
 * cycle of krylov_dim Arnoldi steps, the cycle every solver runs, from a
 * fixed pseudo-random start vector, for each of the ncand candidates cand[i]
 * (0 or 1: one operator application per Gram-Schmidt step; 2..64: s-step
 * blocks); after a warm-up cycle (which sets the Newton shifts, as in a
 * solve) the best of three cycles counts, and a candidate whose blocks trip
 * the conditioning guard pays for its fallback.  The fastest candidate is
 * applied to the context and written to *best; us[i] (host) receives each
 * candidate's cycle time in microseconds.  1 <= ncand <= 16.  Overwrites the
 * context's Krylov workspace (no solve may be in progress on the stream). */
int kry_autotune_sstep(kry_ctx* ctx, const int32_t* cand, int32_t ncand, int32_t* best, double* us);

/* Apply a previously measured launch-shape choice (cpt_* fields of *t). */
int kry_set_tune(kry_ctx* ctx, const kry_tune* t);

/* Transmitted power and its gradient w.r.t. per-cell permittivity.
 * The loss is the period-averaged Poynting flux of the time-harmonic parts
 * Im(e^{i w t} z_w) of Corollary 3 through the plane z = plane_k, summed over
 * the frequencies:
 *     L = sum_w 1/2 Re sum_{i,j} [z_Ex conj(Hy_bar) - z_Ey conj(Hx_bar)],
 * Hbar = (z_H[plane_k - 1] + z_H[plane_k]) / 2 (the paper computes no
 * gradients; this is the differentiation form of the solver).  dL/d eps is
 * obtained with one adjoint shifted solve per frequency, (A^T + i w) lam =
 * dL/dz, solved as (A + i w) x = P M^{-1} dL/dz through the identity
 * A^T = M P A P M^{-1}, P = diag(I_H, -I_E); the forward fields z_w are the
 * saved state of the forward pass.
 * omegas: host, n_omega.  b: device complex interleaved FP64; one shared
 * column (b_per_omega = 0) or n_omega columns.  1 <= plane_k <= nz - 1.
 * loss: host, one double.  dL_deps: device, nx*ny*nz doubles (overwritten),
 * or NULL to evaluate the loss only (no adjoint solves).
 * Shifted residual target: opts.tol relative.  stats may be NULL. */
int kry_grad(kry_ctx* ctx, const double* omegas, int32_t n_omega, const double* b,
             int32_t b_per_omega, int32_t plane_k, double* loss, double* dL_deps,
             kry_stats* stats);

/* Record of column `col` of the last kry_solve_multifreq call (single-vector
 * path).  KRY_EINVAL if the last call left no record for col.  out: host. */
int kry_column_stats(const kry_ctx* ctx, int32_t col, kry_col_stats* out);

/* The |y_hat(t)|_M series of column `col` of the last kry_solve_multifreq
 * call: sample k is the start of the k-th restart in time of the transient
 * (t[k], |y_hat(t[k])|_M, and ms[k], the wall time of that restart), then a
 * last sample at the end (t = T or the time the remainder was dropped,
 * ms = 0).  Writes min(cap, len) samples into the host arrays (any may be
 * NULL) and returns len, the series' length, or a negative error code. */
int kry_norm_series(const kry_ctx* ctx, int32_t col, double* t, double* norm, double* ms, int32_t cap);

/* Flux at a finite time T, the transient included, and its gradient w.r.t.
 * per-cell permittivity.  The field is the whole solution of Corollary 3,
 * y_w(T) = Im(e^{i w T} z_w) - e^{-T A} Im z_w (equation (split1); the
 * transient solves the homogeneous problem (y_homo)), and the loss is its
 * instantaneous Poynting flux through the plane z = plane_k, summed over the
 * frequencies:
 *     L = sum_w sum_{i,j} [Ex Hy_bar - Ey Hx_bar](y_w(T)),
 * Hy_bar, Hx_bar the means of the H planes plane_k - 1 and plane_k (the
 * paper computes no gradients).  With g = dF/dy(T), dL/d eps has a term
 * through z (one adjoint shifted solve per frequency, right-hand side
 * e^{i w T} g - e^{-T A^T} g, by the identity A^T = M P A P M^{-1}) and a
 * term through e^{-TA}, the Frechet derivative of the exponential: the
 * integral over [0, T] of e^{-(T-s)A^T} g against (dA) e^{-sA} Im z.  Both
 * transients (forward from Im z, adjoint from P M^{-1} g) run by restarts
 * in time with the start vector of every step kept; each step's Krylov
 * basis is regenerated once from it, and the integral over every interval
 * where a forward and an adjoint step overlap is a small matrix of the two
 * projected problems, integrated by Gauss-Legendre panels on the host, and
 * applied per cell on the GPU.
 * Arguments as for kry_grad, plus T >= 0 (host).  Workspace allocated per
 * call: 2 (m + 3) vectors of the storage type, 3 FP64 n-vectors, and one
 * checkpoint vector per time step of each transient.  Targets: shifted
 * residuals opts.tol relative; each transient's error below opts.tol
 * relative to its start vector.  stats may be NULL. */
int kry_grad_transient(kry_ctx* ctx, const double* omegas, int32_t n_omega, const double* b,
                       int32_t b_per_omega, int32_t plane_k, double T, double* loss,
                       double* dL_deps, kry_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* KRY_H */
