/*
 * adef2.h - C ABI of the MI355X (gfx950) restricted-system A-DEF2 solver.
 *
 * Solves the restricted SPD system of a state-constrained optimal control
 * problem (paper: "Online Spectral Deflation for State Constrained Optimal
 * Control Problems", arXiv 2606.17971, Sec. 2 "Reduced inactive set system",
 * eq. (reduced)):
 *
 *      S_II x_I = b_I,      I = { i : active_mask[i] == 0 },
 *
 * with A-DEF2 deflated, Jacobi-preconditioned conjugate gradients (Alg. 1,
 * projected search directions; App. "CG stopping criterion"), using reference
 * modes Z computed once on the full domain and restricted to I online
 * (Sec. "Core idea: reference eigenmode basis", Alg. 3 "Online workflow").
 *
 * Conventions
 *   - Pointers documented as "device" point to device memory of the GPU that
 *     was current when the context was created; "host" pointers to host
 *     memory.  The caller owns every pointer it passes; the library copies
 *     what it keeps and owns its internal buffers.
 *   - All device work is ordered on the context's HIP stream.  Calls that fill
 *     host outputs synchronise that stream before returning.
 *   - Return codes: 0 = OK; < 0 = error (context unchanged, message in
 *     adef2_last_error); > 0 = warning with a valid, flagged result.
 *   - Vectors are in global order (length n).  Entries on the active set are
 *     ignored on input and returned as 0.
 *   - Operators must be banded/stencil matrices: at most ADEF2_MAX_DIAGS
 *     distinct diagonals (column - row offsets).  Others give
 *     ADEF2_E_UNSUPPORTED.  This is deliberate: every operator the paper
 *     builds is a finite-difference stencil on a structured grid (App.
 *     "Finite difference discretization"), and the diagonal format needs no
 *     column indices, so the restricted operator is a mask over the full
 *     grid and the matvec streams only coefficients and vectors.  A general
 *     sparse S would need a sliced-ELL restricted submatrix per instance.
 *   - Not thread-safe per context; distinct contexts are independent.
 */
#ifndef ADEF2_H
#define ADEF2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADEF2_MAX_DIAGS 32   /* distinct diagonals of S (A: 16)           */
#define ADEF2_MAX_K     64   /* deflation rank (shared + per-instance)   */

enum adef2_status {
  ADEF2_OK = 0,
  ADEF2_E_ARG = -1,         /* invalid argument (sizes, NaN, null pointer)  */
  ADEF2_E_STATE = -2,       /* call order: restrict before set_reference,
                               solve before restrict                         */
  ADEF2_E_HIP = -3,         /* HIP runtime error                             */
  ADEF2_E_NOMEM = -4,       /* device allocation failed                      */
  ADEF2_E_NOT_SPD = -5,     /* non-positive diagonal or breakdown (p.Sp<=0)  */
  ADEF2_E_UNSUPPORTED = -6, /* operator has more than ADEF2_MAX_DIAGS diags  */
  ADEF2_E_NOCONV = -7,      /* an iterative setup step (the eigensolver of
                               adef2_pod for M > 256) did not converge       */
  ADEF2_W_FALLBACK = 1,     /* cond(E) > tau_cond or Cholesky of E failed:
                               solved as plain Jacobi-PCG (Alg. 3, Remark
                               tau_cond)                                     */
  ADEF2_W_MAXIT = 2,        /* not converged within maxit; x = last iterate  */
  ADEF2_W_STAGNATED = 3     /* refinement modes: the FP64 residual b - S x
                               stopped decreasing above tol (its best value did
                               not halve over 4 outer steps whose segments
                               converged on their own equation, i.e. were not
                               stopped by segment_maxit): the attainable
                               accuracy of FP64 x was reached (when cond(S_II)
                               is ~1e10 the FP64 rounding of the exact solution
                               already has a relative residual ~1e-10); x is
                               the last iterate                              */
};

enum adef2_precision {
  ADEF2_FP64 = 0,           /* all vectors, S, Z and W in FP64 (the paper's
                               setting, App. "GPU implementation")           */
  ADEF2_FP32_REFINE = 1,    /* inner A-DEF2 segments with FP32 S, Z, W and
                               vectors (FP64 accumulation of dot products);
                               FP64 outer residual b - S x and FP64 x; the
                               k x k coarse algebra stays FP64               */
  ADEF2_MIXED_REFINE = 2,   /* as FP32_REFINE but with FP64 vectors: the
                               operator values and the Z / W panels (most of
                               the bytes) are FP32, every vector and every
                               accumulation FP64.  Needed when cond(S) is
                               beyond 1 / FP32 roundoff: an FP32 vector's own
                               rounding noise is then amplified by
                               lambda_max / lambda of the modes it carries  */
  ADEF2_FP64_REFINE = 3     /* FP64 segments (everything as in ADEF2_FP64),
                               each run until its recurrence residual is
                               below tol/2 (inner_rtol does not apply), then
                               the FP64 residual b - S x replaces it; the stop
                               is decided by the true residual.  For cond(S)
                               so large that the FP64 recurrence residual
                               drifts away from the true one (squared 3D
                               operators with coefficient jumps)             */
};

enum adef2_precond {
  ADEF2_JACOBI = 0,         /* K = diag(S_II)^{-1} (Sec. A-DEF2; App. stopping) */
  ADEF2_NONE = 1            /* identity (test option)                        */
};

typedef struct {
  double tau_cond;      /* solve-time fallback threshold on cond(E); 1e10
                           (Remark tau_cond)                                 */
  double drop_rel;      /* restricted-basis column dropped when its part
                           orthogonal to earlier columns is <= drop_rel times
                           its own norm; 1e-6.  With FP32 panels (refinement
                           modes) at least 1e-3: the independent part of a
                           column carries the FP32 rounding of the whole
                           column amplified by the inverse of that ratio     */
  int32_t maxit;        /* iteration cap (total over refinement sweeps);
                           100000 (App. "CG stopping criterion")             */
  int32_t precision;    /* enum adef2_precision                              */
  int32_t precond;      /* enum adef2_precond                                */
  double inner_rtol;    /* FP32_REFINE and MIXED_REFINE: a segment ends when its
                           recurrence residual fell to inner_rtol times the
                           FP64 residual it started from (or below tol/2
                           relative to ||b_I||); the FP64 residual b - S x
                           then replaces it and the search direction carries
                           on (residual replacement); 1e-2                   */
  int32_t max_sweeps;   /* refinement modes: cap on segments; 2000           */
  int32_t segment_maxit; /* refinement modes: a segment also ends after this
                           many iterations (periodic residual replacement);
                           < 0 = no cap, 0 = by precision (1000 with FP32
                           vectors, which drift from the FP64 residual; none
                           with FP64 vectors, where forced replacements
                           perturb CG near the accuracy floor).  The
                           direction is carried over unless the FP64
                           residual exceeds the segment's final recurrence
                           residual by more than 2x (drift), when the next
                           segment restarts; 0                              */
  int32_t check_every;  /* iterations per captured chunk (one HIP graph of
                           check_every iterations of every kernel); 32      */
  int32_t rows_per_thread; /* rows per thread of the per-instance iteration
                           kernels (tile height 256 or 512 rows): 1 or 2, or
                           0 = tuned on the first solve of each
                           configuration                                    */
  int32_t profile;      /* 1 = time kernels with HIP events (adef2_get_stats) */
  int32_t w_mode;       /* how the iteration forms W^T z (W = S_II Z_I):
                           1 = read the stored W; 2 = Z^T (S_II z), one more
                           stencil pass instead of reading W, with the FP64
                           operator and modes (z is rough, so FP32 rounding of
                           S or Z would be amplified by cond(S)), in
                           tile-major kernels that read each row of a shared
                           Z once for the whole batch (matrix-core panel
                           products); 3 = as 2 with per-instance kernels;
                           2 and 3 need FP64 vectors (E_UNSUPPORTED with
                           FP32_REFINE); 4 = tile-major boundary form: one
                           block per tile and group of instances updates
                           x, r, z and forms [Z^T z | Z^T r] for the whole
                           group on the matrix cores (the shared modes are
                           read once per group), with W^T z = Lambda Z^T z +
                           the boundary rows of W - Lambda Z (see
                           w_boundary); needs MIXED_REFINE, modes shared by
                           all instances that are all eigenvectors of the
                           reference operator, and w_boundary != 0
                           (E_UNSUPPORTED otherwise); 0 = tuned on the first
                           solve of each configuration (4 and 5 are
                           candidates whenever they apply); 5 = as 4 with the
                           stencil passes tile-major as well (coefficients of
                           a row read once for a group of instances; at most
                           16 diagonals per stencil).  Tuning runs every candidate for
                           the first 64 iterations from the same start, keeps
                           the fastest per context (batch size, precision,
                           basis width, operator form, N) and reuses it, so
                           repeated solves in one context are bitwise
                           reproducible                                     */
  int32_t w_boundary;   /* 1: with FP32 panels, reference modes that are
                           eigenvectors of the reference operator B
                           (||B z - mu z|| <= 1e-6 |mu| ||z||, tested at
                           set_reference) keep W = S_II Z_I as
                           W - lambda Z, lambda = a mu + c, which vanishes
                           except on inactive rows coupled to the active set
                           (up to the eigen-residual, of the order of the
                           FP32 rounding of W itself); the iteration then
                           reads W only on those rows and takes
                           lambda Z^T z from the shared modes.  2 (default):
                           as 1 when every shared reference mode passes the
                           test, else 0.  0: W stored and read whole      */
  int32_t graph;        /* 1 (default): each chunk of check_every iterations
                           is captured once into a HIP graph (per kernel
                           arguments) and replayed on a private stream of the
                           context, ordered against its stream by events;
                           0: kernels launched one by one.  profile = 1
                           launches one by one                             */
  int32_t ritz_keep;    /* Rayleigh-Ritz reselection (Sec. "Ritz
                           re-selection"): 0 (default) off; 0 < r: after
                           restriction and orthonormalisation the kept
                           columns form a candidate pool, and the r
                           eigenvectors of the pool's projected operator
                           with the smallest Ritz values become the
                           deflation basis (no effect when r >= the kept
                           columns).  cond(E) is then the ratio of the
                           largest to the smallest kept Ritz value, and
                           the deflation rank min(r, k_eff).  The iteration
                           kernels still read the whole pool.              */
  double tau_safe;      /* conditioning bound of the POD safe merge (Alg. 2):
                           the merge stops at the first candidate whose
                           trial basis has cond(Z^T S_II Z) > tau_safe; used
                           by adef2_pod_enrich when its tau_safe <= 0; 1e4
                           (Sec. "Conditioning-based safe merge")            */
  double tau_dep;       /* POD candidates whose part orthogonal to the columns
                           before them is at most tau_dep of their restricted
                           norm are skipped (Alg. 2); the effective bound is
                           max(drop_rel, tau_dep); 1e-10                     */
  int32_t poll_max;     /* chunks enqueued between two host polls, at most:
                           convergence is decided on the device (blocks of a
                           finished instance exit at once), and the host
                           enqueues as many chunks as the slowest iterating
                           instance is estimated to need (the decay of its
                           residual since the last poll, halved), between 1
                           and poll_max; 1 = poll after every chunk; 16    */
  int32_t learned_objective; /* training objective of the learned enrichment,
                           fixed when adef2_learned_prepare runs: 0 = energy
                           capture (the fraction of the solution's energy
                           the coarse correction with [Z_I, V_I] leaves);
                           1 = deflated spectrum (log of the sum of the
                           Ritz values of the Jacobi-preconditioned
                           operator, deflated by Z_I, on span(V_I):
                           small when V_I holds the slow modes that CG
                           would otherwise have to resolve); 0             */
  int32_t op_fused;     /* operator pass of the factored form S = alpha A^T A
                           + shift I inside the iteration: 1 = fused, one
                           kernel per iteration forms t = A p for a tile of
                           rows and the stencil reach around it in LDS and
                           applies A^T to it there (t never reaches HBM);
                           -1 = two passes (t = A p written to HBM, then
                           A^T t); 0 (default) = tuned on the first solve
                           of each configuration, after the tile height and
                           w_mode, whenever the fused pass applies, at
                           tile heights of 2, 4 and 8 times the stencil
                           reach, with one instance per block or (five-
                           point stencils, four LDS copies within 64 KiB)
                           four instances sharing each row's coefficients
                           (the fastest is kept; 1 takes 4 times the reach,
                           or the nearest that fits, one instance per
                           block).  It applies to the
                           factored form when a tile of twice the stencil
                           reach plus that reach on both sides fits 64 KiB
                           of LDS (2D grids up to about 2000 points wide;
                           not 3D grids, whose reach is a whole plane); 1
                           is E_UNSUPPORTED otherwise.  Same arithmetic per
                           row as the two passes; only the summation tree
                           of p.S p differs                                 */
  int32_t op_rows;      /* tile height of the fused operator pass in rows (a
                           multiple of 256): 0 = the candidates above (tuned)
                           or 4 times the reach (op_fused = 1); a tile and
                           its halo that do not fit give E_UNSUPPORTED; 0   */
  int32_t op_group;     /* instances per block of the fused pass: 1, or 4
                           (five-point stencils: the coefficients of a row
                           are loaded once for four instances, each with its
                           own LDS copy of A p, so four copies must fit 64
                           KiB); 0 = tuned (op_fused = 0) or 1 (op_fused =
                           1); 0                                            */
  int32_t sweep_async;  /* refinement modes: 1 (default) = an instance whose
                           segment ends starts its next one at the end of the
                           same chunk of iterations (correction, FP64
                           residual, outer test and the next segment's set-up
                           run inside the chunk, for the instances concerned
                           only), so no instance waits for the others'
                           segments; 0 = every instance's segment must end
                           before the host starts the next segment for all.
                           The arithmetic of every instance is the same
                           either way (same iterations, same x)             */
  int32_t update_ws;    /* update kernel of the tile-major boundary-form path
                           (w_mode 4 and 5, at most 32 modes): 1 = warp-
                           specialised, each block of 8 waves owns a run of
                           tiles, 4 waves update x, r, z of one tile while
                           the other 4 form the previous tile's projections
                           on the matrix cores (the products overlap the
                           loads; one partial sum per run and instance);
                           -1 = one block per tile; 0 (default) = tuned on
                           the first solve after the operator form.  1 is
                           E_UNSUPPORTED where the tile-major path does not
                           apply or above 32 modes                          */
} adef2_opts;

typedef struct adef2_ctx adef2_ctx;

/* Fill *opts with the defaults listed above. */
void adef2_default_opts(adef2_opts *opts);

/* Create a context on the current device.  opts may be NULL (defaults).
 * hip_stream: a hipStream_t (NULL = the default stream). */
int adef2_create(adef2_ctx **ctx, const adef2_opts *opts, void *hip_stream);
int adef2_destroy(adef2_ctx *ctx);
/* Replace the options (does not touch reference data or restrictions). */
int adef2_set_opts(adef2_ctx *ctx, const adef2_opts *opts);

/* Reference operator and modes (Sec. "Core idea", App. "Matrix assembly").
 *   n        : number of unknowns N.
 *   row_ptr  : device int64[n+1]; col_idx: device int32[nnz]; vals: device
 *              f64[nnz]: S in CSR, symmetric positive definite, sorted columns.
 *   k        : number of reference modes (0 <= k <= ADEF2_MAX_K).
 *   Z        : device f64[n*k], column-major (Z[j*n + i]); may be NULL if k = 0.
 * S is converted on the device to a diagonal format (FP64 + FP32 copies); Z is
 * copied (FP64 + FP32).  Invalidates any restriction. */
int adef2_set_reference(adef2_ctx *ctx, int64_t n, const int64_t *row_ptr,
                        const int32_t *col_idx, const double *vals, int64_t nnz,
                        int32_t k, const double *Z);

/* Reference operator given in the paper's Schur-complement form
 * M = alpha A^T A + shift I (Sec. "Reduced inactive set system", eq. schur,
 * with the mass-weighted scaling folded into alpha and shift).
 *   row_ptr, col_idx, vals: device CSR of the state operator A (n x n, any
 *   sparsity with at most 32 distinct diagonals; need not be symmetric).
 *   alpha > 0, shift >= 0; A must have full column rank when shift == 0.
 *   k, Z: as in adef2_set_reference.
 * The restricted operator is applied as S_II v = alpha A[:,I]^T (A[:,I] v) +
 * shift v (two stencil passes).  Its rounding error grows with cond(A) rather
 * than cond(A^T A), which keeps FP32 sweeps usable when cond(S) exceeds
 * 1 / FP32 unit roundoff.  Invalidates any restriction. */
int adef2_set_reference_factored(adef2_ctx *ctx, int64_t n, const int64_t *row_ptr,
                                 const int32_t *col_idx, const double *vals, int64_t nnz,
                                 double alpha, double shift, int32_t k, const double *Z);

/* Operator family S = a * S_ref + c * I applied to later restrict/solve calls,
 * S_ref being the operator of the last set_reference call (a > 0; S must stay
 * positive definite).  Default a = 1, c = 0. */
int adef2_set_operator_scale(adef2_ctx *ctx, double a, double c);

/* Inactive-set compaction (eq. reduced; App. "Matrix assembly and active set
 * restriction").  mask: device uint8[n] (1 = active, 0 = inactive).
 * Outputs (device): I int32[n] (first *n_inactive entries = inactive indices,
 * ascending), g2l int32[n] (position in I, or -1 where active).
 * n_inactive: host out.  Exact integer result. */
int adef2_compact(adef2_ctx *ctx, const uint8_t *mask, int64_t n, int32_t *I,
                  int32_t *g2l, int64_t *n_inactive);

/* adef2_compact without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same outputs as adef2_compact (I, g2l: device
 * int32[n], may be NULL); the count goes to n_inactive_dev (device int64[1],
 * may be NULL) and, when n_inactive (host) is not NULL, also to the host
 * after one synchronisation of the context's stream (pass NULL to stay
 * asynchronous, e.g. under capture).  Its chunk counts and offsets live in a
 * static device array of the library (520 KiB per GPU, held until the
 * process ends): n <= 2^28 (E_ARG beyond).  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other streams or threads) race;
 * calls ordered on one stream do not.  Nothing in it needs clearing: each
 * call writes the counts and offsets before reading them.  E_STATE when the
 * context's device is not current. */
int adef2_compact_noalloc(adef2_ctx *ctx, const uint8_t *mask, int64_t n, int32_t *I,
                          int32_t *g2l, int64_t *n_inactive_dev, int64_t *n_inactive);

/* Restrict to the inactive set of mask (device uint8[n]) and build the coarse
 * space: restricted modes Z_I, their orthonormalisation (CholQR with column
 * dropping, folded into the k x k coarse matrix), W = S_II Z_I,
 * E = Z^T S_II Z (orthonormal basis), cond(E) and its Cholesky factor
 * (Sec. A-DEF2; Alg. 3 restrict .. form E, fallback test).
 * n_inactive, k_eff, cond_E: host outs (may be NULL).  k_eff = 0 means the
 * fallback (plain Jacobi-PCG) will be used; cond_E is +inf when Cholesky of E
 * failed.  Returns ADEF2_W_FALLBACK in that case. */
int adef2_restrict(adef2_ctx *ctx, const uint8_t *active_mask, int64_t *n_inactive,
                   int32_t *k_eff, double *cond_E);

/* Solve S_II x_I = b_I for the current restriction.
 *   b  : device f64[n] (b on the active set ignored).
 *   x0 : device f64[n] warm start, or NULL for x0 = 0 (Remark warm start).
 *   tol: stop when ||b_I - S_II x_I||_2 <= tol ||b_I||_2 (recurrence residual,
 *        App. "CG stopping criterion"; in FP32_REFINE mode the FP64 residual).
 *   x  : device f64[n] out, 0 on the active set.
 *   iters, relres_true (||b - S x||/||b|| recomputed in FP64), cond_E: host
 *   outs (may be NULL).  iters counts CG iterations (all sweeps). */
int adef2_solve(adef2_ctx *ctx, const double *b, const double *x0, double tol,
                double *x, int32_t *iters, double *relres_true, double *cond_E);

/* Batched solve of B independent instances in one launch sequence (shared S
 * and Z; per-instance masks, operator scales, right-hand sides and
 * tolerances).
 *   masks: device uint8[B*n]; b, x: device f64[B*n] (instance-major).
 *   a, c : host f64[B] operator scales (S_m = a_m S_ref + c_m I), or NULL (1, 0).
 *   theta: device f32[B*4] problem parameters, or NULL.  When given (after
 *          adef2_pod / adef2_set_pod_modes and adef2_learned_set_params), each
 *          instance's coarse basis is [Z_I, V_I] with V = Phi C(theta)^T, the 8
 *          learned enrichment vectors; if cond(E) of that basis exceeds
 *          tau_learned (or its setup fails) the instance falls back to the
 *          plain restricted reference modes (Alg. 2's conditioning guard used
 *          as the safeguard of the learned addition).
 *   tol  : relative tolerance, as in adef2_solve.
 *   tol_each: host f64[B] per-instance tolerances replacing tol, or NULL.
 *          E_ARG when any tolerance is not positive and finite.
 *   iters, status (enum adef2_status per instance), relres_true, cond_E,
 *   n_inactive, learned (1 = learned vectors in use): host arrays of B entries
 *   (each may be NULL).
 * Returns the most severe per-instance status. */
int adef2_solve_batched(adef2_ctx *ctx, int32_t B, const uint8_t *masks,
                        const double *b, const double *a, const double *c,
                        const float *theta, double tol, const double *tol_each,
                        double *x, int32_t *iters, int32_t *status,
                        double *relres_true, double *cond_E, int64_t *n_inactive,
                        int32_t *learned);

/* ---- learned coarse-space enrichment (offline training on the device) ----
 * The enrichment vectors are V = Phi C^T, Phi = p POD modes of solution
 * snapshots (Sec. "Online POD enrichment": SVD of the mean-centred snapshot
 * matrix), C = MLP(theta) (8 x p; MLP 4 -> 128 -> 128 -> 8p, erf-GELU, BF16
 * weights, FP32 accumulation).  Training objective (opts.learned_objective):
 *   0: the fraction of the solution's energy norm that the A-DEF2 coarse
 *      correction with [Z_I, V_I] leaves unresolved,
 *      L = 1 - (b_Z^T G_ZZ^-1 b_Z + s^T (C H C^T)^-1 s) / b^T x;
 *   1: the deflated spectrum, L = log tr((C N C^T)^-1 C H C^T), the sum of
 *      the Ritz values of D^-1 S_II (D = diag(S_II)) on span(V_I) after the
 *      candidates are made S_II-orthogonal to Z_I;
 * H = P~^T S_II P~, N = P~^T D P~, s = C (P~^T b) with P~ = Phi_I - Z_I
 * G_ZZ^-1 G_ZP (Grams of [Z_I, Phi_I] under S_II).  Requires the factored
 * operator.  Parameter vector: 83200 FP32 values, packed
 * W1[128][4], b1[128], W2[128][128], b2[128], W3[512][128], b3[512]. */

/* POD modes of M snapshot columns X (device f64[n*M], column-major;
 * 2 <= M <= 8192, 1 <= p < M, p <= 64) by the method of snapshots: the
 * left singular vectors of the mean-centred snapshot matrix (Sec. "Online
 * POD enrichment") from the eigenpairs of its M x M Gram.  M <= 256: cyclic
 * Jacobi on the whole Gram.  M > 256: block subspace iteration with
 * Rayleigh-Ritz on p + max(32, p/2) columns until every wanted pair has
 * ||G v - theta v|| <= 1e-10 theta + 1e-13 theta_1 (E_NOCONV after 500
 * iterations; the count is in adef2_stats.pod_iters).  Device memory:
 * 8 (n M + 17 M^2) bytes at most while it runs.  Keeps Phi in the context;
 * Phi_out (device f64[n*p]) and sigma (host f64[p]) may be NULL. */
int adef2_pod(adef2_ctx *ctx, int32_t M, const double *X, int32_t p, double *Phi_out,
              double *sigma);
/* Use given POD modes (device f64[n*p], column-major) instead. */
/* Learned enrichment in one call (the paper's POD space, Sec. "Online POD
 * enrichment", with the network of the learned addition):
 *   p     : POD modes, 1 <= p <= 64; Phi: device f64[n*p], column-major
 *           (FP64: the expansion V = Phi C^T is formed in FP64 and rounded
 *           only for the FP32 panels of the refinement modes).
 *   mlp_params: host f32[83200] packed parameters (layout above; BF16 compute
 *           copies are made on the device), or NULL to keep the current ones.
 *   n_vec : enrichment vectors per instance; the network emits 8 (any other
 *           value gives E_UNSUPPORTED).
 *   tau_learned: cond(E) bound of the enriched basis (>= 1), as in
 *           adef2_learned_set_params.
 * E_STATE before set_reference, E_ARG for bad sizes or k + 8 > ADEF2_MAX_K. */
int adef2_set_enrichment(adef2_ctx *ctx, int32_t p, const double *Phi, const float *mlp_params,
                         int32_t n_vec, double tau_learned);
int adef2_set_pod_modes(adef2_ctx *ctx, int32_t p, const double *Phi);
/* MLP parameters (host f32[83200]); resets the Adam state.  tau_learned: the
 * cond(E) bound of the enriched basis (>= 1; 1e8 in the learned workload).
 * With FP32 panels (refinement modes) the bound used is at most 1.7e4, where
 * the FP32 coarse solve's error u32 cond(E) reaches 1e-3. */
int adef2_learned_set_params(adef2_ctx *ctx, const float *params, double tau_learned);
int adef2_learned_get_params(adef2_ctx *ctx, float *params);
/* Training samples: masks (device u8[M*n]), right-hand sides b and solutions
 * xsol (device f64[M*n]), theta (device f32[M*4]), operator scales (host, or
 * NULL).  Computes per sample H (p x p), g (p), b_Z^T G_ZZ^-1 b_Z, b^T x,
 * and N (p x p) when opts.learned_objective = 1; the objective is fixed for
 * these samples until the next call.  E_ARG when a sample has
 * b_I^T x_I <= 0 (x is not the solution, or b_I = 0); E_UNSUPPORTED when
 * k*k + k*(p+1) (+ k*p for objective 1) > 20352 (159 KiB of LDS; k = 64
 * with p = 64 fits both objectives). */
int adef2_learned_prepare(adef2_ctx *ctx, int32_t M, const uint8_t *masks, const double *b,
                          const double *xsol, const float *theta, const double *a,
                          const double *c);
/* Loss per prepared sample (host f64[M]) and the gradient of the mean loss
 * w.r.t. the parameters (host f32[83200]) at the current parameters. */
int adef2_learned_loss_grad(adef2_ctx *ctx, double *loss, float *grad);
/* steps full-batch Adam steps (Kingma & Ba 2015; beta 0.9/0.999, eps 1e-8);
 * loss_hist (host f64[steps], may be NULL) receives the mean loss per step. */
int adef2_learned_train(adef2_ctx *ctx, int32_t steps, float lr, double *loss_hist);
/* MLP outputs for M parameter vectors: theta device f32[M*4] -> out device
 * f32[M*512] (C row-major 8 x 64 per sample). */
int adef2_learned_forward(adef2_ctx *ctx, int32_t M, const float *theta, float *out);

/* y = S_II x on the current restriction (global layout, FP64); test hook for
 * the restricted operator.  x, y: device f64[n]. */
int adef2_apply_restricted(adef2_ctx *ctx, const double *x, double *y);

/* Coarse data of the current restriction: E in the orthonormalised basis of
 * the kept columns (host f64[k*k], leading k_eff x k_eff block, column-major),
 * kept column flags (host int32[k]).  Either may be NULL. */
int adef2_coarse_info(adef2_ctx *ctx, double *E, int32_t *kept, int32_t *k_eff,
                      double *cond_E);

/* Offline coarse-grid reference basis (Sec. "Coarse-grid eigenmode
 * prolongation", eq. (prolong), Alg. 4): r coarse-grid modes on the
 * nc^dim interior grid are interpolated linearly to the n^dim fine grid
 * (tensor product of the 1D interpolation with zero Dirichlet values,
 * coarse nodes at (j+1)/(nc+1)) and orthonormalised by two passes of
 * Cholesky QR; a column whose part orthogonal to the kept columns before it
 * is at most tau_sv times its own norm is dropped (the paper leaves tau_sv's
 * value open; 1e-10 is a sensible default).  Needs no reference operator.
 *   dim 2 or 3; Zc: device f64[r * nc^dim], column-major, lexicographic
 *   with x fastest; Z_out: device f64[r * n^dim], column-major: the first
 *   *r_out (host int32, may be NULL) columns are orthonormal, the rest 0.
 *   1 <= r <= ADEF2_MAX_K, 1 <= nc <= n, n^dim <= 2^31.
 * Returns E_ARG on bad sizes, E_NOT_SPD if every column is dropped. */
int adef2_prolong_basis(adef2_ctx *ctx, int32_t dim, int64_t n, int64_t nc, int32_t r,
                        const double *Zc, double tau_sv, double *Z_out, int32_t *r_out);

/* Reference eigenmodes on the GPU (the offline eigensolve of Sec. "Core
 * idea: reference eigenmode basis" and of the coarse grid in Alg. 4, which
 * the paper runs with ARPACK): the r smallest eigenpairs of the reference
 * operator by block inverse iteration with Rayleigh-Ritz.  Each step solves
 * S Y = X for the r columns with adef2_solve_batched (empty active sets, the
 * context's options and reference modes as deflation, tolerance inner_tol),
 * projects on span(Y) (E = Y^T X = Y^T S Y, G = Y^T Y) and takes the Ritz
 * vectors as the next block, until every relative residual
 * ||S z_j - lambda_j z_j|| / lambda_j (with S z_j from the solve) is <= tol.
 *   X0: device f64[r*n] start block (column-major, full rank);
 *   Z_out: device f64[r*n] orthonormal Ritz vectors, ascending Ritz values;
 *   lambda_out, resid_out: host f64[r] (may be NULL); iters_out: host int32.
 * The Ritz values of a block of r converge at the rate lambda_j /
 * lambda_{r+1}: take a few more columns than needed.  Returns W_MAXIT when
 * max_iter steps end first, E_NOT_SPD if the block loses rank. */
int adef2_reference_eigs(adef2_ctx *ctx, int32_t r, const double *X0, int32_t max_iter, double tol,
                         double inner_tol, double *Z_out, double *lambda_out, double *resid_out,
                         int32_t *iters_out);

/* Online POD enrichment with the conditioning-based safe merge (Sec.
 * "Online POD enrichment", Sec. "Conditioning-based safe merge", Alg. 2):
 * the first p POD modes held by ctx (adef2_pod or adef2_set_pod_modes)
 * become candidate columns after the k reference modes.  At every later
 * restriction each instance appends them in order (by decreasing singular
 * value): a candidate numerically inside the span of the columns before it
 * is skipped, and the first candidate whose trial basis gives
 * cond(Z^T S_II Z) > tau_safe ends the merge (1e4 in the paper).  For the
 * causal use the caller keeps the archive of past full-state solutions and
 * calls adef2_pod + adef2_pod_enrich between batches.  p = 0 restores the
 * reference modes alone.  Exclusive with the learned enrichment (a solve
 * with theta ignores the candidates' merge rule).
 * tau_safe <= 0 takes opts.tau_safe; candidates are also skipped below
 * opts.tau_dep (see adef2_opts).
 * Returns E_ARG for p < 0, k + p > ADEF2_MAX_K or 0 < tau_safe < 1; E_STATE
 * before set_reference or when fewer than p POD modes are held. */
int adef2_pod_enrich(adef2_ctx *ctx, int32_t p, double tau_safe);

/* Primal active-set iteration of the state-constrained problem (the
 * appendix algorithm on active-set identification, around eq. (reduced)) for
 * B instances on the reference operator M (a = 1, c = 0): cold start
 * y = 0, A = {}; each outer step fixes y_A = psi_A, solves
 * M_II y_I = (y_d)_I - M_IA psi_A with adef2_solve_batched (the instances
 * still iterating form the batch) and predicts A = {i : y_i > psi_i - tau};
 * an instance stops when the prediction repeats its active set.
 *   y_d, psi : device f64[B*n] desired state and bound, global order.
 *   tau      : active-set tolerance (1e-10 in the paper); tol: inner CG tolerance.
 *   y        : device f64[B*n] out, the state (psi on the active set).
 *   masks_out: device u8[B*n] out (1 = active), may be NULL.
 *   outer, inner_iters, status: host int32[B] (may be NULL): outer steps,
 *   CG iterations summed over them, and the worst inner status, raised to
 *   W_MAXIT when max_outer steps end without a repeat.
 * Returns the most severe per-instance status (negative = error). */
int adef2_active_set_batched(adef2_ctx *ctx, int32_t B, const double *y_d, const double *psi,
                             double tau, double tol, int32_t max_outer, double *y,
                             uint8_t *masks_out, int32_t *outer, int32_t *inner_iters,
                             int32_t *status);

/* Iteration-kernel variant used by the last solve on ctx: rows per thread
 * (1 or 2) and w_mode (1 .. 5 as in adef2_opts), whether fixed by the
 * options or tuned.  ms (host f32[10], may be NULL) receives the trial times
 * of the tuned candidates, rows per thread outer, w_mode inner, restricted to
 * the candidates tried (0 when not tuned).  E_STATE before the first solve. */
int adef2_variant(adef2_ctx *ctx, int32_t *rows_per_thread, int32_t *w_mode, float *ms);

/* Operator form used by the last solve on ctx (see opts.op_fused): fused
 * (1) or two passes (0), the fused pass's tile height in rows and its
 * instances per block (1, or 4 when the coefficients of a row are shared by
 * a group of instances; both 0 when not fused), and in ms (host f32[7], may
 * be NULL) the tuning trial times with the chosen rows per thread and
 * w_mode: ms[0] two passes, ms[1..3] the fused pass at tile heights of 2, 4
 * and 8 times the stencil reach (rounded up to 256 rows), ms[4..6] the same
 * with 4 instances per block (0 where a height does not fit or nothing was
 * tuned).  E_STATE before the first solve. */
int adef2_operator_variant(adef2_ctx *ctx, int32_t *fused, int32_t *tile_rows, int32_t *group, float *ms);

/* Update kernel used by the last solve on ctx (see opts.update_ws):
 * warp-specialised (1) or one block per tile (0), the tiles per block (0
 * when the tile-major path is not in use), and in ms (host f32[2], may be
 * NULL) the tuning trial times of the two forms (0 when not tuned).
 * E_STATE before the first solve. */
int adef2_update_variant(adef2_ctx *ctx, int32_t *warp_specialised, int32_t *tiles_per_block, float *ms);

#define ADEF2_STATS_KERNELS 24
typedef struct {
  int32_t n_kernels;            /* entries filled                           */
  const char *name[ADEF2_STATS_KERNELS];
  int64_t launches[ADEF2_STATS_KERNELS];
  double total_ms[ADEF2_STATS_KERNELS];  /* HIP-event time summed over launches */
  double alg_bytes[ADEF2_STATS_KERNELS]; /* algorithmic bytes summed over launches */
  int64_t polls;                /* host reads of the device convergence state
                                   (counted in every mode, not only profile) */
  int64_t pod_iters;            /* subspace iterations of the last adef2_pod
                                   (0: direct eigensolver, M <= 256)         */
} adef2_stats;

/* Per-kernel timings collected while opts.profile = 1, and the number of
 * host polls since the last reset. */
int adef2_get_stats(adef2_ctx *ctx, adef2_stats *stats);
int adef2_reset_stats(adef2_ctx *ctx);

/* Message of the last error on ctx (or of the last failed create when ctx is
 * NULL).  Valid until the next call on ctx. */
const char *adef2_last_error(const adef2_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADEF2_H */
