/*
 * Plain FP64 A-DEF2 deflated, Jacobi-preconditioned CG on a restricted
 * system S_II x = b_I given in CSR, with OpenMP loops over the rows.
 *
 * TEST INFRASTRUCTURE ONLY (CPU baseline and a second CPU check of the
 * Python oracle): only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code with the GPU library.
 *
 * The steps follow the projected reading of Alg. 1 (Sec. "Online deflated
 * solve (A-DEF2)") taken by the Python oracle: with an orthonormal basis Z of
 * the restricted reference modes, W = S Z, E = Z^T W (Cholesky, reused every
 * iteration, App. "GPU implementation"), K = diag(S_II)^{-1}:
 *   c0 = E^{-1} Z^T b;  x = Z c0;  r = b - W c0
 *   y  = K r - Z E^{-1} (W^T K r - Z^T r)       (y = P K r + Q r)
 *   p  = y;  rho = r.y
 *   while ||r|| > tol ||b|| and it < maxit      (App. "CG stopping criterion")
 *     w = S p;  alpha = rho / p.w;  x += alpha p;  r -= alpha w
 *     y = K r - Z E^{-1} (W^T K r - Z^T r);  rho' = r.y
 *     p = y + (rho' / rho) p;  rho = rho'
 * Dot products are OpenMP reductions; the k x k solves are serial.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* y = S x, CSR */
static void spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, const double* x,
                 double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * x[ci[e]];
    y[i] = s;
  }
}

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* g[q] = sum_i A[q][i] u[i] - B[q][i] v[i] for q < k (column-major n x k) */
static void panel_dots(int64_t n, int k, const double* A, const double* u, const double* B,
                       const double* v, double* g) {
  for (int q = 0; q < k; ++q) g[q] = 0.0;
  if (k == 0) return;
#pragma omp parallel
  {
    double* loc = (double*)calloc((size_t)k, sizeof(double));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const double ui = u[i], vi = v ? v[i] : 0.0;
      for (int q = 0; q < k; ++q) {
        double t = A[(size_t)q * n + i] * ui;
        if (B) t -= B[(size_t)q * n + i] * vi;
        loc[q] += t;
      }
    }
#pragma omp critical
    for (int q = 0; q < k; ++q) g[q] += loc[q];
    free(loc);
  }
}

/* lower Cholesky of the k x k matrix E (row-major, in place); 0 on success */
static int cholesky(int k, double* E) {
  for (int j = 0; j < k; ++j) {
    double d = E[j * k + j];
    for (int l = 0; l < j; ++l) d -= E[j * k + l] * E[j * k + l];
    if (!(d > 0.0)) return -1;
    d = sqrt(d);
    E[j * k + j] = d;
    for (int i = j + 1; i < k; ++i) {
      double s = E[i * k + j];
      for (int l = 0; l < j; ++l) s -= E[i * k + l] * E[j * k + l];
      E[i * k + j] = s / d;
    }
  }
  return 0;
}

/* c = E^{-1} g with the lower factor L (L L^T c = g) */
static void chol_solve(int k, const double* L, const double* g, double* c) {
  for (int i = 0; i < k; ++i) {
    double s = g[i];
    for (int l = 0; l < i; ++l) s -= L[i * k + l] * c[l];
    c[i] = s / L[i * k + i];
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = c[i];
    for (int l = i + 1; l < k; ++l) s -= L[l * k + i] * c[l];
    c[i] = s / L[i * k + i];
  }
}

/* out = base - Z c (or base + Z c with sign = +1), column-major Z */
static void combine(int64_t n, int k, const double* Z, const double* c, const double* base, double sign,
                    double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += Z[(size_t)q * n + i] * c[q];
    out[i] = (base ? base[i] : 0.0) + sign * s;
  }
}

/*
 * n, rp, ci, v : restricted CSR (rows sorted, diagonal present).
 * k, Z         : orthonormal restricted basis, column-major n x k (k may be 0).
 * b            : right-hand side (length n);  x: solution out (length n).
 * nthreads     : OpenMP threads (<= 0: the runtime's default).
 * Outputs: iters, converged (0/1), setup_s and solve_s (wall seconds of the
 * coarse setup and of the iteration).  Returns 0, or -1 when Cholesky of E
 * fails (the instance is then solved without deflation, as Alg. 3 falls back),
 * or -2 on allocation failure.
 */
int cpu_adef2(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, int32_t k,
              const double* Z, const double* b, double tol, int32_t maxit, int32_t nthreads, double* x,
              int32_t* iters, int32_t* converged, double* setup_s, double* solve_s) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const double t0 = omp_get_wtime();
  int rc = 0;
  double* dinv = (double*)malloc(sizeof(double) * n);
  double* r = (double*)malloc(sizeof(double) * n);
  double* z = (double*)malloc(sizeof(double) * n);
  double* y = (double*)malloc(sizeof(double) * n);
  double* p = (double*)malloc(sizeof(double) * n);
  double* w = (double*)malloc(sizeof(double) * n);
  double* W = (double*)malloc(sizeof(double) * (size_t)n * (k > 0 ? k : 1));
  double* E = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k * k : 1));
  double* g = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
  double* c = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
  if (!dinv || !r || !z || !y || !p || !w || !W || !E || !g || !c) { rc = -2; goto done; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double d = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
      if (ci[e] == i) d = v[e];
    dinv[i] = 1.0 / d;
  }
  /* coarse space: W = S Z, E = (Z^T W + W^T Z) / 2, Cholesky */
  for (int q = 0; q < k; ++q) spmv(n, rp, ci, v, Z + (size_t)q * n, W + (size_t)q * n);
  for (int a = 0; a < k; ++a)
    for (int bq = 0; bq <= a; ++bq) {
      const double e1 = dot(n, Z + (size_t)a * n, W + (size_t)bq * n);
      const double e2 = dot(n, Z + (size_t)bq * n, W + (size_t)a * n);
      E[a * k + bq] = E[bq * k + a] = 0.5 * (e1 + e2);
    }
  if (k > 0 && cholesky(k, E) != 0) { rc = -1; k = 0; }
  const double t1 = omp_get_wtime();
  /* deflated start */
  panel_dots(n, k, Z, b, NULL, NULL, g);
  if (k > 0) chol_solve(k, E, g, c);
  combine(n, k, Z, c, NULL, 1.0, x);          /* x = Z c0 */
  combine(n, k, W, c, b, -1.0, r);            /* r = b - W c0 */
  const double bnorm = sqrt(dot(n, b, b));
  int it = 0;
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(double) * n);
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    panel_dots(n, k, W, z, Z, r, g);
    if (k > 0) chol_solve(k, E, g, c);
    combine(n, k, Z, c, z, -1.0, y);
    double rho = dot(n, r, y);
    memcpy(p, y, sizeof(double) * n);
    while (sqrt(dot(n, r, r)) > tol * bnorm && it < maxit) {
      spmv(n, rp, ci, v, p, w);
      const double alpha = rho / dot(n, p, w);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * w[i];
        z[i] = dinv[i] * r[i];
      }
      panel_dots(n, k, W, z, Z, r, g);
      if (k > 0) chol_solve(k, E, g, c);
      combine(n, k, Z, c, z, -1.0, y);
      const double rho_new = dot(n, r, y);
      const double beta = rho_new / rho;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) p[i] = y[i] + beta * p[i];
      rho = rho_new;
      ++it;
    }
  }
  *iters = it;
  *converged = (bnorm == 0.0) || sqrt(dot(n, r, r)) <= tol * bnorm;
  *setup_s = t1 - t0;
  *solve_s = omp_get_wtime() - t1;
done:
  free(dinv); free(r); free(z); free(y); free(p); free(w); free(W); free(E); free(g); free(c);
  return rc;
}

int cpu_max_threads(void) { return omp_get_max_threads(); }
