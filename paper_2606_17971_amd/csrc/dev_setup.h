// Per-reference and per-restriction kernels: diagonal-format conversion,
// inactive-set compaction, W = S_II Z_I with the Gram matrices Z_I^T Z_I and
// Z_I^T W, and the one-workgroup k x k coarse setup.
#pragma once
#include "dev_vec.h"
#include "dev_tile.h"

namespace adef2 {

// ---------------------------------------------------------------------------
// compaction: I = { i : sel[i] == 0 } ascending, g2l, count   (exact)
// Three passes: per-chunk counts, scan of the counts, per-chunk scatter.
// ---------------------------------------------------------------------------
constexpr int CMP_ITEMS = 16;                 // items per thread
constexpr int CMP_CHUNK = TPB * CMP_ITEMS;    // items per block

__global__ void __launch_bounds__(TPB) k_compact_count(int64_t n, const uint8_t* sel, int* counts,
                                                       int nchunks) {
  const int m = blockIdx.y;
  const uint8_t* s = sel + (size_t)m * n;
  const int64_t base = (int64_t)blockIdx.x * CMP_CHUNK + (int64_t)threadIdx.x * CMP_ITEMS;
  int c = 0;
#pragma unroll
  for (int j = 0; j < CMP_ITEMS; ++j) {
    const int64_t i = base + j;
    if (i < n && s[i] == 0) ++c;
  }
  __shared__ int red[NWAVE];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NWAVE; ++w) t += red[w];
    counts[(size_t)m * nchunks + blockIdx.x] = t;
  }
}

// exclusive scan of counts (one block per instance); total -> totals[m]
__global__ void __launch_bounds__(TPB) k_compact_scan(const int* counts, int* offsets, int nchunks,
                                                      long long* totals, Inst* inst) {
  const int m = blockIdx.x;
  const int* c = counts + (size_t)m * nchunks;
  int* o = offsets + (size_t)m * nchunks;
  __shared__ int wsum[NWAVE];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int base = 0; base < nchunks; base += TPB) {
    const int j = base + threadIdx.x;
    const int v = j < nchunks ? c[j] : 0;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = carry;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    if (j < nchunks) o[j] = before + incl - v;
    __syncthreads();
    if (threadIdx.x == TPB - 1) carry = before + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (totals) totals[m] = carry;
    if (inst) inst[m].n_inactive = carry;
  }
}

__global__ void __launch_bounds__(TPB) k_compact_scatter(int64_t n, const uint8_t* sel,
                                                         const int* offsets, int nchunks, int* I,
                                                         int* g2l) {
  const int m = blockIdx.y;
  const uint8_t* s = sel + (size_t)m * n;
  const int64_t base = (int64_t)blockIdx.x * CMP_CHUNK + (int64_t)threadIdx.x * CMP_ITEMS;
  uint8_t f[CMP_ITEMS];
  int c = 0;
#pragma unroll
  for (int j = 0; j < CMP_ITEMS; ++j) {
    const int64_t i = base + j;
    f[j] = (i < n) ? (s[i] == 0) : 0;
    c += f[j];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = c;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  __shared__ int wsum[NWAVE];
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int pos = offsets[(size_t)m * nchunks + blockIdx.x] + incl - c;
  for (int w = 0; w < wid; ++w) pos += wsum[w];
  int* Im = I ? I + (size_t)m * n : nullptr;
  int* Gm = g2l ? g2l + (size_t)m * n : nullptr;
#pragma unroll
  for (int j = 0; j < CMP_ITEMS; ++j) {
    const int64_t i = base + j;
    if (i < n) {
      if (f[j]) {
        if (Im) Im[pos] = (int)i;
        if (Gm) Gm[i] = pos;
        ++pos;
      } else if (Gm) {
        Gm[i] = -1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// CSR -> diagonal format
// ---------------------------------------------------------------------------
// flags[off + n - 1] = 0 for every diagonal offset present (flags preset to 1)
__global__ void k_mark_offsets(int64_t n, const int64_t* rp, const int* col, uint8_t* flags,
                               int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
    const int64_t j = col[e];
    if (j < 0 || j >= n) { *bad = 1; continue; }
    flags[j - i + n - 1] = 0;
  }
}

// which = 0: offsets op.offs (assembled S, diag = main diagonal, must be > 0);
// which = 1: offsets op.offs1 (factor A of S = alpha A^T A + c I; diag unused)
__global__ void k_csr_to_dia(int64_t n, const int64_t* rp, const int* col, const double* val,
                             OpGeom op, int which, double* dia64, float* dia32, double* diag,
                             int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int D = which ? op.D1 : op.D;
  const int* offs = which ? op.offs1 : op.offs;
  double dg = 0.0, rs = 0.0;
  int slot0 = -1;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
    const int off = (int)((int64_t)col[e] - i);
    int lo = 0, hi = D - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] < off) lo = mid + 1; else hi = mid;
    }
    if (offs[lo] != off) { *bad = 1; continue; }
    const double v = val[e];
    if (!(v == v) || v == INFINITY || v == -INFINITY) *bad = 2;
    dia64[(size_t)lo * n + i] = v;
    dia32[(size_t)lo * n + i] = (float)v;
    rs += v;
    if (off == 0) { dg = v; slot0 = lo; }
  }
  // FP32 copy in difference form: the offset-0 slot holds the FP64 row sum
  // (also for a row that has no diagonal entry of its own)
  for (int d = 0; d < D; ++d)
    if (offs[d] == 0) slot0 = d;
  if (slot0 >= 0) dia32[(size_t)slot0 * n + i] = (float)rs;
  if (!which) {
    diag[i] = dg;
    if (!(dg > 0.0)) *bad = 3;
  }
}

// A^T in diagonal format from A: A^T[i, i - o] = A[i - o, i], and row i - o
// of A holds that entry in its diagonal d (offset o = offs1[d]) at position
// i - o; so diagonal d' = D1-1-d of A^T (offset -offs1[d]) holds
// A[d][i - offs1[d]].  Also the diagonal of A^T A (squared column norms of A)
// for the Jacobi preconditioner.
__global__ void k_dia_transpose(OpGeom op, const double* A64, double* AT64, float* AT32, double* diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = op.N;
  if (i >= n) return;
  double cn = 0.0, rs = 0.0;
  int slot0 = -1;
  for (int d = 0; d < op.D1; ++d) {
    const int64_t j = i - op.offs1[d];
    const double v = (j >= 0 && j < n) ? A64[(size_t)d * n + j] : 0.0;
    const int dt = op.D1 - 1 - d;
    AT64[(size_t)dt * n + i] = v;
    AT32[(size_t)dt * n + i] = (float)v;
    cn += v * v;
    rs += v;
    if (op.offs1[d] == 0) slot0 = dt;   // offsets of A^T are -offs1: offset 0 maps to itself
  }
  // FP32 copy in difference form (row sum of A^T in the offset-0 slot)
  if (slot0 >= 0) AT32[(size_t)slot0 * n + i] = (float)rs;
  diag[i] = cn;
}

// T[m][q] = A Ztilde[q] on all rows, Ztilde = Z with the active rows of
// instance m set to zero (factored operator, setup of W).
__global__ void k_stencil_modes(OpGeom op, const double* A64, const double* Z64, int64_t zs,
                                const uint8_t* mask, int KP, double* T) {
  const int q = blockIdx.y;
  const int m = blockIdx.z;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const uint8_t* mk = mask + (size_t)m * N;
  const double* Zq = Z64 + (size_t)m * zs + (size_t)q * N;
  double acc = 0.0;
  for (int e = 0; e < op.D1; ++e) {
    const int64_t j = i + op.offs1[e];
    if (j >= 0 && j < N && mk[j] == 0) acc += A64[(size_t)e * N + i] * Zq[j];
  }
  T[((size_t)m * KP + q) * N + i] = acc;
}

// ---------------------------------------------------------------------------
// Reference modes as eigenvectors of the base operator B (A^T A for the
// factored form, the assembled stencil otherwise): BZ = B Z on the full
// domain, then per column the Rayleigh quotient mu_q = z^T B z / z^T z and
// the flag eig_q = ||B z - mu_q z|| <= tol |mu_q| ||z||.
// ---------------------------------------------------------------------------
__global__ void k_ref_inner(OpGeom op, const double* A64, const double* Z64, double* T) {
  const int q = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const double* Zq = Z64 + (size_t)q * N;
  double acc = 0.0;
  for (int e = 0; e < op.D1; ++e) {
    const int64_t j = i + op.offs1[e];
    if (j >= 0 && j < N) acc += A64[(size_t)e * N + i] * Zq[j];
  }
  T[(size_t)q * N + i] = acc;
}

__global__ void k_ref_outer(OpGeom op, const double* dia64, const double* src, double* BZ) {
  const int q = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const double* sq = src + (size_t)q * N;
  double acc = 0.0;
  for (int d = 0; d < op.D; ++d) {
    const int64_t j = i + op.offs[d];
    if (j >= 0 && j < N) acc += dia64[(size_t)d * N + i] * sq[j];
  }
  BZ[(size_t)q * N + i] = acc;
}

// one block per column; two passes (mu first, then the residual) so that the
// residual is not a difference of nearly equal sums
__global__ void __launch_bounds__(TPB) k_ref_stats(int64_t N, int k, const double* Z64, const double* BZ,
                                                   double tol, double* mu, uint8_t* eig) {
  __shared__ double red[TPB / 64 * 2];
  __shared__ double tot[2];
  const int q = blockIdx.x;
  const double* z = Z64 + (size_t)q * N;
  const double* bz = BZ + (size_t)q * N;
  double v[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < N; i += TPB) {
    v[0] += z[i] * bz[i];
    v[1] += z[i] * z[i];
  }
  block_sum<2, TPB / 64>(v, red, tot);
  const double zz = tot[1];
  const double m = zz > 0.0 ? tot[0] / zz : 0.0;
  double r[1] = {0.0};
  for (int64_t i = threadIdx.x; i < N; i += TPB) {
    const double e = bz[i] - m * z[i];
    r[0] += e * e;
  }
  __syncthreads();
  block_sum<1, TPB / 64>(r, red, tot);
  if (threadIdx.x == 0) {
    mu[q] = m;
    eig[q] = (q < k && zz > 0.0 && sqrt(tot[0]) <= tol * fabs(m) * sqrt(zz)) ? 1 : 0;
  }
}

// Rows of the inactive set whose row of S couples to the active set: there
// W = S_II Z_I differs from (S Z)_I = Z_I Lambda.  Factored S: h_l = row l of
// A touches an active column; boundary_i = row i of A^T touches an l with h_l.
__global__ void k_bnd_inner(OpGeom op, const double* A64, const uint8_t* masks, uint8_t* h) {
  const int m = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const uint8_t* mk = masks + (size_t)m * N;
  uint8_t f = 0;
  for (int e = 0; e < op.D1; ++e) {
    const int64_t j = i + op.offs1[e];
    if (j >= 0 && j < N && mk[j] && A64[(size_t)e * N + i] != 0.0) f = 1;
  }
  h[(size_t)m * N + i] = f;
}

__global__ void k_bnd_outer(OpGeom op, const double* dia64, const uint8_t* masks, const uint8_t* src,
                            uint8_t* bnd) {
  const int m = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const uint8_t* mk = masks + (size_t)m * N;
  const uint8_t* sm = src + (size_t)m * N;
  uint8_t f = 0;
  if (mk[i] == 0)
    for (int d = 0; d < op.D; ++d) {
      const int64_t j = i + op.offs[d];
      if (j >= 0 && j < N && sm[j] && dia64[(size_t)d * N + i] != 0.0) f = 1;
    }
  bnd[(size_t)m * N + i] = f;
}

// ---------------------------------------------------------------------------
// Offline coarse-grid reference basis (Sec. "Coarse-grid eigenmode
// prolongation", eq. (prolong), Alg. 4)
// ---------------------------------------------------------------------------
// 1D linear interpolation weights of fine node i: coarse nodes at positions
// (j+1)/(nc+1), zero values at 0 and 1.  Integer arithmetic locates the
// interval exactly.  lo/hi are coarse indices (-1: boundary, weight unused).
__device__ __forceinline__ void hat_weights(int64_t i, int64_t n, int64_t nc, int64_t* lo, double* wlo,
                                            int64_t* hi, double* whi) {
  const int64_t num = (i + 1) * (nc + 1);
  const int64_t j = num / (n + 1);                 // left node, 0 = boundary
  const double w = (double)(num - j * (n + 1)) / (double)(n + 1);
  *lo = (j >= 1 && j <= nc) ? j - 1 : -1;
  *wlo = 1.0 - w;
  *hi = (j + 1 >= 1 && j + 1 <= nc && w != 0.0) ? j : -1;
  *whi = w;
}

// Pt[q][i] = (P Zc[q])(i) with P the tensor product of the 1D operator
// (lexicographic, x fastest); dim 2 or 3
__global__ void k_prolong(int dim, int64_t n, int64_t nc, const double* Zc, double* Pt) {
  const int q = blockIdx.y;
  const int64_t Nf = dim == 2 ? n * n : n * n * n;
  const int64_t Nc = dim == 2 ? nc * nc : nc * nc * nc;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nf) return;
  int64_t lo[3], hi[3];
  double wl[3], wh[3];
  int64_t rem = i;
  for (int d = 0; d < dim; ++d) {
    hat_weights(rem % n, n, nc, &lo[d], &wl[d], &hi[d], &wh[d]);
    rem /= n;
  }
  const double* z = Zc + (size_t)q * Nc;
  double acc = 0.0;
  const int ncorner = 1 << dim;
  for (int cidx = 0; cidx < ncorner; ++cidx) {
    int64_t off = 0, stride = 1;
    double wt = 1.0;
    bool ok = true;
    for (int d = 0; d < dim; ++d) {
      const bool up = (cidx >> d) & 1;
      const int64_t node = up ? hi[d] : lo[d];
      ok = ok && node >= 0;
      wt *= up ? wh[d] : wl[d];
      off += (node >= 0 ? node : 0) * stride;
      stride *= nc;
    }
    if (ok) acc += wt * z[off];
  }
  Pt[(size_t)q * Nf + i] = acc;
}

// Cholesky of the Gram G (r x r, row-major, r <= 64) with column dropping:
// column j is kept when its part orthogonal to the kept columns before it
// exceeds tau times its own norm.  T = R^-1 of the kept columns (row-major,
// stride r), their indices kidx and count kp.  One thread does the O(r^3)
// work in LDS (an offline step).
__global__ void k_chol_drop(int r, const double* G, double tau, double* T, int* kidx, int* kp_out) {
  __shared__ double A[64 * 64];
  __shared__ double Ti[64 * 64];
  __shared__ int kid[64];
  if (threadIdx.x != 0) return;
  for (int e = 0; e < r * r; ++e) A[e] = G[e];
  int kp = 0;
  for (int j = 0; j < r; ++j) {
    const double g0 = G[j * r + j];
    const double d = A[j * r + j];
    if (g0 > 0.0 && d > tau * tau * g0 && d == d) {
      const double rjj = sqrt(d);
      for (int l = j + 1; l < r; ++l) A[j * r + l] /= rjj;
      A[j * r + j] = rjj;
      for (int l = j + 1; l < r; ++l)
        for (int mm = l; mm < r; ++mm) A[l * r + mm] -= A[j * r + l] * A[j * r + mm];
      kid[kp++] = j;
    } else {
      for (int l = 0; l < r; ++l) A[j * r + l] = 0.0;
    }
  }
  // R of the kept columns (upper) and its inverse by back substitution
  for (int c = 0; c < kp; ++c) {
    for (int i = 0; i < kp; ++i) Ti[i * 64 + c] = 0.0;
    Ti[c * 64 + c] = 1.0 / A[kid[c] * r + kid[c]];
    for (int i = c - 1; i >= 0; --i) {
      double sum = 0.0;
      for (int mm = i + 1; mm <= c; ++mm) sum += A[kid[i] * r + kid[mm]] * Ti[mm * 64 + c];
      Ti[i * 64 + c] = -sum / A[kid[i] * r + kid[i]];
    }
  }
  for (int a = 0; a < kp; ++a)
    for (int b = 0; b < kp; ++b) T[a * r + b] = Ti[a * 64 + b];
  for (int a = 0; a < kp; ++a) kidx[a] = kid[a];
  *kp_out = kp;
}

// Y[a] = sum_{b <= a} X[kidx[b]] T[b][a]  (columns of length Nf, T stride r)
__global__ void k_apply_tri(int64_t Nf, int r, const int* kidx, const double* T, const double* X,
                            double* Y) {
  const int a = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nf) return;
  double acc = 0.0;
  for (int b = 0; b <= a; ++b) acc += X[(size_t)kidx[b] * Nf + i] * T[b * r + a];
  Y[(size_t)a * Nf + i] = acc;
}

// ---------------------------------------------------------------------------
// Reference eigenmodes by block inverse iteration with Rayleigh-Ritz: with
// S Y = X (one batched solve per step) the projected pair is E = Y^T X,
// G = Y^T Y, and S Z = X T for the Ritz vectors Z = Y T.
// ---------------------------------------------------------------------------
// Cholesky G = R^T R, T1 = R^-1 (upper) and F = T1^T sym(E) T1, all r x r
// row-major (r <= 64).  One thread in LDS (r^3 work per step); *fail = 1
// when G is not numerically positive definite.
__global__ void k_rr_reduce(int r, const double* G, const double* E, double* T1g, double* F, int* fail) {
  __shared__ double A[64 * 64];
  __shared__ double Ti[64 * 64];
  if (threadIdx.x != 0) return;
  for (int e = 0; e < r * r; ++e) A[e] = G[e];
  int bad = 0;
  for (int j = 0; j < r && !bad; ++j) {
    const double d = A[j * r + j];
    if (!(d > 0.0) || !(d < INFINITY)) { bad = 1; break; }
    const double rjj = sqrt(d);
    for (int l = j + 1; l < r; ++l) A[j * r + l] /= rjj;
    A[j * r + j] = rjj;
    for (int l = j + 1; l < r; ++l)
      for (int mm = l; mm < r; ++mm) A[l * r + mm] -= A[j * r + l] * A[j * r + mm];
  }
  *fail = bad;
  if (bad) return;
  for (int c = 0; c < r; ++c) {
    for (int i = 0; i < r; ++i) Ti[i * 64 + c] = 0.0;
    Ti[c * 64 + c] = 1.0 / A[c * r + c];
    for (int i = c - 1; i >= 0; --i) {
      double sum = 0.0;
      for (int mm = i + 1; mm <= c; ++mm) sum += A[i * r + mm] * Ti[mm * 64 + c];
      Ti[i * 64 + c] = -sum / A[i * r + i];
    }
  }
  // A <- sym(E) T1, then F = T1^T A
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double sum = 0.0;
      for (int mm = 0; mm <= b; ++mm) sum += 0.5 * (E[a * r + mm] + E[mm * r + a]) * Ti[mm * 64 + b];
      A[a * 64 + b] = sum;
    }
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double sum = 0.0;
      for (int mm = 0; mm <= a; ++mm) sum += Ti[mm * 64 + a] * A[mm * 64 + b];
      F[a * r + b] = sum;
    }
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) T1g[a * r + b] = Ti[a * 64 + b];
}

// Ritz values in ascending order and T = T1 V with the columns permuted alike
__global__ void k_rr_finish(int r, const double* T1, const double* V, const double* ev, double* T, double* lam) {
  __shared__ int ord[64];
  if (threadIdx.x != 0) return;
  for (int i = 0; i < r; ++i) ord[i] = i;
  for (int i = 0; i < r; ++i) {
    int best = i;
    for (int j = i + 1; j < r; ++j)
      if (ev[ord[j]] < ev[ord[best]]) best = j;
    const int t = ord[i]; ord[i] = ord[best]; ord[best] = t;
  }
  for (int j = 0; j < r; ++j) {
    lam[j] = ev[ord[j]];
    for (int a = 0; a < r; ++a) {
      double sum = 0.0;
      for (int b = a; b < r; ++b) sum += T1[a * r + b] * V[b * r + ord[j]];
      T[a * r + j] = sum;
    }
  }
}

// Z = Y T (Ritz vectors) and D = X T - Z diag(lam) = S Z - Z diag(lam)
__global__ void k_ritz_vectors(int64_t N, int r, const double* T, const double* lam, const double* X,
                               const double* Y, double* Z, double* D) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double z = 0.0, sx = 0.0;
  for (int b = 0; b < r; ++b) {
    const double t = T[b * r + j];
    z += Y[(size_t)b * N + i] * t;
    sx += X[(size_t)b * N + i] * t;
  }
  Z[(size_t)j * N + i] = z;
  D[(size_t)j * N + i] = sx - lam[j] * z;
}

// ---------------------------------------------------------------------------
// Primal active-set outer loop (state-constrained problems): the instances
// still iterating are addressed through idx (instance of batch slot j).
// ---------------------------------------------------------------------------
// psi restricted to the active set, padded layout: ps[j][i] = mask ? psi : 0
__global__ void k_ocp_psi(int64_t N, const int* idx, const uint8_t* mk, const double* psi, int64_t vs,
                          double* ps) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int m = idx[j];
  ps[(size_t)j * vs + i] = mk[(size_t)m * N + i] ? psi[(size_t)m * N + i] : 0.0;
}

// t = A ps on all rows (factored operator; ps padded, zero halo)
__global__ void k_ocp_inner(OpGeom op, const double* A64, const double* ps, int64_t vs, double* t) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const double* pj = ps + (size_t)j * vs;
  double acc = 0.0;
  for (int e = 0; e < op.D1; ++e) acc += A64[(size_t)e * N + i] * pj[i + op.offs1[e]];
  t[(size_t)j * vs + i] = acc;
}

// right-hand side of eq. (reduced): b = (y_d)_I - M_IA psi_A, with M_IA psi_A
// = (M ps)_I (ps vanishes on I); M = alpha A^T A + shift I (factored: src = t)
// or the assembled stencil (src = ps); also the batch slot's mask
__global__ void k_ocp_rhs(OpGeom op, const double* dia64, int factored, double alpha, const int* idx,
                          const uint8_t* mk, const double* yd, const double* src, int64_t vs, double* b,
                          uint8_t* msub) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  const int m = idx[j];
  const uint8_t a = mk[(size_t)m * N + i];
  msub[(size_t)j * N + i] = a;
  double v = 0.0;
  if (!a) {
    const double* sj = src + (size_t)j * vs;
    double acc = 0.0;
    for (int d = 0; d < op.D; ++d) acc += dia64[(size_t)d * N + i] * sj[i + op.offs[d]];
    v = yd[(size_t)m * N + i] - (factored ? alpha * acc : acc);
  }
  b[(size_t)j * N + i] = v;
}

// y = psi on the active set, the solve elsewhere; next active set
// {y > psi - tau}; changed[j] = 1 when it differs from the current one
__global__ void k_ocp_update(int64_t N, const int* idx, uint8_t* mk, const double* x, const double* psi,
                             double tau, double* y, int* changed) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int m = idx[j];
  const size_t gi = (size_t)m * N + i;
  const uint8_t old = mk[gi];
  const double pv = psi[gi];
  const double yv = old ? pv : x[(size_t)j * N + i];
  y[gi] = yv;
  const uint8_t nw = (yv > pv - tau) ? 1 : 0;
  mk[gi] = nw;
  if (nw != old) changed[j] = 1;
}

// Z (column-major n x k, FP64) -> Z64 / Z32 (column-major n x KP, zero padded)
__global__ void k_copy_modes(int64_t n, int k, int KP, const double* Z, double* Z64, float* Z32) {
  const int q = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (q < k) ? Z[(size_t)q * n + i] : 0.0;
  if (!(v == v)) return;
  Z64[(size_t)q * n + i] = v;
  Z32[(size_t)q * n + i] = (float)v;
}

// Row-major copy of the shared modes for the tile-major kernels:
// ZT[i][q] = Z[q][i] (the products there read 16 consecutive columns of a row).
template <typename T>
__global__ void k_modes_rowmajor(int64_t n, int KP, const T* Z, T* ZT) {
  const int q = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ZT[(size_t)i * KP + q] = Z[(size_t)q * n + i];
}

// Boundary rows of each instance (flags bnd, rows where W - Lambda Z does not
// vanish), compacted tile by tile for k_update_tm.  Launched with one block of
// UB_ROWS threads per (tile, instance).
__global__ void __launch_bounds__(UB_ROWS) k_bnd_count(int64_t N, int ntiles, const uint8_t* bnd, int* cnt) {
  const int tile = blockIdx.x, m = blockIdx.y;
  const int64_t i = (int64_t)tile * UB_ROWS + threadIdx.x;
  const int f = (i < N && bnd[(size_t)m * N + i]) ? 1 : 0;
  const int c = __syncthreads_count(f);
  if (threadIdx.x == 0) cnt[(size_t)m * ntiles + tile] = c;
}

// Exclusive prefix sums of the [B][ntiles] counts (one block of 1024 threads,
// each scanning a contiguous chunk): off[m][t] = entries before tile t of
// instance m, off[m][ntiles] = end of instance m; *total = all entries.
__global__ void __launch_bounds__(1024) k_bnd_scan(int B, int ntiles, const int* cnt, int* off,
                                                   int* total) {
  __shared__ int part[1024];
  const int n = B * ntiles;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
  int s = 0;
  for (int e = lo; e < hi; ++e) s += cnt[e];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < 1024; ++w) { const int v = part[w]; part[w] = run; run += v; }
    *total = run;
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int e = lo; e < hi; ++e) {
    const int m = e / ntiles, tl = e - m * ntiles;
    off[(size_t)m * (ntiles + 1) + tl] = run;
    run += cnt[e];
    if (tl == ntiles - 1) off[(size_t)m * (ntiles + 1) + ntiles] = run;
  }
}

// Entry e = off[m][tile] + (rank of the row among the tile's flagged rows):
// bidx[e] = row, bW[e][q] = W_m[q][row] (W stored as W - Lambda Z)
template <typename M>
__global__ void __launch_bounds__(UB_ROWS) k_bnd_fill(int64_t N, int ntiles, int KP, const uint8_t* bnd,
                                                      const int* off, const M* W, int* bidx, M* bW) {
  __shared__ int wcnt[UB_ROWS / 64];
  const int tile = blockIdx.x, m = blockIdx.y;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t i = (int64_t)tile * UB_ROWS + threadIdx.x;
  const bool f = i < N && bnd[(size_t)m * N + i];
  const unsigned long long bal = __ballot(f);
  if (lane == 0) wcnt[wid] = __popcll(bal);
  __syncthreads();
  if (!f) return;
  int pos = off[(size_t)m * (ntiles + 1) + tile] + __popcll(bal & ((1ull << lane) - 1ull));
  for (int w = 0; w < wid; ++w) pos += wcnt[w];
  bidx[pos] = (int)i;
  const M* Wm = W + (size_t)m * KP * N;
  for (int q = 0; q < KP; ++q) bW[(size_t)pos * KP + q] = Wm[(size_t)q * N + i];
}

// ---------------------------------------------------------------------------
// W = S_II Z_I (stored as V), and per instance the Gram matrices
//   G = Z_I^T Z_I,  E = Z_I^T W   (FP64, deterministic tree reduction)
// Each block walks sub-tiles of GR rows; the Gram outputs are distributed over
// the threads (OPT outputs each) and accumulated in registers.
// ---------------------------------------------------------------------------
template <int KP> struct GramCfg {
  static constexpr int GR = KP > 32 ? 32 : 64;                 // rows per sub-tile
  static constexpr int NOUT = 2 * KP * KP;
  static constexpr int OPT = (NOUT + TPB - 1) / TPB;           // outputs per thread
  static constexpr int CG = TPB / GR;                          // column groups
  static constexpr int CPG = (KP + CG - 1) / CG;               // columns per group
  static constexpr int LDS = (2 * GR * KP > NOUT ? 2 * GR * KP : NOUT);
};

// src: stencil source columns, Z itself (assembled operator; read masked) or
// T = A Ztilde of this instance (factored operator; read unmasked).
template <typename V, int KP>
__global__ void __launch_bounds__(TPB) k_spmm_gram(OpGeom op, const double* dia64, const double* Z64,
                                                    int64_t zs, const double* src, int factored,
                                                    const uint8_t* mask, V* W, Inst* inst,
                                                    double* part, unsigned* ctr, RedGeom g,
                                                    double* gram, int nsub, const double* mu,
                                                    const uint8_t* eig, int ne) {
  using C = GramCfg<KP>;
  __shared__ double lds[C::LDS];
  double* zt = lds;                 // [GR][KP]
  double* wt = lds + C::GR * KP;    // [GR][KP]
  const int m = blockIdx.y;
  const Inst* S = inst + m;
  const int64_t N = op.N;
  const uint8_t* mk = mask + (size_t)m * N;
  V* Wm = W + (size_t)m * KP * N;
  const double sa = S->a, sc = S->c;
  double acc[C::OPT];
#pragma unroll
  for (int o = 0; o < C::OPT; ++o) acc[o] = 0.0;
  const int row = threadIdx.x % C::GR;
  const int cg = threadIdx.x / C::GR;
  for (int st = blockIdx.x; st < nsub; st += gridDim.x) {
    const int64_t i = (int64_t)st * C::GR + row;
    const bool act = (i >= N) || mk[i] != 0;
#pragma unroll
    for (int cc = 0; cc < C::CPG; ++cc) {
      const int q = cg * C::CPG + cc;
      if (q < KP) {
        double wv = 0.0, zv = 0.0;
        if (!act) {
          const double* Zq = Z64 + (size_t)m * zs + (size_t)q * N;
          const double* Sq = factored ? src + ((size_t)m * KP + q) * N : Zq;
          double s = 0.0;
          for (int d = 0; d < op.D; ++d) {
            const int64_t j = i + op.offs[d];
            if (j >= 0 && j < N && (factored || mk[j] == 0)) s += dia64[(size_t)d * N + i] * Sq[j];
          }
          zv = Zq[i];
          wv = sa * s + sc * zv;
          // eigen columns are stored as W - lambda Z (zero away from the
          // active-set boundary up to the eigen-residual); E uses W itself
          const double lam = (q < ne && eig[q]) ? sa * mu[q] + sc : 0.0;
          Wm[(size_t)q * N + i] = (V)(wv - lam * zv);
        } else if (i < N) {
          Wm[(size_t)q * N + i] = (V)0;
        }
        zt[row * KP + q] = zv;
        wt[row * KP + q] = wv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < C::OPT; ++o) {
      const int idx = threadIdx.x + o * TPB;
      if (idx < C::NOUT) {
        const bool isE = idx >= KP * KP;
        const int e = isE ? idx - KP * KP : idx;
        const int jr = e / KP, jc = e % KP;
        const double* rhs = isE ? wt : zt;
        double s = 0.0;
        for (int r2 = 0; r2 < C::GR; ++r2) s += zt[r2 * KP + jr] * rhs[r2 * KP + jc];
        acc[o] += s;
      }
    }
    __syncthreads();
  }
  // block partial: each output owned by exactly one thread
#pragma unroll
  for (int o = 0; o < C::OPT; ++o) {
    const int idx = threadIdx.x + o * TPB;
    if (idx < C::NOUT) lds[idx] = acc[o];
  }
  __syncthreads();
  double* pm = part + (size_t)m * g.ptotal * C::NOUT;
  unsigned* cm = ctr + (size_t)m * g.ctotal;
  tree_reduce(g, blockIdx.x, C::NOUT, pm, cm, lds, gram + (size_t)m * C::NOUT);
}

// ---------------------------------------------------------------------------
// One-workgroup coarse setup per instance (k x k, FP64, LDS):
//   R = chol(G) with column dropping; T = R^{-1};  F = T^T E T (E of the
//   orthonormal basis Z_I T); cond(F) by cyclic Jacobi; F = L L^T;
//   C = T F^{-1} T^T (= E_raw^{-1} on the kept columns).
// Fallback (kk = 0, C = 0) when cond(F) > tau_cond or Cholesky fails.
// ---------------------------------------------------------------------------
struct CoarseArgs {
  const double* gram;    // [B][2][KP][KP]  (G, then E; row-major)
  double* C;             // [B][KP][KP]
  double* Finfo;         // [B][KP][KP] column-major, leading k' x k'
  int* kept;             // [B][KP]
  Inst* inst;
  int k;                 // true number of modes (<= KP)
  double drop_rel;
  double tau_dep;        // POD candidates (columns k_safe..): also dropped when their part
                         //   orthogonal to the kept columns is <= tau_dep of their norm
  double tau_cond;
  int k_base;            // > 0: columns k_base.. are learned enrichment vectors;
  double tau_learned;    //   if cond(E) exceeds tau_learned (or the setup fails)
                         //   the instance retries with the first k_base columns
  int ritz_keep;         // 0 < r < kept columns: Rayleigh-Ritz reselection of
                         //   the r smallest Ritz vectors of the restricted pool
  int k_safe;            // > 0: columns k_safe.. are POD candidates merged by the
  double tau_safe;       //   conditioning rule (cond <= tau_safe) of the safe merge
};

// Cyclic Jacobi on the leading n x n block of the symmetric matrix A (LDS,
// row stride KP) in parallel round-robin order; V (LDS, may be null)
// accumulates the rotations (V <- V J).  On return diag(A) holds the
// eigenvalues.  Every thread of the block calls it with the same n.
template <int KP>
__device__ void jacobi_eig(double* A, double* V, int n, double* rc, double* rs, int* rp_, int* rq_,
                           double* red) {
  const int tid = threadIdx.x;
  const int M = (n + 1) & ~1;
  const int npair = M / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    // off-diagonal mass
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += TPB) {
      const int aa = e / n, bb = e % n;
      const double v = A[aa * KP + bb];
      if (aa != bb) off += v * v; else dia += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if ((tid & 63) == 0) red[tid >> 6] = off;
    __syncthreads();
    double offt = 0.0;
    for (int w = 0; w < NWAVE; ++w) offt += red[w];
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = dia;
    __syncthreads();
    double diat = 0.0;
    for (int w = 0; w < NWAVE; ++w) diat += red[w];
    __syncthreads();
    if (!(offt > 1e-30 * diat)) break;
    for (int rnd = 0; rnd < M - 1; ++rnd) {
      for (int t = tid; t < npair; t += TPB) {
        int p, q;
        if (t == 0) { p = rnd; q = M - 1; }
        else { p = (rnd + t) % (M - 1); q = (rnd - t + (M - 1)) % (M - 1); }
        if (p > q) { const int tt = p; p = q; q = tt; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * KP + q];
          if (fabs(apq) > 1e-300) {
            const double app = A[p * KP + p], aqq = A[q * KP + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        rp_[t] = p; rq_[t] = q; rc[t] = c; rs[t] = s;
      }
      __syncthreads();
      for (int e = tid; e < npair * n; e += TPB) {      // A <- A J (columns)
        const int t = e / n, i = e % n;
        const int p = rp_[t], q = rq_[t];
        if (q < n) {
          const double c = rc[t], s = rs[t];
          const double aip = A[i * KP + p], aiq = A[i * KP + q];
          A[i * KP + p] = c * aip - s * aiq;
          A[i * KP + q] = s * aip + c * aiq;
          if (V) {                                        // V <- V J
            const double vip = V[i * KP + p], viq = V[i * KP + q];
            V[i * KP + p] = c * vip - s * viq;
            V[i * KP + q] = s * vip + c * viq;
          }
        }
      }
      __syncthreads();
      for (int e = tid; e < npair * n; e += TPB) {      // A <- J^T A (rows)
        const int t = e / n, j = e % n;
        const int p = rp_[t], q = rq_[t];
        if (q < n) {
          const double c = rc[t], s = rs[t];
          const double apj = A[p * KP + j], aqj = A[q * KP + j];
          A[p * KP + j] = c * apj - s * aqj;
          A[q * KP + j] = s * apj + c * aqj;
        }
      }
      __syncthreads();
    }
  }
}

// Largest and smallest diagonal entries of the leading n x n block of A.
template <int KP>
__device__ __forceinline__ double diag_cond(const double* A, int n) {
  double lmin = INFINITY, lmax = -INFINITY;
  for (int i = 0; i < n; ++i) {
    lmin = fmin(lmin, A[i * KP + i]);
    lmax = fmax(lmax, A[i * KP + i]);
  }
  return (lmin > 0.0) ? lmax / lmin : INFINITY;
}

template <int KP>
__global__ void __launch_bounds__(TPB) k_coarse(CoarseArgs ca) {
  constexpr int K = KP > 0 ? KP : 1;
  __shared__ double A0[K * K];   // G -> R, later tmp / Jacobi work / X
  __shared__ double A1[K * K];   // T
  __shared__ double A2[K * K];   // E -> F -> L
  __shared__ int kidx[K];
  __shared__ int s_keep, s_kp, s_fail;
  __shared__ double s_d;
  __shared__ double rc[K / 2 + 1], rs[K / 2 + 1];
  __shared__ int rp_[K / 2 + 1], rq_[K / 2 + 1];
  __shared__ double red[NWAVE];
  __shared__ double gdiag[K];    // diag(G), later the selected Ritz values
  __shared__ int ord[K];
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  Inst* S = ca.inst + m;
  const double* G = ca.gram + (size_t)m * 2 * KP * KP;
  const double* E = G + KP * KP;
  __shared__ int s_retry;
  for (int attempt = 0; attempt < 2; ++attempt) {
  const int k = attempt == 0 ? ca.k : ca.k_base;
  for (int e = tid; e < KP * KP; e += TPB) A0[e] = G[e];
  for (int e = tid; e < KP; e += TPB) gdiag[e] = G[e * KP + e];
  __syncthreads();

  // --- Cholesky of G with column dropping (upper R, row j = R[j][:]) ---
  int kp = 0;
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double d = A0[j * KP + j];
      const double g0 = gdiag[j];
      const double dr = (ca.k_safe > 0 && j >= ca.k_safe) ? fmax(ca.drop_rel, ca.tau_dep) : ca.drop_rel;
      const double thr = dr * dr * g0;
      s_keep = (g0 > 0.0) && (d > thr) && (d == d);
      s_d = s_keep ? sqrt(d) : 0.0;
      if (s_keep) kidx[kp] = j;
    }
    __syncthreads();
    const bool keep = s_keep;
    const double rjj = s_d;
    if (keep) {
      for (int l = j + 1 + tid; l < k; l += TPB) A0[j * KP + l] /= rjj;
      if (tid == 0) A0[j * KP + j] = rjj;
      __syncthreads();
      const int rem = k - j - 1;
      for (int e = tid; e < rem * rem; e += TPB) {
        const int l = j + 1 + e / rem, mm = j + 1 + e % rem;
        if (mm >= l) A0[l * KP + mm] -= A0[j * KP + l] * A0[j * KP + mm];
      }
      ++kp;
    } else {
      for (int l = tid; l < k; l += TPB) A0[j * KP + l] = 0.0;
    }
    __syncthreads();
  }
  // --- compact R to kept columns: Rc[a][b] = R[kidx[a]][kidx[b]] -> A1 temp ---
  for (int e = tid; e < kp * kp; e += TPB) {
    const int aa = e / kp, bb = e % kp;
    A1[aa * KP + bb] = (bb >= aa) ? A0[kidx[aa] * KP + kidx[bb]] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < kp * kp; e += TPB) A0[(e / kp) * KP + e % kp] = A1[(e / kp) * KP + e % kp];
  __syncthreads();
  // --- T = R^{-1} (upper), one column per thread ---
  for (int c = tid; c < kp; c += TPB) {
    for (int i = 0; i < kp; ++i) A1[i * KP + c] = 0.0;
    A1[c * KP + c] = 1.0 / A0[c * KP + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int mm = i + 1; mm <= c; ++mm) s += A0[i * KP + mm] * A1[mm * KP + c];
      A1[i * KP + c] = -s / A0[i * KP + i];
    }
  }
  // --- E on kept columns -> A2 ---
  for (int e = tid; e < kp * kp; e += TPB) {
    const int aa = e / kp, bb = e % kp;
    A2[aa * KP + bb] = 0.5 * (E[kidx[aa] * KP + kidx[bb]] + E[kidx[bb] * KP + kidx[aa]]);
  }
  __syncthreads();
  // --- tmp = E T (A0), F = T^T tmp (A2) ---
  for (int e = tid; e < kp * kp; e += TPB) {
    const int aa = e / kp, bb = e % kp;
    double s = 0.0;
    for (int mm = 0; mm <= bb; ++mm) s += A2[aa * KP + mm] * A1[mm * KP + bb];
    A0[aa * KP + bb] = s;
  }
  __syncthreads();
  for (int e = tid; e < kp * kp; e += TPB) {
    const int aa = e / kp, bb = e % kp;
    double s = 0.0;
    for (int mm = 0; mm <= aa; ++mm) s += A1[mm * KP + aa] * A0[mm * KP + bb];
    A2[aa * KP + bb] = s;
  }
  __syncthreads();
  for (int e = tid; e < kp * kp; e += TPB) {      // symmetrise, export, Jacobi copy
    const int aa = e / kp, bb = e % kp;
    const double v = 0.5 * (A2[aa * KP + bb] + A2[bb * KP + aa]);
    A0[aa * KP + bb] = v;
    ca.Finfo[(size_t)m * KP * KP + bb * KP + aa] = v;
  }
  __syncthreads();
  // Safe merge of POD candidates (Sec. "Conditioning-based safe merge",
  // Alg. 2).  The Cholesky above already orthogonalised every candidate
  // against the kept columns before it and skipped dependent ones; the
  // leading q x q block of F is E of the first q kept columns in an
  // orthonormal basis, and by Cauchy interlacing its condition number
  // grows with q.  Stopping at the first candidate whose trial basis
  // exceeds tau_safe is therefore keeping the longest prefix within it,
  // found by bisection over the candidates.
  if (ca.k_safe > 0 && ca.k_base == 0 && ca.k_safe < k && kp > 0) {
    int ne = 0;
    while (ne < kp && kidx[ne] < ca.k_safe) ++ne;      // kept eigenmode columns
    if (kp > ne) {
      for (int e = tid; e < kp * kp; e += TPB) A2[(e / kp) * KP + e % kp] = A0[(e / kp) * KP + e % kp];
      int lo = ne, hi = kp;
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        __syncthreads();
        for (int e = tid; e < mid * mid; e += TPB) A0[(e / mid) * KP + e % mid] = A2[(e / mid) * KP + e % mid];
        __syncthreads();
        jacobi_eig<KP>(A0, nullptr, mid, rc, rs, rp_, rq_, red);
        const double cm = diag_cond<KP>(A0, mid);
        if (cm <= ca.tau_safe) lo = mid; else hi = mid - 1;
      }
      __syncthreads();
      kp = lo;
      for (int e = tid; e < kp * kp; e += TPB) A0[(e / kp) * KP + e % kp] = A2[(e / kp) * KP + e % kp];
      __syncthreads();
    }
  }
  // Ritz reselection (Sec. "Ritz re-selection"): the eigenvectors of F are
  // accumulated in A2 (the Cholesky of F is not needed on that path)
  const bool ritz = ca.ritz_keep > 0 && ca.ritz_keep < kp;
  const int nx = ritz ? ca.ritz_keep : kp;
  for (int e = tid; e < kp * kp; e += TPB) {
    const int aa = e / kp, bb = e % kp;
    A2[aa * KP + bb] = ritz ? (aa == bb ? 1.0 : 0.0) : A0[aa * KP + bb];
  }
  for (int j = tid; j < KP; j += TPB) {
    int f = 0;
    for (int a2 = 0; a2 < kp; ++a2) f |= (kidx[a2] == j);
    ca.kept[(size_t)m * KP + j] = f;
  }
  __syncthreads();

  // --- cyclic Jacobi eigenvalues of F (A0) ---
  double cond = 1.0;
  if (kp > 0) {
    jacobi_eig<KP>(A0, ritz ? A2 : nullptr, kp, rc, rs, rp_, rq_, red);
    double lmin = INFINITY, lmax = -INFINITY;
    for (int i = 0; i < kp; ++i) {
      lmin = fmin(lmin, A0[i * KP + i]);
      lmax = fmax(lmax, A0[i * KP + i]);
    }
    cond = (lmin > 0.0) ? lmax / lmin : INFINITY;
  }
  __syncthreads();
  if (ritz) {
    // ascending Ritz values; keep the ritz_keep smallest
    if (tid == 0) {
      for (int i = 0; i < kp; ++i) ord[i] = i;
      for (int i = 0; i < nx; ++i) {
        int best = i;
        for (int j = i + 1; j < kp; ++j)
          if (A0[ord[j] * KP + ord[j]] < A0[ord[best] * KP + ord[best]]) best = j;
        const int t = ord[i]; ord[i] = ord[best]; ord[best] = t;
      }
      for (int i = 0; i < nx; ++i) gdiag[i] = A0[ord[i] * KP + ord[i]];
    }
    __syncthreads();
    cond = (gdiag[0] > 0.0) ? gdiag[nx - 1] / gdiag[0] : INFINITY;
  }

  // --- Cholesky F = L L^T (lower, in A2) ---
  if (tid == 0) s_fail = ritz ? !(gdiag[0] > 0.0) : 0;
  __syncthreads();
  for (int j = 0; j < (ritz ? 0 : kp); ++j) {
    if (tid == 0) {
      const double d = A2[j * KP + j];
      if (!(d > 0.0) || !(d < INFINITY)) s_fail = 1;
      s_d = s_fail ? 1.0 : sqrt(d);
    }
    __syncthreads();
    if (s_fail) break;
    const double ljj = s_d;
    for (int l = j + 1 + tid; l < kp; l += TPB) A2[l * KP + j] /= ljj;
    if (tid == 0) A2[j * KP + j] = ljj;
    __syncthreads();
    const int rem = kp - j - 1;
    for (int e = tid; e < rem * rem; e += TPB) {
      const int l = j + 1 + e / rem, mm = j + 1 + e % rem;
      if (mm <= l) A2[l * KP + mm] -= A2[l * KP + j] * A2[mm * KP + j];
    }
    __syncthreads();
  }
  const bool enriched = attempt == 0 && ca.k_base > 0 && ca.k_base < ca.k;
  const double tau = enriched ? fmin(ca.tau_cond, ca.tau_learned) : ca.tau_cond;
  const bool fallback = (kp == 0) || s_fail || !(cond <= tau);
  if (tid == 0) s_retry = enriched && fallback;
  __syncthreads();
  if (s_retry) continue;     // plain reference basis as fallback (uniform)
  // --- X = L^{-1} T^T (A0), one column per thread; with Ritz reselection
  //     X = Lambda_r^{-1/2} Y_r^T T^T (r rows), so C = X^T X is the coarse
  //     inverse of the selected basis Z T Y_r in pool coordinates ---
  if (!fallback && ritz) {
    for (int e = tid; e < nx * kp; e += TPB) {
      const int i = e / kp, c = e % kp;
      const int col = ord[i];
      double s = 0.0;
      for (int mm = c; mm < kp; ++mm) s += A2[mm * KP + col] * A1[c * KP + mm];
      A0[i * KP + c] = s / sqrt(gdiag[i]);
    }
  } else if (!fallback) {
    for (int c = tid; c < kp; c += TPB) {
      for (int i = 0; i < kp; ++i) {
        double s = A1[c * KP + i];                 // (T^T)[i][c] = T[c][i]
        for (int mm = 0; mm < i; ++mm) s -= A2[i * KP + mm] * A0[mm * KP + c];
        A0[i * KP + c] = s / A2[i * KP + i];
      }
    }
  }
  __syncthreads();
  // --- C = X^T X scattered to KP x KP ---
  double* Cm = ca.C + (size_t)m * KP * KP;
  for (int e = tid; e < KP * KP; e += TPB) Cm[e] = 0.0;
  __syncthreads();
  if (!fallback) {
    for (int e = tid; e < kp * kp; e += TPB) {
      const int aa = e / kp, bb = e % kp;
      double s = 0.0;
      for (int i = 0; i < nx; ++i) s += A0[i * KP + aa] * A0[i * KP + bb];
      Cm[kidx[aa] * KP + kidx[bb]] = s;
    }
  }
  if (tid == 0) {
    S->cond = (kp > 0 && s_fail) ? INFINITY : cond;
    S->k_eff = kp;
    S->kk = fallback ? 0 : kp;
    S->learned = enriched && !fallback;
    if (fallback && k > 0 && S->setup_status == 0) S->setup_status = 1;
  }
  break;
  }
}

}  // namespace adef2
