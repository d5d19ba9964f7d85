// Kernels of the learned coarse-space enrichment: POD of solution snapshots,
// per-sample loss data, the MLP theta -> C (BF16 weights, FP32 accumulation),
// its loss gradient, backward pass and Adam, and the basis expansion
// V = Phi C^T appended to the shared reference modes.
#pragma once
#include "dev_setup.h"

namespace adef2 {

// ---------------------------------------------------------------------------
// Tall-skinny Gram  out[m] = X_m^T Y_m  (FP64), optional row mask (rows with
// mask != 0 skipped).  X_m = X + m*sx (N x nx column-major), Y_m likewise.
// Grid (row blocks, output tiles, B); partial sums per row block are written
// to part[m][rb][nx][ny] and summed by k_gram_finish in a fixed order.
// ---------------------------------------------------------------------------
constexpr int GT = 64;    // output tile edge
constexpr int GROWS = 32; // rows staged per step

__global__ void __launch_bounds__(TPB) k_gram_ts(int64_t N, int nx, int ny, const double* X, int64_t sx,
                                                 const double* Y, int64_t sy, const uint8_t* mask,
                                                 int64_t smask, int rows_per_block, double* part) {
  __shared__ double xs[GROWS][GT];
  __shared__ double ys[GROWS][GT];
  const int m = blockIdx.z;
  const int ntx = (nx + GT - 1) / GT;
  const int tx = blockIdx.y % ntx, ty = blockIdx.y / ntx;
  const double* Xm = X + (size_t)m * sx;
  const double* Ym = Y + (size_t)m * sy;
  const uint8_t* mk = mask ? mask + (size_t)m * smask : nullptr;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(N, r0 + rows_per_block);
  double acc[GT * GT / TPB];
#pragma unroll
  for (int o = 0; o < GT * GT / TPB; ++o) acc[o] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += GROWS) {
    for (int e = threadIdx.x; e < GROWS * GT; e += TPB) {
      const int rr = e / GT, cc = e % GT;
      const int64_t i = rb + rr;
      const bool on = i < r1 && (!mk || mk[i] == 0);
      const int cx = tx * GT + cc, cy = ty * GT + cc;
      xs[rr][cc] = (on && cx < nx) ? Xm[(size_t)cx * N + i] : 0.0;
      ys[rr][cc] = (on && cy < ny) ? Ym[(size_t)cy * N + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < GT * GT / TPB; ++o) {
      const int idx = threadIdx.x + o * TPB;
      const int a = idx / GT, b = idx % GT;
      double s = 0.0;
      for (int rr = 0; rr < GROWS; ++rr) s += xs[rr][a] * ys[rr][b];
      acc[o] += s;
    }
    __syncthreads();
  }
  const int nrb = gridDim.x;
#pragma unroll
  for (int o = 0; o < GT * GT / TPB; ++o) {
    const int idx = threadIdx.x + o * TPB;
    const int a = tx * GT + idx / GT, b = ty * GT + idx % GT;
    if (a < nx && b < ny) part[(((size_t)m * nrb + blockIdx.x) * nx + a) * ny + b] = acc[o];
  }
}

__global__ void k_gram_finish(int nrb, int nx, int ny, const double* part, double* out) {
  const int m = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx * ny) return;
  double s = 0.0;
  for (int r = 0; r < nrb; ++r) s += part[((size_t)m * nrb + r) * nx * ny + e];
  out[(size_t)m * nx * ny + e] = s;
}

// row means of X (N x M) and centred copy Xc = X - mean
__global__ void k_center(int64_t N, int M, const double* X, double* Xc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int j = 0; j < M; ++j) s += X[(size_t)j * N + i];
  const double mu = s / M;
  for (int j = 0; j < M; ++j) Xc[(size_t)j * N + i] = X[(size_t)j * N + i] - mu;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix A (global
// memory, row-major) with eigenvectors accumulated in V (V[i][j] = entry i of
// eigenvector j).  One workgroup; parallel round-robin pairs.
// ---------------------------------------------------------------------------
constexpr int JMAX = 256;

__global__ void __launch_bounds__(1024) k_jacobi_eig(int n, double* A, double* V, double* evals) {
  __shared__ double rc[JMAX / 2], rs[JMAX / 2];
  __shared__ int rp_[JMAX / 2], rq_[JMAX / 2];
  __shared__ double red[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  const int M = (n + 1) & ~1;
  const int npair = M / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      const double v = A[e];
      if (e / n != e % n) off += v * v; else dia += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if ((tid & 63) == 0) red[tid >> 6] = off;
    __syncthreads();
    double offt = 0.0;
    for (int w = 0; w < nt / 64; ++w) offt += red[w];
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = dia;
    __syncthreads();
    double diat = 0.0;
    for (int w = 0; w < nt / 64; ++w) diat += red[w];
    __syncthreads();
    if (!(offt > 1e-30 * diat)) break;
    for (int rnd = 0; rnd < M - 1; ++rnd) {
      for (int t = tid; t < npair; t += nt) {
        int p, q;
        if (t == 0) { p = rnd; q = M - 1; }
        else { p = (rnd + t) % (M - 1); q = (rnd - t + (M - 1)) % (M - 1); }
        if (p > q) { const int tt = p; p = q; q = tt; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          if (fabs(apq) > 1e-300) {
            const double app = A[p * n + p], aqq = A[q * n + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        rp_[t] = p; rq_[t] = q; rc[t] = c; rs[t] = s;
      }
      __syncthreads();
      for (int e = tid; e < npair * n; e += nt) {        // A J and V J (columns)
        const int t = e / n, i = e % n;
        const int p = rp_[t], q = rq_[t];
        if (q < n) {
          const double c = rc[t], s = rs[t];
          const double aip = A[i * n + p], aiq = A[i * n + q];
          A[i * n + p] = c * aip - s * aiq;
          A[i * n + q] = s * aip + c * aiq;
          const double vip = V[i * n + p], viq = V[i * n + q];
          V[i * n + p] = c * vip - s * viq;
          V[i * n + q] = s * vip + c * viq;
        }
      }
      __syncthreads();
      for (int e = tid; e < npair * n; e += nt) {        // J^T A (rows)
        const int t = e / n, j = e % n;
        const int p = rp_[t], q = rq_[t];
        if (q < n) {
          const double c = rc[t], s = rs[t];
          const double apj = A[p * n + j], aqj = A[q * n + j];
          A[p * n + j] = c * apj - s * aqj;
          A[q * n + j] = s * apj + c * aqj;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += nt) evals[i] = A[i * n + i];
}

// Phi[:, j] = Xc v_c / sqrt(lambda_c), c = sel[j] (eigenvalue order,
// descending; identity when sel is null); entry m of eigenvector c at
// V[m * vsm + c * vsc]
__global__ void k_pod_modes(int64_t N, int M, int p, const double* Xc, const double* V, int64_t vsm,
                            int64_t vsc, const int* sel, const double* evals, double* Phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= N || j >= p) return;
  const int c = sel ? sel[j] : j;
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += Xc[(size_t)m * N + i] * V[(size_t)m * vsm + (size_t)c * vsc];
  const double lam = evals[c];
  Phi[(size_t)j * N + i] = lam > 0.0 ? s / sqrt(lam) : 0.0;
}

// ---------------------------------------------------------------------------
// Subspace iteration for the leading eigenpairs of a large snapshot Gram
// (M > JMAX): blocks of L orthonormal columns are multiplied by G, rotated
// by the Rayleigh-Ritz eigenvectors of Q^T G Q and re-orthonormalised
// (scaled Gram + eigen-decomposition, "SVQB"), until the residuals of the
// wanted Ritz pairs are small.
// ---------------------------------------------------------------------------
constexpr int SYB = 8;   // columns per thread in k_symm_block

// Y[:, j] = G Q[:, j], G symmetric M x M (row-major: row i is column i, so
// the loads along m are coalesced across threads); Q, Y column-major M x L.
__global__ void __launch_bounds__(256) k_symm_block(int M, int L, const double* G, const double* Q,
                                                    double* Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = blockIdx.y * SYB;
  if (i >= M) return;
  double s[SYB];
#pragma unroll
  for (int c = 0; c < SYB; ++c) s[c] = 0.0;
  for (int m = 0; m < M; ++m) {
    const double g = G[(size_t)m * M + i];
#pragma unroll
    for (int c = 0; c < SYB; ++c)
      if (j0 + c < L) s[c] += g * Q[(size_t)(j0 + c) * M + m];
  }
#pragma unroll
  for (int c = 0; c < SYB; ++c)
    if (j0 + c < L) Y[(size_t)(j0 + c) * M + i] = s[c];
}

// out[:, c] = scale[c] * sum_l A[:, l] pre[l] W[l][col(c)], col(c) = sel[c]
// (or c); A, out column-major M x L, W row-major L x L (entry l of column j
// at W[l * L + j]).  pre / scale / sel may be null (ones / identity).
__global__ void k_comb_cols(int M, int L, const double* A, const double* pre, const double* W,
                            const int* sel, const double* scale, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= M) return;
  const int col = sel ? sel[c] : c;
  double s = 0.0;
  for (int l = 0; l < L; ++l) s += A[(size_t)l * M + i] * (pre ? pre[l] : 1.0) * W[(size_t)l * L + col];
  out[(size_t)c * M + i] = scale ? s * scale[c] : s;
}

// SVQB pre-scaling: dsc[l] = C[l][l]^-1/2 (0 for a zero column) and
// C <- D C D, symmetrised.  One workgroup.
__global__ void k_svqb_scale(int L, double* C, double* dsc) {
  for (int l = threadIdx.x; l < L; l += blockDim.x) {
    const double d = C[(size_t)l * L + l];
    dsc[l] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int a = e / L, b = e % L;
    if (a > b) continue;
    const double v = 0.5 * (C[(size_t)a * L + b] + C[(size_t)b * L + a]) * dsc[a] * dsc[b];
    C[(size_t)a * L + b] = v;
    C[(size_t)b * L + a] = v;
  }
}

// SVQB post-scaling: inv[c] = d[c]^-1/2 for eigenvalues above drop * max(d),
// else 0 (the direction is dropped: a zero column).  One workgroup.
__global__ void k_svqb_inv(int L, const double* d, double drop, double* inv) {
  __shared__ double mx;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int l = 0; l < L; ++l) m = fmax(m, d[l]);
    mx = m;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < L; l += blockDim.x) inv[l] = d[l] > drop * mx ? 1.0 / sqrt(d[l]) : 0.0;
}

// H <- (H + H^T) / 2 (L x L).  One workgroup.
__global__ void k_symmetrize(int L, double* H) {
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int a = e / L, b = e % L;
    if (a >= b) continue;
    const double v = 0.5 * (H[(size_t)a * L + b] + H[(size_t)b * L + a]);
    H[(size_t)a * L + b] = v;
    H[(size_t)b * L + a] = v;
  }
}

// res[c] = || YW[:, c] - th[c] QW[:, c] ||_2 (one workgroup per column)
__global__ void __launch_bounds__(256) k_ritz_resid(int M, const double* QW, const double* YW,
                                                    const double* th, double* res) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const double r = YW[(size_t)c * M + i] - th[c] * QW[(size_t)c * M + i];
    s += r * r;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) res[c] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// deterministic start block: entries uniform in [-1, 1) from a 64-bit mix
// of the entry index (splitmix64 finaliser)
__global__ void k_start_block(int64_t n, double* Q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  uint64_t z = (uint64_t)e + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  Q[e] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// ---------------------------------------------------------------------------
// Per-sample loss data from the Grams of [Z | Phi] (one workgroup per sample):
//   G = [Z|P]^T S [Z|P]  ((k+p) x (k+p)),  bZP = [Z|P]^T b,
//   H = Gpp - Gpz Gzz^-1 Gzp, g = bP - Gpz Gzz^-1 bZ, e0 = bZ^T Gzz^-1 bZ.
// Gzz is factorised by Cholesky (with the same column dropping as the coarse
// setup: dependent columns contribute nothing).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_loss_data(int k, int p, const double* G, const double* bzp,
                                                    double* H, double* gv, double* e0v, double drop_rel,
                                                    const double* Gd, double* Nout) {
  extern __shared__ double sm[];
  double* L = sm;                 // k x k Cholesky (lower)
  double* A = L + k * k;          // k x (p+1): Gzz^-1 [Gzp | bZ]
  double* GA = A + k * (p + 1);   // k x p: Dzz Gzz^-1 Gzp (with Gd only)
  __shared__ int s_keep[64];
  __shared__ double s_d;
  const int m = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = k + p;
  const double* Gm = G + (size_t)m * n * n;
  const double* bm = bzp + (size_t)m * n;
  for (int e = tid; e < k * k; e += nt) L[e] = Gm[(e / k) * n + e % k];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double d = L[j * k + j];
      const double g0 = Gm[j * n + j];
      s_keep[j] = (g0 > 0.0) && (d > drop_rel * drop_rel * g0);
      s_d = s_keep[j] ? sqrt(d) : 0.0;
    }
    __syncthreads();
    if (s_keep[j]) {
      for (int l = j + 1 + tid; l < k; l += nt) L[l * k + j] /= s_d;
      if (tid == 0) L[j * k + j] = s_d;
      __syncthreads();
      const int rem = k - j - 1;
      for (int e = tid; e < rem * rem; e += nt) {
        const int l = j + 1 + e / rem, q = j + 1 + e % rem;
        if (q <= l) L[l * k + q] -= L[l * k + j] * L[q * k + j];
      }
    } else {
      for (int l = tid; l < k; l += nt) { L[l * k + j] = 0.0; L[j * k + l] = 0.0; }
    }
    __syncthreads();
  }
  // A[:, c] = Gzz^-1 rhs_c  (forward then backward substitution, one column per thread)
  for (int c = tid; c < p + 1; c += nt) {
    for (int i = 0; i < k; ++i) {
      double s = (c < p) ? Gm[i * n + k + c] : bm[i];
      for (int q = 0; q < i; ++q) s -= L[i * k + q] * A[q * (p + 1) + c];
      A[i * (p + 1) + c] = s_keep[i] ? s / L[i * k + i] : 0.0;
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = A[i * (p + 1) + c];
      for (int q = i + 1; q < k; ++q) s -= L[q * k + i] * A[q * (p + 1) + c];
      A[i * (p + 1) + c] = s_keep[i] ? s / L[i * k + i] : 0.0;
    }
  }
  __syncthreads();
  double* Hm = H + (size_t)m * p * p;
  for (int e = tid; e < p * p; e += nt) {
    const int a = e / p, b = e % p;
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += Gm[q * n + k + a] * A[q * (p + 1) + b];
    const double h1 = Gm[(k + a) * n + k + b] - s;
    double s2 = 0.0;
    for (int q = 0; q < k; ++q) s2 += Gm[q * n + k + b] * A[q * (p + 1) + a];
    const double h2 = Gm[(k + b) * n + k + a] - s2;
    Hm[e] = 0.5 * (h1 + h2);
  }
  for (int a = tid; a < p; a += nt) {
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += Gm[q * n + k + a] * A[q * (p + 1) + p];
    gv[(size_t)m * p + a] = bm[k + a] - s;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += bm[q] * A[q * (p + 1) + p];
    e0v[m] = s;
  }
  if (!Gd) return;
  // N = P~^T D P~ with P~ = P - Z Gzz^-1 Gzp (the candidates made
  // S-orthogonal to Z) from the D-weighted Gram Gd of [Z | P]:
  //   N = Dpp - Dpz A - A^T Dzp + A^T Dzz A,  A = Gzz^-1 Gzp
  const double* Dm = Gd + (size_t)m * n * n;
  for (int e = tid; e < k * p; e += nt) {
    const int q = e / p, b = e % p;
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += Dm[q * n + r] * A[r * (p + 1) + b];
    GA[e] = s;
  }
  __syncthreads();
  double* Nm = Nout + (size_t)m * p * p;
  for (int e = tid; e < p * p; e += nt) {
    const int a = e / p, b = e % p;
    double s1 = Dm[(k + a) * n + k + b], s2 = Dm[(k + b) * n + k + a];
    for (int q = 0; q < k; ++q) {
      const double aqa = A[q * (p + 1) + a], aqb = A[q * (p + 1) + b];
      s1 += aqa * GA[q * p + b] - Dm[(k + a) * n + q] * aqb - aqa * Dm[q * n + k + b];
      s2 += aqb * GA[q * p + a] - Dm[(k + b) * n + q] * aqa - aqb * Dm[q * n + k + a];
    }
    Nm[e] = 0.5 * (s1 + s2);
  }
}

// DV[q] = D V[q] on inactive rows (0 on active ones), D = diag(S_II) =
// a diag + c of the instance (one->a, one->c)
__global__ void k_dscale_cols(int64_t N, const double* Vb, const double* diag, const uint8_t* mask,
                              const Inst* one, double* DV) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= N) return;
  DV[(size_t)q * N + i] = mask[i] ? 0.0 : (one->a * diag[i] + one->c) * Vb[(size_t)q * N + i];
}

// ---------------------------------------------------------------------------
// MLP 4 -> 128 -> 128 -> (NV x P) with exact erf-GELU.  Weights in BF16
// (row-major [out][in]), biases FP32, FP32 accumulation.  One block per
// sample; activations kept for the backward pass.
// ---------------------------------------------------------------------------
constexpr int MD0 = 4, MD1 = 128, MD2 = 128, MD3 = 512;
constexpr int MLP_NV = 8, MLP_P = 64;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {    // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.3989422804014327f;
}

struct MLPW {            // BF16 compute copies and FP32 biases (device)
  const uint16_t* W1; const float* b1;
  const uint16_t* W2; const float* b2;
  const uint16_t* W3; const float* b3;
};

// theta: [B][4]; act: [B][A1 128 | H1 128 | A2 128 | H2 128]; out: [B][512]
__global__ void __launch_bounds__(512) k_mlp_fwd(int B, const float* theta, MLPW w, float* act, float* out) {
  __shared__ float x0[MD0], h1[MD1], h2[MD2];
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  if (s >= B) return;
  if (t < MD0) x0[t] = theta[s * MD0 + t];
  __syncthreads();
  float* as = act + (size_t)s * 4 * MD1;
  if (t < MD1) {
    float a = w.b1[t];
    for (int k = 0; k < MD0; ++k) a += bf2f(w.W1[t * MD0 + k]) * x0[k];
    as[t] = a;
    h1[t] = gelu_f(a);
    as[MD1 + t] = h1[t];
  }
  __syncthreads();
  if (t < MD2) {
    float a = w.b2[t];
    for (int k = 0; k < MD1; ++k) a += bf2f(w.W2[t * MD1 + k]) * h1[k];
    as[2 * MD1 + t] = a;
    h2[t] = gelu_f(a);
    as[3 * MD1 + t] = h2[t];
  }
  __syncthreads();
  if (t < MD3) {
    float a = w.b3[t];
    for (int k = 0; k < MD2; ++k) a += bf2f(w.W3[t * MD2 + k]) * h2[k];
    out[(size_t)s * MD3 + t] = a;
  }
}

// Loss and dL/dC of one sample.  C (NV x p) is the leading p columns of
// out reshaped NV x 64 (row-major); H is p x p and g has p entries:
//   s = C g, T = C H C^T + eps I, u = T^-1 s,
//   L = 1 - (e0 + s.u) / bx,  dL/dC = -(2 u g^T - 2 u u^T C H) / bx.
// Output columns p..63 get zero gradient.  dout is scaled by wscale
// (1 / batch size).
__global__ void __launch_bounds__(512) k_loss_grad(int B, int p, const float* out, const double* H,
                                                   const double* gv, const double* e0v, const double* bxv,
                                                   double eps, float wscale, float* dout, double* lossv) {
  __shared__ double Hs[MLP_P * MLP_P];
  __shared__ double C[MLP_NV * MLP_P], CH[MLP_NV * MLP_P];
  __shared__ double T[MLP_NV * MLP_NV], sv[MLP_NV], u[MLP_NV], gs[MLP_P];
  const int smp = blockIdx.x, t = threadIdx.x;
  if (smp >= B) return;
  const double* Hm = H + (size_t)smp * p * p;
  for (int e = t; e < p * p; e += blockDim.x) Hs[e] = Hm[e];
  for (int e = t; e < MLP_NV * p; e += blockDim.x) C[e] = out[(size_t)smp * MD3 + (e / p) * MLP_P + e % p];
  for (int e = t; e < p; e += blockDim.x) gs[e] = gv[(size_t)smp * p + e];
  __syncthreads();
  for (int e = t; e < MLP_NV * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    double s = 0.0;
    for (int q = 0; q < p; ++q) s += C[i * p + q] * Hs[q * p + j];
    CH[e] = s;
  }
  if (t < MLP_NV) {
    double s = 0.0;
    for (int q = 0; q < p; ++q) s += C[t * p + q] * gs[q];
    sv[t] = s;
  }
  __syncthreads();
  if (t < MLP_NV * MLP_NV) {
    const int i = t / MLP_NV, j = t % MLP_NV;
    double s = 0.0;
    for (int q = 0; q < p; ++q) s += CH[i * p + q] * C[j * p + q];
    T[t] = s + (i == j ? eps : 0.0);
  }
  __syncthreads();
  if (t == 0) {      // 8 x 8 Cholesky solve T u = s (symmetrised T)
    double Lc[MLP_NV * MLP_NV];
    bool ok = true;
    for (int j = 0; j < MLP_NV && ok; ++j) {
      double d = T[j * MLP_NV + j];
      for (int q = 0; q < j; ++q) d -= Lc[j * MLP_NV + q] * Lc[j * MLP_NV + q];
      if (!(d > 0.0)) { ok = false; break; }
      Lc[j * MLP_NV + j] = sqrt(d);
      for (int l = j + 1; l < MLP_NV; ++l) {
        double v = 0.5 * (T[l * MLP_NV + j] + T[j * MLP_NV + l]);
        for (int q = 0; q < j; ++q) v -= Lc[l * MLP_NV + q] * Lc[j * MLP_NV + q];
        Lc[l * MLP_NV + j] = v / Lc[j * MLP_NV + j];
      }
    }
    double y[MLP_NV];
    for (int i = 0; i < MLP_NV; ++i) {
      double v = sv[i];
      for (int q = 0; q < i && ok; ++q) v -= Lc[i * MLP_NV + q] * y[q];
      y[i] = ok ? v / Lc[i * MLP_NV + i] : 0.0;
    }
    for (int i = MLP_NV - 1; i >= 0; --i) {
      double v = y[i];
      for (int q = i + 1; q < MLP_NV && ok; ++q) v -= Lc[q * MLP_NV + i] * u[q];
      u[i] = ok ? v / Lc[i * MLP_NV + i] : 0.0;
    }
    double su = 0.0;
    for (int i = 0; i < MLP_NV; ++i) su += sv[i] * u[i];
    lossv[smp] = 1.0 - (e0v[smp] + su) / bxv[smp];
  }
  __syncthreads();
  const double ib = 1.0 / bxv[smp];
  for (int e = t; e < MLP_NV * MLP_P; e += blockDim.x) {
    const int i = e / MLP_P, j = e % MLP_P;
    double gr = 0.0;
    if (j < p) {
      double uCH = 0.0;
      for (int q = 0; q < MLP_NV; ++q) uCH += u[q] * CH[q * p + j];
      gr = -(2.0 * u[i] * gs[j] - 2.0 * u[i] * uCH) * ib;
    }
    dout[(size_t)smp * MD3 + e] = (float)(gr * wscale);
  }
}

// Deflated-spectrum loss of one sample and its gradient.  C (NV x p) as in
// k_loss_grad; H and N (p x p) are the S_II- and D-weighted Grams of the
// candidates made S_II-orthogonal to the reference modes.  With
// T = C H C^T and U = C N C^T, R = tr(U^-1 T) is the sum of the Ritz values
// of the Jacobi-preconditioned deflated operator on the span of the NV
// enrichment vectors:
//   L = log R,  dL/dC = 2 (U^-1 C H - U^-1 T U^-1 C N) / R.
// A sample whose U is not positive definite (rank-deficient C) gets a NaN
// loss and zero gradient.
__global__ void __launch_bounds__(512) k_loss_grad_spec(int B, int p, const float* out, const double* H,
                                                        const double* Nv, float wscale, float* dout,
                                                        double* lossv) {
  __shared__ double buf[MLP_P * MLP_P];
  __shared__ double C[MLP_NV * MLP_P], CH[MLP_NV * MLP_P], CN[MLP_NV * MLP_P];
  __shared__ double T[MLP_NV * MLP_NV], U[MLP_NV * MLP_NV], X[MLP_NV * MLP_NV], P[MLP_NV * MLP_NV];
  __shared__ double s_r;
  const int smp = blockIdx.x, t = threadIdx.x;
  if (smp >= B) return;
  for (int e = t; e < MLP_NV * p; e += blockDim.x) C[e] = out[(size_t)smp * MD3 + (e / p) * MLP_P + e % p];
  for (int pass = 0; pass < 2; ++pass) {
    const double* src = (pass == 0 ? H : Nv) + (size_t)smp * p * p;
    double* dst = pass == 0 ? CH : CN;
    __syncthreads();
    for (int e = t; e < p * p; e += blockDim.x) buf[e] = src[e];
    __syncthreads();
    for (int e = t; e < MLP_NV * p; e += blockDim.x) {
      const int i = e / p, j = e % p;
      double s = 0.0;
      for (int q = 0; q < p; ++q) s += C[i * p + q] * buf[q * p + j];
      dst[e] = s;
    }
  }
  __syncthreads();
  if (t < 2 * MLP_NV * MLP_NV) {
    const int w = t / (MLP_NV * MLP_NV), o = t % (MLP_NV * MLP_NV);
    const int i = o / MLP_NV, j = o % MLP_NV;
    const double* src = w == 0 ? CH : CN;
    double s = 0.0;
    for (int q = 0; q < p; ++q) s += src[i * p + q] * C[j * p + q];
    (w == 0 ? T : U)[o] = s;
  }
  __syncthreads();
  if (t == 0) {      // X = U^-1 by Cholesky (symmetrised U), R = tr(X T), P = X T X
    double Lc[MLP_NV * MLP_NV];
    bool ok = true;
    for (int j = 0; j < MLP_NV && ok; ++j) {
      double d = U[j * MLP_NV + j];
      for (int q = 0; q < j; ++q) d -= Lc[j * MLP_NV + q] * Lc[j * MLP_NV + q];
      if (!(d > 0.0)) { ok = false; break; }
      Lc[j * MLP_NV + j] = sqrt(d);
      for (int l = j + 1; l < MLP_NV; ++l) {
        double v = 0.5 * (U[l * MLP_NV + j] + U[j * MLP_NV + l]);
        for (int q = 0; q < j; ++q) v -= Lc[l * MLP_NV + q] * Lc[j * MLP_NV + q];
        Lc[l * MLP_NV + j] = v / Lc[j * MLP_NV + j];
      }
    }
    for (int c = 0; c < MLP_NV; ++c) {
      double y[MLP_NV];
      for (int i = 0; i < MLP_NV; ++i) {
        double v = (i == c) ? 1.0 : 0.0;
        for (int q = 0; q < i && ok; ++q) v -= Lc[i * MLP_NV + q] * y[q];
        y[i] = ok ? v / Lc[i * MLP_NV + i] : 0.0;
      }
      for (int i = MLP_NV - 1; i >= 0; --i) {
        double v = y[i];
        for (int q = i + 1; q < MLP_NV && ok; ++q) v -= Lc[q * MLP_NV + i] * X[q * MLP_NV + c];
        X[i * MLP_NV + c] = ok ? v / Lc[i * MLP_NV + i] : 0.0;
      }
    }
    double r = 0.0;
    for (int i = 0; i < MLP_NV; ++i)
      for (int j = 0; j < MLP_NV; ++j) r += X[i * MLP_NV + j] * 0.5 * (T[j * MLP_NV + i] + T[i * MLP_NV + j]);
    double XT[MLP_NV * MLP_NV];
    for (int i = 0; i < MLP_NV; ++i)
      for (int j = 0; j < MLP_NV; ++j) {
        double v = 0.0;
        for (int q = 0; q < MLP_NV; ++q) v += X[i * MLP_NV + q] * 0.5 * (T[q * MLP_NV + j] + T[j * MLP_NV + q]);
        XT[i * MLP_NV + j] = v;
      }
    for (int i = 0; i < MLP_NV; ++i)
      for (int j = 0; j < MLP_NV; ++j) {
        double v = 0.0;
        for (int q = 0; q < MLP_NV; ++q) v += XT[i * MLP_NV + q] * X[q * MLP_NV + j];
        P[i * MLP_NV + j] = v;
      }
    ok = ok && r > 0.0 && isfinite(r);
    s_r = ok ? r : 0.0;
    lossv[smp] = ok ? log(r) : __builtin_nan("");
  }
  __syncthreads();
  const double r = s_r;
  for (int e = t; e < MLP_NV * MLP_P; e += blockDim.x) {
    const int i = e / MLP_P, j = e % MLP_P;
    double gr = 0.0;
    if (j < p && r > 0.0) {
      double v = 0.0;
      for (int q = 0; q < MLP_NV; ++q) v += X[i * MLP_NV + q] * CH[q * p + j] - P[i * MLP_NV + q] * CN[q * p + j];
      gr = 2.0 * v / r;
    }
    dout[(size_t)smp * MD3 + e] = (float)(gr * wscale);
  }
}

// per-sample backward through the activations: dA2 (128), dA1 (128)
__global__ void __launch_bounds__(128) k_mlp_bwd_act(int B, MLPW w, const float* act, const float* dout,
                                                     float* dA2, float* dA1) {
  __shared__ float d2[MD2];
  const int s = blockIdx.x, t = threadIdx.x;
  if (s >= B) return;
  const float* as = act + (size_t)s * 4 * MD1;
  float g = 0.0f;
  for (int j = 0; j < MD3; ++j) g += dout[(size_t)s * MD3 + j] * bf2f(w.W3[j * MD2 + t]);
  d2[t] = g * gelu_d(as[2 * MD1 + t]);
  dA2[(size_t)s * MD2 + t] = d2[t];
  __syncthreads();
  float g1 = 0.0f;
  for (int j = 0; j < MD2; ++j) g1 += d2[j] * bf2f(w.W2[j * MD1 + t]);
  dA1[(size_t)s * MD1 + t] = g1 * gelu_d(as[t]);
}

// weight / bias gradients summed over the batch:
//   dW[o][i] = sum_s dA[s][o] X[s][i],  db[o] = sum_s dA[s][o]
__global__ void k_mlp_wgrad(int B, int nout, int nin, const float* dA, int ldA, const float* X, int ldX,
                            int offX, float* dW, float* db) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nout * nin) {
    const int o = e / nin, i = e % nin;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dA[(size_t)b * ldA + o] * X[(size_t)b * ldX + offX + i];
    dW[e] = s;
  }
  if (e < nout) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dA[(size_t)b * ldA + e];
    db[e] = s;
  }
}

// Adam (Kingma & Ba 2015) on FP32 master parameters; refreshes the BF16 copy
__global__ void k_adam(int n, float* p, const float* g, float* mo, float* ve, uint16_t* bf, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float m = b1 * mo[i] + (1.0f - b1) * gi;
  const float v = b2 * ve[i] + (1.0f - b2) * gi * gi;
  mo[i] = m;
  ve[i] = v;
  const float pn = p[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  p[i] = pn;
  if (bf) bf[i] = f2bf(pn);
}

__global__ void k_to_bf16(int n, const float* p, uint16_t* bf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) bf[i] = f2bf(p[i]);
}

// Per-instance basis [Z | V_m], V_m = Phi C_m^T  (column-major, KP columns,
// FP64 and FP32), C_m = out[m] reshaped NV x P.
__global__ void k_expand_basis(int64_t N, int k, int KP, int p, const double* Z, const double* Phi,
                               const float* out, double* Zb64, float* Zb32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  const int m = blockIdx.z;
  if (i >= N) return;
  double v = 0.0;
  if (q < k) {
    v = Z[(size_t)q * N + i];
  } else if (q < k + MLP_NV) {
    const float* Cm = out + (size_t)m * MD3 + (size_t)(q - k) * MLP_P;
    for (int j = 0; j < p; ++j) v += (double)Cm[j] * Phi[(size_t)j * N + i];
  }
  Zb64[((size_t)m * KP + q) * N + i] = v;
  Zb32[((size_t)m * KP + q) * N + i] = (float)v;
}

// W[:, q] = a A^T T[:, q] + c Vtilde[:, q] on inactive rows (0 on active
// rows): S_II applied to the columns of V (factored operator, FP64).
__global__ void k_outer_cols(OpGeom op, const double* AT64, const double* T, const double* Vb,
                             const uint8_t* mask, const Inst* one, double* Wv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  const int64_t N = op.N;
  if (i >= N) return;
  double v = 0.0;
  if (mask[i] == 0) {
    const double* Tq = T + (size_t)q * N;
    double acc = 0.0;
    for (int d = 0; d < op.D; ++d) {
      const int64_t j = i + op.offs[d];
      if (j >= 0 && j < N) acc += AT64[(size_t)d * N + i] * Tq[j];
    }
    v = one->a * acc + one->c * Vb[(size_t)q * N + i];
  }
  Wv[(size_t)q * N + i] = v;
}

}  // namespace adef2
