// Streaming kernels of the restricted A-DEF2 solve (gfx950, wave64).
//
// Data layout (all in HBM, global node order, lexicographic, x fastest):
//   S     : diagonal format, dia[d * N + i] = S[i, i + offs[d]] (0 if absent)
//   Z     : column-major N x KP (shared by all instances, zero padded columns)
//   W     : per instance, column-major N x KP, W = S_II Z_I
//   x,r,z,p,w : per instance, length N + 2H with H zero halo entries on both
//           sides, so the stencil reads i + offs[d] need no bounds test;
//           entries on the active set are kept at exactly 0, which makes
//           S (masked vector) restricted to inactive rows equal to S_II.
// Every kernel processes rows of one instance per blockIdx.y.
#pragma once
#include "dev_common.h"

namespace adef2 {

constexpr int MAXD = 64;

struct OpGeom {
  int64_t N;
  int D;
  int ntiles;        // tiles covering N rows
  int ntiles_pad;    // multiple of 8 (XCD mapping)
  int offs[MAXD];
};

template <typename V>
struct IterArgs {
  OpGeom op;
  const V* dia;            // [D][N]
  const uint8_t* mask;     // [B][N]
  const V* dinv;           // [B][N]
  const V* Z;              // [KP][N]
  const V* W;              // [B][KP][N]
  V* x; V* r; V* z; V* p; V* w;   // padded, pointer to instance 0 interior
  int64_t vs;              // padded vector stride
  Inst* inst;              // [B]
  const double* C;         // [B][KP][KP] row-major coarse operator E^{-1}
  double* part;            // reduction partials
  unsigned* ctr;           // reduction counters
  RedGeom g;
  int32_t maxit;
  // init only
  const double* src;       // [B][N] right-hand side of the sweep
  const double* x0;        // padded FP64 warm start (stride x0s) or null
  int64_t x0s;
  double thresh_scale;     // thresh2 = thresh_scale * ||src_I||^2
};

template <int RPT> struct Rows { static constexpr int PB = TPB * RPT; };

// coef[q] = sum_l C[q][l] g[l]  (finisher only; g, coef in LDS/global)
template <int KP>
__device__ __forceinline__ void coarse_apply(const double* Cm, const double* g, double* coef) {
  for (int q = threadIdx.x; q < KP; q += blockDim.x) {
    double s = 0.0;
    for (int l = 0; l < KP; ++l) s += Cm[q * KP + l] * g[l];
    coef[q] = s;
  }
}

// ---------------------------------------------------------------------------
// init: r0 = src - S x0 (or src), g = Z^T r0, ||src||^2;  finisher: c0 = C g
// ---------------------------------------------------------------------------
template <typename V, int KP, int RPT>
__global__ void __launch_bounds__(TPB) k_init(IterArgs<V> a) {
  constexpr int NV = KP + 1;
  __shared__ double red[NWAVE * NV];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  const int m = blockIdx.y;
  Inst* S = a.inst + m;
  if (S->outer_done) return;
  const int tile = xcd_tile(blockIdx.x, a.op.ntiles_pad);
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const double* src = a.src + (size_t)m * N;
  V* x = a.x + m * a.vs;
  V* r = a.r + m * a.vs;
  const double sa = S->a, sc = S->c;
  double v[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = 0.0;
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        const double s = src[i];
        double r0 = s, xv = 0.0;
        if (a.x0) {
          const double* x0 = a.x0 + m * a.x0s;
          double acc = 0.0;
          for (int d = 0; d < a.op.D; ++d) acc += (double)a.dia[(size_t)d * N + i] * x0[i + a.op.offs[d]];
          xv = x0[i];
          r0 = s - (sa * acc + sc * xv);
        }
        x[i] = (V)xv;
        r[i] = (V)r0;
        v[KP] += s * s;
#pragma unroll
        for (int q = 0; q < KP; ++q) v[q] += (double)a.Z[(size_t)q * N + i] * r0;
      }
    }
  }
  block_sum<NV>(v, red, bv);
  double* part = a.part + (size_t)m * a.g.ptotal * NV;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, NV, part, ctr, bv, tot)) return;
  if (threadIdx.x == 0) {
    const double bb = tot[KP];
    S->bb = bb;
    S->thresh2 = a.thresh_scale * bb;
    S->done = 0;
    S->sweep_iters = 0;
    S->fresh = 1;
    if (!(bb < INFINITY)) { S->done = 1; S->outer_done = 1; S->status = -1; }
    else if (bb == 0.0) { S->done = 1; }
  }
  if (S->kk > 0) coarse_apply<KP>(a.C + (size_t)m * KP * KP, tot, S->coef);
  else for (int q = threadIdx.x; q < KP; q += blockDim.x) S->coef[q] = 0.0;
}

// ---------------------------------------------------------------------------
// init2: x += Z c0, r -= W c0, z = K r;  rho = r.z, ||r||^2, g = W^T z
// ---------------------------------------------------------------------------
template <typename V, int KP, int RPT>
__global__ void __launch_bounds__(TPB) k_init2(IterArgs<V> a) {
  constexpr int NV = KP + 2;
  __shared__ double red[NWAVE * NV];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  __shared__ double cf[KP > 0 ? KP : 1];
  const int m = blockIdx.y;
  Inst* S = a.inst + m;
  if (S->outer_done) return;
  const int tile = xcd_tile(blockIdx.x, a.op.ntiles_pad);
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  V* x = a.x + m * a.vs;
  if (S->done) {   // zero right-hand side: x = 0 is the solution
    if (S->bb == 0.0 && tile < a.op.ntiles) {
      for (int rr = 0; rr < RPT; ++rr) {
        const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
        if (i < N) x[i] = (V)0;
      }
    }
    return;
  }
  V* r = a.r + m * a.vs;
  V* z = a.z + m * a.vs;
  const V* dinv = a.dinv + (size_t)m * N;
  const V* W = a.W + (size_t)m * KP * N;
  const bool defl = S->kk > 0;
  for (int q = threadIdx.x; q < KP; q += blockDim.x) cf[q] = S->coef[q];
  __syncthreads();
  double v[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = 0.0;
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        double xv = (double)x[i], rv = (double)r[i];
        if (defl) {
#pragma unroll
          for (int q = 0; q < KP; ++q) {
            xv += (double)a.Z[(size_t)q * N + i] * cf[q];
            rv -= (double)W[(size_t)q * N + i] * cf[q];
          }
        }
        const double zv = (double)dinv[i] * rv;
        x[i] = (V)xv;
        r[i] = (V)rv;
        z[i] = (V)zv;
        const double zq = (double)(V)zv;
        v[KP] += rv * zq;
        v[KP + 1] += rv * rv;
        if (defl) {
#pragma unroll
          for (int q = 0; q < KP; ++q) v[q] += (double)W[(size_t)q * N + i] * zq;
        }
      }
    }
  }
  block_sum<NV>(v, red, bv);
  double* part = a.part + (size_t)m * a.g.ptotal * NV;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, NV, part, ctr, bv, tot)) return;
  const bool stop = !(tot[KP + 1] > S->thresh2);
  if (threadIdx.x == 0) {
    S->rho = tot[KP];
    S->rr = tot[KP + 1];
    S->beta = 0.0;
    S->fresh = 1;
    if (stop) S->done = 1;
  }
  if (!stop && defl) coarse_apply<KP>(a.C + (size_t)m * KP * KP, tot, S->coef);
}

// ---------------------------------------------------------------------------
// p = z - Z c + beta p   (A-DEF2 projected search direction)
// ---------------------------------------------------------------------------
template <typename V, int KP, int RPT>
__global__ void __launch_bounds__(TPB) k_pupdate(IterArgs<V> a) {
  __shared__ double cf[KP > 0 ? KP : 1];
  const int m = blockIdx.y;
  const Inst* S = a.inst + m;
  if (S->done) return;
  const int tile = xcd_tile(blockIdx.x, a.op.ntiles_pad);
  if (tile >= a.op.ntiles) return;
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const V* z = a.z + m * a.vs;
  V* p = a.p + m * a.vs;
  const bool defl = S->kk > 0;
  const double beta = S->fresh ? 0.0 : S->beta;
  const bool keep = !S->fresh;
  for (int q = threadIdx.x; q < KP; q += blockDim.x) cf[q] = S->coef[q];
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
    if (i < N && mk[i] == 0) {
      double pv = (double)z[i];
      if (defl) {
#pragma unroll
        for (int q = 0; q < KP; ++q) pv -= (double)a.Z[(size_t)q * N + i] * cf[q];
      }
      if (keep) pv += beta * (double)p[i];
      p[i] = (V)pv;
    }
  }
}

// ---------------------------------------------------------------------------
// w = S_II p, p.w;  finisher: alpha = rho / p.w
// ---------------------------------------------------------------------------
template <typename V, int KP, int RPT>
__global__ void __launch_bounds__(TPB) k_spmv(IterArgs<V> a) {
  __shared__ double red[NWAVE];
  __shared__ double bv[1];
  __shared__ double tot[1];
  const int m = blockIdx.y;
  Inst* S = a.inst + m;
  if (S->done) return;
  const int tile = xcd_tile(blockIdx.x, a.op.ntiles_pad);
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const V* p = a.p + m * a.vs;
  V* w = a.w + m * a.vs;
  const double sa = S->a, sc = S->c;
  double v[1] = {0.0};
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        double acc = 0.0;
        for (int d = 0; d < a.op.D; ++d)
          acc += (double)a.dia[(size_t)d * N + i] * (double)p[i + a.op.offs[d]];
        const double pi = (double)p[i];
        const double wv = sa * acc + sc * pi;
        w[i] = (V)wv;
        v[0] += pi * (double)(V)wv;
      }
    }
  }
  block_sum<1>(v, red, bv);
  double* part = a.part + (size_t)m * a.g.ptotal * 1;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, 1, part, ctr, bv, tot)) return;
  if (threadIdx.x == 0) {
    const double pw = tot[0];
    S->pw = pw;
    if (!(pw > 0.0) || !(pw < INFINITY)) {
      S->done = 1;
      S->outer_done = 1;
      S->status = -5;
    } else {
      S->alpha = S->rho / pw;
    }
  }
}

// ---------------------------------------------------------------------------
// x += alpha p, r -= alpha w, z = K r;  r.z, ||r||^2, g = W^T z
// finisher: stopping test, beta, coef = C g
// ---------------------------------------------------------------------------
template <typename V, int KP, int RPT>
__global__ void __launch_bounds__(TPB) k_update(IterArgs<V> a) {
  constexpr int NV = KP + 2;
  __shared__ double red[NWAVE * NV];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  const int m = blockIdx.y;
  Inst* S = a.inst + m;
  if (S->done) return;
  const int tile = xcd_tile(blockIdx.x, a.op.ntiles_pad);
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  V* x = a.x + m * a.vs;
  V* r = a.r + m * a.vs;
  V* z = a.z + m * a.vs;
  const V* p = a.p + m * a.vs;
  const V* w = a.w + m * a.vs;
  const V* dinv = a.dinv + (size_t)m * N;
  const V* W = a.W + (size_t)m * KP * N;
  const bool defl = S->kk > 0;
  const double alpha = S->alpha;
  double v[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = 0.0;
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        const double xv = (double)x[i] + alpha * (double)p[i];
        const double rv = (double)r[i] - alpha * (double)w[i];
        const V rq = (V)rv;
        const V zq = (V)((double)dinv[i] * (double)rq);
        x[i] = (V)xv;
        r[i] = rq;
        z[i] = zq;
        v[KP] += (double)rq * (double)zq;
        v[KP + 1] += (double)rq * (double)rq;
        if (defl) {
#pragma unroll
          for (int q = 0; q < KP; ++q) v[q] += (double)W[(size_t)q * N + i] * (double)zq;
        }
      }
    }
  }
  block_sum<NV>(v, red, bv);
  double* part = a.part + (size_t)m * a.g.ptotal * NV;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, NV, part, ctr, bv, tot)) return;
  __shared__ int s_go;
  if (threadIdx.x == 0) {
    const double rz = tot[KP], rr = tot[KP + 1];
    S->iters += 1;
    S->sweep_iters += 1;
    S->rr = rr;
    int go = 0;
    if (!(rr > S->thresh2)) {
      S->done = 1;
      if (!(rr < INFINITY)) { S->outer_done = 1; S->status = -5; }
    } else if (S->iters >= a.maxit) {
      S->done = 1;
      S->outer_done = 1;
      S->status = 2;
    } else {
      S->beta = rz / S->rho;
      S->rho = rz;
      S->fresh = 0;
      go = 1;
    }
    s_go = go;
  }
  __syncthreads();
  if (s_go && defl) coarse_apply<KP>(a.C + (size_t)m * KP * KP, tot, S->coef);
}

// ---------------------------------------------------------------------------
// FP64 outer residual: r64 = b - S_II x64 (optionally stored), ||r64||^2,
// ||b_I||^2; finisher applies the outer stopping test (refinement mode).
// ---------------------------------------------------------------------------
struct ResidArgs {
  OpGeom op;
  const double* dia;       // FP64 [D][N]
  const uint8_t* mask;
  const double* b;         // [B][N]
  const double* x;         // padded FP64 [B][vs]
  int64_t vs;
  double* r64;             // [B][N] or null
  Inst* inst;
  double* part; unsigned* ctr; RedGeom g;
  int32_t first;           // compute ||b_I||^2 (first outer step)
  int32_t decide;          // apply the outer stopping rule
  double tol2;
  int32_t maxit, max_sweeps;
};

template <int RPT>
__global__ void __launch_bounds__(TPB) k_resid64(ResidArgs a) {
  __shared__ double red[NWAVE * 2];
  __shared__ double bv[2];
  __shared__ double tot[2];
  const int m = blockIdx.y;
  Inst* S = a.inst + m;
  if (S->outer_done && a.decide) return;
  const int tile = xcd_tile(blockIdx.x, a.op.ntiles_pad);
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const double* b = a.b + (size_t)m * N;
  const double* x = a.x + m * a.vs;
  const double sa = S->a, sc = S->c;
  double v[2] = {0.0, 0.0};
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        double acc = 0.0;
        for (int d = 0; d < a.op.D; ++d) acc += a.dia[(size_t)d * N + i] * x[i + a.op.offs[d]];
        const double bi = b[i];
        const double rv = bi - (sa * acc + sc * x[i]);
        if (a.r64) a.r64[(size_t)m * N + i] = rv;
        v[0] += rv * rv;
        v[1] += bi * bi;
      }
    }
  }
  block_sum<2>(v, red, bv);
  double* part = a.part + (size_t)m * a.g.ptotal * 2;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, 2, part, ctr, bv, tot)) return;
  if (threadIdx.x == 0) {
    S->rr64 = tot[0];
    if (a.first) S->bb64 = tot[1];
    if (a.decide) {
      const double bb = S->bb64;
      if (!(bb < INFINITY) || !(tot[0] < INFINITY)) { S->outer_done = 1; S->status = -1; }
      else if (!(tot[0] > a.tol2 * bb)) { S->outer_done = 1; }
      else if (S->iters >= a.maxit || S->sweeps >= a.max_sweeps) { S->outer_done = 1; S->status = 2; }
      S->done = 1;
    }
  }
}

// x64 += d (FP32 correction of the last sweep)
template <int RPT>
__global__ void __launch_bounds__(TPB) k_accumulate(OpGeom op, const uint8_t* mask, const float* d,
                                                    double* x64, int64_t vs, Inst* inst) {
  const int m = blockIdx.y;
  Inst* S = inst + m;
  if (S->outer_done) return;
  const int tile = xcd_tile(blockIdx.x, op.ntiles_pad);
  if (tile >= op.ntiles) return;
  const int64_t N = op.N;
  const uint8_t* mk = mask + (size_t)m * N;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * TPB + threadIdx.x;
    if (i < N && mk[i] == 0) x64[m * vs + i] += (double)d[m * vs + i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) S->sweeps += 1;
}

// out[i] = x[i] on inactive rows, 0 on active rows (instance-major, unpadded)
__global__ void k_scatter_out(int64_t N, const uint8_t* mask, const double* x, int64_t vs, double* out,
                              const Inst* inst) {
  const int m = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const bool act = mask[(size_t)m * N + i] != 0;
  out[(size_t)m * N + i] = act ? 0.0 : x[m * vs + i];
  (void)inst;
}

template <typename V>
__global__ void k_fill(V* p, int64_t n, V val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < n; j += stride) p[j] = val;
}

// padded copy: dst[m*vs + i] = src[m*N + i]
__global__ void k_copy_padded(int64_t N, const double* src, double* dst, int64_t vs) {
  const int m = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[m * vs + i] = src[(size_t)m * N + i];
}

// dst[i] = src[i] on inactive rows, 0 on active rows (padded destination)
__global__ void k_mask_copy_padded(int64_t N, const uint8_t* mask, const double* src, double* dst,
                                   int64_t vs) {
  const int m = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[m * vs + i] = mask[(size_t)m * N + i] ? 0.0 : src[(size_t)m * N + i];
}

// y = S_II x (global layout, FP64): x padded with zeros on the active set
__global__ void k_apply64(OpGeom op, const double* dia, const uint8_t* mask, const double* x,
                          double* y, const Inst* inst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  double v = 0.0;
  if (mask[i] == 0) {
    double acc = 0.0;
    for (int d = 0; d < op.D; ++d) acc += dia[(size_t)d * N + i] * x[i + op.offs[d]];
    v = inst->a * acc + inst->c * x[i];
  }
  y[i] = v;
}

// Jacobi preconditioner of the restricted operator: dinv = 1 / (a d + c) on
// inactive rows (1 without preconditioner), 0 on active rows.
template <typename V>
__global__ void k_dinv(int64_t N, const double* diag, const uint8_t* mask, V* dinv, Inst* inst,
                       int precond_none) {
  const int m = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  Inst* S = inst + m;
  const bool act = mask[(size_t)m * N + i] != 0;
  double v = 0.0;
  if (!act) {
    const double dd = S->a * diag[i] + S->c;
    if (!(dd > 0.0)) S->setup_status = -5;
    v = precond_none ? 1.0 : 1.0 / dd;
  }
  dinv[(size_t)m * N + i] = (V)v;
}

}  // namespace adef2
