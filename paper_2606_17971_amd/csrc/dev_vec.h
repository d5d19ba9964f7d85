// Kernels of the host runtime's translation unit: the FP64 outer residual of
// the refinement modes, the inner stencil of the factored operator, the fused
// operator pass of the factored form (one instance or a group of four per
// block), the accumulation of FP32 corrections, scatter / copy / fill
// helpers, the restricted matvec test hook and the Jacobi preconditioner.
#pragma once
#include "dev_tile.h"

namespace adef2 {

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
  const double* sv;        // stencil source: x, or A x (factored)
  int64_t vs;
  double* r64;             // [B][N] or null
  Inst* inst;
  double* part; unsigned* ctr; RedGeom g;
  int32_t first;           // compute ||b_I||^2 (first outer step)
  int32_t decide;          // apply the outer stopping rule
  int32_t maxit, max_sweeps;
  int32_t stall_steps;     // outer steps without halving before W_STAGNATED
  int32_t trans_mode;      // only instances whose sweep has ended (sweep transition)
};

template <int RPT>
__global__ void __launch_bounds__(IPB) k_resid64(ResidArgs a) {
  __shared__ double red[NIWAVE * 2];
  __shared__ double bv[2];
  __shared__ double tot[2];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->outer_done && a.decide) return;
  if (a.trans_mode && !S->done) return;
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const double* b = a.b + (size_t)m * N;
  const double* x = a.x + m * a.vs;
  const double* sv = a.sv + m * a.vs;
  const double sa = S->a, sc = S->c;
  double v[2] = {0.0, 0.0};
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * IPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        double acc = 0.0;
        for (int d = 0; d < a.op.D; ++d) acc += a.dia[(size_t)d * N + i] * sv[i + a.op.offs[d]];
        const double bi = b[i];
        const double rv = bi - (sa * acc + sc * x[i]);
        if (a.r64) a.r64[(size_t)m * N + i] = rv;
        v[0] += rv * rv;
        v[1] += bi * bi;
      }
    }
  }
  block_sum<2, NIWAVE>(v, red, bv);
  double* part = a.part + (size_t)m * a.g.ptotal * 2;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, 2, part, ctr, bv, tot)) return;
  if (threadIdx.x == 0) {
    S->rr64_prev = a.first ? INFINITY : S->rr64;
    S->rr64 = tot[0];
    if (a.first) S->bb64 = tot[1];
    if (a.decide) {
      const double bb = S->bb64;
      const double r2 = tot[0];
      // Drift: the FP64 residual exceeds the recurrence residual the sweep
      // ended with by more than 2x (while the iteration is accurate the two
      // agree to a few per cent); the next sweep then restarts its direction.
      // Attainable-accuracy guard: the best FP64 residual has not halved over
      // the last stall_steps sweeps that converged on their own equation (a
      // sweep stopped by the segment cap is no evidence: CG's residual 2-norm
      // is not monotone)
      S->drift = a.first ? 0 : (r2 > 4.0 * S->rr);
      if (a.first || r2 < 0.25 * S->rr64_best) { S->rr64_best = r2; S->stall = 0; }
      else if (!S->capped) S->stall += 1;
      if (!(bb < INFINITY) || !(r2 < INFINITY)) { S->outer_done = 1; S->status = -1; }
      else if (!(r2 > S->tol2 * bb)) { S->outer_done = 1; }
      else if (S->stall >= a.stall_steps) { S->outer_done = 1; S->status = 3; }
      else if (S->iters >= a.maxit || S->sweeps >= a.max_sweeps) { S->outer_done = 1; S->status = 2; }
      S->done = 1;
    }
  }
}

// Inner stencil of the factored operator on all rows: t = A v (v is zero on
// the active set, so t = A[:, I] v_I).  skip: 1 = skip instances whose sweep is
// done, 2 = skip finished solves, 3 = only instances whose sweep has ended
// (sweep transition), 0 = none.
template <typename VM, typename VI, typename VO, int RPT>
__global__ void __launch_bounds__(IPB) k_stencil1(OpGeom op, const VM* dia1, const VI* v, VO* t,
                                                  int64_t vs, const Inst* inst, int skip) {
  int tile, m;
  tile_inst(op.ntiles_pad, tile, m);
  const Inst* S = inst + m;
  if ((skip == 1 && S->done) || (skip == 2 && S->outer_done) || (skip == 3 && (S->outer_done || !S->done)))
    return;
  if (tile >= op.ntiles) return;
  const int64_t N = op.N;
  const VI* vm = v + m * vs;
  VO* tm = t + m * vs;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * IPB + threadIdx.x;
    if (i < N) {
      tm[i] = (VO)stencil_row(dia1, op.offs1, op.D1, op.d01, N, i, vm);
    }
  }
}

// ---------------------------------------------------------------------------
// Fused operator pass of the factored form: w = a A^T (A p) + c p on the
// inactive rows of one tile, p.w, and alpha = rho / p.w.  One block per
// (tile, instance), tile = of_rows consecutive rows [i0, i0 + R).  The inner
// product t = A p is formed for rows [i0 - Ho, i0 + R + Ho) (Ho = the reach of
// the outer stencil A^T) into LDS and never written to HBM; rows outside
// [0, N) hold 0, as the zero halo of the padded t does.  The arithmetic of
// each row (difference form for FP32 coefficients, t rounded to the vector
// type) is that of k_stencil1 followed by k_spmv; only the p.w reduction tree
// differs (one leaf per fused tile).  The rows of the halo are recomputed by
// the neighbouring tiles' blocks (2 Ho / R more inner stencil work, from L2).
// Dynamic LDS: (R + 2 Ho) doubles.
// ---------------------------------------------------------------------------
// One row of a stencil from its coefficients cw[] and source values vw[]
// (DC diagonals, already loaded): the arithmetic and order of stencil_row
// (difference form with FP32 coefficients when the stencil has an offset-0
// slot d0).
template <typename M, int DC>
__device__ __forceinline__ double stencil_combine(const double (&cw)[DC], const double (&vw)[DC], int d0) {
  double acc = 0.0;
  if constexpr (sizeof(M) == 4) {
    if (d0 >= 0) {
      double vi = 0.0, dg = 0.0;
#pragma unroll
      for (int d = 0; d < DC; ++d)
        if (d == d0) { vi = vw[d]; dg = cw[d]; }
      acc = dg * vi;
#pragma unroll
      for (int d = 0; d < DC; ++d)
        if (d != d0) acc += cw[d] * (vw[d] - vi);
      return acc;
    }
  }
#pragma unroll
  for (int d = 0; d < DC; ++d) acc += cw[d] * vw[d];
  return acc;
}

// DC: diagonals of both stencils known at compile time (0 = any: one row at
// a time through stencil_row).  With DC > 0 each thread loads the
// coefficients and sources of OU rows before it combines any of them, so
// their loads are in flight together (row indices are clamped into range so
// that no load is conditional; rows out of range are discarded).
template <typename V, typename M, int DC>
__global__ void __launch_bounds__(IPB) k_opfused(IterArgs<V, M> a) {
  constexpr int OU = DC > 0 ? 4 : 1;
  constexpr int DX = DC > 0 ? DC : 1;
  extern __shared__ double ts[];
  __shared__ double red[NIWAVE];
  __shared__ double bv[1];
  __shared__ double tot[1];
  int tile, m;
  tile_inst(a.of_ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->done) return;
  const int64_t N = a.op.N;
  const int R = a.of_rows, Ho = a.of_halo;
  const int64_t i0 = (int64_t)tile * R;
  const V* p = a.p + m * a.vs;
  const uint8_t* mk = a.mask + (size_t)m * N;
  V* w = a.w + m * a.vs;
  const double sa = S->a, sc = S->c;
  double v[1] = {0.0};
  const bool live = tile < a.of_ntiles;
  if (live) {
    const int L = R + 2 * Ho;
    for (int e0 = threadIdx.x; e0 < L; e0 += OU * IPB) {
      double tv[OU];
      if constexpr (DC > 0) {
        double cw[OU][DX], vw[OU][DX];
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          const int64_t j = i0 - Ho + e0 + u * IPB;
          const int64_t jc = j < 0 ? 0 : (j >= N ? N - 1 : j);
#pragma unroll
          for (int d = 0; d < DC; ++d) {
            cw[u][d] = (double)a.dia1[(size_t)d * N + jc];
            vw[u][d] = (double)p[jc + a.op.offs1[d]];
          }
        }
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          const int64_t j = i0 - Ho + e0 + u * IPB;
          tv[u] = (j < 0 || j >= N) ? 0.0 : (double)(V)stencil_combine<M, DX>(cw[u], vw[u], a.op.d01);
        }
      } else {
        const int64_t j = i0 - Ho + e0;
        tv[0] = (j >= 0 && j < N) ? (double)(V)stencil_row(a.dia1, a.op.offs1, a.op.D1, a.op.d01, N, j, p) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < OU; ++u)
        if (e0 + u * IPB < L) ts[e0 + u * IPB] = tv[u];
    }
  }
  __syncthreads();
  if (live) {
    for (int e0 = threadIdx.x; e0 < R; e0 += OU * IPB) {
      double wv[OU], pv[OU];
      bool ok[OU];
      if constexpr (DC > 0) {
        double cw[OU][DX], vw[OU][DX];
        uint8_t mv[OU];
        int ec[OU];
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          const int e = e0 + u * IPB;
          const int64_t i = i0 + (e < R ? e : R - 1);
          const int64_t ic = i < N ? i : N - 1;      // i0 <= ic < min(i0 + R, N)
          ec[u] = (int)(ic - i0) + Ho;
          mv[u] = mk[ic];
          pv[u] = (double)p[ic];
#pragma unroll
          for (int d = 0; d < DC; ++d) cw[u][d] = (double)a.dia[(size_t)d * N + ic];
          ok[u] = (e < R) & (i < N);
        }
#pragma unroll
        for (int u = 0; u < OU; ++u) {
#pragma unroll
          for (int d = 0; d < DC; ++d) vw[u][d] = ts[ec[u] + a.op.offs[d]];
          ok[u] = ok[u] & (mv[u] == 0);
          wv[u] = sa * stencil_combine<M, DX>(cw[u], vw[u], a.op.d0) + sc * pv[u];
        }
      } else {
        const int64_t i = i0 + e0;
        ok[0] = i < N && mk[i] == 0;
        pv[0] = wv[0] = 0.0;
        if (ok[0]) {
          double acc = 0.0;
          const int d0 = a.op.d0, li = e0 + Ho;
          if (sizeof(M) == 4 && d0 >= 0) {
            const double ti = ts[li];
            acc = (double)a.dia[(size_t)d0 * N + i] * ti;
            for (int d = 0; d < a.op.D; ++d)
              if (d != d0) acc += (double)a.dia[(size_t)d * N + i] * (ts[li + a.op.offs[d]] - ti);
          } else {
            for (int d = 0; d < a.op.D; ++d) acc += (double)a.dia[(size_t)d * N + i] * ts[li + a.op.offs[d]];
          }
          pv[0] = (double)p[i];
          wv[0] = sa * acc + sc * pv[0];
        }
      }
#pragma unroll
      for (int u = 0; u < OU; ++u) {
        if (!ok[u]) continue;
        w[i0 + e0 + u * IPB] = (V)wv[u];
        v[0] += pv[u] * (double)(V)wv[u];
      }
    }
  }
  block_sum<1, NIWAVE>(v, red, bv);
  double* part = a.part + (size_t)m * a.gof.ptotal;
  unsigned* ctr = a.ctr + (size_t)m * a.gof.ctotal;
  if (!tree_reduce(a.gof, tile, 1, part, ctr, bv, tot)) return;
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

// Grouped form of the fused operator pass: one block per tile and group of
// G instances, so the coefficients of a row (shared by every instance) are
// loaded once for the group instead of once per instance; each instance has
// its own LDS copy of t (dynamic LDS: G (R + 2 Ho) doubles).  Same per-row
// arithmetic as k_opfused; the p.w trees of the group's instances advance
// together (tree_reduce_multi).  DC > 0 only; OU rows per thread and step.
template <typename V, typename M, int DC, int G>
__global__ void __launch_bounds__(IPB) k_opfused_g(IterArgs<V, M> a) {
  static_assert(DC > 0 && G >= 2 && G <= 8, "grouped fused pass: compile-time stencil, 2..8 instances");
  constexpr int OU = 2;
  extern __shared__ double ts[];
  __shared__ double red[NIWAVE * G];
  __shared__ double bvv[G];
  __shared__ double tot[G];
  int tile, grp;
  tile_group(a.of_ntiles_pad, a.of_ngroups, tile, grp);
  const int g0 = grp * G;
  const int Gn = min(G, a.B - g0);
  unsigned act = 0u;
  double sa[G], sc[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    sa[j] = sc[j] = 0.0;
    if (j < Gn) {
      const Inst* S = a.inst + g0 + j;
      if (!S->done) {
        act |= 1u << j;
        sa[j] = S->a;
        sc[j] = S->c;
      }
    }
  }
  if (!act) return;
  const int64_t N = a.op.N;
  const int R = a.of_rows, Ho = a.of_halo;
  const int L = R + 2 * Ho;
  const int64_t i0 = (int64_t)tile * R;
  double v[G];
#pragma unroll
  for (int j = 0; j < G; ++j) v[j] = 0.0;
  const bool live = tile < a.of_ntiles;
  if (live) {
    for (int e0 = threadIdx.x; e0 < L; e0 += OU * IPB) {
      double cw[OU][DC];
      int64_t jc[OU];
#pragma unroll
      for (int u = 0; u < OU; ++u) {
        const int64_t j = i0 - Ho + e0 + u * IPB;
        jc[u] = j < 0 ? 0 : (j >= N ? N - 1 : j);
#pragma unroll
        for (int d = 0; d < DC; ++d) cw[u][d] = (double)a.dia1[(size_t)d * N + jc[u]];
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (!((act >> g) & 1u)) continue;
        const V* p = a.p + (g0 + g) * a.vs;
        double vw[OU][DC];
#pragma unroll
        for (int u = 0; u < OU; ++u)
#pragma unroll
          for (int d = 0; d < DC; ++d) vw[u][d] = (double)p[jc[u] + a.op.offs1[d]];
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          const int e = e0 + u * IPB;
          const int64_t j = i0 - Ho + e;
          const double tv = (j < 0 || j >= N) ? 0.0 : (double)(V)stencil_combine<M, DC>(cw[u], vw[u], a.op.d01);
          if (e < L) ts[g * L + e] = tv;
        }
      }
    }
  }
  __syncthreads();
  if (live) {
    for (int e0 = threadIdx.x; e0 < R; e0 += OU * IPB) {
      double cw[OU][DC];
      int64_t ic[OU];
      int ec[OU];
      bool ok[OU];
#pragma unroll
      for (int u = 0; u < OU; ++u) {
        const int e = e0 + u * IPB;
        const int64_t i = i0 + (e < R ? e : R - 1);
        ic[u] = i < N ? i : N - 1;      // i0 <= ic < min(i0 + R, N)
        ec[u] = (int)(ic[u] - i0) + Ho;
        ok[u] = (e < R) & (i < N);
#pragma unroll
        for (int d = 0; d < DC; ++d) cw[u][d] = (double)a.dia[(size_t)d * N + ic[u]];
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (!((act >> g) & 1u)) continue;
        const int m = g0 + g;
        const V* p = a.p + m * a.vs;
        const uint8_t* mk = a.mask + (size_t)m * N;
        V* w = a.w + m * a.vs;
        uint8_t mv[OU];
        double pv[OU], wv[OU];
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          mv[u] = mk[ic[u]];
          pv[u] = (double)p[ic[u]];
        }
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          double vw[DC];
#pragma unroll
          for (int d = 0; d < DC; ++d) vw[d] = ts[g * L + ec[u] + a.op.offs[d]];
          wv[u] = sa[g] * stencil_combine<M, DC>(cw[u], vw, a.op.d0) + sc[g] * pv[u];
        }
#pragma unroll
        for (int u = 0; u < OU; ++u) {
          if (!(ok[u] && mv[u] == 0)) continue;
          w[i0 + e0 + u * IPB] = (V)wv[u];
          v[g] += pv[u] * (double)(V)wv[u];
        }
      }
    }
  }
  block_sum<G, NIWAVE>(v, red, bvv);
  const unsigned fin = tree_reduce_multi(a.gof, tile, 1, act, G, a.part + (size_t)g0 * a.gof.ptotal,
                                         (size_t)a.gof.ptotal, a.ctr + (size_t)g0 * a.gof.ctotal,
                                         (size_t)a.gof.ctotal, bvv, tot);
  if (threadIdx.x < G && ((fin >> threadIdx.x) & 1u)) {
    Inst* S = a.inst + g0 + threadIdx.x;
    const double pw = tot[threadIdx.x];
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

// x64 += d (correction of the sweep that has just ended; instances still in
// their sweep are skipped)
template <typename V, int RPT>
__global__ void __launch_bounds__(IPB) k_accumulate(OpGeom op, const uint8_t* mask, const V* d,
                                                    double* x64, int64_t vs, Inst* inst) {
  int tile, m;
  tile_inst(op.ntiles_pad, tile, m);
  Inst* S = inst + m;
  if (S->outer_done || !S->done) return;
  if (tile >= op.ntiles) return;
  const int64_t N = op.N;
  const uint8_t* mk = mask + (size_t)m * N;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * IPB + threadIdx.x;
    if (i < N && mk[i] == 0) x64[m * vs + i] += (double)d[m * vs + i];
  }
  if (tile == 0 && threadIdx.x == 0) S->sweeps += 1;
}

// end of a chunk's sweep transitions: no instance has a pending init2
__global__ void k_trans_clear(Inst* inst, int B) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < B) inst[m].trans = 0;
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
                          const double* sv, double* y, const Inst* inst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = op.N;
  if (i >= N) return;
  double v = 0.0;
  if (mask[i] == 0) {
    double acc = 0.0;
    for (int d = 0; d < op.D; ++d) acc += dia[(size_t)d * N + i] * sv[i + op.offs[d]];
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
