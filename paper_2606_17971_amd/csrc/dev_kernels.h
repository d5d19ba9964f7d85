// Streaming kernels of the restricted A-DEF2 solve (gfx950, wave64).
//
// Data layout (all in HBM, global node order, lexicographic, x fastest):
//   S     : diagonal format, dia[d * N + i] = S[i, i + offs[d]] (0 if absent),
//           or, for S = alpha A^T A + c I, the two stencils A (dia1, offs1) and
//           A^T (dia, offs): S_II v = alpha (A^T (A v))_I + c v for v zero on
//           the active set, applied as t = A v on all rows, then A^T t
//   Z     : column-major N x KP (shared by all instances, zero padded columns)
//   W     : per instance, column-major N x KP, W = S_II Z_I
//   x,r,z,p,w : per instance, length N + 2H with H zero halo entries on both
//           sides, so the stencil reads i + offs[d] need no bounds test;
//           entries on the active set are kept at exactly 0, which makes
//           S (masked vector) restricted to inactive rows equal to S_II.
// Tile kernels map blocks to (tile, instance) with tile_inst().
#pragma once
#include "../../include/adef2.h"
#include "dev_common.h"

namespace adef2 {

constexpr int MAXD = ADEF2_MAX_DIAGS;   // diagonals of S, or of A^T (factored)
constexpr int MAXD1 = 16;               // diagonals of A (factored)

struct OpGeom {
  int64_t N;
  int D;             // outer stencil: S (assembled) or A^T (factored)
  int D1;            // inner stencil A (factored), 0 when assembled
  int ntiles;        // tiles covering N rows
  int ntiles_pad;    // multiple of 8 (XCD mapping)
  int offs[MAXD];
  int offs1[MAXD1];
  int d0;            // slot of offset 0 in the outer stencil (-1: none)
  int d01;           // slot of offset 0 in the inner stencil (-1: none)
};

// One row of a diagonal-format stencil, sum_d a_d[i] v[i + o_d].  FP32
// coefficient arrays store, in the offset-0 slot, the row sum of the FP64
// row instead of its diagonal entry, and are applied in difference form
//   rowsum_i v_i + sum_{d != 0} a_d[i] (v[i + o_d] - v_i)
// (the same value in exact arithmetic).  Rounding a coefficient to FP32 then
// perturbs only a flux a_d (v_j - v_i), which is small on smooth v; in the
// direct form the rounded coefficients no longer cancel (zero row sums of the
// interior rows of a conservative stencil) and add an O(u32) zeroth-order
// term that swamps the smallest eigenvalues of A^T A.
template <typename M, typename VI>
__device__ __forceinline__ double stencil_row(const M* dia, const int* offs, int D, int d0,
                                              int64_t N, int64_t i, const VI* v) {
  double acc = 0.0;
  if constexpr (sizeof(M) == 4) {
    if (d0 >= 0) {
      const double vi = (double)v[i];
      acc = (double)dia[(size_t)d0 * N + i] * vi;
      for (int d = 0; d < D; ++d)
        if (d != d0) acc += (double)dia[(size_t)d * N + i] * ((double)v[i + offs[d]] - vi);
      return acc;
    }
  }
  for (int d = 0; d < D; ++d) acc += (double)dia[(size_t)d * N + i] * (double)v[i + offs[d]];
  return acc;
}

// V: type of the per-instance vectors; M: type of the operator values and of
// the Z / W panels (FP32 in the mixed-precision modes).
template <typename V, typename M>
struct IterArgs {
  OpGeom op;
  const M* dia;            // [D][N] outer stencil
  const M* dia1;           // [D1][N] inner stencil (factored operator)
  V* t;                    // padded inner product A p (factored operator)
  const uint8_t* mask;     // [B][N]
  const V* dinv;           // [B][N]
  const M* Z;              // [KP][N] shared, or [B][KP][N] per instance
  int64_t zs;              // instance stride of Z (0: shared by all instances)
  // with a per-instance basis whose first kb columns are the shared modes,
  // those columns are read from the shared copy (one stream through L2 for
  // the whole batch instead of one per instance)
  const M* Zsh;            // [kb][N] shared leading columns
  const double* Zsh64;
  int32_t kb;              // columns q < kb come from Zsh (KP when zs == 0)
  // boundary form of W for reference modes that are eigenvectors of the base
  // operator B (S = a B + c I): column q < ne with eig[q] stores W - lambda Z,
  // lambda = a mu[q] + c, which vanishes (to the eigen-residual) except on
  // rows flagged in bnd; then W^T z = lambda Z^T z + sum over those rows
  const double* mu;        // [KP] Rayleigh quotients of the reference modes for B
  const uint8_t* eig;      // [KP]
  const uint8_t* bnd;      // [B][N]
  int32_t ne;              // 0: W stored whole
  const M* wzero;          // a zero in device memory: the W load of a row that
                           // needs no W reads it (one cached line, no branch)
  const M* W;              // [B][KP][N]
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
  const double* x0sv;      // stencil source for S x0: x0, or A x0 (factored)
  int64_t x0s;
  double thresh_scale;     // thresh2 = max(thresh_scale [* tol2] * ||src_I||^2,
  double thresh_floor;     //               thresh_floor * tol2 * ||b_I||^2), tol2 per instance
  int32_t thresh_rel_tol;  // multiply thresh_scale by the instance's tol2
  int32_t carry_dir;       // keep the previous sweep's search direction
  int32_t trans_mode;      // init / init2 of a sweep transition: only instances whose
                           // sweep ended (init) or that init set up (init2)
  int32_t seg_maxit;       // a sweep ends after this many iterations (0 = none)
  // W-free projection: FP64 operator and modes (see k_zproj)
  const double* dia64;     // [D][N]
  const double* dia1_64;   // [D1][N]
  const double* Z64;       // [KP][N] shared, or [B][KP][N] per instance
  // tile-major kernels (k_pupdate_bt, k_zproj_bt): BT_ROWS-row tiles
  int32_t B;               // instances
  int32_t bt_ntiles, bt_ntiles_pad;
  int32_t bt_nblk_pad;     // k_zproj_bt blocks (BT_TPB tiles each), multiple of 8
  RedGeom gbt;             // reduction tree over the k_zproj_bt blocks
  // tile-major kernels of the shared reference modes (k_pupdate_tm,
  // k_update_tm): UB_ROWS-row tiles, instance groups of UB_G / PB_G
  int32_t ub_ntiles, ub_ntiles_pad;
  int32_t ub_ngroups, pb_ngroups, sg_ngroups;
  RedGeom gub;             // reduction tree over the tiles (one leaf per tile)
  const M* ZT;             // [N][KP] row-major copy of the shared modes
  const double* diag;      // [N] diagonal of the reference stencil (Jacobi: 1 / (a d + c))
  int32_t precond_none;
  // boundary rows of each instance (rows of W - lambda Z that are not zero),
  // compacted tile by tile: entries btoff[m][t] .. btoff[m][t + 1] - 1 of
  // instance m lie in tile t, entry e is row bidx[e] with values bW[e][0..KP)
  const int32_t* btoff;    // [B][ub_ntiles + 1]
  const int32_t* bidx;
  const M* bW;
  double* ftot;            // [B][slices][2 KP + 2] slice totals of the tile-major finisher
  unsigned* fctr;          // [B] arrival counters of the tile-major finisher
  int32_t fin_leaves;      // partial sums per instance that the finisher adds (tiles,
                           // or runs of ws_T tiles for the warp-specialised update)
  int32_t ws_T, ws_cpx;    // warp-specialised update: tiles per block, runs per XCD
  // fused operator pass of the factored form (k_opfused): of_rows-row tiles,
  // inner product A p staged in LDS over of_halo extra rows on each side
  int32_t of_rows, of_halo;
  int32_t of_ntiles, of_ntiles_pad;
  int32_t of_ngroups;      // instance groups of the grouped pass (k_opfused_g)
  RedGeom gof;             // reduction tree over the fused tiles
};

template <int RPT> struct Rows { static constexpr int PB = IPB * RPT; };

// column q of instance m's basis (FP32/FP64 panel type M, or FP64)
template <typename V, typename M>
__device__ __forceinline__ const M* zcol(const IterArgs<V, M>& a, int m, int q) {
  return q < a.kb ? a.Zsh + (size_t)q * a.op.N : a.Z + (size_t)m * a.zs + (size_t)q * a.op.N;
}
template <typename V, typename M>
__device__ __forceinline__ const double* zcol64(const IterArgs<V, M>& a, int m, int q) {
  return q < a.kb ? a.Zsh64 + (size_t)q * a.op.N : a.Z64 + (size_t)m * a.zs + (size_t)q * a.op.N;
}

// Row tile of one iteration block: IPB * RPT consecutive rows starting at
// base; thread t owns rows base + t + j * IPB.

// Panel products of a whole block: for the NQ columns q = 0..NQ-1 (column q
// of the panel at col(q), multiplied with the LDS vector vec(q)), wave w
// sums the columns w, w + NIWAVE, ... over the tile rows and lane 0 stores
// the totals in out[q].  Rows and columns are fully unrolled so that each
// lane has all of its column loads in flight at once (with a handful of
// outstanding loads per lane these reductions are latency bound far below
// HBM bandwidth).  The LDS vectors are zero on rows that do not take part,
// so only rows past N need a guard (last tile).
template <typename M, int RPT, int NQ, typename ColF, typename VecF>
__device__ __forceinline__ void panel_dots(int64_t base, int64_t N, ColF col, VecF vec, double* out) {
  constexpr int R = Rows<RPT>::PB;
  constexpr int NQW = (NQ + NIWAVE - 1) / NIWAVE;   // columns per wave
  constexpr int PG = 4;                              // columns per group (loads in flight)
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool full = base + R <= N;
#pragma unroll 1
  for (int s0 = 0; s0 < NQW; s0 += PG) {
    double acc[PG];
#pragma unroll
    for (int g = 0; g < PG; ++g) acc[g] = 0.0;
    if (full) {
#pragma unroll
      for (int g = 0; g < PG; ++g) {
        const int q = wid + (s0 + g) * NIWAVE;
        if (s0 + g < NQW && q < NQ) {
          const M* c = col(q);
          const double* v = vec(q);
#pragma unroll
          for (int j = lane; j < R; j += 64) acc[g] += (double)c[base + j] * v[j];
        }
      }
    } else {
#pragma unroll
      for (int g = 0; g < PG; ++g) {
        const int q = wid + (s0 + g) * NIWAVE;
        if (s0 + g < NQW && q < NQ) {
          const M* c = col(q);
          const double* v = vec(q);
          for (int j = lane; j < R && base + j < N; j += 64) acc[g] += (double)c[base + j] * v[j];
        }
      }
    }
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      const int q = wid + (s0 + g) * NIWAVE;
      if (s0 + g < NQW && q < NQ) {
        const double t = wave_sum(acc[g]);
        if (lane == 0) out[q] = t;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// init: r0 = src - S x0 (or src), g = Z^T r0, ||src||^2;  finisher: c0 = C g
// ---------------------------------------------------------------------------
template <typename V, typename M, int KP, int RPT>
__global__ void __launch_bounds__(IPB) k_init(IterArgs<V, M> a) {
  constexpr int R = Rows<RPT>::PB;
  constexpr int NV = KP + 1;
  __shared__ double vl[R];
  __shared__ uint8_t act[R];
  __shared__ double red[NIWAVE];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->outer_done || (a.trans_mode && !S->done)) return;
  const int64_t N = a.op.N;
  const int64_t base = (int64_t)tile * R;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const double* src = a.src + (size_t)m * N;
  V* x = a.x + m * a.vs;
  V* r = a.r + m * a.vs;
  const double sa = S->a, sc = S->c;
  double bb = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int j = rr * IPB + threadIdx.x;
    const int64_t i = base + j;
    const bool on = (tile < a.op.ntiles) && i < N && mk[i] == 0;
    double r0 = 0.0;
    if (on) {
      const double s = src[i];
      double xv = 0.0;
      r0 = s;
      if (a.x0) {
        const double* x0 = a.x0 + m * a.x0s;
        const double* sv = a.x0sv + m * a.x0s;
        double acc = 0.0;
        for (int d = 0; d < a.op.D; ++d) acc += (double)a.dia[(size_t)d * N + i] * sv[i + a.op.offs[d]];
        xv = x0[i];
        r0 = s - (sa * acc + sc * xv);
      }
      x[i] = (V)xv;
      r[i] = (V)r0;
      bb += s * s;
    }
    vl[j] = r0;
    act[j] = !on;
  }
  {
    double v1[1] = {bb};
    block_sum<1, NIWAVE>(v1, red, bv + KP);
  }
  {
    __shared__ const M* colp[KP > 0 ? KP : 1];
    for (int q = threadIdx.x; q < KP; q += blockDim.x) colp[q] = zcol(a, m, q);
    __syncthreads();
    panel_dots<M, RPT, KP>(base, N, [&](int q) { return colp[q]; },
                           [&](int) { return (const double*)vl; }, bv);
  }
  __syncthreads();
  double* part = a.part + (size_t)m * a.g.ptotal * NV;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, NV, part, ctr, bv, tot)) return;
  if (threadIdx.x == 0) {
    const double b2 = tot[KP];
    S->bb = b2;
    S->thresh2 = fmax(a.thresh_scale * (a.thresh_rel_tol ? S->tol2 : 1.0) * b2,
                      a.thresh_floor * S->tol2 * S->bb64);
    S->done = 0;
    S->sweep_iters = 0;
    S->fresh = 1;
    if (a.trans_mode) S->trans = 1;
    if (!(b2 < INFINITY)) { S->done = 1; S->outer_done = 1; S->status = -1; }
    else if (b2 == 0.0) { S->done = 1; }
  }
  const double* Cm = a.C + (size_t)m * KP * KP;
  for (int q = threadIdx.x; q < KP; q += blockDim.x) {
    double s = 0.0;
    if (S->kk > 0)
      for (int l = 0; l < KP; ++l) s += Cm[q * KP + l] * tot[l];
    S->coef[q] = s;
  }
}

// ---------------------------------------------------------------------------
// A-DEF2 preconditioned residual y = P K r + Q r  (P = I - Z E^-1 W^T,
// Q = Z E^-1 Z^T): its coarse coordinates are c = E^-1 (W^T z - Z^T r) and
// y = z - Z c.  The finisher of a reduction holding
//   tot = [W^T z (KP) | Z^T r (KP) | r.z | r.r]
// forms c (stored in S->coef) and returns r.y = r.z - (Z^T r).c.
// ---------------------------------------------------------------------------
template <int KP>
__device__ __forceinline__ double adef2_direction(const double* Cm, const double* tot, Inst* S,
                                                  bool defl) {
  constexpr int K1 = KP > 0 ? KP : 1;
  __shared__ double gl[K1], cl[K1];
  __shared__ double s_rho;
  if (defl) {
    for (int q = threadIdx.x; q < KP; q += blockDim.x) gl[q] = tot[q] - tot[KP + q];
    __syncthreads();
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
      double s = 0.0;
#pragma unroll 4
      for (int l = 0; l < KP; ++l) s += Cm[q * KP + l] * gl[l];
      cl[q] = s;
      S->coef[q] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double corr = 0.0;
    if (defl)
#pragma unroll 4
      for (int q = 0; q < KP; ++q) corr += tot[KP + q] * cl[q];
    s_rho = tot[2 * KP] - corr;
  }
  __syncthreads();
  return s_rho;
}

// [W^T z | Z^T r] with the boundary form of W.  The tile's boundary rows are
// compacted into an LDS list (wave ballots and prefix counts, so the order is
// fixed); an eigen column then takes one dense pass over Z (serving Z^T z
// and Z^T r) and a short pass over the listed rows of its stored panel
// W - lambda Z; a non-eigen column (learned vectors) reads its W whole.
template <typename V, typename M, int KP, int RPT>
__device__ __forceinline__ void spectral_dots(const IterArgs<V, M>& a, int m, int64_t base, const M* W,
                                              const double* zl, const double* rl, double* out) {
  constexpr int R = Rows<RPT>::PB;
  constexpr int NQW = (KP + NIWAVE - 1) / NIWAVE;
  constexpr int NCH = R / 64;                       // 64-row chunks of the tile
  __shared__ int blist[R];
  __shared__ int bcnt[NCH + 1];
  const int64_t N = a.op.N;
  const uint8_t* bm = a.bnd + (size_t)m * N;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // chunk c = rows 64 c .. 64 c + 63, handled by wave c % NIWAVE
  for (int c = wid; c < NCH; c += NIWAVE) {
    const int64_t i = base + 64 * c + lane;
    const bool f = i < N && bm[i] != 0;
    const unsigned long long bal = __ballot(f);
    if (lane == 0) bcnt[c + 1] = __popcll(bal);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bcnt[0] = 0;
    for (int c = 0; c < NCH; ++c) bcnt[c + 1] += bcnt[c];
  }
  __syncthreads();
  for (int c = wid; c < NCH; c += NIWAVE) {
    const int64_t i = base + 64 * c + lane;
    const bool f = i < N && bm[i] != 0;
    const unsigned long long bal = __ballot(f);
    if (f) blist[bcnt[c] + __popcll(bal & ((1ull << lane) - 1ull))] = 64 * c + lane;
  }
  __syncthreads();
  const int nb = bcnt[NCH];
  const Inst* S = a.inst + m;
  const bool full = base + R <= N;
#pragma unroll
  for (int s = 0; s < NQW; ++s) {
    const int q = wid + s * NIWAVE;
    if (q < KP) {
      const M* zc = zcol(a, m, q) + base;
      const M* wc = W + (size_t)q * N + base;
      const bool e = q < a.ne && a.eig[q];
      double aw = 0.0, az = 0.0, ar = 0.0;
      if (e) {
        if (full) {
#pragma unroll
          for (int j = lane; j < R; j += 64) {
            const double zv = (double)zc[j];
            az += zv * zl[j];
            ar += zv * rl[j];
          }
        } else {
          for (int j = lane; j < R && base + j < N; j += 64) {
            const double zv = (double)zc[j];
            az += zv * zl[j];
            ar += zv * rl[j];
          }
        }
        for (int t = lane; t < nb; t += 64) {
          const int j = blist[t];
          aw += (double)wc[j] * zl[j];
        }
      } else {
        if (full) {
#pragma unroll
          for (int j = lane; j < R; j += 64) {
            aw += (double)wc[j] * zl[j];
            ar += (double)zc[j] * rl[j];
          }
        } else {
          for (int j = lane; j < R && base + j < N; j += 64) {
            aw += (double)wc[j] * zl[j];
            ar += (double)zc[j] * rl[j];
          }
        }
      }
      aw = wave_sum(aw);
      az = wave_sum(az);
      ar = wave_sum(ar);
      if (lane == 0) {
        const double lam = e ? S->a * a.mu[q] + S->c : 0.0;
        out[q] = aw + lam * az;
        out[KP + q] = ar;
      }
    }
  }
}

// Second half of init2 / update: block sums of [W^T z | Z^T r | r.z | r.r]
// for the tile (z, r already in LDS), then the reduction tree.
template <typename V, typename M, int KP, int RPT, bool SPEC = false>
__device__ __forceinline__ bool reduce_directions(const IterArgs<V, M>& a, int m, int tile, int64_t base,
                                                  const M* W, bool defl, double rz, double rr2,
                                                  const double* zl, const double* rl,
                                                  const uint8_t* act, double* red, double* bv,
                                                  double* tot) {
  constexpr int NV = 2 * KP + 2;
  {
    double v2[2] = {rz, rr2};
    block_sum<2, NIWAVE>(v2, red, bv + 2 * KP);
  }
  const int64_t N = a.op.N;
  if constexpr (SPEC) {
    if (defl) spectral_dots<V, M, KP, RPT>(a, m, base, W, zl, rl, bv);
    else
      for (int q = threadIdx.x; q < 2 * KP; q += blockDim.x) bv[q] = 0.0;
  } else if (defl) {
    // column base pointers computed once per block (the shared/per-instance
    // choice of zcol inside the unrolled loop costs ~2x the registers)
    __shared__ const M* colp[KP > 0 ? 2 * KP : 1];
    for (int q = threadIdx.x; q < 2 * KP; q += blockDim.x)
      colp[q] = q < KP ? W + (size_t)q * N : zcol(a, m, q - KP);
    __syncthreads();
    panel_dots<M, RPT, 2 * KP>(
        base, N, [&](int q) { return colp[q]; }, [&](int q) { return q < KP ? zl : rl; }, bv);
  } else {
    for (int q = threadIdx.x; q < 2 * KP; q += blockDim.x) bv[q] = 0.0;
  }
  __syncthreads();
  double* part = a.part + (size_t)m * a.g.ptotal * NV;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  return tree_reduce(a.g, tile, NV, part, ctr, bv, tot);
}

// ---------------------------------------------------------------------------
// init2: x += Z c0, r -= W c0, z = K r;  W^T z, Z^T r, r.z, ||r||^2
// ---------------------------------------------------------------------------
template <typename V, typename M, int KP, int RPT>
__global__ void __launch_bounds__(IPB) k_init2(IterArgs<V, M> a) {
  constexpr int R = Rows<RPT>::PB;
  constexpr int NV = 2 * KP + 2;
  __shared__ double zl[R], rl[R];
  __shared__ uint8_t act[R];
  __shared__ double red[NIWAVE * 2];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  __shared__ double cf[KP > 0 ? KP : 1];
  __shared__ double lamq[KP > 0 ? KP : 1];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->outer_done || (a.trans_mode && !S->trans)) return;
  const int64_t N = a.op.N;
  const int64_t base = (int64_t)tile * R;
  const uint8_t* mk = a.mask + (size_t)m * N;
  V* x = a.x + m * a.vs;
  if (S->done) {   // zero right-hand side: x = 0 is the solution
    if (S->bb == 0.0 && tile < a.op.ntiles) {
      for (int rr = 0; rr < RPT; ++rr) {
        const int64_t i = base + rr * IPB + threadIdx.x;
        if (i < N) x[i] = (V)0;
      }
    }
    return;
  }
  V* r = a.r + m * a.vs;
  V* z = a.z + m * a.vs;
  const V* dinv = a.dinv + (size_t)m * N;
  const M* W = a.W + (size_t)m * KP * N;
  const bool defl = S->kk > 0;
  for (int q = threadIdx.x; q < KP; q += blockDim.x) {
    cf[q] = S->coef[q];
    lamq[q] = (q < a.ne && a.eig[q]) ? S->a * a.mu[q] + S->c : 0.0;
  }
  __syncthreads();
  double rz = 0.0, rr2 = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int j = rr * IPB + threadIdx.x;
    const int64_t i = base + j;
    const bool on = (tile < a.op.ntiles) && i < N && mk[i] == 0;
    double rv = 0.0, zv = 0.0;
    if (on) {
      double xv = (double)x[i];
      rv = (double)r[i];
      if (defl) {
#pragma unroll
        for (int q = 0; q < KP; ++q) {
          const double zq = (double)zcol(a, m, q)[i];
          xv += zq * cf[q];
          rv -= ((double)W[(size_t)q * N + i] + lamq[q] * zq) * cf[q];
        }
      }
      const V rq = (V)rv;
      const V zq = (V)((double)dinv[i] * (double)rq);
      x[i] = (V)xv;
      r[i] = rq;
      z[i] = zq;
      rv = (double)rq;
      zv = (double)zq;
      rz += rv * zv;
      rr2 += rv * rv;
    }
    zl[j] = zv;
    rl[j] = rv;
    act[j] = !on;
  }
  __syncthreads();
  if (!reduce_directions<V, M, KP, RPT>(a, m, tile, base, W, defl, rz, rr2, zl, rl, act, red, bv, tot))
    return;
  const bool stop = !(tot[2 * KP + 1] > S->thresh2);
  double rho = 0.0;
  if (!stop) rho = adef2_direction<KP>(a.C + (size_t)m * KP * KP, tot, S, defl);
  if (threadIdx.x == 0) {
    S->rr = tot[2 * KP + 1];
    // residual replacement: continue the previous direction, p = y + beta p,
    // unless the last sweep drifted from the FP64 residual
    const bool carry = a.carry_dir && S->has_dir && S->rho_end > 0.0 && rho > 0.0 && !S->drift;
    S->beta = carry ? rho / S->rho_end : 0.0;
    S->fresh = carry ? 0 : 1;
    S->rho = rho;
    if (stop) S->done = 1;
  }
}

// ---------------------------------------------------------------------------
// p = z - Z c + beta p   (A-DEF2 search direction)
// ---------------------------------------------------------------------------
template <typename V, typename M, int KP, int RPT>
__global__ void __launch_bounds__(IPB) k_pupdate(IterArgs<V, M> a) {
  __shared__ double cf[KP > 0 ? KP : 1];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  const Inst* S = a.inst + m;
  if (S->done) return;
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
    const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * IPB + threadIdx.x;
    if (i < N && mk[i] == 0) {
      double pv = (double)z[i];
      if (defl) {
#pragma unroll
        for (int q = 0; q < KP; ++q) pv -= (double)zcol(a, m, q)[i] * cf[q];
      }
      if (keep) pv += beta * (double)p[i];
      p[i] = (V)pv;
    }
  }
}

// ---------------------------------------------------------------------------
// w = S_II p, p.w;  finisher: alpha = rho / p.w
// ---------------------------------------------------------------------------
template <typename V, typename M, int KP, int RPT>
__global__ void __launch_bounds__(IPB) k_spmv(IterArgs<V, M> a) {
  __shared__ double red[NIWAVE];
  __shared__ double bv[1];
  __shared__ double tot[1];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->done) return;
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const V* p = a.p + m * a.vs;
  const V* sv = (a.op.D1 ? a.t : a.p) + m * a.vs;
  V* w = a.w + m * a.vs;
  const double sa = S->a, sc = S->c;
  double v[1] = {0.0};
  if (tile < a.op.ntiles) {
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * IPB + threadIdx.x;
      if (i < N && mk[i] == 0) {
        const double acc = stencil_row(a.dia, a.op.offs, a.op.D, a.op.d0, N, i, sv);
        const double pi = (double)p[i];
        const double wv = sa * acc + sc * pi;
        w[i] = (V)wv;
        v[0] += pi * (double)(V)wv;
      }
    }
  }
  block_sum<1, NIWAVE>(v, red, bv);
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

// Finisher of an iteration's last reduction, tot = [W^T z | Z^T r | r.z | r.r]:
// iteration count, stopping tests (tolerance, segment cap, maxit), then the
// next coarse coordinates and beta.
template <int KP>
__device__ __forceinline__ void update_finish(const double* Cm, const double* tot, Inst* S, bool defl,
                                              int32_t maxit, int32_t seg_maxit) {
  __shared__ int s_go;
  if (threadIdx.x == 0) {
    const double rrt = tot[2 * KP + 1];
    S->iters += 1;
    S->sweep_iters += 1;
    S->rr = rrt;
    int go = 0;
    if (!(rrt > S->thresh2) || (seg_maxit > 0 && S->sweep_iters >= seg_maxit)) {
      S->done = 1;
      S->capped = (rrt > S->thresh2);
      go = 2;                       // sweep ends: keep r.y for the next sweep
      if (!(rrt < INFINITY)) { S->outer_done = 1; S->status = -5; go = 0; }
    } else if (S->iters >= maxit) {
      S->done = 1;
      S->outer_done = 1;
      S->status = 2;
    } else {
      go = 1;
    }
    s_go = go;
  }
  __syncthreads();
  if (!s_go) return;
  const double rho = adef2_direction<KP>(Cm, tot, S, defl);
  if (threadIdx.x == 0) {
    if (s_go == 1) {
      S->beta = rho / S->rho;
      S->rho = rho;
      S->fresh = 0;
    } else {
      S->rho_end = rho;
      S->has_dir = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// x += alpha p, r -= alpha w, z = K r;  W^T z, Z^T r, r.z, ||r||^2
// finisher: stopping test on ||r||, beta = r.y / rho, coarse coordinates
// ---------------------------------------------------------------------------
// SPEC: W in the boundary form (a.ne > 0), a separate instantiation so that
// the default kernel carries neither its code nor its LDS
template <typename V, typename M, int KP, int RPT, bool SPEC = false>
__global__ void __launch_bounds__(IPB) k_update(IterArgs<V, M> a) {
  constexpr int R = Rows<RPT>::PB;
  constexpr int NV = 2 * KP + 2;
  __shared__ double zl[R], rl[R];
  __shared__ uint8_t act[R];
  __shared__ double red[NIWAVE * 2];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->done) return;
  const int64_t N = a.op.N;
  const int64_t base = (int64_t)tile * R;
  const uint8_t* mk = a.mask + (size_t)m * N;
  V* x = a.x + m * a.vs;
  V* r = a.r + m * a.vs;
  V* z = a.z + m * a.vs;
  const V* p = a.p + m * a.vs;
  const V* w = a.w + m * a.vs;
  const V* dinv = a.dinv + (size_t)m * N;
  const M* W = a.W + (size_t)m * KP * N;
  const bool defl = S->kk > 0;
  const double alpha = S->alpha;
  double rz = 0.0, rr2 = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int j = rr * IPB + threadIdx.x;
    const int64_t i = base + j;
    const bool on = (tile < a.op.ntiles) && i < N && mk[i] == 0;
    double rv = 0.0, zv = 0.0;
    if (on) {
      const double xv = (double)x[i] + alpha * (double)p[i];
      const V rq = (V)((double)r[i] - alpha * (double)w[i]);
      const V zq = (V)((double)dinv[i] * (double)rq);
      x[i] = (V)xv;
      r[i] = rq;
      z[i] = zq;
      rv = (double)rq;
      zv = (double)zq;
      rz += rv * zv;
      rr2 += rv * rv;
    }
    zl[j] = zv;
    rl[j] = rv;
    act[j] = !on;
  }
  __syncthreads();
  if (!reduce_directions<V, M, KP, RPT, SPEC>(a, m, tile, base, W, defl, rz, rr2, zl, rl, act, red, bv, tot))
    return;
  update_finish<KP>(a.C + (size_t)m * KP * KP, tot, S, defl, a.maxit, a.seg_maxit);
}

// ---------------------------------------------------------------------------
// W-free variant of the update: W^T z = Z^T (S_II z), so the per-instance
// panel W is not read in the iteration.  k_update_nw streams x, r, z;
// k_zproj then forms u = S_II z row by row (from t = A z for the factored
// operator) and reduces [Z^T u | Z^T r | r.z | r.r] with one pass over Z.
// The preconditioned residual z is rough, so S z is of the size of
// ||S|| ||z|| while Z^T S z is of the size of the small eigenvalues times
// ||z||: rounding S, Z or z to FP32 would leave an error of u32 cond(S)
// relative to it.  This variant therefore needs FP64 vectors and always
// reads the FP64 operator and FP64 modes (shared by all instances of a batch,
// so their traffic is paid once per launch, not per instance).
// ---------------------------------------------------------------------------
template <typename V, typename M, int KP, int RPT>
__global__ void __launch_bounds__(IPB) k_update_nw(IterArgs<V, M> a) {
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  const Inst* S = a.inst + m;
  if (S->done) return;
  if (tile >= a.op.ntiles) return;
  const int64_t N = a.op.N;
  const uint8_t* mk = a.mask + (size_t)m * N;
  V* x = a.x + m * a.vs;
  V* r = a.r + m * a.vs;
  V* z = a.z + m * a.vs;
  const V* p = a.p + m * a.vs;
  const V* w = a.w + m * a.vs;
  const V* dinv = a.dinv + (size_t)m * N;
  const double alpha = S->alpha;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int64_t i = (int64_t)tile * Rows<RPT>::PB + rr * IPB + threadIdx.x;
    if (i < N && mk[i] == 0) {
      x[i] = (V)((double)x[i] + alpha * (double)p[i]);
      const V rq = (V)((double)r[i] - alpha * (double)w[i]);
      r[i] = rq;
      z[i] = (V)((double)dinv[i] * (double)rq);
    }
  }
}

template <typename V, typename M, int KP, int RPT>
__global__ void __launch_bounds__(IPB) k_zproj(IterArgs<V, M> a) {
  constexpr int R = Rows<RPT>::PB;
  constexpr int NV = 2 * KP + 2;
  __shared__ double ul[R], rl[R];
  __shared__ uint8_t act[R];
  __shared__ double red[NIWAVE * 2];
  __shared__ double bv[NV];
  __shared__ double tot[NV];
  int tile, m;
  tile_inst(a.op.ntiles_pad, tile, m);
  Inst* S = a.inst + m;
  if (S->done) return;
  const int64_t N = a.op.N;
  const int64_t base = (int64_t)tile * R;
  const uint8_t* mk = a.mask + (size_t)m * N;
  const V* r = a.r + m * a.vs;
  const V* z = a.z + m * a.vs;
  static_assert(sizeof(V) == 8, "the W-free projection needs FP64 vectors");
  const V* sv = (a.op.D1 ? a.t : a.z) + m * a.vs;
  const bool defl = S->kk > 0;
  const double sa = S->a, sc = S->c;
  double rz = 0.0, rr2 = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int j = rr * IPB + threadIdx.x;
    const int64_t i = base + j;
    const bool on = (tile < a.op.ntiles) && i < N && mk[i] == 0;
    double rv = 0.0, uv = 0.0;
    if (on) {
      const double zv = (double)z[i];
      rv = (double)r[i];
      rz += rv * zv;
      rr2 += rv * rv;
      if (defl) uv = sa * stencil_row(a.dia64, a.op.offs, a.op.D, a.op.d0, N, i, sv) + sc * zv;
    }
    ul[j] = uv;
    rl[j] = rv;
    act[j] = !on;
  }
  __syncthreads();
  {
    double v2[2] = {rz, rr2};
    block_sum<2, NIWAVE>(v2, red, bv + 2 * KP);
  }
  if (defl) {
    __shared__ const double* colp[KP > 0 ? KP : 1];
    for (int q = threadIdx.x; q < KP; q += blockDim.x) colp[q] = zcol64(a, m, q);
    __syncthreads();
    panel_dots<double, RPT, 2 * KP>(
        base, N, [&](int q) { return colp[q < KP ? q : q - KP]; },
        [&](int q) { return q < KP ? (const double*)ul : (const double*)rl; }, bv);
  } else {
    for (int q = threadIdx.x; q < 2 * KP; q += blockDim.x) bv[q] = 0.0;
  }
  __syncthreads();
  double* part = a.part + (size_t)m * a.g.ptotal * NV;
  unsigned* ctr = a.ctr + (size_t)m * a.g.ctotal;
  if (!tree_reduce(a.g, tile, NV, part, ctr, bv, tot)) return;
  update_finish<KP>(a.C + (size_t)m * KP * KP, tot, S, defl, a.maxit, a.seg_maxit);
}

// ---------------------------------------------------------------------------
// Tile-major kernels for a basis shared by all instances.  One block owns a
// tile of BT_ROWS rows for every instance of the batch, so each row of Z is
// read once per launch instead of once per instance (with B instances the
// per-instance kernels pull the Z tile B times through L2, which bounds them
// well below HBM bandwidth).
//   k_pupdate_bt: p_m = z_m - Z c_m + beta_m p_m; the thread keeps its row of
//     Z in registers and loops over the instances.
//   k_zproj_bt: the panel products of the W-free update for all instances
//     as one FP64 matrix product per tile, [Z^T u_m, Z^T r_m]_m = Z^T V with
//     V = [u_1 r_1 ... u_G r_G] (BT_ROWS x 2G, staged in LDS), on the matrix
//     cores (v_mfma_f64_16x16x4): lane l feeds A[l%16][l/16] = Z[row][q] and
//     B[l/16][l%16] = V[row][c], and holds D[4j + l/16][l%16] in element j.
//     Then one reduction tree per instance, whose finisher ends the
//     iteration as k_update does.
// ---------------------------------------------------------------------------
constexpr int BT_ROWS = 128;   // rows per tile
constexpr int BT_SL = 4;       // instance slices: threads per row
constexpr int BT_THREADS = BT_ROWS * BT_SL;   // 8 waves
constexpr int BT_G = 16;       // instances per group (2 BT_G = 32 MFMA columns)
constexpr int BT_GS = BT_G / BT_SL;           // instances per slice

template <typename V, typename M, int KP>
__global__ void __launch_bounds__(BT_THREADS) k_pupdate_bt(IterArgs<V, M> a) {
  constexpr int K1 = KP > 0 ? KP : 1;
  __shared__ M zt[K1][BT_ROWS];
  __shared__ double cf[BT_G][K1];
  __shared__ double sb[BT_G];
  __shared__ int sk[BT_G];
  const int tile = xcd_tile(blockIdx.x, a.bt_ntiles_pad);
  if (tile >= a.bt_ntiles) return;
  const int64_t N = a.op.N;
  const int t = threadIdx.x;
  const int rl = t % BT_ROWS, sl = t / BT_ROWS;
  const int64_t i = (int64_t)tile * BT_ROWS + rl;
  const bool row = i < N;
  for (int e = t; e < KP * BT_ROWS; e += BT_THREADS) {      // Z tile, coalesced along rows
    const int q = e / BT_ROWS, r = e % BT_ROWS;
    const int64_t gi = (int64_t)tile * BT_ROWS + r;
    zt[q][r] = gi < N ? a.Z[(size_t)q * N + gi] : (M)0;
  }
  for (int g0 = 0; g0 < a.B; g0 += BT_G) {
    const int G = min(BT_G, a.B - g0);
    __syncthreads();
    if (t < BT_G) {
      int k = 0;
      double b = 0.0;
      if (t < G) {
        const Inst* S = a.inst + g0 + t;
        k = S->done ? 0 : (S->kk > 0 ? 2 : 1);
        b = S->fresh ? 0.0 : S->beta;
      }
      sk[t] = k;
      sb[t] = b;
    }
    for (int e = t; e < G * KP; e += BT_THREADS) {
      const int j = e / K1, q = e % K1;
      cf[j][q] = a.inst[g0 + j].coef[q];
    }
    __syncthreads();
    if (!row) continue;
#pragma unroll
    for (int jj = 0; jj < BT_GS; ++jj) {
      const int j = sl * BT_GS + jj;
      if (!sk[j]) continue;
      const int m = g0 + j;
      // loads issued regardless of the mask (all arrays span N rows); the
      // store is skipped on active rows, where p stays 0
      const bool on = a.mask[(size_t)m * N + i] == 0;
      V* p = a.p + m * a.vs;
      double pv = (double)a.z[m * a.vs + i] + sb[j] * (double)p[i];
      if (sk[j] == 2) {
#pragma unroll
        for (int q = 0; q < KP; ++q) pv -= (double)zt[q][rl] * cf[j][q];
      }
      if (on) p[i] = (V)pv;
    }
  }
}

typedef double bt_d4 __attribute__((ext_vector_type(4)));

// k_zproj_bt: each block walks BT_TPB consecutive tiles and keeps summing into
// its matrix-core accumulators, so the reduction tree has one leaf per block.
constexpr int BT_TPB = 4;

template <typename M, int KP>
__global__ void __launch_bounds__(BT_THREADS) __attribute__((amdgpu_waves_per_eu(4, 8))) k_zproj_bt(IterArgs<double, M> a) {
  constexpr int KQ = (KP + 15) / 16 * 16;          // Z columns padded to the MFMA tile
  constexpr int NC = 2 * BT_G;                     // V columns
  constexpr int NV = 2 * KP + 2;
  constexpr int NQT = KQ / 16;                     // q tiles (0 when KP = 0: no coarse space)
  constexpr int NT = NQT * (NC / 16);              // output tiles
  constexpr int NWV = BT_THREADS / 64;             // waves
  constexpr int TPW = NT > 0 ? (NT + NWV - 1) / NWV : 1;   // output tiles per wave
  constexpr int KS = BT_ROWS / 4;                  // MFMA k steps per tile
  constexpr int DR = 8;                            // stencil diagonals kept in registers
  __shared__ double vs[BT_ROWS][NC + 1];
  __shared__ double bvs[BT_G * NV];                // block sums, instance-major
  __shared__ double tots[BT_G * NV];
  __shared__ double red[NWV][2 * BT_GS];
  __shared__ int sk[BT_G];
  const int blk = xcd_tile(blockIdx.x, a.bt_nblk_pad);   // leaf of the reduction tree
  const int64_t N = a.op.N;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int rl = t % BT_ROWS, sl = t / BT_ROWS;    // waves 2 sl, 2 sl + 1 hold slice sl
  const int D = a.op.D;
  for (int g0 = 0; g0 < a.B; g0 += BT_G) {
    const int G = min(BT_G, a.B - g0);
    __syncthreads();
    if (t < BT_G) {
      int k = 0;
      if (t < G) {
        const Inst* S = a.inst + g0 + t;
        k = S->done ? 0 : (S->kk > 0 ? 2 : 1);
      }
      sk[t] = k;
    }
    __syncthreads();
    double rzv[BT_GS], rrv[BT_GS];
#pragma unroll
    for (int jj = 0; jj < BT_GS; ++jj) { rzv[jj] = 0.0; rrv[jj] = 0.0; }
    bt_d4 acc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) acc[s] = bt_d4{0.0, 0.0, 0.0, 0.0};
    for (int tt = 0; tt < BT_TPB; ++tt) {
      const int tile = blk * BT_TPB + tt;
      const int64_t base = (int64_t)tile * BT_ROWS;
      const int64_t i = base + rl;
      const bool row = (tile < a.bt_ntiles) && i < N;
      // V = [u r] for this thread's slice of instances on its row
      double cw[DR];
#pragma unroll
      for (int d = 0; d < DR; ++d) cw[d] = (row && d < D) ? a.dia64[(size_t)d * N + i] : 0.0;
#pragma unroll
      for (int jj = 0; jj < BT_GS; ++jj) {
        const int j = sl * BT_GS + jj;
        double uv = 0.0, rv = 0.0;
        if (sk[j] && row) {
          const int m = g0 + j;
          const bool on = a.mask[(size_t)m * N + i] == 0;
          const double zv = a.z[m * a.vs + i];       // zero on active rows
          rv = a.r[m * a.vs + i];
          rzv[jj] += rv * zv;
          rrv[jj] += rv * rv;
          if (sk[j] == 2 && on) {
            const double* sv = (a.op.D1 ? a.t : a.z) + m * a.vs;
            double sacc = 0.0;
            if (D <= DR) {
#pragma unroll
              for (int d = 0; d < DR; ++d)
                if (d < D) sacc += cw[d] * sv[i + a.op.offs[d]];
            } else {
              for (int d = 0; d < D; ++d) sacc += a.dia64[(size_t)d * N + i] * sv[i + a.op.offs[d]];
            }
            const Inst* S = a.inst + m;
            uv = S->a * sacc + S->c * zv;
          }
        }
        vs[rl][2 * j] = uv;
        vs[rl][2 * j + 1] = rv;
      }
      __syncthreads();
      // [Z^T u | Z^T r] += Z_tile^T V_tile on the matrix cores, one output tile
      // per wave; the wave's A operands (Z^T, FP64) are loaded first
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        const int ot = wid + s * NWV;
        if (ot < NT) {
          const int qt = ot / (NC / 16), ct = ot % (NC / 16);
          const int cb = ct * 16 + (lane & 15), kr = lane >> 4;
          const int qa = qt * 16 + (lane & 15);
          // A operands in chunks of 8 k steps (fewer live registers)
          for (int k0 = 0; k0 < KS; k0 += 8) {
            double av[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int64_t gi = base + 4 * (k0 + k) + kr;
              av[k] = (qa < KP && tile < a.bt_ntiles && gi < N) ? a.Z64[(size_t)qa * N + gi] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
              acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k], vs[4 * (k0 + k) + kr][cb], acc[s], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
    // block sums: D[q][c], q = 16 qt + 4 e + kr, c = cb: u (even c) or r (odd c) of instance c / 2
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      const int ot = wid + s * NWV;
      if (ot < NT) {
        const int qt = ot / (NC / 16), ct = ot % (NC / 16);
        const int cb = ct * 16 + (lane & 15), kr = lane >> 4;
        const int jj = cb >> 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = qt * 16 + 4 * e + kr;
          if (q < KP) bvs[jj * NV + (cb & 1) * KP + q] = acc[s][e];
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < BT_GS; ++jj) {
      const double s1 = wave_sum(rzv[jj]);
      const double s2 = wave_sum(rrv[jj]);
      if (lane == 0) { red[wid][2 * jj] = s1; red[wid][2 * jj + 1] = s2; }
    }
    __syncthreads();
    for (int e = t; e < BT_G * 2; e += BT_THREADS) {   // slice j / BT_GS: waves 2 sl, 2 sl + 1
      const int j = e >> 1, w2 = e & 1;
      const int s2 = j / BT_GS, jj = j % BT_GS;
      bvs[j * NV + 2 * KP + w2] = red[2 * s2][2 * jj + w2] + red[2 * s2 + 1][2 * jj + w2];
    }
    __syncthreads();
    unsigned act = 0u;
    for (int j = 0; j < G; ++j)
      if (sk[j]) act |= 1u << j;
    const unsigned fin = tree_reduce_multi(a.gbt, blk, NV, act, G,
                                           a.part + (size_t)g0 * a.gbt.ptotal * NV, (size_t)a.gbt.ptotal * NV,
                                           a.ctr + (size_t)g0 * a.gbt.ctotal, (size_t)a.gbt.ctotal, bvs, tots);
    for (int j = 0; j < G; ++j) {
      if (!((fin >> j) & 1u)) continue;
      Inst* S = a.inst + g0 + j;
      update_finish<KP>(a.C + (size_t)(g0 + j) * KP * KP, tots + j * NV, S, S->kk > 0, a.maxit, a.seg_maxit);
      __syncthreads();
    }
  }
}

}  // namespace adef2
