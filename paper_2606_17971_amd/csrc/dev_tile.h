// Tile-major iteration kernels for reference modes shared by every instance
// of a batch (gfx950, wave64, FP64 matrix cores).
//
// One block owns a tile of UB_ROWS consecutive rows for a group of
// instances, so each row of the shared modes is fetched once per group
// instead of once per instance, and the products with the shared modes run
// on the matrix cores (v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4e + l/16][l%16] in element e).  The modes are
// stored in FP32 or FP64 and widened exactly, the vectors are FP64, so the
// products are FP64 dot products in a fixed summation order.
//
//   k_pupdate_tm: p_j = z_j - Z c_j + beta_j p_j for PB_G = 16 instances.
//     For each 16-row slice, D[j][row] = sum_q c_j[q] Z[row][q] is one 16 x 16
//     output tile (A = the coarse coordinates, B = 16 rows of Z); the masks
//     of a wave's four slices are loaded first, and two slices are in
//     flight at a time.
//   k_update_tm: x_j += alpha_j p_j, r_j -= alpha_j w_j, z_j = K r_j for
//     UB_G = 8 instances, then [Z^T z_j | Z^T r_j] for all of them as
//     Z_tile^T [z_1 r_1 ... z_8 r_8] (KQ x 16 outputs), r_j.z_j and r_j.r_j
//     from the same staged tile (32 threads per instance), and W^T z from the
//     boundary form of W = S_II Z_I: every reference mode q is an eigenvector
//     of the reference operator B (S = a B + c I, B z_q = mu_q z_q), so
//     W = Lambda Z_I + (W - Lambda Z_I) with Lambda_q = a mu_q + c, and the
//     second term vanishes except on inactive rows whose stencil reaches the
//     active set (up to the eigen-residual).  Those rows are kept in a
//     compact list per instance and tile (row, W - Lambda Z), so
//       W^T z = Lambda Z^T z + (sum over the listed rows).
//     The Jacobi scaling 1 / (a d_i + c) is formed from the shared diagonal
//     of the reference stencil.  The block sums of each tile are stored with
//     plain stores; k_finish_tm reduces them (fixed order, many blocks per
//     instance) and ends the iteration as k_update's finisher does.  A
//     multi-level tree of agent-scope atomics inside the update kernel cost
//     more than the update's own traffic.
#pragma once
#include "dev_kernels.h"

namespace adef2 {

constexpr int UB_ROWS = 256;      // rows per tile
constexpr int UB_THREADS = 256;   // one row per thread, 4 waves
constexpr int UB_G = 8;           // instances per update block: 2 UB_G = 16 matrix-core columns
constexpr int PB_G = 16;          // instances per p-update block: 16 matrix-core rows
static_assert(UB_THREADS == 32 * UB_G, "the update's dot products take 32 threads per instance");

typedef double tm_d4 __attribute__((ext_vector_type(4)));

// Block -> (tile, instance group): XCD x (blocks are dispatched to the 8 XCDs
// round-robin) owns a contiguous range of tiles, and the groups of one tile
// run back to back on it, so a tile's rows of Z come from that XCD's L2 for
// every group after the first.  Launched with ntiles_pad * ngroups blocks.
__device__ __forceinline__ void tile_group(int ntiles_pad, int ngroups, int& tile, int& grp) {
  const int bid = blockIdx.x;
  const int j = bid >> 3;
  tile = (bid & 7) * (ntiles_pad >> 3) + j / ngroups;
  grp = j % ngroups;
}

// ---------------------------------------------------------------------------
// p_j = z_j - Z c_j + beta_j p_j
// ---------------------------------------------------------------------------
template <typename M, int KP>
__global__ void __launch_bounds__(UB_THREADS) k_pupdate_tm(IterArgs<double, M> a) {
  constexpr int KS = KP / 4;
  constexpr int KS1 = KS > 0 ? KS : 1;
  constexpr int K1 = KP > 0 ? KP : 1;
  __shared__ double cf[PB_G][K1 + 1];
  __shared__ double s_beta[PB_G];
  __shared__ int s_k[PB_G];
  __shared__ int s_keep[PB_G];
  int tile, grp;
  tile_group(a.ub_ntiles_pad, a.pb_ngroups, tile, grp);
  if (tile >= a.ub_ntiles) return;
  const int g0 = grp * PB_G;
  const int G = min(PB_G, a.B - g0);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int64_t N = a.op.N;
  const int64_t base = (int64_t)tile * UB_ROWS;
  const int cn = lane & 15, kk = lane >> 4;
  if (t < PB_G) {
    int k = 0, keep = 0;
    double b = 0.0;
    if (t < G) {
      const Inst* S = a.inst + g0 + t;
      k = S->done ? 0 : (S->kk > 0 ? 2 : 1);
      keep = !S->fresh;
      b = S->fresh ? 0.0 : S->beta;
    }
    s_k[t] = k; s_keep[t] = keep; s_beta[t] = b;
  }
  for (int e = t; e < PB_G * KP; e += UB_THREADS) {
    const int j = e / K1, q = e - j * K1;
    double v = 0.0;
    if (j < G) {
      const Inst* S = a.inst + g0 + j;
      if (!S->done && S->kk > 0) v = S->coef[q];
    }
    cf[j][q] = v;
  }
  // masks of the wave's four 16-row slices: they do not depend on the
  // instance state, so they are loaded (unconditionally, indices clamped)
  // before the barrier and kept only for iterating instances after it
  uint8_t mk[4][4];
#pragma unroll
  for (int s0 = 0; s0 < 4; ++s0) {
    const int64_t i = base + 64 * wid + 16 * s0 + cn;
    const int64_t ic = i < N ? i : N - 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * e + kk;
      mk[s0][e] = a.mask[(size_t)(g0 + (j < G ? j : 0)) * N + ic];
    }
  }
  __syncthreads();
  bool any = false;
  for (int j = 0; j < PB_G; ++j) any |= s_k[j] != 0;
  if (!any) return;
#pragma unroll
  for (int s0 = 0; s0 < 4; ++s0) {
    const int64_t i = base + 64 * wid + 16 * s0 + cn;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * e + kk;
      if (!(j < G && i < N && s_k[j])) mk[s0][e] = 1;
    }
  }
  // A operand: the coarse coordinates, A[j = cn][k = kk]; B operand: rows
  // of Z, B[k = kk][row = cn] = Z[row][4 s + kk]
  double av[KS1];
#pragma unroll
  for (int s = 0; s < KS; ++s) av[s] = cf[cn][4 * s + kk];
  // loads of one 16-row slice: the rows of Z first, then the vectors (a
  // wave's loads complete in order, so the products wait for Z only).  With
  // FP32 panels Z is read from its row-major copy: the KP values of a row are
  // one contiguous run that this slice's loads consume whole (in the
  // column-major layout each load takes half of a 128-byte line per column
  // and the other half is left to another slice)
  auto load_slice = [&](int s0, M (&bv)[KS1], double (&zv)[4], double (&pv)[4]) {
    const int64_t i = base + 64 * wid + 16 * s0 + cn;
    const int64_t ic = i < N ? i : N - 1;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if constexpr (sizeof(M) == 4) bv[s] = a.ZT[(size_t)ic * KP + 4 * s + kk];
      else bv[s] = a.Z[(size_t)(4 * s + kk) * N + ic];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * e + kk;
      zv[e] = 0.0;
      pv[e] = 0.0;
      if (!mk[s0][e]) {
        const int64_t o = (int64_t)(g0 + j) * a.vs + i;
        zv[e] = a.z[o];
        if (s_keep[j]) pv[e] = a.p[o];
      }
    }
  };
  // D[j][row] = sum_q c_j[q] Z[row][q] on the matrix cores, then the stores
  auto finish_slice = [&](int s0, const M (&bv)[KS1], const double (&zv)[4], const double (&pv)[4]) {
    const int64_t i = base + 64 * wid + 16 * s0 + cn;
    tm_d4 d = tm_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; ++s)
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], i < N ? (double)bv[s] : 0.0, d, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (mk[s0][e]) continue;
      const int j = 4 * e + kk;
      double pn = zv[e] - d[e];
      if (s_keep[j]) pn += s_beta[j] * pv[e];
      a.p[(int64_t)(g0 + j) * a.vs + i] = pn;
    }
  };
  // two slices in flight: the next slice's loads are issued before this
  // slice's products and stores
  M bv0[KS1], bv1[KS1];
  double zv0[4], pv0[4], zv1[4], pv1[4];
  load_slice(0, bv0, zv0, pv0);
  load_slice(1, bv1, zv1, pv1);
  finish_slice(0, bv0, zv0, pv0);
  load_slice(2, bv0, zv0, pv0);
  finish_slice(1, bv1, zv1, pv1);
  load_slice(3, bv1, zv1, pv1);
  finish_slice(2, bv0, zv0, pv0);
  finish_slice(3, bv1, zv1, pv1);
}

// ---------------------------------------------------------------------------
// x_j += alpha_j p_j, r_j -= alpha_j w_j, z_j = K r_j;
// block sums [W^T z_j | Z^T r_j | r_j.z_j | r_j.r_j] of the tile, stored to
// part[m][tile][0 .. 2 KP + 2) for k_finish_tm
// ---------------------------------------------------------------------------
// Up to 32 modes: at least 4 waves per SIMD, the register budget (<= 128)
// that lets four 256-thread blocks share a CU; the default allocation (3
// waves) left the vector loads' latency exposed (71 vs 81 us at 511^2 x 16).
// Wider bases would spill under that budget and keep the default.
template <typename M, int KP>
__global__ void __launch_bounds__(UB_THREADS) __attribute__((amdgpu_waves_per_eu(KP <= 32 ? 4 : 1, 8)))
k_update_tm(IterArgs<double, M> a) {
  constexpr int KQ = (KP + 15) / 16 * 16;          // columns padded to the matrix-core tile
  constexpr int NQT = KQ / 16;
  constexpr int NV = 2 * KP + 2;
  constexpr int NC = 2 * UB_G;                     // z_j, r_j columns
  constexpr int NWV = UB_THREADS / 64;
  constexpr int ZR = UB_ROWS * NC;                 // [row][NC] tile of z and r
  constexpr int NQG = NQT > 0 ? NQT : 1;           // product tiles
  constexpr int PW = NWV * NQG * 256;              // wave partials of the products
  constexpr int SH = ZR > PW ? ZR : PW;
  constexpr int LPE = KP <= 32 ? 2 : 1;            // boundary entries per wave step
  constexpr int BU = 4;                            // boundary steps loaded ahead
  constexpr int KB = KQ > 0 ? KQ : 1;
  __shared__ double sh[SH];
  __shared__ double bsum[UB_G][KB];
  __shared__ double dots[UB_G][2];                 // r_j.z_j, r_j.r_j of the tile
  __shared__ double s_alpha[UB_G], s_a[UB_G], s_c[UB_G];
  __shared__ int s_k[UB_G];
  int tile, grp;
  tile_group(a.ub_ntiles_pad, a.ub_ngroups, tile, grp);
  const int g0 = grp * UB_G;
  const int G = min(UB_G, a.B - g0);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int64_t N = a.op.N;
  const int64_t base = (int64_t)tile * UB_ROWS;
  const bool in_tile = tile < a.ub_ntiles;
  const int64_t i = base + t;
  const bool row = in_tile && i < N;

  // loads that depend on nothing but the block: boundary list offsets of
  // this wave's instances j = wid + NWV h, masks, the shared diagonal
  int e0[2] = {0, 0}, e1[2] = {0, 0};
  if (KP > 0 && in_tile) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = wid + NWV * h;
      if (j < G) {
        const int32_t* to = a.btoff + (size_t)(g0 + j) * (a.ub_ntiles + 1) + tile;
        e0[h] = to[0];
        e1[h] = to[1];
      }
    }
  }
  uint8_t mk[UB_G];
#pragma unroll
  for (int j = 0; j < UB_G; ++j) mk[j] = (j < G && row) ? a.mask[(size_t)(g0 + j) * N + i] : (uint8_t)1;
  const double dg = row ? a.diag[i] : 0.0;
  if (t < UB_G) {
    int k = 0;
    double al = 0.0, sa = 0.0, sc = 0.0;
    if (t < G) {
      const Inst* S = a.inst + g0 + t;
      k = S->done ? 0 : (S->kk > 0 ? 2 : 1);
      al = S->alpha;
      sa = S->a;
      sc = S->c;
    }
    s_k[t] = k;
    s_alpha[t] = al;
    s_a[t] = sa;
    s_c[t] = sc;
  }
  __syncthreads();
  unsigned act = 0u;
  for (int j = 0; j < UB_G; ++j)
    if (s_k[j]) act |= 1u << j;
  if (!act) return;

  // vector loads of the iterating instances' inactive rows, and the first
  // boundary entries (their list offsets have arrived by now)
  double xv[UB_G], pv[UB_G], rv[UB_G], wv[UB_G];
#pragma unroll
  for (int j = 0; j < UB_G; ++j) {
    xv[j] = pv[j] = rv[j] = wv[j] = 0.0;
    if (s_k[j] && !mk[j]) {
      const int64_t o = (int64_t)(g0 + j) * a.vs + i;
      xv[j] = a.x[o];
      pv[j] = a.p[o];
      rv[j] = a.r[o];
      wv[j] = a.w[o];
    } else {
      mk[j] = 1;
    }
  }
  const int bq = (LPE == 2) ? (lane & 31) : lane;
  const int bsub = (LPE == 2) ? (lane >> 5) : 0;
  double bwv[2][BU];
  int bri[2][BU];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (s_k[wid + NWV * h] != 2) e1[h] = e0[h];
#pragma unroll
    for (int u = 0; u < BU; ++u) {
      const int e = e0[h] + bsub + LPE * u;
      const bool ok = e < e1[h];
      bri[h][u] = ok ? (int)(a.bidx[e] - base) : 0;
      bwv[h][u] = (ok && bq < KP) ? (double)a.bW[(size_t)e * KP + bq] : 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < UB_G; ++j) {
    double zq = 0.0, rq = 0.0;
    if (!mk[j]) {
      const int64_t o = (int64_t)(g0 + j) * a.vs + i;
      const double al = s_alpha[j];
      const double xn = xv[j] + al * pv[j];
      rq = rv[j] - al * wv[j];
      const double dinv = a.precond_none ? 1.0 : 1.0 / (s_a[j] * dg + s_c[j]);
      zq = dinv * rq;
      a.x[o] = xn;
      a.r[o] = rq;
      a.z[o] = zq;
    }
    sh[t * NC + 2 * j] = zq;
    sh[t * NC + 2 * j + 1] = rq;
  }
  __syncthreads();

  // [Z^T z_j | Z^T r_j] on the matrix cores: wave w sums rows 64 w .. 64 w + 63;
  // in k step s lane group kk takes row 64 w + 4 s + kk, so A (row-major Z)
  // reads 4 rows x 16 consecutive columns per instruction
  tm_d4 acc[NQG];
#pragma unroll
  for (int qt = 0; qt < NQG; ++qt) acc[qt] = tm_d4{0.0, 0.0, 0.0, 0.0};
  if constexpr (KP > 0) {
    const int cn = lane & 15, kk = lane >> 4;
    M zraw[16][NQT];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int64_t gi = base + 64 * wid + 4 * s + kk;
#pragma unroll
      for (int qt = 0; qt < NQT; ++qt) {
        const int q = qt * 16 + cn;
        zraw[s][qt] = (q < KP && in_tile && gi < N) ? a.ZT[(size_t)gi * KP + q] : (M)0;
      }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const double bval = sh[(64 * wid + 4 * s + kk) * NC + cn];
#pragma unroll
      for (int qt = 0; qt < NQT; ++qt)
        acc[qt] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)zraw[s][qt], bval, acc[qt], 0, 0, 0);
    }
  }
  // r_j.z_j and r_j.r_j from the staged tile: thread t sums 8 rows of
  // instance j = t / 32, then 5 shuffle steps within its 32 lanes (instead of
  // 16 wave-wide reductions, or a Gram on the matrix cores, whose FP64 rate
  // is the vector rate on this chip)
  {
    const int j = t >> 5, l = t & 31;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int u = 0; u < UB_ROWS / 32; ++u) {
      const int rw = l + 32 * u;
      const double zz = sh[rw * NC + 2 * j], rr = sh[rw * NC + 2 * j + 1];
      s1 += rr * zz;
      s2 += rr * rr;
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      s1 += __shfl_xor(s1, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    if (l == 0) {
      dots[j][0] = s1;
      dots[j][1] = s2;
    }
  }
  // boundary rows: (W - Lambda Z)^T z_j over the tile's listed rows, lanes
  // over the columns, entries in list order (deterministic)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = wid + NWV * h;
    double ab = 0.0;
    if (e1[h] > e0[h]) {
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        const int e = e0[h] + bsub + LPE * u;
        if (e < e1[h]) ab += bwv[h][u] * sh[bri[h][u] * NC + 2 * j];
      }
      for (int e = e0[h] + bsub + LPE * BU; e < e1[h]; e += LPE) {
        const double wq = bq < KP ? (double)a.bW[(size_t)e * KP + bq] : 0.0;
        ab += wq * sh[(int)(a.bidx[e] - base) * NC + 2 * j];
      }
    }
    if (LPE == 2) ab += __shfl_down(ab, 32, 64);
    if (bsub == 0 && bq < KB) bsum[j][bq] = ab;
  }
  __syncthreads();                                  // sh no longer holds [z r]
#pragma unroll
  for (int qt = 0; qt < NQG; ++qt)
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[((wid * NQG + qt) * 4 + e) * 64 + lane] = acc[qt][e];
  __syncthreads();
  // block sums per instance: D[q][c] sits in wave partial (qt = q / 16,
  // e = (q % 16) / 4) at lane 16 (q % 4) + c; stored for the finisher
  for (int o = t; o < UB_G * NV; o += UB_THREADS) {
    const int j = o / NV, v = o - j * NV;
    if (!((act >> j) & 1u)) continue;
    double val = 0.0;
    if (v < 2 * KP) {
      const bool zpart = v < KP;
      const int q = zpart ? v : v - KP;
      const int c = 2 * j + (zpart ? 0 : 1);
      const int qt = q >> 4, e = (q & 15) >> 2, ln = (q & 3) * 16 + c;
      double dsum = 0.0;
      for (int w = 0; w < NWV; ++w) dsum += sh[((w * NQG + qt) * 4 + e) * 64 + ln];
      val = zpart ? (s_a[j] * a.mu[q] + s_c[j]) * dsum + bsum[j][q] : dsum;
    } else {
      val = dots[j][v - 2 * KP];
    }
    a.part[((size_t)(g0 + j) * a.ub_ntiles_pad + tile) * NV + v] = val;
  }
}

// ---------------------------------------------------------------------------
// Warp-specialised form of the update (up to 32 modes): one block of 8 waves
// owns an instance group and a run of T consecutive tiles.  Waves 0-3 do
// the vector work of tile q (x, r, z for the group's 8 instances) and stage
// [z r] into zr[q & 1], while waves 4-7 form the projections of tile q - 1
// from zr[(q - 1) & 1]: the matrix-core products with the shared modes, the
// boundary rows, r.z and r.r.  One barrier per step; the two halves work on
// different tiles, so the products overlap the next tile's loads (within one
// wave they could not: a wave's vector-memory counter completes in order).
// The products, boundary sums and dot products accumulate over the run in
// registers, and each block stores one partial per instance (the run's
// leaf) for k_finish_tm.  Same per-row arithmetic as k_update_tm; the sums
// are added tile by tile within a run.
// ---------------------------------------------------------------------------
constexpr int WS_THREADS = 512;

template <typename M, int KP>
__global__ void __launch_bounds__(WS_THREADS) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_update_ws(IterArgs<double, M> a) {
  static_assert(KP > 0 && KP <= 32, "warp-specialised update: 1..32 modes");
  constexpr int KQ = (KP + 15) / 16 * 16;
  constexpr int NQT = KQ / 16;
  constexpr int NV = 2 * KP + 2;
  constexpr int NC = 2 * UB_G;
  constexpr int ZR = UB_ROWS * NC;
  constexpr int LPE = 2;
  constexpr int BU = 4;
  __shared__ double zr[2][ZR];
  __shared__ double s_alpha[UB_G], s_a[UB_G], s_c[UB_G];
  __shared__ int s_k[UB_G];
  const int per = a.ub_ntiles_pad >> 3;
  const int xcd = blockIdx.x & 7, jb = blockIdx.x >> 3;
  const int grp = jb % a.ub_ngroups, run = jb / a.ub_ngroups;
  const int T = a.ws_T;
  const int tb = xcd * per + run * T;
  const int te = min(tb + T, (xcd + 1) * per);
  const int leaf = xcd * a.ws_cpx + run;
  const int g0 = grp * UB_G;
  const int G = min(UB_G, a.B - g0);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const bool memw = wid < 4;
  const int tt = t & 255;
  const int64_t N = a.op.N;
  if (t < UB_G) {
    int k = 0;
    double al = 0.0, sa = 0.0, sc = 0.0;
    if (t < G) {
      const Inst* S = a.inst + g0 + t;
      k = S->done ? 0 : (S->kk > 0 ? 2 : 1);
      al = S->alpha;
      sa = S->a;
      sc = S->c;
    }
    s_k[t] = k;
    s_alpha[t] = al;
    s_a[t] = sa;
    s_c[t] = sc;
  }
  __syncthreads();
  unsigned act = 0u;
  for (int j = 0; j < UB_G; ++j)
    if (s_k[j]) act |= 1u << j;
  if (!act) return;
  // product waves: running sums over the run's tiles
  const int cw = wid - 4;
  const int cn = lane & 15, kk = lane >> 4;
  const int bq = lane & 31, bsub = lane >> 5;
  tm_d4 acc[NQT];
#pragma unroll
  for (int qt = 0; qt < NQT; ++qt) acc[qt] = tm_d4{0.0, 0.0, 0.0, 0.0};
  double ab[2] = {0.0, 0.0};
  double d1 = 0.0, d2 = 0.0;
  for (int q = 0; q <= te - tb; ++q) {
    if (memw) {
      if (tb + q < te) {
        const int tile = tb + q;
        const int64_t i = (int64_t)tile * UB_ROWS + tt;
        const bool row = tile < a.ub_ntiles && i < N;
        const int64_t ic = row ? i : 0;
        uint8_t mk[UB_G];
#pragma unroll
        for (int j = 0; j < UB_G; ++j) {
          const uint8_t mv = a.mask[(size_t)(g0 + (j < G ? j : 0)) * N + ic];
          mk[j] = (j < G && row && s_k[j]) ? mv : (uint8_t)1;
        }
        const double dg = a.diag[ic];
        double xv[UB_G], pv[UB_G], rv[UB_G], wv[UB_G];
#pragma unroll
        for (int j = 0; j < UB_G; ++j) {
          xv[j] = pv[j] = rv[j] = wv[j] = 0.0;
          if (!mk[j]) {
            const int64_t o = (int64_t)(g0 + j) * a.vs + i;
            xv[j] = a.x[o];
            pv[j] = a.p[o];
            rv[j] = a.r[o];
            wv[j] = a.w[o];
          }
        }
        double* zb = zr[q & 1];
#pragma unroll
        for (int j = 0; j < UB_G; ++j) {
          double zq = 0.0, rq = 0.0;
          if (!mk[j]) {
            const int64_t o = (int64_t)(g0 + j) * a.vs + i;
            const double al = s_alpha[j];
            const double xn = xv[j] + al * pv[j];
            rq = rv[j] - al * wv[j];
            const double dinv = a.precond_none ? 1.0 : 1.0 / (s_a[j] * dg + s_c[j]);
            zq = dinv * rq;
            a.x[o] = xn;
            a.r[o] = rq;
            a.z[o] = zq;
          }
          zb[tt * NC + 2 * j] = zq;
          zb[tt * NC + 2 * j + 1] = rq;
        }
      }
    } else if (q >= 1) {
      const int tile = tb + q - 1;
      const int64_t base = (int64_t)tile * UB_ROWS;
      const bool in_tile = tile < a.ub_ntiles;
      const double* zb = zr[(q - 1) & 1];
      // boundary lists of this wave's instances j = cw + 4 h
      int e0[2] = {0, 0}, e1[2] = {0, 0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = cw + 4 * h;
        if (in_tile && j < G && s_k[j] == 2) {
          const int32_t* to = a.btoff + (size_t)(g0 + j) * (a.ub_ntiles + 1) + tile;
          e0[h] = to[0];
          e1[h] = to[1];
        }
      }
      M zraw[16][NQT];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int64_t gi = base + 64 * cw + 4 * s + kk;
#pragma unroll
        for (int qt = 0; qt < NQT; ++qt) {
          const int qq = qt * 16 + cn;
          zraw[s][qt] = (qq < KP && in_tile && gi < N) ? a.ZT[(size_t)gi * KP + qq] : (M)0;
        }
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const double bval = zb[(64 * cw + 4 * s + kk) * NC + cn];
#pragma unroll
        for (int qt = 0; qt < NQT; ++qt)
          acc[qt] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)zraw[s][qt], bval, acc[qt], 0, 0, 0);
      }
      {
        const int ct = t - 256, j = ct >> 5, l = ct & 31;
#pragma unroll
        for (int u = 0; u < UB_ROWS / 32; ++u) {
          const int rw = l + 32 * u;
          const double zz = zb[rw * NC + 2 * j], rr = zb[rw * NC + 2 * j + 1];
          d1 += rr * zz;
          d2 += rr * rr;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = cw + 4 * h;
        for (int e = e0[h] + bsub; e < e1[h]; e += LPE) {
          const double wq = bq < KP ? (double)a.bW[(size_t)e * KP + bq] : 0.0;
          ab[h] += wq * zb[(int)(a.bidx[e] - base) * NC + 2 * j];
        }
      }
    }
    __syncthreads();
  }
  // run totals: the product waves' partials into zr[0], the boundary sums and
  // dot products into zr[1]; then one partial per instance for the finisher
  double* pw = zr[0];
  double* bs = zr[1];                              // [UB_G][32] boundary sums, then [UB_G][2] dots
  if (!memw) {
#pragma unroll
    for (int qt = 0; qt < NQT; ++qt)
#pragma unroll
      for (int e = 0; e < 4; ++e) pw[((cw * NQT + qt) * 4 + e) * 64 + lane] = acc[qt][e];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v = ab[h] + __shfl_down(ab[h], 32, 64);
      if (bsub == 0) bs[(cw + 4 * h) * 32 + bq] = v;
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      d1 += __shfl_xor(d1, off, 64);
      d2 += __shfl_xor(d2, off, 64);
    }
    const int ct = t - 256;
    if ((ct & 31) == 0) {
      bs[UB_G * 32 + 2 * (ct >> 5)] = d1;
      bs[UB_G * 32 + 2 * (ct >> 5) + 1] = d2;
    }
  }
  __syncthreads();
  for (int o = t; o < UB_G * NV; o += WS_THREADS) {
    const int j = o / NV, v = o - j * NV;
    if (!((act >> j) & 1u)) continue;
    double val = 0.0;
    if (v < 2 * KP) {
      const bool zpart = v < KP;
      const int q = zpart ? v : v - KP;
      const int c = 2 * j + (zpart ? 0 : 1);
      const int qt = q >> 4, e = (q & 15) >> 2, ln = (q & 3) * 16 + c;
      double dsum = 0.0;
      for (int w = 0; w < 4; ++w) dsum += pw[((w * NQT + qt) * 4 + e) * 64 + ln];
      val = zpart ? (s_a[j] * a.mu[q] + s_c[j]) * dsum + bs[j * 32 + q] : dsum;
    } else {
      val = bs[UB_G * 32 + 2 * j + (v - 2 * KP)];
    }
    a.part[((size_t)(g0 + j) * a.fin_leaves + leaf) * NV + v] = val;
  }
}

// ---------------------------------------------------------------------------
// Finisher of the tile-major update: per instance the tile sums
// part[m][tile][0 .. NV) are reduced in a fixed order.  Block (ch, sc, m)
// covers FC values of slice sc of the tiles (thread (v, s) sums value v over
// the slice's tiles s, s + FS, ..., then the FS partial sums are added in
// order) and publishes them with agent-scope stores to ftot[m][sc]; the last
// of the instance's blocks (agent-scope counter) adds the slices in order
// and ends the iteration (stopping tests, beta, coarse coordinates) as
// k_update does.  Grid (ceil(NV / FC), slices, B); the slice count divides
// ub_ntiles_pad (fin_slices).
// ---------------------------------------------------------------------------
constexpr int FC = 16;
constexpr int FS = UB_THREADS / FC;
constexpr int FIN_MAX_SLICES = 8;

// slices of the finisher for a padded tile count (a multiple of 8): at
// least 64 tiles each, at most FIN_MAX_SLICES
inline int fin_slices(int ntiles_pad) {
  int s = 1;
  while (s < FIN_MAX_SLICES && ntiles_pad % (2 * s) == 0 && ntiles_pad / (2 * s) >= 64) s *= 2;
  return s;
}

template <typename M, int KP>
__global__ void __launch_bounds__(UB_THREADS) k_finish_tm(IterArgs<double, M> a) {
  constexpr int NV = 2 * KP + 2;
  __shared__ double sl[UB_THREADS];
  __shared__ double tots[NV];
  __shared__ int s_last;
  const int m = blockIdx.z, ch = blockIdx.x, sc = blockIdx.y;
  const int nsl = gridDim.y;
  const unsigned nblk = gridDim.x * gridDim.y;
  Inst* S = a.inst + m;
  if (S->done) return;
  const int t = threadIdx.x;
  const int v = ch * FC + (t % FC), sidx = t / FC;
  const int tps = a.fin_leaves / nsl;
  const double* pm = a.part + ((size_t)m * a.fin_leaves + (size_t)sc * tps) * NV;
  double acc = 0.0;
  if (v < NV)
    for (int tl = sidx; tl < tps; tl += FS) acc += pm[(size_t)tl * NV + v];
  sl[t] = acc;
  __syncthreads();
  if (t < FC && ch * FC + t < NV) {
    double tot = 0.0;
    for (int s2 = 0; s2 < FS; ++s2) tot += sl[s2 * FC + t];
    st_coherent(&a.ftot[((size_t)m * nsl + sc) * NV + ch * FC + t], tot);
  }
  wait_mem();
  __syncthreads();
  if (t == 0) {
    const unsigned old = __hip_atomic_fetch_add(&a.fctr[m], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (old == nblk - 1);
    if (s_last) __hip_atomic_store(&a.fctr[m], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (!s_last) return;
  for (int e = t; e < NV; e += UB_THREADS) {
    double tot = 0.0;
    for (int q = 0; q < nsl; ++q) tot += ld_coherent(&a.ftot[((size_t)m * nsl + q) * NV + e]);
    tots[e] = tot;
  }
  __syncthreads();
  update_finish<KP>(a.C + (size_t)m * KP * KP, tots, S, S->kk > 0, a.maxit, a.seg_maxit);
}

// ---------------------------------------------------------------------------
// Stencil passes of the tile-major path: one block per tile and group of
// SG_G instances.  The stencil coefficients of a row are loaded once for the
// group (every instance shares them); each thread then applies them to its
// row of every instance of the group.
//   k_stencil1_tm: t_j = A p_j on all rows (inner stencil of the factored
//                  operator)
//   k_spmv_tm:     w_j = a_j (A^T t_j, or S p_j) + c_j p_j on inactive rows,
//                  and the tile sums of p_j.w_j into part[m][tile];
//   k_alpha_tm:    adds those tile sums in a fixed order and sets
//                  alpha_j = rho_j / p_j.w_j (breakdown test as in k_spmv).
// ---------------------------------------------------------------------------
constexpr int SG_G = 8;    // instances per stencil block
constexpr int SDR = 16;    // stencil diagonals held in registers (tile-major path needs D, D1 <= SDR)

// One row of a diagonal-format stencil with the row's coefficients cw[] in
// registers: the arithmetic and order of stencil_row (difference form for
// FP32 coefficients).
template <typename M, int DR>
__device__ __forceinline__ double stencil_row_reg(const double* cw, const int* offs, int D, int d0, int64_t i,
                                                  const double* v) {
  double acc = 0.0;
  if constexpr (sizeof(M) == 4) {
    if (d0 >= 0) {
      const double vi = v[i];
      double dg = 0.0;
#pragma unroll
      for (int d = 0; d < DR; ++d)
        if (d == d0) dg = cw[d];
      acc = dg * vi;
#pragma unroll
      for (int d = 0; d < DR; ++d)
        if (d < D && d != d0) acc += cw[d] * (v[i + offs[d]] - vi);
      return acc;
    }
  }
#pragma unroll
  for (int d = 0; d < DR; ++d)
    if (d < D) acc += cw[d] * v[i + offs[d]];
  return acc;
}

template <typename M>
__global__ void __launch_bounds__(UB_THREADS) k_stencil1_tm(IterArgs<double, M> a) {
  int tile, grp;
  tile_group(a.ub_ntiles_pad, a.sg_ngroups, tile, grp);
  if (tile >= a.ub_ntiles) return;
  const int g0 = grp * SG_G;
  const int G = min(SG_G, a.B - g0);
  const int64_t N = a.op.N;
  const int64_t i = (int64_t)tile * UB_ROWS + threadIdx.x;
  if (i >= N) return;
  const int D1 = a.op.D1;
  bool live[SG_G];
#pragma unroll
  for (int j = 0; j < SG_G; ++j) live[j] = j < G && !a.inst[g0 + j].done;
  double cw[SDR];
#pragma unroll
  for (int d = 0; d < SDR; ++d) cw[d] = d < D1 ? (double)a.dia1[(size_t)d * N + i] : 0.0;
  double tv[SG_G];
#pragma unroll
  for (int j = 0; j < SG_G; ++j)
    tv[j] = live[j] ? stencil_row_reg<M, SDR>(cw, a.op.offs1, D1, a.op.d01, i, a.p + (int64_t)(g0 + j) * a.vs)
                    : 0.0;
#pragma unroll
  for (int j = 0; j < SG_G; ++j)
    if (live[j]) a.t[(int64_t)(g0 + j) * a.vs + i] = tv[j];
}

template <typename M>
__global__ void __launch_bounds__(UB_THREADS) k_spmv_tm(IterArgs<double, M> a) {
  constexpr int NWV = UB_THREADS / 64;
  __shared__ double red[NWV][SG_G];
  int tile, grp;
  tile_group(a.ub_ntiles_pad, a.sg_ngroups, tile, grp);
  const int g0 = grp * SG_G;
  const int G = min(SG_G, a.B - g0);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int64_t N = a.op.N;
  const int64_t i = (int64_t)tile * UB_ROWS + t;
  const bool row = tile < a.ub_ntiles && i < N;
  const int D = a.op.D;
  bool live[SG_G];
  bool any = false;
#pragma unroll
  for (int j = 0; j < SG_G; ++j) {
    live[j] = j < G && !a.inst[g0 + j].done;
    any |= live[j];
  }
  if (!any) return;
  uint8_t mk[SG_G];
#pragma unroll
  for (int j = 0; j < SG_G; ++j) mk[j] = (live[j] && row) ? a.mask[(size_t)(g0 + j) * N + i] : (uint8_t)1;
  double cw[SDR];
#pragma unroll
  for (int d = 0; d < SDR; ++d) cw[d] = (row && d < D) ? (double)a.dia[(size_t)d * N + i] : 0.0;
  const double* sv = a.op.D1 ? a.t : a.p;
  double wv[SG_G], pw[SG_G];
#pragma unroll
  for (int j = 0; j < SG_G; ++j) {
    wv[j] = 0.0;
    pw[j] = 0.0;
    if (!mk[j]) {
      const Inst* S = a.inst + g0 + j;
      const int64_t o = (int64_t)(g0 + j) * a.vs;
      const double acc = stencil_row_reg<M, SDR>(cw, a.op.offs, D, a.op.d0, i, sv + o);
      const double pi = a.p[o + i];
      wv[j] = S->a * acc + S->c * pi;
      pw[j] = pi * wv[j];
    }
  }
#pragma unroll
  for (int j = 0; j < SG_G; ++j) {
    if (!mk[j]) a.w[(int64_t)(g0 + j) * a.vs + i] = wv[j];
    const double s = wave_sum(pw[j]);
    if (lane == 0) red[wid][j] = s;
  }
  __syncthreads();
  if (t < G && live[t]) {
    double s = 0.0;
    for (int w = 0; w < NWV; ++w) s += red[w][t];
    a.part[(size_t)(g0 + t) * a.ub_ntiles_pad + tile] = s;
  }
}

template <typename M>
__global__ void __launch_bounds__(UB_THREADS) k_alpha_tm(IterArgs<double, M> a) {
  __shared__ double red[UB_THREADS / 64];
  __shared__ double tot[1];
  const int m = blockIdx.x;
  Inst* S = a.inst + m;
  if (S->done) return;
  double v[1] = {0.0};
  const double* pm = a.part + (size_t)m * a.ub_ntiles_pad;
  for (int tl = threadIdx.x; tl < a.ub_ntiles_pad; tl += UB_THREADS) v[0] += pm[tl];
  block_sum<1, UB_THREADS / 64>(v, red, tot);
  if (threadIdx.x == 0) {
    const double pwt = tot[0];
    S->pw = pwt;
    if (!(pwt > 0.0) || !(pwt < INFINITY)) {
      S->done = 1;
      S->outer_done = 1;
      S->status = -5;
    } else {
      S->alpha = S->rho / pwt;
    }
  }
}

}  // namespace adef2
