// Device helpers shared by the solver kernels: constants, per-instance state,
// wave/block reductions and the deterministic reduction tree.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adef2 {

constexpr int TPB = 256;            // threads per block of the setup kernels
constexpr int NWAVE = TPB / 64;     // wave64
constexpr int IPB = 256;            // threads per block of the iteration kernels
constexpr int NIWAVE = IPB / 64;
constexpr int KMAX = 64;            // max deflation rank (padded to a multiple of 8)
constexpr int RED_FAN = 16;         // fan-in of the reduction tree
constexpr int RED_MAXLEV = 6;

// Per-instance solve state, resident in device memory.  Written only by the
// block that finishes a reduction tree (or by the one-block coarse kernel);
// read by every block of the following kernels.
struct Inst {
  double a, c;          // operator scale: S = a * S_ref + c * I
  double bb;            // ||src_I||^2 of the current sweep (b, or the FP64 residual)
  double thresh2;       // sweep stops when ||r||^2 <= thresh2
  double rho;           // r.z
  double alpha, beta;
  double rr;            // ||r||^2 after the last update
  double pw;            // p.Sp of the last iteration
  double cond;          // cond(E) of the orthonormalised coarse basis
  double bb64;          // ||b_I||^2 (FP64, outer)
  double rho_end;       // r.y at the end of the last sweep (direction carried over)
  double rr64_prev;     // outer residual before the last one
  double rr64_best;     // smallest outer residual so far
  double rr64;          // ||b_I - S_II x||^2 of the last outer residual
  double tol2;          // squared relative tolerance of this instance
  int32_t iters;        // CG iterations, all sweeps
  int32_t sweep_iters;
  int32_t done;         // current sweep finished (kernels skip the instance)
  int32_t outer_done;   // solve finished
  int32_t status;       // enum adef2_status of the solve
  int32_t setup_status; // enum adef2_status of the restriction (fallback, ...)
  int32_t kk;           // coarse dimension in use (0: plain Jacobi-PCG)
  int32_t fresh;        // next p update starts a new direction
  int32_t drift;        // last outer residual > 10x the sweep's recurrence residual
  int32_t capped;       // the last sweep ended at the segment cap, not at its tolerance
  int32_t n_inactive;
  int32_t k_eff;        // kept restricted modes
  int32_t sweeps;
  int32_t has_dir;      // a search direction from the previous sweep exists
  int32_t stall;        // outer steps since the best residual last halved
  int32_t learned;      // the learned enrichment vectors are in the coarse space
  int32_t trans;        // a new sweep was set up in this chunk's transition (init2 pending)
  double coef[KMAX];    // coarse coefficients of the next x / p update
};

// Geometry of the reduction tree: level 0 has one node per tile, level l has
// ceil(n_{l-1} / RED_FAN) nodes, the last level has one node.
struct RedGeom {
  int nlev;
  int n[RED_MAXLEV];
  int pofs[RED_MAXLEV];     // node offsets into the partial-sum array
  int cofs[RED_MAXLEV];     // node offsets into the counter array (levels >= 1)
  int ptotal;               // nodes per instance
  int ctotal;               // counters per instance
};

// Agent-scope (all XCDs) loads and stores of reduction partials.  They bypass
// the non-coherent per-XCD L2 state for these addresses only, so the
// reduction needs no L2-wide writeback/invalidate fence.
__device__ __forceinline__ double ld_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until this thread's outstanding memory operations have completed
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sums of NV per-thread values.  The result lands in out[0..NV)
// (LDS), valid after the call for every thread.  red: LDS [NWAVE * NV].
template <int NV, int NW = NWAVE>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double s = wave_sum(v[j]);
    if (lane == 0) red[wid * NV + j] = s;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NV; j += blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w * NV + j];
    out[j] = s;
  }
  __syncthreads();
}

// Deterministic multi-block reduction.  Every block of a launch calls this
// once with its block sums in bval[0..nv) (LDS).  The block that completes the
// tree returns true with the totals in out[0..nv); all others return false.
// Partial sums are combined in a fixed order (node index), so results do not
// depend on block scheduling.  Counters are reset by their finisher.
// Publication protocol: partials are written with agent-scope stores and each
// thread waits for their completion before the block's barrier; only then is
// the node counter incremented (agent-scope atomic).  The block that observes
// the last arrival reads the partials with agent-scope loads.
__device__ inline bool tree_reduce(const RedGeom& g, int tile, int nv, double* part,
                                   unsigned* ctr, const double* bval, double* out) {
  __shared__ int s_last;
  if (g.nlev == 1) {
    for (int j = threadIdx.x; j < nv; j += blockDim.x) out[j] = bval[j];
    __syncthreads();
    return true;
  }
  int node = tile;
  for (int j = threadIdx.x; j < nv; j += blockDim.x)
    st_coherent(&part[(size_t)(g.pofs[0] + node) * nv + j], bval[j]);
  for (int l = 1; l < g.nlev; ++l) {
    wait_mem();
    __syncthreads();
    const int parent = node / RED_FAN;
    const int first = parent * RED_FAN;
    const int cnt = min(RED_FAN, g.n[l - 1] - first);
    if (threadIdx.x == 0) {
      unsigned old = __hip_atomic_fetch_add(&ctr[g.cofs[l] + parent], 1u, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      s_last = (old == (unsigned)(cnt - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    if (threadIdx.x == 0) __hip_atomic_store(&ctr[g.cofs[l] + parent], 0u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    const bool top = (l == g.nlev - 1);
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
      double s = 0.0;
      for (int i = 0; i < cnt; ++i) s += ld_coherent(&part[(size_t)(g.pofs[l - 1] + first + i) * nv + j]);
      if (top) out[j] = s;
      else st_coherent(&part[(size_t)(g.pofs[l] + parent) * nv + j], s);
    }
    node = parent;
  }
  __syncthreads();
  return true;
}

// tree_reduce for up to 32 instances at once that share the tile geometry:
// instance j (active when bit j of act is set) has its block sums in
// bval[j * nv ..], partials at part + pstride * j and counters at
// ctr + cstride * j.  The counter updates of all instances are issued
// together (one thread each), so a block pays one round trip per level
// instead of one per instance.  Returns the set of instances whose tree this
// block completed; their totals are in out[j * nv ..].
__device__ inline unsigned tree_reduce_multi(const RedGeom& g, int tile, int nv, unsigned act, int G,
                                             double* part, size_t pstride, unsigned* ctr, size_t cstride,
                                             const double* bval, double* out) {
  __shared__ unsigned s_last;
  if (g.nlev == 1) {
    for (int e = threadIdx.x; e < G * nv; e += blockDim.x) out[e] = bval[e];
    __syncthreads();
    return act;
  }
  int node = tile;
  for (int e = threadIdx.x; e < G * nv; e += blockDim.x) {
    const int j = e / nv, v = e - j * nv;
    if ((act >> j) & 1u) st_coherent(&part[pstride * j + (size_t)(g.pofs[0] + node) * nv + v], bval[e]);
  }
  if (threadIdx.x == 0) s_last = 0u;
  for (int l = 1; l < g.nlev; ++l) {
    wait_mem();
    __syncthreads();
    const int parent = node / RED_FAN;
    const int first = parent * RED_FAN;
    const int cnt = min(RED_FAN, g.n[l - 1] - first);
    if (threadIdx.x < G && ((act >> threadIdx.x) & 1u)) {
      unsigned* c = ctr + cstride * threadIdx.x + g.cofs[l] + parent;
      const unsigned old = __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old == (unsigned)(cnt - 1)) {
        __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicOr(&s_last, 1u << threadIdx.x);
      }
    }
    __syncthreads();
    act = s_last;
    __syncthreads();                  // every thread has read s_last before it is cleared
    if (threadIdx.x == 0) s_last = 0u;
    if (!act) return 0u;
    const bool top = (l == g.nlev - 1);
    for (int e = threadIdx.x; e < G * nv; e += blockDim.x) {
      const int j = e / nv, v = e - j * nv;
      if (!((act >> j) & 1u)) continue;
      double sum = 0.0;
      for (int i = 0; i < cnt; ++i)
        sum += ld_coherent(&part[pstride * j + (size_t)(g.pofs[l - 1] + first + i) * nv + v]);
      if (top) out[e] = sum;
      else st_coherent(&part[pstride * j + (size_t)(g.pofs[l] + parent) * nv + v], sum);
    }
    node = parent;
  }
  __syncthreads();
  return act;
}

// Map a workgroup id to a tile so that each XCD (workgroups are dispatched to
// the 8 XCDs round-robin) owns a contiguous range of tiles: stencil neighbours
// of a tile then mostly hit the same XCD's L2.  ntiles_pad % 8 == 0.
__device__ __forceinline__ int xcd_tile(int bid, int ntiles_pad) {
  const int per = ntiles_pad >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Block -> (tile, instance) for the batched iteration kernels, launched with
// ntiles_pad * B one-dimensional blocks.  XCD x (blocks are dispatched to the
// 8 XCDs round-robin) owns a contiguous range of tiles, and within an XCD the
// B instances of one tile run back to back: the operator stencils and the
// shared Z panel of a tile are then fetched from HBM about once per XCD and
// re-used from its L2 by the other instances.
__device__ __forceinline__ void tile_inst(int ntiles_pad, int& tile, int& m) {
  const int B = gridDim.x / ntiles_pad;
  const int bid = blockIdx.x;
  const int j = bid >> 3;
  tile = (bid & 7) * (ntiles_pad >> 3) + j / B;
  m = j % B;
}

}  // namespace adef2
