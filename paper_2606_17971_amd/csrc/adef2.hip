// Host runtime and C ABI of the restricted A-DEF2 solver (see include/adef2.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adef2.h"
#include "dev_learned.h"
#include "iter_tab.h"

using namespace adef2;

// Scratch of the no-allocation compaction (adef2_compact_noalloc): chunk
// counts, chunk offsets and the inactive count for masks of up to
// NOALLOC_MAX_N entries (520 KiB).  Every GPU the library runs on holds one
// copy until the process ends.  Host code never passes the symbol itself:
// it uses the device address from hipGetSymbolAddress, taken once per device
// with that device current (at adef2_create, or at the entry point's first
// call on a device) and kept in g_scratch.
constexpr int64_t NOALLOC_MAX_N = (int64_t)1 << 28;
constexpr int64_t NOALLOC_CHUNKS = NOALLOC_MAX_N / adef2::CMP_CHUNK;
constexpr size_t NOALLOC_BYTES = (size_t)NOALLOC_CHUNKS * 2 * sizeof(int) + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEV = 64;
void* g_scratch[NOALLOC_MAX_DEV] = {};
std::mutex g_scratch_mu;

// device address of this device's scratch (dev must be current); null on failure
void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

std::string g_create_error;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int round8(int k) { return (k + 7) & ~7; }
constexpr double FP32_DROP = 1e-3;   // column-drop threshold with FP32 panels
// eigen-residual bound for the boundary form of W (FP32 panels only): an
// interior row of W - Lambda Z then holds at most 1e-6 |lambda| of its mode,
// the order of the FP32 rounding (6e-8) of the stored W that the mixed
// iteration carries anyway; the FP64 residual replacement keeps the accuracy
constexpr double EIG_TOL = 1e-6;
constexpr double FP32_COND = 1e-3 / 5.96e-8;   // learned cond(E) bound with FP32 panels

enum KernelId { KI_INIT = 0, KI_INIT2, KI_PUPDATE, KI_SPMV, KI_UPDATE, KI_RESID, KI_ACCUM,
                KI_GRAM, KI_COARSE, KI_COMPACT, KI_UPDATE_NW, KI_ZPROJ, KI_PUPDATE_BT, KI_ZPROJ_BT,
                KI_PUPDATE_TM, KI_UPDATE_TM, KI_FINISH_TM, KI_STENCIL, KI_OPFUSED, KI_COUNT };
static_assert(KI_COUNT <= ADEF2_STATS_KERNELS, "adef2_stats holds ADEF2_STATS_KERNELS entries");
const char* kKernelNames[KI_COUNT] = {"init", "init2", "pupdate", "spmv", "update", "resid64",
                                      "accumulate", "spmm_gram", "coarse", "compact", "update_nw",
                                      "zproj", "pupdate_bt", "zproj_bt", "pupdate_tm", "update_tm",
                                      "finish_tm", "stencil1", "opfused"};

}  // namespace

struct adef2_ctx {
  adef2_opts o{};
  hipStream_t st = nullptr;
  // captured chunks of iterations (HIP graphs), replayed on a private stream
  // ordered against st by events
  hipStream_t gst = nullptr;
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  struct GraphEntry { std::vector<char> key; hipGraphExec_t exec; };
  std::vector<GraphEntry> graphs;
  int dev = 0;
  std::string err;

  // reference operator and modes
  bool have_ref = false;
  int64_t N = 0;
  int D = 0, H = 0, k = 0, KP = 0;
  std::vector<int> offs;
  double* dia64 = nullptr;
  float* dia32 = nullptr;
  double* diag = nullptr;
  double* Z64 = nullptr;
  float* Z32 = nullptr;
  float* ZT32 = nullptr;           // [N][KP] row-major copy (tile-major kernels)
  double scale_a = 1.0, scale_c = 0.0;
  // factored operator S = alpha A^T A + shift I: inner stencil A (dia1),
  // outer stencil A^T (dia64/dia32 above, offsets offs)
  bool factored = false;
  int D1 = 0;
  std::vector<int> offs1;
  double* dia1_64 = nullptr;
  float* dia1_32 = nullptr;
  double alpha_ref = 1.0, shift_ref = 0.0;
  // POD enrichment: the first k_ref columns of Z are the reference modes;
  // columns k_safe.. (k_safe > 0) are POD candidates for the safe merge
  int k_ref = 0, k_safe = 0;
  double tau_safe = 1e4;
  // current coarse basis: shared reference modes (zs = 0) or a per-instance
  // basis [Z | V_m] of the learned enrichment (zs = KP * N, k_base = k of Z)
  int64_t zs = 0;
  int k_base = 0;
  int KPalloc = -1;

  // learned enrichment: POD pool Phi (N x p), MLP parameters, training data
  int p = 0;
  double* Phi = nullptr;
  float* mlp = nullptr;          // FP32 master parameters (packed)
  uint16_t* mlp_bf = nullptr;    // BF16 compute copy (same layout)
  float* mlp_g = nullptr;        // gradients
  float* mlp_m = nullptr;        // Adam first moments
  float* mlp_v = nullptr;        // Adam second moments
  int adam_t = 0;
  bool have_mlp = false;
  int Mtr = 0;
  float* theta_tr = nullptr;
  double *Htr = nullptr, *gtr = nullptr, *e0tr = nullptr, *bxtr = nullptr;
  double* Ntr = nullptr;          // [M][p][p] D-weighted Grams (deflated-spectrum objective)
  int obj_tr = 0;                 // objective the training samples were prepared for
  float *act = nullptr, *mout = nullptr, *dout = nullptr, *dA1 = nullptr, *dA2 = nullptr;
  double* lossv = nullptr;
  int Mcap_mlp = 0;
  double* Zb64 = nullptr;        // [B][KP][N] per-instance basis
  float* Zb32 = nullptr;
  size_t zb_cap = 0;             // elements allocated in Zb64 / Zb32
  double* Zsh64 = nullptr;       // shared reference modes while Z points at Zb
  float* Zsh32 = nullptr;
  // reference modes as eigenvectors of the base operator (boundary form of W)
  double* mu64 = nullptr;        // [KP] Rayleigh quotients
  uint8_t* eigf = nullptr;       // [KP] eigen-residual <= EIG_TOL
  int n_eig = 0;                 // columns flagged
  uint8_t* bnd = nullptr;        // [B][N] boundary rows of the current restriction
  uint8_t* hb = nullptr;         // [B][N] scratch of the boundary test
  double* zero64 = nullptr;      // 64 zero words (branch-free skipped loads)
  int ne = 0;                    // columns in boundary form for the current restriction
  // boundary rows compacted per instance and tile (tile-major boundary-form
  // update): counts, offsets [B][ub_ntiles + 1], rows and W - Lambda Z rows
  bool tm_ok = false;            // the current restriction supports the tile-major update
  int* bcnt = nullptr;
  double* ftot = nullptr;        // [B][slices][2 KP + 2] slice totals of the tile-major finisher
  unsigned* fctr = nullptr;      // [B] its arrival counters
  int* btoff = nullptr;
  int* btot = nullptr;
  int* bidx = nullptr;
  float* bW32 = nullptr;
  size_t bcap = 0;               // entries allocated in bidx / bW32
  int64_t nbnd = 0;              // entries of the current restriction
  double tau_learned = 1e8;

  // restriction / batch state
  bool restricted = false;
  int B = 0, Bcap = 0, prec = ADEF2_FP64;
  int64_t vs = 0;
  uint8_t* masks = nullptr;
  int* I = nullptr;
  int* g2l = nullptr;
  int* ccount = nullptr;
  int* cofs = nullptr;
  long long* ntot = nullptr;
  Inst* inst = nullptr;
  Inst* inst_h = nullptr;        // pinned mirror
  double* C = nullptr;
  double* Finfo = nullptr;
  int* kept = nullptr;
  double* gram = nullptr;
  double* v64[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  float* v32[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double* W64 = nullptr;
  float* W32 = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  double* x64 = nullptr;         // padded (refinement mode)
  double* r64 = nullptr;         // unpadded [B][N]
  double* x0pad = nullptr;       // padded warm start
  double* t64 = nullptr;         // padded A v (factored operator, FP64)
  float* t32 = nullptr;          // padded A v (factored operator, FP32 sweeps)
  double* Tm = nullptr;          // [B][KP][N] A Ztilde (factored operator setup)
  double* part = nullptr;
  unsigned* ctr = nullptr;
  size_t part_elems = 0, ctr_elems = 0;
  std::vector<size_t> bytes;     // allocation sizes (for growth)

  // geometry and variant of the streaming kernels
  int rpt = 2;
  int wfree = 0;                 // W^T z as Z^T (S z), W not read: 1 tile-major, 2 per instance;
                                 // 3: tile-major boundary form (k_pupdate_tm / k_update_tm)
  bool solved = false;           // a solve ran (variant is meaningful)
  int ntiles = 0, ntiles_pad = 0;
  int bt_ntiles = 0, bt_ntiles_pad = 0;   // tile-major kernels (BT_ROWS-row tiles)
  int bt_nblk_pad = 0;                     // k_zproj_bt blocks (BT_TPB tiles each)
  int ub_ntiles = 0, ub_ntiles_pad = 0;    // tile-major boundary-form kernels (UB_ROWS-row tiles)
  RedGeom g_ub{};
  RedGeom g_bt{};
  // fused operator pass of the factored form (k_opfused), 0 = two passes
  int opf = 0;
  int opg = 1;                   // instances per block of the fused pass (1, or 4: k_opfused_g)
  int uws = 0;                   // warp-specialised update (k_update_ws) instead of k_update_tm
  int ws_T = 1, ws_cpx = 0;      // its tiles per block and runs per XCD
  int of_rows = 0, of_halo = 0, of_ntiles = 0, of_ntiles_pad = 0;
  RedGeom g_of{};
  // opo: the op_fused option the entry was tuned under; opf: rows of the
  // fused operator pass (0 = two passes), opg its instances per block;
  // ms_op: trial times of the two passes and of the fused pass at each
  // candidate tile height, one instance per block [1..3] and four [4..6],
  // with the chosen rpt / wfree
  // uwo: the update_ws option tuned under; uws: the update form kept; ms_uw:
  // trial times of the per-tile and warp-specialised updates
  struct Tuned { int B, prec, KP, fact, tm; int64_t N; int rpt, wfree; float ms[10]; int opo, opf, opg; float ms_op[7];
                 int uwo, uws; float ms_uw[2]; int fro, fwo; };
  std::vector<Tuned> tuned;      // autotuned variants per configuration
  RedGeom g_iter{};
  int gram_blocks = 0;
  RedGeom g_gram{};

  // profiling
  struct Ev { int id; hipEvent_t a, b; double bytes; };
  std::vector<Ev> ev_pending;
  std::vector<hipEvent_t> ev_pool;
  int64_t st_launch[KI_COUNT] = {};
  double st_ms[KI_COUNT] = {};
  double st_bytes[KI_COUNT] = {};
  int64_t st_polls = 0;          // host polls of the device state (all solves since reset)
  int64_t pod_iters = 0;         // subspace iterations of the last POD (0: Jacobi on the whole Gram)
  std::vector<long long> nI_host;
  std::vector<double> tol_h;     // per-instance tolerances of the current solve
};

namespace {

int fail(adef2_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, ADEF2_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
int dalloc(adef2_ctx* c, T** p, size_t count) {
  if (*p) { hipFree(*p); *p = nullptr; }
  if (count == 0) return ADEF2_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, ADEF2_E_NOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                      " bytes failed: " + hipGetErrorString(e));
  }
  return ADEF2_OK;
}

RedGeom make_geom(int nleaf) {
  RedGeom g{};
  int n = nleaf, l = 0, p = 0, c = 0;
  g.n[0] = n;
  g.pofs[0] = 0;
  g.cofs[0] = 0;
  p += n;
  while (n > 1) {
    n = (int)cdiv(n, RED_FAN);
    ++l;
    g.n[l] = n;
    g.pofs[l] = p;
    g.cofs[l] = c;
    p += n;
    c += n;
  }
  g.nlev = l + 1;
  g.ptotal = p;
  g.ctotal = c;
  return g;
}

// padded vectors hold H zeros before and after each instance's N entries;
// kernels receive the address of instance 0's first interior entry
template <typename T>
T* interior(const adef2_ctx* c, T* base) { return base ? base + c->H : nullptr; }

OpGeom op_geom(const adef2_ctx* c) {
  OpGeom g{};
  g.N = c->N;
  g.D = c->D;
  g.ntiles = c->ntiles;
  g.ntiles_pad = c->ntiles_pad;
  for (int d = 0; d < c->D; ++d) g.offs[d] = c->offs[d];
  g.D1 = c->factored ? c->D1 : 0;
  for (int d = 0; d < g.D1; ++d) g.offs1[d] = c->offs1[d];
  g.d0 = g.d01 = -1;
  for (int d = 0; d < g.D; ++d) if (g.offs[d] == 0) g.d0 = d;
  for (int d = 0; d < g.D1; ++d) if (g.offs1[d] == 0) g.d01 = d;
  return g;
}

void drop_graphs(adef2_ctx* c) {
  for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

void free_all(adef2_ctx* c) {
  drop_graphs(c);
  if (c->gev_in) { hipEventDestroy(c->gev_in); c->gev_in = nullptr; }
  if (c->gev_out) { hipEventDestroy(c->gev_out); c->gev_out = nullptr; }
  if (c->gst) { hipStreamDestroy(c->gst); c->gst = nullptr; }
  auto F = [](void* p) { if (p) hipFree(p); };
  F(c->dia64); F(c->dia32); F(c->diag); F(c->Z64); F(c->Z32);
  F(c->masks); F(c->I); F(c->g2l); F(c->ccount); F(c->cofs); F(c->ntot); F(c->inst);
  F(c->C); F(c->Finfo); F(c->kept); F(c->gram);
  for (int j = 0; j < 5; ++j) { F(c->v64[j]); F(c->v32[j]); }
  F(c->W64); F(c->W32); F(c->dinv64); F(c->dinv32); F(c->x64); F(c->r64); F(c->x0pad);
  F(c->t64); F(c->t32); F(c->Tm); F(c->dia1_64); F(c->dia1_32);
  F(c->part); F(c->ctr);
  F(c->Phi); F(c->mlp); F(c->mlp_bf); F(c->mlp_g); F(c->mlp_m); F(c->mlp_v); F(c->theta_tr);
  F(c->Htr); F(c->Ntr); F(c->gtr); F(c->e0tr); F(c->bxtr); F(c->act); F(c->mout); F(c->dout); F(c->dA1);
  F(c->dA2); F(c->lossv); F(c->Zb64); F(c->Zb32); F(c->mu64); F(c->eigf); F(c->bnd); F(c->hb); F(c->zero64);
  F(c->ZT32); F(c->bcnt); F(c->ftot); F(c->fctr); F(c->btoff); F(c->btot); F(c->bidx); F(c->bW32);
  if (c->inst_h) hipHostFree(c->inst_h);
  for (auto& e : c->ev_pending) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
  for (auto e : c->ev_pool) hipEventDestroy(e);
}

// ---------------------------------------------------------------- profiling
hipEvent_t ev_get(adef2_ctx* c) {
  if (!c->ev_pool.empty()) { hipEvent_t e = c->ev_pool.back(); c->ev_pool.pop_back(); return e; }
  hipEvent_t e;
  hipEventCreate(&e);
  return e;
}

void ev_harvest(adef2_ctx* c) {
  for (auto& e : c->ev_pending) {
    float ms = 0.f;
    hipEventSynchronize(e.b);
    hipEventElapsedTime(&ms, e.a, e.b);
    c->st_launch[e.id] += 1;
    c->st_ms[e.id] += ms;
    c->st_bytes[e.id] += e.bytes;
    c->ev_pool.push_back(e.a);
    c->ev_pool.push_back(e.b);
  }
  c->ev_pending.clear();
}

template <typename F>
void timed(adef2_ctx* c, int id, double bytes, F&& launch) {
  if (!c->o.profile) { launch(); return; }
  hipEvent_t a = ev_get(c), b = ev_get(c);
  hipEventRecord(a, c->st);
  launch();
  hipEventRecord(b, c->st);
  c->ev_pending.push_back({id, a, b, bytes});
  if (c->ev_pending.size() >= 2048) ev_harvest(c);
}

// ------------------------------------------------------------ kernel tables
// precision modes: vectors FP64 unless FP32_REFINE; operator values and Z/W
// panels FP64 only in FP64 mode
inline bool vec64(int prec) { return prec != ADEF2_FP32_REFINE; }
inline bool mat64(int prec) { return prec == ADEF2_FP64 || prec == ADEF2_FP64_REFINE; }

template <typename V, typename M>
KTab<V, M> pick(int KP, int rpt) {
  if (rpt == 2) return pick_kp<V, M, 2>(KP);
  return pick_kp<V, M, 1>(KP);
}

template <int RPT>
void (*pick_resid(void))(ResidArgs) { return k_resid64<RPT>; }

void (*resid_fn(int rpt))(ResidArgs) {
  if (rpt == 2) return k_resid64<2>;
  return k_resid64<1>;
}
template <typename VM, typename VI, typename VO>
void (*stencil1_fn(int rpt))(OpGeom, const VM*, const VI*, VO*, int64_t, const Inst*, int) {
  if (rpt == 2) return k_stencil1<VM, VI, VO, 2>;
  return k_stencil1<VM, VI, VO, 1>;
}

template <typename V>
void (*accum_fn(int rpt))(OpGeom, const uint8_t*, const V*, double*, int64_t, Inst*) {
  if (rpt == 2) return k_accumulate<V, 2>;
  return k_accumulate<V, 1>;
}

template <typename V>
void launch_gram(adef2_ctx* c, const V* dummy_tag, V* W) {
  (void)dummy_tag;
  OpGeom og = op_geom(c);
  dim3 grid(c->gram_blocks, c->B);
  int nsub = 0;
#define GRAM_CASE(KPV)                                                                       \
  case KPV:                                                                                  \
    nsub = (int)cdiv(c->N, GramCfg<KPV>::GR);                                                \
    hipLaunchKernelGGL((k_spmm_gram<V, KPV>), grid, dim3(TPB), 0, c->st, og, c->dia64, c->Z64, \
                       c->zs, c->Tm, (int)c->factored, c->masks, W, c->inst, c->part, c->ctr,        \
                       c->g_gram, c->gram, nsub, c->mu64, c->eigf, c->ne);                   \
    break;
  switch (c->KP) {
    GRAM_CASE(8) GRAM_CASE(16) GRAM_CASE(24) GRAM_CASE(32) GRAM_CASE(40) GRAM_CASE(48)
    GRAM_CASE(56) GRAM_CASE(64)
    default: break;
  }
#undef GRAM_CASE
}

void launch_coarse(adef2_ctx* c) {
  CoarseArgs ca{};
  ca.gram = c->gram;
  ca.C = c->C;
  ca.Finfo = c->Finfo;
  ca.kept = c->kept;
  ca.inst = c->inst;
  ca.k = c->k;
  // with FP32 panels the part of a column orthogonal to the earlier ones
  // carries the FP32 rounding of the whole column amplified by 1/|R_jj|: keep
  // only columns whose independent part is at least FP32_DROP of their norm
  ca.drop_rel = mat64(c->prec) ? c->o.drop_rel : std::max(c->o.drop_rel, FP32_DROP);
  ca.tau_cond = c->o.tau_cond;
  ca.k_base = c->k_base;
  ca.ritz_keep = c->o.ritz_keep;
  ca.k_safe = c->k_safe;
  ca.tau_safe = c->tau_safe;
  ca.tau_dep = c->o.tau_dep;
  // with FP32 panels the coarse solve errs by ~u32 cond(E): cap the learned
  // basis' bound so that this stays below 1e-3
  ca.tau_learned = mat64(c->prec) ? c->tau_learned : std::min(c->tau_learned, FP32_COND);
#define COARSE_CASE(KPV) \
  case KPV: hipLaunchKernelGGL((k_coarse<KPV>), dim3(c->B), dim3(TPB), 0, c->st, ca); break;
  switch (c->KP) {
    COARSE_CASE(8) COARSE_CASE(16) COARSE_CASE(24) COARSE_CASE(32) COARSE_CASE(40)
    COARSE_CASE(48) COARSE_CASE(56) COARSE_CASE(64)
    default: break;
  }
#undef COARSE_CASE
}

// -------------------------------------------------------- buffer management
// Tile geometry of the streaming kernels for rpt rows per thread (the
// reduction scratch is sized for rpt = 1, the largest tile count).
// Tile heights of the fused operator pass: 2, 4 and 8 times the reach Ho of
// the outer stencil, rounded up to 256 rows (the LDS halo adds Ho / R on
// each side of inner-stencil work), kept while the tile and its halo fit
// 64 KiB of LDS.  None for an assembled operator; none for a 3D grid, whose
// reach is a whole plane.  The default (op_fused = 1 with nothing tuned) is
// the middle candidate that applies.
int opf_halo(const adef2_ctx* c) {
  int ho = 0;
  for (int o : c->offs) ho = std::max(ho, std::abs(o));
  return ho;
}

std::vector<int> opf_candidates(const adef2_ctx* c) {
  std::vector<int> r;
  if (!c->factored || c->D1 == 0) return r;
  const int64_t ho = opf_halo(c);
  for (int64_t f : {2, 4, 8}) {
    const int64_t R = std::max<int64_t>(256, cdiv(f * ho, (int64_t)256) * 256);
    if ((R + 2 * ho) * 8 <= 64 * 1024 && (r.empty() || r.back() != R)) r.push_back((int)R);
  }
  return r;
}

int opf_default_rows(const adef2_ctx* c) {
  const std::vector<int> r = opf_candidates(c);
  return r.empty() ? 0 : r[r.size() / 2];
}

// opf: rows of the fused operator pass's tiles (0 = two passes); opg: its
// instances per block
void set_variant(adef2_ctx* c, int rpt, int wfree, int opf = 0, int opg = 1, int uws = 0) {
  c->rpt = rpt;
  c->wfree = wfree;
  c->of_rows = opf;
  c->opf = c->of_rows > 0;
  c->opg = c->opf ? opg : 1;
  c->of_halo = c->opf ? opf_halo(c) : 0;
  c->of_ntiles = c->opf ? (int)cdiv(c->N, (int64_t)c->of_rows) : 0;
  c->of_ntiles_pad = (int)cdiv(c->of_ntiles, 8) * 8;
  c->g_of = make_geom(std::max(c->of_ntiles_pad, 8));
  c->ntiles = (int)cdiv(c->N, (int64_t)IPB * rpt);
  c->ntiles_pad = (int)cdiv(c->ntiles, 8) * 8;
  c->g_iter = make_geom(c->ntiles_pad);
  c->bt_ntiles = (int)cdiv(c->N, (int64_t)BT_ROWS);
  c->bt_ntiles_pad = (int)cdiv(c->bt_ntiles, 8) * 8;
  c->bt_nblk_pad = (int)cdiv(cdiv(c->bt_ntiles, BT_TPB), 8) * 8;
  c->g_bt = make_geom(c->bt_nblk_pad);
  c->ub_ntiles = (int)cdiv(c->N, (int64_t)UB_ROWS);
  c->ub_ntiles_pad = (int)cdiv(c->ub_ntiles, 8) * 8;
  c->g_ub = make_geom(c->ub_ntiles_pad);
  // warp-specialised update: runs of ws_T tiles, the smallest power of two
  // that keeps the grid within two 512-thread blocks per CU
  c->uws = uws;
  const int per = c->ub_ntiles_pad / 8, ng = (int)cdiv(std::max(c->B, 1), UB_G);
  c->ws_T = 1;
  while (c->ws_T < per && 8 * ng * cdiv(per, c->ws_T) > 512) c->ws_T *= 2;
  c->ws_cpx = (int)cdiv(per, c->ws_T);
}

// partial sums per instance that k_finish_tm adds
int fin_leaves(const adef2_ctx* c) { return c->uws ? 8 * c->ws_cpx : c->ub_ntiles_pad; }

template <typename V>
void fill(adef2_ctx* c, V* p, size_t n, V v);

int ensure_batch(adef2_ctx* c, int B, int prec) {
  const int64_t N = c->N;
  const int KP = c->KP;
  set_variant(c, (c->o.rows_per_thread >= 2) ? c->o.rows_per_thread : 1, c->o.w_mode >= 2 ? c->o.w_mode - 1 : 0);
  const int64_t nsub_max = cdiv(N, 32);
  int gb = (int)std::max<int64_t>(8, std::min<int64_t>(256, 2048 / std::max(B, 1)));
  gb = (int)std::min<int64_t>(gb, nsub_max);
  c->gram_blocks = std::max(gb, 1);
  c->g_gram = make_geom(c->gram_blocks);
  const bool same = (B <= c->Bcap) && (prec == c->prec) && c->vs == N + 2 * c->H && KP == c->KPalloc;
  c->B = B;
  if (same) return ADEF2_OK;
  int rc;
  c->Bcap = B;
  c->KPalloc = KP;
  c->prec = prec;
  c->vs = N + 2 * c->H;
  const size_t BN = (size_t)B * N;
  const size_t BV = (size_t)B * c->vs;
  const int nchunks = (int)cdiv(N, CMP_CHUNK);
  if ((rc = dalloc(c, &c->masks, BN))) return rc;
  if ((rc = dalloc(c, &c->I, BN))) return rc;
  if ((rc = dalloc(c, &c->g2l, BN))) return rc;
  if ((rc = dalloc(c, &c->ccount, (size_t)B * nchunks))) return rc;
  if ((rc = dalloc(c, &c->cofs, (size_t)B * nchunks))) return rc;
  if ((rc = dalloc(c, &c->ntot, (size_t)B))) return rc;
  if ((rc = dalloc(c, &c->inst, (size_t)B))) return rc;
  if (c->inst_h) hipHostFree(c->inst_h);
  c->inst_h = nullptr;
  HIPCHK(c, hipHostMalloc((void**)&c->inst_h, sizeof(Inst) * B));
  const size_t kk = (size_t)std::max(KP, 1) * std::max(KP, 1);
  if ((rc = dalloc(c, &c->C, (size_t)B * kk))) return rc;
  if ((rc = dalloc(c, &c->Finfo, (size_t)B * kk))) return rc;
  if ((rc = dalloc(c, &c->kept, (size_t)B * std::max(KP, 1)))) return rc;
  if ((rc = dalloc(c, &c->gram, (size_t)B * 2 * kk))) return rc;
  const bool v64 = vec64(prec), m64 = mat64(prec);
  for (int j = 0; j < 5; ++j) {
    if ((rc = dalloc(c, &c->v64[j], v64 ? BV : 0))) return rc;
    if ((rc = dalloc(c, &c->v32[j], v64 ? 0 : BV))) return rc;
  }
  if ((rc = dalloc(c, &c->W64, m64 ? BN * KP : 0))) return rc;
  if ((rc = dalloc(c, &c->W32, m64 ? 0 : BN * KP))) return rc;
  if ((rc = dalloc(c, &c->dinv64, v64 ? BN : 0))) return rc;
  if ((rc = dalloc(c, &c->dinv32, v64 ? 0 : BN))) return rc;
  if ((rc = dalloc(c, &c->x64, prec == ADEF2_FP64 ? 0 : BV))) return rc;
  if ((rc = dalloc(c, &c->r64, prec == ADEF2_FP64 ? 0 : BN))) return rc;
  if ((rc = dalloc(c, &c->x0pad, BV))) return rc;
  if ((rc = dalloc(c, &c->t64, c->factored ? BV : 0))) return rc;
  if ((rc = dalloc(c, &c->t32, (c->factored && !v64) ? BV : 0))) return rc;
  if ((rc = dalloc(c, &c->Tm, c->factored ? BN * KP : 0))) return rc;
  if ((rc = dalloc(c, &c->bnd, BN)) || (rc = dalloc(c, &c->hb, BN)) || (rc = dalloc(c, &c->zero64, 64)))
    return rc;
  if ((rc = dalloc(c, &c->ftot, (size_t)B * FIN_MAX_SLICES * (2 * KP + 2))) || (rc = dalloc(c, &c->fctr, (size_t)B + 16)))
    return rc;
  HIPCHK(c, hipMemsetAsync(c->fctr, 0, ((size_t)B + 16) * sizeof(unsigned), c->st));
  if ((rc = dalloc(c, &c->bcnt, (size_t)B * c->ub_ntiles)) ||
      (rc = dalloc(c, &c->btoff, (size_t)B * (c->ub_ntiles + 1))) || (rc = dalloc(c, &c->btot, 1)))
    return rc;
  fill<double>(c, c->zero64, 64, 0.0);
  // reduction scratch: enough for the iteration kernels (NV <= KP+2) and the
  // Gram kernel (NV = 2 KP^2); geometry is recomputed per call from B
  const size_t pi = (size_t)std::max(make_geom((int)cdiv(cdiv(N, IPB), 8) * 8).ptotal,
                                     make_geom((int)cdiv(cdiv(N, BT_ROWS), 8) * 8).ptotal) *
                    (2 * KP + 2);
  const size_t pg = (size_t)make_geom(256).ptotal * 2 * kk;
  c->part_elems = (size_t)B * std::max(pi, pg);
  c->ctr_elems = (size_t)B * std::max({make_geom((int)cdiv(cdiv(N, IPB), 8) * 8).ctotal,
                                       make_geom((int)cdiv(cdiv(N, BT_ROWS), 8) * 8).ctotal,
                                       make_geom(256).ctotal}) + 16;
  if ((rc = dalloc(c, &c->part, c->part_elems))) return rc;
  if ((rc = dalloc(c, &c->ctr, c->ctr_elems))) return rc;
  HIPCHK(c, hipMemsetAsync(c->ctr, 0, c->ctr_elems * sizeof(unsigned), c->st));
  return ADEF2_OK;
}

template <typename V>
void fill(adef2_ctx* c, V* p, size_t n, V v) {
  if (!p || n == 0) return;
  int blocks = (int)std::min<int64_t>(cdiv((int64_t)n, 256), 8192);
  hipLaunchKernelGGL((k_fill<V>), dim3(blocks), dim3(256), 0, c->st, p, (int64_t)n, v);
}

// restrict B instances whose masks are already in c->masks; a, c per instance
int restrict_batch(adef2_ctx* c, const double* a_h, const double* c_h) {
  const int B = c->B;
  const int64_t N = c->N;
  const int nchunks = (int)cdiv(N, CMP_CHUNK);
  // instance state
  for (int m = 0; m < B; ++m) {
    Inst& s = c->inst_h[m];
    std::memset(&s, 0, sizeof(Inst));
    const double ua = a_h ? a_h[m] : c->scale_a;
    const double uc = c_h ? c_h[m] : c->scale_c;
    if (!(ua > 0.0) || !std::isfinite(ua) || !std::isfinite(uc))
      return fail(c, ADEF2_E_ARG, "operator scale a must be > 0");
    // kernels apply S = s.a * (stencil) + s.c * I
    s.a = c->factored ? ua * c->alpha_ref : ua;
    s.c = c->factored ? ua * c->shift_ref + uc : uc;
    s.cond = 1.0;
  }
  HIPCHK(c, hipMemcpyAsync(c->inst, c->inst_h, sizeof(Inst) * B, hipMemcpyHostToDevice, c->st));
  // compaction
  timed(c, KI_COMPACT, (double)B * (2.0 * N + 8.0 * N), [&] {
    hipLaunchKernelGGL(k_compact_count, dim3(nchunks, B), dim3(TPB), 0, c->st, N, c->masks,
                       c->ccount, nchunks);
    hipLaunchKernelGGL(k_compact_scan, dim3(B), dim3(TPB), 0, c->st, c->ccount, c->cofs, nchunks,
                       c->ntot, c->inst);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nchunks, B), dim3(TPB), 0, c->st, N, c->masks,
                       c->cofs, nchunks, c->I, c->g2l);
  });
  // preconditioner and zeroed vectors
  dim3 g1((unsigned)cdiv(N, 256), B);
  const size_t BV = (size_t)B * c->vs;
  if (c->prec != ADEF2_FP64) fill<double>(c, c->x64, BV, 0.0);
  if (vec64(c->prec)) {
    hipLaunchKernelGGL((k_dinv<double>), g1, dim3(256), 0, c->st, N, c->diag, c->masks, c->dinv64,
                       c->inst, c->o.precond == ADEF2_NONE);
    for (int j = 0; j < 5; ++j) fill<double>(c, c->v64[j], BV, 0.0);
  } else {
    hipLaunchKernelGGL((k_dinv<float>), g1, dim3(256), 0, c->st, N, c->diag, c->masks, c->dinv32,
                       c->inst, c->o.precond == ADEF2_NONE);
    for (int j = 0; j < 5; ++j) fill<float>(c, c->v32[j], BV, 0.0f);
    fill<double>(c, c->x64, BV, 0.0);
    fill<float>(c, c->t32, BV, 0.0f);
  }
  fill<double>(c, c->x0pad, BV, 0.0);
  fill<double>(c, c->t64, BV, 0.0);
  // boundary form of W: FP32 panels and reference modes that are eigenvectors
  // (w_boundary 1: the eigen columns; 2: only when every shared reference
  // mode is one, which also enables the tile-major boundary-form update)
  const bool wb = c->o.w_boundary == 1 || (c->o.w_boundary == 2 && c->zs == 0 && c->n_eig == c->k);
  c->ne = (c->KP > 0 && wb && !mat64(c->prec) && c->n_eig > 0) ? (c->zs ? c->k_base : c->k) : 0;
  c->tm_ok = c->ne > 0 && c->zs == 0 && c->n_eig == c->k && vec64(c->prec) && c->ZT32 != nullptr;
  c->nbnd = 0;
  if (c->ne > 0) {
    OpGeom og = op_geom(c);
    if (c->factored) {
      hipLaunchKernelGGL(k_bnd_inner, g1, dim3(256), 0, c->st, og, c->dia1_64, c->masks, c->hb);
      hipLaunchKernelGGL(k_bnd_outer, g1, dim3(256), 0, c->st, og, c->dia64, c->masks, c->hb, c->bnd);
    } else {
      hipLaunchKernelGGL(k_bnd_outer, g1, dim3(256), 0, c->st, og, c->dia64, c->masks, c->masks, c->bnd);
    }
  }
  // coarse space
  if (c->KP > 0) {
    const double wbytes = (mat64(c->prec) ? 8.0 : 4.0);
    timed(c, KI_GRAM, (double)B * N * (c->D * 8.0 + c->KP * (8.0 + wbytes) + 1.0), [&] {
      if (c->factored) {
        hipLaunchKernelGGL(k_stencil_modes, dim3((unsigned)cdiv(N, 256), c->KP, B), dim3(256), 0,
                           c->st, op_geom(c), c->dia1_64, c->Z64, c->zs, c->masks, c->KP, c->Tm);
      }
      if (mat64(c->prec)) launch_gram<double>(c, nullptr, c->W64);
      else launch_gram<float>(c, nullptr, c->W32);
    });
    timed(c, KI_COARSE, 0.0, [&] { launch_coarse(c); });
    if (c->tm_ok) {
      // boundary rows (W - Lambda Z != 0) compacted per instance and tile
      const dim3 gb((unsigned)c->ub_ntiles, B);
      hipLaunchKernelGGL(k_bnd_count, gb, dim3(UB_ROWS), 0, c->st, N, c->ub_ntiles, c->bnd, c->bcnt);
      hipLaunchKernelGGL(k_bnd_scan, dim3(1), dim3(1024), 0, c->st, B, c->ub_ntiles, c->bcnt, c->btoff,
                         c->btot);
      int tot = 0;
      HIPCHK(c, hipMemcpyAsync(&tot, c->btot, sizeof(int), hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
      if ((size_t)tot > c->bcap) {
        int rc;
        const size_t cap = (size_t)tot + tot / 4 + 1024;
        c->bcap = 0;
        if ((rc = dalloc(c, &c->bidx, cap)) || (rc = dalloc(c, &c->bW32, cap * c->KP))) return rc;
        c->bcap = cap;
      }
      c->nbnd = tot;
      if (tot > 0)
        hipLaunchKernelGGL((k_bnd_fill<float>), gb, dim3(UB_ROWS), 0, c->st, N, c->ub_ntiles, c->KP,
                           c->bnd, c->btoff, c->W32, c->bidx, c->bW32);
    }
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->inst_h, c->inst, sizeof(Inst) * B, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->restricted = true;
  c->nI_host.assign(B, 0);
  int worst = ADEF2_OK;
  for (int m = 0; m < B; ++m) {
    c->nI_host[m] = c->inst_h[m].n_inactive;
    const int s = c->inst_h[m].setup_status;
    if (s < 0) worst = std::min(worst, s);
    else if (worst >= 0) worst = std::max(worst, s);
  }
  if (worst == ADEF2_E_NOT_SPD) {
    c->restricted = false;
    return fail(c, ADEF2_E_NOT_SPD, "restricted operator has a non-positive diagonal entry");
  }
  return worst;
}

template <typename V, typename M>
IterArgs<V, M> iter_args(adef2_ctx* c) {
  IterArgs<V, M> a{};
  a.op = op_geom(c);
  a.mask = c->masks;
  a.inst = c->inst;
  a.C = c->C;
  a.part = c->part;
  a.ctr = c->ctr;
  a.g = c->g_iter;
  a.maxit = c->o.maxit;
  a.vs = c->vs;
  a.zs = c->zs;
  a.dia64 = c->dia64;
  a.dia1_64 = c->dia1_64;
  a.Z64 = c->Z64;
  a.kb = c->zs ? c->k_base : c->KP;
  a.mu = c->mu64;
  a.eig = c->eigf;
  a.bnd = c->bnd;
  a.ne = c->ne;
  a.wzero = (const M*)c->zero64;
  a.Zsh64 = c->zs ? c->Zsh64 : c->Z64;
  a.B = c->B;
  a.bt_ntiles = c->bt_ntiles;
  a.bt_ntiles_pad = c->bt_ntiles_pad;
  a.bt_nblk_pad = c->bt_nblk_pad;
  a.gbt = c->g_bt;
  a.ub_ntiles = c->ub_ntiles;
  a.ub_ntiles_pad = c->ub_ntiles_pad;
  a.ub_ngroups = (int)cdiv(c->B, UB_G);
  a.pb_ngroups = (int)cdiv(c->B, PB_G);
  a.sg_ngroups = (int)cdiv(c->B, SG_G);
  a.gub = c->g_ub;
  a.diag = c->diag;
  a.precond_none = c->o.precond == ADEF2_NONE;
  a.btoff = c->btoff;
  a.bidx = c->bidx;
  a.ftot = c->ftot;
  a.fctr = c->fctr;
  a.fin_leaves = fin_leaves(c);
  a.ws_T = c->ws_T;
  a.ws_cpx = c->ws_cpx;
  a.of_rows = c->of_rows;
  a.of_halo = c->of_halo;
  a.of_ntiles = c->of_ntiles;
  a.of_ntiles_pad = c->of_ntiles_pad;
  a.of_ngroups = (int)cdiv(c->B, c->opg);
  a.gof = c->g_of;
  if constexpr (sizeof(M) == 8) {
    a.ZT = nullptr;
    a.bW = nullptr;
  } else {
    a.ZT = (const M*)c->ZT32;
    a.bW = (const M*)c->bW32;
  }
  if constexpr (sizeof(M) == 8) {
    a.dia1 = (const M*)c->dia1_64;
    a.dia = (const M*)c->dia64;
    a.Z = (const M*)c->Z64;
    a.W = (const M*)c->W64;
    a.Zsh = (const M*)(c->zs ? c->Zsh64 : c->Z64);
  } else {
    a.dia1 = (const M*)c->dia1_32;
    a.dia = (const M*)c->dia32;
    a.Z = (const M*)c->Z32;
    a.W = (const M*)c->W32;
    a.Zsh = (const M*)(c->zs ? c->Zsh32 : c->Z32);
  }
  if constexpr (sizeof(V) == 8) {
    a.t = (V*)interior(c, c->t64);
    a.dinv = (const V*)c->dinv64;
    a.x = (V*)interior(c, c->v64[0]); a.r = (V*)interior(c, c->v64[1]);
    a.z = (V*)interior(c, c->v64[2]); a.p = (V*)interior(c, c->v64[3]);
    a.w = (V*)interior(c, c->v64[4]);
  } else {
    a.t = (V*)interior(c, c->t32);
    a.dinv = (const V*)c->dinv32;
    a.x = (V*)interior(c, c->v32[0]); a.r = (V*)interior(c, c->v32[1]);
    a.z = (V*)interior(c, c->v32[2]); a.p = (V*)interior(c, c->v32[3]);
    a.w = (V*)interior(c, c->v32[4]);
  }
  return a;
}

// algorithmic bytes per launch (per instance: inactive rows only); wv / wm =
// bytes per vector entry / per operator or panel entry
struct ByteModel { double init, init2, pupdate, stencil, spmv, update, resid, accum, update_nw, zproj, update_tm,
                   finish_tm, opfused; };
// Algorithmic bytes per launch.  Per-instance data (vectors, W, the mask) is
// counted for every instance still iterating at the last poll (a finished
// instance's blocks exit at their first instruction); operands shared by
// all instances (Z, the stencil coefficients) are counted once per launch,
// over min(N, total inactive rows) rows for Z and the outer stencil and N
// rows for the inner stencil of the factored operator.
ByteModel byte_model(const adef2_ctx* c, double wv, double wm, bool sweep_active = true) {
  const double k = c->KP > 0 ? (double)c->k : 0.0;
  double nI = 0.0;
  int nact = 0;
  for (int m = 0; m < c->B; ++m) {
    const Inst& s = c->inst_h[m];
    const bool act = sweep_active ? !(s.done || s.outer_done) : !s.outer_done;
    if (act && m < (int)c->nI_host.size()) { nI += (double)c->nI_host[m]; ++nact; }
  }
  ByteModel b{};
  if (nact == 0) return b;
  const double N1 = (double)c->N;
  const double Nall = N1 * nact;                     // mask bytes, inner-stencil rows
  const double U = std::min(N1, nI);                 // rows of shared operands used
  // Z: shared; with a per-instance basis only the columns past k_base are per instance
  const double kb = c->zs ? (double)c->k_base : k;
  const double zsh = (U * kb + (c->zs ? nI * (k - kb) : 0.0)) * wm;
  const double D = c->D, D1 = c->D1;
  b.init = nI * (8.0 + 2 * wv) + zsh + Nall;                   // src -> x, r; Z^T r
  b.init2 = nI * (k * wm + 6 * wv) + zsh + Nall;               // W c0, x r z dinv
  b.pupdate = nI * 3 * wv + zsh + Nall;                        // z, p -> p; Z c
  const double outer = nI * 3 * wv + U * D * wm + Nall;        // t (or p), p -> w; A^T or S
  const double inner = c->factored ? (Nall * 2 * wv + N1 * D1 * wm) : 0.0;   // t = A v
  b.stencil = inner;
  b.spmv = outer;
  // fused pass: p on all rows (the inner stencil's source), the mask, w on
  // the inactive rows, both stencils' coefficients once; t stays in LDS
  b.opfused = Nall * wv + nI * wv + Nall + N1 * D1 * wm + U * D * wm;
  b.update = nI * (k * wm + 8 * wv) + zsh + Nall;              // W, Z; x p r w dinv -> x r z
  b.update_nw = nI * 8 * wv + Nall;                            // x p r w dinv -> x r z
  // x p r w -> x r z; the Jacobi scaling from the shared diagonal (N rows once);
  // Z once (row-major copy); the boundary rows' list entries
  b.update_tm = nI * 7 * wv + Nall + N1 * 8.0 + zsh + (double)c->nbnd * (4.0 + k * wm);
  // tile partial sums of the iterating instances, the slice totals written and read back
  const double nv = 2.0 * (double)c->KP + 2.0;
  b.finish_tm = (double)nact * nv * 8.0 * ((double)fin_leaves(c) + 2.0 * fin_slices(fin_leaves(c)));
  // (t = A z), z, r; Z^T u, Z^T r with the FP64 operator and modes
  const double inner64 = c->factored ? (Nall * 2 * wv + N1 * D1 * 8.0) : 0.0;
  b.zproj = inner64 + nI * 3 * wv + U * D * 8.0 + zsh * (8.0 / wm) + Nall;
  if (c->factored)
    b.resid = Nall * 16.0 + N1 * D1 * 8.0 + nI * 8.0 * 4 + U * D * 8.0 + Nall;
  else
    b.resid = nI * 8.0 * 3 + U * D * 8.0 + Nall;
  b.accum = nI * (wv + 16.0) + Nall;
  return b;
}

int poll(adef2_ctx* c, bool outer, bool* all_done) {
  c->st_polls += 1;
  HIPCHK(c, hipMemcpyAsync(c->inst_h, c->inst, sizeof(Inst) * c->B, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  bool ad = true;
  for (int m = 0; m < c->B; ++m) {
    const Inst& s = c->inst_h[m];
    if (outer ? !s.outer_done : !(s.done || s.outer_done)) { ad = false; break; }
  }
  *all_done = ad;
  return ADEF2_OK;
}

// FP64 outer residual r64 = b - S_II x (stored when store), its norm and the
// outer stopping rule (decide); trans_mode: only instances whose sweep has
// ended (sweep transitions inside a chunk)
ResidArgs resid_args(const adef2_ctx* c, const double* b, const double* xpad, int first, int decide, bool store,
                     int trans_mode) {
  ResidArgs ra{};
  ra.op = op_geom(c);
  ra.dia = c->dia64;
  ra.mask = c->masks;
  ra.b = b;
  ra.x = xpad;
  ra.sv = xpad;
  ra.vs = c->vs;
  ra.r64 = store ? c->r64 : nullptr;
  ra.inst = c->inst;
  ra.part = c->part;
  ra.ctr = c->ctr;
  ra.g = c->g_iter;
  ra.first = first;
  ra.decide = decide;
  ra.maxit = c->o.maxit;
  ra.max_sweeps = c->o.max_sweeps;
  ra.stall_steps = 4;
  ra.trans_mode = trans_mode;
  return ra;
}

// the residual kernel (after t = A x for the factored operator, stencil skip
// mode as in k_stencil1) on stream s
void launch_resid(adef2_ctx* c, ResidArgs ra, const double* xpad, hipStream_t s, int skip) {
  if (c->factored) {
    hipLaunchKernelGGL((stencil1_fn<double, double, double>(c->rpt)), dim3(c->ntiles_pad * c->B), dim3(IPB), 0, s,
                       ra.op, c->dia1_64, xpad, interior(c, c->t64), c->vs, c->inst, skip);
    ra.sv = interior(c, c->t64);
  }
  hipLaunchKernelGGL(resid_fn(c->rpt), dim3(c->ntiles_pad * c->B), dim3(IPB), 0, s, ra);
}

// run one A-DEF2 sweep in precision V for all instances: init, init2, then
// chunks of iterations until every instance's sweep is done
// Instantiated graph of one chunk of iterations for these kernel arguments:
// captured on the private stream the first time, then reused while the
// arguments (buffers, geometry, variant) are unchanged.  Up to 24
// configurations are kept per context.
template <typename V, typename M, typename F>
int chunk_graph(adef2_ctx* c, const IterArgs<V, M>& a, int chunk, int variant, const void* tag, F&& launch_chunk,
                hipGraphExec_t* out) {
  std::vector<char> key(sizeof(a) + 4 * sizeof(int) + sizeof(tag));
  std::memcpy(key.data(), &a, sizeof(a));
  const int extra[4] = {(int)sizeof(V), (int)sizeof(M), chunk, variant * 16 + c->rpt};
  std::memcpy(key.data() + sizeof(a), extra, sizeof(extra));
  std::memcpy(key.data() + sizeof(a) + sizeof(extra), &tag, sizeof(tag));
  for (auto& g : c->graphs)
    if (g.key == key) { *out = g.exec; return ADEF2_OK; }
  if (!c->gst) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->gev_in, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->gev_out, hipEventDisableTiming));
  }
  hipGraph_t graph = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal));
  launch_chunk(c->gst);
  const hipError_t ce = hipStreamEndCapture(c->gst, &graph);
  if (ce != hipSuccess) return fail(c, ADEF2_E_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(c, ADEF2_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
  if (c->graphs.size() >= 24) {
    hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({key, exec});
  *out = exec;
  return ADEF2_OK;
}

// max_chunks > 0 stops after that many chunks (tuning trials).
template <typename V, typename M>
// b_outer != null: refinement with sweep transitions inside the chunks (each
// instance starts its next sweep at the end of the chunk in which its sweep
// ended; x64 accumulates the corrections; the run ends when every instance
// meets the outer test), b_outer being the right-hand side of the solve
int run_sweep(adef2_ctx* c, const double* src, const double* x0pad, double thresh_scale, int rel_tol,
              double thresh_floor, int carry_dir, int max_chunks = 0, const double* b_outer = nullptr) {
  // tile-major boundary-form kernels (w_mode 4): shared eigen-basis, FP64 vectors
  const bool tm = (c->wfree == 3 || c->wfree == 4) && c->KP > 0 && sizeof(V) == 8 && c->tm_ok;
  const bool wfree = (c->wfree == 1 || c->wfree == 2) && c->KP > 0 && sizeof(V) == 8;
  // tile-major kernels (w_mode 2) need the basis shared by all instances
  const bool bt = wfree && c->wfree == 1 && c->zs == 0;
  const dim3 gbt(c->bt_ntiles_pad);
  const dim3 gpt((unsigned)(c->ub_ntiles_pad * cdiv(c->B, PB_G)));
  const dim3 gut((unsigned)(c->ub_ntiles_pad * cdiv(c->B, UB_G)));
  const dim3 gfin((unsigned)cdiv(2 * c->KP + 2, FC), (unsigned)fin_slices(fin_leaves(c)), (unsigned)c->B);
  const dim3 gws((unsigned)(8 * cdiv(c->B, UB_G) * c->ws_cpx));
  // tile-major stencil passes: coefficients of a row held in registers
  const bool stm = tm && c->wfree == 4 && c->D <= SDR && (!c->factored || c->D1 <= SDR);
  const dim3 gst((unsigned)(c->ub_ntiles_pad * cdiv(c->B, SG_G)));
  // fused operator pass: one block per (fused tile, instance), or per
  // (fused tile, group of 4 instances), A p in LDS
  const dim3 gof((unsigned)(c->of_ntiles_pad * cdiv(c->B, c->opg)));
  const size_t of_lds = (size_t)c->opg * (c->of_rows + 2 * c->of_halo) * sizeof(double);
  // five-point stencils (2D grids) with the diagonal count known at compile time
  auto opk = (c->D == 5 && c->D1 == 5) ? (c->opg == 4 ? k_opfused_g<V, M, 5, 4> : k_opfused<V, M, 5>)
                                       : k_opfused<V, M, 0>;
  // four LDS copies of up to 64 KiB together, plus the kernel's static LDS:
  // above the default per-launch bound
  if (c->opf) HIPCHK(c, hipFuncSetAttribute((const void*)opk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)of_lds));
  IterArgs<V, M> a = iter_args<V, M>(c);
  a.src = src;
  a.x0 = x0pad;
  a.x0s = c->vs;
  a.thresh_scale = thresh_scale;
  a.thresh_rel_tol = rel_tol;
  a.thresh_floor = thresh_floor;
  a.carry_dir = carry_dir;
  // segment cap: explicit (> 0), none (< 0), or by precision (0): FP32
  // vectors drift from the FP64 residual and need periodic replacement, FP64
  // vectors do not (forced replacements perturb CG near the accuracy floor)
  const int sm = c->o.segment_maxit;
  a.seg_maxit = (c->prec == ADEF2_FP64) ? 0 : (sm > 0 ? sm : (sm == 0 && !vec64(c->prec) ? 1000 : 0));
  KTab<V, M> kt = pick<V, M>(c->KP, c->rpt);
  BtTab<M> btt{};
  if constexpr (sizeof(V) == 8)
    if (bt || tm) btt = pick_bt<M>(c->KP);
  dim3 grid(c->ntiles_pad * c->B), blk(IPB);
  ByteModel bm = byte_model(c, (double)sizeof(V), (double)sizeof(M), false);
  const OpGeom og = a.op;
  auto st1 = stencil1_fn<M, V, V>(c->rpt);
  a.x0sv = x0pad;
  if (x0pad && c->factored) {
    // S x0 needs t = A x0 first (FP64 warm start, FP64 sweeps only)
    hipLaunchKernelGGL((stencil1_fn<double, double, double>(c->rpt)), grid, blk, 0, c->st, og,
                       c->dia1_64, x0pad, interior(c, c->t64), c->vs, c->inst, 2);
    a.x0sv = interior(c, c->t64);
  }
  timed(c, KI_INIT, bm.init, [&] { hipLaunchKernelGGL(kt.init, grid, blk, 0, c->st, a); });
  timed(c, KI_INIT2, bm.init2, [&] { hipLaunchKernelGGL(kt.init2, grid, blk, 0, c->st, a); });
  HIPCHK(c, hipGetLastError());
  // sweep transitions: the next sweep's init and init2 carry the direction
  // over and touch only the instances whose sweep has ended
  IterArgs<V, M> at = a;
  at.carry_dir = 1;
  at.trans_mode = 1;
  const ResidArgs ra_t = resid_args(c, b_outer, interior(c, c->x64), 0, 1, true, 1);
  const ByteModel bm64 = byte_model(c, 8.0, 8.0, false);
  const int chunk = std::max(1, c->o.check_every);
  // one chunk of iterations on stream s (kernel arguments are the same for
  // every iteration: all per-iteration state lives in device memory)
  auto launch_chunk = [&](hipStream_t s) {
    for (int it = 0; it < chunk; ++it) {
      if constexpr (sizeof(V) == 8) {
        if (tm)
          timed(c, KI_PUPDATE_TM, bm.pupdate,
                [&] { hipLaunchKernelGGL(btt.pupdate_tm, gpt, dim3(UB_THREADS), 0, s, a); });
        else if (bt)
          timed(c, KI_PUPDATE_BT, bm.pupdate,
                [&] { hipLaunchKernelGGL(btt.pupdate_bt, gbt, dim3(BT_THREADS), 0, s, a); });
      }
      if (!tm && !bt)
        timed(c, KI_PUPDATE, bm.pupdate, [&] { hipLaunchKernelGGL(kt.pupdate, grid, blk, 0, s, a); });
      if (c->opf)
        timed(c, KI_OPFUSED, bm.opfused,
              [&] { hipLaunchKernelGGL(opk, gof, blk, of_lds, s, a); });
      if (c->factored && !c->opf)
        timed(c, KI_STENCIL, bm.stencil, [&] {
          if constexpr (sizeof(V) == 8)
            if (stm) hipLaunchKernelGGL(btt.stencil1_tm, gst, dim3(UB_THREADS), 0, s, a);
          if (!stm)
            hipLaunchKernelGGL(st1, grid, blk, 0, s, og, a.dia1, (const V*)a.p, a.t, c->vs, c->inst, 1);
        });
      if (!c->opf) timed(c, KI_SPMV, bm.spmv, [&] {
        if constexpr (sizeof(V) == 8) {
          if (stm) {
            hipLaunchKernelGGL(btt.spmv_tm, gst, dim3(UB_THREADS), 0, s, a);
            hipLaunchKernelGGL(btt.alpha_tm, dim3((unsigned)c->B), dim3(UB_THREADS), 0, s, a);
          }
        }
        if (!stm) hipLaunchKernelGGL(kt.spmv, grid, blk, 0, s, a);
      });
      if (tm) {
        if constexpr (sizeof(V) == 8)
        {
          timed(c, KI_UPDATE_TM, bm.update_tm, [&] {
            if (c->uws) hipLaunchKernelGGL(btt.update_ws, gws, dim3(WS_THREADS), 0, s, a);
            else hipLaunchKernelGGL(btt.update_tm, gut, dim3(UB_THREADS), 0, s, a);
          });
          timed(c, KI_FINISH_TM, bm.finish_tm,
                [&] { hipLaunchKernelGGL(btt.finish_tm, gfin, dim3(UB_THREADS), 0, s, a); });
        }
      } else if (!wfree) {
        timed(c, KI_UPDATE, bm.update, [&] {
          hipLaunchKernelGGL((c->ne > 0 ? kt.update_spec : kt.update), grid, blk, 0, s, a);
        });
      } else {
        timed(c, KI_UPDATE_NW, bm.update_nw,
              [&] { hipLaunchKernelGGL(kt.update_nw, grid, blk, 0, s, a); });
        timed(c, bt ? KI_ZPROJ_BT : KI_ZPROJ, bm.zproj, [&] {
          if (c->factored)
            hipLaunchKernelGGL((stencil1_fn<double, V, V>(c->rpt)), grid, blk, 0, s, og, c->dia1_64,
                               (const V*)a.z, a.t, c->vs, c->inst, 1);
          if (bt) {
            if constexpr (sizeof(V) == 8)
              hipLaunchKernelGGL(btt.zproj_bt, dim3(c->bt_nblk_pad), dim3(BT_THREADS), 0, s, a);
          } else
            hipLaunchKernelGGL(kt.zproj, grid, blk, 0, s, a);
        });
      }
    }
    if (b_outer) {
      // instances whose sweep ended in this chunk: the correction into x64,
      // the FP64 residual and the outer test, then the next sweep's set-up
      timed(c, KI_ACCUM, bm.accum, [&] {
        hipLaunchKernelGGL(accum_fn<V>(c->rpt), grid, blk, 0, s, og, c->masks, (const V*)a.x,
                           interior(c, c->x64), c->vs, c->inst);
      });
      timed(c, KI_RESID, bm64.resid, [&] { launch_resid(c, ra_t, interior(c, c->x64), s, 3); });
      timed(c, KI_INIT, bm.init, [&] { hipLaunchKernelGGL(kt.init, grid, blk, 0, s, at); });
      timed(c, KI_INIT2, bm.init2, [&] { hipLaunchKernelGGL(kt.init2, grid, blk, 0, s, at); });
      hipLaunchKernelGGL(k_trans_clear, dim3((unsigned)cdiv(c->B, 64)), dim3(64), 0, s, c->inst, c->B);
    }
  };
  hipGraphExec_t gexec = nullptr;
  if (c->o.graph && !c->o.profile) {
    // the key names every choice that changes the launches: the W mode code
    // itself (w_mode 4 and 5 differ only in the stencil kernels), the
    // operator form and the boundary form
    int rc = chunk_graph<V, M>(c, a, chunk,
                               (c->uws << 13) | ((b_outer ? 1 : 0) << 12) | (c->opg << 9) | ((int)c->opf << 8) | (c->wfree << 4) |
                                   ((int)tm << 3) | ((int)bt << 2) | ((int)wfree << 1) | (c->ne > 0 ? 1 : 0),
                               b_outer, launch_chunk, &gexec);
    if (rc) return rc;
  }
  // Convergence is decided on the device (finished instances' blocks exit at
  // once); the host only has to notice that every instance is done.  Between
  // polls it enqueues as many chunks as the slowest instance is estimated to
  // still need: the decay of its squared residual since the last poll,
  // extrapolated to its threshold, halved for safety (CG's residual is not
  // monotone), at least one chunk, at most poll_max chunks.
  const int pmax = std::max(1, c->o.poll_max);
  std::vector<double> prev_rr(c->B, 0.0);
  std::vector<int> prev_it(c->B, -1);
  int64_t launched = 0;
  for (;;) {
    bool ad = false;
    int rc = poll(c, b_outer != nullptr, &ad);
    if (rc) return rc;
    if (ad) break;
    // every instance stops at maxit on the device; this guards the host loop
    if (launched > (int64_t)c->o.maxit + (int64_t)(pmax + 2) * chunk)
      return fail(c, ADEF2_E_HIP, "iteration kernels made no progress");
    double est = 0.0;
    for (int m = 0; m < c->B; ++m) {
      const Inst& s = c->inst_h[m];
      if (s.done || s.outer_done) continue;
      double rem = chunk;
      if (prev_it[m] >= 0 && s.sweep_iters > prev_it[m] && s.rr > 0.0 && prev_rr[m] > s.rr &&
          s.thresh2 > 0.0) {
        const double rate = std::log(prev_rr[m] / s.rr) / (double)(s.sweep_iters - prev_it[m]);
        rem = std::log(s.rr / s.thresh2) / rate;
      }
      rem = std::min(rem, (double)(c->o.maxit - s.iters));
      est = std::max(est, rem);
      prev_rr[m] = s.rr;
      prev_it[m] = s.sweep_iters;
    }
    // with sweep transitions the horizon is the outer test, which the sweep
    // residuals do not predict: poll_max chunks between polls
    int nrep = b_outer ? pmax : (int)std::min<double>((double)pmax, std::max(1.0, std::floor(0.5 * est / chunk)));
    if (max_chunks > 0) nrep = std::min<int64_t>(nrep, std::max<int64_t>(1, max_chunks - launched / chunk));
    for (int rep = 0; rep < nrep; ++rep) {
      launched += chunk;
      if (c->o.profile) bm = byte_model(c, (double)sizeof(V), (double)sizeof(M), true);
      if (gexec) {
        HIPCHK(c, hipEventRecord(c->gev_in, c->st));
        HIPCHK(c, hipStreamWaitEvent(c->gst, c->gev_in, 0));
        HIPCHK(c, hipGraphLaunch(gexec, c->gst));
        HIPCHK(c, hipEventRecord(c->gev_out, c->gst));
        HIPCHK(c, hipStreamWaitEvent(c->st, c->gev_out, 0));
      } else {
        launch_chunk(c->st);
      }
      HIPCHK(c, hipGetLastError());
    }
    if (max_chunks > 0 && launched >= (int64_t)max_chunks * chunk) break;
  }
  return ADEF2_OK;
}

int resid64(adef2_ctx* c, const double* b, const double* xpad, int first, int decide, bool store) {
  const ResidArgs ra = resid_args(c, b, xpad, first, decide, store, 0);
  const ByteModel bm = byte_model(c, 8.0, 8.0, false);
  timed(c, KI_RESID, bm.resid, [&] { launch_resid(c, ra, xpad, c->st, decide ? 2 : 0); });
  HIPCHK(c, hipGetLastError());
  return ADEF2_OK;
}

// reset per-solve state (keep restriction results)
int reset_solve_state(adef2_ctx* c) {
  for (int m = 0; m < c->B; ++m) {
    Inst& s = c->inst_h[m];
    s.iters = 0; s.sweep_iters = 0; s.done = 0; s.outer_done = 0; s.status = 0; s.sweeps = 0;
    s.has_dir = 0; s.rho_end = 0.0; s.stall = 0; s.rr64_best = INFINITY; s.drift = 0;
    s.capped = 0; s.trans = 0;
    s.rr = 0; s.rr64 = 0; s.bb64 = 0;
    const double t = m < (int)c->tol_h.size() ? c->tol_h[m] : 1e-8;
    s.tol2 = t * t;
  }
  HIPCHK(c, hipMemcpyAsync(c->inst, c->inst_h, sizeof(Inst) * c->B, hipMemcpyHostToDevice, c->st));
  return ADEF2_OK;
}

// Variant of the iteration kernels: rows per thread (tile height) and
// whether W is read each iteration.  Fixed by the options, or tuned once per
// (batch size, precision, basis width, operator form, N) on the first solve:
// every candidate runs the solve's first two chunks of iterations from the
// same start and the fastest is kept for this context, so repeated solves of
// one configuration use the same kernels (and give identical results).
int choose_variant(adef2_ctx* c, const double* b) {
  const int fr = c->o.rows_per_thread, fw = c->o.w_mode, fo = c->o.op_fused;
  if (fw >= 2 && !vec64(c->prec))
    return fail(c, ADEF2_E_UNSUPPORTED, "W-free iterations need FP64 vectors (FP64 or MIXED_REFINE)");
  std::vector<int> rpts = (fr == 1 || fr == 2) ? std::vector<int>{fr} : std::vector<int>{1, 2};
  const bool stm_ok = c->D <= SDR && (!c->factored || c->D1 <= SDR);
  if (fw == 5 && !stm_ok)
    return fail(c, ADEF2_E_UNSUPPORTED, "tile-major stencil passes need at most 16 diagonals");
  if ((fw == 4 || fw == 5) && !c->tm_ok)
    return fail(c, ADEF2_E_UNSUPPORTED,
                "the tile-major boundary-form update needs FP32 panels with FP64 vectors (MIXED_REFINE), "
                "reference modes shared by all instances that are eigenvectors of the reference operator, "
                "and w_boundary enabled");
  // fused operator pass: the (tile height, instances per block) candidates
  // the options allow; slot: where a candidate's trial time is reported
  const int64_t ho = opf_halo(c);
  const bool five = c->D == 5 && c->D1 == 5;
  auto fits = [&](int R, int G) {
    return c->factored && c->D1 > 0 && R >= 256 && R % 256 == 0 && (G == 1 || (G == 4 && five)) &&
           (int64_t)G * (R + 2 * ho) * 8 <= 64 * 1024;
  };
  struct OpC { int R, G, slot; };
  std::vector<OpC> opc;
  {
    const std::vector<int> Rs = c->o.op_rows > 0 ? std::vector<int>{c->o.op_rows} : opf_candidates(c);
    const std::vector<int> Gs = c->o.op_group > 0 ? std::vector<int>{c->o.op_group} : std::vector<int>{1, 4};
    for (size_t q = 0; q < Rs.size(); ++q)
      for (int G : Gs)
        if (fits(Rs[q], G) && (G == 1 || c->B > 1))
          opc.push_back({Rs[q], G, 1 + (G == 4 ? 3 : 0) + (int)std::min<size_t>(q, 2)});
  }
  // op_fused = 1: the given tile height and group, else 4 times the reach
  // (or the nearest candidate that fits) with one instance per block
  const int R1 = c->o.op_rows > 0 ? c->o.op_rows : opf_default_rows(c);
  const int G1 = c->o.op_group > 0 ? c->o.op_group : 1;
  if (fo == 1 && !fits(R1, G1))
    return fail(c, ADEF2_E_UNSUPPORTED,
                "the fused operator pass needs the factored operator with a stencil reach whose tile and "
                "halo fit 64 KiB of LDS (2D grids up to about 2000 points wide; 4 instances per block: "
                "five-point stencils and four such copies)");
  std::vector<int> wfs = (fw == 1 || c->KP == 0 || !vec64(c->prec)) ? std::vector<int>{0}
                         : (fw == 2 ? std::vector<int>{1}
                         : (fw == 3 ? std::vector<int>{2}
                         : (fw == 4 ? std::vector<int>{3}
                         : (fw == 5 ? std::vector<int>{4} : std::vector<int>{0, 1, 2}))));
  if (fw == 0 && c->tm_ok && c->KP > 0 && vec64(c->prec)) {
    wfs.push_back(3);
    if (stm_ok) wfs.push_back(4);
  }
  // operator form: fused (1) or two passes (0); tuned only when it applies
  // and the option leaves it open
  const bool tune_op = fo == 0 && !opc.empty();
  const int op0 = fo == 1 ? R1 : 0, og0 = fo == 1 ? G1 : 1;
  // update form of the tile-major path: per tile (k_update_tm) or
  // warp-specialised runs of tiles (k_update_ws, up to 32 modes)
  const int fu = c->o.update_ws;
  const bool ws_ok = c->tm_ok && c->KP > 0 && c->KP <= 32 && vec64(c->prec);
  if (fu == 1 && !ws_ok)
    return fail(c, ADEF2_E_UNSUPPORTED,
                "the warp-specialised update needs the tile-major boundary-form path with at most 32 modes");
  const bool tune_uw = fu == 0 && ws_ok;
  const int uw0 = fu == 1 ? 1 : 0;
  if (rpts.size() * wfs.size() == 1 && !tune_op && !tune_uw) {
    set_variant(c, rpts[0], wfs[0], op0, og0, uw0);
    return ADEF2_OK;
  }
  const int fact = c->factored ? 1 : 0;
  const int tmk = c->tm_ok ? 1 : 0;
  const int opo = fo + 4 * c->o.op_group + 32 * c->o.op_rows;   // the operator options tuned under
  for (const auto& t : c->tuned)
    if (t.B == c->B && t.prec == c->prec && t.KP == c->KP && t.fact == fact && t.tm == tmk &&
        t.N == c->N && t.opo == opo && t.uwo == fu && t.fro == fr && t.fwo == fw) {
      set_variant(c, t.rpt, t.wfree, t.opf, t.opg, t.uws);
      return ADEF2_OK;
    }
  const int prof = c->o.profile;
  c->o.profile = 0;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  adef2_ctx::Tuned best{c->B, c->prec, c->KP, fact, tmk, c->N, rpts[0], wfs[0], {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
                        opo, op0, og0, {0, 0, 0, 0, 0, 0, 0}, fu, uw0, {0, 0}, fr, fw};
  // one trial: the solve's first two chunks of iterations from the same start
  auto trial = [&](int rpt, int wf, int opf, int opg, int uws, float* ms) -> int {
    set_variant(c, rpt, wf, opf, opg, uws);
    int rc = reset_solve_state(c);
    if (rc) return rc;
    if (c->prec != ADEF2_FP64) {
      fill<double>(c, c->x64, (size_t)c->B * c->vs, 0.0);
      if ((rc = resid64(c, b, interior(c, c->x64), 1, 1, true))) return rc;
    }
    HIPCHK(c, hipEventRecord(e0, c->st));
    if (c->prec == ADEF2_FP64)
      rc = run_sweep<double, double>(c, b, nullptr, 1.0, 1, 0.0, 0, 2);
    else if (mat64(c->prec))
      rc = run_sweep<double, double>(c, c->r64, nullptr, 0.0, 0, 0.25, 0, 2);
    else if (vec64(c->prec))
      rc = run_sweep<double, float>(c, c->r64, nullptr, c->o.inner_rtol * c->o.inner_rtol, 0, 0.25, 0, 2);
    else
      rc = run_sweep<float, float>(c, c->r64, nullptr, c->o.inner_rtol * c->o.inner_rtol, 0, 0.25, 0, 2);
    if (rc) return rc;
    HIPCHK(c, hipEventRecord(e1, c->st));
    HIPCHK(c, hipEventSynchronize(e1));
    HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
    return ADEF2_OK;
  };
  float best_ms = INFINITY;
  int rc = ADEF2_OK, ci = 0;
  // stage 1: tile height and W mode, with the operator form the option fixes
  // (two passes while the form is tuned)
  for (int rpt : rpts) {
    for (int wf : wfs) {
      float ms = 0.0f;
      if ((rc = trial(rpt, wf, op0, og0, uw0, &ms))) break;
      best.ms[ci++] = ms;
      if (ms < best_ms) { best_ms = ms; best.rpt = rpt; best.wfree = wf; }
    }
    if (rc) break;
  }
  // stage 2: the fused operator pass at each candidate tile height, with
  // the winner of stage 1
  if (!rc && tune_op) {
    best.ms_op[0] = best_ms;
    for (size_t q = 0; q < opc.size() && !rc; ++q) {
      float ms = 0.0f;
      rc = trial(best.rpt, best.wfree, opc[q].R, opc[q].G, uw0, &ms);
      best.ms_op[opc[q].slot] = ms;
      if (!rc && ms < best_ms) { best_ms = ms; best.opf = opc[q].R; best.opg = opc[q].G; }
    }
  }
  // stage 3: the warp-specialised update, when the tile-major path won
  if (!rc && tune_uw && (best.wfree == 3 || best.wfree == 4)) {
    float ms = 0.0f;
    rc = trial(best.rpt, best.wfree, best.opf, best.opg, 1, &ms);
    best.ms_uw[0] = best_ms;
    best.ms_uw[1] = ms;
    if (!rc && ms < best_ms) { best_ms = ms; best.uws = 1; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->o.profile = prof;
  if (rc) return rc;
  c->tuned.push_back(best);
  set_variant(c, best.rpt, best.wfree, best.opf, best.opg, best.uws);
  return ADEF2_OK;
}

// Solve all B restricted instances; b, x instance-major unpadded [B][N].
// tols: host f64[B] per-instance tolerances, or null for tol everywhere
int solve_batch(adef2_ctx* c, const double* b, const double* x0, double tol, double* x,
                const double* tols = nullptr) {
  const int B = c->B;
  const int64_t N = c->N;
  c->tol_h.assign(B, tol);
  if (tols)
    for (int m = 0; m < B; ++m) c->tol_h[m] = tols[m];
  for (int m = 0; m < B; ++m)
    if (!(c->tol_h[m] > 0.0) || !std::isfinite(c->tol_h[m]))
      return fail(c, ADEF2_E_ARG, "tol must be positive and finite");
  int rc;
  if ((rc = choose_variant(c, b))) return rc;
  if ((rc = reset_solve_state(c))) return rc;
  dim3 gc((unsigned)cdiv(N, 256), B);
  const double* x0p = nullptr;
  if (x0) {
    // warm start restricted to the inactive set (zero on active rows)
    hipLaunchKernelGGL(k_mask_copy_padded, gc, dim3(256), 0, c->st, N, c->masks, x0,
                       interior(c, c->x0pad), c->vs);
    x0p = interior(c, c->x0pad);
  }
  double* xres = nullptr;
  if (c->prec == ADEF2_FP64) {
    if ((rc = run_sweep<double, double>(c, b, x0p, 1.0, 1, 0.0, 0))) return rc;
    xres = interior(c, c->v64[0]);
    if ((rc = resid64(c, b, xres, 1, 0, false))) return rc;
  } else {
    if (x0p) {
      HIPCHK(c, hipMemcpyAsync(c->x64, c->x0pad, sizeof(double) * (size_t)B * c->vs,
                               hipMemcpyDeviceToDevice, c->st));
    } else {
      fill<double>(c, c->x64, (size_t)B * c->vs, 0.0);
    }
    if ((rc = resid64(c, b, interior(c, c->x64), 1, 1, true))) return rc;
    const bool v64 = vec64(c->prec), m64 = mat64(c->prec);
    // FP64 segments run until their recurrence residual is below tol/2: an
    // FP64 recurrence stays close to the true residual over many orders of
    // magnitude, and every restart costs CG's accumulated Krylov space
    const double in2 = m64 ? 0.0 : c->o.inner_rtol * c->o.inner_rtol;
    const double mb = m64 ? 8.0 : 4.0;
    ByteModel bm = byte_model(c, v64 ? 8.0 : 4.0, mb, false);
    if (c->o.sweep_async) {
      // every instance moves to its next segment at the end of the chunk in
      // which its segment ended
      rc = m64 ? run_sweep<double, double>(c, c->r64, nullptr, in2, 0, 0.25, 0, 0, b)
               : v64 ? run_sweep<double, float>(c, c->r64, nullptr, in2, 0, 0.25, 0, 0, b)
                     : run_sweep<float, float>(c, c->r64, nullptr, in2, 0, 0.25, 0, 0, b);
      if (rc) return rc;
    }
    for (int sweep = 0; !c->o.sweep_async; ++sweep) {
      bool ad = false;
      if ((rc = poll(c, true, &ad))) return rc;
      if (ad) break;
      if (sweep > c->o.max_sweeps + 1) return fail(c, ADEF2_E_HIP, "refinement made no progress");
      bm = byte_model(c, v64 ? 8.0 : 4.0, mb, false);
      // segment on the correction equation S d = r64 (FP32 operator and
      // panels, or FP64 in FP64_REFINE); it ends when its recurrence
      // residual fell by inner_rtol (or below tol ||b|| / 2); the FP64
      // residual then replaces it and the search direction carries on
      rc = m64 ? run_sweep<double, double>(c, c->r64, nullptr, in2, 0, 0.25, sweep > 0)
               : v64 ? run_sweep<double, float>(c, c->r64, nullptr, in2, 0, 0.25, sweep > 0)
                     : run_sweep<float, float>(c, c->r64, nullptr, in2, 0, 0.25, sweep > 0);
      if (rc) return rc;
      timed(c, KI_ACCUM, bm.accum, [&] {
        if (v64)
          hipLaunchKernelGGL(accum_fn<double>(c->rpt), dim3(c->ntiles_pad * B), dim3(IPB), 0, c->st,
                             op_geom(c), c->masks, interior(c, c->v64[0]), interior(c, c->x64),
                             c->vs, c->inst);
        else
          hipLaunchKernelGGL(accum_fn<float>(c->rpt), dim3(c->ntiles_pad * B), dim3(IPB), 0, c->st,
                             op_geom(c), c->masks, interior(c, c->v32[0]), interior(c, c->x64),
                             c->vs, c->inst);
      });
      if ((rc = resid64(c, b, interior(c, c->x64), 0, 1, true))) return rc;
    }
    xres = interior(c, c->x64);
  }
  hipLaunchKernelGGL(k_scatter_out, gc, dim3(256), 0, c->st, N, c->masks, xres, c->vs, x, c->inst);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->inst_h, c->inst, sizeof(Inst) * B, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (c->o.profile) ev_harvest(c);
  c->solved = true;
  return ADEF2_OK;
}

int combine_status(const Inst& s) {
  if (s.status < 0) return s.status;
  if (s.setup_status < 0) return s.setup_status;
  return std::max(s.status, s.setup_status);
}

int worst_of(int a, int b) {
  if (a < 0 || b < 0) return std::min(a, b);
  return std::max(a, b);
}

bool valid_opts(const adef2_opts* o) {
  return o->maxit > 0 &&
         (o->precision == ADEF2_FP64 || o->precision == ADEF2_FP32_REFINE ||
          o->precision == ADEF2_MIXED_REFINE || o->precision == ADEF2_FP64_REFINE) &&
         (o->precond == ADEF2_JACOBI || o->precond == ADEF2_NONE) && o->inner_rtol > 0.0 &&
         o->inner_rtol < 1.0 && o->max_sweeps > 0 && o->drop_rel >= 0.0 && o->tau_cond > 0.0 &&
         (o->rows_per_thread == 0 || o->rows_per_thread == 1 || o->rows_per_thread == 2) &&
         o->w_mode >= 0 && o->w_mode <= 5 && o->w_boundary >= 0 && o->w_boundary <= 2 &&
         (o->graph == 0 || o->graph == 1) && o->ritz_keep >= 0 && o->ritz_keep <= ADEF2_MAX_K &&
         o->tau_safe >= 1.0 && o->tau_dep >= 0.0 && o->tau_dep < 1.0 && o->poll_max >= 1 &&
         (o->learned_objective == 0 || o->learned_objective == 1) &&
         (o->op_fused >= -1 && o->op_fused <= 1) && o->op_rows >= 0 && o->op_rows % 256 == 0 &&
         o->op_rows <= (1 << 16) && (o->op_group == 0 || o->op_group == 1 || o->op_group == 4) &&
         (o->sweep_async == 0 || o->sweep_async == 1) && o->update_ws >= -1 && o->update_ws <= 1;
}

}  // namespace

// Packed MLP parameter layout (FP32 master / BF16 copy share offsets)
constexpr int OW1 = 0, OB1 = OW1 + MD1 * MD0, OW2 = OB1 + MD1, OB2 = OW2 + MD2 * MD1,
              OW3 = OB2 + MD2, OB3 = OW3 + MD3 * MD2, NPARAM = OB3 + MD3;

MLPW mlp_view(const adef2_ctx* c) {
  MLPW w;
  w.W1 = c->mlp_bf + OW1; w.b1 = c->mlp + OB1;
  w.W2 = c->mlp_bf + OW2; w.b2 = c->mlp + OB2;
  w.W3 = c->mlp_bf + OW3; w.b3 = c->mlp + OB3;
  return w;
}

int ensure_mlp_batch(adef2_ctx* c, int M) {
  if (M <= c->Mcap_mlp) return ADEF2_OK;
  int rc;
  if ((rc = dalloc(c, &c->act, (size_t)M * 4 * MD1)) || (rc = dalloc(c, &c->mout, (size_t)M * MD3)) ||
      (rc = dalloc(c, &c->dout, (size_t)M * MD3)) || (rc = dalloc(c, &c->dA1, (size_t)M * MD1)) ||
      (rc = dalloc(c, &c->dA2, (size_t)M * MD2)) || (rc = dalloc(c, &c->lossv, (size_t)M)))
    return rc;
  c->Mcap_mlp = M;
  return ADEF2_OK;
}

void mlp_forward_launch(adef2_ctx* c, int M, const float* theta) {
  hipLaunchKernelGGL(k_mlp_fwd, dim3(M), dim3(512), 0, c->st, M, theta, mlp_view(c), c->act, c->mout);
}

// fwd + loss gradient + backward over the M prepared samples; gradient of the
// mean loss in c->mlp_g
void mlp_grad_launch(adef2_ctx* c, int M) {
  mlp_forward_launch(c, M, c->theta_tr);
  if (c->obj_tr == 1)
    hipLaunchKernelGGL(k_loss_grad_spec, dim3(M), dim3(512), 0, c->st, M, c->p, c->mout, c->Htr, c->Ntr,
                       1.0f / (float)M, c->dout, c->lossv);
  else
    hipLaunchKernelGGL(k_loss_grad, dim3(M), dim3(512), 0, c->st, M, c->p, c->mout, c->Htr, c->gtr, c->e0tr,
                       c->bxtr, 0.0, 1.0f / (float)M, c->dout, c->lossv);
  hipLaunchKernelGGL(k_mlp_bwd_act, dim3(M), dim3(128), 0, c->st, M, mlp_view(c), c->act, c->dout,
                     c->dA2, c->dA1);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)cdiv(MD3 * MD2, 256)), dim3(256), 0, c->st, M, MD3, MD2,
                     c->dout, MD3, c->act, 4 * MD1, 3 * MD1, c->mlp_g + OW3, c->mlp_g + OB3);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)cdiv(MD2 * MD1, 256)), dim3(256), 0, c->st, M, MD2, MD1,
                     c->dA2, MD2, c->act, 4 * MD1, MD1, c->mlp_g + OW2, c->mlp_g + OB2);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)cdiv(MD1 * MD0, 256)), dim3(256), 0, c->st, M, MD1, MD0,
                     c->dA1, MD1, c->theta_tr, MD0, 0, c->mlp_g + OW1, c->mlp_g + OB1);
}

// Swaps the shared reference basis for the per-instance enriched basis
// [Z | Phi C_m^T] for the duration of one batched solve.
struct BasisSwap {
  adef2_ctx* c;
  bool active = false;
  double* Z64s = nullptr;
  float* Z32s = nullptr;
  int k0 = 0, KP0 = 0;
  explicit BasisSwap(adef2_ctx* cc) : c(cc) {}
  int enrich(int B, const float* theta) {
    int rc;
    if ((rc = ensure_mlp_batch(c, B))) return rc;
    mlp_forward_launch(c, B, theta);
    const int k = c->k, KPe = round8(k + MLP_NV);
    const size_t need = (size_t)B * KPe * c->N;
    if (need > c->zb_cap) {
      c->zb_cap = 0;
      if ((rc = dalloc(c, &c->Zb64, need)) || (rc = dalloc(c, &c->Zb32, need))) return rc;
      c->zb_cap = need;
    }
    hipLaunchKernelGGL(k_expand_basis, dim3((unsigned)cdiv(c->N, 256), KPe, B), dim3(256), 0, c->st,
                       c->N, k, KPe, c->p, c->Z64, c->Phi, c->mout, c->Zb64, c->Zb32);
    HIPCHK(c, hipGetLastError());
    Z64s = c->Z64; Z32s = c->Z32; k0 = c->k; KP0 = c->KP;
    c->Zsh64 = c->Z64; c->Zsh32 = c->Z32;
    c->Z64 = c->Zb64; c->Z32 = c->Zb32;
    c->k_base = k;
    c->k = k + MLP_NV;
    c->KP = KPe;
    c->zs = (int64_t)KPe * c->N;
    active = true;
    return ADEF2_OK;
  }
  ~BasisSwap() {
    if (!active) return;
    c->Z64 = Z64s; c->Z32 = Z32s;
    c->Zsh64 = nullptr; c->Zsh32 = nullptr;
    c->k = k0; c->KP = KP0;
    c->k_base = 0;
    c->zs = 0;
  }
};

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

void adef2_default_opts(adef2_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tau_cond = 1e10;
  o->drop_rel = 1e-6;
  o->maxit = 100000;
  o->precision = ADEF2_FP64;
  o->precond = ADEF2_JACOBI;
  o->inner_rtol = 1e-2;
  o->max_sweeps = 2000;
  o->check_every = 32;
  o->segment_maxit = 0;
  o->rows_per_thread = 0;
  o->profile = 0;
  o->w_mode = 0;
  o->w_boundary = 2;
  o->graph = 1;
  o->ritz_keep = 0;
  o->tau_safe = 1e4;
  o->tau_dep = 1e-10;
  o->poll_max = 16;
  o->learned_objective = 0;
  o->op_fused = 0;
  o->op_rows = 0;
  o->op_group = 0;
  o->sweep_async = 1;
  o->update_ws = 0;
}

int adef2_create(adef2_ctx** out, const adef2_opts* opts, void* stream) {
  if (!out) { g_create_error = "null context pointer"; return ADEF2_E_ARG; }
  *out = nullptr;
  adef2_opts o;
  adef2_default_opts(&o);
  if (opts) o = *opts;
  if (!valid_opts(&o)) { g_create_error = "invalid options"; return ADEF2_E_ARG; }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { g_create_error = "no HIP device"; return ADEF2_E_HIP; }
  adef2_ctx* c = new adef2_ctx();
  c->o = o;
  c->st = (hipStream_t)stream;
  c->dev = dev;
  scratch_ptr(dev);          // the no-allocation entry point's scratch, once per device
  *out = c;
  return ADEF2_OK;
}

int adef2_destroy(adef2_ctx* c) {
  if (!c) return ADEF2_E_ARG;
  hipStreamSynchronize(c->st);
  free_all(c);
  delete c;
  return ADEF2_OK;
}

int adef2_set_opts(adef2_ctx* c, const adef2_opts* o) {
  if (!c || !o) return ADEF2_E_ARG;
  if (!valid_opts(o)) return fail(c, ADEF2_E_ARG, "invalid options");
  const bool prec_changed = o->precision != c->o.precision;
  const bool rpt_changed = o->rows_per_thread != c->o.rows_per_thread;
  const bool precond_changed = o->precond != c->o.precond;
  const bool coarse_changed = o->tau_cond != c->o.tau_cond || o->drop_rel != c->o.drop_rel ||
                              o->ritz_keep != c->o.ritz_keep;
  c->o = *o;
  if (prec_changed || rpt_changed || precond_changed || coarse_changed) c->restricted = false;
  return ADEF2_OK;
}

}  // extern "C"

namespace {

// CSR (device) -> diagonal format.  Finds the distinct column-row offsets on
// the device (flag array + compaction), then scatters the values.
// which = 0: assembled S (c->offs, c->dia64/32, c->diag); which = 1: factor A
// (c->offs1, c->dia1_64/32).
int load_dia(adef2_ctx* c, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
             const double* vals, int which) {
  const size_t nf = (size_t)(2 * n - 1);
  uint8_t* flags = nullptr;
  int* bad = nullptr;
  int* Iofs = nullptr;
  int* cnt = nullptr;
  int* ofs = nullptr;
  long long* tot = nullptr;
  const int nch = (int)cdiv((int64_t)nf, CMP_CHUNK);
  auto cleanup = [&] {
    if (flags) hipFree(flags);
    if (bad) hipFree(bad);
    if (Iofs) hipFree(Iofs);
    if (cnt) hipFree(cnt);
    if (ofs) hipFree(ofs);
    if (tot) hipFree(tot);
  };
  int rc;
  if ((rc = dalloc(c, &flags, nf)) || (rc = dalloc(c, &bad, 1)) || (rc = dalloc(c, &Iofs, nf)) ||
      (rc = dalloc(c, &cnt, nch)) || (rc = dalloc(c, &ofs, nch)) || (rc = dalloc(c, &tot, 1))) {
    cleanup();
    return rc;
  }
  hipMemsetAsync(flags, 1, nf, c->st);
  hipMemsetAsync(bad, 0, sizeof(int), c->st);
  hipLaunchKernelGGL(k_mark_offsets, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->st, n, row_ptr,
                     col_idx, flags, bad);
  hipLaunchKernelGGL(k_compact_count, dim3(nch, 1), dim3(TPB), 0, c->st, (int64_t)nf, flags, cnt, nch);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(TPB), 0, c->st, cnt, ofs, nch, tot, (Inst*)nullptr);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nch, 1), dim3(TPB), 0, c->st, (int64_t)nf, flags, ofs,
                     nch, Iofs, (int*)nullptr);
  long long D = 0;
  int badh = 0;
  hipMemcpyAsync(&D, tot, sizeof(long long), hipMemcpyDeviceToHost, c->st);
  hipMemcpyAsync(&badh, bad, sizeof(int), hipMemcpyDeviceToHost, c->st);
  if (hipStreamSynchronize(c->st) != hipSuccess) { cleanup(); return fail(c, ADEF2_E_HIP, "sync failed"); }
  if (badh) { cleanup(); return fail(c, ADEF2_E_ARG, "column index out of range"); }
  const int dmax = which ? MAXD1 : ADEF2_MAX_DIAGS;
  if (D > dmax || D <= 0) {
    cleanup();
    return fail(c, ADEF2_E_UNSUPPORTED, "operator has " + std::to_string(D) +
                                            " distinct diagonals (max " + std::to_string(dmax) + ")");
  }
  std::vector<int> pos(D);
  hipMemcpyAsync(pos.data(), Iofs, sizeof(int) * D, hipMemcpyDeviceToHost, c->st);
  hipStreamSynchronize(c->st);
  std::vector<int>& off = which ? c->offs1 : c->offs;
  off.resize(D);
  bool has0 = false;
  for (int d = 0; d < D; ++d) {
    off[d] = (int)(pos[d] - (n - 1));
    has0 |= off[d] == 0;
  }
  if (!which && !has0) { cleanup(); return fail(c, ADEF2_E_NOT_SPD, "operator has no main diagonal"); }
  double** d64 = which ? &c->dia1_64 : &c->dia64;
  float** d32 = which ? &c->dia1_32 : &c->dia32;
  if ((rc = dalloc(c, d64, (size_t)D * n)) || (rc = dalloc(c, d32, (size_t)D * n)) ||
      (!which && (rc = dalloc(c, &c->diag, (size_t)n)))) {
    cleanup();
    return rc;
  }
  hipMemsetAsync(*d64, 0, sizeof(double) * D * n, c->st);
  hipMemsetAsync(*d32, 0, sizeof(float) * D * n, c->st);
  OpGeom og{};
  og.N = n;
  if (which) {
    og.D1 = (int)D;
    for (int d = 0; d < D; ++d) og.offs1[d] = off[d];
  } else {
    og.D = (int)D;
    for (int d = 0; d < D; ++d) og.offs[d] = off[d];
  }
  hipMemsetAsync(bad, 0, sizeof(int), c->st);
  hipLaunchKernelGGL(k_csr_to_dia, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->st, n, row_ptr,
                     col_idx, vals, og, which, *d64, *d32, c->diag, bad);
  hipMemcpyAsync(&badh, bad, sizeof(int), hipMemcpyDeviceToHost, c->st);
  hipError_t e = hipStreamSynchronize(c->st);
  cleanup();
  if (e != hipSuccess) return fail(c, ADEF2_E_HIP, std::string("set_reference: ") + hipGetErrorString(e));
  if (badh == 2) return fail(c, ADEF2_E_ARG, "operator has non-finite values");
  if (badh == 3) return fail(c, ADEF2_E_NOT_SPD, "operator has a non-positive diagonal entry");
  if (badh) return fail(c, ADEF2_E_ARG, "inconsistent operator structure");
  return ADEF2_OK;
}

// Rayleigh quotients of the reference modes for the base operator and the
// eigen flags (relative eigen-residual <= EIG_TOL), on the full domain.
int eigen_test(adef2_ctx* c) {
  const int64_t n = c->N;
  const int KP = c->KP;
  int rc;
  if ((rc = dalloc(c, &c->mu64, (size_t)KP)) || (rc = dalloc(c, &c->eigf, (size_t)KP))) return rc;
  double *T = nullptr, *BZ = nullptr;
  if ((rc = dalloc(c, &BZ, (size_t)KP * n)) || (c->factored && (rc = dalloc(c, &T, (size_t)KP * n)))) {
    if (BZ) hipFree(BZ);
    return rc;
  }
  OpGeom og = op_geom(c);
  const dim3 g((unsigned)cdiv(n, 256), KP);
  if (c->factored) {
    hipLaunchKernelGGL(k_ref_inner, g, dim3(256), 0, c->st, og, c->dia1_64, c->Z64, T);
    hipLaunchKernelGGL(k_ref_outer, g, dim3(256), 0, c->st, og, c->dia64, T, BZ);
  } else {
    hipLaunchKernelGGL(k_ref_outer, g, dim3(256), 0, c->st, og, c->dia64, c->Z64, BZ);
  }
  hipLaunchKernelGGL(k_ref_stats, dim3(KP), dim3(TPB), 0, c->st, n, c->k, c->Z64, BZ, EIG_TOL, c->mu64,
                     c->eigf);
  std::vector<uint8_t> e(KP);
  hipError_t err = hipMemcpyAsync(e.data(), c->eigf, KP, hipMemcpyDeviceToHost, c->st);
  if (err == hipSuccess) err = hipStreamSynchronize(c->st);
  hipFree(BZ);
  if (T) hipFree(T);
  if (err != hipSuccess) return fail(c, ADEF2_E_HIP, std::string("eigen test: ") + hipGetErrorString(err));
  c->n_eig = 0;
  for (int q = 0; q < KP; ++q) c->n_eig += e[q];
  return ADEF2_OK;
}

int load_modes(adef2_ctx* c, int64_t n, int32_t k, const double* Z) {
  c->k = k;
  c->KP = round8(k);
  c->n_eig = 0;
  int rc;
  if (c->KP > 0) {
    if ((rc = dalloc(c, &c->Z64, (size_t)c->KP * n)) || (rc = dalloc(c, &c->Z32, (size_t)c->KP * n)))
      return rc;
    hipLaunchKernelGGL(k_copy_modes, dim3((unsigned)cdiv(n, 256), c->KP), dim3(256), 0, c->st, n, k,
                       c->KP, Z, c->Z64, c->Z32);
    if ((rc = dalloc(c, &c->ZT32, (size_t)c->KP * n))) return rc;
    hipLaunchKernelGGL((k_modes_rowmajor<float>), dim3((unsigned)cdiv(n, 256), c->KP), dim3(256), 0, c->st,
                       n, c->KP, c->Z32, c->ZT32);
    HIPCHK(c, hipGetLastError());
    if ((rc = eigen_test(c))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  return ADEF2_OK;
}

int check_ref_args(adef2_ctx* c, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                   const double* vals, int64_t nnz, int32_t k, const double* Z) {
  if (n <= 0 || n > (int64_t)1 << 30 || !row_ptr || !col_idx || !vals || nnz <= 0)
    return fail(c, ADEF2_E_ARG, "invalid operator arguments");
  if (k < 0 || k > ADEF2_MAX_K || (k > 0 && !Z)) return fail(c, ADEF2_E_ARG, "invalid k or Z");
  return ADEF2_OK;
}

}  // namespace

extern "C" {

int adef2_set_reference(adef2_ctx* c, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                        const double* vals, int64_t nnz, int32_t k, const double* Z) {
  if (!c) return ADEF2_E_ARG;
  int rc = check_ref_args(c, n, row_ptr, col_idx, vals, nnz, k, Z);
  if (rc) return rc;
  c->have_ref = false;
  c->restricted = false;
  c->Bcap = 0;
  c->factored = false;
  c->N = n;
  if ((rc = load_dia(c, n, row_ptr, col_idx, vals, 0))) return rc;
  c->D = (int)c->offs.size();
  c->D1 = 0;
  int maxoff = 0;
  for (int o : c->offs) maxoff = std::max(maxoff, std::abs(o));
  c->H = ((maxoff + 63) / 64) * 64;
  if ((rc = load_modes(c, n, k, Z))) return rc;
  c->k_ref = k;
  c->k_safe = 0;
  c->have_ref = true;
  return ADEF2_OK;
}

int adef2_set_reference_factored(adef2_ctx* c, int64_t n, const int64_t* row_ptr,
                                 const int32_t* col_idx, const double* vals, int64_t nnz,
                                 double alpha, double shift, int32_t k, const double* Z) {
  if (!c) return ADEF2_E_ARG;
  int rc = check_ref_args(c, n, row_ptr, col_idx, vals, nnz, k, Z);
  if (rc) return rc;
  if (!(alpha > 0.0) || !std::isfinite(alpha) || !(shift >= 0.0) || !std::isfinite(shift))
    return fail(c, ADEF2_E_ARG, "alpha must be > 0 and shift >= 0");
  c->have_ref = false;
  c->restricted = false;
  c->Bcap = 0;
  c->factored = true;
  c->N = n;
  if ((rc = load_dia(c, n, row_ptr, col_idx, vals, 1))) return rc;
  c->D1 = (int)c->offs1.size();
  c->D = c->D1;
  c->offs.resize(c->D);
  for (int d = 0; d < c->D; ++d) c->offs[d] = -c->offs1[c->D1 - 1 - d];
  if ((rc = dalloc(c, &c->dia64, (size_t)c->D * n)) || (rc = dalloc(c, &c->dia32, (size_t)c->D * n)) ||
      (rc = dalloc(c, &c->diag, (size_t)n)))
    return rc;
  OpGeom og{};
  og.N = n;
  og.D1 = c->D1;
  for (int d = 0; d < c->D1; ++d) og.offs1[d] = c->offs1[d];
  hipLaunchKernelGGL(k_dia_transpose, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->st, og,
                     c->dia1_64, c->dia64, c->dia32, c->diag);
  HIPCHK(c, hipStreamSynchronize(c->st));
  int maxoff = 0;
  for (int o : c->offs1) maxoff = std::max(maxoff, std::abs(o));
  c->H = ((maxoff + 63) / 64) * 64;
  c->alpha_ref = alpha;
  c->shift_ref = shift;
  if ((rc = load_modes(c, n, k, Z))) return rc;
  c->k_ref = k;
  c->k_safe = 0;
  c->have_ref = true;
  return ADEF2_OK;
}

int adef2_set_operator_scale(adef2_ctx* c, double a, double cc) {
  if (!c) return ADEF2_E_ARG;
  if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(cc)) return fail(c, ADEF2_E_ARG, "invalid scale");
  c->scale_a = a;
  c->scale_c = cc;
  c->restricted = false;
  return ADEF2_OK;
}

int adef2_compact(adef2_ctx* c, const uint8_t* mask, int64_t n, int32_t* I, int32_t* g2l,
                  int64_t* n_inactive) {
  if (!c || !mask || n < 0) return ADEF2_E_ARG;
  if (n == 0) { if (n_inactive) *n_inactive = 0; return ADEF2_OK; }
  const int nch = (int)cdiv(n, CMP_CHUNK);
  int* cnt = nullptr;
  int* ofs = nullptr;
  long long* tot = nullptr;
  int rc;
  if ((rc = dalloc(c, &cnt, nch)) || (rc = dalloc(c, &ofs, nch)) || (rc = dalloc(c, &tot, 1))) {
    if (cnt) hipFree(cnt);
    if (ofs) hipFree(ofs);
    return rc;
  }
  hipLaunchKernelGGL(k_compact_count, dim3(nch, 1), dim3(TPB), 0, c->st, n, mask, cnt, nch);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(TPB), 0, c->st, cnt, ofs, nch, tot, (Inst*)nullptr);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nch, 1), dim3(TPB), 0, c->st, n, mask, ofs, nch, I, g2l);
  long long t = 0;
  hipMemcpyAsync(&t, tot, sizeof(long long), hipMemcpyDeviceToHost, c->st);
  hipError_t e = hipStreamSynchronize(c->st);
  hipFree(cnt);
  hipFree(ofs);
  hipFree(tot);
  if (e != hipSuccess) return fail(c, ADEF2_E_HIP, hipGetErrorString(e));
  if (n_inactive) *n_inactive = t;
  return ADEF2_OK;
}

int adef2_compact_noalloc(adef2_ctx* c, const uint8_t* mask, int64_t n, int32_t* I, int32_t* g2l,
                          int64_t* n_inactive_dev, int64_t* n_inactive) {
  if (!c || n < 0 || (n > 0 && !mask)) return ADEF2_E_ARG;
  if (n > NOALLOC_MAX_N)
    return fail(c, ADEF2_E_ARG, "compact_noalloc: n exceeds the 2^28 mask entries its static scratch holds");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->dev) return fail(c, ADEF2_E_STATE, "compact_noalloc: the context's device is not current");
  void* base = scratch_ptr(dev);
  if (!base) return fail(c, ADEF2_E_HIP, "compact_noalloc: hipGetSymbolAddress of the scratch failed");
  const int nch = (int)cdiv(n, CMP_CHUNK);
  int* cnt = (int*)base;
  int* ofs = cnt + NOALLOC_CHUNKS;
  long long* tot = (long long*)(ofs + NOALLOC_CHUNKS);
  long long* tdst = n_inactive_dev ? (long long*)n_inactive_dev : tot;
  if (n == 0) {
    hipLaunchKernelGGL((k_fill<long long>), dim3(1), dim3(64), 0, c->st, tdst, (int64_t)1, 0LL);
  } else {
    // counts and offsets are written in full before they are read: nothing to clear
    hipLaunchKernelGGL(k_compact_count, dim3(nch, 1), dim3(TPB), 0, c->st, n, mask, cnt, nch);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(TPB), 0, c->st, cnt, ofs, nch, tdst, (Inst*)nullptr);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nch, 1), dim3(TPB), 0, c->st, n, mask, ofs, nch, I, g2l);
  }
  HIPCHK(c, hipGetLastError());
  if (n_inactive) {
    long long t = 0;
    HIPCHK(c, hipMemcpyAsync(&t, tdst, sizeof(long long), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    *n_inactive = t;
  }
  return ADEF2_OK;
}

int adef2_restrict(adef2_ctx* c, const uint8_t* mask, int64_t* n_inactive, int32_t* k_eff,
                   double* cond_E) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "restrict before set_reference");
  if (!mask) return fail(c, ADEF2_E_ARG, "null mask");
  c->restricted = false;
  int rc = ensure_batch(c, 1, c->o.precision);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->masks, mask, (size_t)c->N, hipMemcpyDeviceToDevice, c->st));
  rc = restrict_batch(c, nullptr, nullptr);
  if (rc < 0) return rc;
  if (n_inactive) *n_inactive = c->inst_h[0].n_inactive;
  if (k_eff) *k_eff = c->inst_h[0].k_eff;
  if (cond_E) *cond_E = c->inst_h[0].cond;
  return rc;
}

int adef2_solve(adef2_ctx* c, const double* b, const double* x0, double tol, double* x,
                int32_t* iters, double* relres_true, double* cond_E) {
  if (!c) return ADEF2_E_ARG;
  if (!c->restricted || c->B != 1) return fail(c, ADEF2_E_STATE, "solve before restrict");
  if (!b || !x) return fail(c, ADEF2_E_ARG, "null vector");
  int rc = solve_batch(c, b, x0, tol, x);
  if (rc) return rc;
  const Inst& s = c->inst_h[0];
  if (iters) *iters = s.iters;
  if (relres_true) *relres_true = s.bb64 > 0 ? std::sqrt(s.rr64 / s.bb64) : 0.0;
  if (cond_E) *cond_E = s.cond;
  const int st = combine_status(s);
  if (st == ADEF2_E_ARG) return fail(c, st, "non-finite right-hand side or residual");
  if (st == ADEF2_E_NOT_SPD) return fail(c, st, "breakdown: p.Sp <= 0 (operator not SPD)");
  return st;
}

int adef2_solve_batched(adef2_ctx* c, int32_t B, const uint8_t* masks, const double* b,
                        const double* a, const double* cs, const float* theta, double tol,
                        const double* tol_each, double* x,
                        int32_t* iters, int32_t* status, double* relres_true, double* cond_E,
                        int64_t* n_inactive, int32_t* learned) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "solve_batched before set_reference");
  if (B <= 0 || !masks || !b || !x) return fail(c, ADEF2_E_ARG, "invalid batch arguments");
  if (theta && (!c->have_mlp || c->p <= 0))
    return fail(c, ADEF2_E_STATE, "learned enrichment requested before POD modes and MLP parameters");
  if (theta && c->k + MLP_NV > ADEF2_MAX_K)
    return fail(c, ADEF2_E_ARG, "k + 8 learned vectors exceeds ADEF2_MAX_K");
  c->restricted = false;
  int rc;
  BasisSwap swap(c);
  if (theta) {
    if ((rc = swap.enrich(B, theta))) return rc;
  }
  rc = ensure_batch(c, B, c->o.precision);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->masks, masks, (size_t)B * c->N, hipMemcpyDeviceToDevice, c->st));
  rc = restrict_batch(c, a, cs);
  if (rc < 0) return rc;
  rc = solve_batch(c, b, nullptr, tol, x, tol_each);
  if (rc) return rc;
  int worst = ADEF2_OK;
  for (int m = 0; m < B; ++m)
    if (learned) learned[m] = c->inst_h[m].learned;
  for (int m = 0; m < B; ++m) {
    const Inst& s = c->inst_h[m];
    const int st = combine_status(s);
    worst = worst_of(worst, st);
    if (iters) iters[m] = s.iters;
    if (status) status[m] = st;
    if (relres_true) relres_true[m] = s.bb64 > 0 ? std::sqrt(s.rr64 / s.bb64) : 0.0;
    if (cond_E) cond_E[m] = s.cond;
    if (n_inactive) n_inactive[m] = s.n_inactive;
  }
  return worst;
}

int adef2_apply_restricted(adef2_ctx* c, const double* x, double* y) {
  if (!c) return ADEF2_E_ARG;
  if (!c->restricted || c->B != 1) return fail(c, ADEF2_E_STATE, "apply before restrict");
  if (!x || !y) return fail(c, ADEF2_E_ARG, "null vector");
  const int64_t N = c->N;
  double* tmp = nullptr;
  int rc;
  if ((rc = dalloc(c, &tmp, (size_t)c->vs))) return rc;
  fill<double>(c, tmp, (size_t)c->vs, 0.0);
  const dim3 g((unsigned)cdiv(N, 256), 1);
  hipLaunchKernelGGL(k_mask_copy_padded, g, dim3(256), 0, c->st, N, c->masks, x, tmp + c->H, c->vs);
  const double* sv = tmp + c->H;
  if (c->factored) {
    hipLaunchKernelGGL((stencil1_fn<double, double, double>(c->rpt)), dim3(c->ntiles_pad),
                       dim3(IPB), 0, c->st, op_geom(c), c->dia1_64, tmp + c->H,
                       interior(c, c->t64), c->vs, c->inst, 0);
    sv = interior(c, c->t64);
  }
  hipLaunchKernelGGL(k_apply64, g, dim3(256), 0, c->st, op_geom(c), c->dia64, c->masks, tmp + c->H,
                     sv, y, c->inst);
  hipError_t e = hipStreamSynchronize(c->st);
  hipFree(tmp);
  if (e != hipSuccess) return fail(c, ADEF2_E_HIP, hipGetErrorString(e));
  return ADEF2_OK;
}

int adef2_prolong_basis(adef2_ctx* c, int32_t dim, int64_t n, int64_t nc, int32_t r, const double* Zc,
                        double tau_sv, double* Z_out, int32_t* r_out) {
  if (!c) return ADEF2_E_ARG;
  if ((dim != 2 && dim != 3) || nc < 1 || n < nc || r < 1 || r > ADEF2_MAX_K || !(tau_sv >= 0.0) || !Zc ||
      !Z_out)
    return fail(c, ADEF2_E_ARG, "prolong_basis: need dim 2 or 3, 1 <= nc <= n, 1 <= r <= ADEF2_MAX_K");
  const double nf_d = std::pow((double)n, dim);
  if (nf_d > (double)((int64_t)1 << 31)) return fail(c, ADEF2_E_ARG, "prolong_basis: fine grid too large");
  const int64_t Nf = dim == 2 ? n * n : n * n * n;
  const int rpb = 4096;
  const int nrb = (int)cdiv(Nf, rpb);
  const int nt = (int)cdiv(r, GT);
  double *Pt = nullptr, *Q1 = nullptr, *part = nullptr, *G = nullptr, *T = nullptr;
  int *kidx = nullptr, *kpd = nullptr;
  auto cleanup = [&] {
    for (void* q : {(void*)Pt, (void*)Q1, (void*)part, (void*)G, (void*)T, (void*)kidx, (void*)kpd})
      if (q) hipFree(q);
  };
  int rc;
  if ((rc = dalloc(c, &Pt, (size_t)Nf * r)) || (rc = dalloc(c, &Q1, (size_t)Nf * r)) ||
      (rc = dalloc(c, &part, (size_t)nrb * r * r)) || (rc = dalloc(c, &G, (size_t)r * r)) ||
      (rc = dalloc(c, &T, (size_t)r * r)) || (rc = dalloc(c, &kidx, (size_t)r)) || (rc = dalloc(c, &kpd, 1))) {
    cleanup();
    return rc;
  }
  hipLaunchKernelGGL(k_prolong, dim3((unsigned)cdiv(Nf, 256), r), dim3(256), 0, c->st, dim, n, nc, Zc, Pt);
  // two passes of Cholesky QR; the first drops dependent columns
  const double* X = Pt;
  int ncol = r, kp = 0;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_gram_ts, dim3(nrb, nt * nt, 1), dim3(TPB), 0, c->st, Nf, ncol, ncol, X, (int64_t)0, X,
                       (int64_t)0, (const uint8_t*)nullptr, (int64_t)0, rpb, part);
    hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv(ncol * ncol, 256), 1), dim3(256), 0, c->st, nrb, ncol,
                       ncol, part, G);
    hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(64), 0, c->st, ncol, G, pass == 0 ? tau_sv : 0.0, T, kidx,
                       kpd);
    int kph = 0;
    if (hipMemcpyAsync(&kph, kpd, sizeof(int), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess) {
      cleanup();
      return fail(c, ADEF2_E_HIP, "prolong_basis: device error");
    }
    if (kph == 0 || (pass == 1 && kph != ncol)) {
      cleanup();
      return fail(c, ADEF2_E_NOT_SPD, "prolong_basis: prolonged modes are numerically dependent");
    }
    double* Y = pass == 0 ? Q1 : Z_out;
    hipLaunchKernelGGL(k_apply_tri, dim3((unsigned)cdiv(Nf, 256), kph), dim3(256), 0, c->st, Nf, ncol, kidx, T,
                       X, Y);
    X = Q1;
    ncol = kph;
    kp = kph;
  }
  if (kp < r) HIPCHK(c, hipMemsetAsync(Z_out + (size_t)kp * Nf, 0, sizeof(double) * Nf * (r - kp), c->st));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  cleanup();
  if (r_out) *r_out = kp;
  return ADEF2_OK;
}

int adef2_reference_eigs(adef2_ctx* c, int32_t r, const double* X0, int32_t max_iter, double tol,
                         double inner_tol, double* Z_out, double* lambda_out, double* resid_out,
                         int32_t* iters_out) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "reference_eigs before set_reference");
  if (r < 1 || r > ADEF2_MAX_K || !X0 || !Z_out || max_iter < 1 || !(tol > 0.0) || !(inner_tol > 0.0))
    return fail(c, ADEF2_E_ARG, "reference_eigs: need 1 <= r <= ADEF2_MAX_K, max_iter >= 1, tol > 0");
  const int64_t N = c->N;
  const int rpb = 4096;
  const int nrb = (int)cdiv(N, rpb);
  double *X = nullptr, *Y = nullptr, *Zb = nullptr, *D = nullptr, *part = nullptr, *G = nullptr, *E = nullptr;
  double *T1 = nullptr, *F = nullptr, *V = nullptr, *ev = nullptr, *T = nullptr, *lam = nullptr, *Gd = nullptr;
  uint8_t* mk = nullptr;
  int* fl = nullptr;
  auto cleanup = [&] {
    for (void* q : {(void*)X, (void*)Y, (void*)Zb, (void*)D, (void*)part, (void*)G, (void*)E, (void*)T1, (void*)F,
                    (void*)V, (void*)ev, (void*)T, (void*)lam, (void*)Gd, (void*)mk, (void*)fl})
      if (q) hipFree(q);
  };
  const size_t NR = (size_t)N * r, RR = (size_t)r * r;
  int rc;
  if ((rc = dalloc(c, &X, NR)) || (rc = dalloc(c, &Y, NR)) || (rc = dalloc(c, &Zb, NR)) || (rc = dalloc(c, &D, NR)) ||
      (rc = dalloc(c, &part, (size_t)nrb * RR)) || (rc = dalloc(c, &G, RR)) || (rc = dalloc(c, &E, RR)) ||
      (rc = dalloc(c, &T1, RR)) || (rc = dalloc(c, &F, RR)) || (rc = dalloc(c, &V, RR)) ||
      (rc = dalloc(c, &ev, (size_t)r)) || (rc = dalloc(c, &T, RR)) || (rc = dalloc(c, &lam, (size_t)r)) ||
      (rc = dalloc(c, &Gd, RR)) || (rc = dalloc(c, &mk, NR)) || (rc = dalloc(c, &fl, 1))) {
    cleanup();
    return rc;
  }
  HIPCHK(c, hipMemcpyAsync(X, X0, sizeof(double) * NR, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipMemsetAsync(mk, 0, NR, c->st));        // no active points: the full operator
  auto gram = [&](const double* A, const double* Bm, double* out) {
    hipLaunchKernelGGL(k_gram_ts, dim3(nrb, 1, 1), dim3(TPB), 0, c->st, N, r, r, A, (int64_t)0, Bm, (int64_t)0,
                       (const uint8_t*)nullptr, (int64_t)0, rpb, part);
    hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv(RR, 256), 1), dim3(256), 0, c->st, nrb, r, r, part, out);
  };
  std::vector<int32_t> st(r), its(r);
  std::vector<double> gd(RR), lh(r), res(r, INFINITY);
  int it = 0;
  const dim3 gv((unsigned)cdiv(N, 256), r);
  for (it = 1; it <= max_iter; ++it) {
    rc = adef2_solve_batched(c, r, mk, X, nullptr, nullptr, nullptr, inner_tol, nullptr, Y, its.data(), st.data(), nullptr,
                             nullptr, nullptr, nullptr);
    if (rc < 0) { cleanup(); return rc; }
    gram(Y, Y, G);
    gram(Y, X, E);
    hipLaunchKernelGGL(k_rr_reduce, dim3(1), dim3(64), 0, c->st, r, G, E, T1, F, fl);
    hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(1024), 0, c->st, r, F, V, ev);
    hipLaunchKernelGGL(k_rr_finish, dim3(1), dim3(64), 0, c->st, r, T1, V, ev, T, lam);
    hipLaunchKernelGGL(k_ritz_vectors, gv, dim3(256), 0, c->st, N, r, T, lam, X, Y, Zb, D);
    gram(D, D, Gd);
    int flh = 0;
    HIPCHK(c, hipMemcpyAsync(&flh, fl, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(gd.data(), Gd, sizeof(double) * RR, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(lh.data(), lam, sizeof(double) * r, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (flh) { cleanup(); return fail(c, ADEF2_E_NOT_SPD, "reference_eigs: the iterated block lost rank"); }
    double worst = 0.0;
    for (int j = 0; j < r; ++j) {
      res[j] = std::sqrt(std::max(gd[(size_t)j * r + j], 0.0)) / std::fabs(lh[j]);
      worst = std::max(worst, res[j]);
    }
    std::swap(X, Zb);
    if (worst <= tol) break;
  }
  const bool conv = it <= max_iter;
  if (!conv) it = max_iter;
  HIPCHK(c, hipMemcpyAsync(Z_out, X, sizeof(double) * NR, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (lambda_out) for (int j = 0; j < r; ++j) lambda_out[j] = lh[j];
  if (resid_out) for (int j = 0; j < r; ++j) resid_out[j] = res[j];
  if (iters_out) *iters_out = it;
  cleanup();
  return conv ? ADEF2_OK : ADEF2_W_MAXIT;
}

int adef2_active_set_batched(adef2_ctx* c, int32_t B, const double* y_d, const double* psi, double tau,
                             double tol, int32_t max_outer, double* y, uint8_t* masks_out, int32_t* outer,
                             int32_t* inner_iters, int32_t* status) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "active_set_batched before set_reference");
  if (B <= 0 || !y_d || !psi || !y || max_outer <= 0 || !(tau >= 0.0) || !(tol > 0.0))
    return fail(c, ADEF2_E_ARG, "invalid active-set arguments");
  const int64_t N = c->N;
  const int64_t vs = N + 2 * c->H;
  uint8_t *mk = nullptr, *msub = nullptr;
  double *bsub = nullptr, *xsub = nullptr, *ps = nullptr, *t = nullptr;
  int *idx = nullptr, *chg = nullptr;
  auto cleanup = [&] {
    for (void* q : {(void*)mk, (void*)msub, (void*)bsub, (void*)xsub, (void*)ps, (void*)t, (void*)idx,
                    (void*)chg})
      if (q) hipFree(q);
  };
  int rc;
  if ((rc = dalloc(c, &mk, (size_t)B * N)) || (rc = dalloc(c, &msub, (size_t)B * N)) ||
      (rc = dalloc(c, &bsub, (size_t)B * N)) || (rc = dalloc(c, &xsub, (size_t)B * N)) ||
      (rc = dalloc(c, &ps, (size_t)B * vs)) || (c->factored && (rc = dalloc(c, &t, (size_t)B * vs))) ||
      (rc = dalloc(c, &idx, (size_t)B)) || (rc = dalloc(c, &chg, (size_t)B))) {
    cleanup();
    return rc;
  }
  HIPCHK(c, hipMemsetAsync(mk, 0, (size_t)B * N, c->st));               // cold start: A = {}
  fill<double>(c, ps, (size_t)B * vs, 0.0);                               // zero halos
  if (t) fill<double>(c, t, (size_t)B * vs, 0.0);
  std::vector<int> conv(B, 0), outer_h(B, 0), inner_h(B, 0), st_h(B, 0);
  std::vector<int32_t> it_b(B), st_b(B);
  std::vector<int> act, chg_h(B);
  OpGeom og = op_geom(c);
  int worst = ADEF2_OK;
  for (int k = 0; k < max_outer; ++k) {
    act.clear();
    for (int m = 0; m < B; ++m)
      if (!conv[m]) act.push_back(m);
    if (act.empty()) break;
    const int Bs = (int)act.size();
    HIPCHK(c, hipMemcpyAsync(idx, act.data(), sizeof(int) * Bs, hipMemcpyHostToDevice, c->st));
    const dim3 g((unsigned)cdiv(N, 256), Bs);
    double* psi_i = ps + c->H;                 // interior of slot 0 (stride vs)
    hipLaunchKernelGGL(k_ocp_psi, g, dim3(256), 0, c->st, N, idx, mk, psi, vs, psi_i);
    const double* src = psi_i;
    if (c->factored) {
      hipLaunchKernelGGL(k_ocp_inner, g, dim3(256), 0, c->st, og, c->dia1_64, psi_i, vs, t + c->H);
      src = t + c->H;
    }
    hipLaunchKernelGGL(k_ocp_rhs, g, dim3(256), 0, c->st, og, c->dia64, (int)c->factored,
                       c->factored ? c->alpha_ref : 1.0, idx, mk, y_d, src, vs, bsub, msub);
    HIPCHK(c, hipGetLastError());
    rc = adef2_solve_batched(c, Bs, msub, bsub, nullptr, nullptr, nullptr, tol, nullptr, xsub, it_b.data(),
                             st_b.data(), nullptr, nullptr, nullptr, nullptr);
    if (rc < 0) { cleanup(); return rc; }
    HIPCHK(c, hipMemsetAsync(chg, 0, sizeof(int) * Bs, c->st));
    hipLaunchKernelGGL(k_ocp_update, g, dim3(256), 0, c->st, N, idx, mk, xsub, psi, tau, y, chg);
    HIPCHK(c, hipMemcpyAsync(chg_h.data(), chg, sizeof(int) * Bs, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (int j = 0; j < Bs; ++j) {
      const int m = act[j];
      outer_h[m] = k + 1;
      inner_h[m] += it_b[j];
      if (st_b[j] < 0 || st_h[m] < 0) st_h[m] = std::min(st_h[m], (int)st_b[j]);
      else st_h[m] = std::max(st_h[m], (int)st_b[j]);
      if (!chg_h[j]) conv[m] = 1;
    }
  }
  for (int m = 0; m < B; ++m) {
    if (!conv[m] && st_h[m] >= 0) st_h[m] = std::max(st_h[m], (int)ADEF2_W_MAXIT);
    if (st_h[m] < 0) worst = std::min(worst, st_h[m]);
    else if (worst >= 0) worst = std::max(worst, st_h[m]);
    if (outer) outer[m] = outer_h[m];
    if (inner_iters) inner_iters[m] = inner_h[m];
    if (status) status[m] = st_h[m];
  }
  if (masks_out) HIPCHK(c, hipMemcpyAsync(masks_out, mk, (size_t)B * N, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  cleanup();
  return worst;
}

int adef2_variant(adef2_ctx* c, int32_t* rows_per_thread, int32_t* w_mode, float* ms) {
  if (!c) return ADEF2_E_ARG;
  if (!c->solved) return fail(c, ADEF2_E_STATE, "variant before the first solve");
  if (rows_per_thread) *rows_per_thread = c->rpt;
  if (w_mode) *w_mode = c->wfree + 1;
  if (ms) {
    for (int i = 0; i < 10; ++i) ms[i] = 0.0f;
    const int fact = c->factored ? 1 : 0;
    for (const auto& t : c->tuned)
      if (t.B == c->B && t.prec == c->prec && t.KP == c->KP && t.fact == fact && t.N == c->N)
        for (int i = 0; i < 10; ++i) ms[i] = t.ms[i];
  }
  return ADEF2_OK;
}

int adef2_operator_variant(adef2_ctx* c, int32_t* fused, int32_t* tile_rows, int32_t* group, float* ms) {
  if (!c) return ADEF2_E_ARG;
  if (!c->solved) return fail(c, ADEF2_E_STATE, "operator_variant before the first solve");
  if (fused) *fused = c->opf;
  if (tile_rows) *tile_rows = c->of_rows;
  if (group) *group = c->opf ? c->opg : 0;
  if (ms) {
    for (int q = 0; q < 7; ++q) ms[q] = 0.0f;
    const int fact = c->factored ? 1 : 0;
    for (const auto& t : c->tuned)
      if (t.B == c->B && t.prec == c->prec && t.KP == c->KP && t.fact == fact && t.N == c->N &&
          t.opo == c->o.op_fused + 4 * c->o.op_group + 32 * c->o.op_rows)
        for (int q = 0; q < 7; ++q) ms[q] = t.ms_op[q];
  }
  return ADEF2_OK;
}

int adef2_update_variant(adef2_ctx* c, int32_t* warp_specialised, int32_t* tiles_per_block, float* ms) {
  if (!c) return ADEF2_E_ARG;
  if (!c->solved) return fail(c, ADEF2_E_STATE, "update_variant before the first solve");
  const bool tm = (c->wfree == 3 || c->wfree == 4) && c->tm_ok;
  if (warp_specialised) *warp_specialised = tm && c->uws;
  if (tiles_per_block) *tiles_per_block = tm && c->uws ? c->ws_T : (tm ? 1 : 0);
  if (ms) {
    ms[0] = ms[1] = 0.0f;
    const int fact = c->factored ? 1 : 0;
    for (const auto& t : c->tuned)
      if (t.B == c->B && t.prec == c->prec && t.KP == c->KP && t.fact == fact && t.N == c->N &&
          t.uwo == c->o.update_ws) {
        ms[0] = t.ms_uw[0];
        ms[1] = t.ms_uw[1];
      }
  }
  return ADEF2_OK;
}

int adef2_coarse_info(adef2_ctx* c, double* E, int32_t* kept, int32_t* k_eff, double* cond_E) {
  if (!c) return ADEF2_E_ARG;
  if (!c->restricted) return fail(c, ADEF2_E_STATE, "coarse_info before restrict");
  const int KP = c->KP;
  if (KP > 0 && E) {
    std::vector<double> h((size_t)KP * KP);
    HIPCHK(c, hipMemcpy(h.data(), c->Finfo, sizeof(double) * KP * KP, hipMemcpyDeviceToHost));
    const int ke = c->inst_h[0].k_eff;
    for (int j = 0; j < c->k; ++j)
      for (int i = 0; i < c->k; ++i) E[(size_t)j * c->k + i] = (i < ke && j < ke) ? h[(size_t)j * KP + i] : 0.0;
  }
  if (KP > 0 && kept) {
    std::vector<int> h(KP);
    HIPCHK(c, hipMemcpy(h.data(), c->kept, sizeof(int) * KP, hipMemcpyDeviceToHost));
    for (int j = 0; j < c->k; ++j) kept[j] = h[j];
  }
  if (k_eff) *k_eff = c->inst_h[0].k_eff;
  if (cond_E) *cond_E = c->inst_h[0].cond;
  return ADEF2_OK;
}

int adef2_get_stats(adef2_ctx* c, adef2_stats* s) {
  if (!c || !s) return ADEF2_E_ARG;
  ev_harvest(c);
  std::memset(s, 0, sizeof(*s));
  s->n_kernels = KI_COUNT;
  for (int i = 0; i < KI_COUNT; ++i) {
    s->name[i] = kKernelNames[i];
    s->launches[i] = c->st_launch[i];
    s->total_ms[i] = c->st_ms[i];
    s->alg_bytes[i] = c->st_bytes[i];
  }
  s->polls = c->st_polls;
  s->pod_iters = c->pod_iters;
  return ADEF2_OK;
}

int adef2_reset_stats(adef2_ctx* c) {
  if (!c) return ADEF2_E_ARG;
  ev_harvest(c);
  for (int i = 0; i < KI_COUNT; ++i) { c->st_launch[i] = 0; c->st_ms[i] = 0; c->st_bytes[i] = 0; }
  c->st_polls = 0;
  return ADEF2_OK;
}

}  // extern "C"

namespace {
constexpr size_t LOSS_LDS_MAX = 159 * 1024;   // dynamic LDS of k_loss_data (160 KiB less its static part)
constexpr int POD_MAX_M = 8192;   // snapshots per POD call
constexpr int POD_MAXIT = 500;    // subspace iterations (M > JMAX)

// leading p eigenpairs of the symmetric M x M snapshot Gram G (device,
// row-major) by block subspace iteration with Rayleigh-Ritz and SVQB
// re-orthonormalisation.  V: device column-major M x p; th: host,
// descending.  Converged when every wanted Ritz pair has
// ||G v - theta v|| <= 1e-10 theta + 1e-13 theta_1.
int gram_top_eigs(adef2_ctx* c, int M, const double* G, int p, double* V, std::vector<double>& th) {
  const int L = std::min(M - 1, p + std::max(32, p / 2));
  const size_t ML = (size_t)M * L, LL = (size_t)L * L;
  double *Q = nullptr, *Y = nullptr, *QW = nullptr, *YW = nullptr, *C = nullptr, *U = nullptr, *d = nullptr,
         *dsc = nullptr, *inv = nullptr, *ths = nullptr, *res = nullptr, *part = nullptr;
  int* sel = nullptr;
  auto cleanup = [&] {
    for (void* q : {(void*)Q, (void*)Y, (void*)QW, (void*)YW, (void*)C, (void*)U, (void*)d, (void*)dsc,
                    (void*)inv, (void*)ths, (void*)res, (void*)part, (void*)sel})
      if (q) hipFree(q);
  };
  const int nt = (int)cdiv(L, GT);
  int rc;
  if ((rc = dalloc(c, &Q, ML)) || (rc = dalloc(c, &Y, ML)) || (rc = dalloc(c, &QW, ML)) ||
      (rc = dalloc(c, &YW, ML)) || (rc = dalloc(c, &C, LL)) || (rc = dalloc(c, &U, LL)) ||
      (rc = dalloc(c, &d, (size_t)L)) || (rc = dalloc(c, &dsc, (size_t)L)) || (rc = dalloc(c, &inv, (size_t)L)) ||
      (rc = dalloc(c, &ths, (size_t)L)) || (rc = dalloc(c, &res, (size_t)L)) || (rc = dalloc(c, &part, LL)) ||
      (rc = dalloc(c, &sel, (size_t)L))) { cleanup(); return rc; }
  const dim3 gcol((unsigned)cdiv(M, 256), (unsigned)L);
  // out = A^T B (L x L, row-major) over the M rows, one row block
  auto gram = [&](const double* A, const double* Bm, double* out) {
    hipLaunchKernelGGL(k_gram_ts, dim3(1, nt * nt, 1), dim3(TPB), 0, c->st, (int64_t)M, L, L, A, (int64_t)0, Bm,
                       (int64_t)0, (const uint8_t*)nullptr, (int64_t)0, M, part);
    hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv(LL, 256), 1), dim3(256), 0, c->st, 1, L, L, part, out);
  };
  // Qout = orthonormal basis of span(Z) (Qout != Z)
  auto svqb = [&](const double* Z, double* Qout) {
    gram(Z, Z, C);
    hipLaunchKernelGGL(k_svqb_scale, dim3(1), dim3(1024), 0, c->st, L, C, dsc);
    hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(1024), 0, c->st, L, C, U, d);
    hipLaunchKernelGGL(k_svqb_inv, dim3(1), dim3(256), 0, c->st, L, d, 1e-14, inv);
    hipLaunchKernelGGL(k_comb_cols, gcol, dim3(256), 0, c->st, M, L, Z, dsc, U, (const int*)nullptr, inv, Qout);
  };
  hipLaunchKernelGGL(k_start_block, dim3((unsigned)cdiv(ML, 256)), dim3(256), 0, c->st, (int64_t)ML, Y);
  svqb(Y, QW);
  svqb(QW, Q);
  std::vector<double> dh(L), thh(L), rh(L);
  std::vector<int> idx(L);
  for (int it = 0; it < POD_MAXIT; ++it) {
    hipLaunchKernelGGL(k_symm_block, dim3((unsigned)cdiv(M, 256), (unsigned)cdiv(L, SYB)), dim3(256), 0, c->st,
                       M, L, G, Q, Y);
    gram(Q, Y, C);
    hipLaunchKernelGGL(k_symmetrize, dim3(1), dim3(1024), 0, c->st, L, C);
    hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(1024), 0, c->st, L, C, U, d);
    hipMemcpyAsync(dh.data(), d, sizeof(double) * L, hipMemcpyDeviceToHost, c->st);
    if (hipStreamSynchronize(c->st) != hipSuccess) { cleanup(); return fail(c, ADEF2_E_HIP, "pod subspace sync"); }
    for (int i = 0; i < L; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return dh[a] > dh[b]; });
    for (int i = 0; i < L; ++i) thh[i] = dh[idx[i]];
    hipMemcpyAsync(sel, idx.data(), sizeof(int) * L, hipMemcpyHostToDevice, c->st);
    hipMemcpyAsync(ths, thh.data(), sizeof(double) * L, hipMemcpyHostToDevice, c->st);
    hipLaunchKernelGGL(k_comb_cols, gcol, dim3(256), 0, c->st, M, L, Q, (const double*)nullptr, U, sel,
                       (const double*)nullptr, QW);
    hipLaunchKernelGGL(k_comb_cols, gcol, dim3(256), 0, c->st, M, L, Y, (const double*)nullptr, U, sel,
                       (const double*)nullptr, YW);
    hipLaunchKernelGGL(k_ritz_resid, dim3(L), dim3(256), 0, c->st, M, QW, YW, ths, res);
    hipMemcpyAsync(rh.data(), res, sizeof(double) * L, hipMemcpyDeviceToHost, c->st);
    if (hipStreamSynchronize(c->st) != hipSuccess) { cleanup(); return fail(c, ADEF2_E_HIP, "pod subspace sync"); }
    bool done = true;
    for (int j = 0; j < p; ++j)
      if (!(rh[j] <= 1e-10 * std::fabs(thh[j]) + 1e-13 * std::fabs(thh[0]))) done = false;
    if (done) {
      hipMemcpyAsync(V, QW, sizeof(double) * (size_t)M * p, hipMemcpyDeviceToDevice, c->st);
      const hipError_t e = hipStreamSynchronize(c->st);
      cleanup();
      if (e != hipSuccess) return fail(c, ADEF2_E_HIP, hipGetErrorString(e));
      th.assign(thh.begin(), thh.begin() + p);
      c->pod_iters = it + 1;
      return ADEF2_OK;
    }
    // next block: the Ritz vectors multiplied by G, orthonormalised twice
    svqb(YW, Y);
    svqb(Y, Q);
  }
  cleanup();
  return fail(c, ADEF2_E_NOCONV, "pod: the subspace iteration on the snapshot Gram did not converge");
}
}  // namespace

extern "C" {

int adef2_pod(adef2_ctx* c, int32_t M, const double* X, int32_t p, double* Phi_out, double* sigma) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "pod before set_reference");
  if (M < 2 || M > POD_MAX_M || p < 1 || p > MLP_P || p >= M || !X)
    return fail(c, ADEF2_E_ARG, "need 2 <= M <= 8192 snapshots and 1 <= p < M, p <= 64");
  const int64_t N = c->N;
  const bool direct = M <= JMAX;
  double *Xc = nullptr, *part = nullptr, *G = nullptr, *V = nullptr, *ev = nullptr;
  int* sel = nullptr;
  // at most 16 row blocks of partial Grams (16 M^2 doubles)
  const int rpb = (int)std::max<int64_t>(4096, cdiv(N, 16));
  const int nrb = (int)cdiv(N, rpb);
  const int nt = (int)cdiv(M, GT);
  auto cleanup = [&] { for (void* q : {(void*)Xc, (void*)part, (void*)G, (void*)V, (void*)ev, (void*)sel}) if (q) hipFree(q); };
  int rc;
  if ((rc = dalloc(c, &Xc, (size_t)N * M)) || (rc = dalloc(c, &part, (size_t)nrb * M * M)) ||
      (rc = dalloc(c, &G, (size_t)M * M)) || (rc = dalloc(c, &V, direct ? (size_t)M * M : (size_t)M * p)) ||
      (rc = dalloc(c, &ev, direct ? (size_t)M : (size_t)p)) || (rc = dalloc(c, &sel, (size_t)p))) { cleanup(); return rc; }
  hipLaunchKernelGGL(k_center, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, c->st, N, M, X, Xc);
  hipLaunchKernelGGL(k_gram_ts, dim3(nrb, nt * nt, 1), dim3(TPB), 0, c->st, N, M, M, Xc, (int64_t)0, Xc,
                     (int64_t)0, (const uint8_t*)nullptr, (int64_t)0, rpb, part);
  hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv((int64_t)M * M, 256), 1), dim3(256), 0, c->st, nrb, M, M,
                     part, G);
  hipFree(part);
  part = nullptr;
  std::vector<double> th;
  if (direct) {
    hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(1024), 0, c->st, M, G, V, ev);
    std::vector<double> evh(M);
    hipMemcpyAsync(evh.data(), ev, sizeof(double) * M, hipMemcpyDeviceToHost, c->st);
    if (hipStreamSynchronize(c->st) != hipSuccess) { cleanup(); return fail(c, ADEF2_E_HIP, "pod sync"); }
    // order the eigenvalues (descending) on the host: p indices only
    std::vector<int> idx(M);
    for (int i = 0; i < M; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return evh[i] > evh[j]; });
    hipMemcpyAsync(sel, idx.data(), sizeof(int) * p, hipMemcpyHostToDevice, c->st);
    for (int j = 0; j < p; ++j) th.push_back(evh[idx[j]]);
    c->pod_iters = 0;
  } else {
    if ((rc = gram_top_eigs(c, M, G, p, V, th))) { cleanup(); return rc; }
    hipMemcpyAsync(ev, th.data(), sizeof(double) * p, hipMemcpyHostToDevice, c->st);
  }
  if ((rc = dalloc(c, &c->Phi, (size_t)N * p))) { cleanup(); return rc; }
  // Phi[:, j] = Xc v_j / sqrt(theta_j)
  if (direct)
    hipLaunchKernelGGL(k_pod_modes, dim3((unsigned)cdiv(N, 256), p), dim3(256), 0, c->st, N, M, p, Xc, V,
                       (int64_t)M, (int64_t)1, sel, ev, c->Phi);
  else
    hipLaunchKernelGGL(k_pod_modes, dim3((unsigned)cdiv(N, 256), p), dim3(256), 0, c->st, N, M, p, Xc, V,
                       (int64_t)1, (int64_t)M, (const int*)nullptr, ev, c->Phi);
  if (Phi_out) hipMemcpyAsync(Phi_out, c->Phi, sizeof(double) * N * p, hipMemcpyDeviceToDevice, c->st);
  hipError_t e = hipStreamSynchronize(c->st);
  cleanup();
  if (e != hipSuccess) return fail(c, ADEF2_E_HIP, hipGetErrorString(e));
  if (sigma) for (int j = 0; j < p; ++j) sigma[j] = th[j] > 0 ? std::sqrt(th[j]) : 0.0;
  c->p = p;
  return ADEF2_OK;
}

int adef2_set_pod_modes(adef2_ctx* c, int32_t p, const double* Phi) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "set_pod_modes before set_reference");
  if (p < 1 || p > MLP_P || !Phi) return fail(c, ADEF2_E_ARG, "1 <= p <= 64 and Phi required");
  int rc;
  if ((rc = dalloc(c, &c->Phi, (size_t)c->N * p))) return rc;
  HIPCHK(c, hipMemcpyAsync(c->Phi, Phi, sizeof(double) * c->N * p, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->p = p;
  return ADEF2_OK;
}

int adef2_set_enrichment(adef2_ctx* c, int32_t p, const double* Phi, const float* mlp_params,
                         int32_t n_vec, double tau_learned) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "set_enrichment before set_reference");
  if (n_vec != MLP_NV)
    return fail(c, ADEF2_E_UNSUPPORTED, "set_enrichment: the network emits 8 enrichment vectors (n_vec = 8)");
  if (p < 1 || p > MLP_P || !Phi) return fail(c, ADEF2_E_ARG, "set_enrichment: 1 <= p <= 64 and Phi required");
  if (c->k + MLP_NV > ADEF2_MAX_K)
    return fail(c, ADEF2_E_ARG, "set_enrichment: k + 8 enrichment vectors exceeds ADEF2_MAX_K");
  if (mlp_params && !(tau_learned >= 1.0)) return fail(c, ADEF2_E_ARG, "tau_learned must be >= 1");
  int rc = adef2_set_pod_modes(c, p, Phi);
  if (rc) return rc;
  if (mlp_params) return adef2_learned_set_params(c, mlp_params, tau_learned);
  return ADEF2_OK;
}

int adef2_pod_enrich(adef2_ctx* c, int32_t p, double tau_safe) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref) return fail(c, ADEF2_E_STATE, "pod_enrich before set_reference");
  if (tau_safe <= 0.0) tau_safe = c->o.tau_safe;
  if (p < 0 || (p > 0 && !(tau_safe >= 1.0)) || c->k_ref + p > ADEF2_MAX_K)
    return fail(c, ADEF2_E_ARG, "pod_enrich: need 0 <= p, k + p <= ADEF2_MAX_K and tau_safe >= 1");
  if (p > 0 && (!c->Phi || p > c->p)) return fail(c, ADEF2_E_STATE, "pod_enrich: fewer POD modes held than p");
  const int64_t N = c->N;
  const int kn = c->k_ref + p;
  double* Zt = nullptr;
  int rc;
  if (kn > 0) {
    if ((rc = dalloc(c, &Zt, (size_t)N * kn))) return rc;
    if (c->k_ref > 0)
      HIPCHK(c, hipMemcpyAsync(Zt, c->Z64, sizeof(double) * N * c->k_ref, hipMemcpyDeviceToDevice, c->st));
    if (p > 0)
      HIPCHK(c, hipMemcpyAsync(Zt + (size_t)N * c->k_ref, c->Phi, sizeof(double) * N * p,
                               hipMemcpyDeviceToDevice, c->st));
  }
  drop_graphs(c);
  HIPCHK(c, hipStreamSynchronize(c->st));     // Zt is read from the old Z64
  rc = load_modes(c, N, kn, Zt);
  if (Zt) {
    hipStreamSynchronize(c->st);
    hipFree(Zt);
  }
  if (rc) return rc;
  c->k_safe = p > 0 ? c->k_ref : 0;
  c->tau_safe = tau_safe;
  c->restricted = false;
  return ADEF2_OK;
}

int adef2_learned_set_params(adef2_ctx* c, const float* params, double tau_learned) {
  if (!c || !params) return ADEF2_E_ARG;
  if (!(tau_learned >= 1.0)) return fail(c, ADEF2_E_ARG, "tau_learned must be >= 1");
  int rc;
  if (!c->mlp) {
    if ((rc = dalloc(c, &c->mlp, NPARAM)) || (rc = dalloc(c, &c->mlp_bf, NPARAM)) ||
        (rc = dalloc(c, &c->mlp_g, NPARAM)) || (rc = dalloc(c, &c->mlp_m, NPARAM)) ||
        (rc = dalloc(c, &c->mlp_v, NPARAM)))
      return rc;
  }
  HIPCHK(c, hipMemcpyAsync(c->mlp, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->st));
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)cdiv(NPARAM, 256)), dim3(256), 0, c->st, NPARAM, c->mlp, c->mlp_bf);
  HIPCHK(c, hipMemsetAsync(c->mlp_m, 0, sizeof(float) * NPARAM, c->st));
  HIPCHK(c, hipMemsetAsync(c->mlp_v, 0, sizeof(float) * NPARAM, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->adam_t = 0;
  c->tau_learned = tau_learned;
  c->have_mlp = true;
  return ADEF2_OK;
}

int adef2_learned_get_params(adef2_ctx* c, float* params) {
  if (!c || !params) return ADEF2_E_ARG;
  if (!c->have_mlp) return fail(c, ADEF2_E_STATE, "no MLP parameters");
  HIPCHK(c, hipMemcpy(params, c->mlp, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  return ADEF2_OK;
}

int adef2_learned_prepare(adef2_ctx* c, int32_t M, const uint8_t* masks, const double* b,
                          const double* xsol, const float* theta, const double* a_h, const double* c_h) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_ref || c->p <= 0) return fail(c, ADEF2_E_STATE, "learned_prepare needs set_reference and POD modes");
  if (!c->factored) return fail(c, ADEF2_E_UNSUPPORTED, "learned enrichment needs the factored operator");
  if (M <= 0 || !masks || !b || !xsol || !theta) return fail(c, ADEF2_E_ARG, "invalid training arguments");
  const int64_t N = c->N;
  const int k = c->k, p = c->p, nb = k + p;
  const int obj = c->o.learned_objective;
  const size_t lds = sizeof(double) * ((size_t)k * k + (size_t)k * (p + 1) + (obj == 1 ? (size_t)k * p : 0));
  // k_loss_data keeps the k x k Cholesky factor and its solves in LDS: up to
  // 159 KiB of gfx950's 160 KiB per workgroup (k = 64, p = 64 fits either
  // objective)
  if (lds > LOSS_LDS_MAX)
    return fail(c, ADEF2_E_UNSUPPORTED, "learned_prepare: k*k + k*(p+1) (+ k*p for the deflated-spectrum "
                                        "objective) must fit 20352 doubles (159 KiB of LDS)");
  if (lds > 65536)
    HIPCHK(c, hipFuncSetAttribute((const void*)k_loss_data, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int rc;
  c->Mtr = 0;
  if ((rc = dalloc(c, &c->theta_tr, (size_t)M * MD0)) || (rc = dalloc(c, &c->Htr, (size_t)M * p * p)) ||
      (rc = dalloc(c, &c->gtr, (size_t)M * p)) || (rc = dalloc(c, &c->e0tr, (size_t)M)) ||
      (rc = dalloc(c, &c->bxtr, (size_t)M)) || (obj == 1 && (rc = dalloc(c, &c->Ntr, (size_t)M * p * p))))
    return rc;
  HIPCHK(c, hipMemcpyAsync(c->theta_tr, theta, sizeof(float) * M * MD0, hipMemcpyDeviceToDevice, c->st));
  double *VB = nullptr, *T = nullptr, *Wv = nullptr, *part = nullptr, *G = nullptr, *bz = nullptr, *bx1 = nullptr;
  double *DV = nullptr, *Gd = nullptr;
  Inst* one = nullptr;
  const int rpb = 4096;
  const int nrb = (int)cdiv(N, rpb);
  const int nt = (int)cdiv(nb, GT);
  auto cleanup = [&] {
    for (void* q : {(void*)VB, (void*)T, (void*)Wv, (void*)part, (void*)G, (void*)bz, (void*)bx1, (void*)one,
                    (void*)DV, (void*)Gd})
      if (q) hipFree(q);
  };
  if ((rc = dalloc(c, &VB, (size_t)N * nb)) || (rc = dalloc(c, &T, (size_t)N * nb)) ||
      (rc = dalloc(c, &Wv, (size_t)N * nb)) || (rc = dalloc(c, &part, (size_t)nrb * nb * nb)) ||
      (rc = dalloc(c, &G, (size_t)nb * nb)) || (rc = dalloc(c, &bz, (size_t)nb)) ||
      (rc = dalloc(c, &bx1, 1)) || (rc = dalloc(c, &one, 1)) ||
      (obj == 1 && ((rc = dalloc(c, &DV, (size_t)N * nb)) || (rc = dalloc(c, &Gd, (size_t)nb * nb))))) {
    cleanup();
    return rc;
  }
  // [Z | Phi] (k reference modes first)
  HIPCHK(c, hipMemcpyAsync(VB, c->Z64, sizeof(double) * N * k, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(VB + (size_t)N * k, c->Phi, sizeof(double) * N * p, hipMemcpyDeviceToDevice, c->st));
  OpGeom og = op_geom(c);
  std::vector<double> bxh(M);
  for (int m = 0; m < M; ++m) {
    const uint8_t* mk = masks + (size_t)m * N;
    Inst ih{};
    const double ua = a_h ? a_h[m] : c->scale_a, uc = c_h ? c_h[m] : c->scale_c;
    ih.a = ua * c->alpha_ref;
    ih.c = ua * c->shift_ref + uc;
    hipMemcpyAsync(one, &ih, sizeof(Inst), hipMemcpyHostToDevice, c->st);
    // S_II [Z | Phi] restricted: T = A Vtilde on all rows, W = a A^T T + c Vtilde (inactive rows)
    hipLaunchKernelGGL(k_stencil_modes, dim3((unsigned)cdiv(N, 256), nb, 1), dim3(256), 0, c->st, og,
                       c->dia1_64, VB, (int64_t)0, mk, nb, T);
    hipLaunchKernelGGL(k_outer_cols, dim3((unsigned)cdiv(N, 256), nb), dim3(256), 0, c->st, og, c->dia64,
                       T, VB, mk, one, Wv);
    hipLaunchKernelGGL(k_gram_ts, dim3(nrb, nt * nt, 1), dim3(TPB), 0, c->st, N, nb, nb, VB, (int64_t)0,
                       Wv, (int64_t)0, mk, (int64_t)0, rpb, part);
    hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv(nb * nb, 256), 1), dim3(256), 0, c->st, nrb, nb,
                       nb, part, G);
    hipLaunchKernelGGL(k_gram_ts, dim3(nrb, nt, 1), dim3(TPB), 0, c->st, N, nb, 1, VB, (int64_t)0,
                       b + (size_t)m * N, (int64_t)0, mk, (int64_t)0, rpb, part);
    hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv(nb, 256), 1), dim3(256), 0, c->st, nrb, nb, 1,
                       part, bz);
    hipLaunchKernelGGL(k_gram_ts, dim3(nrb, 1, 1), dim3(TPB), 0, c->st, N, 1, 1, b + (size_t)m * N,
                       (int64_t)0, xsol + (size_t)m * N, (int64_t)0, mk, (int64_t)0, rpb, part);
    hipLaunchKernelGGL(k_gram_finish, dim3(1, 1), dim3(256), 0, c->st, nrb, 1, 1, part, c->bxtr + m);
    if (obj == 1) {   // D-weighted Gram of [Z | Phi] on the inactive rows, D = diag(S_II)
      hipLaunchKernelGGL(k_dscale_cols, dim3((unsigned)cdiv(N, 256), nb), dim3(256), 0, c->st, N, VB, c->diag,
                         mk, one, DV);
      hipLaunchKernelGGL(k_gram_ts, dim3(nrb, nt * nt, 1), dim3(TPB), 0, c->st, N, nb, nb, VB, (int64_t)0,
                         DV, (int64_t)0, mk, (int64_t)0, rpb, part);
      hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)cdiv(nb * nb, 256), 1), dim3(256), 0, c->st, nrb, nb,
                         nb, part, Gd);
    }
    // the kernel indexes its one sample through blockIdx.x = 0; shift the outputs
    hipLaunchKernelGGL(k_loss_data, dim3(1), dim3(1024), lds, c->st, k, p, G, bz, c->Htr + (size_t)m * p * p,
                       c->gtr + (size_t)m * p, c->e0tr + m, c->o.drop_rel, (const double*)Gd,
                       obj == 1 ? c->Ntr + (size_t)m * p * p : (double*)nullptr);
  }
  hipError_t e = hipStreamSynchronize(c->st);
  cleanup();
  if (e != hipSuccess) return fail(c, ADEF2_E_HIP, std::string("learned_prepare: ") + hipGetErrorString(e));
  // b^T x* > 0 for an SPD system and b != 0: it normalises the loss
  HIPCHK(c, hipMemcpy(bxh.data(), c->bxtr, sizeof(double) * M, hipMemcpyDeviceToHost));
  for (int m = 0; m < M; ++m)
    if (!(bxh[m] > 0.0) || !std::isfinite(bxh[m]))
      return fail(c, ADEF2_E_ARG, "learned_prepare: sample " + std::to_string(m) +
                                      " has b_I^T x_I <= 0 (not a solution, or b_I = 0)");
  c->Mtr = M;
  c->obj_tr = obj;
  return ADEF2_OK;
}

int adef2_learned_loss_grad(adef2_ctx* c, double* loss, float* grad) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_mlp || c->Mtr <= 0) return fail(c, ADEF2_E_STATE, "learned_loss_grad needs parameters and prepared samples");
  int rc;
  if ((rc = ensure_mlp_batch(c, c->Mtr))) return rc;
  mlp_grad_launch(c, c->Mtr);
  HIPCHK(c, hipGetLastError());
  if (loss) HIPCHK(c, hipMemcpyAsync(loss, c->lossv, sizeof(double) * c->Mtr, hipMemcpyDeviceToHost, c->st));
  if (grad) HIPCHK(c, hipMemcpyAsync(grad, c->mlp_g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return ADEF2_OK;
}

int adef2_learned_train(adef2_ctx* c, int32_t steps, float lr, double* loss_hist) {
  if (!c) return ADEF2_E_ARG;
  if (!c->have_mlp || c->Mtr <= 0) return fail(c, ADEF2_E_STATE, "learned_train needs parameters and prepared samples");
  if (steps < 0 || !(lr > 0.0f)) return fail(c, ADEF2_E_ARG, "invalid training arguments");
  int rc;
  const int M = c->Mtr;
  if ((rc = ensure_mlp_batch(c, M))) return rc;
  std::vector<double> lh(M);
  const float b1 = 0.9f, b2 = 0.999f;
  for (int it = 0; it < steps; ++it) {
    mlp_grad_launch(c, M);
    c->adam_t += 1;
    const float c1 = 1.0f - std::pow(b1, (float)c->adam_t), c2 = 1.0f - std::pow(b2, (float)c->adam_t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)cdiv(NPARAM, 256)), dim3(256), 0, c->st, NPARAM, c->mlp,
                       c->mlp_g, c->mlp_m, c->mlp_v, c->mlp_bf, lr, b1, b2, 1e-8f, c1, c2);
    if (loss_hist) {
      HIPCHK(c, hipMemcpyAsync(lh.data(), c->lossv, sizeof(double) * M, hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
      double sum = 0.0;
      for (double v : lh) sum += v;
      loss_hist[it] = sum / M;
    }
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  return ADEF2_OK;
}

int adef2_learned_forward(adef2_ctx* c, int32_t M, const float* theta, float* out) {
  if (!c || M <= 0 || !theta || !out) return ADEF2_E_ARG;
  if (!c->have_mlp) return fail(c, ADEF2_E_STATE, "no MLP parameters");
  int rc;
  if ((rc = ensure_mlp_batch(c, M))) return rc;
  mlp_forward_launch(c, M, theta);
  HIPCHK(c, hipMemcpyAsync(out, c->mout, sizeof(float) * M * MD3, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return ADEF2_OK;
}

const char* adef2_last_error(const adef2_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
