// Kernel tables of the iteration kernels.  The instantiations live in their
// own translation units (iter_inst.hip per vector / panel type and tile
// height, iter_bt.hip for the tile-major kernels) so that the library builds
// in parallel; the host runtime only sees these declarations.
#pragma once
#include "dev_tile.h"

namespace adef2 {

// per-instance kernels: one block per (tile, instance)
template <typename V, typename M>
struct KTab {
  void (*init)(IterArgs<V, M>);
  void (*init2)(IterArgs<V, M>);
  void (*pupdate)(IterArgs<V, M>);
  void (*spmv)(IterArgs<V, M>);
  void (*update)(IterArgs<V, M>);
  void (*update_nw)(IterArgs<V, M>);
  void (*zproj)(IterArgs<V, M>);
  void (*update_spec)(IterArgs<V, M>);
};

// defined in iter_inst.hip for V, M in {(double, double), (double, float),
// (float, float)} and RPT in {1, 2}; KP in {0, 8, ..., 64}
template <typename V, typename M, int RPT>
KTab<V, M> pick_kp(int KP);

// tile-major kernels of a basis shared by every instance (FP64 vectors):
// the W-free pair (pupdate_bt, zproj_bt) and the boundary-form pair
// (pupdate_tm, update_tm)
template <typename M>
struct BtTab {
  void (*pupdate_bt)(IterArgs<double, M>);
  void (*zproj_bt)(IterArgs<double, M>);
  void (*pupdate_tm)(IterArgs<double, M>);
  void (*update_tm)(IterArgs<double, M>);
  void (*finish_tm)(IterArgs<double, M>);
  void (*stencil1_tm)(IterArgs<double, M>);
  void (*spmv_tm)(IterArgs<double, M>);
  void (*alpha_tm)(IterArgs<double, M>);
  void (*update_ws)(IterArgs<double, M>);   // warp-specialised update (KP <= 32; null above)
};

// defined in iter_bt.hip for M in {double, float}
template <typename M>
BtTab<M> pick_bt(int KP);

}  // namespace adef2
