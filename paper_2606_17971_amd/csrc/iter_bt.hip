// Instantiations of the tile-major iteration kernels (shared basis, FP64
// vectors) for FP64 and FP32 panels.
#include "iter_tab.h"

namespace adef2 {

template <typename M, int KP>
static BtTab<M> make_bt() {
  if constexpr (KP <= 32)
    return {k_pupdate_bt<double, M, KP>, k_zproj_bt<M, KP>, k_pupdate_tm<M, KP>, k_update_tm<M, KP>,
            k_finish_tm<M, KP>, k_stencil1_tm<M>, k_spmv_tm<M>, k_alpha_tm<M>, k_update_ws<M, KP>};
  else
    return {k_pupdate_bt<double, M, KP>, k_zproj_bt<M, KP>, k_pupdate_tm<M, KP>, k_update_tm<M, KP>,
            k_finish_tm<M, KP>, k_stencil1_tm<M>, k_spmv_tm<M>, k_alpha_tm<M>, nullptr};
}

template <typename M>
BtTab<M> pick_bt(int KP) {
  switch (KP) {
    case 8: return make_bt<M, 8>();
    case 16: return make_bt<M, 16>();
    case 24: return make_bt<M, 24>();
    case 32: return make_bt<M, 32>();
    case 40: return make_bt<M, 40>();
    case 48: return make_bt<M, 48>();
    case 56: return make_bt<M, 56>();
    default: return make_bt<M, 64>();
  }
}

template BtTab<double> pick_bt<double>(int);
template BtTab<float> pick_bt<float>(int);

}  // namespace adef2
