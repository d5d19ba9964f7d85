// Instantiations of the per-instance iteration kernels for one vector type
// ITER_V, panel type ITER_M and tile height ITER_RPT (rows per thread); the
// build compiles this file once per combination.
#include "iter_tab.h"

#ifndef ITER_V
#error "ITER_V, ITER_M and ITER_RPT must be defined"
#endif

namespace adef2 {

template <typename V, typename M, int KP, int RPT>
static KTab<V, M> make_tab() {
  if constexpr (sizeof(V) == 8)
    return {k_init<V, M, KP, RPT>, k_init2<V, M, KP, RPT>, k_pupdate<V, M, KP, RPT>,
            k_spmv<V, M, KP, RPT>, k_update<V, M, KP, RPT>, k_update_nw<V, M, KP, RPT>,
            k_zproj<V, M, KP, RPT>, k_update<V, M, KP, RPT, true>};
  else
    return {k_init<V, M, KP, RPT>, k_init2<V, M, KP, RPT>, k_pupdate<V, M, KP, RPT>,
            k_spmv<V, M, KP, RPT>, k_update<V, M, KP, RPT>, nullptr, nullptr,
            k_update<V, M, KP, RPT, true>};
}

template <typename V, typename M, int R>
KTab<V, M> pick_kp(int KP) {
  switch (KP) {
    case 0: return make_tab<V, M, 0, R>();
    case 8: return make_tab<V, M, 8, R>();
    case 16: return make_tab<V, M, 16, R>();
    case 24: return make_tab<V, M, 24, R>();
    case 32: return make_tab<V, M, 32, R>();
    case 40: return make_tab<V, M, 40, R>();
    case 48: return make_tab<V, M, 48, R>();
    case 56: return make_tab<V, M, 56, R>();
    default: return make_tab<V, M, 64, R>();
  }
}

template KTab<ITER_V, ITER_M> pick_kp<ITER_V, ITER_M, ITER_RPT>(int);

}  // namespace adef2
