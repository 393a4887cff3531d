// Instantiates the regression kernels of one feature count (ESIM_REGRESS_F,
// set by the build) and fills its dispatch table.
#include "esim_regress_impl.h"

#ifndef ESIM_REGRESS_F
#error "ESIM_REGRESS_F must be defined"
#endif

#define ESIM_CAT2(a, b) a##b
#define ESIM_CAT(a, b) ESIM_CAT2(a, b)

namespace esim {

void ESIM_CAT(regress_table_, ESIM_REGRESS_F)(RegressTable& t) {
  constexpr int F = ESIM_REGRESS_F;
  t.general[0][0] = regress_kernel<F, 1, false, false>;
  t.general[0][1] = regress_kernel<F, 1, true, false>;
  t.general[1][0] = regress_kernel<F, 2, false, false>;
  t.general[1][1] = regress_kernel<F, 2, true, false>;
  t.general[2][0] = regress_kernel<F, 4, false, false>;
  t.general[2][1] = regress_kernel<F, 4, true, false>;
  t.general[3][0] = regress_kernel<F, 8, false, false>;
  t.general[3][1] = regress_kernel<F, 8, true, false>;
  t.general[4][0] = regress_kernel<F, 16, false, false>;
  t.general[4][1] = regress_kernel<F, 16, true, false>;
  t.onepass[0] = regress_kernel<F, 16, false, false, true>;
  t.onepass[1] = regress_kernel<F, 16, true, false, true>;
  t.kappa[0] = regress_kernel<F, 1, false, false, false, true>;
  t.kappa[1] = regress_kernel<F, 1, true, false, false, true>;
  // the compensated-FP32 variant is compiled for the feature counts of the
  // workloads (7 and 10) and for the default lane counts
#if ESIM_REGRESS_F == 7 || ESIM_REGRESS_F == 10
  t.c32[0][0] = regress_kernel<F, 4, false, true>;
  t.c32[0][1] = regress_kernel<F, 4, true, true>;
  t.c32[1][0] = regress_kernel<F, 16, false, true>;
  t.c32[1][1] = regress_kernel<F, 16, true, true>;
#endif
}

}  // namespace esim
