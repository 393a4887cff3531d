// Dispatch of the regression kernels (templates in esim_regress_impl.h, one
// translation unit per feature count).
#include <mutex>

#include "esim_internal.h"

namespace esim {

void regress_table_1(RegressTable&);
void regress_table_2(RegressTable&);
void regress_table_3(RegressTable&);
void regress_table_4(RegressTable&);
void regress_table_5(RegressTable&);
void regress_table_6(RegressTable&);
void regress_table_7(RegressTable&);
void regress_table_8(RegressTable&);
void regress_table_9(RegressTable&);
void regress_table_10(RegressTable&);
void regress_table_11(RegressTable&);
void regress_table_12(RegressTable&);

namespace {

const RegressTable* table(int F) {
  static RegressTable tabs[ESIM_MAX_F + 1];
  static std::once_flag once;
  std::call_once(once, [] {
    void (*fill[ESIM_MAX_F + 1])(RegressTable&) = {
        nullptr,          regress_table_1, regress_table_2,  regress_table_3, regress_table_4,
        regress_table_5,  regress_table_6, regress_table_7,  regress_table_8, regress_table_9,
        regress_table_10, regress_table_11, regress_table_12};
    for (int f = 1; f <= ESIM_MAX_F; ++f) fill[f](tabs[f]);
  });
  return (F >= 1 && F <= ESIM_MAX_F) ? &tabs[F] : nullptr;
}

KernelFn pick(int F, int lanes, bool f16) {
  const RegressTable* t = table(F);
  const int li = lanes == 1 ? 0 : lanes == 2 ? 1 : lanes == 4 ? 2 : lanes == 8 ? 3 : lanes == 16 ? 4 : -1;
  return (t && li >= 0) ? t->general[li][f16] : nullptr;
}

KernelFn pick_onepass(int F, bool f16) {
  const RegressTable* t = table(F);
  return t ? t->onepass[f16] : nullptr;
}

KernelFn pick_c32(int F, int lanes, bool f16) {
  const RegressTable* t = table(F);
  const int li = lanes == 4 ? 0 : lanes == 16 ? 1 : -1;
  return (t && li >= 0) ? t->c32[li][f16] : nullptr;
}

}  // namespace

int regress_supported_lanes(int F) { return (F >= 1 && F <= ESIM_MAX_F) ? 0x1 | 0x2 | 0x4 | 0x8 | 0x10 : 0; }

bool regress_supports(int F, int lanes, int precision) {
  if (precision == ESIM_GRAM_F32C) return pick_c32(F, lanes, false) != nullptr;
  return pick(F, lanes, false) != nullptr;
}

hipError_t launch_regress(const RegressArgs& a, int F, bool f16, int precision, int lanes,
                          int blocks_per_cu, int max_r, const DeviceShape& dev, hipStream_t s) {
  // the condition estimate (FP64 Gram) has an instance of its own, one lane
  // per item (the caller sizes the groups for one lane)
  const RegressTable* tab = table(F);
  KernelFn fn = precision == ESIM_GRAM_F32C ? pick_c32(F, lanes, f16)
                : a.kappa ? (tab ? tab->kappa[f16] : nullptr)
                : (lanes == 16 && 2 * max_r + 1 <= 16) ? pick_onepass(F, f16)
                                                       : pick(F, lanes, f16);
  if (!fn) return hipErrorInvalidValue;
  int64_t blocks = (a.max_groups + kWavesPerBlock - 1) / kWavesPerBlock;
  const int64_t cap = static_cast<int64_t>(dev.cus) * blocks_per_cu;
  if (blocks > cap) blocks = cap;
  blocks = (blocks + dev.xcds - 1) / dev.xcds * dev.xcds;   // a multiple of the XCDs (see GroupIter)
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace esim
