// Launchers of the bandwidth-optimised regression (esim_bandwidth.hip).
#pragma once

#include "esim_internal.h"

namespace esim {

constexpr int kMaxBandwidths = 8;

struct BandwidthArgs {
  const ClipDev* clip;          // single clip (device)
  int32_t t;                    // frame of every regression
  const int64_t* items;         // nullptr = every pixel of the clip
  const int32_t* count;         // work-list length (device)
  int64_t n_out;                // output stride (>= HW when dense)
  const float* vy;              // [T][H][W] MC variance of y
  int32_t K;                    // candidates
  double scale[kMaxBandwidths]; // h / h_k (the plan's h over the candidate)
  double h[kMaxBandwidths];     // candidate bandwidths
  float* alpha;                 // [n_out]
  float* beta;                  // [D][n_out] nullable
  float* hsel;                  // [n_out] nullable
  float* sure;                  // [n_out] nullable
};

hipError_t launch_log_variance(const float* E, const float* var, float* vy, int64_t n, int spp, float eps,
                               hipStream_t s);
hipError_t launch_bandwidth(const BandwidthArgs& a, int F, bool f16, int64_t max_items, int r, hipStream_t s);

}  // namespace esim
