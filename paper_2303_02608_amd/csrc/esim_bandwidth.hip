// Bandwidth-optimised regression (Sec. 3, bandwidth optimisation): the global
// bandwidth h of eq. (5) chosen per regression from K candidates by the
// smallest estimated mean squared error of alpha.
//
// alpha_h = e_0^T A_h^{-1} g_h is linear in the observations y, and its weight
// on the centre sample (w_c = 1, z_c = e_0) is v_0 / W_h with v = A_h^{-1} e_0.
// With sigma_c^2 the MC variance of y_c, Stein's unbiased risk estimate
//     SURE(h) = (alpha_h - y_c)^2 + 2 sigma_c^2 v_0 / W_h - sigma_c^2
// estimates E[(alpha_h - f_c)^2] (squared bias plus variance).
//
//   log_variance_kernel  sigma^2 of y = log(E + eps) from the radiance sample
//                        variance: var / spp / (E + eps)^2 (delta method).
//   bandwidth_*_kernel   per regression (dense: one lane per pixel of frame t;
//                        work lists: 16 lanes per item, one window column
//                        each) and candidate: the window loop of the
//                        regression with the regressors scaled to that h, the
//                        W-normalised system with the ridge in those units,
//                        Cholesky, theta and v; the outputs of the candidate
//                        with the smallest SURE (the first of equal ones) are
//                        written.
#include <cmath>
#include <cstdint>

#include "esim_bandwidth.h"
#include "esim_internal.h"
#include "esim_wlr.h"

namespace esim {
namespace {

__global__ void __launch_bounds__(256)
log_variance_kernel(const float* __restrict__ E, const float* __restrict__ var, float* __restrict__ vy,
                    int64_t n, float inv_spp, float eps) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float e = E[i] + eps;
    vy[i] = var[i] * inv_spp / (e * e);
  }
}

// The candidates of one item in lane j of its L-lane group (L = 1: the lane
// owns the item; L = 16: one window column per lane, the sums combined with
// DPP; ONE: every lane owns exactly one column).  Lane j == 0 writes output i.
template <int F, bool F16, int L, bool ONE>
__device__ __forceinline__ void bandwidth_item(const BandwidthArgs& a, const ClipDev& C, int64_t i,
                                               int64_t pix, bool active, int j) {
  constexpr int P = F + 3;
  const int f0 = max(0, a.t - C.tr), f1 = min(C.T, a.t + C.tr + 1);
  const int64_t cen = static_cast<int64_t>(a.t) * C.HW + pix;
  const double yc = C.y[cen];
  const double s2 = a.vy[cen];
  const bool writer = active && j == 0;
  if (writer) {
    a.alpha[i] = __builtin_nanf("");
    if (a.hsel) a.hsel[i] = __builtin_nanf("");
    if (a.sure) a.sure[i] = __builtin_nanf("");
  }
  double best = INFINITY;
  for (int k = 0; k < a.K; ++k) {
    const double sc = a.scale[k];            // h / h_k: regressors in h_k-scaled units
    ItemGeom<F, F16, double> g;
    make_geom(g, C, pix, a.t, f0, f1, active);
#pragma unroll
    for (int d = 0; d < F + 2; ++d) g.sf[d] *= sc;
#pragma unroll
    for (int f = 0; f < F; ++f) g.xcs[f] *= sc;
    g.vx_step *= sc;
    g.vy_step *= sc;
    Gram<F, double> gm;
    if constexpr (ONE) {
      gm.zero_onepass();
      window_loop<F, L, F16, double>(
          g, j, [&](double) {},
          [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
            gm.add_onepass(w, yd, v, vy);
          },
          [&](double vx) { gm.fold_onepass(vx); });
    } else {
      gm.zero_snap();
      window_loop<F, L, F16, double>(
          g, j, [&](double) { gm.pass_begin_snap(); },
          [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
            gm.add_onepass(w, yd, v, vy);
          },
          [&](double vx) { gm.pass_end_snap(vx); });
    }
    gm.template lane_sum<L>();
    // the W-normalised system; the ridge lambda on beta in units u reads
    // lambda (sf_j sc)^2 on the scaled unknowns
    const double iW = 1.0 / gm.SW;
    const double lam = C.ridge * sc * sc;
    double M[P * (P + 1) / 2], rhs[P], th[P], e0[P], v[P];
    M[tri(0, 0)] = 1.0;
    M[tri(1, 0)] = gm.A0x * iW;
    M[tri(2, 0)] = gm.A0y * iW;
    M[tri(1, 1)] = gm.Axx * iW + lam * C.c2[0];
    M[tri(2, 1)] = gm.Axy * iW;
    M[tri(2, 2)] = gm.Ayy * iW + lam * C.c2[1];
    rhs[0] = gm.g0 * iW;
    rhs[1] = gm.gx * iW;
    rhs[2] = gm.gy * iW;
    {
      int q = 0;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        M[tri(3 + f, 0)] = gm.A0f[f] * iW;
        M[tri(3 + f, 1)] = gm.Axf[f] * iW;
        M[tri(3 + f, 2)] = gm.Ayf[f] * iW;
        rhs[3 + f] = gm.gf[f] * iW;
#pragma unroll
        for (int e = f; e < F; ++e) {
          M[tri(3 + e, 3 + f)] = gm.Aff[q] * iW + (e == f ? lam * C.c2[2 + f] : 0.0);
          ++q;
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < P; ++jj) e0[jj] = jj == 0 ? 1.0 : 0.0;
    cholesky_inplace<P, double>(M);
    chol_solve<P, double>(M, rhs, th);
    chol_solve<P, double>(M, e0, v);
    const double d = th[0] - yc;
    const double sure = d * d + 2.0 * s2 * v[0] * iW - s2;
    if (active && sure < best) {              // NaN (a failed factor) never wins
      best = sure;
      if (writer) {
        a.alpha[i] = static_cast<float>(th[0]);
        if (a.beta)
#pragma unroll
          for (int jj = 0; jj < F + 2; ++jj)
            a.beta[jj * a.n_out + i] = static_cast<float>(th[1 + jj] * C.sf[jj] * sc);
        if (a.hsel) a.hsel[i] = static_cast<float>(a.h[k]);
        if (a.sure) a.sure[i] = static_cast<float>(sure);
      }
    }
  }
}

// Up to 8 features the window loop's accumulators fit half the register file:
// two waves per SIMD, as for the regression (a wave's memory and scalar work
// then issues beside the other wave's FMAs).
template <int F>
constexpr int bandwidth_waves_per_simd() {
  return F <= 8 ? 2 : 1;
}

// Dense: one lane per pixel of frame t.
template <int F, bool F16>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bandwidth_waves_per_simd<F>())))
bandwidth_dense_kernel(BandwidthArgs a) {
  const ClipDev& C = *a.clip;
  const int64_t n = C.HW;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  // uniform trip count per block: lanes past n idle with weight 0
  for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    const bool active = i < n;
    bandwidth_item<F, F16, 1, false>(a, C, i, active ? i : 0, active, 0);
  }
}

// Work list: kListLanes lanes per item (scattered pixels: the lanes of an item
// read adjacent columns, so its loads coalesce), the one-pass Gram when every
// lane owns one column.
constexpr int kListLanes = 16;
template <int F, bool F16, bool ONE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bandwidth_waves_per_simd<F>())))
bandwidth_list_kernel(BandwidthArgs a) {
  const ClipDev& C = *a.clip;
  const int64_t n = max(static_cast<int64_t>(0), min(static_cast<int64_t>(a.count[0]), a.n_out));
  constexpr int ipb = 256 / kListLanes;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * ipb;
  const int j = threadIdx.x % kListLanes;
  for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * ipb; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x / kListLanes;
    bool active = i < n;
    int64_t pix = 0;
    if (active) {
      const int64_t it = a.items[i];
      active = it >= 0 && item_clip(it) == 0 && item_pixel(it) < C.HW;
      pix = active ? item_pixel(it) : 0;
    }
    bandwidth_item<F, F16, kListLanes, ONE>(a, C, i, pix, active, j);
  }
}

using BandwidthFn = void (*)(BandwidthArgs);

// kind 0: dense; 1: work list, one-pass; 2: work list, pass-snapshot
template <int F>
BandwidthFn pick(bool f16, int kind) {
  if (kind == 0) return f16 ? bandwidth_dense_kernel<F, true> : bandwidth_dense_kernel<F, false>;
  if (kind == 1) return f16 ? bandwidth_list_kernel<F, true, true> : bandwidth_list_kernel<F, false, true>;
  return f16 ? bandwidth_list_kernel<F, true, false> : bandwidth_list_kernel<F, false, false>;
}

BandwidthFn bandwidth_fn(int F, bool f16, int kind) {
  switch (F) {
    case 1: return pick<1>(f16, kind);
    case 2: return pick<2>(f16, kind);
    case 3: return pick<3>(f16, kind);
    case 4: return pick<4>(f16, kind);
    case 5: return pick<5>(f16, kind);
    case 6: return pick<6>(f16, kind);
    case 7: return pick<7>(f16, kind);
    case 8: return pick<8>(f16, kind);
    case 9: return pick<9>(f16, kind);
    case 10: return pick<10>(f16, kind);
    case 11: return pick<11>(f16, kind);
    case 12: return pick<12>(f16, kind);
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_log_variance(const float* E, const float* var, float* vy, int64_t n, int spp, float eps,
                               hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(log_variance_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, E, var, vy, n,
                     1.0f / static_cast<float>(spp), eps);
  return hipGetLastError();
}

hipError_t launch_bandwidth(const BandwidthArgs& a, int F, bool f16, int64_t max_items, int r, hipStream_t s) {
  const int kind = a.items ? (2 * r + 1 <= kListLanes ? 1 : 2) : 0;
  const BandwidthFn k = bandwidth_fn(F, f16, kind);
  if (!k) return hipErrorInvalidValue;
  const int64_t per_block = a.items ? 256 / kListLanes : 256;
  int64_t blocks = (max_items + per_block - 1) / per_block;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace esim
