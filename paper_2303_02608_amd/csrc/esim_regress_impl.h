// Weighted local regression (Sec. 2.1, eqs. 3-5) on gfx950: kernel templates.
// Each feature count is instantiated in a translation unit of its own
// (esim_regress_inst.hip); esim_regress.hip dispatches.
//
// One regression ("item") is the minimiser of
//     (1/W) sum_i w_i (y_i - alpha - beta^T u_i)^2 + ridge * |beta|^2,
//     u_i = x^i - x^c,  w_i = exp(-1/2 sum_j (u_ij / (h b_j))^2),  W = sum_i w_i,
// over the window |dx|, |dy| <= r, |dt| <= tr (truncated at image borders and
// clip ends), with x = (px / r, py / r, f_0 .. f_{F-1}).
//
// Mapping.  A wave holds G = 64 / L items; the L lanes of an item split the
// 2r+1 window columns, so for one column pass the coordinate regressor is
// constant in a lane and every Gram entry that involves it is formed once per
// pass instead of once per sample (esim_wlr.h).  Dense launches use L = 1
// (64 items per wave, no cross-lane sums), work lists L = 16 (4 items per
// wave, one column per lane).  Loads are raw buffer loads
// (SGPR resource + VGPR offset, the channel stride in the SGPR offset),
// coalesced over the L adjacent columns of an item and over the G adjacent
// items of a dense wave.
//
// Precision.  The weight exponent is summed in FP64 from FP64 differences of
// the FP32 inputs and exponentiated with the FP32 hardware exp2 (about 1e-7
// relative).  Gram, right-hand side and Cholesky are FP64: without packed FP32
// (disabled by the compile flags) an FP64 FMA issues at the same rate as an
// FP32 one on CDNA4, and the windows are ill-conditioned (kappa up to ~1e6
// with a 1e-6 ridge), which FP32 accumulation does not survive at the 1e-4
// contract.
//
// After the window loop the L lane partials are summed with DPP, every lane of
// the item factors the (F+3)x(F+3) system redundantly (registers only) and the
// lanes share the output writes.  The optional condition output is Hager's
// 1-norm estimate on the factor.
#pragma once
#include <type_traits>

#include "esim_wlr.h"

namespace esim {
namespace {

// One group of a launch: G = 64 / L items, g * G + slot for the lane's slot,
// below n_items (work lists) or the pixels of group g (dense).
//
// C32 selects the reduced-precision variant: FP32 regressors and weights,
// FP32 Gram with block-compensated sums (GramC), FP32 Cholesky, and an FP64
// re-solve of the same compensated Gram for items whose Hager condition
// estimate exceeds kappa_fp64.  ONE selects the one-pass Gram (every lane
// owns one window column).
// Rows of window data in flight in the interior one-pass loop.
constexpr int kRing = 3;

// KAPPA: the instance that writes the condition estimate (FP64 Gram, one lane
// per item); the estimate's code stays out of the other instances, whose
// register budget it would raise.
template <int F, int L, bool F16, bool C32, bool ONE, bool KAPPA>
__device__ __forceinline__ void regress_group(const RegressArgs& a, int64_t g, int64_t n_items) {
  constexpr int D = F + 2;
  constexpr int P = F + 3;
  constexpr int G = kWave / L;
  using Real = typename std::conditional<C32, float, double>::type;

  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / L;
  const int j = lane % L;
  {
    // ---- which item, clip, pixel and frame this lane group works on.  Items
    //      are bounds-checked (clip, pixel, frame); invalid ones are skipped.
    int my_cl = 0;
    int64_t my_pix = 0, idx_out = 0;
    int my_t = a.t;
    bool valid = false;
    if (a.items) {
      const int64_t i = g * G + slot;
      const int64_t it = i < n_items ? a.items[i] : -1;
      if (it >= 0) {
        const int c = item_clip(it);
        if (c < a.nclips) {
          const int64_t p = item_pixel(it);
          const int fr = a.t >= 0 ? a.t : item_frame(it);
          if (p < a.clips[c].HW && fr >= 0 && fr < a.clips[c].T) {
            valid = true;
            my_cl = c;
            my_pix = p;
            my_t = fr;
          }
        }
      }
      idx_out = i;
    } else {
      for (int c = 1; c < a.nclips; ++c)
        if (a.clips[c].grp_off[lanes_index(L)] <= g) my_cl = c;
      const int64_t p = (g - a.clips[my_cl].grp_off[lanes_index(L)]) * G + slot;
      valid = p < a.clips[my_cl].HW && a.t < a.clips[my_cl].T;
      my_pix = valid ? p : 0;
      idx_out = a.clips[my_cl].pix_off + p;
    }
    // Waterfall over the clips present in the wave (one round when the work
    // list keeps each wave inside one clip, as the threshold call does).
    uint64_t todo = __ballot(valid);
    while (todo != 0) {
      const int cl = __builtin_amdgcn_readfirstlane(
          __shfl(my_cl, __ffsll(static_cast<unsigned long long>(todo)) - 1));
      const bool active = valid && my_cl == cl && ((todo >> lane) & 1ull);
      todo &= ~__ballot(active);
      const ClipDev& C = a.clips[cl];
      // frames held by the buffer resources: the window of a uniform frame, or
      // the whole clip when items carry their own frame
      const int f0 = a.t >= 0 ? max(0, a.t - C.tr) : 0;
      const int f1 = a.t >= 0 ? min(C.T, a.t + C.tr + 1) : C.T;
      // Interior waves of the one-pass (work-list) instances: every item's
      // window lies inside the image and the clip, so the window loop runs
      // without per-row validity tests; lanes without an item then take the
      // geometry of the first item (weights 0).  The other instances keep the
      // checked loop only: a second loop variant costs them registers (many
      // spills at F = 10, one wave per SIMD).
      const int fr = active ? my_t : (a.t >= 0 ? a.t : 0);
      const int prow = static_cast<int>(my_pix / C.W), pcol = static_cast<int>(my_pix - prow * C.W);
      const bool inside = prow >= C.r && prow + C.r < C.H && pcol >= C.r && pcol + C.r < C.W &&
                          fr - C.tr >= 0 && fr + C.tr < C.T;
      const uint64_t act = __ballot(active);
      const bool full = ONE && !C32 && __ballot(active && !inside) == 0;
      int64_t gpix = active ? my_pix : 0;
      int gfr = fr;
      if (full) {
        const int src = __ffsll(static_cast<unsigned long long>(act)) - 1;
        const int64_t p0 = __shfl(my_pix, src);
        const int t0 = __shfl(fr, src);
        if (!active) {
          gpix = p0;
          gfr = t0;
        }
      }
      ItemGeom<F, F16, Real> geo;
      make_geom(geo, C, gpix, gfr, f0, f1, active);

      double th[P], rhs[P], Syy, iW, kap = 0.0;
      if constexpr (!C32) {
        Gram<F, double> gm;
        auto add = [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
          gm.add_onepass(w, yd, v, vy);
        };
        if constexpr (ONE) {
          // every lane owns one column (2r + 1 <= L, checked by the launcher)
          gm.zero_onepass();
          if (full)
            window_loop_ring<F, L, F16, kRing>(geo, j, [&](double) {}, add,
                                               [&](double vx) { gm.fold_onepass(vx); });
          else
            window_loop<F, L, F16, double>(geo, j, [&](double) {}, add, [&](double vx) { gm.fold_onepass(vx); });
        } else {
          gm.zero_snap();
          window_loop<F, L, F16, double>(geo, j, [&](double) { gm.pass_begin_snap(); }, add,
                                         [&](double vx) { gm.pass_end_snap(vx); });
        }
        gm.template lane_sum<L>();
        double M[P * (P + 1) / 2], anorm;
        iW = gram_solve<F, double>(gm, C, M, rhs, th, anorm);
        Syy = gm.Syy;
        if constexpr (KAPPA) {
          equilibrate_factor<P, double>(M);
          kap = anorm * hager_inv_norm1<P, double>(M);
        } else {
          (void)anorm;
        }
      } else {
        GramC<F> gc;
        gc.zero();
        window_loop<F, L, F16, float>(
            geo, j, [&](float) { gc.pass_begin(); },
            [&](float w, float yd, const float (&v)[F], float vy, int, int, int, bool) {
              gc.add(w, yd, v, vy);
            },
            [&](float vx) { gc.pass_end(vx); });
        gc.template lane_sum<L>();
        Gram<F, float> g32;
        gc.values(g32);
        float M32[P * (P + 1) / 2], r32[P], t32[P], an32;
        iW = gram_solve<F, float>(g32, C, M32, r32, t32, an32);
        equilibrate_factor<P, float>(M32);
        kap = static_cast<double>(an32) * static_cast<double>(hager_inv_norm1<P, float>(M32));
        const bool fallback = !(kap <= C.kappa_fp64);
        Syy = g32.Syy;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          th[i] = t32[i];
          rhs[i] = r32[i];
        }
        if (__ballot(fallback && active) != 0) {
          Gram<F, double> g64;
          gc.values(g64);
          double M[P * (P + 1) / 2], r64[P], t64[P], an64;
          const double iW64 = gram_solve<F, double>(g64, C, M, r64, t64, an64);
          if (fallback) {
            iW = iW64;
            Syy = g64.Syy;
#pragma unroll
            for (int i = 0; i < P; ++i) {
              th[i] = t64[i];
              rhs[i] = r64[i];
            }
          }
        }
      }

      // ---- outputs (the lanes of an item share the writes: lane j of the
      //      group writes components j, j + L, ...; each component's value is
      //      picked by a select over the L candidates of its round, so a lane
      //      forms one address per round instead of one per component)
      if (active && a.update_state) {
        if (j == 0) {
          C.st_alpha[my_pix] = static_cast<float>(th[0]);
          C.st_tref[my_pix] = my_t;
        }
#pragma unroll
        for (int k = 0; k < (F + L - 1) / L; ++k) {
          const int f = j + k * L;
          if (f < F) {
            double bv = 0.0;
#pragma unroll
            for (int ff = k * L; ff < (k + 1) * L && ff < F; ++ff)
              if (ff == f) bv = th[3 + ff] * C.sf[2 + ff];
            C.st_beta[f * C.HW + my_pix] = static_cast<float>(bv);
            C.st_xref[f * C.HW + my_pix] = feat_value(C, my_t, f, my_pix);
          }
        }
      }
      if (active && a.alpha) {
        if (j == 0) {
          a.alpha[idx_out] = static_cast<float>(th[0]);
          if (a.resid) {
            // at the solution (A + Lambda) theta = rhs, so
            // R = Syy/W - theta^T rhs - theta^T Lambda theta
            double tg = 0.0, bb = 0.0;
#pragma unroll
            for (int i = 0; i < P; ++i) tg = fma(th[i], rhs[i], tg);
#pragma unroll
            for (int i = 1; i < P; ++i) bb = fma(th[i] * C.c2[i - 1], th[i], bb);
            a.resid[idx_out] = static_cast<float>(Syy * iW - tg - C.ridge * bb);
          }
          if (a.kappa && (KAPPA || C32)) a.kappa[idx_out] = static_cast<float>(kap);
        }
        if (a.beta) {
#pragma unroll
          for (int k = 0; k < (D + L - 1) / L; ++k) {
            const int d = j + k * L;
            if (d < D) {
              double bv = 0.0;
#pragma unroll
              for (int dd = k * L; dd < (k + 1) * L && dd < D; ++dd)
                if (dd == d) bv = th[1 + dd] * C.sf[dd];
              a.beta[static_cast<int64_t>(d) * a.n_out + idx_out] = static_cast<float>(bv);
            }
          }
        }
      }
    }  // waterfall
  }
}

// FP64 instances up to 8 features keep their window-loop accumulators within
// half the register file and run two waves per SIMD (a wave's scalar and
// memory instructions then issue beside the other wave's FMAs); larger F, and
// the compensated-FP32 variant, run one.
template <int F, bool C32>
constexpr int regress_waves_per_simd() {
  return (!C32 && F <= 8) ? 2 : 1;
}

template <int F, int L, bool F16, bool C32, bool ONE = false, bool KAPPA = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(regress_waves_per_simd<F, C32>())))
regress_kernel(RegressArgs a) {
  constexpr int G = kWave / L;
  // the device count is clamped to the output length: item i writes index i
  const int64_t n_items =
      a.items ? max(static_cast<int64_t>(0), min(static_cast<int64_t>(a.count[0]), a.n_out)) : 0;
  const int64_t ngroups = a.items ? (n_items + G - 1) / G : a.n_dense_groups;
  GroupIter it(ngroups, a.nxcd, a.items ? nullptr : a.xcd_bounds);
  int64_t g;
  while (it.next(g)) regress_group<F, L, F16, C32, ONE, KAPPA>(a, g, n_items);
}

}  // namespace
}  // namespace esim
