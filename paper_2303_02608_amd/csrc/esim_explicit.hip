// Explicit Delta R threshold (Sec. 2.2: eq. (7) and the R of eq. (4) summed
// over a window, instead of the closed form of Prop. 1).
//
//   explicit_flag_kernel  one lane per pixel of a 256-pixel block (the block
//                         layout of the closed-form flag kernel, so the same
//                         scatter compacts it).  With the stored plane
//                         (alpha, beta over D: bxy and beta) and, in
//                         bandwidth-scaled regressors v, theta_j = beta_j h b_j:
//                           pass 1, the last-event window (frame t_ref, centre
//                           x^c = the features at t_ref):
//                             r_i    = y_i - alpha - theta^T v_i
//                             rhat_i = r_i + beta^T (x_hat^c - x^c)
//                           (last-window reading: R, R_hat and the mean of
//                           rhat all come from this pass);
//                           pass 2 (new-window reading), frame t's window with
//                           weights and v about x_hat^c:
//                             rhat_i = y_i - alpha - theta^T v_i
//                         Delta R = |R_hat - R|; flag when Delta R >= C^2;
//                         dl = s sqrt(Delta R), s the sign of the weighted
//                         mean of rhat (-1 when 0).  Sums in FP64, weights in
//                         FP32 from the regression's window loop.
#include <cmath>
#include <cstdint>

#include "esim_compact.h"
#include "esim_internal.h"
#include "esim_wlr.h"

namespace esim {
namespace {

template <int F, bool F16>
__global__ void __launch_bounds__(kBlock)
explicit_flag_kernel(const ClipDev* __restrict__ clips, int nclips, int t, float* __restrict__ dl,
                     Workspace ws, const int64_t* __restrict__ ev_count) {
  __shared__ int wcount[kWavesPerBlock];
  const int64_t b = blockIdx.x;
  const int cl = block_clip(clips, nclips, b);
  const ClipDev& C = clips[cl];
  const int64_t p = (b - C.blk_off) * kBlock + threadIdx.x;
  const bool frame_ok = t >= 1 && t < C.T;      // uniform in the block
  const bool in = frame_ok && p < C.HW;
  bool flag = false, pos = false;
  if (frame_ok) {
    const int64_t pc = in ? p : 0;              // idle lanes read pixel 0 with weight 0
    const int tref = min(max(C.st_tref[pc], 0), C.T - 1);
    // the plane in scaled regressors: pred = alpha + sum_j th_j v_j
    const double alpha = C.st_alpha[pc];
    const double thx = static_cast<double>(C.st_bxy[pc]) / C.sf[0];
    const double thy = static_cast<double>(C.st_bxy[C.HW + pc]) / C.sf[1];
    double th[F];
    double shift = 0.0;                         // beta^T (x_hat^c - x^c)
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const double bf = C.st_beta[f * C.HW + pc];
      th[f] = bf / C.sf[2 + f];
      shift = fma(bf, static_cast<double>(feat_value(C, t, f, pc)) - C.st_xref[f * C.HW + pc], shift);
    }
    const bool new_window = C.thr == ESIM_THRESHOLD_NEW_WINDOW;
    double sw = 0.0, sr2 = 0.0, sh = 0.0, sh2 = 0.0;
    double base = alpha;                        // alpha + th_x v_x of the column pass
    {
      ItemGeom<F, F16, double> g;
      make_geom(g, C, pc, tref, 0, C.T, in);
      window_loop<F, 1>(
          g, 0, [&](double vx) { base = fma(thx, vx, alpha); },
          [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
            double pr = fma(thy, vy, base);
#pragma unroll
            for (int f = 0; f < F; ++f) pr = fma(th[f], v[f], pr);
            const double r = yd - pr;
            const double rh = r + shift;
            const double wr = w * r, wh = w * rh;
            sw += w;
            sr2 = fma(wr, r, sr2);
            sh += wh;
            sh2 = fma(wh, rh, sh2);
          },
          [&](double) {});
    }
    const double R = sr2 / sw;
    double Rh = sh2 / sw, mean = sh / sw;
    if (new_window) {
      ItemGeom<F, F16, double> g;
      make_geom(g, C, pc, t, 0, C.T, in);
      double sw2 = 0.0, s1 = 0.0, s2 = 0.0;
      window_loop<F, 1>(
          g, 0, [&](double vx) { base = fma(thx, vx, alpha); },
          [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
            double pr = fma(thy, vy, base);
#pragma unroll
            for (int f = 0; f < F; ++f) pr = fma(th[f], v[f], pr);
            const double rh = yd - pr;
            const double wh = w * rh;
            sw2 += w;
            s1 += wh;
            s2 = fma(wh, rh, s2);
          },
          [&](double) {});
      Rh = s2 / sw2;
      mean = s1 / sw2;
    }
    if (in) {
      const double d = fabs(Rh - R);
      flag = d >= C.C * C.C;
      pos = mean > 0.0;
      if (dl) dl[C.pix_off + p] = static_cast<float>(pos ? sqrt(d) : -sqrt(d));
    }
  } else if (p < C.HW && dl) {
    dl[C.pix_off + p] = __builtin_nanf("");
  }
  const int w = threadIdx.x / kWave;
  const uint64_t fm = __ballot(flag);
  const uint64_t pm = __ballot(flag && pos);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    ws.flags[b * kWavesPerBlock + w] = fm;
    ws.pol[b * kWavesPerBlock + w] = pm;
    wcount[w] = __popcll(fm);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) s += wcount[k];
    ws.bcount[b] = s;
    if (b == 0) ws.misc[0] = ev_count ? *ev_count : 0;
  }
}

using ExplicitFn = void (*)(const ClipDev*, int, int, float*, Workspace, const int64_t*);

template <int F>
constexpr ExplicitFn pick(bool f16) {
  return f16 ? explicit_flag_kernel<F, true> : explicit_flag_kernel<F, false>;
}

ExplicitFn explicit_kernel(int F, bool f16) {
  switch (F) {
    case 1: return pick<1>(f16);
    case 2: return pick<2>(f16);
    case 3: return pick<3>(f16);
    case 4: return pick<4>(f16);
    case 5: return pick<5>(f16);
    case 6: return pick<6>(f16);
    case 7: return pick<7>(f16);
    case 8: return pick<8>(f16);
    case 9: return pick<9>(f16);
    case 10: return pick<10>(f16);
    case 11: return pick<11>(f16);
    case 12: return pick<12>(f16);
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_explicit_flag(const ClipDev* clips, int nclips, int64_t nblk, int t, int F, bool f16,
                                float* dl, const Workspace& ws, const int64_t* ev_count, hipStream_t s) {
  const ExplicitFn k = explicit_kernel(F, f16);
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s, clips, nclips, t, dl, ws,
                     ev_count);
  return hipGetLastError();
}

}  // namespace esim
