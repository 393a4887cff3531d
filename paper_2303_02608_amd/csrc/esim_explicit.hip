// Explicit Delta R thresholds (Sec. 2.2: eq. (7) and the R of eq. (4) as window
// sums, instead of the closed form of Prop. 1).
//
// In bandwidth-scaled regressors v (theta_j = beta_j h b_j) the stored plane
// predicts alpha + theta^T v, and over a window of frame tt about the centre
// (p, tt) a sample's residual is r_i = y_i - alpha - theta^T v_i.
//
//   moments_*_kernel      when a model is stored (frame t, uniform over the
//                         launch): W, sum w r, sum w r^2 over the plane's own
//                         window -> rmom = (R, m1 = sum w r / W).  Dense: one
//                         lane per pixel, row-major window walk (a wave reads
//                         64 neighbouring pixels of a row); work lists
//                         (scattered pixels): 16 lanes per item, one window
//                         column each, summed with DPP.
//   explicit_flag_kernel  per pixel at frame t, with d = beta^T (x_hat^c - x^c)
//                         over the F buffer channels:
//                           last-event window: the samples stay those of t_ref
//                           and every translated residual is r_i + d, so
//                           R_hat = R + 2 d m1 + d^2 and the mean is m1 + d;
//                           frame t's window: W, sum w r_hat, sum w r_hat^2
//                           summed over the window of frame t about x_hat^c
//                           (row-major walk);
//                         Delta R = |R_hat - R|; flag when Delta R >= C^2;
//                         dl = s sqrt(Delta R), s the sign of the mean (-1 when
//                         0).  Fills the ballots and block counts of the
//                         closed-form flag kernel (same block layout), so the
//                         same scatter compacts it.
// Sums in FP64; weights in FP32 from the regression's window loop.
#include <cmath>
#include <cstdint>

#include "esim_compact.h"
#include "esim_internal.h"
#include "esim_wlr.h"

namespace esim {
namespace {

// The stored plane of pixel p in scaled regressors.
template <int F>
struct Plane {
  double alpha, thx, thy, th[F];
};

template <int F>
__device__ __forceinline__ void load_plane(const ClipDev& C, int64_t p, Plane<F>& P) {
  P.alpha = C.st_alpha[p];
  P.thx = static_cast<double>(C.st_bxy[p]) / C.sf[0];
  P.thy = static_cast<double>(C.st_bxy[C.HW + p]) / C.sf[1];
#pragma unroll
  for (int f = 0; f < F; ++f) P.th[f] = static_cast<double>(C.st_beta[f * C.HW + p]) / C.sf[2 + f];
}

// W, sum w r, sum w r^2 of the plane over the window of frame tt about the
// centre (pix, tt) (weights and v about that centre's feature vector); with
// L > 1 lane j of the item's L-lane group takes the columns j, j + L, ...
// and the sums are of those columns.
template <int F, bool F16, int L = 1>
__device__ __forceinline__ void window_sums(const ClipDev& C, int64_t pix, int tt, bool active,
                                            const Plane<F>& P, double& sw, double& s1, double& s2,
                                            int j = 0) {
  ItemGeom<F, F16, double> g;
  make_geom(g, C, pix, tt, max(0, tt - C.tr), min(C.T, tt + C.tr + 1), active);
  double base = P.alpha;                  // alpha + th_x v_x of the column pass
  sw = s1 = s2 = 0.0;
  window_loop<F, L>(
      g, j, [&](double vx) { base = fma(P.thx, vx, P.alpha); },
      [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
        double pr = fma(P.thy, vy, base);
#pragma unroll
        for (int f = 0; f < F; ++f) pr = fma(P.th[f], v[f], pr);
        const double r = yd - pr;
        const double wr = w * r;
        sw += w;
        s1 += wr;
        s2 = fma(wr, r, s2);
      },
      [&](double) {});
}

// The same sums with one lane per pixel, walking the window row by row
// (columns innermost): the 64 lanes of a wave read 64 neighbouring pixels of
// one row, and the 2r + 1 shifted reads of that row hit the same cache lines,
// where a column-major walk would fetch every row once per column pass.
// Samples outside the image read the centre with weight 0.
template <int F, bool F16>
__device__ __forceinline__ void window_sums_rows(const ClipDev& C, int64_t pix, int tt, bool active,
                                                 const Plane<F>& P, double& sw, double& s1, double& s2) {
  constexpr uint32_t ES = F16 ? 2u : 4u;
  constexpr double K = kHalfLog2e;
  const int W = C.W, H = C.H, r = C.r;
  const uint32_t HW = static_cast<uint32_t>(C.HW);
  const int f0 = max(0, tt - C.tr), f1 = min(C.T, tt + C.tr + 1);
  const __amdgpu_buffer_rsrc_t ry =
      make_rsrc(C.y + static_cast<uint64_t>(f0) * HW, static_cast<uint64_t>(f1 - f0) * HW * 4u);
  const __amdgpu_buffer_rsrc_t rf =
      make_rsrc(static_cast<const char*>(C.feat) + static_cast<uint64_t>(f0) * F * HW * ES,
                static_cast<uint64_t>(f1 - f0) * F * HW * ES);
  const int py = static_cast<int>(pix / W), px = static_cast<int>(pix - static_cast<int64_t>(py) * W);
  const uint32_t fc = static_cast<uint32_t>(tt - f0);
  double sf[F], xcs[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    sf[f] = C.sf[2 + f];
    xcs[f] = static_cast<double>(ld_feat<F16>(rf, (fc * F * HW + static_cast<uint32_t>(pix)) * ES,
                                              f * HW * ES)) * sf[f];
  }
  const double vxs = C.sf[0] / r, vys = C.sf[1] / r;
  sw = s1 = s2 = 0.0;
  for (int fr = 0; fr < f1 - f0; ++fr) {
    for (int dy = -r; dy <= r; ++dy) {
      const int row = py + dy;
      const bool row_ok = active && row >= 0 && row < H;
      const double vy = dy * vys;
      const double ky = K * vy * vy;
      const double by = fma(P.thy, vy, P.alpha);
#pragma unroll 3
      for (int dx = -r; dx <= r; ++dx) {
        const int col = px + dx;
        const bool ok = row_ok && col >= 0 && col < W;
        // frame (relative to f0) and pixel of the sample, or the centre
        const uint32_t fs = ok ? static_cast<uint32_t>(fr) : fc;
        const uint32_t ps = ok ? static_cast<uint32_t>(row * W + col) : static_cast<uint32_t>(pix);
        const uint32_t fe = fs * F * HW + ps;
        const float yv = ld_f32(ry, (fs * HW + ps) * 4u, 0);
        double q = 0.0, pr = fma(P.thx, dx * vxs, by);
#pragma unroll
        for (int f = 0; f < F; ++f) {
          const double v = fma(static_cast<double>(ld_feat<F16>(rf, fe * ES, f * HW * ES)), sf[f], -xcs[f]);
          q = fma(v, v, q);
          pr = fma(P.th[f], v, pr);
        }
        const double vx = dx * vxs;
        const float ew = __builtin_amdgcn_exp2f(static_cast<float>(fma(q, K, fma(K * vx, vx, ky))));
        const double w = ok ? static_cast<double>(ew) : 0.0;
        const double res = static_cast<double>(yv) - pr;
        const double wr = w * res;
        sw += w;
        s1 += wr;
        s2 = fma(wr, res, s2);
      }
    }
  }
}

// Work-list form: L lanes per item over the regression's column-major loop.
template <int F, bool F16, int L>
__device__ __forceinline__ void store_moments(const ClipDev& C, int64_t p, int t, bool active, int j) {
  Plane<F> P;
  load_plane<F>(C, p, P);
  double sw, s1, s2;
  window_sums<F, F16, L>(C, p, t, active, P, sw, s1, s2, j);
  sw = group_sum<L>(sw);
  s1 = group_sum<L>(s1);
  s2 = group_sum<L>(s2);
  if (active && j == 0) {
    C.st_rmom[p] = static_cast<float>(s2 / sw);
    C.st_rmom[C.HW + p] = static_cast<float>(s1 / sw);
  }
}

constexpr int kListLanes = 16;                   // lanes per work-list item
constexpr int kItemsPerBlock = kBlock / kListLanes;

// Dense: every pixel of the plan, in the flag kernel's block layout.
template <int F, bool F16>
__global__ void __launch_bounds__(kBlock)
moments_dense_kernel(const ClipDev* __restrict__ clips, int nclips, int t) {
  const int64_t b = blockIdx.x;
  const ClipDev& C = clips[block_clip(clips, nclips, b)];
  const int64_t p = (b - C.blk_off) * kBlock + threadIdx.x;
  if (t < 0 || t >= C.T) return;                 // uniform in the block
  const bool active = p < C.HW;
  const int64_t pc = active ? p : 0;
  Plane<F> P;
  load_plane<F>(C, pc, P);
  double sw, s1, s2;
  window_sums_rows<F, F16>(C, pc, t, active, P, sw, s1, s2);
  if (active) {
    C.st_rmom[p] = static_cast<float>(s2 / sw);
    C.st_rmom[C.HW + p] = static_cast<float>(s1 / sw);
  }
}

// Work list: kListLanes lanes per item, grid-stride over the items.
template <int F, bool F16>
__global__ void __launch_bounds__(kBlock)
moments_list_kernel(const ClipDev* __restrict__ clips, int nclips, int t, const int64_t* __restrict__ worklist,
                    const int32_t* __restrict__ count, int64_t max_items) {
  const int64_t n = max(static_cast<int64_t>(0), min(static_cast<int64_t>(count[0]), max_items));
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kItemsPerBlock;
  const int j = threadIdx.x % kListLanes;
  for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * kItemsPerBlock; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x / kListLanes;
    const int64_t it = i < n ? worklist[i] : -1;
    const int cl = it < 0 ? -1 : item_clip(it);
    bool pending = it >= 0 && cl < nclips;
    // one pass per clip present in the wave (almost always one), so that the
    // clip descriptor is wave-uniform
    while (__ballot(pending)) {
      const int src = __ffsll(static_cast<unsigned long long>(__ballot(pending))) - 1;
      const int cw = __builtin_amdgcn_readfirstlane(__shfl(cl, src));
      const ClipDev& C = clips[cw];
      const bool mine = pending && cl == cw;
      const int64_t p = mine ? item_pixel(it) : 0;
      const bool active = mine && p < C.HW && t < C.T;
      store_moments<F, F16, kListLanes>(C, active ? p : 0, t < C.T ? t : 0, active, j);
      pending = pending && !mine;
    }
  }
}

template <int F, bool F16, bool NEW>
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
    double d = 0.0;                             // beta^T (x_hat^c - x^c)
    for (int f = 0; f < F; ++f)
      d = fma(static_cast<double>(C.st_beta[f * C.HW + pc]),
              static_cast<double>(feat_value(C, t, f, pc)) - C.st_xref[f * C.HW + pc], d);
    const double R = C.st_rmom[pc], m1 = C.st_rmom[C.HW + pc];
    double dR, mean;
    if constexpr (NEW) {
      Plane<F> P;
      load_plane<F>(C, pc, P);
      double sw, s1, s2;
      window_sums_rows<F, F16>(C, pc, t, in, P, sw, s1, s2);
      dR = s2 / sw - R;
      mean = s1 / sw;
    } else {
      dR = d * (2.0 * m1 + d);
      mean = m1 + d;
    }
    if (in) {
      const double a = fabs(dR);
      flag = a >= C.C * C.C;
      pos = mean > 0.0;
      if (dl) dl[C.pix_off + p] = static_cast<float>(pos ? sqrt(a) : -sqrt(a));
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
    int64_t s = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) s += wcount[k];
    ws.bcount[b] = s;
    if (b == 0) ws.misc[0] = ev_count ? *ev_count : 0;
  }
}

using ExplicitFn = void (*)(const ClipDev*, int, int, float*, Workspace, const int64_t*);
using MomentsDenseFn = void (*)(const ClipDev*, int, int);
using MomentsListFn = void (*)(const ClipDev*, int, int, const int64_t*, const int32_t*, int64_t);

template <int F>
struct Pick {
  static ExplicitFn flag(bool f16, bool nw) {
    return f16 ? (nw ? explicit_flag_kernel<F, true, true> : explicit_flag_kernel<F, true, false>)
               : (nw ? explicit_flag_kernel<F, false, true> : explicit_flag_kernel<F, false, false>);
  }
  static MomentsDenseFn dense(bool f16) {
    return f16 ? moments_dense_kernel<F, true> : moments_dense_kernel<F, false>;
  }
  static MomentsListFn list(bool f16) {
    return f16 ? moments_list_kernel<F, true> : moments_list_kernel<F, false>;
  }
};

template <template <int> class P, class Fn>
auto by_f(int F, Fn&& fn) -> decltype(fn(P<1>{})) {
  switch (F) {
    case 1: return fn(P<1>{});
    case 2: return fn(P<2>{});
    case 3: return fn(P<3>{});
    case 4: return fn(P<4>{});
    case 5: return fn(P<5>{});
    case 6: return fn(P<6>{});
    case 7: return fn(P<7>{});
    case 8: return fn(P<8>{});
    case 9: return fn(P<9>{});
    case 10: return fn(P<10>{});
    case 11: return fn(P<11>{});
    case 12: return fn(P<12>{});
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_explicit_flag(const ClipDev* clips, int nclips, int64_t nblk, int t, int F, bool f16,
                                int thr, float* dl, const Workspace& ws, const int64_t* ev_count,
                                hipStream_t s) {
  const bool nw = thr == ESIM_THRESHOLD_NEW_WINDOW;
  const ExplicitFn k = by_f<Pick>(F, [&](auto p) { return decltype(p)::flag(f16, nw); });
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s, clips, nclips, t, dl, ws,
                     ev_count);
  return hipGetLastError();
}

hipError_t launch_moments(const ClipDev* clips, int nclips, int64_t nblk, int t, int F, bool f16,
                          const int64_t* worklist, const int32_t* count, int64_t max_items,
                          hipStream_t s) {
  if (!worklist) {
    const MomentsDenseFn k = by_f<Pick>(F, [&](auto p) { return decltype(p)::dense(f16); });
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s, clips, nclips, t);
    return hipGetLastError();
  }
  const MomentsListFn k = by_f<Pick>(F, [&](auto p) { return decltype(p)::list(f16); });
  if (!k) return hipErrorInvalidValue;
  int64_t blocks = (max_items + kItemsPerBlock - 1) / kItemsPerBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, clips, nclips, t, worklist,
                     count, max_items);
  return hipGetLastError();
}

}  // namespace esim
