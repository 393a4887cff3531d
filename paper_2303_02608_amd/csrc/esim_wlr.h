// Window geometry and the streamed window loop of one weighted local
// regression (Sec. 2.1, eqs. 4-5), shared by the forward and adjoint kernels.
//
// Regressors are kept in bandwidth-scaled units v_j = u_j / (h b_j): the
// weight exponent is then sum_j v_j^2 (eq. 5 with a Gaussian fall-off) and
// the fit in v equals the fit in u with beta_j = theta_j / (h b_j) and the
// ridge scaled to lambda / (h b_j)^2.
//
// The L lanes of an item split the window columns (lane j takes dx = -r + j,
// -r + j + L, ...); for one column pass v_x is constant in the lane.  The rows
// (dt, dy) of a column are software-pipelined in registers (window_loop): the
// loads of a row are issued two rows ahead of its use.  Rows outside the image
// (or past the last row) read the valid centre pixel and get weight 0.
#pragma once

#include <type_traits>

#include "esim_internal.h"

namespace esim {

constexpr double kHalfLog2e = -0.72134752044448170368;  // -log2(e) / 2

template <int F, bool F16, class Real = double>
struct ItemGeom {
  static constexpr uint32_t ES = F16 ? 2u : 4u;
  __amdgpu_buffer_rsrc_t ry, rf;
  uint32_t HW, vcen_f, vcen_y;
  int W, H, T, r, tr, px, py, fc, tt, dt_lo, dt_hi;
  bool active;
  Real sf[F + 2];
  Real xcs[F];
  Real vx_step, vy_step;
};

// Fills the geometry of the item at (pix, tt) of clip C.  f0/f1 are the frames
// the buffer resources cover (a uniform frame's window, or the whole clip).
template <int F, bool F16, class Real>
__device__ __forceinline__ void make_geom(ItemGeom<F, F16, Real>& g, const ClipDev& C, int64_t pix,
                                          int tt, int f0, int f1, bool active) {
  constexpr uint32_t ES = ItemGeom<F, F16, Real>::ES;
  g.W = C.W;
  g.H = C.H;
  g.T = C.T;
  g.r = C.r;
  g.tr = C.tr;
  g.HW = static_cast<uint32_t>(C.HW);
  g.active = active;
  g.tt = tt;
  g.ry = make_rsrc(C.y + static_cast<uint64_t>(f0) * g.HW, static_cast<uint64_t>(f1 - f0) * g.HW * 4u);
  g.rf = make_rsrc(static_cast<const char*>(C.feat) + static_cast<uint64_t>(f0) * F * g.HW * ES,
                   static_cast<uint64_t>(f1 - f0) * F * g.HW * ES);
  g.py = static_cast<int>(pix / g.W);
  g.px = static_cast<int>(pix - static_cast<int64_t>(g.py) * g.W);
  g.fc = tt - f0;
  g.vcen_f = (static_cast<uint32_t>(g.fc) * F * g.HW + static_cast<uint32_t>(pix)) * ES;
  g.vcen_y = (static_cast<uint32_t>(g.fc) * g.HW + static_cast<uint32_t>(pix)) * 4u;
#pragma unroll
  for (int d = 0; d < F + 2; ++d) g.sf[d] = static_cast<Real>(C.sf[d]);
#pragma unroll
  for (int f = 0; f < F; ++f)
    g.xcs[f] = static_cast<Real>(ld_feat<F16>(g.rf, g.vcen_f, f * g.HW * ES)) * g.sf[2 + f];
  g.vx_step = static_cast<Real>(C.sf[0] / g.r);
  g.vy_step = static_cast<Real>(C.sf[1] / g.r);
  g.dt_lo = max(-g.tr, -tt);
  g.dt_hi = min(g.tr, g.T - 1 - tt);
}

// Runs the window of one item in lane j of its L-lane group.
//   pass_begin(vx)                      before each column pass
//   sample(w, yd, v[F], vy, dx, dt, dy, ok) for every row of the window in
//                                       the lane's column; ok is false (and
//                                       w = 0) outside the image and for idle
//                                       columns
//   pass_end(vx)                        after each column pass
//
// The rows of a column form a three-stage software pipeline: the loads of row
// k+2 are in flight while the weight of row k+1 is computed and row k is
// accumulated, so the exponential's latency overlaps independent Gram work.
// The loop takes two rows per iteration (see the loop for an odd row count).
// Row offsets advance by uniform (SGPR) amounts; only the validity test and
// the select are per lane.
//
// FULL: the caller guarantees that the window of every lane's item lies
// entirely inside the image and the clip (|dx|, |dy| <= r and |dt| <= tr all
// valid; lanes without an item carry the geometry of one that has).  Then no
// row needs a validity test or an address select: a lane's column offset is
// fixed for the pass, the row offset is uniform, and only the lane's own
// weight switch (no item, or the idle column of a lane group wider than the
// window) remains.
template <int F, int L, bool F16, class Real, bool FULL = false, class PassBegin, class Sample,
          class PassEnd>
__device__ __forceinline__ void window_loop(const ItemGeom<F, F16, Real>& g, int j,
                                            PassBegin&& pass_begin, Sample&& sample,
                                            PassEnd&& pass_end) {
  constexpr uint32_t ES = ItemGeom<F, F16, Real>::ES;
  constexpr Real K = static_cast<Real>(kHalfLog2e);
  const int r = g.r;
  const int span = 2 * r + 1;
  // FULL: every lane's window spans 2 tr + 1 frames (a uniform count, so the
  // loop bounds and row offsets below stay scalar)
  const int nt = FULL ? 2 * g.tr + 1 : g.dt_hi - g.dt_lo + 1;
  const int nrows = nt * span;
  const int npass = (span + L - 1) / L;
  // per-lane valid row range of the item (rows inside the image)
  const int dy_lo = -min(r, g.py), dy_hi = min(r, g.H - 1 - g.py);
  const uint32_t WES = static_cast<uint32_t>(g.W) * ES, W4 = static_cast<uint32_t>(g.W) * 4u;
  const uint32_t FES = static_cast<uint32_t>(F) * g.HW * ES, HW4 = g.HW * 4u;
  for (int k = 0; k < npass; ++k) {
    const int dx = -r + j + k * L;
    // FULL: an idle column reads the window's last column (weight 0)
    const int col = g.px + (FULL ? min(dx, r) : dx);
    const bool col_ok = g.active && dx <= r && col >= 0 && col < g.W;
    const Real vx = static_cast<Real>(dx) * g.vx_step;
    const Real kx = K * vx * vx;
    pass_begin(vx);
    // offsets of the window's first row (dt_lo, -r) in this column; rows above
    // the image wrap as unsigned and are never used (the select takes the
    // centre instead)
    const uint32_t vf_base = (static_cast<uint32_t>(g.fc + g.dt_lo) * F * g.HW +
                              static_cast<uint32_t>((g.py - r) * g.W + col)) * ES;
    const uint32_t vy_base = (static_cast<uint32_t>(g.fc + g.dt_lo) * g.HW +
                              static_cast<uint32_t>((g.py - r) * g.W + col)) * 4u;
    int ldt = 0, ldy = 0;          // next row to load, relative to (dt_lo, -r)
    auto load_row = [&](float& yv, float (&fv)[F]) -> bool {
      if constexpr (FULL) {
        // rows past the window (the pipeline's look-ahead) repeat the last
        // row; their weights are never used
        const bool in = ldt < nt;
        const uint32_t lt = static_cast<uint32_t>(in ? ldt : nt - 1);
        const uint32_t ly = static_cast<uint32_t>(in ? ldy : span - 1);
        const uint32_t sof = lt * FES + ly * WES;
        const uint32_t soy = lt * HW4 + ly * W4;
        yv = ld_f32(g.ry, vy_base, soy);
#pragma unroll
        for (int f = 0; f < F; ++f) fv[f] = ld_feat<F16>(g.rf, vf_base, sof + f * g.HW * ES);
        if (++ldy == span) {
          ldy = 0;
          ++ldt;
        }
        return col_ok;
      }
      const int dy = ldy - r;
      const bool ok = (ldt <= g.dt_hi - g.dt_lo) & col_ok & (dy >= dy_lo) & (dy <= dy_hi);
      const uint32_t sof = static_cast<uint32_t>(ldt) * FES + static_cast<uint32_t>(ldy) * WES;
      const uint32_t soy = static_cast<uint32_t>(ldt) * HW4 + static_cast<uint32_t>(ldy) * W4;
      const uint32_t vf = ok ? vf_base + sof : g.vcen_f;
      const uint32_t vy = ok ? vy_base + soy : g.vcen_y;
      yv = ld_f32(g.ry, vy, 0);
#pragma unroll
      for (int f = 0; f < F; ++f) fv[f] = ld_feat<F16>(g.rf, vf, f * g.HW * ES);
      if (++ldy == span) {
        ldy = 0;
        ++ldt;
      }
      return ok;
    };
    struct Wt {
      Real w, yd, vy, v[F];
      int dt, dy;
      bool ok;
    };
    int cdt = FULL ? -g.tr : g.dt_lo, cdy = -r;   // next row to weigh
    auto weigh = [&](float yv, const float (&fv)[F], bool ok, Wt& o) {
      o.dy = cdy;
      o.dt = cdt;
      o.ok = ok;
      if (++cdy > r) {
        cdy = -r;
        ++cdt;
      }
      o.vy = static_cast<Real>(o.dy) * g.vy_step;
      Real s0 = 0, s1 = 0;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        o.v[f] = fma(static_cast<Real>(fv[f]), g.sf[2 + f], -g.xcs[f]);
        if (f & 1) s1 = fma(o.v[f], o.v[f], s1);
        else s0 = fma(o.v[f], o.v[f], s0);
      }
      const Real arg = fma(s0 + s1, K, fma(K * o.vy, o.vy, kx));
      const float e = __builtin_amdgcn_exp2f(static_cast<float>(arg));
      o.w = static_cast<Real>(ok ? e : 0.0f);
      o.yd = static_cast<Real>(yv);
    };
    auto use = [&](const Wt& o) { sample(o.w, o.yd, o.v, o.vy, dx, o.dt, o.dy, o.ok); };
    // pipeline prologue: rows 0 and 1 loaded, row 0 weighed, row 2 in flight
    float yA, fA[F], yB, fB[F];
    bool okA = load_row(yA, fA);
    bool okB = load_row(yB, fB) & (1 < nrows);
    Wt wA, wB;
    weigh(yA, fA, okA, wA);
    okA = load_row(yA, fA) & (2 < nrows);
    // FP64: pairs of rows, then an odd last row alone.  FP32 (the compensated
    // variant, whose per-sample body is larger): pairs only, an odd count
    // ending on a weight-0 padding row, which measured faster there.
    constexpr bool kPeel = std::is_same<Real, double>::value;
    const int qend = kPeel ? nrows - 1 : nrows;
    int q = 0;
#pragma unroll 1
    for (; q < qend; q += 2) {
      // wA = row q (weighed), raw B = row q+1, raw A = row q+2
      weigh(yB, fB, okB, wB);
      okB = load_row(yB, fB) & (q + 3 < nrows);
      use(wA);
      weigh(yA, fA, okA, wA);
      okA = load_row(yA, fA) & (q + 4 < nrows);
      use(wB);
    }
    if constexpr (kPeel) {
      if (q < nrows) use(wA);     // odd row count: the last row alone
    }
    pass_end(vx);
  }
}

// The window of one item whose window lies entirely inside the image and the
// clip (the FULL case of window_loop), with a deeper load pipeline: a ring of
// R rows in registers.  Each step weighs and accumulates the oldest row and
// issues the loads of the row R ahead into its slot, so every load has R - 1
// rows of work to arrive (the window rows of scattered work-list items often
// miss the L2).  Same calls and order of samples as window_loop; sample()
// receives dt = dy = 0 (unused by its callers).
template <int F, int L, bool F16, int R, class PassBegin, class Sample, class PassEnd>
__device__ __forceinline__ void window_loop_ring(const ItemGeom<F, F16, double>& g, int j,
                                                 PassBegin&& pass_begin, Sample&& sample,
                                                 PassEnd&& pass_end) {
  constexpr uint32_t ES = ItemGeom<F, F16, double>::ES;
  constexpr double K = kHalfLog2e;
  const int r = g.r;
  const int span = 2 * r + 1;
  const int nt = 2 * g.tr + 1;
  const int nrows = nt * span;
  const int npass = (span + L - 1) / L;
  const uint32_t WES = static_cast<uint32_t>(g.W) * ES, W4 = static_cast<uint32_t>(g.W) * 4u;
  const uint32_t FES = static_cast<uint32_t>(F) * g.HW * ES, HW4 = g.HW * 4u;
  for (int k = 0; k < npass; ++k) {
    const int dx = -r + j + k * L;
    const int col = g.px + min(dx, r);        // an idle column reads the last one (weight 0)
    const bool col_ok = g.active && dx <= r;
    const double vx = static_cast<double>(dx) * g.vx_step;
    const double kx = K * vx * vx;
    pass_begin(vx);
    const uint32_t vf_base = (static_cast<uint32_t>(g.fc - g.tr) * F * g.HW +
                              static_cast<uint32_t>((g.py - r) * g.W + col)) * ES;
    const uint32_t vy_base = (static_cast<uint32_t>(g.fc - g.tr) * g.HW +
                              static_cast<uint32_t>((g.py - r) * g.W + col)) * 4u;
    int ldt = 0, ldy = 0;                     // next row to load (uniform)
    auto load_next = [&](float& yv, float (&fv)[F]) {
      // rows past the window repeat the last row; they are never consumed
      const bool in = ldt < nt;
      const uint32_t lt = static_cast<uint32_t>(in ? ldt : nt - 1);
      const uint32_t ly = static_cast<uint32_t>(in ? ldy : span - 1);
      yv = ld_f32(g.ry, vy_base, lt * HW4 + ly * W4);
#pragma unroll
      for (int f = 0; f < F; ++f) fv[f] = ld_feat<F16>(g.rf, vf_base, lt * FES + ly * WES + f * g.HW * ES);
      if (++ldy == span) {
        ldy = 0;
        ++ldt;
      }
    };
    int cdy = -r;                             // next row to consume (uniform)
    auto consume = [&](float yv, const float (&fv)[F]) {
      const double vy = static_cast<double>(cdy) * g.vy_step;
      if (++cdy > r) cdy = -r;
      double v[F], s0 = 0, s1 = 0;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        v[f] = fma(static_cast<double>(fv[f]), g.sf[2 + f], -g.xcs[f]);
        if (f & 1) s1 = fma(v[f], v[f], s1);
        else s0 = fma(v[f], v[f], s0);
      }
      const double arg = fma(s0 + s1, K, fma(K * vy, vy, kx));
      const float e = __builtin_amdgcn_exp2f(static_cast<float>(arg));
      sample(static_cast<double>(col_ok ? e : 0.0f), static_cast<double>(yv), v, vy, dx, 0, 0, col_ok);
    };
    float ys[R], fs[R][F];
#pragma unroll
    for (int i = 0; i < R; ++i) load_next(ys[i], fs[i]);
    int q = 0;
#pragma unroll 1
    for (; q + R <= nrows; q += R) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        consume(ys[i], fs[i]);
        load_next(ys[i], fs[i]);
      }
    }
    // the last nrows - q rows sit in slots 0 .. nrows - q - 1
#pragma unroll
    for (int i = 0; i + 1 < R; ++i)
      if (q + i < nrows) consume(ys[i], fs[i]);
    pass_end(vx);
  }
}

// Normal equations of one item, accumulated per lane.  Within a column pass
// v_x is constant in a lane, so the entries with a v_x factor are not summed
// per sample: they are v_x times sums of the first-row entries (formed once per
// item by the one-pass form, once per pass by the pass-snapshot form).
template <int F, class Real = double>
struct Gram {
  static constexpr int NA = F * (F + 1) / 2;
  Real SW, A0y, g0, A0f[F];
  Real A0x, Axx, Axy, gx, Axf[F];
  Real Ayy, gy, Syy, Ayf[F], gf[F], Aff[NA];
  Real qW, qY, qG, qF[F];                 // first-row totals at the pass start

  // One-pass form (every lane owns a single window column): the column sums
  // are the totals, and the entries with a v_x factor are formed once after
  // the window loop, so they are not live during it.
  __device__ __forceinline__ void zero_onepass() {
    SW = A0y = g0 = Ayy = gy = Syy = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) A0f[f] = Ayf[f] = gf[f] = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) Aff[k] = 0;
  }
  __device__ __forceinline__ void add_onepass(Real w, Real yd, const Real (&v)[F], Real vy) {
    const Real wy = w * yd;
    const Real wvy = w * vy;
    SW += w;
    A0y += wvy;
    g0 += wy;
    Ayy = fma(wvy, vy, Ayy);
    gy = fma(wy, vy, gy);
    Syy = fma(wy, yd, Syy);
    int qq = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const Real wz = w * v[f];
      A0f[f] += wz;
      Ayf[f] = fma(wvy, v[f], Ayf[f]);
      gf[f] = fma(wz, yd, gf[f]);
#pragma unroll
      for (int e = f; e < F; ++e) {
        Aff[qq] = fma(wz, v[e], Aff[qq]);
        ++qq;
      }
    }
  }
  __device__ __forceinline__ void fold_onepass(Real vx) {
    A0x = vx * SW;
    Axx = vx * vx * SW;
    Axy = vx * A0y;
    gx = vx * g0;
#pragma unroll
    for (int f = 0; f < F; ++f) Axf[f] = vx * A0f[f];
  }
  // Pass-snapshot form: the window loop accumulates as the one-pass form; at
  // each pass start the first-row totals (W, v_y, y and feature sums) are
  // copied, and at its end the entries with a v_x factor take v_x times the
  // pass's increment of them.  The snapshot and the v_x entries are only
  // touched once per pass, so the loop's live accumulators are the one-pass
  // ones.  (The increment is a difference of two FP64 totals of at most
  // 2r + 1 passes: its rounding is of the order of the totals' own.)
  __device__ __forceinline__ void zero_snap() {
    zero_onepass();
    A0x = Axx = Axy = gx = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) Axf[f] = 0;
  }
  __device__ __forceinline__ void pass_begin_snap() {
    qW = SW;
    qY = A0y;
    qG = g0;
#pragma unroll
    for (int f = 0; f < F; ++f) qF[f] = A0f[f];
  }
  __device__ __forceinline__ void pass_end_snap(Real vx) {
    const Real dW = SW - qW;
    A0x = fma(vx, dW, A0x);
    Axx = fma(vx * vx, dW, Axx);
    Axy = fma(vx, A0y - qY, Axy);
    gx = fma(vx, g0 - qG, gx);
#pragma unroll
    for (int f = 0; f < F; ++f) Axf[f] = fma(vx, A0f[f] - qF[f], Axf[f]);
  }
  // Applies one DPP butterfly step to every total; the steps run in sequence
  // over all totals (step-major), so consecutive DPP reads never depend on
  // the previous instruction.
  template <int CTRL>
  __device__ __forceinline__ void dpp_step() {
    auto st = [](Real& v) { v += dpp_d<CTRL>(v); };
    st(SW);
    st(A0y);
    st(g0);
    st(A0x);
    st(Axx);
    st(Axy);
    st(gx);
    st(Ayy);
    st(gy);
    st(Syy);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      st(A0f[f]);
      st(Axf[f]);
      st(Ayf[f]);
      st(gf[f]);
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) st(Aff[k]);
  }
  template <int L>
  __device__ __forceinline__ void lane_sum() {
    if constexpr (L >= 2) dpp_step<0xB1>();
    if constexpr (L >= 4) dpp_step<0x4E>();
    if constexpr (L >= 8) dpp_step<0x141>();
    if constexpr (L >= 16) dpp_step<0x140>();
  }
};

// Neumaier-compensated accumulation: (hi, lo) += x.
__device__ __forceinline__ void neumaier(float& hi, float& lo, float x) {
  const float t = hi + x;
  lo += fabsf(hi) >= fabsf(x) ? (hi - t) + x : (x - t) + hi;
  hi = t;
}

// FP32 normal equations with block-compensated sums: every sample updates
// plain FP32 partials of the current column pass (a block of 2tr+1 times
// 2r+1 samples); at the end of the pass each partial is added to a
// Neumaier-compensated (hi, lo) total, and lane groups merge their totals
// with error-free two-sums.  Values are read back as hi + lo.
template <int F>
struct GramC {
  static constexpr int NA = F * (F + 1) / 2;
  static constexpr int NQ = F + 3;             // qW, qY, qG, qF[F]
  static constexpr int ND = 3 + 2 * F + NA;    // Ayy, gy, Syy, Ayf[F], gf[F], Aff[NA]
  static constexpr int NT = 2 * NQ + 1 + ND;   // q totals, x folds, Axx, directs
  float q[NQ], d[ND];
  float hi[NT], lo[NT];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < NT; ++k) hi[k] = lo[k] = 0.0f;
  }
  __device__ __forceinline__ void pass_begin() {
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < ND; ++k) d[k] = 0.0f;
  }
  __device__ __forceinline__ void add(float w, float yd, const float (&v)[F], float vy) {
    const float wy = w * yd;
    const float wvy = w * vy;
    q[0] += w;
    q[1] += wvy;
    q[2] += wy;
    d[0] = fmaf(wvy, vy, d[0]);
    d[1] = fmaf(wy, vy, d[1]);
    d[2] = fmaf(wy, yd, d[2]);
    int qq = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const float wz = w * v[f];
      q[3 + f] += wz;
      d[3 + f] = fmaf(wvy, v[f], d[3 + f]);
      d[3 + F + f] = fmaf(wz, yd, d[3 + F + f]);
#pragma unroll
      for (int e = f; e < F; ++e) {
        d[3 + 2 * F + qq] = fmaf(wz, v[e], d[3 + 2 * F + qq]);
        ++qq;
      }
    }
  }
  __device__ __forceinline__ void pass_end(float vx) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      neumaier(hi[k], lo[k], q[k]);
      neumaier(hi[NQ + k], lo[NQ + k], vx * q[k]);
    }
    neumaier(hi[2 * NQ], lo[2 * NQ], vx * vx * q[0]);
#pragma unroll
    for (int k = 0; k < ND; ++k) neumaier(hi[2 * NQ + 1 + k], lo[2 * NQ + 1 + k], d[k]);
  }
  template <int L>
  __device__ __forceinline__ void lane_sum() {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      float h = hi[k], l = lo[k];
      auto step = [&](float h2, float l2) {
        const float s = h + h2;
        const float bb = s - h;
        const float err = (h - (s - bb)) + (h2 - bb);
        h = s;
        l = l + l2 + err;
      };
      if constexpr (L >= 2) step(dpp_f<0xB1>(h), dpp_f<0xB1>(l));
      if constexpr (L >= 4) step(dpp_f<0x4E>(h), dpp_f<0x4E>(l));
      if constexpr (L >= 8) step(dpp_f<0x141>(h), dpp_f<0x141>(l));
      if constexpr (L >= 16) step(dpp_f<0x140>(h), dpp_f<0x140>(l));
      hi[k] = h;
      lo[k] = l;
    }
  }
  // Totals in the Gram layout, as Real (hi + lo evaluated in Real).
  template <class Real>
  __device__ __forceinline__ void values(Gram<F, Real>& G) const {
    auto v = [&](int k) { return static_cast<Real>(hi[k]) + static_cast<Real>(lo[k]); };
    G.SW = v(0);
    G.A0y = v(1);
    G.g0 = v(2);
    G.A0x = v(NQ + 0);
    G.Axy = v(NQ + 1);
    G.gx = v(NQ + 2);
    G.Axx = v(2 * NQ);
    G.Ayy = v(2 * NQ + 1);
    G.gy = v(2 * NQ + 2);
    G.Syy = v(2 * NQ + 3);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      G.A0f[f] = v(3 + f);
      G.Axf[f] = v(NQ + 3 + f);
      G.Ayf[f] = v(2 * NQ + 4 + f);
      G.gf[f] = v(2 * NQ + 4 + F + f);
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) G.Aff[k] = v(2 * NQ + 4 + 2 * F + k);
  }
};

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Wave-group iteration with XCD affinity.  Workgroups are dispatched to the
// nxcd XCDs round-robin by block index, so block b runs on XCD b % nxcd.  When
// the grid is a multiple of nxcd blocks, XCD x walks a contiguous range of the
// groups (the x-th of nxcd equal parts, or [xb[x], xb[x + 1]) when a split by
// work is given), which keeps spatially adjacent items (sharing window rows)
// in the same L2; otherwise a plain grid stride is used.
struct GroupIter {
  int64_t g, end, step;
  __device__ __forceinline__ GroupIter(int64_t ngroups, int nxcd, const int64_t* xb = nullptr) {
    const int64_t nblk = gridDim.x;
    const int64_t wib = threadIdx.x / kWave;            // wave in block
    const int64_t wpb = blockDim.x / kWave;
    const int64_t nx = nxcd;
    if (nx > 1 && nblk >= nx && nblk % nx == 0) {
      const int64_t x = blockIdx.x % nx;
      int64_t lo, hi;
      if (xb) {
        lo = xb[x];
        hi = min(ngroups, xb[x + 1]);
      } else {
        const int64_t chunk = (ngroups + nx - 1) / nx;
        lo = x * chunk;
        hi = min(ngroups, (x + 1) * chunk);
      }
      g = lo + (blockIdx.x / nx) * wpb + wib;
      end = hi;
      step = (nblk / nx) * wpb;
    } else {
      g = static_cast<int64_t>(blockIdx.x) * wpb + wib;
      end = ngroups;
      step = nblk * wpb;
    }
  }
  __device__ __forceinline__ bool next(int64_t& out) {
    if (g >= end) return false;
    out = g;
    g += step;
    return true;
  }
};

// Hardware estimates of 1/sqrt(x) and 1/x.
__device__ __forceinline__ double rsq_approx(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float rsq_approx(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rcp_approx(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }

// 1/sqrt(x) refined by two Newton steps from the hardware estimate (each step
// doubles the correct bits; within an ulp or two of the correctly rounded
// value, a short dependent chain instead of the correctly rounded square root
// and divide sequences).
template <class Real>
__device__ __forceinline__ Real rsq_refined(Real x) {
  Real y = rsq_approx(x);
  y = y * fma(Real(-0.5) * x * y, y, Real(1.5));
  y = y * fma(Real(-0.5) * x * y, y, Real(1.5));
  return y;
}

// Solves L L^T x = b with the packed factor (its diagonal holds 1 / L_ii).
template <int P, class Real>
__device__ __forceinline__ void chol_solve(const Real (&M)[P * (P + 1) / 2], const Real (&b)[P],
                                           Real (&x)[P]) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    Real v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= M[tri(i, k)] * x[k];
    x[i] = v * M[tri(i, i)];
  }
#pragma unroll
  for (int i = P - 1; i >= 0; --i) {
    Real v = x[i];
#pragma unroll
    for (int k = i + 1; k < P; ++k) v -= M[tri(k, i)] * x[k];
    x[i] = v * M[tri(i, i)];
  }
}

// In-place packed Cholesky A = L L^T; the diagonal slots receive 1 / L_ii (the
// solves multiply by it), from the refined reciprocal square root of the
// pivot.  A non-positive pivot yields NaN.
template <int P, class Real>
__device__ __forceinline__ void cholesky_inplace(Real (&M)[P * (P + 1) / 2]) {
#pragma unroll
  for (int c = 0; c < P; ++c) {
    Real s = M[tri(c, c)];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= M[tri(c, k)] * M[tri(c, k)];
    Real id = rsq_refined(s);
    id = s > Real(0) ? id : static_cast<Real>(__builtin_nan(""));
    M[tri(c, c)] = id;
#pragma unroll
    for (int i = c + 1; i < P; ++i) {
      Real v = M[tri(i, c)];
#pragma unroll
      for (int k = 0; k < c; ++k) v -= M[tri(i, k)] * M[tri(c, k)];
      M[tri(i, c)] = v * id;
    }
  }
}

// Assembles the W-normalised system in scaled units (unknowns alpha, beta_x,
// beta_y, beta_f..), adds the scaled ridge, factors it in place (packed lower
// Cholesky) and solves for theta.  Returns 1/W.  anorm1 receives the 1-norm of
// the equilibrated matrix S^-1 A S^-1 (S^2 = diag(A), unit diagonal), for the
// condition estimate (equilibrate_factor, hager_inv_norm1).
template <int F, class Real>
__device__ __forceinline__ Real gram_solve(const Gram<F, Real>& G, const ClipDev& C,
                                           Real (&M)[(F + 3) * (F + 4) / 2], Real (&rhs)[F + 3],
                                           Real (&th)[F + 3], Real& anorm1) {
  constexpr int P = F + 3;
  const Real iW = Real(1) / G.SW;
  const Real lam = static_cast<Real>(C.ridge);
  M[tri(0, 0)] = Real(1);
  M[tri(1, 0)] = G.A0x * iW;
  M[tri(2, 0)] = G.A0y * iW;
  M[tri(1, 1)] = G.Axx * iW + lam * static_cast<Real>(C.c2[0]);
  M[tri(2, 1)] = G.Axy * iW;
  M[tri(2, 2)] = G.Ayy * iW + lam * static_cast<Real>(C.c2[1]);
  rhs[0] = G.g0 * iW;
  rhs[1] = G.gx * iW;
  rhs[2] = G.gy * iW;
  {
    int q = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      M[tri(3 + f, 0)] = G.A0f[f] * iW;
      M[tri(3 + f, 1)] = G.Axf[f] * iW;
      M[tri(3 + f, 2)] = G.Ayf[f] * iW;
      rhs[3 + f] = G.gf[f] * iW;
#pragma unroll
      for (int e = f; e < F; ++e) {
        M[tri(3 + e, 3 + f)] = G.Aff[q] * iW + (e == f ? lam * static_cast<Real>(C.c2[2 + f]) : Real(0));
        ++q;
      }
    }
  }
  Real isd[P];
#pragma unroll
  for (int i = 0; i < P; ++i) isd[i] = Real(1) / sqrt(M[tri(i, i)]);
  anorm1 = 0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    Real cs = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) cs += fabs(i >= c ? M[tri(i, c)] : M[tri(c, i)]) * isd[i];
    anorm1 = fmax(anorm1, cs * isd[c]);
  }
  cholesky_inplace<P, Real>(M);
  chol_solve<P, Real>(M, rhs, th);
  return iW;
}


// Turns the packed Cholesky factor of A (diagonal slots holding 1 / L_ii) into
// the factor of the equilibrated As = S^-1 A S^-1, S^2 = diag(A): row i of L
// divided by S_i, with A_ii = sum_k L_ik^2 read off the factor itself.  In
// place; M is no longer A's factor afterwards.  By van der Sluis the rounding
// error of the Cholesky solve is governed by kappa(As), not kappa(A), whose
// diagonal spans the ridge (a constant feature) to 1.
template <int P, class Real>
__device__ __forceinline__ void equilibrate_factor(Real (&M)[P * (P + 1) / 2]) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    // A_ii = L_ii^2 + sum_k L_ik^2, with L_ii = 1 / M_ii (the slot's value)
    const Real lii = rcp_approx(M[tri(i, i)]);
    Real s = lii * lii;
#pragma unroll
    for (int k = 0; k < i; ++k) s += M[tri(i, k)] * M[tri(i, k)];
    // an estimate needs no correctly rounded root: the hardware reciprocal
    // square root (about 1 ulp) keeps this short
    const Real isd = rsq_approx(s), sd = s * isd;
#pragma unroll
    for (int k = 0; k < i; ++k) M[tri(i, k)] *= isd;
    M[tri(i, i)] *= sd;
  }
}

// Estimate of ||A^{-1}||_1 for a symmetric positive definite A from its
// packed Cholesky factor, after Hager (1984) with Higham's refinements (1988,
// the scheme of LAPACK's xLACN2): power-like steps on sign vectors, at most
// five solves with unit vectors, then an extra test vector with alternating
// signs.  kappa_1 is estimated as ||A||_1 times this; the estimate never
// exceeds the true value.
template <int P, class Real>
__device__ __forceinline__ Real hager_inv_norm1(const Real (&M)[P * (P + 1) / 2]) {
  Real b[P], x[P], z[P], xi[P];
  auto norm1 = [&](const Real (&v)[P]) {
    Real s = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) s += fabs(v[i]);
    return s;
  };
  auto argmax_abs = [&](const Real (&v)[P]) {
    int jm = 0;
    Real m = fabs(v[0]);
#pragma unroll
    for (int i = 1; i < P; ++i)
      if (fabs(v[i]) > m) {
        m = fabs(v[i]);
        jm = i;
      }
    return jm;
  };
#pragma unroll
  for (int i = 0; i < P; ++i) b[i] = Real(1) / P;
  chol_solve<P, Real>(M, b, x);
  Real est = norm1(x);
#pragma unroll
  for (int i = 0; i < P; ++i) xi[i] = x[i] >= Real(0) ? Real(1) : Real(-1);
  chol_solve<P, Real>(M, xi, z);
  int j = argmax_abs(z);
#pragma unroll 1
  for (int iter = 0; iter < 4; ++iter) {
#pragma unroll
    for (int i = 0; i < P; ++i) b[i] = i == j ? Real(1) : Real(0);
    chol_solve<P, Real>(M, b, x);
    const Real old = est;
    est = fmax(est, norm1(x));
    bool same = true;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const Real sgn = x[i] >= Real(0) ? Real(1) : Real(-1);
      same = same && sgn == xi[i];
      xi[i] = sgn;
    }
    if (same || !(est > old)) break;
    chol_solve<P, Real>(M, xi, z);
    const int jn = argmax_abs(z);
    if (fabs(z[jn]) == fabs(z[j])) break;
    j = jn;
  }
  // alternating-sign test vector
#pragma unroll
  for (int i = 0; i < P; ++i)
    b[i] = (i & 1 ? Real(-1) : Real(1)) * (Real(1) + static_cast<Real>(i) / static_cast<Real>(P > 1 ? P - 1 : 1));
  chol_solve<P, Real>(M, b, x);
  est = fmax(est, Real(2) * norm1(x) / (Real(3) * P));
  return est;
}

}  // namespace esim
