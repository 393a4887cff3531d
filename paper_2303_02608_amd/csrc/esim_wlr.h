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
// (dt, dy) of a column are streamed through two register buffers so the loads
// of one row are in flight while the other row is used.  Rows outside the
// image (or past the last row) read the valid centre pixel and get weight 0.
#pragma once

#include "esim_internal.h"

namespace esim {

constexpr double kHalfLog2e = -0.72134752044448170368;  // -log2(e) / 2

template <int F, bool F16>
struct ItemGeom {
  static constexpr uint32_t ES = F16 ? 2u : 4u;
  __amdgpu_buffer_rsrc_t ry, rf;
  uint32_t HW, vcen_f, vcen_y;
  int W, H, T, r, tr, px, py, fc, tt, dt_lo, dt_hi;
  bool active;
  double sf[F + 2];
  double xcs[F];
  double vx_step, vy_step;
};

// Fills the geometry of the item at (pix, tt) of clip C.  f0/f1 are the frames
// the buffer resources cover (a uniform frame's window, or the whole clip).
template <int F, bool F16>
__device__ __forceinline__ void make_geom(ItemGeom<F, F16>& g, const ClipDev& C, int64_t pix, int tt,
                                          int f0, int f1, bool active) {
  constexpr uint32_t ES = ItemGeom<F, F16>::ES;
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
  for (int d = 0; d < F + 2; ++d) g.sf[d] = C.sf[d];
#pragma unroll
  for (int f = 0; f < F; ++f)
    g.xcs[f] = static_cast<double>(ld_feat<F16>(g.rf, g.vcen_f, f * g.HW * ES)) * g.sf[2 + f];
  const double rinv = 1.0 / g.r;
  g.vx_step = rinv * g.sf[0];
  g.vy_step = rinv * g.sf[1];
  g.dt_lo = max(-g.tr, -tt);
  g.dt_hi = min(g.tr, g.T - 1 - tt);
}

// Runs the window of one item in lane j of its L-lane group.
//   pass_begin(vx)                      before each column pass
//   sample(w, yd, v[F], vy, dx, dt, dy, ok) for every sample; ok is false
//                                       (and w = 0) outside the image, for
//                                       idle columns and for the weight-0
//                                       padding row of an odd row count, whose
//                                       (dt, dy) lie past the window
//   pass_end(vx)                        after each column pass
template <int F, int L, bool F16, class PassBegin, class Sample, class PassEnd>
__device__ __forceinline__ void window_loop(const ItemGeom<F, F16>& g, int j, PassBegin&& pass_begin,
                                            Sample&& sample, PassEnd&& pass_end) {
  constexpr uint32_t ES = ItemGeom<F, F16>::ES;
  const int r = g.r;
  const int nrows = (g.dt_hi - g.dt_lo + 1) * (2 * r + 1);
  const int npass = (2 * r + 1 + L - 1) / L;
  for (int k = 0; k < npass; ++k) {
    const int dx = -r + j + k * L;
    const int col = g.px + dx;
    const bool col_ok = g.active && dx <= r && col >= 0 && col < g.W;
    const double vx = dx * g.vx_step;
    const double kx = kHalfLog2e * vx * vx;
    pass_begin(vx);
    int ldt = g.dt_lo, ldy = -r;   // next row to load
    auto load_row = [&](float& yv, float (&fv)[F]) -> bool {
      const int row = g.py + ldy;
      // bitwise tests and selects keep the row addressing branch-free
      const bool ok = (ldt <= g.dt_hi) & col_ok & (row >= 0) & (row < g.H);
      const uint32_t pofs = static_cast<uint32_t>(row * g.W + col);
      const uint32_t fr = static_cast<uint32_t>(g.fc + ldt);
      const uint32_t vf_row = (fr * F * g.HW + pofs) * ES;
      const uint32_t vy_row = (fr * g.HW + pofs) * 4u;
      const uint32_t vf = ok ? vf_row : g.vcen_f;
      const uint32_t vy = ok ? vy_row : g.vcen_y;
      yv = ld_f32(g.ry, vy, 0);
#pragma unroll
      for (int f = 0; f < F; ++f) fv[f] = ld_feat<F16>(g.rf, vf, f * g.HW * ES);
      if (++ldy > r) {
        ldy = -r;
        ++ldt;
      }
      return ok;
    };
    int cdt = g.dt_lo, cdy = -r;   // row being used
    auto use_row = [&](float yv, const float (&fv)[F], bool ok) {
      const int dy = cdy, dt = cdt;
      if (++cdy > r) {
        cdy = -r;
        ++cdt;
      }
      const double vy = static_cast<double>(dy) * g.vy_step;
      double v[F];
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        v[f] = fma(static_cast<double>(fv[f]), g.sf[2 + f], -g.xcs[f]);
        if (f & 1) s1 = fma(v[f], v[f], s1);
        else s0 = fma(v[f], v[f], s0);
      }
      const double arg = fma(s0 + s1, kHalfLog2e, fma(kHalfLog2e * vy, vy, kx));
      const float e = __builtin_amdgcn_exp2f(static_cast<float>(arg));
      const double w = static_cast<double>(ok ? e : 0.0f);
      sample(w, static_cast<double>(yv), v, vy, dx, dt, dy, ok);
    };
    // two rows per iteration in one basic block (an odd last row is used with
    // weight 0), so the scheduler can overlap the weight of one row with the
    // accumulation of the other
    float yA, fA[F], yB, fB[F];
    bool okA = load_row(yA, fA), okB;
#pragma unroll 1
    for (int q = 0; q < nrows; q += 2) {
      okB = load_row(yB, fB) & (q + 1 < nrows);
      use_row(yA, fA, okA);
      okA = load_row(yA, fA);
      use_row(yB, fB, okB);
    }
    pass_end(vx);
  }
}

// Normal equations of one item, accumulated per lane (Gram entries with a v_x
// factor are folded once per column pass).
template <int F>
struct Gram {
  static constexpr int NA = F * (F + 1) / 2;
  double SW, A0y, g0, A0f[F];
  double A0x, Axx, Axy, gx, Axf[F];
  double Ayy, gy, Syy, Ayf[F], gf[F], Aff[NA];
  double qW, qY, qG, qF[F];

  __device__ __forceinline__ void zero() {
    SW = A0y = g0 = A0x = Axx = Axy = gx = Ayy = gy = Syy = 0.0;
#pragma unroll
    for (int f = 0; f < F; ++f) A0f[f] = Axf[f] = Ayf[f] = gf[f] = 0.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) Aff[k] = 0.0;
  }
  __device__ __forceinline__ void pass_begin() {
    qW = qY = qG = 0.0;
#pragma unroll
    for (int f = 0; f < F; ++f) qF[f] = 0.0;
  }
  __device__ __forceinline__ void add(double w, double yd, const double (&v)[F], double vy) {
    const double wy = w * yd;
    const double wvy = w * vy;
    qW += w;
    qY += wvy;
    qG += wy;
    Ayy = fma(wvy, vy, Ayy);
    gy = fma(wy, vy, gy);
    Syy = fma(wy, yd, Syy);
    int qq = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const double wz = w * v[f];
      qF[f] += wz;
      Ayf[f] = fma(wvy, v[f], Ayf[f]);
      gf[f] = fma(wz, yd, gf[f]);
#pragma unroll
      for (int e = f; e < F; ++e) {
        Aff[qq] = fma(wz, v[e], Aff[qq]);
        ++qq;
      }
    }
  }
  __device__ __forceinline__ void pass_end(double vx) {
    SW += qW;
    A0y += qY;
    g0 += qG;
    A0x = fma(vx, qW, A0x);
    Axx = fma(vx * vx, qW, Axx);
    Axy = fma(vx, qY, Axy);
    gx = fma(vx, qG, gx);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      A0f[f] += qF[f];
      Axf[f] = fma(vx, qF[f], Axf[f]);
    }
  }
  template <int L>
  __device__ __forceinline__ void lane_sum() {
    if constexpr (L > 1) {
      SW = group_sum<L>(SW);
      A0y = group_sum<L>(A0y);
      g0 = group_sum<L>(g0);
      A0x = group_sum<L>(A0x);
      Axx = group_sum<L>(Axx);
      Axy = group_sum<L>(Axy);
      gx = group_sum<L>(gx);
      Ayy = group_sum<L>(Ayy);
      gy = group_sum<L>(gy);
      Syy = group_sum<L>(Syy);
#pragma unroll
      for (int f = 0; f < F; ++f) {
        A0f[f] = group_sum<L>(A0f[f]);
        Axf[f] = group_sum<L>(Axf[f]);
        Ayf[f] = group_sum<L>(Ayf[f]);
        gf[f] = group_sum<L>(gf[f]);
      }
#pragma unroll
      for (int k = 0; k < NA; ++k) Aff[k] = group_sum<L>(Aff[k]);
    }
  }
};

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Solves L L^T x = b with the packed factor.
template <int P>
__device__ __forceinline__ void chol_solve(const double (&M)[P * (P + 1) / 2], const double (&b)[P],
                                           double (&x)[P]) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= M[tri(i, k)] * x[k];
    x[i] = v / M[tri(i, i)];
  }
#pragma unroll
  for (int i = P - 1; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int k = i + 1; k < P; ++k) v -= M[tri(k, i)] * x[k];
    x[i] = v / M[tri(i, i)];
  }
}


// Assembles the W-normalised system in scaled units (unknowns alpha, beta_x,
// beta_y, beta_f..), adds the scaled ridge, factors it in place (packed lower
// Cholesky) and solves for theta.  Returns 1/W.  dmin/dmax are the extreme
// diagonal entries of the factor.
template <int F>
__device__ __forceinline__ double gram_solve(const Gram<F>& G, const ClipDev& C,
                                             double (&M)[(F + 3) * (F + 4) / 2], double (&rhs)[F + 3],
                                             double (&th)[F + 3], double& dmin, double& dmax) {
  constexpr int P = F + 3;
  const double iW = 1.0 / G.SW;
  M[tri(0, 0)] = 1.0;
  M[tri(1, 0)] = G.A0x * iW;
  M[tri(2, 0)] = G.A0y * iW;
  M[tri(1, 1)] = G.Axx * iW + C.ridge * C.c2[0];
  M[tri(2, 1)] = G.Axy * iW;
  M[tri(2, 2)] = G.Ayy * iW + C.ridge * C.c2[1];
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
        M[tri(3 + e, 3 + f)] = G.Aff[q] * iW + (e == f ? C.ridge * C.c2[2 + f] : 0.0);
        ++q;
      }
    }
  }
  dmin = 1e300;
  dmax = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    double s = M[tri(c, c)];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= M[tri(c, k)] * M[tri(c, k)];
    const double d = s > 0.0 ? sqrt(s) : __builtin_nan("");
    const double id = 1.0 / d;
    M[tri(c, c)] = d;
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
#pragma unroll
    for (int i = c + 1; i < P; ++i) {
      double v = M[tri(i, c)];
#pragma unroll
      for (int k = 0; k < c; ++k) v -= M[tri(i, k)] * M[tri(c, k)];
      M[tri(i, c)] = v * id;
    }
  }
  chol_solve<P>(M, rhs, th);
  return iW;
}

}  // namespace esim
