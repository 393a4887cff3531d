// Weighted local regression (Sec. 2.1, eqs. 3-5) on gfx950.
//
// One regression ("item") is the minimiser of
//     (1/W) sum_i w_i (y_i - alpha - beta^T u_i)^2 + ridge * |beta|^2,
//     u_i = x^i - x^c,  w_i = exp(-1/2 sum_j (u_ij / (h b_j))^2),  W = sum_i w_i,
// over the window |dx|, |dy| <= r, |dt| <= tr (truncated at image borders and
// clip ends), with x = (px / r, py / r, f_0 .. f_{F-1}).
//
// Mapping.  A wave holds G = 64 / L items; the L lanes of an item split the
// 2r+1 window columns (lane j takes dx = -r + j, -r + j + L, ...), so for one
// column pass the coordinate regressor u_x is constant in a lane and every
// Gram entry that involves u_x is folded once per pass instead of once per
// sample.  Loads are raw buffer loads (SGPR resource + VGPR offset, the
// channel stride in the SGPR offset), coalesced over the L adjacent columns of
// an item and over the G adjacent items of a dense wave.
//
// Precision.  The weight exponent is summed in FP64 from FP64 differences of
// the FP32 inputs and exponentiated with the FP32 hardware exp2 (about 1e-7
// relative).  Gram, right-hand side and Cholesky are FP64: without packed FP32
// (disabled in this build) an FP64 FMA issues at the same rate as an FP32 one
// on CDNA4, and the windows are ill-conditioned (kappa up to ~1e6 with a
// 1e-6 ridge), which FP32 accumulation does not survive at the 1e-4 contract.
//
// After the window loop the L lane partials are summed with DPP, every lane of
// the item factors the (F+3)x(F+3) system redundantly (registers only) and the
// lanes share the output writes.
#include "esim_internal.h"

namespace esim {
namespace {

constexpr double kHalfLog2e = -0.72134752044448170368;  // -log2(e) / 2

template <int F, int L, bool F16>
__global__ void __launch_bounds__(256)
regress_kernel(RegressArgs a) {
  constexpr int D = F + 2;
  constexpr int P = F + 3;
  constexpr int G = kWave / L;
  constexpr int NA = F * (F + 1) / 2;
  constexpr uint32_t ES = F16 ? 2u : 4u;

  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / L;
  const int j = lane % L;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) / kWave;
  // the device count is clamped to the output length: item i writes index i
  const int64_t n_items =
      a.items ? max(static_cast<int64_t>(0), min(static_cast<int64_t>(a.count[0]), a.n_out)) : 0;
  const int64_t ngroups = a.items ? (n_items + G - 1) / G : a.n_dense_groups;

  for (int64_t g = wave; g < ngroups; g += nwaves) {
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
    const int W = C.W, H = C.H, T = C.T, r = C.r, tr = C.tr;
    const uint32_t HW = static_cast<uint32_t>(C.HW);
    const int64_t pix = active ? my_pix : 0;
    // inactive lanes read a valid centre pixel of the resource window
    const int tt = active ? my_t : (a.t >= 0 ? a.t : 0);

    // frames held by the buffer resources: the window of a uniform frame, or
    // the whole clip when items carry their own frame
    const int f0 = a.t >= 0 ? max(0, a.t - tr) : 0;
    const int f1 = a.t >= 0 ? min(T, a.t + tr + 1) : T;
    const __amdgpu_buffer_rsrc_t ry =
        make_rsrc(C.y + static_cast<uint64_t>(f0) * HW, static_cast<uint64_t>(f1 - f0) * HW * 4u);
    const __amdgpu_buffer_rsrc_t rf =
        make_rsrc(static_cast<const char*>(C.feat) + static_cast<uint64_t>(f0) * F * HW * ES,
                  static_cast<uint64_t>(f1 - f0) * F * HW * ES);

    const int py = static_cast<int>(pix / W);
    const int px = static_cast<int>(pix - static_cast<int64_t>(py) * W);
    const int fc = tt - f0;
    const uint32_t vcen_f = (static_cast<uint32_t>(fc) * F * HW + static_cast<uint32_t>(pix)) * ES;
    const uint32_t vcen_y = (static_cast<uint32_t>(fc) * HW + static_cast<uint32_t>(pix)) * 4u;

    // Regressors are kept in bandwidth-scaled units v_j = u_j / (h b_j): the
    // weight exponent is then sum_j v_j^2, and the fit in v is the fit in u
    // with beta_j = theta_j / (h b_j) and the ridge scaled to lambda / (h b_j)^2.
    double sf[D], xcs[F];
#pragma unroll
    for (int d = 0; d < D; ++d) sf[d] = C.sf[d];
#pragma unroll
    for (int f = 0; f < F; ++f)
      xcs[f] = static_cast<double>(ld_feat<F16>(rf, vcen_f, f * HW * ES)) * sf[2 + f];

    const double rinv = 1.0 / r;
    const double vx_step = rinv * sf[0], vy_step = rinv * sf[1];
    const int dt_lo = max(-tr, -tt), dt_hi = min(tr, T - 1 - tt);
    const int nrows = (dt_hi - dt_lo + 1) * (2 * r + 1);

    // accumulators (see the header comment for the x-folding)
    double SW = 0, A0y = 0, g0 = 0, A0f[F];
    double A0x = 0, Axx = 0, Axy = 0, gx = 0, Axf[F];
    double Ayy = 0, gy = 0, Syy = 0, Ayf[F], gf[F], Aff[NA];
#pragma unroll
    for (int f = 0; f < F; ++f) A0f[f] = Axf[f] = Ayf[f] = gf[f] = 0.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) Aff[k] = 0.0;

    const int npass = (2 * r + 1 + L - 1) / L;
    for (int k = 0; k < npass; ++k) {
      const int dx = -r + j + k * L;
      const int col = px + dx;
      const bool col_ok = active && dx <= r && col >= 0 && col < W;
      const double vx = dx * vx_step;
      const double kx = kHalfLog2e * vx * vx;
      double qW = 0, qY = 0, qG = 0, qF[F];
#pragma unroll
      for (int f = 0; f < F; ++f) qF[f] = 0.0;

      // The rows (dt, dy) of this column are streamed through two register
      // buffers: the loads of one row are in flight while the other row is
      // accumulated.  Rows outside the image (or past the last row) read the
      // valid centre pixel and get weight 0.
      int ldt = dt_lo, ldy = -r;   // next row to load
      auto load_row = [&](float& yv, float (&fv)[F]) -> bool {
        const int row = py + ldy;
        // bitwise tests and selects keep the row addressing branch-free
        const bool ok = (ldt <= dt_hi) & col_ok & (row >= 0) & (row < H);
        const uint32_t pofs = static_cast<uint32_t>(row * W + col);
        const uint32_t fr = static_cast<uint32_t>(fc + ldt);
        const uint32_t vf_row = (fr * F * HW + pofs) * ES;
        const uint32_t vy_row = (fr * HW + pofs) * 4u;
        const uint32_t vf = ok ? vf_row : vcen_f;
        const uint32_t vy = ok ? vy_row : vcen_y;
        yv = ld_f32(ry, vy, 0);
#pragma unroll
        for (int f = 0; f < F; ++f) fv[f] = ld_feat<F16>(rf, vf, f * HW * ES);
        if (++ldy > r) {
          ldy = -r;
          ++ldt;
        }
        return ok;
      };
      int cdy = -r;                // dy of the row being accumulated
      auto accumulate = [&](float yv, const float (&fv)[F], bool ok) {
        const double vy = static_cast<double>(cdy) * vy_step;
        if (++cdy > r) cdy = -r;
        double v[F];
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int f = 0; f < F; ++f) {
          v[f] = fma(static_cast<double>(fv[f]), sf[2 + f], -xcs[f]);
          if (f & 1) s1 = fma(v[f], v[f], s1);
          else s0 = fma(v[f], v[f], s0);
        }
        const double arg = fma(s0 + s1, kHalfLog2e, fma(kHalfLog2e * vy, vy, kx));
        const float e = __builtin_amdgcn_exp2f(static_cast<float>(arg));
        const double w = static_cast<double>(ok ? e : 0.0f);
        const double yd = static_cast<double>(yv);
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
          for (int e2 = f; e2 < F; ++e2) {
            Aff[qq] = fma(wz, v[e2], Aff[qq]);
            ++qq;
          }
        }
      };
      float yA, fA[F], yB, fB[F];
      bool okA = load_row(yA, fA), okB;
      // two rows per iteration in one basic block (an odd last row is
      // accumulated with weight 0), so the scheduler can overlap the weight of
      // one row with the Gram updates of the other
#pragma unroll 1
      for (int q = 0; q < nrows; q += 2) {
        okB = load_row(yB, fB) & (q + 1 < nrows);
        accumulate(yA, fA, okA);
        okA = load_row(yA, fA);
        accumulate(yB, fB, okB);
      }
      // fold the column pass: every entry with a v_x factor
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

    // ---- sum the L lane partials of each item
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

    // ---- assemble the W-normalised system (packed lower triangle, row-major)
    //      unknown order: alpha, beta_x, beta_y, beta_f0 ..
    double M[P * (P + 1) / 2];
    double rhs[P];
    const double iW = 1.0 / SW;
    auto at = [](int i, int jj) { return i * (i + 1) / 2 + jj; };
    M[at(0, 0)] = 1.0;
    M[at(1, 0)] = A0x * iW;
    M[at(2, 0)] = A0y * iW;
    M[at(1, 1)] = Axx * iW + C.ridge * C.c2[0];
    M[at(2, 1)] = Axy * iW;
    M[at(2, 2)] = Ayy * iW + C.ridge * C.c2[1];
    rhs[0] = g0 * iW;
    rhs[1] = gx * iW;
    rhs[2] = gy * iW;
    {
      int q = 0;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        M[at(3 + f, 0)] = A0f[f] * iW;
        M[at(3 + f, 1)] = Axf[f] * iW;
        M[at(3 + f, 2)] = Ayf[f] * iW;
        rhs[3 + f] = gf[f] * iW;
#pragma unroll
        for (int e = f; e < F; ++e) {
          M[at(3 + e, 3 + f)] = Aff[q] * iW + (e == f ? C.ridge * C.c2[2 + f] : 0.0);
          ++q;
        }
      }
    }

    // ---- Cholesky M = L L^T in place, then L L^T theta = rhs
    double dmin = 1e300, dmax = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      double s = M[at(c, c)];
#pragma unroll
      for (int k = 0; k < c; ++k) s -= M[at(c, k)] * M[at(c, k)];
      const double d = s > 0.0 ? sqrt(s) : __builtin_nan("");
      const double id = 1.0 / d;
      M[at(c, c)] = d;
      dmin = fmin(dmin, d);
      dmax = fmax(dmax, d);
#pragma unroll
      for (int i = c + 1; i < P; ++i) {
        double v = M[at(i, c)];
#pragma unroll
        for (int k = 0; k < c; ++k) v -= M[at(i, k)] * M[at(c, k)];
        M[at(i, c)] = v * id;
      }
    }
    double th[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double v = rhs[i];
#pragma unroll
      for (int k = 0; k < i; ++k) v -= M[at(i, k)] * th[k];
      th[i] = v / M[at(i, i)];
    }
#pragma unroll
    for (int i = P - 1; i >= 0; --i) {
      double v = th[i];
#pragma unroll
      for (int k = i + 1; k < P; ++k) v -= M[at(k, i)] * th[k];
      th[i] = v / M[at(i, i)];
    }

    // ---- outputs (the lanes of an item share the writes)
    if (active) {
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
        if (a.kappa) {
          const double q = dmax / dmin;
          a.kappa[idx_out] = static_cast<float>(q * q);
        }
      }
      if (a.beta) {
#pragma unroll
        for (int d = 0; d < D; ++d)
          if (d % L == j)
            a.beta[static_cast<int64_t>(d) * a.n_out + idx_out] = static_cast<float>(th[1 + d] * sf[d]);
      }
    }
    }  // waterfall
  }
}

using KernelFn = void (*)(RegressArgs);

template <int F, int L>
KernelFn pick_dtype(bool f16) {
  return f16 ? regress_kernel<F, L, true> : regress_kernel<F, L, false>;
}

template <int F>
KernelFn pick_lanes(int lanes, bool f16) {
  switch (lanes) {
    case 2: return pick_dtype<F, 2>(f16);
    case 4: return pick_dtype<F, 4>(f16);
    case 8: return pick_dtype<F, 8>(f16);
    case 16: return pick_dtype<F, 16>(f16);
    default: return nullptr;
  }
}

KernelFn pick(int F, int lanes, bool f16) {
  switch (F) {
    case 1: return pick_lanes<1>(lanes, f16);
    case 2: return pick_lanes<2>(lanes, f16);
    case 3: return pick_lanes<3>(lanes, f16);
    case 4: return pick_lanes<4>(lanes, f16);
    case 5: return pick_lanes<5>(lanes, f16);
    case 6: return pick_lanes<6>(lanes, f16);
    case 7: return pick_lanes<7>(lanes, f16);
    case 8: return pick_lanes<8>(lanes, f16);
    case 9: return pick_lanes<9>(lanes, f16);
    case 10: return pick_lanes<10>(lanes, f16);
    case 11: return pick_lanes<11>(lanes, f16);
    case 12: return pick_lanes<12>(lanes, f16);
    default: return nullptr;
  }
}

}  // namespace

int regress_supported_lanes(int F) { return (F >= 1 && F <= ESIM_MAX_F) ? 0x2 | 0x4 | 0x8 | 0x10 : 0; }

hipError_t launch_regress(const RegressArgs& a, int F, bool f16, int precision, int lanes,
                          int blocks_per_cu, hipStream_t s) {
  (void)precision;
  KernelFn fn = pick(F, lanes, f16);
  if (!fn) return hipErrorInvalidValue;
  const int G = kWave / lanes;
  (void)G;
  int64_t blocks = (a.max_groups + kWavesPerBlock - 1) / kWavesPerBlock;
  const int64_t cap = static_cast<int64_t>(256) * blocks_per_cu;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace esim
