// Plain FP64 CPU oracle of the event simulator (TEST INFRASTRUCTURE ONLY).
//
// This file is the slow, obviously-correct reference the GPU path is checked
// against.  It shares no code, header or constant with the HIP library, and it
// must only be called from tests, the smoke check and the CPU-baseline leg of
// the benchmark.  Everything is double precision; FP16 feature inputs are
// widened bit-exactly.
//
// Paper: Tsuji, Yatagawa, Kubo, Morishima, "Event-based Camera Simulation using
// Monte Carlo Path Tracing with Adaptive Denoising" (arXiv 2303.02608).
//
//   * orc_log_brightness   Sec. 1.1 / Sec. 2.1: L = log E  (the workloads add
//                          eps = 1e-3 inside the log).
//   * orc_regress*         Sec. 2.1, eqs. (3)-(5): first-order weighted local
//                          regression of y over a window of neighbours.
//   * orc_residual_hat     Sec. 2.2, eq. (7): residual of the translated plane,
//                          evaluated explicitly over the last-event window.
//   * orc_explicit         Sec. 2.2, eq. (7) and the R of eq. (4) for a stored
//                          plane, over the last-event window or (the other
//                          reading) over the current frame's window.
//   * orc_run              Sec. 1.1 eq. (1) event rule; Sec. 2.2 threshold
//                          (Prop. 1, eqs. (8)-(9)); the baselines of Sec. 3
//                          ("ESIM" on the noisy frames, "WLR+ESIM").
//   * orc_backward         adjoint of the regression estimate alpha with
//                          respect to y and to the bandwidths b (derived from
//                          eqs. (4)-(5) by implicit differentiation).
//   * orc_cond             2-norm condition number by cyclic Jacobi, for
//                          reporting only.
//   * orc_log_variance     variance of y = log(E_mean + eps) from the sample
//                          variance of the radiance (delta method).
//   * orc_regress_bandwidth the bandwidth-optimised variant of Sec. 3
//                          (bandwidth optimisation): per regression, the
//                          global bandwidth h of eq. (5) chosen from a
//                          candidate set by the smallest estimated mean
//                          squared error of alpha (Stein's unbiased risk
//                          estimate with the MC variance of the centre).
//
// Readings of the paper taken here (where it is silent or loose):
//   - Gaussian fall-off w(u) = exp(-u^2/2); the product over dimensions of
//     eq. (5) is one exponential of the summed squares.
//   - Feature vector x = (px/r, py/r, f_0 .. f_{F-1}): image coordinates in
//     units of the window radius r, other features as supplied.
//   - Window: |dx|, |dy| <= r, |dt| <= tr frames, truncated at image borders
//     and clip ends.  Temporal neighbours are weighted by eq. (5) only.
//   - The system is (D+1)x(D+1) (alpha is an unknown as well).  A ridge
//     lambda >= 0 is added to the beta block of the W-normalised Gram; the
//     alpha row is untouched, so the residuals have weighted mean zero.
//   - Threshold: R_hat uses the window data of the last-event frame with only
//     the centre feature replaced (Fig. 1 caption), so R_hat - R equals
//     (beta^T (x^c - x_hat^c))^2 exactly at the least-squares minimiser; the
//     image-coordinate components of x^c - x_hat^c vanish (same pixel).
//   - An event fires when Delta R >= C^2 (the change "reaches" C), polarity is
//     the sign of beta^T (x_hat^c - x^c), at most one event per pixel and
//     frame, and the reference model is replaced by the new regression.
//   - Exhaustive and raw baselines: L_ref starts at frame 0; an event fires
//     when |L_t - L_ref| >= C, then L_ref <- L_t.
//   - Bandwidth optimisation (the paper names the bias and the MC variance
//     as the criterion but not the estimator): alpha_h = e_0^T A_h^{-1} g_h is
//     linear in the observations, with d alpha_h / d y_c = (w_c / W_h) v_0,
//     v = A_h^{-1} e_0 (w_c = 1, z_c = e_0 at the centre).  With sigma_c^2 the
//     MC variance of y_c, SURE(h) = (alpha_h - y_c)^2 + 2 sigma_c^2 v_0 / W_h
//     - sigma_c^2 estimates E[(alpha_h - f_c)^2] without bias (bias^2 plus
//     variance); the candidate with the smallest SURE is taken (the first of
//     equal ones).  Only h is optimised; b stays as given.
//   - Explicit thresholds (an ablation of Prop. 1): Delta R = |R_hat - R| is
//     evaluated from its definition instead of the closed form.  R is eq. (4)
//     for the stored plane over its own (last-event) window.  R_hat is eq. (7)
//     over either the last-event window (the reading above: then Delta R equals
//     the closed form's dL^2) or the window of the current frame t centred at
//     x_hat^c, with weights of eq. (5) about x_hat^c and the current samples
//     (the other reading, which also sees brightness changes that the features
//     do not explain).  The sign of an event is the sign of the weighted mean
//     of the translated plane's residuals y^i - alpha - beta^T (x^i - x_hat^c),
//     which over the last-event window equals dL; the compared change is
//     sign * sqrt(Delta R), which equals dL in the first reading.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t W, H, T, F;
  const double* y;      // [T][H][W] log-brightness
  const void* feat;     // [T][F][H][W], float32 or float16 bits
  int32_t feat_f16;     // 1 if feat holds IEEE binary16
} orc_clip;

typedef struct {
  int32_t r, tr;        // spatial radius, temporal radius (frames)
  double C;             // contrast threshold
  double h;             // global bandwidth
  const double* b;      // [F+2] per-dimension bandwidths (coords first)
  double ridge;         // lambda on the beta block
} orc_params;

}  // extern "C"

namespace {

double half_bits_to_double(uint16_t hb) {
  const int sign = (hb >> 15) & 1;
  const int ex = (hb >> 10) & 31;
  const int man = hb & 1023;
  double v;
  if (ex == 0) {
    v = std::ldexp(static_cast<double>(man), -24);
  } else if (ex == 31) {
    v = man ? NAN : INFINITY;
  } else {
    v = std::ldexp(static_cast<double>(man + 1024), ex - 25);
  }
  return sign ? -v : v;
}

struct Clip {
  const orc_clip* c;
  double feat(int t, int f, int py, int px) const {
    const size_t i = ((static_cast<size_t>(t) * c->F + f) * c->H + py) * c->W + px;
    if (c->feat_f16) return half_bits_to_double(static_cast<const uint16_t*>(c->feat)[i]);
    return static_cast<double>(static_cast<const float*>(c->feat)[i]);
  }
  double y(int t, int py, int px) const {
    return c->y[(static_cast<size_t>(t) * c->H + py) * c->W + px];
  }
};

// One window sample: its weight, its regressor z = (1, u) and its observation.
struct Sample {
  double w;
  double yv;
  std::vector<double> z;  // length P
  int t, py, px;
};

// Feature vector x = (px/r, py/r, f_0..f_{F-1}) at (t, py, px).
void feature_vector(const Clip& cl, int r, int t, int py, int px, double* x) {
  x[0] = static_cast<double>(px) / r;
  x[1] = static_cast<double>(py) / r;
  for (int f = 0; f < cl.c->F; ++f) x[2 + f] = cl.feat(t, f, py, px);
}

// Eq. (5): w^i = prod_j w((x^i_j - x^c_j) / (h b_j)), w(u) = exp(-u^2/2).
// Collects the window Omega of the centre (t, py, px) with centre features xc.
std::vector<Sample> gather_window(const Clip& cl, const orc_params* p, int t, int py, int px,
                                  const double* xc) {
  const int F = cl.c->F, D = F + 2, P = D + 1;
  std::vector<Sample> out;
  std::vector<double> xi(D);
  for (int tt = t - p->tr; tt <= t + p->tr; ++tt) {
    if (tt < 0 || tt >= cl.c->T) continue;
    for (int yy = py - p->r; yy <= py + p->r; ++yy) {
      if (yy < 0 || yy >= cl.c->H) continue;
      for (int xx = px - p->r; xx <= px + p->r; ++xx) {
        if (xx < 0 || xx >= cl.c->W) continue;
        feature_vector(cl, p->r, tt, yy, xx, xi.data());
        Sample s;
        s.z.assign(P, 0.0);
        s.z[0] = 1.0;
        double q = 0.0;
        for (int j = 0; j < D; ++j) {
          const double u = xi[j] - xc[j];
          s.z[1 + j] = u;
          const double a = u / (p->h * p->b[j]);
          q += a * a;
        }
        s.w = std::exp(-0.5 * q);
        s.yv = cl.y(tt, yy, xx);
        s.t = tt;
        s.py = yy;
        s.px = xx;
        out.push_back(std::move(s));
      }
    }
  }
  return out;
}

// Cholesky factorisation A = L L^T of a symmetric P x P matrix (row-major);
// returns false if a pivot is not positive.
bool cholesky(const std::vector<double>& A, int P, std::vector<double>& L) {
  L.assign(static_cast<size_t>(P) * P, 0.0);
  for (int j = 0; j < P; ++j) {
    double s = A[j * P + j];
    for (int k = 0; k < j; ++k) s -= L[j * P + k] * L[j * P + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    L[j * P + j] = d;
    for (int i = j + 1; i < P; ++i) {
      double v = A[i * P + j];
      for (int k = 0; k < j; ++k) v -= L[i * P + k] * L[j * P + k];
      L[i * P + j] = v / d;
    }
  }
  return true;
}

// Solve L L^T x = rhs.
void chol_solve(const std::vector<double>& L, int P, const double* rhs, double* x) {
  std::vector<double> z(P);
  for (int i = 0; i < P; ++i) {
    double v = rhs[i];
    for (int k = 0; k < i; ++k) v -= L[i * P + k] * z[k];
    z[i] = v / L[i * P + i];
  }
  for (int i = P - 1; i >= 0; --i) {
    double v = z[i];
    for (int k = i + 1; k < P; ++k) v -= L[k * P + i] * x[k];
    x[i] = v / L[i * P + i];
  }
}

// Cyclic Jacobi eigenvalues of a symmetric matrix; returns lambda_max/lambda_min.
double jacobi_cond(std::vector<double> A, int P) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) {
        tot += A[i * P + j] * A[i * P + j];
        if (i != j) off += A[i * P + j] * A[i * P + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < P - 1; ++p)
      for (int q = p + 1; q < P; ++q) {
        const double apq = A[p * P + q];
        if (apq == 0.0) continue;
        const double app = A[p * P + p], aqq = A[q * P + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < P; ++k) {  // A <- A J (columns p, q)
          const double akp = A[k * P + p], akq = A[k * P + q];
          A[k * P + p] = c * akp - s * akq;
          A[k * P + q] = s * akp + c * akq;
        }
        for (int k = 0; k < P; ++k) {  // A <- J^T A (rows p, q)
          const double apk = A[p * P + k], aqk = A[q * P + k];
          A[p * P + k] = c * apk - s * aqk;
          A[q * P + k] = s * apk + c * aqk;
        }
      }
  }
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < P; ++i) {
    lo = std::min(lo, A[i * P + i]);
    hi = std::max(hi, A[i * P + i]);
  }
  if (!(lo > 0.0)) return INFINITY;
  return hi / lo;
}

struct Fit {
  bool ok = false;
  std::vector<double> theta;  // (alpha, beta_0 .. beta_{D-1})
  std::vector<double> A;      // W-normalised Gram with ridge (P x P)
  double W = 0.0, R = 0.0, kappa = NAN;
  std::vector<double> xc;     // centre feature vector
  std::vector<Sample> win;
};

// Eqs. (3)-(5): minimise (1/W) sum_i w^i (y^i - alpha - beta^T (x^i - x^c))^2
// (+ ridge on beta) through the normal equations and a Cholesky solve.
Fit regress(const Clip& cl, const orc_params* p, int t, int py, int px, bool want_kappa,
            bool keep_window) {
  const int F = cl.c->F, D = F + 2, P = D + 1;
  Fit fit;
  fit.xc.assign(D, 0.0);
  feature_vector(cl, p->r, t, py, px, fit.xc.data());
  std::vector<Sample> win = gather_window(cl, p, t, py, px, fit.xc.data());
  std::vector<double> A(static_cast<size_t>(P) * P, 0.0), g(P, 0.0);
  double W = 0.0;
  for (const Sample& s : win) {
    W += s.w;
    for (int i = 0; i < P; ++i) {
      g[i] += s.w * s.yv * s.z[i];
      for (int j = 0; j < P; ++j) A[i * P + j] += s.w * s.z[i] * s.z[j];
    }
  }
  for (double& a : A) a /= W;
  for (double& v : g) v /= W;
  for (int j = 1; j < P; ++j) A[j * P + j] += p->ridge;
  fit.W = W;
  fit.A = A;
  fit.theta.assign(P, NAN);
  std::vector<double> L;
  if (cholesky(A, P, L)) {
    chol_solve(L, P, g.data(), fit.theta.data());
    fit.ok = true;
  }
  // R of eq. (4), evaluated explicitly over the window.
  double R = 0.0;
  for (const Sample& s : win) {
    double pred = 0.0;
    for (int i = 0; i < P; ++i) pred += fit.theta[i] * s.z[i];
    const double e = s.yv - pred;
    R += s.w * e * e;
  }
  fit.R = R / W;
  if (want_kappa) fit.kappa = jacobi_cond(A, P);
  if (keep_window) fit.win = std::move(win);
  return fit;
}

// Eq. (7) evaluated literally: the last-event window (weights, y^i, x^i) and
// plane (alpha, beta), with the centre replaced by x_hat.
double residual_hat(const Fit& fit, const double* xhat, int D) {
  double Rh = 0.0;
  for (const Sample& s : fit.win) {
    // x^i - x_hat = (x^i - x^c) + (x^c - x_hat)
    double pred = fit.theta[0];
    for (int j = 0; j < D; ++j) pred += fit.theta[1 + j] * (s.z[1 + j] + fit.xc[j] - xhat[j]);
    const double e = s.yv - pred;
    Rh += s.w * e * e;
  }
  return Rh / fit.W;
}

// R of eq. (4) for the plane theta (alpha, beta over D) over the window of
// frame tw about centre features xw, and the translated plane's residuals
// rhat_i = y^i - alpha - beta^T (x^i - xhat): returns their weighted mean and
// mean square.  With xw = x^c (the plane's own centre) and tw = t_ref this is
// eq. (7) over the last-event window; with xw = xhat and tw = t, over the
// current frame's window (then R is not formed: the window is not the plane's).
struct WindowResiduals {
  double W = 0.0, R = 0.0, Rhat = 0.0, mean = 0.0;
};

WindowResiduals window_residuals(const Clip& cl, const orc_params* p, int tw, int py, int px,
                                 const double* xw, const double* theta, const double* xhat) {
  const int D = cl.c->F + 2;
  WindowResiduals o;
  std::vector<Sample> win = gather_window(cl, p, tw, py, px, xw);
  double sr2 = 0.0, sh = 0.0, sh2 = 0.0;
  for (const Sample& s : win) {
    // s.z[1 + j] = x^i_j - xw_j
    double pr = theta[0], ph = theta[0];
    for (int j = 0; j < D; ++j) {
      pr += theta[1 + j] * s.z[1 + j];
      ph += theta[1 + j] * (s.z[1 + j] + xw[j] - xhat[j]);
    }
    const double r = s.yv - pr, rh = s.yv - ph;
    o.W += s.w;
    sr2 += s.w * r * r;
    sh += s.w * rh;
    sh2 += s.w * rh * rh;
  }
  o.R = sr2 / o.W;
  o.Rhat = sh2 / o.W;
  o.mean = sh / o.W;
  return o;
}

// Explicit Delta R of the stored plane (theta, centre features at t_ref) at
// frame t (new_window: 0 = last-event window, 1 = frame t's window).  Returns
// the compared change sign(mean) * sqrt(|R_hat - R|); *dR receives |R_hat - R|.
double explicit_change(const Clip& cl, const orc_params* p, int new_window, int tref, int t, int py,
                       int px, const double* theta, double* dR) {
  const int D = cl.c->F + 2;
  std::vector<double> xc(D), xhat(D);
  feature_vector(cl, p->r, tref, py, px, xc.data());
  feature_vector(cl, p->r, t, py, px, xhat.data());
  const WindowResiduals last = window_residuals(cl, p, tref, py, px, xc.data(), theta, xhat.data());
  double Rhat = last.Rhat, mean = last.mean;
  if (new_window) {
    const WindowResiduals cur = window_residuals(cl, p, t, py, px, xhat.data(), theta, xhat.data());
    Rhat = cur.Rhat;
    mean = cur.mean;
  }
  const double d = std::fabs(Rhat - last.R);
  *dR = d;
  return (mean > 0.0 ? 1.0 : -1.0) * std::sqrt(d);
}

int nthreads_or_default(int n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  // namespace

extern "C" {

// y = log(E + eps) in double (Sec. 1.1: L = log E).
void orc_log_brightness(const float* E, double* y, int64_t n, double eps) {
  for (int64_t i = 0; i < n; ++i) y[i] = std::log(static_cast<double>(E[i]) + eps);
}

// One regression (eqs. 3-5).  theta[P] receives (alpha, beta); info[4]
// receives (W, R, kappa, ok).  Returns 0 on success, -1 if the Cholesky
// failed (theta = NaN), -2 on bad arguments.
int orc_regress(const orc_clip* c, const orc_params* p, int t, int px, int py, double* theta,
                double* info, int want_kappa) {
  if (!c || !p || t < 0 || t >= c->T || px < 0 || px >= c->W || py < 0 || py >= c->H) return -2;
  Clip cl{c};
  Fit fit = regress(cl, p, t, py, px, want_kappa != 0, false);
  const int P = c->F + 3;
  for (int i = 0; i < P; ++i) theta[i] = fit.theta[i];
  if (info) {
    info[0] = fit.W;
    info[1] = fit.R;
    info[2] = fit.kappa;
    info[3] = fit.ok ? 1.0 : 0.0;
  }
  return fit.ok ? 0 : -1;
}

// The W-normalised Gram (with ridge) and right-hand side of one regression,
// for checking the solver independently.  A[P*P], g[P].
int orc_normal_equations(const orc_clip* c, const orc_params* p, int t, int px, int py,
                         double* A, double* g, double* Wout) {
  if (!c || !p) return -2;
  Clip cl{c};
  const int F = c->F, D = F + 2, P = D + 1;
  std::vector<double> xc(D);
  feature_vector(cl, p->r, t, py, px, xc.data());
  std::vector<Sample> win = gather_window(cl, p, t, py, px, xc.data());
  std::vector<double> AA(static_cast<size_t>(P) * P, 0.0), gg(P, 0.0);
  double W = 0.0;
  for (const Sample& s : win) {
    W += s.w;
    for (int i = 0; i < P; ++i) {
      gg[i] += s.w * s.yv * s.z[i];
      for (int j = 0; j < P; ++j) AA[i * P + j] += s.w * s.z[i] * s.z[j];
    }
  }
  for (int i = 0; i < P * P; ++i) A[i] = AA[i] / W;
  for (int i = 0; i < P; ++i) g[i] = gg[i] / W;
  for (int j = 1; j < P; ++j) A[j * P + j] += p->ridge;
  *Wout = W;
  return static_cast<int>(win.size());
}

// The window samples of one regression: for each sample (t, py, px, w, z[P]).
// Returns the number of samples (written up to cap).
int orc_window(const orc_clip* c, const orc_params* p, int t, int px, int py, int32_t* pos,
               double* w, double* z, int cap) {
  Clip cl{c};
  const int F = c->F, D = F + 2, P = D + 1;
  std::vector<double> xc(D);
  feature_vector(cl, p->r, t, py, px, xc.data());
  std::vector<Sample> win = gather_window(cl, p, t, py, px, xc.data());
  const int n = static_cast<int>(win.size());
  for (int i = 0; i < n && i < cap; ++i) {
    pos[3 * i + 0] = win[i].t;
    pos[3 * i + 1] = win[i].py;
    pos[3 * i + 2] = win[i].px;
    w[i] = win[i].w;
    for (int j = 0; j < P; ++j) z[static_cast<size_t>(i) * P + j] = win[i].z[j];
  }
  return n;
}

// Regressions at a list of items (t * H * W + py * W + px).  Outputs per item:
// theta[n][P], W[n], R[n], kappa[n] (kappa may be null).  Returns the number
// of failed solves.
int orc_regress_items(const orc_clip* c, const orc_params* p, const int64_t* items, int64_t n,
                      double* theta, double* Wout, double* Rout, double* kappa, int nthreads) {
  Clip cl{c};
  const int P = c->F + 3;
  const int64_t HW = static_cast<int64_t>(c->W) * c->H;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads)) reduction(+ : fails)
  for (int64_t i = 0; i < n; ++i) {
    const int t = static_cast<int>(items[i] / HW);
    const int pix = static_cast<int>(items[i] % HW);
    Fit fit = regress(cl, p, t, pix / c->W, pix % c->W, kappa != nullptr, false);
    for (int j = 0; j < P; ++j) theta[i * P + j] = fit.theta[j];
    if (Wout) Wout[i] = fit.W;
    if (Rout) Rout[i] = fit.R;
    if (kappa) kappa[i] = fit.kappa;
    if (!fit.ok) fails += 1;
  }
  return fails;
}

// Eq. (7) explicitly: R_hat for the plane regressed at (t_ref, py, px) and the
// translated centre x_hat[D].  Returns R_hat; R of that regression in *R.
double orc_residual_hat(const orc_clip* c, const orc_params* p, int t_ref, int px, int py,
                        const double* xhat, double* R) {
  Clip cl{c};
  Fit fit = regress(cl, p, t_ref, py, px, false, true);
  if (R) *R = fit.R;
  return residual_hat(fit, xhat, c->F + 2);
}

// Explicit Delta R for the plane theta[P] = (alpha, beta over D) regressed at
// (t_ref, py, px), at frame t (new_window 0: eq. (7) over the last-event
// window; 1: over frame t's window).  out[4] = (R, R_hat, weighted mean of the
// translated residuals, compared change sign * sqrt(|R_hat - R|)).
int orc_explicit(const orc_clip* c, const orc_params* p, int new_window, int t_ref, int t, int px,
                 int py, const double* theta, double* out) {
  if (!c || !p || !theta || !out || t_ref < 0 || t_ref >= c->T || t < 0 || t >= c->T || px < 0 ||
      px >= c->W || py < 0 || py >= c->H)
    return -2;
  Clip cl{c};
  const int D = c->F + 2;
  std::vector<double> xc(D), xhat(D);
  feature_vector(cl, p->r, t_ref, py, px, xc.data());
  feature_vector(cl, p->r, t, py, px, xhat.data());
  const WindowResiduals last = window_residuals(cl, p, t_ref, py, px, xc.data(), theta, xhat.data());
  WindowResiduals cur = last;
  if (new_window) cur = window_residuals(cl, p, t, py, px, xhat.data(), theta, xhat.data());
  double dR = 0.0;
  out[0] = last.R;
  out[1] = cur.Rhat;
  out[2] = cur.mean;
  out[3] = explicit_change(cl, p, new_window, t_ref, t, py, px, theta, &dR);
  return 0;
}

// Delta-method variance of y = log(E + eps) for the mean E of spp samples with
// unbiased sample variance var: Var[E_mean] = var / spp, dy/dE = 1 / (E + eps).
void orc_log_variance(const float* E, const float* var, int spp, double* vy, int64_t n, double eps) {
  for (int64_t i = 0; i < n; ++i) {
    const double e = static_cast<double>(E[i]) + eps;
    vy[i] = static_cast<double>(var[i]) / spp / (e * e);
  }
}

// Bandwidth-optimised regressions at items (t * H * W + pixel): for each of the
// K candidate global bandwidths hs[k] (replacing p->h in eq. (5)) the
// regression of eqs. (3)-(5), v = A^{-1} e_0 and
//   SURE_k = (alpha_k - y_c)^2 + 2 vy_c v_0 / W_k - vy_c
// with vy ([T][H][W]) the MC variance of y.  Outputs per item: theta[n][P] and
// hsel[n] of the smallest SURE (the first of equal ones), and, nullable,
// alpha_k[n][K] and sure[n][K] of every candidate.  Returns the number of
// failed solves (their SURE is +inf).
int orc_regress_bandwidth(const orc_clip* c, const orc_params* p, const double* hs, int K,
                          const double* vy, const int64_t* items, int64_t n, double* theta, double* hsel,
                          double* alpha_k, double* sure_k, int nthreads) {
  Clip cl{c};
  const int P = c->F + 3;
  const int64_t HW = static_cast<int64_t>(c->W) * c->H;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads)) reduction(+ : fails)
  for (int64_t i = 0; i < n; ++i) {
    const int t = static_cast<int>(items[i] / HW);
    const int pix = static_cast<int>(items[i] % HW);
    const double yc = cl.y(t, pix / c->W, pix % c->W);
    const double s2 = vy[static_cast<int64_t>(t) * HW + pix];
    double best = INFINITY;
    int kbest = 0;
    std::vector<double> th_best(P, NAN);
    for (int k = 0; k < K; ++k) {
      orc_params pk = *p;
      pk.h = hs[k];
      Fit fit = regress(cl, &pk, t, pix / c->W, pix % c->W, false, false);
      double sure = INFINITY;
      std::vector<double> L;
      if (fit.ok && cholesky(fit.A, P, L)) {
        std::vector<double> e0(P, 0.0), v(P);
        e0[0] = 1.0;
        chol_solve(L, P, e0.data(), v.data());
        const double d = fit.theta[0] - yc;
        sure = d * d + 2.0 * s2 * v[0] / fit.W - s2;
      } else {
        ++fails;
      }
      if (alpha_k) alpha_k[i * K + k] = fit.theta[0];
      if (sure_k) sure_k[i * K + k] = sure;
      if (sure < best) {
        best = sure;
        kbest = k;
        th_best = fit.theta;
      }
    }
    for (int j = 0; j < P; ++j) theta[i * P + j] = th_best[j];
    hsel[i] = hs[kbest];
  }
  return fails;
}

double orc_cond(const double* A, int P) {
  std::vector<double> M(A, A + static_cast<size_t>(P) * P);
  return jacobi_cond(M, P);
}

// Modes of orc_run.
enum {
  ORC_THRESHOLDED = 0,
  ORC_EXHAUSTIVE = 1,
  ORC_RAW = 2,
  ORC_EXPLICIT_LAST = 3,
  ORC_EXPLICIT_NEW = 4,
  ORC_EXHAUSTIVE_ALL = 5,
  ORC_RAW_ALL = 6
};

// Event simulation over a whole clip (or a subset of pixels).
//
//   mode 0: the paper's method (Sec. 2.2).  Frame 0 regresses every pixel and
//           stores (alpha, beta, x^c, t_ref); no events.  For t >= 1 the
//           predicted change dL = beta_ref^T (f_t - x_ref) over the F buffer
//           channels is thresholded (dL^2 >= C^2, Prop. 1); flagged pixels
//           emit (px, py, t, sign dL), regress at t and replace the state.
//           With check_identity the residual of eq. (7) is also evaluated
//           explicitly and |R_hat - R - dL^2| is recorded.
//   mode 1: WLR+ESIM: alpha_t for every pixel and frame, eq. (1) on alpha.
//   mode 2: ESIM on the noisy frames: eq. (1) on y.
//   mode 3: as mode 0 with Delta R = |R_hat - R| evaluated explicitly over
//           the last-event window (eqs. (4) and (7)); fires when
//           Delta R >= C^2, with the sign of the translated plane's mean
//           residual.  dl receives sign * sqrt(Delta R).
//   mode 4: as mode 3 with R_hat over the window of the current frame.
//   mode 5, 6: modes 1 and 2 with every crossing (ESIM proper, the event rule
//           of eq. (1) applied to each level the brightness passes between
//           two frames).  The compared brightness L is taken as linear between
//           frames t - 1 and t.  With d = L_t - L_ref, n = floor(|d| / C) and
//           p = sign d, the levels L_ref + k p C (k = 1..n) are events at the
//           times (t - 1) + (L_ref + k p C - L_{t-1}) / (L_t - L_{t-1}); then
//           L_ref <- L_ref + n p C (the last level passed, not L_t).  L_ref
//           starts at L_0, so it stays on the lattice L_0 + C Z.  Everything
//           in double precision, with no bound on n (a non-finite d fires
//           nothing).
//
// pixels: optional list of pixel indices (ascending) to simulate; null = all.
// Events are written in (t, py, px) order up to cap; the total count is
// returned.  dl (nullable, [T][npix]) receives the per-pixel-frame change that
// was compared with C (NaN at t = 0).  nflag (nullable, [T]) counts flagged
// pixels per frame (mode 0) or events per frame.  st_alpha/st_beta/st_xref/
// st_tref (nullable, [npix], [F][npix], [F][npix], [npix]) receive the final
// state of mode 0; st_alpha receives L_ref in modes 1, 2, 5 and 6.  ets
// (nullable, [cap]) receives each event's time in frame units: t, or the
// interpolated crossing time in modes 5 and 6.
int64_t orc_run(const orc_clip* c, const orc_params* p, int mode, const int32_t* pixels,
                int64_t npix_in, int32_t* ex, int32_t* ey, int32_t* et, int8_t* ep, int64_t cap,
                double* dl, int64_t* nflag, double* st_alpha, double* st_beta, double* st_xref,
                int32_t* st_tref, int check_identity, double* max_identity_err, int nthreads,
                double* ets) {
  Clip cl{c};
  const int F = c->F, D = F + 2, P = D + 1, T = c->T;
  const int64_t HW = static_cast<int64_t>(c->W) * c->H;
  const int64_t npix = pixels ? npix_in : HW;
  auto pix_of = [&](int64_t k) -> int64_t { return pixels ? pixels[k] : k; };
  const int nt = nthreads_or_default(nthreads);

  std::vector<double> ref(npix, 0.0);                       // alpha_ref or L_ref
  std::vector<double> beta(static_cast<size_t>(npix) * F, 0.0);
  std::vector<double> xref(static_cast<size_t>(npix) * F, 0.0);
  std::vector<double> theta_full;                           // only for identity check
  std::vector<double> Rref;
  std::vector<int32_t> tref(npix, 0);
  const bool explicit_mode = mode == ORC_EXPLICIT_LAST || mode == ORC_EXPLICIT_NEW;
  const bool thresholded = mode == ORC_THRESHOLDED || explicit_mode;
  if ((check_identity && mode == ORC_THRESHOLDED) || explicit_mode) {
    theta_full.assign(static_cast<size_t>(npix) * P, 0.0);
    Rref.assign(npix, 0.0);
  }
  const bool every = mode == ORC_EXHAUSTIVE_ALL || mode == ORC_RAW_ALL;
  std::vector<signed char> fire(npix, 0);
  std::vector<double> value(npix, 0.0);
  std::vector<double> cur(npix, 0.0), prev(npix, 0.0);   // every crossing: L_t, L_{t-1}
  std::vector<int64_t> ncross(npix, 0);
  double max_err = 0.0;
  int64_t nev = 0;

  auto init_or_update = [&](int64_t k, int t, const Fit& fit) {
    ref[k] = fit.theta[0];
    const int64_t pix = pix_of(k);
    for (int f = 0; f < F; ++f) {
      beta[k * F + f] = fit.theta[3 + f];
      xref[k * F + f] = cl.feat(t, f, static_cast<int>(pix / c->W), static_cast<int>(pix % c->W));
    }
    tref[k] = t;
    if (!theta_full.empty()) {
      for (int j = 0; j < P; ++j) theta_full[k * P + j] = fit.theta[j];
      Rref[k] = fit.R;
    }
  };

  for (int t = 0; t < T; ++t) {
    double frame_err = 0.0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(max : frame_err)
    for (int64_t k = 0; k < npix; ++k) {
      const int64_t pix = pix_of(k);
      const int py = static_cast<int>(pix / c->W), px = static_cast<int>(pix % c->W);
      fire[k] = 0;
      if (thresholded) {
        if (t == 0) {
          Fit fit = regress(cl, p, 0, py, px, false, false);
          init_or_update(k, 0, fit);
          value[k] = NAN;
          continue;
        }
        if (explicit_mode) {
          double dR = 0.0;
          const double v = explicit_change(cl, p, mode == ORC_EXPLICIT_NEW ? 1 : 0, tref[k], t, py, px,
                                           &theta_full[k * P], &dR);
          value[k] = v;
          if (dR >= p->C * p->C) {
            fire[k] = v > 0 ? 1 : -1;
            Fit fit = regress(cl, p, t, py, px, false, false);
            init_or_update(k, t, fit);
          }
          continue;
        }
        double dlh = 0.0;
        for (int f = 0; f < F; ++f)
          dlh += beta[k * F + f] * (cl.feat(t, f, py, px) - xref[k * F + f]);
        value[k] = dlh;
        if (check_identity) {
          // Explicit eq. (7) over the last-event window, compared with Prop. 1.
          Fit old = regress(cl, p, tref[k], py, px, false, true);
          std::vector<double> xhat(old.xc);
          for (int f = 0; f < F; ++f) xhat[2 + f] = cl.feat(t, f, py, px);
          const double Rh = residual_hat(old, xhat.data(), D);
          const double err = std::fabs(std::fabs(Rh - old.R) - dlh * dlh) / std::max(1.0, Rh);
          frame_err = std::max(frame_err, err);
        }
        if (dlh * dlh >= p->C * p->C) {
          fire[k] = dlh > 0 ? 1 : -1;
          Fit fit = regress(cl, p, t, py, px, false, false);
          init_or_update(k, t, fit);
        }
      } else {
        double L;
        if (mode == ORC_EXHAUSTIVE || mode == ORC_EXHAUSTIVE_ALL) {
          Fit fit = regress(cl, p, t, py, px, false, false);
          L = fit.theta[0];
        } else {
          L = cl.y(t, py, px);
        }
        if (t == 0) {
          ref[k] = L;
          cur[k] = L;
          value[k] = NAN;
          continue;
        }
        const double d = L - ref[k];
        value[k] = d;
        if (every) {
          // levels passed; the events and the move of L_ref are taken in the
          // ordered pass below, which needs L_{t-1}
          const double q = std::floor(std::fabs(d) / p->C);
          ncross[k] = (std::isfinite(q) && q >= 1.0) ? static_cast<int64_t>(q) : 0;
          fire[k] = ncross[k] > 0 ? (d > 0 ? 1 : -1) : 0;
          prev[k] = cur[k];
          cur[k] = L;
        } else if (std::fabs(d) >= p->C) {
          fire[k] = d > 0 ? 1 : -1;
          ref[k] = L;
        }
      }
    }
    max_err = std::max(max_err, frame_err);
    int64_t frame_events = 0;
    for (int64_t k = 0; k < npix; ++k) {
      if (dl) dl[static_cast<int64_t>(t) * npix + k] = value[k];
      if (fire[k] == 0) continue;
      const int64_t pix = pix_of(k);
      const int64_t n = every ? ncross[k] : 1;
      for (int64_t j = 1; j <= n; ++j) {
        if (nev < cap) {
          ex[nev] = static_cast<int32_t>(pix % c->W);
          ey[nev] = static_cast<int32_t>(pix / c->W);
          et[nev] = t;
          ep[nev] = fire[k];
          if (ets) {
            if (every) {
              const double level = ref[k] + static_cast<double>(j) * fire[k] * p->C;
              ets[nev] = (t - 1) + (level - prev[k]) / (cur[k] - prev[k]);
            } else {
              ets[nev] = t;
            }
          }
        }
        ++nev;
        ++frame_events;
      }
      if (every) ref[k] += static_cast<double>(n) * fire[k] * p->C;
    }
    if (nflag) nflag[t] = frame_events;
  }
  for (int64_t k = 0; k < npix; ++k) {
    if (st_alpha) st_alpha[k] = ref[k];
    if (thresholded) {
      for (int f = 0; f < F; ++f) {
        if (st_beta) st_beta[static_cast<int64_t>(f) * npix + k] = beta[k * F + f];
        if (st_xref) st_xref[static_cast<int64_t>(f) * npix + k] = xref[k * F + f];
      }
      if (st_tref) st_tref[k] = tref[k];
    }
  }
  if (max_identity_err) *max_identity_err = max_err;
  return nev;
}

// Adjoint of alpha at a list of regressions (items = t * H * W + pixel) with
// upstream gradients galpha[n].  Accumulates into gy[T][H][W] and gb[F+2].
//
// With A = (1/W) sum w z z^T + lambda E (E = diag(0, 1, .., 1)),
// g = (1/W) sum w y z, theta = A^{-1} g, v = A^{-1} e_0, s_i = v^T z_i and
// r_i = y_i - z_i^T theta:
//   d alpha / d y_i   = (w_i / W) s_i
//   d alpha / d w_i   = (s_i r_i - lambda v^T E theta) / W
//   d w_i   / d b_j   = w_i u_ij^2 / (h^2 b_j^3)
int orc_backward(const orc_clip* c, const orc_params* p, const int64_t* items, int64_t n,
                 const double* galpha, double* gy, double* gb) {
  Clip cl{c};
  const int F = c->F, D = F + 2, P = D + 1;
  const int64_t HW = static_cast<int64_t>(c->W) * c->H;
  int fails = 0;
  for (int64_t it = 0; it < n; ++it) {
    const double ga = galpha[it];
    if (ga == 0.0) continue;
    const int t = static_cast<int>(items[it] / HW);
    const int pix = static_cast<int>(items[it] % HW);
    Fit fit = regress(cl, p, t, pix / c->W, pix % c->W, false, true);
    std::vector<double> L;
    if (!cholesky(fit.A, P, L)) {
      ++fails;
      continue;
    }
    std::vector<double> e0(P, 0.0), v(P);
    e0[0] = 1.0;
    chol_solve(L, P, e0.data(), v.data());
    double vEtheta = 0.0;
    for (int j = 1; j < P; ++j) vEtheta += v[j] * fit.theta[j];
    for (const Sample& s : fit.win) {
      double si = 0.0, pred = 0.0;
      for (int j = 0; j < P; ++j) {
        si += v[j] * s.z[j];
        pred += fit.theta[j] * s.z[j];
      }
      const double ri = s.yv - pred;
      gy[(static_cast<int64_t>(s.t) * c->H + s.py) * c->W + s.px] += ga * s.w / fit.W * si;
      const double dadw = (si * ri - p->ridge * vEtheta) / fit.W;
      for (int j = 0; j < D; ++j) {
        const double u = s.z[1 + j];
        const double bj = p->b[j];
        gb[j] += ga * dadw * s.w * u * u / (p->h * p->h * bj * bj * bj);
      }
    }
  }
  return fails;
}

}  // extern "C"
