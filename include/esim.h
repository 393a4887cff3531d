/*
 * esim.h -- C ABI of the MI355X event simulator (libesim.so).
 *
 * The library turns noisy log-brightness frames plus per-pixel feature
 * buffers into DVS events (x, y, t, polarity), following
 * Tsuji, Yatagawa, Kubo, Morishima, "Event-based Camera Simulation using Monte
 * Carlo Path Tracing with Adaptive Denoising", arXiv 2303.02608:
 *
 *   - Sec. 1.1, eq. (1): an event fires when the log-brightness change since
 *     the pixel's last event reaches the contrast threshold C.
 *   - Sec. 2.1, eqs. (2)-(5): weighted local regression (WLR) of the log
 *     brightness y over a window of neighbours, with Gaussian feature weights.
 *   - Sec. 2.2, eqs. (6)-(9) and Prop. 1: the residual of the last-event plane
 *     translated to the new centre feature differs from the plane's own
 *     residual by (beta^T (x^c - x_hat^c))^2; comparing that difference with
 *     C^2 decides whether the regression has to be solved again.
 *   - Sec. 3: the "WLR+ESIM" baseline (regress every pixel of every frame, then
 *     eq. (1)) and the "ESIM" baseline (eq. (1) on the noisy frames).
 *
 * Conventions
 *   - Every data pointer is DEVICE memory owned by the caller, except the
 *     structs passed by pointer (host memory, read during the call only).
 *   - Hot calls (log_brightness, threshold, regress, events, backward) are
 *     asynchronous on the given stream (a hipStream_t; NULL = null stream),
 *     allocate nothing, never synchronise, and may be captured in a hipGraph.
 *     Argument validation is synchronous and happens before anything is
 *     enqueued: on an error nothing has been launched.
 *   - Pixel p of a clip is p = py * W + px; arrays are planar (SoA).
 *   - A work item is an int64: bits [0,32) pixel, bits [32,44) clip index in the
 *     plan, bits [44,63) frame (only used where a call says so).  The value -1
 *     is a padding entry and is skipped.
 *   - Entry points catch every exception; none crosses the ABI.
 */
#ifndef ESIM_H_
#define ESIM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ESIM_MAX_F 12                 /* feature-buffer channels supported   */
#define ESIM_MAX_D (ESIM_MAX_F + 2)   /* plus the two image coordinates      */

typedef enum {
  ESIM_OK = 0,
  ESIM_E_INVAL = -1,        /* bad argument; nothing enqueued                  */
  ESIM_E_HIP = -2,          /* HIP runtime or launch error                     */
  ESIM_E_CAPACITY = -3,     /* a buffer is known to be too small               */
  ESIM_E_UNSUPPORTED = -4   /* valid request outside what the build supports   */
} esim_status;

typedef enum { ESIM_F32 = 0, ESIM_F16 = 1 } esim_dtype;

/* esim_events modes */
typedef enum {
  ESIM_INIT = 0,          /* store the frame's models as the reference state  */
  ESIM_THRESHOLDED = 1,   /* the paper's method (Sec. 2.2)                     */
  ESIM_EXHAUSTIVE = 2,    /* WLR+ESIM: eq. (1) on the regressed alpha           */
  ESIM_RAW = 3            /* ESIM on the noisy frames: eq. (1) on y            */
} esim_mode;

/* Gram precision of the regression */
typedef enum {
  ESIM_GRAM_F64 = 0,      /* FP32 weights, FP64 Gram and FP64 Cholesky (default) */
  ESIM_GRAM_F32C = 1      /* FP32 regressors and weights, FP32 Gram with
                             block-compensated (Neumaier) sums, FP32 Cholesky,
                             FP64 re-solve of the compensated Gram when the
                             Hager condition estimate exceeds kappa_fp64.
                             Compiled for F in {7, 10}, lanes 4 and 16.        */
} esim_precision;

/* How the threshold of a thresholded conversion evaluates Delta R = |R_hat - R|
 * (Sec. 2.2, eqs. (4), (7) and Prop. 1).  The two explicit forms are an
 * ablation of the closed form; they need the state's bxy. */
typedef enum {
  ESIM_THRESHOLD_CLOSED = 0,      /* Prop. 1: Delta R = dL^2 with dL = beta_ref^T
                                     (f_t - xref) over the F buffer channels
                                     (default: the paper's method)            */
  ESIM_THRESHOLD_LAST_WINDOW = 1, /* eq. (7) summed over the last-event window:
                                     the samples, weights and centre of the
                                     frame t_ref, the centre feature replaced
                                     by frame t's; R of eq. (4) over the same
                                     window for the stored plane.  Equal to the
                                     closed form at the least-squares minimiser */
  ESIM_THRESHOLD_NEW_WINDOW = 2   /* eq. (7) summed over frame t's window (its
                                     samples, and weights of eq. (5) about
                                     frame t's centre feature vector); R as
                                     above.  Also sees brightness changes that
                                     the features do not explain              */
} esim_threshold;

/* One clip.  y = log brightness [T][H][W] (see esim_log_brightness); feat =
 * the F feature buffers [T][F][H][W] in feat_dtype.  The image coordinates
 * are implicit features (px / r, py / r). */
typedef struct {
  int32_t W, H, T, F;
  int32_t feat_dtype;
  const float* y;
  const void* feat;
} esim_clip;

/* Method parameters of one clip (Sec. 2.1 eq. 5; Sec. 1.1 eq. 1). */
typedef struct {
  int32_t r;               /* spatial window radius, >= 1                       */
  int32_t tr;              /* temporal radius in frames, >= 0                    */
  double C;                /* contrast threshold, > 0                           */
  double h;                /* global bandwidth, > 0 (paper: 1)                  */
  double b[ESIM_MAX_D];    /* per-dimension bandwidths, coordinates first, > 0  */
  double ridge;            /* lambda >= 0 added to the beta block of the
                              W-normalised Gram (the alpha row is untouched)    */
  int32_t precision;       /* esim_precision                                    */
  double kappa_fp64;       /* ESIM_GRAM_F32C: bound on kappa-hat               */
  int32_t multi_crossing;  /* exhaustive and raw modes: 0 = at most one event per
                              pixel-frame, L_ref reset to the current value (the
                              paper's fixed-interval ESIM, Sec. 3); 1 = ESIM with
                              every crossing: n = floor(|L - L_ref| / C) events,
                              the brightness taken as linear between frames, at
                              the fractional times the levels L_ref + k p C are
                              passed, and L_ref <- L_ref + n p C (n capped at
                              2^20 per pixel-frame).  Needs the state's `last`.
                              Ignored by the thresholded mode.                  */
  int32_t threshold;       /* esim_threshold; the same for every clip of a plan  */
  double dt;               /* time between frames, > 0 and finite (Sec. 3: the
                              frames are rendered at fixed times; the DVS
                              workload uses 1 ms): event times are t * dt     */
} esim_params;

/* Per-pixel reference state (Sec. 2.2: one regression model per pixel, kept
 * until the pixel's next event).  alpha also holds L_ref of the exhaustive and
 * raw baselines.  beta holds only the F buffer channels: the image-coordinate
 * part of x^c - x_hat^c is zero for a pixel. */
typedef struct {
  float* alpha;            /* [H*W]                                              */
  float* beta;             /* [F][H*W]                                           */
  float* xref;             /* [F][H*W]  feature vector at the last event          */
  int32_t* tref;           /* [H*W]     frame of the last event                    */
  float* last;             /* [H*W]     compared value of the previous frame
                              (multi_crossing only; nullable otherwise)         */
  float* bxy;              /* [2][H*W]  image-coordinate components of beta
                              (x, then y) at the last event: the explicit
                              thresholds need the whole plane.  Written, when
                              non-NULL, by esim_events' model updates and by
                              every step of a plan with an explicit threshold
                              (the closed-form step leaves it untouched).     */
  float* rmom;             /* [2][H*W]  window sums of the stored plane over its
                              own (last-event) window, taken when the model is
                              stored: R of eq. (4), then the weighted mean
                              residual m1 = sum w r / W.  Explicit thresholds
                              only (nullable otherwise).                       */
} esim_state;

/* Event sink.  Events are appended in (t, clip, py, px) order at *count (the
 * events of one pixel-frame in time order); an event whose index reaches
 * `capacity` is dropped but still counted, so a caller detects overflow by
 * *count > capacity after synchronising.  `clip` and `ts` may be NULL.
 * `t` receives the frame index; `ts` the event's time in the unit of the
 * clip's dt: t * dt, or with multi_crossing the interpolated crossing time
 * in ((t - 1) * dt, t * dt]. */
typedef struct {
  int32_t* x;
  int32_t* y;
  int32_t* t;
  int8_t* p;               /* polarity, +1 or -1                                */
  int32_t* clip;
  int64_t capacity;
  int64_t* count;          /* device, running total                             */
  float* ts;               /* nullable: time of each event in frame units       */
} esim_events_buf;

typedef struct esim_plan_s* esim_plan;

/* ---- set-up (not hot: these allocate and copy) ------------------------- */

/* Build a plan over nclips clips (1 = the plain single-clip form; > 1 = the
 * batched form).  Copies the clip descriptors, parameters and state pointers
 * to the device and allocates the compaction workspace.  The plan keeps the
 * pointers, not the data: the caller keeps y, feat and the states alive.
 * Errors: E_INVAL (bad shape, F outside 1..ESIM_MAX_F, bad parameter),
 * E_UNSUPPORTED (2^31 pixels or more over the clips, mixed F or feature dtype
 * or threshold form, a window of 4 GiB or more), E_HIP (allocation or copy
 * failed). */
int esim_plan_create(const esim_clip* clips, const esim_params* params,
                     const esim_state* states, int32_t nclips, esim_plan* out);
/* Frees the plan's device buffers and the plan (a null plan is accepted).
 * Returns E_HIP if a free fails; the plan is released in any case. */
int esim_plan_destroy(esim_plan plan);

/* Total pixels over the plan's clips (sum of H*W): the length of dl, of dense
 * regression outputs and of a work list, without padding. */
int64_t esim_plan_pixels(esim_plan plan);
/* Work-list capacity a threshold call may need: the plan's pixels. */
int64_t esim_plan_worklist_capacity(esim_plan plan);
/* First pixel of clip c in the concatenated pixel range. */
int64_t esim_plan_pixel_offset(esim_plan plan, int32_t c);

/* Schedule of the regression kernel (set by the autotuner, or by hand): the
 * lanes that share one regression item in dense launches and in work-list
 * launches (1, 2, 4, 8 or 16; more lanes = more, shorter wave tasks for sparse
 * lists) and the persistent blocks per CU (1..64).  Defaults 1, 16, 4 (4, 16, 4 with
 * ESIM_GRAM_F32C).
 * Errors: E_UNSUPPORTED (lanes not compiled), E_INVAL. */
int esim_plan_set_schedule(esim_plan plan, int32_t lanes_dense, int32_t lanes_list,
                           int32_t blocks_per_cu);

/* ---- hot path ---------------------------------------------------------- */

/* Log brightness (Sec. 1.1, L = log E): y[i] = log(E[i] + eps), elementwise, n values.
 * Errors: E_INVAL (null pointer, n < 0, eps < 0). */
int esim_log_brightness(const float* E, float* y, int64_t n, float eps, void* stream);

/* Threshold and compaction (Sec. 2.2, Prop. 1, eqs. 8-9): for every pixel of every clip with
 * 1 <= t < T, dL = sum_f beta_ref[f] (feat_t[f] - xref[f]) over the F buffer
 * channels (computed in FP64 from the FP32 state), written to dl[pixel offset
 * + p] (NaN for clips inactive at t); a pixel is flagged when dL^2 >= C^2.
 * With an explicit esim_threshold, Delta R = |R_hat - R| comes from window sums
 * of the stored plane (alpha, bxy, beta) in FP64 with FP32 weights as in the
 * regression.  R and m1 are the state's rmom.  Over the last-event window the
 * samples are those of t_ref and only the centre moves, so the translated
 * residuals are r_i + d with d = beta^T (x_hat^c - x^c) and eq. (7) expands
 * exactly: R_hat = R + 2 d m1 + d^2, mean m1 + d.  Over frame t's window
 * R_hat and the mean are summed at frame t.  A pixel is flagged when
 * Delta R >= C^2; dl receives s * sqrt(Delta R), s (the sign of the event)
 * being the sign of the weighted mean of the translated plane's residuals
 * y^i - alpha - beta^T (x^i - x_hat^c) (-1 when the mean is 0).  Over the
 * last-event window s * sqrt(Delta R) is dL up to the m1 term (zero at the
 * least-squares minimiser).  The explicit forms need bxy, rmom and clips
 * whose features stay below 4 GiB (E_UNSUPPORTED otherwise).
 * Flagged pixels are compacted into worklist as items (clip << 32 | p), in
 * ascending (clip, p) order.  count[0] = count[1] = flagged pixels (the work-list
 * length; a wave of the regression may straddle two clips).
 * dl must hold esim_plan_pixels values, worklist
 * esim_plan_worklist_capacity items, count two int32. */
int esim_wlr_threshold(esim_plan plan, int32_t t, float* dl, int64_t* worklist,
                       int32_t* count, void* stream);

/* Weighted local regression (Sec. 2.1, eqs. 3-5): weighted local regression at
 *   - the listed items (worklist != NULL; *count is read on the device and
 *     clamped to n_out, so worklist must hold min(*count, n_out) entries;
 *     item i's results go to index i), or
 *   - every pixel of every clip active at t (worklist == NULL; the results of
 *     pixel p of clip c go to index pixel_offset(c) + p).
 * If t >= 0 every item is regressed at frame t; if t < 0 each item carries its
 * frame in bits [44,63) (then every clip's feature and brightness arrays must
 * stay below 4 GiB).
 * Outputs (n_out = stride of beta, >= the largest index written):
 *   alpha[i]          = fitted value at the centre (eq. 3's f(x^c)),
 *   beta[d * n_out + i] (nullable) = gradient over the D = F + 2 features,
 *                       coordinates first,
 *   resid[i] (nullable) = R of eq. (4) at the minimiser,
 *   kappa[i] (nullable) = kappa-hat: the 1-norm condition number of the
 *                       equilibrated system As = S^-1 A S^-1 (S^2 = diag(A),
 *                       unit diagonal), ||As||_1 times Hager's estimate of
 *                       ||As^{-1}||_1 from A's Cholesky factor; A is the
 *                       W-normalised Gram plus ridge in bandwidth-scaled
 *                       regressors u_j / (h b_j).  A lower bound of
 *                       kappa_1(As), which (van der Sluis) governs the
 *                       rounding error of the Cholesky solve.  With
 *                       ESIM_GRAM_F32C it is the FP32 estimate that decides
 *                       the FP64 re-solve (re-solved iff it exceeds
 *                       kappa_fp64 or is not finite).
 * Errors: E_INVAL (null outputs, n_out too small for dense mode),
 * E_UNSUPPORTED (t < 0 with a clip of 4 GiB or more of features or brightness). */
int esim_wlr_regress(esim_plan plan, int32_t t, const int64_t* worklist, const int32_t* count,
                     int64_t n_out, float* alpha, float* beta, float* resid, float* kappa,
                     void* stream);

/* Events and state updates (Sec. 1.1 eq. 1; Sec. 2.2; Sec. 3):
 *   ESIM_INIT:        every pixel of every clip active at t: state <- (alpha,
 *                     beta over the F buffer channels, feat_t, t; bxy from
 *                     beta's coordinate rows when the state has bxy) from
 *                     dense regression outputs (index pixel_offset(c) + p,
 *                     stride n_out).  No events.  Plans with an explicit
 *                     threshold then sum rmom over each stored plane's window.
 *   ESIM_THRESHOLDED: for the work-list items of a threshold call at t: emit
 *                     (px, py, t, sign dl) and replace the state with the
 *                     item's regression (alpha[i], beta[.., i], bxy and rmom
 *                     as for INIT), feat_t and t.  n_out must be at least
 *                     esim_plan_worklist_capacity (E_INVAL otherwise), so that
 *                     every item a threshold call can list has its outputs.
 *   ESIM_EXHAUSTIVE:  every pixel: d = alpha - state.alpha (L_ref); if
 *                     |d| >= C emit sign d and set L_ref <- alpha.  At t = 0
 *                     (or for a fresh state) call ESIM_INIT first.
 *   ESIM_RAW:         as EXHAUSTIVE with alpha replaced by y_t.  Pass
 *                     alpha = NULL; mode INIT with alpha = NULL stores y_t.
 * dl is the threshold call's output (THRESHOLDED and EXHAUSTIVE/RAW write the
 * compared change to it when non-NULL in the latter two).
 * Errors: E_INVAL (mode, missing buffers, n_out). */
int esim_events(esim_plan plan, int32_t t, int32_t mode, const int64_t* worklist,
                const int32_t* count, float* dl, const float* alpha, const float* beta,
                int64_t n_out, esim_events_buf* ev, void* stream);

/* One frame of a conversion (Sec. 2.2; Sec. 3) with the plan's own work
 * buffers, in as few launches as the step allows; the same results as the
 * per-frame calls above (same kernels and arithmetic):
 *   ESIM_INIT:        regress every pixel active at t and store the models in
 *                     the state (no events).
 *   ESIM_THRESHOLDED: threshold (Prop. 1) at t >= 1, append the flagged
 *                     pixels' events (sign of dL, during the compaction), and
 *                     regress the flagged pixels, each regression writing its
 *                     model straight into the state.  In a plan whose clips'
 *                     windows lie on both sides of 16 columns (2r + 1), the
 *                     compaction puts the two kinds in separate segments of the
 *                     plan's work list and each segment gets its own launch.  With an explicit
 *                     esim_threshold the models pass through the plan's
 *                     buffers (one more launch, so that bxy is written too)
 *                     and a last launch sums rmom over the new planes.
 *   ESIM_EXHAUSTIVE:  regress every pixel, then eq. (1) on alpha (as
 *                     esim_events).
 *   ESIM_RAW:         eq. (1) on y_t.
 * dl (nullable, esim_plan_pixels values) receives the compared change.
 * The plan's internal work list and dense outputs are overwritten; calls on
 * one plan must be ordered on one stream.  Events are appended at *ev->count
 * (the true total is always counted; entries beyond capacity are dropped).
 * Errors: E_INVAL (t, mode, missing state or events buffer), E_UNSUPPORTED. */
int esim_step(esim_plan plan, int32_t t, int32_t mode, float* dl, esim_events_buf* ev,
              void* stream);

/* Adjoint of alpha (eqs. 4-5 differentiated) at n regressions.  items
 * carry their frame (bits [44,63)) and must be distinct; g_alpha[n] is the
 * upstream gradient.  With A the W-normalised Gram plus ridge, theta its
 * solution, v = A^{-1} e_0, s_i = v^T z_i, r_i = y_i - z_i^T theta:
 *   g_y[t'][py'][px'] += sum_items g_alpha (w_i / W) s_i          (gather,
 *                        deterministic: no atomics)
 *   g_b[j]            += sum_items g_alpha sum_i (s_i r_i - lambda v^T E theta)
 *                        / W * w_i u_ij^2 / (h^2 b_j^3),  j < F + 2.
 * The window is recomputed, not stored.  Single-clip plans only; the clip's
 * features and brightness must each stay below 4 GiB, and r <= 25.  scratch: esim_backward_scratch_bytes.
 * Errors: E_INVAL, E_CAPACITY (scratch too small), E_UNSUPPORTED. */
size_t esim_backward_scratch_bytes(esim_plan plan, int64_t n);
int esim_wlr_backward(esim_plan plan, const int64_t* items, int64_t n, const float* g_alpha,
                      float* g_y, double* g_b, void* scratch, size_t scratch_bytes, void* stream);

/* ---- bandwidth optimisation ---------------------------------------------- */

/* MC variance of the log brightness (Sec. 1.1: y = log E): for the mean E of
 * spp radiance samples with unbiased sample variance var, the delta method
 * gives vy[i] = var[i] / spp / (E[i] + eps)^2, elementwise, n values.
 * Errors: E_INVAL (null pointer, n < 0, spp < 1, eps < 0). */
int esim_log_variance(const float* E, const float* var, int32_t spp, float* vy, int64_t n, float eps,
                      void* stream);

/* Bandwidth-optimised regression (Sec. 3, bandwidth optimisation: the
 * bandwidths of eq. (5) chosen per pixel from the bias and the MC variance).
 * The paper gives the criterion, not the estimator; here only the global
 * bandwidth h is chosen, among the K candidates hs[0..K) (host array,
 * replacing the plan's h), by the smallest Stein's unbiased risk estimate of
 * alpha's mean squared error:
 *     SURE(h) = (alpha_h - y_c)^2 + 2 vy_c v_0 / W_h - vy_c,   v = A_h^{-1} e_0,
 * alpha_h's weight on the centre sample being v_0 / W_h.  The first of equal
 * values wins; a failed factor never does (its outputs stay NaN if all fail).
 * Items as in esim_wlr_regress with a frame t >= 0: the work list (item i's
 * results at index i, *count read on the device and clamped to n_out) or, with
 * worklist NULL, every pixel (index p, n_out >= H*W).  Outputs: alpha[i];
 * beta[d * n_out + i] over D (nullable); hsel[i] the chosen h (nullable);
 * sure[i] its SURE (nullable).  vy: [T][H][W], the variance of y
 * (esim_log_variance).  Single-clip plans, FP64 Gram; K window passes per
 * item (one lane per pixel for every pixel of the frame, 16 lanes per item for
 * work lists).
 * Errors: E_INVAL (K outside 1..8, h <= 0, null pointers, n_out),
 * E_UNSUPPORTED (several clips). */
int esim_wlr_regress_bandwidth(esim_plan plan, int32_t t, const int64_t* worklist, const int32_t* count,
                               int64_t n_out, const float* vy, const double* hs, int32_t K, float* alpha,
                               float* beta, float* hsel, float* sure, void* stream);

/* ---- event-set comparison ------------------------------------------------ */

/* Nearest same-polarity neighbour distances (Sec. 3, "Quantitative comparison":
 * events are signed points (x, y, t); precision and recall count the events of
 * one set whose closest event of the same polarity in the other set lies
 * within a distance threshold).  For each of the nq query events, d[i] is the
 * Euclidean distance, in the scaled coordinates (x scale_x, y scale_y,
 * t scale_t), to the nearest of the ns source events with the same polarity
 * (p = +1 or -1), or +inf when none lies within rmax.  The search is exact
 * within rmax.  Events outside [0, W) x [0, H) x [0, T) or with another p are
 * ignored as sources and get +inf as queries.  All arrays are device memory;
 * d is FP64.  scratch: esim_nn_scratch_bytes(W, H, T) bytes of device memory
 * (occupancy bitmaps, overwritten).  The x extent of rmax, rmax / scale_x, must
 * stay below 4096 columns.
 * Errors: E_INVAL (shapes, scales, null pointers), E_CAPACITY (scratch too
 * small), E_UNSUPPORTED (radius too wide). */
size_t esim_nn_scratch_bytes(int32_t W, int32_t H, int32_t T);

/* The same search for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops): the occupancy bitmaps live in a
 * fixed device array of ESIM_NN_STATIC_BYTES bytes inside the library, one
 * per GPU, held until the process ends; nothing is allocated, by the library
 * or by the caller.  Arguments as esim_nn_distances without the scratch.
 * The first call on a device looks the array up (hipGetSymbolAddress);
 * capture a graph only after one call on that device.  Every call on a GPU
 * shares that GPU's array and clears the part it uses first: calls that
 * overlap on one GPU (different streams, or graph replays in flight) race and
 * must be serialised by the caller.
 * Errors: as esim_nn_distances; E_CAPACITY when esim_nn_scratch_bytes(W, H, T)
 * exceeds ESIM_NN_STATIC_BYTES; E_HIP if the array cannot be looked up. */
#define ESIM_NN_STATIC_BYTES ((size_t)32 << 20)
int esim_nn_distances_noalloc(const int32_t* src_x, const int32_t* src_y, const int32_t* src_t,
                              const int8_t* src_p, int64_t ns, const int32_t* qry_x, const int32_t* qry_y,
                              const int32_t* qry_t, const int8_t* qry_p, int64_t nq, int32_t W, int32_t H,
                              int32_t T, double scale_x, double scale_y, double scale_t, double rmax, double* d,
                              void* stream);
int esim_nn_distances(const int32_t* src_x, const int32_t* src_y, const int32_t* src_t,
                      const int8_t* src_p, int64_t ns, const int32_t* qry_x, const int32_t* qry_y,
                      const int32_t* qry_t, const int8_t* qry_p, int64_t nq, int32_t W, int32_t H,
                      int32_t T, double scale_x, double scale_y, double scale_t, double rmax, double* d,
                      void* scratch, size_t scratch_bytes, void* stream);

/* ---- diagnostics ------------------------------------------------------- */
const char* esim_status_string(int status);
/* Message of the last failed call on this thread ("" if none). */
const char* esim_last_error(void);
/* Build information: the offload target and the compiled kernel variants. */
const char* esim_build_info(void);

#ifdef __cplusplus
}
#endif

#endif  /* ESIM_H_ */
