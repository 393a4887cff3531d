// Host side of libesim: plans, argument validation and launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "esim.h"
#include "esim_bandwidth.h"
#include "esim_compact.h"
#include "esim_internal.h"

struct esim_plan_s {
  int nclips = 0;
  int F = 0;
  bool f16 = false;
  std::vector<esim::ClipDev> host;
  esim::ClipDev* dev = nullptr;
  esim::Workspace ws{};
  void* ws_mem = nullptr;
  int64_t npix = 0;
  int64_t nblk = 0;
  int64_t wl_capacity = 0;
  int64_t dense_groups[5] = {0, 0, 0, 0, 0};
  int lanes_dense = 1;     // lanes per regression item, dense launches
  int lanes_list = 16;     // lanes per regression item, work-list launches
  int blocks_per_cu = 4;   // persistent grid: 256 CUs x this many blocks
  uint64_t max_feat_bytes = 0;   // largest feature array of a clip
  uint64_t max_y_bytes = 0;      // largest brightness array of a clip
  esim::DeviceShape shape;       // compute units and XCDs of the plan's device
  // work buffers of esim_step (allocated with the plan)
  void* step_mem = nullptr;
  int64_t* xcd_bounds = nullptr;  // [5 lane counts][kMaxXcds + 1] dense group bounds per XCD (device)
  int64_t* step_wl = nullptr;     // [wl_capacity]
  int32_t* step_count = nullptr;  // [4] (two segments of a split work list)
  // esim_step's split work list: clips whose windows fit 16 columns (the
  // one-pass list instance) in the first segment, wider ones from split_seg
  // on (-1: one segment); the largest r of each segment
  int64_t split_seg = -1;
  int split_r[2] = {0, 0};
  float* step_alpha = nullptr;    // [npix]
  float* step_beta = nullptr;     // [F + 2][npix] (explicit thresholds only)
  int thr = ESIM_THRESHOLD_CLOSED;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int ok() {
  g_last_error.clear();
  return ESIM_OK;
}

int hip_check(hipError_t e, const char* where) {
  if (e != hipSuccess) return fail(ESIM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
  return ok();
}


}  // namespace

namespace esim {

bool query_device_shape(DeviceShape& out) {
  int dev = 0, cus = 0, xccs = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return false;
  if (hipDeviceGetAttribute(&xccs, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || xccs < 1) xccs = 1;
  out.cus = cus;
  out.xcds = xccs > kMaxXcds ? 1 : xccs;
  return true;
}

}  // namespace esim

namespace {

int launch_plan_regress(esim_plan pl, int32_t t, const int64_t* worklist, const int32_t* count,
                        int64_t n_out, float* alpha, float* beta, float* resid, float* kappa,
                        bool update_state, hipStream_t stream, int max_r = -1) {
  // the condition estimate of the FP64 Gram comes from a one-lane instance
  const bool kappa_f64 = kappa && pl->host[0].precision == ESIM_GRAM_F64;
  const int L = kappa_f64 ? 1 : worklist ? pl->lanes_list : pl->lanes_dense;
  if (!esim::regress_supports(pl->F, L, pl->host[0].precision))
    return fail(ESIM_E_UNSUPPORTED, "no kernel instance for this F, lane count and precision");
  esim::RegressArgs a{};
  a.clips = pl->dev;
  a.nclips = pl->nclips;
  a.t = t;
  a.items = worklist;
  a.count = count;
  a.n_dense_groups = pl->dense_groups[esim::lanes_index(L)];
  const int G = esim::kWave / L;
  a.max_groups = worklist ? (std::max<int64_t>(n_out, 1) + G - 1) / G : a.n_dense_groups;
  a.n_out = n_out;
  a.alpha = alpha;
  a.beta = beta;
  a.resid = resid;
  a.kappa = kappa;
  a.update_state = update_state ? 1 : 0;
  a.xcd_bounds = (!worklist && pl->nclips > 1) ? pl->xcd_bounds + (esim::kMaxXcds + 1) * esim::lanes_index(L)
                                                : nullptr;
  a.nxcd = pl->shape.xcds;
  if (max_r < 0)
    for (const auto& c : pl->host) max_r = std::max(max_r, static_cast<int>(c.r));
  return hip_check(esim::launch_regress(a, pl->F, pl->f16, pl->host[0].precision, L, pl->blocks_per_cu,
                                        max_r, pl->shape, stream),
                   "regress");
}

// The every-crossing rule keeps the previous frame's value in the state.
bool multi_state_ok(esim_plan pl) {
  for (const auto& c : pl->host)
    if (c.multi && !c.st_last) return false;
  return true;
}

bool full_state(esim_plan pl) {
  for (const auto& c : pl->host)
    if (!c.st_beta || !c.st_xref || !c.st_alpha || !c.st_tref) return false;
  if (pl->thr != ESIM_THRESHOLD_CLOSED)
    for (const auto& c : pl->host)
      if (!c.st_bxy || !c.st_rmom) return false;
  return true;
}

// The explicit thresholds read the whole stored plane and its window sums.
int explicit_ok(esim_plan pl) {
  if (pl->thr == ESIM_THRESHOLD_CLOSED) return ok();
  for (const auto& c : pl->host)
    if (!c.st_bxy || !c.st_rmom) return fail(ESIM_E_INVAL, "explicit thresholds need the state's bxy and rmom");
  return ok();
}

// After models were stored at frame t (work-list items, or every pixel when
// worklist is null): their window sums, for plans with an explicit threshold.
int store_moments(esim_plan pl, int32_t t, const int64_t* worklist, const int32_t* count, hipStream_t s) {
  if (pl->thr == ESIM_THRESHOLD_CLOSED) return ok();
  return hip_check(esim::launch_moments(pl->dev, pl->nclips, pl->nblk, t, pl->F, pl->f16, worklist, count,
                                        pl->wl_capacity, s),
                   "window sums of the stored planes");
}

// Threshold at t into the plan's workspace, then the compaction (work list,
// count and, with ev, the flagged pixels' events).
int threshold_compact(esim_plan pl, int32_t t, float* dl, int64_t* worklist, int32_t* count,
                      const esim::EventsDev* ev, hipStream_t s, int64_t seg_b = -1) {
  if (pl->thr == ESIM_THRESHOLD_CLOSED)
    return hip_check(esim::launch_flag_compact(pl->dev, pl->nclips, pl->nblk, t, esim::kFlagThreshold, dl,
                                               nullptr, pl->ws, worklist, count, ev, s, seg_b),
                     "threshold");
  int rc = explicit_ok(pl);
  if (rc != ESIM_OK) return rc;
  rc = hip_check(esim::launch_explicit_flag(pl->dev, pl->nclips, pl->nblk, t, pl->F, pl->f16, pl->thr, dl, pl->ws,
                                            ev ? ev->count : nullptr, s),
                 "threshold(explicit)");
  if (rc != ESIM_OK) return rc;
  return hip_check(esim::launch_scatter(pl->dev, pl->nclips, pl->nblk, t, esim::kFlagThreshold, nullptr,
                                        pl->ws, worklist, count, ev, s),
                   "threshold(compaction)");
}

}  // namespace

extern "C" {

const char* esim_status_string(int s) {
  switch (s) {
    case ESIM_OK: return "ok";
    case ESIM_E_INVAL: return "invalid argument";
    case ESIM_E_HIP: return "HIP error";
    case ESIM_E_CAPACITY: return "capacity exceeded";
    case ESIM_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* esim_last_error(void) { return g_last_error.c_str(); }

const char* esim_build_info(void) {
  return "libesim gfx950; regress: F=1..12 x lanes{1,2,4,8,16} x {f32,f16} features, FP64 Gram; "
         "compensated FP32 Gram for F in {7,10} x lanes {4,16}";
}

int esim_plan_create(const esim_clip* clips, const esim_params* params, const esim_state* states,
                     int32_t nclips, esim_plan* out) {
  try {
    if (!out) return fail(ESIM_E_INVAL, "out is null");
    *out = nullptr;
    if (!clips || !params || nclips < 1 || nclips > 4096)
      return fail(ESIM_E_INVAL, "clips/params null or nclips outside 1..4096");
    auto* pl = new esim_plan_s();
    pl->nclips = nclips;
    pl->F = clips[0].F;
    pl->f16 = clips[0].feat_dtype == ESIM_F16;
    int64_t pix = 0, blk = 0, grp[5] = {0, 0, 0, 0, 0};
    int64_t wl = 0;
    for (int c = 0; c < nclips; ++c) {
      const esim_clip& k = clips[c];
      const esim_params& p = params[c];
      char msg[256];
      if (k.W < 1 || k.H < 1 || k.T < 1 || static_cast<int64_t>(k.W) * k.H >= (1ll << 31)) {
        std::snprintf(msg, sizeof msg, "clip %d: bad shape W=%d H=%d T=%d", c, k.W, k.H, k.T);
        delete pl;
        return fail(ESIM_E_INVAL, msg);
      }
      if (k.F < 1 || k.F > ESIM_MAX_F) {
        delete pl;
        return fail(ESIM_E_UNSUPPORTED, "F outside 1..ESIM_MAX_F");
      }
      if (k.F != pl->F || (k.feat_dtype == ESIM_F16) != pl->f16 ||
          (k.feat_dtype != ESIM_F32 && k.feat_dtype != ESIM_F16)) {
        delete pl;
        return fail(ESIM_E_UNSUPPORTED, "all clips of a plan share F and the feature dtype");
      }
      if (!k.y || !k.feat) {
        delete pl;
        return fail(ESIM_E_INVAL, "clip y/feat null");
      }
      if (p.r < 1 || p.r > 64 || p.tr < 0 || p.tr > 16 || !(p.C > 0) || !(p.h > 0) ||
          !(p.ridge >= 0) || std::isinf(p.C)) {
        std::snprintf(msg, sizeof msg, "clip %d: bad params r=%d tr=%d C=%g h=%g ridge=%g", c, p.r,
                      p.tr, p.C, p.h, p.ridge);
        delete pl;
        return fail(ESIM_E_INVAL, msg);
      }
      if (p.precision != ESIM_GRAM_F64 && p.precision != ESIM_GRAM_F32C) {
        delete pl;
        return fail(ESIM_E_INVAL, "bad precision");
      }
      if (c > 0 && p.precision != params[0].precision) {
        delete pl;
        return fail(ESIM_E_UNSUPPORTED, "all clips of a plan share the precision");
      }
      if (!(p.dt > 0) || std::isinf(p.dt)) {
        delete pl;
        return fail(ESIM_E_INVAL, "dt must be positive and finite");
      }
      if (p.threshold < ESIM_THRESHOLD_CLOSED || p.threshold > ESIM_THRESHOLD_NEW_WINDOW) {
        delete pl;
        return fail(ESIM_E_INVAL, "bad threshold");
      }
      if (c > 0 && p.threshold != params[0].threshold) {
        delete pl;
        return fail(ESIM_E_UNSUPPORTED, "all clips of a plan share the threshold form");
      }
      for (int d = 0; d < k.F + 2; ++d)
        if (!(p.b[d] > 0) || std::isinf(p.b[d])) {
          delete pl;
          return fail(ESIM_E_INVAL, "bandwidths b must be positive and finite");
        }
      esim::ClipDev cd{};
      cd.y = k.y;
      cd.feat = k.feat;
      if (states) {
        cd.st_alpha = states[c].alpha;
        cd.st_beta = states[c].beta;
        cd.st_xref = states[c].xref;
        cd.st_tref = states[c].tref;
        cd.st_last = states[c].last;
        cd.st_bxy = states[c].bxy;
        cd.st_rmom = states[c].rmom;
      }
      cd.thr = p.threshold;
      cd.dt = p.dt;
      cd.W = k.W;
      cd.H = k.H;
      cd.T = k.T;
      cd.F = k.F;
      cd.feat_f16 = k.feat_dtype == ESIM_F16;
      cd.r = p.r;
      cd.tr = p.tr;
      cd.precision = p.precision;
      if (p.multi_crossing != 0 && p.multi_crossing != 1) {
        delete pl;
        return fail(ESIM_E_INVAL, "multi_crossing must be 0 or 1");
      }
      cd.multi = p.multi_crossing;
      cd.HW = static_cast<int64_t>(k.W) * k.H;
      cd.pix_off = pix;
      cd.blk_off = blk;
      cd.nblk = (cd.HW + esim::kBlock - 1) / esim::kBlock;
      const int Ls[5] = {1, 2, 4, 8, 16};
      for (int q = 0; q < 5; ++q) {
        cd.grp_off[q] = grp[q];
        grp[q] += (cd.HW + (esim::kWave / Ls[q]) - 1) / (esim::kWave / Ls[q]);
      }
      cd.C = p.C;
      cd.h = p.h;
      cd.ridge = p.ridge;
      cd.kappa_fp64 = p.kappa_fp64;
      for (int d = 0; d < ESIM_MAX_D; ++d) {
        const double bd = d < k.F + 2 ? p.b[d] : 1.0;
        cd.c2[d] = 1.0 / (p.h * bd * p.h * bd);
        cd.sf[d] = 1.0 / (p.h * bd);
        cd.gbk[d] = 1.0 / (p.h * p.h * bd * bd * bd);
      }
      pix += cd.HW;
      blk += cd.nblk;
      wl += cd.HW;
      const uint64_t fb = static_cast<uint64_t>(k.T) * k.F * cd.HW * (cd.feat_f16 ? 2u : 4u);
      const uint64_t wb = static_cast<uint64_t>(2 * p.tr + 1) * k.F * cd.HW * (cd.feat_f16 ? 2u : 4u);
      if (wb >= (1ull << 32) || static_cast<uint64_t>(2 * p.tr + 1) * cd.HW * 4u >= (1ull << 32)) {
        delete pl;
        return fail(ESIM_E_UNSUPPORTED, "the 2*tr+1 frames of a window must stay below 4 GiB");
      }
      pl->max_feat_bytes = std::max(pl->max_feat_bytes, fb);
      pl->max_y_bytes = std::max(pl->max_y_bytes, static_cast<uint64_t>(k.T) * cd.HW * 4u);
      pl->host.push_back(cd);
    }
    if (pix >= (1ll << 31)) {
      // work-list counts are 32-bit, and the split compaction sums them in the
      // low half of 64-bit block counts
      delete pl;
      return fail(ESIM_E_UNSUPPORTED, "a plan holds fewer than 2^31 pixels over its clips");
    }
    // the compensated-FP32 instances exist for 4 and 16 lanes only
    if (params[0].precision == ESIM_GRAM_F32C) pl->lanes_dense = 4;
    pl->thr = params[0].threshold;
    if (!esim::query_device_shape(pl->shape)) {
      delete pl;
      return fail(ESIM_E_HIP, "device attribute query failed");
    }
    pl->npix = pix;
    pl->nblk = blk;
    pl->wl_capacity = wl;
    {
      // the split work list of esim_step (multi-clip plans with windows on
      // both sides of 16 columns)
      int64_t seg = 0;
      bool narrow = false, wide = false;
      for (auto& cd : pl->host) {
        cd.list_class = 2 * cd.r + 1 > 16 ? 1 : 0;
        if (cd.list_class) {
          wide = true;
          pl->split_r[1] = std::max(pl->split_r[1], static_cast<int>(cd.r));
        } else {
          narrow = true;
          seg += cd.HW;
          pl->split_r[0] = std::max(pl->split_r[0], static_cast<int>(cd.r));
        }
      }
      pl->split_seg = narrow && wide ? seg : -1;
    }
    for (int q = 0; q < 5; ++q) pl->dense_groups[q] = grp[q];

    // device memory: descriptors + workspace
    const size_t clip_bytes = sizeof(esim::ClipDev) * nclips;
    auto align = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    size_t off = 0;
    const size_t o_clips = off;
    off = align(off + clip_bytes);
    const size_t o_bcount = off;
    off = align(off + sizeof(int64_t) * blk);
    const size_t o_chunk = off;
    off = align(off + sizeof(int64_t) * ((blk + esim::kChunkBlocks - 1) / esim::kChunkBlocks));
    const size_t o_xcd = off;
    off = align(off + sizeof(int64_t) * 5 * (esim::kMaxXcds + 1));
    const size_t o_flags = off;
    off = align(off + sizeof(uint64_t) * blk * esim::kWavesPerBlock);
    const size_t o_pol = off;
    off = align(off + sizeof(uint64_t) * blk * esim::kWavesPerBlock);
    const size_t o_misc = off;
    off = align(off + sizeof(int64_t) * 4);
    hipError_t e = hipMalloc(&pl->ws_mem, off);
    if (e != hipSuccess) {
      delete pl;
      return hip_check(e, "hipMalloc(plan)");
    }
    char* m = static_cast<char*>(pl->ws_mem);
    pl->dev = reinterpret_cast<esim::ClipDev*>(m + o_clips);
    pl->ws.bcount = reinterpret_cast<int64_t*>(m + o_bcount);
    pl->ws.chunk = reinterpret_cast<int64_t*>(m + o_chunk);
    pl->xcd_bounds = reinterpret_cast<int64_t*>(m + o_xcd);
    pl->ws.flags = reinterpret_cast<uint64_t*>(m + o_flags);
    pl->ws.pol = reinterpret_cast<uint64_t*>(m + o_pol);
    pl->ws.misc = reinterpret_cast<int64_t*>(m + o_misc);
    // Dense launches of a multi-clip plan split the groups between the XCDs
    // by work (window size x groups per clip) rather than by count, since a
    // clip's items cost in proportion to its window.
    const int nx = pl->shape.xcds;
    std::vector<int64_t> xb(5 * (esim::kMaxXcds + 1), 0);
    for (int q = 0; q < 5; ++q) {
      int64_t* row = xb.data() + q * (esim::kMaxXcds + 1);
      double total = 0.0;
      std::vector<double> wc(nclips);
      std::vector<int64_t> gc(nclips);
      for (int c = 0; c < nclips; ++c) {
        const auto& cd = pl->host[c];
        gc[c] = (c + 1 < nclips ? pl->host[c + 1].grp_off[q] : grp[q]) - cd.grp_off[q];
        wc[c] = static_cast<double>(2 * cd.r + 1) * (2 * cd.r + 1) * (2 * cd.tr + 1);
        total += wc[c] * static_cast<double>(gc[c]);
      }
      row[0] = 0;
      row[nx] = grp[q];
      for (int x = 1; x < nx; ++x) {
        const double target = total * x / nx;
        double cum = 0.0;
        int64_t idx = grp[q];
        for (int c = 0; c < nclips; ++c) {
          const double cw = wc[c] * static_cast<double>(gc[c]);
          if (cum + cw >= target) {
            idx = pl->host[c].grp_off[q] +
                  std::min<int64_t>(gc[c], static_cast<int64_t>(std::ceil((target - cum) / wc[c])));
            break;
          }
          cum += cw;
        }
        row[x] = std::max(row[x - 1], idx);
      }
    }
    e = hipMemcpy(pl->dev, pl->host.data(), clip_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m + o_bcount, 0, off - o_bcount);
    if (e == hipSuccess)
      e = hipMemcpy(pl->xcd_bounds, xb.data(), sizeof(int64_t) * xb.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      (void)hipFree(pl->ws_mem);   // the upload's error is the one reported
      delete pl;
      return hip_check(e, "plan upload");
    }
    // esim_step buffers: work list, count, dense alpha
    {
      size_t so = 0;
      const size_t s_wl = so;
      so = align(so + sizeof(int64_t) * std::max<int64_t>(wl, 1));
      const size_t s_cnt = so;
      so = align(so + sizeof(int32_t) * 4);
      const size_t s_al = so;
      so = align(so + sizeof(float) * pix);
      const size_t s_be = so;
      if (pl->thr != ESIM_THRESHOLD_CLOSED) so = align(so + sizeof(float) * (pl->F + 2) * pix);
      e = hipMalloc(&pl->step_mem, so);
      if (e != hipSuccess) {
        (void)hipFree(pl->ws_mem);   // the allocation's error is the one reported
        delete pl;
        return hip_check(e, "hipMalloc(step buffers)");
      }
      char* sm = static_cast<char*>(pl->step_mem);
      pl->step_wl = reinterpret_cast<int64_t*>(sm + s_wl);
      pl->step_count = reinterpret_cast<int32_t*>(sm + s_cnt);
      pl->step_alpha = reinterpret_cast<float*>(sm + s_al);
      if (pl->thr != ESIM_THRESHOLD_CLOSED) pl->step_beta = reinterpret_cast<float*>(sm + s_be);
    }
    *out = pl;
    return ok();
  } catch (const std::exception& ex) {
    return fail(ESIM_E_HIP, ex.what());
  } catch (...) {
    return fail(ESIM_E_HIP, "unknown exception");
  }
}

int esim_plan_destroy(esim_plan pl) {
  if (!pl) return ok();
  hipError_t e = hipSuccess;
  if (pl->ws_mem) e = hipFree(pl->ws_mem);
  if (pl->step_mem) {
    const hipError_t e2 = hipFree(pl->step_mem);
    if (e == hipSuccess) e = e2;
  }
  delete pl;   // the plan is gone either way; a failed free is reported
  return hip_check(e, "hipFree(plan buffers)");
}

int64_t esim_plan_pixels(esim_plan pl) { return pl ? pl->npix : -1; }
int64_t esim_plan_worklist_capacity(esim_plan pl) { return pl ? pl->wl_capacity : -1; }
int64_t esim_plan_pixel_offset(esim_plan pl, int32_t c) {
  if (!pl || c < 0 || c >= pl->nclips) return -1;
  return pl->host[c].pix_off;
}

int esim_log_brightness(const float* E, float* y, int64_t n, float eps, void* stream) {
  try {
    if (n < 0 || !(eps >= 0)) return fail(ESIM_E_INVAL, "n < 0 or eps < 0");
    if (n == 0) return ok();
    if (!E || !y) return fail(ESIM_E_INVAL, "null pointer");
    return hip_check(esim::launch_log(E, y, n, eps, static_cast<hipStream_t>(stream)), "log_brightness");
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_wlr_threshold(esim_plan pl, int32_t t, float* dl, int64_t* worklist, int32_t* count,
                       void* stream) {
  try {
    if (!pl || !dl || !worklist || !count) return fail(ESIM_E_INVAL, "null argument");
    if (t < 0) return fail(ESIM_E_INVAL, "t < 0");
    for (const auto& c : pl->host)
      if (!c.st_beta || !c.st_xref || !c.st_alpha || !c.st_tref)
        return fail(ESIM_E_INVAL, "threshold needs the full state (alpha, beta, xref, tref)");
    return threshold_compact(pl, t, dl, worklist, count, nullptr, static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_wlr_regress(esim_plan pl, int32_t t, const int64_t* worklist, const int32_t* count,
                     int64_t n_out, float* alpha, float* beta, float* resid, float* kappa,
                     void* stream) {
  try {
    if (!pl || !alpha) return fail(ESIM_E_INVAL, "null argument");
    if (worklist && !count) return fail(ESIM_E_INVAL, "worklist without count");
    if (!worklist && t < 0) return fail(ESIM_E_INVAL, "dense regression needs t >= 0");
    if (!worklist && n_out < pl->npix) return fail(ESIM_E_INVAL, "n_out < plan pixels");
    if (n_out < 0) return fail(ESIM_E_INVAL, "n_out < 0");
    if (t < 0 && (pl->max_feat_bytes >= (1ull << 32) || pl->max_y_bytes >= (1ull << 32)))
      return fail(ESIM_E_UNSUPPORTED, "per-item frames need feature and brightness arrays below 4 GiB");
    return launch_plan_regress(pl, t, worklist, count, n_out, alpha, beta, resid, kappa, false,
                               static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_events(esim_plan pl, int32_t t, int32_t mode, const int64_t* worklist, const int32_t* count,
                float* dl, const float* alpha, const float* beta, int64_t n_out, esim_events_buf* ev,
                void* stream) {
  try {
    if (!pl) return fail(ESIM_E_INVAL, "null plan");
    if (t < 0) return fail(ESIM_E_INVAL, "t < 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (const auto& c : pl->host)
      if (!c.st_alpha) return fail(ESIM_E_INVAL, "state alpha is null");
    if (mode == ESIM_INIT) {
      if (alpha && n_out < pl->npix) return fail(ESIM_E_INVAL, "n_out < plan pixels");
      const bool model = alpha && beta && pl->thr != ESIM_THRESHOLD_CLOSED;
      if (model) {
        int rc = explicit_ok(pl);
        if (rc != ESIM_OK) return rc;
      }
      int rc = hip_check(esim::launch_init(pl->dev, pl->nclips, pl->nblk, t, alpha, beta, n_out, s), "init");
      if (rc != ESIM_OK || !model) return rc;
      return store_moments(pl, t, nullptr, nullptr, s);
    }
    if (!ev || !ev->x || !ev->y || !ev->t || !ev->p || !ev->count || ev->capacity < 0)
      return fail(ESIM_E_INVAL, "events buffer incomplete");
    esim::EventsDev ed{ev->x, ev->y, ev->t, ev->p, ev->clip, ev->capacity, ev->count, ev->ts};
    if (mode == ESIM_THRESHOLDED) {
      if (!worklist || !count || !dl || !alpha || !beta)
        return fail(ESIM_E_INVAL, "thresholded events need worklist, count, dl, alpha and beta");
      // every item of the work list needs its model: the outputs must cover the
      // largest work list a threshold call can produce
      if (n_out < pl->wl_capacity)
        return fail(ESIM_E_INVAL, "n_out < work-list capacity (esim_plan_worklist_capacity)");
      for (const auto& c : pl->host)
        if (!c.st_beta || !c.st_xref || !c.st_tref) return fail(ESIM_E_INVAL, "state incomplete");
      int rc = explicit_ok(pl);
      if (rc != ESIM_OK) return rc;
      rc = hip_check(esim::launch_list_events(pl->dev, pl->nclips, t, worklist, count, pl->wl_capacity, dl,
                                              alpha, beta, n_out, pl->ws, ed, s),
                     "events(thresholded)");
      if (rc != ESIM_OK) return rc;
      return store_moments(pl, t, worklist, count, s);
    }
    if (mode == ESIM_EXHAUSTIVE || mode == ESIM_RAW) {
      if (!multi_state_ok(pl)) return fail(ESIM_E_INVAL, "multi_crossing needs the state's last");
      if (mode == ESIM_EXHAUSTIVE && (!alpha || n_out < pl->npix))
        return fail(ESIM_E_INVAL, "exhaustive events need dense alpha (n_out >= plan pixels)");
      return hip_check(esim::launch_flag_compact(pl->dev, pl->nclips, pl->nblk, t,
                                                 mode == ESIM_EXHAUSTIVE ? esim::kFlagExhaustive
                                                                         : esim::kFlagRaw,
                                                 dl, alpha, pl->ws, nullptr, nullptr, &ed, s),
                       "events");
    }
    return fail(ESIM_E_INVAL, "bad mode");
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_step(esim_plan pl, int32_t t, int32_t mode, float* dl, esim_events_buf* ev, void* stream) {
  try {
    if (!pl) return fail(ESIM_E_INVAL, "null plan");
    if (t < 0) return fail(ESIM_E_INVAL, "t < 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (mode == ESIM_INIT || mode == ESIM_THRESHOLDED) {
      if (!full_state(pl)) return fail(ESIM_E_INVAL, "the step needs the full state (alpha, beta, xref, tref)");
    } else {
      for (const auto& c : pl->host)
        if (!c.st_alpha) return fail(ESIM_E_INVAL, "state alpha is null");
    }
    if (mode == ESIM_INIT) {
      if (pl->thr == ESIM_THRESHOLD_CLOSED)
        return launch_plan_regress(pl, t, nullptr, nullptr, pl->npix, nullptr, nullptr, nullptr, nullptr,
                                   true, s);
      // explicit thresholds keep the whole plane: through the plan's buffers
      int rc = launch_plan_regress(pl, t, nullptr, nullptr, pl->npix, pl->step_alpha, pl->step_beta, nullptr,
                                   nullptr, false, s);
      if (rc != ESIM_OK) return rc;
      rc = hip_check(esim::launch_init(pl->dev, pl->nclips, pl->nblk, t, pl->step_alpha, pl->step_beta,
                                       pl->npix, s),
                     "step(init)");
      if (rc != ESIM_OK) return rc;
      return store_moments(pl, t, nullptr, nullptr, s);
    }
    if (!ev || !ev->x || !ev->y || !ev->t || !ev->p || !ev->count || ev->capacity < 0)
      return fail(ESIM_E_INVAL, "events buffer incomplete");
    esim::EventsDev ed{ev->x, ev->y, ev->t, ev->p, ev->clip, ev->capacity, ev->count, ev->ts};
    if (mode == ESIM_THRESHOLDED) {
      // Mixed window widths: the compaction writes the narrow clips' items and
      // the wide ones' into two segments, and each gets its own launch, so the
      // narrow ones run the one-pass list instance (one column per lane)
      // instead of the general one, each launch spread over every XCD.
      const bool split = pl->split_seg >= 0 && pl->thr == ESIM_THRESHOLD_CLOSED && pl->lanes_list == 16 &&
                         pl->host[0].precision == ESIM_GRAM_F64;
      int rc = threshold_compact(pl, t, dl, pl->step_wl, pl->step_count, &ed, s, split ? pl->split_seg : -1);
      if (rc != ESIM_OK) return rc;
      if (split) {
        rc = launch_plan_regress(pl, t, pl->step_wl, pl->step_count, pl->split_seg, nullptr, nullptr, nullptr,
                                 nullptr, true, s, pl->split_r[0]);
        if (rc != ESIM_OK) return rc;
        return launch_plan_regress(pl, t, pl->step_wl + pl->split_seg, pl->step_count + 2,
                                   pl->wl_capacity - pl->split_seg, nullptr, nullptr, nullptr, nullptr, true, s,
                                   pl->split_r[1]);
      }
      if (pl->thr == ESIM_THRESHOLD_CLOSED)
        return launch_plan_regress(pl, t, pl->step_wl, pl->step_count, pl->wl_capacity, nullptr, nullptr,
                                   nullptr, nullptr, true, s);
      rc = launch_plan_regress(pl, t, pl->step_wl, pl->step_count, pl->wl_capacity, pl->step_alpha,
                               pl->step_beta, nullptr, nullptr, false, s);
      if (rc != ESIM_OK) return rc;
      rc = hip_check(esim::launch_list_state(pl->dev, pl->nclips, t, pl->step_wl, pl->step_count,
                                             pl->wl_capacity, pl->step_alpha, pl->step_beta, pl->wl_capacity,
                                             s),
                     "step(state)");
      if (rc != ESIM_OK) return rc;
      return store_moments(pl, t, pl->step_wl, pl->step_count, s);
    }
    if ((mode == ESIM_EXHAUSTIVE || mode == ESIM_RAW) && !multi_state_ok(pl))
      return fail(ESIM_E_INVAL, "multi_crossing needs the state's last");
    if (mode == ESIM_EXHAUSTIVE) {
      int rc = launch_plan_regress(pl, t, nullptr, nullptr, pl->npix, pl->step_alpha, nullptr, nullptr,
                                   nullptr, false, s);
      if (rc != ESIM_OK) return rc;
      return hip_check(esim::launch_flag_compact(pl->dev, pl->nclips, pl->nblk, t, esim::kFlagExhaustive, dl,
                                                 pl->step_alpha, pl->ws, nullptr, nullptr, &ed, s),
                       "step(exhaustive)");
    }
    if (mode == ESIM_RAW)
      return hip_check(esim::launch_flag_compact(pl->dev, pl->nclips, pl->nblk, t, esim::kFlagRaw, dl,
                                                 nullptr, pl->ws, nullptr, nullptr, &ed, s),
                       "step(raw)");
    return fail(ESIM_E_INVAL, "bad mode");
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_log_variance(const float* E, const float* var, int32_t spp, float* vy, int64_t n, float eps,
                      void* stream) {
  try {
    if (n < 0 || spp < 1 || !(eps >= 0)) return fail(ESIM_E_INVAL, "n < 0, spp < 1 or eps < 0");
    if (n == 0) return ok();
    if (!E || !var || !vy) return fail(ESIM_E_INVAL, "null pointer");
    return hip_check(esim::launch_log_variance(E, var, vy, n, spp, eps, static_cast<hipStream_t>(stream)),
                     "log_variance");
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_wlr_regress_bandwidth(esim_plan pl, int32_t t, const int64_t* worklist, const int32_t* count,
                               int64_t n_out, const float* vy, const double* hs, int32_t K, float* alpha,
                               float* beta, float* hsel, float* sure, void* stream) {
  try {
    if (!pl || !alpha || !vy || !hs) return fail(ESIM_E_INVAL, "null argument");
    if (pl->nclips != 1) return fail(ESIM_E_UNSUPPORTED, "bandwidth optimisation takes single-clip plans");
    const esim::ClipDev& hc = pl->host[0];
    if (t < 0 || t >= hc.T) return fail(ESIM_E_INVAL, "t outside the clip");
    if (K < 1 || K > esim::kMaxBandwidths) return fail(ESIM_E_INVAL, "K outside 1..8");
    if (worklist && !count) return fail(ESIM_E_INVAL, "worklist without count");
    if (!worklist && n_out < pl->npix) return fail(ESIM_E_INVAL, "n_out < plan pixels");
    if (n_out < 1) return fail(ESIM_E_INVAL, "n_out < 1");
    esim::BandwidthArgs a{};
    for (int k = 0; k < K; ++k) {
      if (!(hs[k] > 0) || std::isinf(hs[k])) return fail(ESIM_E_INVAL, "bandwidths must be positive and finite");
      a.h[k] = hs[k];
      a.scale[k] = hc.h / hs[k];
    }
    a.clip = pl->dev;
    a.t = t;
    a.items = worklist;
    a.count = count;
    a.n_out = n_out;
    a.vy = vy;
    a.K = K;
    a.alpha = alpha;
    a.beta = beta;
    a.hsel = hsel;
    a.sure = sure;
    return hip_check(esim::launch_bandwidth(a, pl->F, pl->f16, worklist ? std::min(n_out, pl->wl_capacity)
                                                                         : pl->npix,
                                            hc.r, static_cast<hipStream_t>(stream)),
                     "regress_bandwidth");
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

size_t esim_backward_scratch_bytes(esim_plan pl, int64_t n) {
  if (!pl || pl->nclips != 1 || n < 0) return 0;
  return esim::backward_scratch_bytes(pl->host[0], n);
}

int esim_wlr_backward(esim_plan pl, const int64_t* items, int64_t n, const float* g_alpha, float* g_y,
                      double* g_b, void* scratch, size_t scratch_bytes, void* stream) {
  try {
    if (!pl) return fail(ESIM_E_INVAL, "null plan");
    if (pl->nclips != 1) return fail(ESIM_E_UNSUPPORTED, "backward supports single-clip plans");
    if (n < 0) return fail(ESIM_E_INVAL, "n < 0");
    if (n == 0) return ok();
    if (!items || !g_alpha || !g_y || !g_b) return fail(ESIM_E_INVAL, "null argument");
    if (pl->max_feat_bytes >= (1ull << 32) || pl->max_y_bytes >= (1ull << 32))
      return fail(ESIM_E_UNSUPPORTED, "backward needs feature and brightness arrays below 4 GiB");
    if (pl->host[0].r > 25 || esim::backward_gather_lds_bytes(pl->host[0]) > esim::kMaxGatherLds)
      return fail(ESIM_E_UNSUPPORTED, "backward supports window radii up to 25");
    const size_t need = esim::backward_scratch_bytes(pl->host[0], n);
    if (!scratch || scratch_bytes < need) return fail(ESIM_E_CAPACITY, "scratch too small");
    esim::BackwardArgs a{pl->dev, &pl->host[0], items, n, g_alpha, g_y, g_b, scratch, scratch_bytes, pl->shape};
    return hip_check(esim::launch_backward(a, static_cast<hipStream_t>(stream)), "backward");
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

size_t esim_nn_scratch_bytes(int32_t W, int32_t H, int32_t T) {
  if (W < 1 || H < 1 || T < 1) return 0;
  return esim::nn_scratch_bytes(W, H, T);
}

}  // extern "C"

namespace {

// Validation and marshalling shared by the two event-set comparison entry
// points; scratch is the bitmap memory (caller's, or the library's fixed array).
int nn_call(const int32_t* src_x, const int32_t* src_y, const int32_t* src_t, const int8_t* src_p, int64_t ns,
            const int32_t* qry_x, const int32_t* qry_y, const int32_t* qry_t, const int8_t* qry_p, int64_t nq,
            int32_t W, int32_t H, int32_t T, double scale_x, double scale_y, double scale_t, double rmax, double* d,
            void* scratch, size_t scratch_bytes, bool fixed, void* stream) {
  if (W < 1 || H < 1 || T < 1 || ns < 0 || nq < 0) return fail(ESIM_E_INVAL, "bad shape or count");
  if (!(scale_x > 0) || !(scale_y > 0) || !(scale_t > 0) || !(rmax >= 0) || std::isinf(rmax))
    return fail(ESIM_E_INVAL, "scales must be positive and rmax finite and >= 0");
  if ((ns > 0 && (!src_x || !src_y || !src_t || !src_p)) || (nq > 0 && (!qry_x || !qry_y || !qry_t || !qry_p || !d)))
    return fail(ESIM_E_INVAL, "null event array");
  const size_t need = esim::nn_scratch_bytes(W, H, T);
  if (fixed) {
    if (need > ESIM_NN_STATIC_BYTES)
      return fail(ESIM_E_CAPACITY, "the bitmaps of this W x H x T exceed the fixed array (ESIM_NN_STATIC_BYTES)");
    if (!esim::nn_static_scratch(&scratch)) return fail(ESIM_E_HIP, "lookup of the fixed bitmap array failed");
  } else if (!scratch || scratch_bytes < need) {
    return fail(ESIM_E_CAPACITY, "scratch too small");
  }
  const double ex = std::floor(rmax / scale_x), ey = std::floor(rmax / scale_y), et = std::floor(rmax / scale_t);
  if (ex >= 4096) return fail(ESIM_E_UNSUPPORTED, "rmax spans 4096 columns or more");
  esim::NnArgs a{};
  a.sx = src_x;
  a.sy = src_y;
  a.st = src_t;
  a.sp = src_p;
  a.ns = ns;
  a.qx = qry_x;
  a.qy = qry_y;
  a.qt = qry_t;
  a.qp = qry_p;
  a.nq = nq;
  a.W = W;
  a.H = H;
  a.T = T;
  a.scale_x = scale_x;
  a.scale_y = scale_y;
  a.scale_t = scale_t;
  a.rmax = rmax;
  a.rx = static_cast<int>(std::min<double>(ex, W));
  a.ry = static_cast<int>(std::min<double>(ey, H));
  a.rt = static_cast<int>(std::min<double>(et, T));
  a.d = d;
  a.scratch = scratch;
  return hip_check(esim::launch_nn(a, static_cast<hipStream_t>(stream)), "nn_distances");
}

}  // namespace

extern "C" {

int esim_nn_distances(const int32_t* src_x, const int32_t* src_y, const int32_t* src_t, const int8_t* src_p,
                      int64_t ns, const int32_t* qry_x, const int32_t* qry_y, const int32_t* qry_t,
                      const int8_t* qry_p, int64_t nq, int32_t W, int32_t H, int32_t T, double scale_x,
                      double scale_y, double scale_t, double rmax, double* d, void* scratch,
                      size_t scratch_bytes, void* stream) {
  try {
    return nn_call(src_x, src_y, src_t, src_p, ns, qry_x, qry_y, qry_t, qry_p, nq, W, H, T, scale_x, scale_y,
                   scale_t, rmax, d, scratch, scratch_bytes, false, stream);
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

int esim_nn_distances_noalloc(const int32_t* src_x, const int32_t* src_y, const int32_t* src_t,
                              const int8_t* src_p, int64_t ns, const int32_t* qry_x, const int32_t* qry_y,
                              const int32_t* qry_t, const int8_t* qry_p, int64_t nq, int32_t W, int32_t H,
                              int32_t T, double scale_x, double scale_y, double scale_t, double rmax, double* d,
                              void* stream) {
  try {
    return nn_call(src_x, src_y, src_t, src_p, ns, qry_x, qry_y, qry_t, qry_p, nq, W, H, T, scale_x, scale_y,
                   scale_t, rmax, d, nullptr, 0, true, stream);
  } catch (...) {
    return fail(ESIM_E_HIP, "exception");
  }
}

// Schedule override used by the autotuner: lanes per item for dense and for
// work-list launches (1, 2, 4, 8, 16) and persistent blocks per CU.  Not part of
// the hot path.
int esim_plan_set_schedule(esim_plan pl, int32_t lanes_dense, int32_t lanes_list,
                           int32_t blocks_per_cu) {
  if (!pl) return fail(ESIM_E_INVAL, "null plan");
  for (int L : {lanes_dense, lanes_list})
    if (L < 1 || (L & (L - 1)) || !esim::regress_supports(pl->F, L, pl->host[0].precision))
      return fail(ESIM_E_UNSUPPORTED, "lanes per item not compiled for this F and precision");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(ESIM_E_INVAL, "blocks_per_cu outside 1..64");
  pl->lanes_dense = lanes_dense;
  pl->lanes_list = lanes_list;
  pl->blocks_per_cu = blocks_per_cu;
  return ok();
}

}  // extern "C"
