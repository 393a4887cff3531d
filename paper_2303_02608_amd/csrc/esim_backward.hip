// Adjoint of the regression estimate alpha (Sec. 2.1, eqs. 4-5 differentiated).
//
// With A the W-normalised Gram plus ridge Lambda (in bandwidth-scaled units),
// theta = A^{-1} g, v = A^{-1} e_0, s_i = v^T z_i and r_i = y_i - z_i^T theta:
//     d alpha / d y_i = (w_i / W) s_i
//     d alpha / d w_i = (s_i r_i - v^T Lambda theta) / W
//     d w_i / d b_j   = w_i u_ij^2 / (h^2 b_j^3) = w_i v_ij^2 / b_j
// (alpha does not depend on the scaling of the regressors, so the scaled system
// gives the same derivatives).
//
// Kernels, all deterministic (no atomics on values):
//   fill_map / map_items  a dense (frame, pixel) -> item index map
//   adjoint_kernel        per item: the window's Gram, Cholesky, theta and v
//                         (the window is recomputed, not stored by the forward
//                         pass); writes the item's record c = g_alpha v / W,
//                         theta, q = g_alpha v^T Lambda theta / W
//   gather_kernel         per input sample (frame, pixel): for every item whose
//                         window holds it, in a fixed order, recomputes the
//                         sample's weight and regressors from the item's
//                         centre features and record, adds w_i c^T z_i to g_y
//                         and accumulates w_i (c^T z_i r_i - q) z_ij^2 for the
//                         bandwidths.  A wave owns 8 x 8 samples and walks the
//                         items staged in LDS one at a time, every lane reading
//                         the same record (a broadcast); per-block partials
//   reduce_gb_*           fixed-order two-level sum of the per-block partials
#include "esim_wlr.h"

namespace esim {
namespace {

constexpr int kAdjLanes = 4;        // lanes per item, windows wider than 16 columns
constexpr int kAdjLanesWide = 16;   // lanes per item, windows of at most 16 columns
constexpr int kRedBlocks = 256;
constexpr int kAdjRing = 3;      // rows of window loads in flight in the interior loop
constexpr int kGatherTile = 16;     // input pixels of a gather block: 16 x 16, four waves of 8 x 8
constexpr int kGatherThreads = 256;
constexpr int kGatherWaves = kGatherThreads / kWave;
constexpr size_t kGatherLdsBudget = 40960;    // four blocks per CU
constexpr int kGatherSlots = 4;              // region slots per thread and step of the gather's scan
constexpr size_t kGatherCountBytes = sizeof(int32_t) * 2 * kGatherSlots * kGatherWaves;

struct BwdDev {
  int32_t* item_map;   // [T*HW]
  double* rec;         // [n][2P + 1] per-item records (c, theta, q)
  double* gbpart;      // [npart][D] per-gather-block bandwidth partials
  double* gbblk;       // [kRedBlocks][D]
  int64_t n;
  int64_t npart;
};

__global__ void __launch_bounds__(256) fill_map_kernel(int32_t* m, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) m[i] = -1;
}

__device__ __forceinline__ bool item_ok(const ClipDev& C, int64_t it, const float* g_alpha, int64_t i,
                                        int64_t& pix, int& t) {
  if (it < 0 || item_clip(it) != 0) return false;
  pix = item_pixel(it);
  t = item_frame(it);
  return pix < C.HW && t >= 0 && t < C.T && g_alpha[i] != 0.0f;
}

__global__ void __launch_bounds__(256)
map_items_kernel(const ClipDev* __restrict__ clips, const int64_t* __restrict__ items, int64_t n,
                 const float* __restrict__ g_alpha, int32_t* item_map) {
  const ClipDev& C = clips[0];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t pix;
    int t;
    if (item_ok(C, items[i], g_alpha, i, pix, t)) item_map[static_cast<int64_t>(t) * C.HW + pix] = static_cast<int32_t>(i);
  }
}

template <int F, int L, bool F16, bool ONE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(F <= 8 ? 2 : 1)))
adjoint_kernel(const ClipDev* __restrict__ clips, const int64_t* __restrict__ items,
               const float* __restrict__ g_alpha, BwdDev bd, int nxcd) {
  constexpr int P = F + 3;
  constexpr int R = 2 * P + 1;
  constexpr int G = kWave / L;
  const ClipDev& C = clips[0];
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / L;
  const int j = lane % L;
  const int64_t ngroups = (bd.n + G - 1) / G;
  GroupIter it_groups(ngroups, nxcd);
  int64_t g;
  while (it_groups.next(g)) {
    const int64_t i = g * G + slot;
    int64_t pix = 0;
    int t = 0;
    const bool active = i < bd.n && item_ok(C, items[i], g_alpha, i, pix, t);
    const uint64_t act = __ballot(active);
    if (act == 0) continue;
    // Interior waves (every item's window inside the image and the clip) of
    // the one-column-per-lane instance run the window loop without per-row
    // validity tests; lanes without an item then take the first item's
    // geometry with weight 0.
    const int prow = static_cast<int>(pix / C.W), pcol = static_cast<int>(pix - static_cast<int64_t>(prow) * C.W);
    const bool inside = prow >= C.r && prow + C.r < C.H && pcol >= C.r && pcol + C.r < C.W &&
                        t - C.tr >= 0 && t + C.tr < C.T;
    const bool full = ONE && __ballot(active && !inside) == 0;
    int64_t gpix = active ? pix : 0;
    int gt = active ? t : 0;
    if (full) {
      const int src = __ffsll(static_cast<unsigned long long>(act)) - 1;
      const int64_t p0 = __shfl(pix, src);
      const int t0 = __shfl(t, src);
      if (!active) {
        gpix = p0;
        gt = t0;
      }
    }
    ItemGeom<F, F16, double> geo;
    make_geom(geo, C, gpix, gt, 0, C.T, active);

    Gram<F, double> gm;
    auto add = [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
      gm.add_onepass(w, yd, v, vy);
    };
    if constexpr (ONE) {
      // every lane owns one column of the window (2r + 1 <= L, checked by the launcher)
      gm.zero_onepass();
      if (full)
        window_loop_ring<F, L, F16, kAdjRing>(geo, j, [&](double) {}, add,
                                              [&](double vx) { gm.fold_onepass(vx); });
      else
        window_loop<F, L, F16, double>(geo, j, [&](double) {}, add, [&](double vx) { gm.fold_onepass(vx); });
    } else {
      gm.zero_snap();
      window_loop<F, L, F16, double>(geo, j, [&](double) { gm.pass_begin_snap(); }, add,
                                     [&](double vx) { gm.pass_end_snap(vx); });
    }
    gm.template lane_sum<L>();
    double M[P * (P + 1) / 2], rhs[P], th[P], anorm;
    const double iW = gram_solve<F, double>(gm, C, M, rhs, th, anorm);
    double e0[P], vv[P];
#pragma unroll
    for (int k = 0; k < P; ++k) e0[k] = k == 0 ? 1.0 : 0.0;
    chol_solve<P, double>(M, e0, vv);
    double vLt = 0.0;      // v^T Lambda theta (Lambda = scaled ridge on the beta block)
#pragma unroll
    for (int k = 1; k < P; ++k) vLt = fma(vv[k] * (C.ridge * C.c2[k - 1]), th[k], vLt);
    if (active && j == 0) {
      const double gw = static_cast<double>(g_alpha[i]) * iW;
      double* o = bd.rec + i * R;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        o[k] = gw * vv[k];
        o[P + k] = th[k];
      }
      o[2 * P] = gw * vLt;
    }
  }
}

// LDS bytes of one staged item of the gather: its record, its centre features
// (scaled) and its packed position in the block's item region.
size_t gather_item_bytes(int F) {
  const int P = F + 3;
  return sizeof(double) * (2 * P + 1) + sizeof(double) * F + sizeof(int32_t);
}

// Items staged at a time (the LDS budget, less the per-wave counts).
int gather_capacity(int F) {
  return static_cast<int>((kGatherLdsBudget - kGatherCountBytes) / gather_item_bytes(F));
}

// One block per (input frame tq, 16 x 16 tile of input pixels); wave w owns the
// 8 x 8 sub-tile (w & 1, w >> 1), lane l the sample (l & 7, l >> 3) in it.
// The block's item region is the (frame, row, column) slots whose window can
// reach the tile: rows yc, frames tc and columns x within r (tr) of it, taken
// in a fixed order (tc ascending, then yc, then x), 1024 slots per step, four
// per thread.  A step's present items (the frame-pixel map holds their index) are
// compacted in that order into an LDS buffer of cap items (records, centre
// features, positions): a wave ballot and prefix per set of 256 slots, and the
// waves' counts exchanged through LDS.  When the next item would not fit, every wave walks
// the buffer in order, skipping the items out of reach of all of its lanes
// (64 positions tested per ballot), and each lane whose window holds the item
// adds its sample's terms.  The order of every sum is fixed, so g_y and the
// partials do not depend on scheduling.
template <int F>
__global__ void __launch_bounds__(kGatherThreads) __attribute__((amdgpu_waves_per_eu(F <= 8 ? 4 : 1)))
gather_kernel(const ClipDev* __restrict__ clips, BwdDev bd, float* __restrict__ g_y, int cap) {
  constexpr int D = F + 2;
  constexpr int P = F + 3;
  constexpr int R = 2 * P + 1;
  constexpr double K = kHalfLog2e;
  extern __shared__ double sm[];
  const ClipDev& C = clips[0];
  const int r = C.r, tr = C.tr, W = C.W, H = C.H, T = C.T;
  const int ncol = kGatherTile + 2 * r;                        // at most 66 (r <= 25)
  double* srec = sm;                                            // [cap][R]
  double* sxcs = srec + static_cast<size_t>(cap) * R;           // [cap][F]
  int32_t* spos = reinterpret_cast<int32_t*>(sxcs + static_cast<size_t>(cap) * F);  // [cap] (row << 8) | column
  int32_t* wcnt = spos + cap;                                   // [2][slots][waves] present items per wave and step
  const int ntx = (W + kGatherTile - 1) / kGatherTile;
  const int nty = (H + kGatherTile - 1) / kGatherTile;
  int64_t b = blockIdx.x;
  const int tx = static_cast<int>(b % ntx);
  b /= ntx;
  const int ty = static_cast<int>(b % nty);
  const int tq = static_cast<int>(b / nty);
  const int bx0 = tx * kGatherTile, by0 = ty * kGatherTile;
  const int lane = static_cast<int>(threadIdx.x) & (kWave - 1);
  const int wv = static_cast<int>(threadIdx.x) / kWave;
  const int wx0 = bx0 + 8 * (wv & 1), wy0 = by0 + 8 * (wv >> 1);
  const int xq = wx0 + (lane & 7), yq = wy0 + (lane >> 3);
  const bool in = xq < W && yq < H;
  const int xs = bx0 - r;                      // image column of region column 0
  // region columns whose items reach the wave's columns: wc0 .. wc0 + 7 + 2r
  const int wc0 = wx0 - r - xs;
  const int64_t pq = in ? static_cast<int64_t>(yq) * W + xq : 0;
  double fi[F];
#pragma unroll
  for (int f = 0; f < F; ++f) fi[f] = in ? static_cast<double>(feat_value(C, tq, f, pq)) : 0.0;
  const double yi = in ? static_cast<double>(C.y[static_cast<int64_t>(tq) * C.HW + pq]) : 0.0;
  double sf[F];
#pragma unroll
  for (int f = 0; f < F; ++f) sf[f] = C.sf[2 + f];
  const double vx_step = C.sf[0] / r, vy_step = C.sf[1] / r;
  double acc = 0.0;
  double gb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) gb[d] = 0.0;
  const int t0 = max(0, tq - tr), t1 = min(T - 1, tq + tr);
  const int ntc = t1 - t0 + 1;
  const int yc0 = max(0, by0 - r), yc1 = min(H - 1, by0 + kGatherTile - 1 + r);
  const int nry = yc1 - yc0 + 1;
  // slot s: row k = s / ncol = (tc - t0) nry + yc - yc0, column s % ncol (frame
  // by frame, so that every buffer holds items of all the tile's rows and all
  // four waves have work in every walk)
  const int nslot = nry * ntc * ncol;
  auto map_entry = [&](int s) -> int32_t {
    if (s >= nslot) return -1;
    const int k = s / ncol, c = s - k * ncol, x = xs + c;
    if (x < 0 || x >= W) return -1;
    const int yc = yc0 + k % nry, tc = t0 + k / nry;
    return bd.item_map[static_cast<int64_t>(tc) * C.HW + static_cast<int64_t>(yc) * W + x];
  };

  // Walks buffer entries 0 .. n - 1 in order.
  auto walk = [&](int n) {
    for (int i0 = 0; i0 < n; i0 += kWave) {
      const int ii = i0 + lane;
      const int pp = ii < n ? spos[ii] : 0;
      const int prow = pp >> 8, pcol = pp & 255;
      const int yc = yc0 + prow;
      // items out of reach of every lane of the wave are skipped (ballot)
      uint64_t m = __ballot(ii < n && yc >= wy0 - r && yc <= wy0 + 7 + r && pcol >= wc0 && pcol <= wc0 + 7 + 2 * r);
      while (m != 0) {
        const int bi = __ffsll(static_cast<unsigned long long>(m)) - 1;
        m &= m - 1;
        const int pu = __builtin_amdgcn_readlane(pp, bi);
        const int dy = yq - (yc0 + (pu >> 8));
        const int dx = xq - (xs + (pu & 255));
        if (!in || dy < -r || dy > r || dx < -r || dx > r) continue;
        const int q = i0 + bi;
        const double* rc = srec + static_cast<size_t>(q) * R;
        const double* xc = sxcs + static_cast<size_t>(q) * F;
        // the sample's regressors and weight as the item's window pass forms them
        const double vy = static_cast<double>(dy) * vy_step;
        const double kyy = K * vy;
        const double vx = static_cast<double>(dx) * vx_step;
        double v[F];
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int f = 0; f < F; ++f) {
          v[f] = fma(fi[f], sf[f], -xc[f]);
          if (f & 1) s1 = fma(v[f], v[f], s1);
          else s0 = fma(v[f], v[f], s0);
        }
        const double arg = fma(s0 + s1, K, fma(kyy, vy, K * vx * vx));
        const double w = static_cast<double>(__builtin_amdgcn_exp2f(static_cast<float>(arg)));
        double cs = fma(rc[1], vx, fma(rc[2], vy, rc[0]));
        double pred = fma(rc[P + 1], vx, fma(rc[P + 2], vy, rc[P]));
#pragma unroll
        for (int f = 0; f < F; ++f) {
          cs = fma(rc[3 + f], v[f], cs);
          pred = fma(rc[P + 3 + f], v[f], pred);
        }
        acc = fma(w, cs, acc);
        const double kq = w * fma(cs, yi - pred, -rc[2 * P]);
        gb[0] = fma(kq, vx * vx, gb[0]);
        gb[1] = fma(kq, vy * vy, gb[1]);
#pragma unroll
        for (int f = 0; f < F; ++f) gb[2 + f] = fma(kq, v[f] * v[f], gb[2 + f]);
      }
    }
  };

  // Steps of 256 slots fill the buffer; a walk empties it when a step's items
  // overflow it (the step is then resumed) and once after the last step.  One
  // walk site, so that the walk is compiled once.
  const int tid = static_cast<int>(threadIdx.x);
  int seq = 0;                                 // items of the region found so far (block-uniform)
  int base = 0;                                // sequence number of buffer entry 0
  int par = 0;
  int s = tid;                                 // this thread's first slot of the current step
  int32_t it[kGatherSlots];
  int mine[kGatherSlots];
  bool resume = false;
  int32_t next_it[kGatherSlots];
#pragma unroll
  for (int u = 0; u < kGatherSlots; ++u) {
    it[u] = -1;
    mine[u] = 0;
    next_it[u] = map_entry(s + u * kGatherThreads);
  }
  for (;;) {
    int nwalk = 0;                             // block-uniform
    const bool last = !resume && s - tid >= nslot;
    if (last) {
      nwalk = seq - base;
    } else {
      if (!resume) {
        int below[kGatherSlots];
#pragma unroll
        for (int u = 0; u < kGatherSlots; ++u) {
          it[u] = next_it[u];
          // in flight while this step is compacted and staged
          next_it[u] = map_entry(s + (kGatherSlots + u) * kGatherThreads);
          const uint64_t bal = __ballot(it[u] >= 0);
          below[u] = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(bal >> 32),
                                               __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0));
          if (lane == 0) wcnt[(par * kGatherSlots + u) * kGatherWaves + wv] = __popcll(bal);
        }
        __syncthreads();                       // counts visible
#pragma unroll
        for (int u = 0; u < kGatherSlots; ++u) {
          int total = 0, off = 0;
#pragma unroll
          for (int w2 = 0; w2 < kGatherWaves; ++w2) {
            const int c = wcnt[(par * kGatherSlots + u) * kGatherWaves + w2];
            total += c;
            off += w2 < wv ? c : 0;
          }
          mine[u] = seq + off + below[u];
          seq += total;
        }
        par ^= 1;
      }
#pragma unroll
      for (int u = 0; u < kGatherSlots; ++u) {
        if (it[u] >= 0 && mine[u] >= base && mine[u] < base + cap) {
          const int e = mine[u] - base;
          const int su = s + u * kGatherThreads;
          const int k = su / ncol, c = su - k * ncol;
          const int yc = yc0 + k % nry, tc = t0 + k / nry;
          const double* src = bd.rec + static_cast<int64_t>(it[u]) * R;
#pragma unroll
          for (int j = 0; j < R; ++j) srec[static_cast<size_t>(e) * R + j] = src[j];
          const int64_t p = static_cast<int64_t>(yc) * W + xs + c;
#pragma unroll
          for (int f = 0; f < F; ++f)
            sxcs[static_cast<size_t>(e) * F + f] = static_cast<double>(feat_value(C, tc, f, p)) * sf[f];
          spos[e] = ((yc - yc0) << 8) | c;
        }
      }
      resume = seq > base + cap;
      if (resume) nwalk = cap;
      else s += kGatherSlots * kGatherThreads;
    }
    if (nwalk > 0) {
      __syncthreads();                         // the buffer is staged
      walk(nwalk);
      __syncthreads();                         // its reads are done
      base += nwalk;
    }
    if (last) break;
  }
  if (in && acc != 0.0) g_y[static_cast<int64_t>(tq) * C.HW + pq] += static_cast<float>(acc);
  // bandwidth partials of the block: a fixed butterfly inside each wave, then
  // the waves in order
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) gb[d] += __shfl_xor(gb[d], o);
  __syncthreads();                             // the last walk's reads are done
  if (lane == 0)
#pragma unroll
    for (int d = 0; d < D; ++d) sm[wv * D + d] = gb[d];
  __syncthreads();
  if (threadIdx.x < D) {
    double s = 0.0;
    for (int w2 = 0; w2 < kGatherWaves; ++w2) s += sm[w2 * D + threadIdx.x];
    bd.gbpart[static_cast<int64_t>(blockIdx.x) * D + threadIdx.x] = s * C.sf[threadIdx.x] * C.h;
  }
}

template <int D>
__global__ void __launch_bounds__(256) reduce_gb_blocks(BwdDev bd) {
  __shared__ double sh[256][D];
  double acc[D];
#pragma unroll
  for (int d = 0; d < D; ++d) acc[d] = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < bd.npart;
       i += static_cast<int64_t>(gridDim.x) * 256)
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] += bd.gbpart[i * D + d];
#pragma unroll
  for (int d = 0; d < D; ++d) sh[threadIdx.x][d] = acc[d];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (static_cast<int>(threadIdx.x) < o)
#pragma unroll
      for (int d = 0; d < D; ++d) sh[threadIdx.x][d] += sh[threadIdx.x + o][d];
    __syncthreads();
  }
  if (threadIdx.x < D) bd.gbblk[blockIdx.x * D + threadIdx.x] = sh[0][threadIdx.x];
}

__global__ void reduce_gb_final(BwdDev bd, int nblk, int D, double* g_b) {
  const int d = threadIdx.x;
  if (d >= D) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += bd.gbblk[b * D + d];
  g_b[d] += s;
}

using AdjFn = void (*)(const ClipDev*, const int64_t*, const float*, BwdDev, int);
using GatherFn = void (*)(const ClipDev*, BwdDev, float*, int);

template <int F>
AdjFn pick_adj(bool f16, bool wide) {
  if (wide)
    return f16 ? adjoint_kernel<F, kAdjLanesWide, true, true> : adjoint_kernel<F, kAdjLanesWide, false, true>;
  return f16 ? adjoint_kernel<F, kAdjLanes, true, false> : adjoint_kernel<F, kAdjLanes, false, false>;
}

AdjFn pick(int F, bool f16, bool wide) {
  switch (F) {
    case 1: return pick_adj<1>(f16, wide);
    case 2: return pick_adj<2>(f16, wide);
    case 3: return pick_adj<3>(f16, wide);
    case 4: return pick_adj<4>(f16, wide);
    case 5: return pick_adj<5>(f16, wide);
    case 6: return pick_adj<6>(f16, wide);
    case 7: return pick_adj<7>(f16, wide);
    case 8: return pick_adj<8>(f16, wide);
    case 9: return pick_adj<9>(f16, wide);
    case 10: return pick_adj<10>(f16, wide);
    case 11: return pick_adj<11>(f16, wide);
    case 12: return pick_adj<12>(f16, wide);
    default: return nullptr;
  }
}

GatherFn pick_gather(int F) {
  switch (F) {
    case 1: return gather_kernel<1>;
    case 2: return gather_kernel<2>;
    case 3: return gather_kernel<3>;
    case 4: return gather_kernel<4>;
    case 5: return gather_kernel<5>;
    case 6: return gather_kernel<6>;
    case 7: return gather_kernel<7>;
    case 8: return gather_kernel<8>;
    case 9: return gather_kernel<9>;
    case 10: return gather_kernel<10>;
    case 11: return gather_kernel<11>;
    case 12: return gather_kernel<12>;
    default: return nullptr;
  }
}

using RedFn = void (*)(BwdDev);
template <int D>
RedFn red() { return reduce_gb_blocks<D>; }
RedFn pick_red(int D) {
  switch (D) {
    case 3: return red<3>();
    case 4: return red<4>();
    case 5: return red<5>();
    case 6: return red<6>();
    case 7: return red<7>();
    case 8: return red<8>();
    case 9: return red<9>();
    case 10: return red<10>();
    case 11: return red<11>();
    case 12: return red<12>();
    case 13: return red<13>();
    case 14: return red<14>();
    default: return nullptr;
  }
}

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

int64_t gather_blocks(const ClipDev& hc) {
  return static_cast<int64_t>(hc.T) * ((hc.H + kGatherTile - 1) / kGatherTile) *
         ((hc.W + kGatherTile - 1) / kGatherTile);
}

struct Layout {
  size_t map, rec, gbpart, gbblk, total;
};

Layout layout(const ClipDev& hc, int64_t n) {
  Layout l{};
  const int D = hc.F + 2, P = hc.F + 3;
  size_t off = 0;
  l.map = off;
  off = align256(off + sizeof(int32_t) * static_cast<size_t>(hc.T) * hc.HW);
  l.rec = off;
  off = align256(off + sizeof(double) * (2 * P + 1) * static_cast<size_t>(n));
  l.gbpart = off;
  off = align256(off + sizeof(double) * D * static_cast<size_t>(gather_blocks(hc)));
  l.gbblk = off;
  off = align256(off + sizeof(double) * kRedBlocks * D);
  l.total = off;
  return l;
}

unsigned grid_for(int64_t n, int64_t cap) {
  int64_t b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

size_t backward_scratch_bytes(const ClipDev& hc, int64_t n) { return layout(hc, n).total; }

size_t backward_gather_lds_bytes(const ClipDev& hc) {
  return gather_item_bytes(hc.F) * gather_capacity(hc.F) + kGatherCountBytes;
}

hipError_t launch_backward(const BackwardArgs& a, hipStream_t s) {
  const ClipDev& hc = *a.host_clip;
  const int F = hc.F, D = F + 2;
  // 16 lanes per item (one column each) when the window has at most 16 columns
  const bool wide = 2 * hc.r + 1 <= kAdjLanesWide;
  AdjFn adj = pick(F, hc.feat_f16 != 0, wide);
  GatherFn gat = pick_gather(F);
  RedFn rb = pick_red(D);
  if (!adj || !gat || !rb) return hipErrorInvalidValue;
  const Layout l = layout(hc, a.n);
  char* m = static_cast<char*>(a.scratch);
  const int64_t gblocks = gather_blocks(hc);
  BwdDev bd{reinterpret_cast<int32_t*>(m + l.map), reinterpret_cast<double*>(m + l.rec),
            reinterpret_cast<double*>(m + l.gbpart), reinterpret_cast<double*>(m + l.gbblk), a.n, gblocks};
  const int64_t map_n = static_cast<int64_t>(hc.T) * hc.HW;
  hipLaunchKernelGGL(fill_map_kernel, dim3(grid_for(map_n, 4096)), dim3(256), 0, s, bd.item_map, map_n);
  hipLaunchKernelGGL(map_items_kernel, dim3(grid_for(a.n, 4096)), dim3(256), 0, s, a.clip, a.items, a.n,
                     a.g_alpha, bd.item_map);
  const int L = wide ? kAdjLanesWide : kAdjLanes;
  const int G = kWave / L;
  int64_t blocks = ((a.n + G - 1) / G + kWavesPerBlock - 1) / kWavesPerBlock;
  const int64_t cap = static_cast<int64_t>(a.dev.cus) * 8;
  if (blocks > cap) blocks = cap;
  blocks = (blocks + a.dev.xcds - 1) / a.dev.xcds * a.dev.xcds;   // a multiple of the XCDs (see GroupIter)
  hipLaunchKernelGGL(adj, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, a.clip, a.items, a.g_alpha, bd,
                     a.dev.xcds);
  const size_t lds = std::max(backward_gather_lds_bytes(hc), sizeof(double) * kGatherWaves * D);
  hipLaunchKernelGGL(gat, dim3(static_cast<unsigned>(gblocks)), dim3(kGatherThreads), lds, s, a.clip, bd, a.g_y,
                     gather_capacity(F));
  hipLaunchKernelGGL(rb, dim3(kRedBlocks), dim3(256), 0, s, bd);
  hipLaunchKernelGGL(reduce_gb_final, dim3(1), dim3(64), 0, s, bd, kRedBlocks, D, a.g_b);
  return hipGetLastError();
}

}  // namespace esim
