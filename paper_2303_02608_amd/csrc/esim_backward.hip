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
//   adjoint_kernel        per item: recompute the window, Gram, Cholesky,
//                         theta and v (the window is not stored by the forward
//                         pass); a second window pass writes each sample's
//                         contribution g_alpha (w_i / W) s_i to the item's slot
//                         and sums the bandwidth gradient over the item's lanes
//   gather_kernel         per input (frame, pixel): sums, in a fixed order, the
//                         contributions of every item whose window holds it
//                         (item rows staged in LDS per tile of an input row)
//   reduce_gb_*           fixed-order two-level sum of the per-item b gradients
#include "esim_wlr.h"

namespace esim {
namespace {

constexpr int kAdjLanes = 4;        // lanes per item, windows wider than 16 columns
constexpr int kAdjLanesWide = 16;   // lanes per item, windows of at most 16 columns
constexpr int kRedBlocks = 256;

struct BwdDev {
  int32_t* item_map;   // [T*HW]
  float* contrib;      // [n][S]
  double* gbpart;      // [n][D]
  double* gbblk;       // [kRedBlocks][D]
  int64_t S;           // window slots per item: (2r+1)^2 (2tr+1)
  int64_t n;
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

template <int F, int L, bool F16>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(F <= 8 ? 2 : 1)))
adjoint_kernel(const ClipDev* __restrict__ clips, const int64_t* __restrict__ items,
               const float* __restrict__ g_alpha, BwdDev bd, int nxcd) {
  constexpr int D = F + 2;
  constexpr int P = F + 3;
  constexpr int G = kWave / L;
  const ClipDev& C = clips[0];
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / L;
  const int j = lane % L;
  const int64_t ngroups = (bd.n + G - 1) / G;
  const int r = C.r, tr = C.tr;
  const int span = 2 * r + 1;
  GroupIter it_groups(ngroups, nxcd);
  int64_t g;
  while (it_groups.next(g)) {
    const int64_t i = g * G + slot;
    int64_t pix = 0;
    int t = 0;
    const bool active = i < bd.n && item_ok(C, items[i], g_alpha, i, pix, t);
    if (__ballot(active) == 0) {
      if (i < bd.n && j == 0)
        for (int d = 0; d < D; ++d) bd.gbpart[i * D + d] = 0.0;
      continue;
    }
    ItemGeom<F, F16, double> geo;
    make_geom(geo, C, active ? pix : 0, active ? t : 0, 0, C.T, active);

    Gram<F, double> gm;
    gm.zero_snap();
    window_loop<F, L, F16, double>(
        geo, j, [&](double) { gm.pass_begin_snap(); },
        [&](double w, double yd, const double (&v)[F], double vy, int, int, int, bool) {
          gm.add_onepass(w, yd, v, vy);
        },
        [&](double vx) { gm.pass_end_snap(vx); });
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
    const double ga = active ? static_cast<double>(g_alpha[i]) : 0.0;
    float* ci = bd.contrib + (active ? i : 0) * bd.S;

    double gb[D];
#pragma unroll
    for (int d = 0; d < D; ++d) gb[d] = 0.0;
    double cur_vx = 0.0;
    window_loop<F, L, F16, double>(
        geo, j, [&](double vx) { cur_vx = vx; },
        [&](double w, double yd, const double (&v)[F], double vy, int dx, int dt, int dy, bool ok) {
          double s = fma(vv[1], cur_vx, fma(vv[2], vy, vv[0]));
          double pred = fma(th[1], cur_vx, fma(th[2], vy, th[0]));
#pragma unroll
          for (int f = 0; f < F; ++f) {
            s = fma(vv[3 + f], v[f], s);
            pred = fma(th[3 + f], v[f], pred);
          }
          const double res = yd - pred;
          // only in-image samples have a slot the gather reads
          if (ok) ci[((dt + tr) * span + (dy + r)) * span + (dx + r)] = static_cast<float>(ga * w * iW * s);
          const double k = ga * (s * res - vLt) * iW * w;
          gb[0] = fma(k, cur_vx * cur_vx, gb[0]);
          gb[1] = fma(k, vy * vy, gb[1]);
#pragma unroll
          for (int f = 0; f < F; ++f) gb[2 + f] = fma(k, v[f] * v[f], gb[2 + f]);
        },
        [&](double) {});
#pragma unroll
    for (int d = 0; d < D; ++d) gb[d] = group_sum<L>(gb[d]);
    if (i < bd.n && j == 0) {
#pragma unroll
      for (int d = 0; d < D; ++d)
        bd.gbpart[i * D + d] = active ? gb[d] * C.sf[d] * C.h : 0.0;   // / b_d = * sf_d * h
    }
  }
}

// One block per (frame, row, tile of kGatherTile columns) of inputs.  For each
// item row (tc, yc) that can reach the tile, in ascending order, the block
// stages the map row and the items' contributions to this input row (2r + 1
// consecutive slots per item, coalesced) in LDS; each thread then adds, for
// its input column, the items at xc = xq - r .. xq + r in ascending order.
// The order of the sum (tc, yc, xc ascending) is fixed, so the result does not
// depend on scheduling.
constexpr int kGatherTile = 256;

__global__ void __launch_bounds__(kGatherTile)
gather_kernel(const ClipDev* __restrict__ clips, BwdDev bd, float* __restrict__ g_y) {
  extern __shared__ float sm[];
  const ClipDev& C = clips[0];
  const int r = C.r, tr = C.tr, W = C.W, H = C.H, T = C.T;
  const int span = 2 * r + 1;
  const int seg = kGatherTile + 2 * r;                 // staged columns
  int32_t* mrow = reinterpret_cast<int32_t*>(sm);      // [seg]
  float* cx = sm + seg;                                // [seg][span]
  const int ntile = (W + kGatherTile - 1) / kGatherTile;
  const int64_t b = blockIdx.x;
  const int tile = static_cast<int>(b % ntile);
  const int64_t rowq = b / ntile;                      // tq * H + yq
  const int tq = static_cast<int>(rowq / H), yq = static_cast<int>(rowq % H);
  const int x_lo = tile * kGatherTile;
  const int xs = x_lo - r;                             // column of staged index 0
  const int xq = x_lo + static_cast<int>(threadIdx.x);
  const int lane = static_cast<int>(threadIdx.x) & (kWave - 1);
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  double acc = 0.0;
  const int t0 = max(0, tq - tr), t1 = min(T - 1, tq + tr);
  const int y0 = max(0, yq - r), y1 = min(H - 1, yq + r);
  // item rows (tc, yc) in ascending order, k = (tc - t0) * ny + (yc - y0); the
  // map entries of row k + 1 are loaded into registers while row k is used
  const int ny = y1 - y0 + 1;
  const int nrow = (t1 - t0 + 1) * ny;
  constexpr int kPer = 2;                              // staged columns per thread (seg <= 2 tile)
  auto load_map = [&](int k, int32_t (&v)[kPer]) {
    const int tc = t0 + k / ny, yc = y0 + k % ny;
    const int32_t* row = bd.item_map + static_cast<int64_t>(tc) * C.HW + static_cast<int64_t>(yc) * W;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int c = static_cast<int>(threadIdx.x) + q * kGatherTile;
      const int x = xs + c;
      v[q] = (c < seg && x >= 0 && x < W) ? row[x] : -1;
    }
  };
  int32_t nxt[kPer];
  if (nrow > 0) load_map(0, nxt);
  for (int k = 0; k < nrow; ++k) {
    const int tc = t0 + k / ny, yc = y0 + k % ny;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int c = static_cast<int>(threadIdx.x) + q * kGatherTile;
      if (c < seg) mrow[c] = nxt[q];
    }
    __syncthreads();
    if (k + 1 < nrow) load_map(k + 1, nxt);
    // each wave walks the present items of its 64-column chunks (a
    // wave-uniform loop over the ballot); the lanes load the items' slots,
    // coalesced 4 (2r + 1)-byte reads: four items per step for windows of at
    // most 16 columns, one otherwise
    const int64_t sbase = static_cast<int64_t>((tq - tc + tr) * span + (yq - yc + r)) * span;
    for (int base = wave * kWave; base < seg; base += kGatherTile) {
      const int c = base + lane;
      const int32_t it = c < seg ? mrow[c] : -1;
      uint64_t mask = __ballot(it >= 0);
      if (span <= 16) {
        // four items per step, 16 lanes each (lane q * 16 + m takes slot m of
        // the q-th next item)
        const int q = lane >> 4, m = lane & 15;
        while (mask != 0) {
          int bits[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            bits[u] = mask != 0 ? __ffsll(static_cast<unsigned long long>(mask)) - 1 : -1;
            if (mask != 0) mask &= mask - 1;
          }
          const int bq = q == 0 ? bits[0] : q == 1 ? bits[1] : q == 2 ? bits[2] : bits[3];
          const int32_t itc = __shfl(it, bq < 0 ? 0 : bq);
          if (bq >= 0 && m < span)
            cx[(base + bq) * span + m] = bd.contrib[static_cast<int64_t>(itc) * bd.S + sbase + m];
        }
      } else {
        while (mask != 0) {
          const int bit = __ffsll(static_cast<unsigned long long>(mask)) - 1;
          mask &= mask - 1;
          const int32_t itc = __shfl(it, bit);
          for (int mm = lane; mm < span; mm += kWave)
            cx[(base + bit) * span + mm] = bd.contrib[static_cast<int64_t>(itc) * bd.S + sbase + mm];
        }
      }
    }
    __syncthreads();
    if (xq < W) {
      // items at xc = xq - r + m (staged index threadIdx.x + m), slot x-index span - 1 - m
      for (int m = 0; m < span; ++m) {
        const int c = static_cast<int>(threadIdx.x) + m;
        if (mrow[c] >= 0) acc += static_cast<double>(cx[c * span + (span - 1 - m)]);
      }
    }
    __syncthreads();
  }
  if (xq < W && acc != 0.0) g_y[rowq * W + xq] += static_cast<float>(acc);
}

template <int D>
__global__ void __launch_bounds__(256) reduce_gb_blocks(BwdDev bd) {
  __shared__ double sh[256][D];
  double acc[D];
#pragma unroll
  for (int d = 0; d < D; ++d) acc[d] = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < bd.n;
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

template <int F>
AdjFn pick_adj(bool f16, bool wide) {
  if (wide) return f16 ? adjoint_kernel<F, kAdjLanesWide, true> : adjoint_kernel<F, kAdjLanesWide, false>;
  return f16 ? adjoint_kernel<F, kAdjLanes, true> : adjoint_kernel<F, kAdjLanes, false>;
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

struct Layout {
  size_t map, contrib, gbpart, gbblk, total;
  int64_t S;
};

Layout layout(const ClipDev& hc, int64_t n) {
  Layout l{};
  const int D = hc.F + 2;
  l.S = static_cast<int64_t>(2 * hc.r + 1) * (2 * hc.r + 1) * (2 * hc.tr + 1);
  size_t off = 0;
  l.map = off;
  off = align256(off + sizeof(int32_t) * static_cast<size_t>(hc.T) * hc.HW);
  l.contrib = off;
  off = align256(off + sizeof(float) * static_cast<size_t>(n) * l.S);
  l.gbpart = off;
  off = align256(off + sizeof(double) * static_cast<size_t>(n) * D);
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
  return sizeof(float) * static_cast<size_t>(kGatherTile + 2 * hc.r) * (2 * hc.r + 2);
}

hipError_t launch_backward(const BackwardArgs& a, hipStream_t s) {
  const ClipDev& hc = *a.host_clip;
  const int F = hc.F, D = F + 2;
  // 16 lanes per item (one column each) when the window has at most 16
  // columns: an item's contributions to a window row are then one coalesced
  // 4(2r+1)-byte store
  const bool wide = 2 * hc.r + 1 <= kAdjLanesWide;
  AdjFn adj = pick(F, hc.feat_f16 != 0, wide);
  RedFn rb = pick_red(D);
  if (!adj || !rb) return hipErrorInvalidValue;
  const Layout l = layout(hc, a.n);
  char* m = static_cast<char*>(a.scratch);
  BwdDev bd{reinterpret_cast<int32_t*>(m + l.map), reinterpret_cast<float*>(m + l.contrib),
            reinterpret_cast<double*>(m + l.gbpart), reinterpret_cast<double*>(m + l.gbblk), l.S, a.n};
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
  const size_t lds = backward_gather_lds_bytes(hc);
  const int64_t gblocks = static_cast<int64_t>(hc.T) * hc.H * ((hc.W + kGatherTile - 1) / kGatherTile);
  hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(gblocks)), dim3(kGatherTile), lds, s, a.clip, bd,
                     a.g_y);
  hipLaunchKernelGGL(rb, dim3(kRedBlocks), dim3(256), 0, s, bd);
  hipLaunchKernelGGL(reduce_gb_final, dim3(1), dim3(64), 0, s, bd, kRedBlocks, D, a.g_b);
  return hipGetLastError();
}

}  // namespace esim
