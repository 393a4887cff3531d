// Nearest same-polarity neighbour distances between two event sets, for the
// event-set comparison of Sec. 3 (quantitative comparison: events as signed
// points (x, y, t); precision and recall count the events whose nearest
// same-polarity event of the other set lies within a threshold).
//
//   bitmap_clear_kernel  zero the occupancy bitmaps (a fill kernel, so a call
//                        can sit in a captured graph)
//   bitmap_set_kernel    one bit per source event in the bitmap of its
//                        polarity: [2][T][H][ceil(W / 32)] words (atomicOr:
//                        the result does not depend on the order)
//   nn_kernel            per query event: for the frames and rows of the box
//                        |dt| <= rt, |dy| <= ry, visited centre-out, the
//                        nearest set bit of the row within |dx| <= rx of the
//                        query column (count leading/trailing zeros over the
//                        row's words); the smallest scaled distance (FP64)
//                        wins, and rows whose (dt, dy) offset alone cannot beat
//                        it are not visited.  With rx, ry, rt the lattice
//                        extents of the radius rmax, this is the exact nearest
//                        neighbour within rmax.
#include <cmath>
#include <cstdint>
#include <mutex>

#include "esim.h"
#include "esim_internal.h"

// Occupancy bitmaps of esim_nn_distances_noalloc: a fixed device array, so that
// call allocates nothing.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code this name is a host-side stand-in, not
// a device address: the device address is obtained once per device with
// hipGetSymbolAddress (nn_static_scratch) and only that address is used.
static __device__ __align__(256) uint32_t scratch[ESIM_NN_STATIC_BYTES / sizeof(uint32_t)];

namespace esim {
namespace {

__global__ void __launch_bounds__(256) bitmap_clear_kernel(uint32_t* __restrict__ bm, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) bm[i] = 0u;
}

__global__ void __launch_bounds__(256)
bitmap_set_kernel(uint32_t* __restrict__ bm, const int32_t* __restrict__ x, const int32_t* __restrict__ y,
                  const int32_t* __restrict__ t, const int8_t* __restrict__ p, int64_t n, int W, int H, int T,
                  int64_t wpr) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int xi = x[i], yi = y[i], ti = t[i], pi = p[i];
    if (xi < 0 || xi >= W || yi < 0 || yi >= H || ti < 0 || ti >= T || (pi != 1 && pi != -1)) continue;
    const int pl = pi > 0 ? 0 : 1;
    const int64_t w = ((static_cast<int64_t>(pl) * T + ti) * H + yi) * wpr + (xi >> 5);
    atomicOr(bm + w, 1u << (xi & 31));
  }
}

// Distance in columns from x to the nearest set bit of row within [lo, hi]
// (lo <= x <= hi), or -1 if none.
__device__ __forceinline__ int nearest_bit(const uint32_t* __restrict__ row, int x, int lo, int hi) {
  int best = -1;
  // right: lowest set bit in [x, hi]
  for (int w = x >> 5; w <= (hi >> 5); ++w) {
    uint32_t m = row[w];
    const int b0 = w << 5;
    if (b0 < x) m &= ~0u << (x - b0);
    if (b0 + 31 > hi) m &= (hi - b0 >= 31) ? ~0u : ((1u << (hi - b0 + 1)) - 1u);
    if (m) {
      best = b0 + __builtin_ctz(m) - x;
      break;
    }
  }
  // left: highest set bit in [lo, x - 1], only if it can be nearer
  const int lim = best < 0 ? x - lo : min(best - 1, x - lo);
  if (lim > 0) {
    const int l2 = x - lim;
    for (int w = (x - 1) >> 5; w >= (l2 >> 5); --w) {
      uint32_t m = row[w];
      const int b0 = w << 5;
      if (b0 + 31 > x - 1) m &= (x - 1 - b0 >= 31) ? ~0u : ((1u << (x - 1 - b0 + 1)) - 1u);
      if (b0 < l2) m &= ~0u << (l2 - b0);
      if (m) {
        const int d = x - (b0 + 31 - __builtin_clz(m));
        if (best < 0 || d < best) best = d;
        break;
      }
    }
  }
  return best;
}

__global__ void __launch_bounds__(256)
nn_kernel(const uint32_t* __restrict__ bm, const int32_t* __restrict__ qx, const int32_t* __restrict__ qy,
          const int32_t* __restrict__ qt, const int8_t* __restrict__ qp, int64_t nq, int W, int H, int T,
          int64_t wpr, double sx, double sy, double st, int rx, int ry, int rt, double rmax,
          double* __restrict__ d) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nq; i += stride) {
    const int xi = qx[i], yi = qy[i], ti = qt[i], pi = qp[i];
    double best = INFINITY;
    if (xi >= 0 && xi < W && yi >= 0 && yi < H && ti >= 0 && ti < T && (pi == 1 || pi == -1)) {
      const int pl = pi > 0 ? 0 : 1;
      const int lo = max(0, xi - rx), hi = min(W - 1, xi + rx);
      // frames and rows centre-out (0, -1, +1, -2, +2, ...): |dt| and |dy| never
      // decrease, so once a row's offset alone reaches the best distance every
      // later row of the frame (and, at dy = 0, every later frame) does too
      for (int kt = 0; kt <= 2 * rt; ++kt) {
        const int dt = (kt & 1) ? -((kt + 1) >> 1) : (kt >> 1);
        const double et = dt * st;
        if (et * et >= best) break;
        const int tc = ti + dt;
        if (tc < 0 || tc >= T) continue;
        for (int ky = 0; ky <= 2 * ry; ++ky) {
          const int dy = (ky & 1) ? -((ky + 1) >> 1) : (ky >> 1);
          const double ey = dy * sy;
          const double base = fma(et, et, ey * ey);
          if (base >= best) break;
          const int yc = yi + dy;
          if (yc < 0 || yc >= H) continue;
          const uint32_t* row = bm + ((static_cast<int64_t>(pl) * T + tc) * H + yc) * wpr;
          const int dx = nearest_bit(row, xi, lo, hi);
          if (dx >= 0) {
            const double ex = dx * sx;
            best = min(best, fma(ex, ex, base));
          }
        }
      }
    }
    const double dist = sqrt(best);
    d[i] = dist <= rmax ? dist : INFINITY;
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

bool nn_static_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
    addr[dev] = p;
  }
  *out = addr[dev];
  return true;
}

size_t nn_scratch_bytes(int W, int H, int T) {
  const int64_t wpr = (static_cast<int64_t>(W) + 31) / 32;
  return sizeof(uint32_t) * 2 * static_cast<size_t>(T) * H * wpr;
}

hipError_t launch_nn(const NnArgs& a, hipStream_t s) {
  const int64_t wpr = (static_cast<int64_t>(a.W) + 31) / 32;
  const int64_t words = 2 * static_cast<int64_t>(a.T) * a.H * wpr;
  uint32_t* bm = static_cast<uint32_t*>(a.scratch);
  hipLaunchKernelGGL(bitmap_clear_kernel, dim3(grid_for(words)), dim3(256), 0, s, bm, words);
  if (a.ns > 0)
    hipLaunchKernelGGL(bitmap_set_kernel, dim3(grid_for(a.ns)), dim3(256), 0, s, bm, a.sx, a.sy, a.st, a.sp,
                       a.ns, a.W, a.H, a.T, wpr);
  if (a.nq > 0)
    hipLaunchKernelGGL(nn_kernel, dim3(grid_for(a.nq)), dim3(256), 0, s, bm, a.qx, a.qy, a.qt, a.qp, a.nq, a.W,
                       a.H, a.T, wpr, a.scale_x, a.scale_y, a.scale_t, a.rx, a.ry, a.rt, a.rmax, a.d);
  return hipGetLastError();
}

}  // namespace esim
