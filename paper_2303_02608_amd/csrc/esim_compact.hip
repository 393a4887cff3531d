// Threshold, compaction, event emission and state updates (HBM-bound).
//
//   log_kernel         Sec. 1.1: y = log(E + eps) (log4_kernel: 16-byte
//                      accesses when both arrays are 16-byte aligned).
//   flag_kernel        per pixel of a 256-pixel block:
//                        threshold  - Prop. 1 / eqs. 8-9: dL = beta_ref^T (f_t -
//                                     x_ref) over the F buffer channels (the
//                                     image-coordinate part is zero for a
//                                     pixel); flag when dL^2 >= C^2;
//                        exhaustive - eq. 1 on the regressed alpha against L_ref;
//                        raw        - eq. 1 on y against L_ref;
//                      wave ballots of the flags and polarities, block counts;
//                      block 0 records the event base.
//   chunk_kernel       totals of chunks of kChunkBlocks block counts (only for
//                      grids above kDirectPrefixBlocks blocks).
//   scatter_kernel     each block's offset: the sum of the counts of the
//                      blocks before it, read directly (or as chunk totals plus
//                      the counts inside its chunk), with no inter-block
//                      signalling; rank = offset + popcounts of
//                      the ballots below the lane; writes the work list
//                      (threshold) and/or the events; the last block writes
//                      the count and advances the event count.
//   list_events_kernel events of the work-list items and the state update
//                      (Sec. 2.2: the model at the last event is kept until the
//                      pixel's next event); advance_kernel then advances the
//                      event count.
//   init_kernel        state <- the models of frame t (no events).
#include "esim_internal.h"
#include "esim_compact.h"

namespace esim {
namespace {

__global__ void __launch_bounds__(256) log_kernel(const float* __restrict__ E, float* __restrict__ y,
                                                  int64_t n, float eps) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = logf(E[i] + eps);
}

// The same with 16-byte accesses (both pointers 16-byte aligned): four values
// per lane and iteration; the n % 4 last values by the first lanes.
__global__ void __launch_bounds__(256) log4_kernel(const float4* __restrict__ E, float4* __restrict__ y,
                                                   int64_t n, float eps) {
  const int64_t n4 = n >> 2;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t id = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t i = id; i < n4; i += stride) {
    const float4 e = E[i];
    y[i] = make_float4(logf(e.x + eps), logf(e.y + eps), logf(e.z + eps), logf(e.w + eps));
  }
  const int64_t tail = n - (n4 << 2);
  if (id < tail) {
    const float* Es = reinterpret_cast<const float*>(E);
    float* ys = reinterpret_cast<float*>(y);
    ys[(n4 << 2) + id] = logf(Es[(n4 << 2) + id] + eps);
  }
}

// Levels L_ref + k p C passed by a change d (every-crossing rule): floor(|d| / C),
// at most kMaxCrossings (so that block and wave sums of counts stay in int32).
constexpr double kMaxCrossings = 1048576.0;
__device__ __forceinline__ int crossings(double d, double C) {
  const double n = floor(fabs(d) / C);
  return n >= 1.0 ? static_cast<int>(fmin(n, kMaxCrossings)) : 0;
}

// Exclusive prefix of one int per thread of a kBlock-thread block.
__device__ int block_exclusive_scan(int v) {
  __shared__ int wsum[kWavesPerBlock];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; ++k) before += wsum[k];
  return before + x - v;
}

__global__ void __launch_bounds__(kBlock)
flag_kernel(const ClipDev* __restrict__ clips, int nclips, int t, int mode, float* __restrict__ dl,
            const float* __restrict__ alpha, Workspace ws, const int64_t* __restrict__ ev_count, int split) {
  __shared__ int wcount[kWavesPerBlock];
  const int64_t b = blockIdx.x;
  const int cl = block_clip(clips, nclips, b);
  const ClipDev& C = clips[cl];
  const int64_t p = (b - C.blk_off) * kBlock + threadIdx.x;
  const bool in = p < C.HW && t >= 0 && t < C.T;
  bool flag = false, pos = false;
  int ncross = 0;
  if (in) {
    float val = __builtin_nanf("");
    if (mode == kFlagThreshold) {
      if (t >= 1) {
        double d = 0.0;
        for (int f = 0; f < C.F; ++f) {
          const double bf = C.st_beta[f * C.HW + p];
          const double xf = C.st_xref[f * C.HW + p];
          d = fma(bf, static_cast<double>(feat_value(C, t, f, p)) - xf, d);
        }
        flag = d * d >= C.C * C.C;
        pos = d > 0.0;
        val = static_cast<float>(d);
      }
    } else {
      const float L = mode == kFlagExhaustive ? alpha[C.pix_off + p]
                                              : C.y[static_cast<int64_t>(t) * C.HW + p];
      if (t == 0) {
        C.st_alpha[p] = L;
        if (C.multi) C.st_last[p] = L;
      } else {
        const double d = static_cast<double>(L) - static_cast<double>(C.st_alpha[p]);
        val = static_cast<float>(d);
        if (C.multi) {
          // every crossing: the scatter writes the events and updates the state
          ncross = crossings(d, C.C);
          flag = ncross > 0;
          pos = d > 0.0;
        } else if (fabs(d) >= C.C) {
          flag = true;
          pos = d > 0.0;
          C.st_alpha[p] = L;
        }
      }
    }
    if (dl) dl[C.pix_off + p] = val;
  }
  const int w = threadIdx.x / kWave;
  const uint64_t fm = __ballot(flag);
  const uint64_t pm = __ballot(flag && pos);
  int wc = __popcll(fm);
  if (C.multi && mode != kFlagThreshold) {   // uniform: one clip per block
    wc = ncross;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) wc += __shfl_xor(wc, o);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    ws.flags[b * kWavesPerBlock + w] = fm;
    ws.pol[b * kWavesPerBlock + w] = pm;
    wcount[w] = wc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) s += wcount[k];
    // a split compaction counts the second segment's items in the high half,
    // so one prefix sum gives both ranks (the totals stay below 2^32)
    if (split && C.list_class) s |= s << 32;
    ws.bcount[b] = s;
    // the event base of this step (the count is advanced by the scatter)
    if (b == 0) ws.misc[0] = ev_count ? *ev_count : 0;
  }
}

// Sum of a[lo, hi) by one block of kBlock threads.
template <class V>
__device__ int64_t block_sum(const V* __restrict__ a, int64_t lo, int64_t hi) {
  __shared__ int64_t red[kWavesPerBlock];
  int64_t s = 0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) s += a[k];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  int64_t tot = 0;
#pragma unroll
  for (int k = 0; k < kWavesPerBlock; ++k) tot += red[k];
  return tot;
}

// Counts of blocks [0, b): directly, or (chunked) the chunk totals before b's
// chunk plus the counts inside it.
__device__ int64_t counts_before(const Workspace& ws, int64_t b, bool chunked) {
  if (!chunked) return block_sum(ws.bcount, 0, b);
  const int64_t c = b / kChunkBlocks;
  const int64_t s = block_sum(ws.chunk, 0, c);
  return s + block_sum(ws.bcount, c * kChunkBlocks, b);
}

// Block c: the total count of blocks [c * kChunkBlocks, (c + 1) * kChunkBlocks).
__global__ void __launch_bounds__(kBlock) chunk_kernel(Workspace ws, int64_t nblk) {
  const int64_t c = blockIdx.x;
  const int64_t t = block_sum(ws.bcount, c * kChunkBlocks, min(nblk, (c + 1) * kChunkBlocks));
  if (threadIdx.x == 0) ws.chunk[c] = t;
}

__global__ void __launch_bounds__(kBlock)
scatter_kernel(const ClipDev* __restrict__ clips, int nclips, int t, int mode, Workspace ws, int chunked,
               const float* __restrict__ alpha, int64_t* __restrict__ worklist, int32_t* __restrict__ count,
               EventsDev ev, int64_t seg_b) {
  constexpr int64_t kLow = 0xFFFFFFFFll;
  const int64_t b = blockIdx.x;
  const int64_t packed = counts_before(ws, b, chunked != 0);
  const int64_t off0 = packed & kLow;         // flagged pixels before this block
  const int64_t offb0 = packed >> 32;         // of them in second-segment clips (split only)
  const int64_t base = ws.misc[0];
  if (b == gridDim.x - 1 && threadIdx.x == 0) {
    const int64_t tp = packed + ws.bcount[b];
    const int64_t total = tp & kLow;
    if (count) {
      const int64_t nb = seg_b >= 0 ? tp >> 32 : 0;
      count[0] = static_cast<int32_t>(total - nb);
      count[1] = static_cast<int32_t>(total - nb);
      if (seg_b >= 0) {
        count[2] = static_cast<int32_t>(nb);
        count[3] = static_cast<int32_t>(nb);
      }
    }
    if (ev.count) *ev.count = base + total;
  }
  const int cl = block_clip(clips, nclips, b);
  const ClipDev& C = clips[cl];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (C.multi && mode != kFlagThreshold) {   // uniform: one clip per block
    // every-crossing rule: n events per pixel at the interpolated times the
    // levels L_ref + k p C are passed; then L_ref += n p C and L_last = L
    const int64_t p = (b - C.blk_off) * kBlock + threadIdx.x;
    const bool in = p < C.HW && t >= 1 && t < C.T;
    float L = 0.0f, Lref = 0.0f, Llast = 0.0f;
    int n = 0;
    if (in) {
      L = mode == kFlagExhaustive ? alpha[C.pix_off + p] : C.y[static_cast<int64_t>(t) * C.HW + p];
      Lref = C.st_alpha[p];
      Llast = C.st_last[p];
      n = crossings(static_cast<double>(L) - static_cast<double>(Lref), C.C);
    }
    const int64_t off = off0 + block_exclusive_scan(n);
    if (n > 0) {
      const double d = static_cast<double>(L) - static_cast<double>(Lref);
      const int pol = d > 0.0 ? 1 : -1;
      const double step = pol * C.C;               // exact: C times +-1
      const double den = static_cast<double>(L) - static_cast<double>(Llast);
      for (int k = 1; k <= n; ++k) {
        const int64_t e = base + off + (k - 1);
        if (e >= ev.capacity) break;
        const double level = static_cast<double>(Lref) + static_cast<double>(k) * step;
        ev.x[e] = static_cast<int32_t>(p % C.W);
        ev.y[e] = static_cast<int32_t>(p / C.W);
        ev.t[e] = t;
        ev.p[e] = static_cast<int8_t>(pol);
        if (ev.clip) ev.clip[e] = cl;
        if (ev.ts) ev.ts[e] = static_cast<float>(((t - 1) + (level - static_cast<double>(Llast)) / den) * C.dt);
      }
      // the reference level is kept in FP32 like the rest of the state
      C.st_alpha[p] = static_cast<float>(static_cast<double>(Lref) + static_cast<double>(n) * step);
    }
    if (in) C.st_last[p] = L;
    return;
  }
  const uint64_t m = ws.flags[b * kWavesPerBlock + w];
  if (!((m >> lane) & 1ull)) return;
  const int64_t p = (b - C.blk_off) * kBlock + threadIdx.x;
  int64_t rank = 0;                           // among the block's flagged pixels
  for (int k = 0; k < w; ++k) rank += __popcll(ws.flags[b * kWavesPerBlock + k]);
  rank += __popcll(m & ((1ull << lane) - 1ull));
  const int64_t off = off0 + rank;
  if (mode == kFlagThreshold && worklist) {
    // a block lies in one clip, so its items all go to the same segment
    const int64_t pos = seg_b < 0 ? off : C.list_class ? seg_b + offb0 + rank : off0 - offb0 + rank;
    worklist[pos] = (static_cast<int64_t>(cl) << 32) | p;
  }
  if (ev.x) {
    const int64_t e = base + off;
    if (e < ev.capacity) {
      const bool pos = (ws.pol[b * kWavesPerBlock + w] >> lane) & 1ull;
      ev.x[e] = static_cast<int32_t>(p % C.W);
      ev.y[e] = static_cast<int32_t>(p / C.W);
      ev.t[e] = t;
      ev.p[e] = pos ? 1 : -1;
      if (ev.clip) ev.clip[e] = cl;
      if (ev.ts) ev.ts[e] = static_cast<float>(t * C.dt);
    }
  }
}

// The model of regression output i (alpha[i], beta[d * n_out + i] over D,
// coordinates first) becomes pixel p's reference state at frame t.
__device__ __forceinline__ void store_model(const ClipDev& C, int64_t p, int t, int64_t i,
                                            const float* __restrict__ alpha,
                                            const float* __restrict__ beta, int64_t n_out) {
  C.st_alpha[p] = alpha[i];
  if (beta && C.st_beta)
    for (int f = 0; f < C.F; ++f) C.st_beta[f * C.HW + p] = beta[(2 + f) * n_out + i];
  if (beta && C.st_bxy) {
    C.st_bxy[p] = beta[i];
    C.st_bxy[C.HW + p] = beta[n_out + i];
  }
  if (C.st_xref)
    for (int f = 0; f < C.F; ++f) C.st_xref[f * C.HW + p] = feat_value(C, t, f, p);
  if (C.st_tref) C.st_tref[p] = t;
}

__device__ void list_events_body(const ClipDev* __restrict__ clips, int nclips, int t,
                                 const int64_t* __restrict__ worklist, int64_t n, int64_t base,
                                 int64_t stride, const float* __restrict__ dl,
                                 const float* __restrict__ alpha, const float* __restrict__ beta,
                                 int64_t n_out, const Workspace& ws, const EventsDev& ev);

__global__ void __launch_bounds__(256)
list_events_kernel(const ClipDev* __restrict__ clips, int nclips, int t, const int64_t* __restrict__ worklist,
                   const int32_t* __restrict__ count, const float* __restrict__ dl,
                   const float* __restrict__ alpha, const float* __restrict__ beta, int64_t n_out,
                   int64_t max_items, Workspace ws, EventsDev ev) {
  // the device count is clamped to the work-list capacity and output length
  const int64_t n = max(static_cast<int64_t>(0),
                        min(static_cast<int64_t>(count[0]), min(max_items, n_out)));
  const int64_t base = *ev.count;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  list_events_body(clips, nclips, t, worklist, n, base, stride, dl, alpha, beta, n_out, ws, ev);
}

// Advances the event count after list_events_kernel (which read it as its base).
__global__ void advance_kernel(int64_t* __restrict__ ev_count, const int32_t* __restrict__ count) {
  if (threadIdx.x == 0) *ev_count += count[1];
}

__device__ void list_events_body(const ClipDev* __restrict__ clips, int nclips, int t,
                                 const int64_t* __restrict__ worklist, int64_t n, int64_t base,
                                 int64_t stride, const float* __restrict__ dl,
                                 const float* __restrict__ alpha, const float* __restrict__ beta,
                                 int64_t n_out, const Workspace& ws, const EventsDev& ev) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t it = worklist[i];
    if (it < 0) continue;
    const int cl = static_cast<int>((it >> 32) & 0xFFF);
    if (cl >= nclips) continue;
    const ClipDev& C = clips[cl];
    const int64_t p = it & 0xFFFFFFFFll;
    if (p >= C.HW || t >= C.T) continue;
    const int64_t e = base + i;
    const float d = dl[C.pix_off + p];
    if (e >= 0 && e < ev.capacity) {
      ev.x[e] = static_cast<int32_t>(p % C.W);
      ev.y[e] = static_cast<int32_t>(p / C.W);
      ev.t[e] = t;
      ev.p[e] = d > 0.0f ? 1 : -1;
      if (ev.clip) ev.clip[e] = cl;
      if (ev.ts) ev.ts[e] = static_cast<float>(t * C.dt);
    }
    store_model(C, p, t, i, alpha, beta, n_out);
  }
}

__global__ void __launch_bounds__(256)
list_state_kernel(const ClipDev* __restrict__ clips, int nclips, int t, const int64_t* __restrict__ worklist,
                  const int32_t* __restrict__ count, const float* __restrict__ alpha,
                  const float* __restrict__ beta, int64_t n_out, int64_t max_items) {
  const int64_t n = max(static_cast<int64_t>(0),
                        min(static_cast<int64_t>(count[0]), min(max_items, n_out)));
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t it = worklist[i];
    if (it < 0) continue;
    const int cl = static_cast<int>((it >> 32) & 0xFFF);
    if (cl >= nclips) continue;
    const ClipDev& C = clips[cl];
    const int64_t p = it & 0xFFFFFFFFll;
    if (p >= C.HW || t >= C.T) continue;
    store_model(C, p, t, i, alpha, beta, n_out);
  }
}

__global__ void __launch_bounds__(kBlock)
init_kernel(const ClipDev* __restrict__ clips, int nclips, int t, const float* __restrict__ alpha,
            const float* __restrict__ beta, int64_t n_out) {
  const int64_t b = blockIdx.x;
  const int cl = block_clip(clips, nclips, b);
  const ClipDev& C = clips[cl];
  const int64_t p = (b - C.blk_off) * kBlock + threadIdx.x;
  if (p >= C.HW || t < 0 || t >= C.T) return;
  if (!alpha) {
    C.st_alpha[p] = C.y[static_cast<int64_t>(t) * C.HW + p];
    return;
  }
  store_model(C, p, t, C.pix_off + p, alpha, beta, n_out);
}

}  // namespace

hipError_t launch_log(const float* E, float* y, int64_t n, float eps, hipStream_t s) {
  const bool vec = (reinterpret_cast<uintptr_t>(E) % 16 == 0) && (reinterpret_cast<uintptr_t>(y) % 16 == 0);
  const int64_t per = vec ? 4 : 1;
  int64_t blocks = (n / per + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (vec)
    hipLaunchKernelGGL(log4_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(E), reinterpret_cast<float4*>(y), n, eps);
  else
    hipLaunchKernelGGL(log_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, E, y, n, eps);
  return hipGetLastError();
}

hipError_t launch_flag_compact(const ClipDev* clips, int nclips, int64_t nblk, int t, int mode,
                               float* dl, const float* alpha, const Workspace& ws, int64_t* worklist,
                               int32_t* count, const EventsDev* ev, hipStream_t s, int64_t seg_b) {
  int64_t* wl = mode == kFlagThreshold ? worklist : nullptr;
  if (!wl) seg_b = -1;
  hipLaunchKernelGGL(flag_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s, clips, nclips,
                     t, mode, dl, alpha, ws, ev ? ev->count : nullptr, seg_b >= 0 ? 1 : 0);
  return launch_scatter(clips, nclips, nblk, t, mode, alpha, ws, wl, count, ev, s, seg_b);
}

hipError_t launch_scatter(const ClipDev* clips, int nclips, int64_t nblk, int t, int mode,
                          const float* alpha, const Workspace& ws, int64_t* worklist, int32_t* count,
                          const EventsDev* ev, hipStream_t s, int64_t seg_b) {
  int64_t* wl = mode == kFlagThreshold ? worklist : nullptr;
  if (!wl) seg_b = -1;
  const int chunked = nblk > kDirectPrefixBlocks ? 1 : 0;
  if (chunked)
    hipLaunchKernelGGL(chunk_kernel, dim3(static_cast<unsigned>((nblk + kChunkBlocks - 1) / kChunkBlocks)),
                       dim3(kBlock), 0, s, ws, nblk);
  EventsDev none{};
  hipLaunchKernelGGL(scatter_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s, clips, nclips,
                     t, mode, ws, chunked, alpha, wl, wl ? count : nullptr, ev ? *ev : none, seg_b);
  return hipGetLastError();
}

hipError_t launch_list_events(const ClipDev* clips, int nclips, int t, const int64_t* worklist,
                              const int32_t* count, int64_t max_items, const float* dl,
                              const float* alpha, const float* beta, int64_t n_out,
                              const Workspace& ws, const EventsDev& ev, hipStream_t s) {
  int64_t blocks = (max_items + 255) / 256;
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(list_events_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, clips,
                     nclips, t, worklist, count, dl, alpha, beta, n_out, max_items, ws, ev);
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, ev.count, count);
  return hipGetLastError();
}

hipError_t launch_list_state(const ClipDev* clips, int nclips, int t, const int64_t* worklist,
                             const int32_t* count, int64_t max_items, const float* alpha,
                             const float* beta, int64_t n_out, hipStream_t s) {
  int64_t blocks = (max_items + 255) / 256;
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(list_state_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, clips, nclips,
                     t, worklist, count, alpha, beta, n_out, max_items);
  return hipGetLastError();
}

hipError_t launch_init(const ClipDev* clips, int nclips, int64_t nblk, int t, const float* alpha,
                       const float* beta, int64_t n_out, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s, clips, nclips, t,
                     alpha, beta, n_out);
  return hipGetLastError();
}

}  // namespace esim
