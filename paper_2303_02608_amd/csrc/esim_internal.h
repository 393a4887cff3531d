// Internal declarations of libesim (device descriptors, load helpers,
// cross-lane reductions and the launchers each source file provides).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "esim.h"

namespace esim {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // threads of flag/scatter blocks
constexpr int kWavesPerBlock = kBlock / kWave;

// Device descriptor of one clip of a plan.
struct ClipDev {
  const float* y;          // [T][H][W]
  const void* feat;        // [T][F][H][W]
  float* st_alpha;         // [HW]
  float* st_beta;          // [F][HW]
  float* st_xref;          // [F][HW]
  int32_t* st_tref;        // [HW]
  float* st_last;          // [HW] previous frame's compared value (multi-crossing)
  int32_t W, H, T, F;
  int32_t feat_f16, r, tr, precision;
  int32_t multi;           // every-crossing event rule in the exhaustive/raw modes
  int64_t HW;
  int64_t pix_off;         // first pixel in the concatenated pixel range
  int64_t blk_off;         // first kBlock-pixel block of the flag/scatter grid
  int64_t nblk;            // kBlock-pixel blocks of this clip
  int64_t grp_off[5];      // first dense wave-group, per lanes-per-item 1,2,4,8,16
  double C, h, ridge, kappa_fp64;
  double c2[ESIM_MAX_D];   // 1 / (h b_j)^2
  double sf[ESIM_MAX_D];   // 1 / (h b_j)
  double gbk[ESIM_MAX_D];  // 1 / (h^2 b_j^3)
  float* st_bxy;           // [2][HW] coordinate components of beta (nullable)
  float* st_rmom;          // [2][HW] R and mean residual of the stored plane (nullable)
  int32_t thr;             // esim_threshold
  double dt;               // time between frames (event times t * dt)
  int32_t list_class;      // 1: esim_step's split work list puts this clip's items in its second
                           // segment (windows wider than 16 columns), 0 otherwise
};

// Shape of the device a plan runs on, queried once when the plan is created:
// compute units and the XCDs (L2 domains) they are grouped in.  Workgroups are
// dispatched to the XCDs round-robin by block index.
struct DeviceShape {
  int cus = 1;
  int xcds = 1;
};
constexpr int kMaxXcds = 32;
// The current device's shape (hipDeviceAttributeMultiProcessorCount and
// hipDeviceAttributeNumberOfXccs); returns false if a query fails.
bool query_device_shape(DeviceShape& out);

// Compaction workspace of a plan (device).
struct Workspace {
  int64_t* bcount;         // [nblk] flagged pixels per block; a split compaction also adds the
                           // count times 2^32 for blocks of second-segment clips
  uint64_t* flags;         // [nblk][kWavesPerBlock] flag ballots
  uint64_t* pol;           // [nblk][kWavesPerBlock] positive-polarity ballots
  int64_t* misc;           // [4] [0] event base of the current step
  int64_t* chunk;          // [ceil(nblk / kChunkBlocks)] counts per chunk of blocks
};

constexpr int64_t kChunkBlocks = 1024;     // blocks per chunk of the two-level prefix

// Stored feature value f of pixel p at frame t (FP16 storage converted).
__device__ __forceinline__ float feat_value(const ClipDev& C, int t, int f, int64_t p) {
  const int64_t i = (static_cast<int64_t>(t) * C.F + f) * C.HW + p;
  if (C.feat_f16) {
    const uint16_t h = static_cast<const uint16_t*>(C.feat)[i];
    return static_cast<float>(__builtin_bit_cast(_Float16, h));
  }
  return static_cast<const float*>(C.feat)[i];
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint64_t bytes) {
  const uint32_t n = bytes >= 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(bytes);
  // Raw (stride 0) buffer; the third dword selects 32-bit data for the gfx9 family.
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                           static_cast<int>(n), 0x00020000);
}

__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ float ld_f16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
  return static_cast<float>(__builtin_bit_cast(_Float16, h));
}

template <bool F16>
__device__ __forceinline__ float ld_feat(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (F16) return ld_f16(r, voff, soff);
  else return ld_f32(r, voff, soff);
}

// Lane-group sum with DPP.  After dpp_sum<L>(v) every lane of each aligned
// group of L lanes (L in 1, 2, 4, 8, 16) holds the group's sum:
//   quad_perm [1,0,3,2] and [2,3,0,1] give quad sums; row_half_mirror maps
//   each quad onto the other quad of its half-row; row_mirror maps each
//   half-row onto the other half of its row.
// All lanes take part and every source lane of these controls lies inside the
// row, so no lane keeps an "old" value (bound_ctrl set, full masks).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b & 0xFFFFFFFFu), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                        static_cast<uint32_t>(lo));
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF,
                                                            0xF, true));
}

template <int L>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (L >= 2) v += dpp_d<0xB1>(v);
  if constexpr (L >= 4) v += dpp_d<0x4E>(v);
  if constexpr (L >= 8) v += dpp_d<0x141>(v);
  if constexpr (L >= 16) v += dpp_d<0x140>(v);
  return v;
}

template <int L>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (L >= 2) v += dpp_f<0xB1>(v);
  if constexpr (L >= 4) v += dpp_f<0x4E>(v);
  if constexpr (L >= 8) v += dpp_f<0x141>(v);
  if constexpr (L >= 16) v += dpp_f<0x140>(v);
  return v;
}

__host__ __device__ constexpr int lanes_index(int L) {
  return L == 1 ? 0 : L == 2 ? 1 : L == 4 ? 2 : L == 8 ? 3 : 4;
}

// Work item fields.
__device__ __forceinline__ int item_clip(int64_t it) { return static_cast<int>((it >> 32) & 0xFFF); }
__device__ __forceinline__ int64_t item_pixel(int64_t it) { return it & 0xFFFFFFFFll; }
__device__ __forceinline__ int item_frame(int64_t it) { return static_cast<int>(it >> 44); }

// ---- launchers (host) -----------------------------------------------------

struct RegressArgs {
  const ClipDev* clips;
  int32_t nclips;
  int32_t t;                // >= 0 uniform frame, < 0 frame from the item
  const int64_t* items;     // nullptr = dense
  const int32_t* count;
  int64_t n_dense_groups;   // dense: wave-groups over all clips (for the chosen L)
  int64_t max_groups;       // upper bound of groups (grid sizing)
  int64_t n_out;
  float* alpha;             // nullable when update_state is set
  float* beta;
  float* resid;
  float* kappa;
  int32_t update_state;     // write each item's model into its clip state (Sec. 2.2)
  const int64_t* xcd_bounds;  // dense multi-clip launches: [nxcd + 1] group bounds per XCD (device)
  int32_t nxcd;               // XCDs of the device (group-to-XCD mapping)
};

// Regression launcher: picks the kernel instance for (F, dtype, precision)
// and the lanes-per-item L; returns hipSuccess or the launch error.
using KernelFn = void (*)(RegressArgs);

// Regression kernels of one feature count: general [lanes 1, 2, 4, 8, 16][f16],
// one-pass [f16], compensated FP32 [lanes 4, 16][f16] (null where not compiled).
struct RegressTable {
  KernelFn general[5][2] = {};
  KernelFn onepass[2] = {};
  KernelFn c32[2][2] = {};
  KernelFn kappa[2] = {};      // FP64 Gram with the condition estimate, one lane per item
};

hipError_t launch_regress(const RegressArgs& a, int F, bool f16, int precision, int lanes,
                          int blocks_per_cu, int max_r, const DeviceShape& dev, hipStream_t s);
int regress_supported_lanes(int F);
bool regress_supports(int F, int lanes, int precision);

struct BackwardArgs {
  const ClipDev* clip;      // single clip (device)
  const ClipDev* host_clip; // the same, host copy
  const int64_t* items;
  int64_t n;
  const float* g_alpha;
  float* g_y;
  double* g_b;
  void* scratch;
  size_t scratch_bytes;
  DeviceShape dev;
};
size_t backward_scratch_bytes(const ClipDev& hc, int64_t n);
// LDS of the gather kernel's item buffer (records, centre features and
// positions of the items staged at a time, and the per-wave counts).
size_t backward_gather_lds_bytes(const ClipDev& hc);
constexpr size_t kMaxGatherLds = 65536;
hipError_t launch_backward(const BackwardArgs& a, hipStream_t s);

// Nearest same-polarity neighbour distances (event-set comparison).
struct NnArgs {
  const int32_t *sx, *sy, *st;  // source events
  const int8_t* sp;
  int64_t ns;
  const int32_t *qx, *qy, *qt;  // query events
  const int8_t* qp;
  int64_t nq;
  int W, H, T;
  double scale_x, scale_y, scale_t, rmax;
  int rx, ry, rt;               // lattice extents of rmax
  double* d;
  void* scratch;
};
size_t nn_scratch_bytes(int W, int H, int T);
hipError_t launch_nn(const NnArgs& a, hipStream_t s);
// Device address of the fixed bitmap array of esim_nn_distances_noalloc on
// the current device (ESIM_NN_STATIC_BYTES bytes), looked up on the first call
// per device; false if the lookup fails.
bool nn_static_scratch(void** out);

// Explicit Delta R threshold (dense over the plan's pixels at frame t): fills
// dl and the flag/polarity ballots and block counts of the compaction
// workspace, like the closed-form flag kernel.
hipError_t launch_explicit_flag(const ClipDev* clips, int nclips, int64_t nblk, int t, int F, bool f16,
                                int thr, float* dl, const Workspace& ws, const int64_t* ev_count,
                                hipStream_t s);
// Window sums (R, mean residual) of the stored planes of the pixels updated at
// frame t: the work-list items (worklist non-null, *count of them, at most
// max_items) or every pixel of the plan (dense, nblk kBlock-pixel blocks).
hipError_t launch_moments(const ClipDev* clips, int nclips, int64_t nblk, int t, int F, bool f16,
                          const int64_t* worklist, const int32_t* count, int64_t max_items,
                          hipStream_t s);

}  // namespace esim
