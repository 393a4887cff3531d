// Launchers of the threshold / compaction / event kernels.
#pragma once

#include "esim_internal.h"

namespace esim {

enum { kFlagThreshold = 0, kFlagExhaustive = 1, kFlagRaw = 2 };

// Clip of kBlock-pixel block b of a flag/scatter grid.
__device__ __forceinline__ int block_clip(const ClipDev* clips, int nclips, int64_t b) {
  int cl = 0;
  for (int c = 1; c < nclips; ++c)
    if (clips[c].blk_off <= b) cl = c;
  return cl;
}

// Device view of an esim_events_buf.
struct EventsDev {
  int32_t* x;
  int32_t* y;
  int32_t* t;
  int8_t* p;
  int32_t* clip;
  int64_t capacity;
  int64_t* count;
  float* ts;
};

hipError_t launch_log(const float* E, float* y, int64_t n, float eps, hipStream_t s);

// Grids of at most this many blocks skip the chunk kernel: each scatter block
// sums the counts before it (at most 16 KiB of reads); larger grids sum chunk
// totals and the counts inside their chunk.
constexpr int64_t kDirectPrefixBlocks = 4096;

// flag -> (scan) -> scatter.  mode kFlagThreshold writes the work list and
// count (count[0] = count[1] = flagged pixels), and with ev also appends the
// flagged pixels' events (the sign of the threshold's change); the other
// modes append events to ev.
// Split work list (kFlagThreshold, seg_b >= 0): the items of clips with
// list_class 0 go to worklist[0, nA) and those of list_class 1 to
// worklist[seg_b, seg_b + nB), each segment in ascending (clip, p) order;
// count[0] = count[1] = nA, count[2] = count[3] = nB (count holds four).
// The events keep their order, (clip, p) ascending over all clips.
hipError_t launch_flag_compact(const ClipDev* clips, int nclips, int64_t nblk, int t, int mode,
                               float* dl, const float* alpha, const Workspace& ws, int64_t* worklist,
                               int32_t* count, const EventsDev* ev, hipStream_t s, int64_t seg_b = -1);

// The compaction after a flag kernel that has already filled ws (chunk totals
// when needed, then the scatter), as in launch_flag_compact (no split).
hipError_t launch_scatter(const ClipDev* clips, int nclips, int64_t nblk, int t, int mode,
                          const float* alpha, const Workspace& ws, int64_t* worklist, int32_t* count,
                          const EventsDev* ev, hipStream_t s, int64_t seg_b = -1);

// State <- the models of the work-list items (alpha[i], beta[.., i]), feat_t
// and t, without events (the step's explicit-threshold path).
hipError_t launch_list_state(const ClipDev* clips, int nclips, int t, const int64_t* worklist,
                             const int32_t* count, int64_t max_items, const float* alpha,
                             const float* beta, int64_t n_out, hipStream_t s);

hipError_t launch_list_events(const ClipDev* clips, int nclips, int t, const int64_t* worklist,
                              const int32_t* count, int64_t max_items, const float* dl,
                              const float* alpha, const float* beta, int64_t n_out,
                              const Workspace& ws, const EventsDev& ev, hipStream_t s);

hipError_t launch_init(const ClipDev* clips, int nclips, int64_t nblk, int t, const float* alpha,
                       const float* beta, int64_t n_out, hipStream_t s);

}  // namespace esim
