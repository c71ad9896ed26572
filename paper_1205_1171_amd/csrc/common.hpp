// Shared declarations of the hull library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hull3d.h"

namespace hull {

constexpr int kNil = -1;
constexpr int64_t kMaxN = int64_t(1) << 26;      // points of one hull
// points of a batch: the workspace of 2^28 points (about 924 bytes per
// point) still fits the 288 GB of one MI355X
constexpr int64_t kMaxTotal = int64_t(1) << 28;
constexpr int32_t kMaxCoord = 1 << 29;
constexpr int64_t kMaxWideXY = int64_t(1) << 30;  // wide range: |x|, |y|
constexpr int64_t kMaxWideZ = int64_t(1) << 42;   // wide range: |z|
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortThreads * kSortItems;  // keys per radix tile
constexpr int kRadixBits = 8;
constexpr int kBuckets = 1 << kRadixBits;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kSortThreads * kScanItems;
constexpr int kStrideBlocks = 1024;  // grid of the grid-stride kernels
constexpr int kScanDevGrid = 128;    // tile blocks per job of a device-length scan
constexpr int kSegKeep = 4;  // bridge events a walk segment keeps from its counting pass
constexpr int kMinWalkSegment = 4;  // fewest child events per walk segment
constexpr int kWorkBins = 1024;     // child-event counts told apart when ordering merges

// Slots of the per-run counter region of the parallel merge strategy.
constexpr int kCtrTouched = 2;   // per-point link-change lists allocated this level
constexpr int kCtrMerges = 4;    // merges of the level
constexpr int kCtrEvents = 5;    // child events of the level
constexpr int kCtrSegments = 6;  // walk segments of the level
constexpr int kCtrBridge = 7;    // bridge events of the level
constexpr int kCtrSlots = 8;     // size of the region (int32 words)
static_assert(kCtrBridge < kCtrSlots, "counter region too small");

// Device-side status words at the head of every workspace.
struct Header {
  int32_t err;      // first error seen on the device (HULL_* code), 0 = none
  int32_t minx;     // minimum x (sort key origin)
  int32_t maxx;     // maximum x
  int32_t nbits;    // bits of (maxx - minx): radix passes actually needed
  int32_t pad[60];  // keeps the header one 256-byte line
};

// One movie event: the face (a, w, b) of ranks a < w < b whose middle vertex w
// enters (kind = 1) or leaves (kind = 0) the kinetic chain, and the standard
// part of its time rounded to float.  One 16-byte record (one vector load);
// the kind is the top bit of the middle rank (ranks are below 2^29).
struct __align__(16) Event {
  int a;
  int wk;  // w | kind << 31
  int b;
  float t;  // NaN: not covered by the filter
  __host__ __device__ int w() const { return wk & 0x7fffffff; }
  __host__ __device__ int kind() const { return (int)((unsigned)wk >> 31); }
};

__host__ __device__ inline Event make_event(int a, int w, int b, int kind, double t) {
  Event e;
  e.a = a;
  e.wk = (int)((unsigned)w | ((unsigned)kind << 31));
  e.b = b;
  e.t = (float)t;
  return e;
}

// A link-change list entry of the parallel merge strategy: the child event's
// (a, w | kind << 31, b) and a key that is first the event's slot in the input
// movies (the list's sort key: a movie is in time order) and, once the list
// is sorted, the bits of its time (the fields of an Event).
struct __align__(16) Entry {
  int a;
  int wk;
  int b;
  int key;
  __host__ __device__ int w() const { return wk & 0x7fffffff; }
  __host__ __device__ int kind() const { return (int)((unsigned)wk >> 31); }
};

// Offsets (bytes) of every workspace region for n points in H hulls.
struct Plan {
  size_t header, keys0, vals0, keys1, vals1, counts, pts, hid, off1;
  size_t pv0[2], nx0[2], lk[2];
  size_t ev[2][2], len[2][2];  // [run][buffer]
  // the level schedule (merge list, trailing blocks)
  size_t mcnt, moff, tcnt, toff, tlist, mlist;
  size_t perm[2], wbins[2];  // per run: merges in work order, work histogram
  // parallel merge strategy, per run
  size_t cntR[2], cntL[2], offR[2], offL[2], curR[2], curL[2], claimR[2], claimL[2];
  size_t entR[2], entL[2], ctr[2], touched[2];
  size_t ecnt[2], eoff[2], cslot[2], cmerge[2];
  size_t segS[2], segBase[2], segMerge[2], segB[2], segCnt[2], segOff[2], segUV[2];
  size_t segTmp[2], segTmpUV[2];  // the first kSegKeep bridge events of each segment
  size_t bev[2], buv[2], nB[2], boff[2], uv0[2], surv[2], jb[2], pre[2];
  size_t aR[2], aL[2], aT[2], wf[2];
  // status words of the parallel strategy's one-launch scans (kChainJobs x chain_stride)
  size_t chain_words;
  int64_t chain_stride;
  // face counts of the hulls of a batch
  size_t fcnt;
  size_t total;
  int64_t n, H, tiles, count_len, mcap, seg_cap;
};

// min_seg: the smallest walk segment (child events) the plan must hold;
// pt_bytes: size of a point by rank (16: int4, standard range; 32: WPt, wide).
Plan make_plan(int64_t n, int64_t H, int min_seg = kMinWalkSegment, int pt_bytes = 16);

// The HIP error behind the last HULL_EHIP of this host thread.
void note_hip_error(hipError_t e);

#define HULL_LAUNCH_CHECK()                         \
  do {                                              \
    hipError_t e_ = hipGetLastError();              \
    if (e_ != hipSuccess) {                         \
      ::hull::note_hip_error(e_);                   \
      return HULL_EHIP;                             \
    }                                               \
  } while (0)

// Entry of every call that launches: an error left pending by earlier,
// unrelated HIP calls of this thread is cleared, so that the launch checks
// see the call's own launches only.
inline void clear_stale_hip_error() { (void)hipGetLastError(); }

// One hull (lower and/or upper run) of n points: sort, every merge level,
// faces (the body of hull_lower / hull_full).  int32 rows: the standard
// range; int64 rows: the wide range (hull_full_wide and friends).
int32_t hull_runs(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, hipStream_t s, bool lower, bool upper,
                  void* const* events, int32_t nevents);
int32_t hull_runs(const int64_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, hipStream_t s, bool lower, bool upper,
                  void* const* events, int32_t nevents);

// Workspace bytes of the wide-range entry points (int64 rows) and of the
// float entry points (the wide hull plus the snapped rows), for n points.
size_t wide_workspace_bytes(int64_t n);
size_t f32_workspace_bytes(int64_t n);

// Clear the device status words (a kernel, so that the call can be captured).
void init_header(Header* h, hipStream_t s);

// Sort: ranks by (hull, x, index within the hull).  Fills pts (PT: int4 x, y,
// z, index within the hull from int32 rows; WPt from int64 rows, by rank).
// hull_off (device [H + 1]) may be NULL for a single hull.
template <class InT, class PT>
int32_t sort_points(const InT* d_xyz, int64_t n, const int64_t* hull_off, int64_t H, char* ws,
                    const Plan& pl, hipStream_t s);

// Exclusive scans of int32 (in place allowed), each in one launch (a chained
// scan): up to kMaxScanJobs arrays of the same add and cap, each of a length
// read from device memory (len = *d_len + add, never more than cap; a null
// d_len: cap itself).  Job j publishes one status word per tile at words +
// j * wstride (wstride >= cap / 4096 rounded up); epoch (1 .. 2^30 - 1) tells
// this scan's words from those of earlier scans that used the same words,
// which must hold zero or another epoch.
constexpr int kMaxScanJobs = 8;
constexpr int kChainJobs = 16;  // job slots of the status words (a parallel level's scans)
struct ScanJob {
  const int32_t* in;
  int32_t* out;
  const int32_t* d_len;
  int32_t* total;  // if set: receives the sum of the scanned entries (the scan's total)
};
struct ScanJobs {
  ScanJob j[kMaxScanJobs];
  int count;
};
int32_t exclusive_scan_chained(const ScanJobs& J, int add, int64_t cap, unsigned long long* words,
                               int64_t wstride, unsigned epoch, Header* h, hipStream_t s);
// One array of host-known length (slot 0 of the words).
int32_t scan_chained_i32(const int32_t* in, int32_t* out, int64_t len, unsigned long long* words,
                         int64_t wstride, unsigned epoch, Header* h, hipStream_t s);
// Epochs of the one-launch scans of a call: the sort's passes 1..8, level k's
// scans 8k + 1..7, the face offsets kChainEpochFaces.  The sort clears the
// words at the start of every call.
constexpr unsigned kChainEpochFaces = 8 * 28 + 1;
// Zero count 64-bit words (a kernel: capturable).
void zero_words(unsigned long long* w, int64_t count, hipStream_t s);

}  // namespace hull
