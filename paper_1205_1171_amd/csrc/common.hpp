// Shared declarations of the hull library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hull3d.h"

namespace hull {

constexpr int kNil = -1;
constexpr int64_t kMaxN = int64_t(1) << 26;
constexpr int32_t kMaxCoord = 1 << 29;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortThreads * kSortItems;  // keys per radix tile
constexpr int kRadixBits = 8;
constexpr int kBuckets = 1 << kRadixBits;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kSortThreads * kScanItems;

// Device-side status words at the head of every workspace.
struct Header {
  int32_t err;      // first error seen on the device (HULL_* code), 0 = none
  int32_t minx;     // minimum x (sort key origin)
  int32_t maxx;     // maximum x
  int32_t nbits;    // bits of (maxx - minx): radix passes actually needed
  int32_t pad[60];  // keeps the header one 256-byte line
};

// One movie event: the face (a, w, b) of ranks a < w < b whose middle vertex w
// enters (kind = 1) or leaves (kind = 0) the kinetic chain; the event time's
// standard part is kept beside it in a parallel double array.
struct Event {
  int a, w, b, kind;
};

// Offsets (bytes) of every workspace region for a single hull of n points.
struct Plan {
  size_t header, keys0, vals0, keys1, vals1, counts, partials, pts;
  size_t pv0[2], nx0[2], pv[2], nx[2];
  size_t ev[2][2], tau[2][2], len[2][2];  // [run][buffer]
  // parallel merge strategy, per run
  size_t cntR[2], cntL[2], offR[2], offL[2], curR[2], curL[2], entR[2], entL[2];
  size_t entRt[2], entLt[2], segS[2], segBase[2], segMerge[2], segCnt[2], segOff[2];
  size_t bev[2], btau[2], buv[2], nB[2], uv0[2], surv[2], jb[2], pre[2];
  size_t total;
  int64_t n, tiles, count_len, partial_len;
};

Plan make_plan(int64_t n);

inline int32_t hip_status(hipError_t e) { return e == hipSuccess ? HULL_OK : HULL_EHIP; }

#define HULL_LAUNCH_CHECK()                         \
  do {                                              \
    hipError_t e_ = hipGetLastError();              \
    if (e_ != hipSuccess) return HULL_EHIP;         \
  } while (0)

// Clear the device status words (a kernel, so that the call can be captured).
void init_header(Header* h, hipStream_t s);

// Sort: ranks by (x, input index).  Fills pts (int4 x, y, z, i by rank).
int32_t sort_points(const int32_t* d_xyz, int64_t n, char* ws, const Plan& pl, hipStream_t s);

// Exclusive scan of int32 counts (device, in place into `out`).
int32_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t len, int32_t* partials,
                           hipStream_t s);

// Runs for one hull: lower (run 0) and/or upper (run 1).
int32_t hull_runs(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, hipStream_t s, bool lower, bool upper,
                  void* const* events, int32_t nevents);

}  // namespace hull
