// Workspace plan: offsets of every device buffer of a single hull (host).
#include <algorithm>

#include "common.hpp"

namespace hull {

static int64_t scan_partials_needed(int64_t len) { return (len + kScanBlock - 1) / kScanBlock; }

// ---------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Plan make_plan(int64_t n) {
  Plan p{};
  int64_t nn = n > 0 ? n : 1;
  p.n = n;
  p.tiles = (nn + kTile - 1) / kTile;
  p.count_len = p.tiles * kBuckets;
  p.partial_len = std::max(scan_partials_needed(p.count_len), scan_partials_needed(2 * nn + 1)) + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  p.header = take(sizeof(Header));
  p.keys0 = take(nn * 4);
  p.vals0 = take(nn * 4);
  p.keys1 = take(nn * 4);
  p.vals1 = take(nn * 4);
  p.counts = take(p.count_len * 4);
  p.partials = take(p.partial_len * 4);
  p.pts = take(nn * sizeof(int4));
  for (int r = 0; r < 2; ++r) {
    p.pv0[r] = take(nn * 4);
    p.nx0[r] = take(nn * 4);
    p.pv[r] = take(nn * 4);
    p.nx[r] = take(nn * 4);
    for (int b = 0; b < 2; ++b) {
      p.ev[r][b] = take(2 * nn * sizeof(Event));
      p.tau[r][b] = take(2 * nn * sizeof(double));
      p.len[r][b] = take(nn * 4);
    }
    p.cntR[r] = take(nn * 4);
    p.cntL[r] = take(nn * 4);
    p.offR[r] = take(nn * 4);
    p.offL[r] = take(nn * 4);
    p.curR[r] = take(nn * 4);
    p.curL[r] = take(nn * 4);
    p.entR[r] = take(4 * nn * sizeof(Event));
    p.entL[r] = take(4 * nn * sizeof(Event));
    p.entRt[r] = take(4 * nn * sizeof(double));
    p.entLt[r] = take(4 * nn * sizeof(double));
    p.segS[r] = take((nn + 2) * 4);
    p.segBase[r] = take((nn + 2) * 4);
    p.segMerge[r] = take((nn + 2) * 4);
    p.segCnt[r] = take((nn + 2) * 4);
    p.segOff[r] = take((nn + 2) * 4);
    p.bev[r] = take(2 * nn * sizeof(Event));
    p.btau[r] = take(2 * nn * sizeof(double));
    p.buv[r] = take(2 * nn * sizeof(int2));
    p.nB[r] = take(nn * 4);
    p.uv0[r] = take(nn * sizeof(int2));
    p.surv[r] = take((2 * nn + 1) * 4);
    p.jb[r] = take(2 * nn * 4);
    p.pre[r] = take((2 * nn + 1) * 4);
  }
  p.total = off;
  return p;
}

}  // namespace hull
