// Workspace plan: offsets of every device buffer for n points in H hulls (host).
#include <algorithm>

#include "common.hpp"

namespace hull {

static thread_local int32_t g_last_hip_error = 0;

void note_hip_error(hipError_t e) { g_last_hip_error = (int32_t)e; }

static int64_t scan_tiles(int64_t len) { return (len + kScanBlock - 1) / kScanBlock; }

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Plan make_plan(int64_t n, int64_t H, int min_seg, int pt_bytes) {
  Plan p{};
  const int64_t nn = n > 0 ? n : 1;
  const int64_t hh = H > 0 ? H : 1;
  p.n = n;
  p.H = H;
  p.tiles = (nn + kTile - 1) / kTile;
  p.count_len = p.tiles * kBuckets;
  // merges of one level: sum over hulls of floor(ceil(n_h / w) / 2) <= n / 2
  p.mcap = nn / 2 + 1;
  // walk segments of one level: sum over merges of 1 + events / G, events <= 2n
  p.seg_cap = p.mcap + (2 * nn) / std::max(min_seg, 1) + 1;
  int64_t longest = std::max<int64_t>({p.count_len, 2 * nn + 1, p.seg_cap + 1, hh + 1});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  p.header = take(sizeof(Header));
  p.chain_stride = scan_tiles(longest) + 1;
  p.chain_words = take(kChainJobs * p.chain_stride * sizeof(unsigned long long));
  p.pts = take(nn * (size_t)pt_bytes);
  p.off1 = take(2 * sizeof(int64_t));
  p.mcnt = take((hh + 1) * 4);
  p.moff = take((hh + 1) * 4);
  p.tcnt = take((hh + 1) * 4);
  p.toff = take((hh + 1) * 4);
  p.tlist = take(hh * 4);
  p.mlist = take(p.mcap * sizeof(int2));
  for (int r = 0; r < 2; ++r) {
    p.perm[r] = take(p.mcap * 4);
    p.wbins[r] = take(kWorkBins * 4);
  }
  p.fcnt = take((hh + 1) * 4);
  for (int r = 0; r < 2; ++r) {
    p.pv0[r] = take(nn * 4);
    p.nx0[r] = take(nn * 4);
    p.lk[r] = take(nn * sizeof(int2));
    for (int b = 0; b < 2; ++b) {
      p.ev[r][b] = take(2 * nn * sizeof(Event));
      p.len[r][b] = take(nn * 4);
    }
    p.cntR[r] = take(nn * 4);
    p.cntL[r] = take(nn * 4);
    p.offR[r] = take(nn * 4);
    p.offL[r] = take(nn * 4);
    p.curR[r] = take(nn * 4);
    p.curL[r] = take(nn * 4);
    p.claimR[r] = take(nn * 4);
    p.claimL[r] = take(nn * 4);
    p.entR[r] = take(3 * nn * sizeof(Entry));
    if (r == 0) {
      // the sort's buffers live only until the points are gathered, before
      // any merge: they share run 0's entry lists (48 bytes per point)
      size_t o = p.entR[0];
      auto sub = [&](size_t bytes) {
        size_t q = o;
        o = align256(o + bytes);
        return q;
      };
      p.keys0 = sub(nn * 4);
      p.vals0 = sub(nn * 4);
      p.keys1 = sub(nn * 4);
      p.vals1 = sub(nn * 4);
      p.hid = sub(nn * 4);
      p.counts = sub(p.count_len * 4);
      static_assert(3 * sizeof(Entry) >= 20, "sort buffers must fit in the entry lists");
    }
    p.entL[r] = take(3 * nn * sizeof(Entry));
    p.ctr[r] = take(kCtrSlots * sizeof(int32_t));
    p.touched[r] = take(2 * nn * 4);
    p.ecnt[r] = take((p.mcap + 1) * 4);
    p.eoff[r] = take((p.mcap + 1) * 4);
    p.cslot[r] = take(2 * nn * 4);
    p.cmerge[r] = take(2 * nn * 4);
    p.segS[r] = take((p.mcap + 1) * 4);
    p.segBase[r] = take((p.mcap + 1) * 4);
    p.segMerge[r] = take((p.seg_cap + 1) * 4);
    p.segB[r] = take((p.seg_cap + 1) * 4);
    p.segCnt[r] = take((p.seg_cap + 1) * 4);
    p.segOff[r] = take((p.seg_cap + 1) * 4);
    p.segUV[r] = take((p.seg_cap + 1) * sizeof(int2));
    p.segTmp[r] = take((p.seg_cap + 1) * kSegKeep * sizeof(Event));
    p.segTmpUV[r] = take((p.seg_cap + 1) * kSegKeep * sizeof(int2));
    p.bev[r] = take(2 * nn * sizeof(Event));
    p.buv[r] = take(2 * nn * sizeof(int2));
    p.nB[r] = take((p.mcap + 1) * 4);
    p.boff[r] = take((p.mcap + 1) * 4);
    p.uv0[r] = take(p.mcap * sizeof(int2));
    p.aR[r] = take((2 * nn + 1) * 4);
    p.aL[r] = take((2 * nn + 1) * 4);
    p.aT[r] = take((2 * nn + 1) * 4);
    // per-event survival flags and prefix sums are written after the list
    // allocation counts are last read (place, before the walk): same space
    p.surv[r] = p.aR[r];
    p.jb[r] = p.aL[r];
    p.pre[r] = p.aT[r];
    p.wf[r] = take(2 * nn);
  }
  p.total = off;
  return p;
}

}  // namespace hull

extern "C" int32_t hull_last_hip_error(void) { return hull::g_last_hip_error; }
