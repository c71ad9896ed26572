// Events of a movie as comparison candidates, and their exact order.
#pragma once
#include "common.hpp"
#include "predicates.hpp"

namespace hull {

struct Cand {
  Tri t;
  double st;  // standard part of tau (NaN: not covered by the fast path)
  int kind;   // 1 insertion, 0 deletion
};

// Pointers of one run (lower or upper) for the lane-serial merge strategy.
// pts: the points by rank, int4 (x, y, z, w) on the standard range or WPt on
// the wide range (the kernels are instantiated for each).
struct RunPtrs {
  const void* pts;
  int* pv0;
  int* nx0;
  int2* lk;  // working links of the level: (pv, nx) of each point
  const Event* ev_in;
  const int* len_in;
  Event* ev_out;
  int* len_out;
  int zs;
};

// Working links (pv, nx) of a merge's points, in one of three places.  The
// merge kernels read and write them only through get / set_pv / set_nx /
// set, so one merge loop serves all three.
//
// In global memory: one int2 per point, indexed like the point array.
struct GlobalLinks {
  int2* p;
  __device__ __forceinline__ int2 get(int i) const { return p[i]; }
  __device__ __forceinline__ void set_pv(int i, int v) const { p[i].x = v; }
  __device__ __forceinline__ void set_nx(int i, int v) const { p[i].y = v; }
  __device__ __forceinline__ void set(int i, int pv, int nx) const { p[i] = make_int2(pv, nx); }
};

// In LDS, as block-local ranks (kNil stays -1) in a narrow signed type: one
// lane's merge of up to kLinkLdsLane points in int8, a lane group's merge in
// int16 while the block's groups need at most kLinkLdsGroupBytes.  Entry i
// sits at p[i * STRIDE] (STRIDE 64: the entries of a wave's 64 lanes
// interleaved, so that a wave-wide access spans consecutive banks).  Indices
// and link values are block-local.
constexpr int kLinkLdsLane = 128;
constexpr int kLinkLdsGroupBytes = 32768;
template <class T>
struct __align__(2 * sizeof(T)) LinkPair {
  T pv, nx;
};
template <class T, int STRIDE>
struct LdsLinks {
  LinkPair<T>* p;
  __device__ __forceinline__ int2 get(int i) const {
    const LinkPair<T> e = p[i * STRIDE];
    return make_int2(e.pv, e.nx);
  }
  __device__ __forceinline__ void set_pv(int i, int v) const { p[i * STRIDE].pv = (T)v; }
  __device__ __forceinline__ void set_nx(int i, int v) const { p[i * STRIDE].nx = (T)v; }
  __device__ __forceinline__ void set(int i, int pv, int nx) const {
    LinkPair<T> e;
    e.pv = (T)pv;
    e.nx = (T)nx;
    p[i * STRIDE] = e;
  }
};

// In LDS as above, for a merge loop that works in global ranks: indices and
// link values are shifted by the block start on the way in and out.
template <class T>
struct LdsLinksShifted {
  LinkPair<T>* p;
  int base;
  __device__ __forceinline__ int2 get(int i) const {
    const LinkPair<T> e = p[i - base];
    return make_int2(e.pv < 0 ? kNil : e.pv + base, e.nx < 0 ? kNil : e.nx + base);
  }
  __device__ __forceinline__ void set_pv(int i, int v) const {
    p[i - base].pv = (T)(v == kNil ? -1 : v - base);
  }
  __device__ __forceinline__ void set_nx(int i, int v) const {
    p[i - base].nx = (T)(v == kNil ? -1 : v - base);
  }
  __device__ __forceinline__ void set(int i, int pv, int nx) const {
    LinkPair<T> e;
    e.pv = (T)(pv == kNil ? -1 : pv - base);
    e.nx = (T)(nx == kNil ? -1 : nx - base);
    p[i - base] = e;
  }
};

// The hulls of a call (rank offsets) and the level schedule built for every
// level on the device: the merges (pairs of adjacent blocks inside a hull)
// and the unpaired trailing blocks that are copied across.
struct Sched {
  const int64_t* off;  // [H + 1] rank offsets of the hulls
  int64_t H;
  int* moff;           // [H + 1] merges before each hull; moff[H] = merges of the level
  int2* mlist;         // [mcap] (s, e) of each merge, m = s + half
  int* toff;           // [H + 1] trailing blocks before each hull; toff[H] = their count
  int* tlist;          // [H] trailing block starts
  int64_t mcap;
};

struct LevelArgs {
  RunPtrs run[2];
  int* perm[2];   // per run: merge of each lane (nullptr: lane g takes merge g)
  int* wbins[2];  // per run: histogram, then cursors, of the work order
  Header* h;
  Sched S;
  int64_t n;
  int64_t half;   // size of a left block
  int64_t width;  // size of a merged block
};
// Exact (time, rank triple) order of two events (cold path).  Arguments
// go by value so that callers keep their candidates in registers.
template <class PT>
__device__ __noinline__ int tri_cmp_exact(const PT* pts, Tri A, Tri B, int zs) {
  Coef ca, cb;
  coef_of(pts[A.a], pts[A.w], pts[A.b], zs, ca);
  coef_of(pts[B.a], pts[B.w], pts[B.b], zs, cb);
  int s = tau_cmp_exact(ca, cb);
  if (s) return s;
  if (A.a != B.a) return A.a < B.a ? -1 : 1;
  if (A.w != B.w) return A.w < B.w ? -1 : 1;
  if (A.b != B.b) return A.b < B.b ? -1 : 1;
  return 0;
}

// Leading terms of D and N of a triple, exact in int64: D0, N0 (the
// unperturbed orientations) and D1, N1 (their e1 coefficients).
struct Lead {
  int64_t d0, n0, d1, n1;
};

__device__ __forceinline__ Lead lead_of(int4 P, int4 Q, int4 R, int zs) {
  const int dx1 = dif32(Q.x, P.x), dx2 = dif32(R.x, P.x);
  const int dy1 = dif32(Q.y, P.y), dy2 = dif32(R.y, P.y);
  const int dz1 = dif32(Q.z, P.z), dz2 = dif32(R.z, P.z);
  const int di1 = Q.w - P.w, di2 = R.w - P.w;
  Lead L;
  L.d0 = mul32(dx1, dy2) - mul32(dx2, dy1);
  L.n0 = zs * (mul32(dx1, dz2) - mul32(dx2, dz1));
  L.d1 = mul32(di1, dy2) - mul32(di2, dy1);
  L.n1 = zs * (mul32(di1, dz2) - mul32(di2, dz1));
  return L;
}

// Exact order when the double filter cannot decide.  The first three
// coefficients of N_A D_B - N_B D_A (monomials 1, e1, e1^2) fit int128:
//   N0a D0b - N0b D0a,  N0a D1b + N1a D0b - N0b D1a - N1b D0a,  N1a D1b - N1b D1a.
// They decide every tie of the standard parts that comes from a pair of
// points with equal x (all triples on such a pair share a standard part),
// with no 256-bit arithmetic; only when all three vanish (or D0 = D1 = 0)
// does the full cascade run.
// Sign of tau_A - tau_B from coefficients 1-3 of both leading terms; 0 when
// they do not decide (all three vanish, or D0 = D1 = 0 on a side).
__device__ __forceinline__ int lead_cmp(const Lead& a, const Lead& b) {
  const int sa = a.d0 ? (a.d0 > 0 ? 1 : -1) : (a.d1 > 0) - (a.d1 < 0);
  const int sb = b.d0 ? (b.d0 > 0 ? 1 : -1) : (b.d1 > 0) - (b.d1 < 0);
  if (sa && sb) {
    i128 p = (i128)a.n0 * b.d0 - (i128)b.n0 * a.d0;
    if (!p) {
      p = (i128)a.n0 * b.d1 + (i128)a.n1 * b.d0 - (i128)b.n0 * a.d1 - (i128)b.n1 * a.d0;
      if (!p) p = (i128)a.n1 * b.d1 - (i128)b.n1 * a.d1;
    }
    if (p) return (p > 0 ? 1 : -1) * sa * sb;
  }
  return 0;
}

__device__ __forceinline__ int tri_cmp_mid_body(const int4* pts, Tri A, Tri B, int zs) {
  const int s = lead_cmp(lead_of(pts[A.a], pts[A.w], pts[A.b], zs),
                         lead_of(pts[B.a], pts[B.w], pts[B.b], zs));
  return s ? s : tri_cmp_exact(pts, A, B, zs);
}

// The same on the wide range, where D0, N0, D1, N1 need int128 and their
// products may not fit it (N0 D0 up to 2^138): the three coefficients are
// taken in int128 when every leading term's bit length leaves the products
// below 2^124 (so that no sum of four overflows), which covers, for
// instance, all lifted points of |x|, |y| <= 2^20 (N up to 2^70, D up to
// 2^48); otherwise the full cascade decides.
struct WLead {
  i128 d0, n0, d1, n1;
};

__device__ __forceinline__ WLead lead_of(const WPt& P, const WPt& Q, const WPt& R, int zs) {
  const int64_t dx1 = (int64_t)Q.x - P.x, dx2 = (int64_t)R.x - P.x;
  const int64_t dy1 = (int64_t)Q.y - P.y, dy2 = (int64_t)R.y - P.y;
  const int64_t dz1 = Q.z - P.z, dz2 = R.z - P.z;
  const int64_t di1 = Q.w - P.w, di2 = R.w - P.w;
  WLead L;
  L.d0 = (i128)dx1 * dy2 - (i128)dx2 * dy1;
  L.n0 = zs * ((i128)dx1 * dz2 - (i128)dx2 * dz1);
  L.d1 = (i128)di1 * dy2 - (i128)di2 * dy1;
  L.n1 = zs * ((i128)di1 * dz2 - (i128)di2 * dz1);
  return L;
}

__device__ __forceinline__ int bits128(i128 v) {
  const u128 u = v < 0 ? (u128)(-v) : (u128)v;
  const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
  return hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
}

__device__ __forceinline__ int lead_cmp(const WLead& a, const WLead& b) {
  const int sa = a.d0 ? (a.d0 > 0 ? 1 : -1) : (a.d1 > 0) - (a.d1 < 0);
  const int sb = b.d0 ? (b.d0 > 0 ? 1 : -1) : (b.d1 > 0) - (b.d1 < 0);
  const int mn = max(max(bits128(a.n0), bits128(a.n1)), max(bits128(b.n0), bits128(b.n1)));
  const int md = max(max(bits128(a.d0), bits128(a.d1)), max(bits128(b.d0), bits128(b.d1)));
  if (sa && sb && mn + md <= 124) {
    i128 p = a.n0 * b.d0 - b.n0 * a.d0;
    if (!p) {
      p = a.n0 * b.d1 + a.n1 * b.d0 - b.n0 * a.d1 - b.n1 * a.d0;
      if (!p) p = a.n1 * b.d1 - b.n1 * a.d1;
    }
    if (p) return (p > 0 ? 1 : -1) * sa * sb;
  }
  return 0;
}

__device__ __forceinline__ int tri_cmp_mid_body(const WPt* pts, Tri A, Tri B, int zs) {
  const int s = lead_cmp(lead_of(pts[A.a], pts[A.w], pts[A.b], zs),
                         lead_of(pts[B.a], pts[B.w], pts[B.b], zs));
  return s ? s : tri_cmp_exact(pts, A, B, zs);
}

// The mid tier as a call (kernels with many live registers) ...
template <class PT>
__device__ __noinline__ int tri_cmp_mid(const PT* pts, Tri A, Tri B, int zs) {
  return tri_cmp_mid_body(pts, A, B, zs);
}

// Order of two events: 0 for the same triple, else the standard-part filter,
// then the mid tier (inlined with kInlineMid: the lane-serial merge, where
// exact standard-part ties are frequent and a call costs more than the
// registers).
template <bool kInlineMid = false, class PT>
__device__ __forceinline__ int ev_cmp(const PT* pts, const Cand& A, const Cand& B, int zs) {
  if (A.t.a == B.t.a && A.t.w == B.t.w && A.t.b == B.t.b) return 0;
  int s = std_cmp(A.st, B.st);
  if (s) return s;
  return kInlineMid ? tri_cmp_mid_body(pts, A.t, B.t, zs) : tri_cmp_mid(pts, A.t, B.t, zs);
}

// The same order for callers that hold both triples' points (A's as a0, a1,
// a2 and B's as b0, b1, b2, in rank order): the mid tier then needs no loads
// and no call; only the full cascade (rare) reloads them.
template <class PT>
__device__ __forceinline__ int ev_cmp_pts(const PT* pts, const Cand& A, const PT& a0, const PT& a1,
                                          const PT& a2, const Cand& B, const PT& b0, const PT& b1,
                                          const PT& b2, int zs) {
  if (A.t.a == B.t.a && A.t.w == B.t.w && A.t.b == B.t.b) return 0;
  const int s = std_cmp(A.st, B.st);
  if (s) return s;
  const int m = lead_cmp(lead_of(a0, a1, a2, zs), lead_of(b0, b1, b2, zs));
  return m ? m : tri_cmp_exact(pts, A.t, B.t, zs);
}

// The same for a candidate A whose points the caller holds (a0, a1, a2) against
// an event B: a tie loads only B's points.
template <class PT>
__device__ __forceinline__ int ev_cmp_half(const PT* pts, const Cand& A, const PT& a0, const PT& a1,
                                           const PT& a2, const Cand& B, int zs) {
  if (A.t.a == B.t.a && A.t.w == B.t.w && A.t.b == B.t.b) return 0;
  const int s = std_cmp(A.st, B.st);
  if (s) return s;
  const int m = lead_cmp(lead_of(a0, a1, a2, zs), lead_of(pts[B.t.a], pts[B.t.w], pts[B.t.b], zs));
  return m ? m : tri_cmp_exact(pts, A.t, B.t, zs);
}

// Perturbed sign of D when D0 = D1 = 0 (cold path).
template <class PT>
__device__ __noinline__ int d_sign_slow(PT P, PT Q, PT R) {
  Coef c;
  coef_of(P, Q, R, 1, c);
  return c.dsign;
}

// Perturbed sign of D(a, b, c) (xy orientation).
__device__ __forceinline__ int d_sign(int4 P, int4 Q, int4 R) {
  const int dy1 = dif32(Q.y, P.y), dy2 = dif32(R.y, P.y);
  const int64_t D0 = mul32(dif32(Q.x, P.x), dy2) - mul32(dif32(R.x, P.x), dy1);
  if (D0) return D0 > 0 ? 1 : -1;
  const int64_t D1 = mul32(Q.w - P.w, dy2) - mul32(R.w - P.w, dy1);
  if (D1) return D1 > 0 ? 1 : -1;
  return d_sign_slow(P, Q, R);
}

// The same on the wide range (D0 up to 2^63: int128; D1 up to 2^58).
__device__ __forceinline__ int d_sign(const WPt& P, const WPt& Q, const WPt& R) {
  const int64_t dy1 = (int64_t)Q.y - P.y, dy2 = (int64_t)R.y - P.y;
  const i128 D0 = (i128)((int64_t)Q.x - P.x) * dy2 - (i128)((int64_t)R.x - P.x) * dy1;
  if (D0) return D0 > 0 ? 1 : -1;
  const int64_t D1 = (int64_t)(Q.w - P.w) * dy2 - (int64_t)(R.w - P.w) * dy1;
  if (D1) return D1 > 0 ? 1 : -1;
  return d_sign_slow(P, Q, R);
}

template <class PT>
__device__ __forceinline__ Cand make_cand(const PT* pts, int a, int w, int b, const PT& A,
                                          const PT& W, const PT& B, int kind, int zs) {
  Cand c;
  c.t = Tri{a, w, b};
  c.kind = kind;
  c.st = tau_std(A, W, B, zs);
  return c;
}

// Largest i in [0, count) with off[i] <= x (off non-decreasing, off[0] <= x).
__device__ __forceinline__ int find_owner(const int* off, int count, int64_t x) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ Cand cand_of(const Event* ev, int64_t q) {
  const Event E = ev[q];
  Cand c;
  c.t = Tri{E.a, E.w(), E.b};
  c.kind = E.kind();
  c.st = (double)E.t;
  return c;
}

// Pointers of one run for the parallel (bridge walk and scatter) strategy.
// Everything is sized by the events of the level, not by the points: child
// events are enumerated into a compact list, and per-point lists exist only
// for the points those events touch.
struct ParRun {
  const void* pts;  // int4 or WPt, as in RunPtrs
  int* pv0;
  int* nx0;
  const Event* ev_in;
  const int* len_in;
  Event* ev_out;
  int* len_out;
  int* cntR;      // per point: # child events changing nx(p)
  int* cntL;      // per point: # child events changing pv(p)
  int* offR;      // per point: start of its list
  int* offL;
  int* curR;
  int* curL;
  int* claimR;    // per point: level that allocated its list
  int* claimL;
  int stamp;      // this level's claim stamp: lists of other points are empty
  Entry* entR;    // link-change events grouped by point, time-sorted (by slot)
  Entry* entL;
  int* ctr;       // [kCtrSlots]: touched lists; level totals of merges, child events,
                  // walk segments, bridge events
  int* touched;   // (point << 1 | side) of every allocated list
  int* ecnt;      // per merge: child events (mcap + 1)
  int* eoff;      // exclusive scan of ecnt
  int* cslot;     // per child event: its slot in the input movies
  int* cmerge;    // per child event: its merge
  int* segS;      // per merge: # time segments of its bridge walk
  int* segBase;   // exclusive scan of segS
  int* segMerge;  // per segment: its merge
  int* segB;      // per segment: input-movie slot of the child event it starts after (-1: -inf)
  int* segCnt;    // per segment: # bridge events
  int* segOff;    // exclusive scan of segCnt
  int2* segUV;    // per segment: the bridge at its start (found by the counting pass)
  Event* segTmp;  // per segment: its first kSegKeep bridge events (counting pass)
  int2* segTmpUV; // and the bridges after them
  Event* bev;     // bridge events of merge (s, e) at slots [2s, 2s + nB)
  int2* buv;      // (u, v) after each bridge event
  int* nB;        // per merge: # bridge events
  int* boff;      // exclusive scan of nB
  int2* uv0;      // per merge: the bridge at -inf
  int* surv;      // per child event: survives into the merged movie (+1 entry)
  int* jb;        // per child event: # bridge events before it
  int* pre;       // exclusive scan of surv
  int* aR;        // per child event: list entries (R side) of the lists it allocates,
  int* aL;        //   then their start (exclusive scan); L side
  int* aT;        //   touched lists it allocates, then their start
  unsigned char* wf;  // per child event: which of its lists it allocates (bits R a, R w, L b, L w)
  int zs;
};

struct ParLevel {
  ParRun run[2];
  Header* h;
  Sched S;
  int k;            // level: input blocks of 2^(k-1) points, merged blocks of 2^k
  int seg_events;   // child events per walk segment
  int64_t seg_cap;  // bound on the walk segments of a level
  int64_t ecap;     // bound on the child events of a level (2n)
  unsigned long long* chain_words;  // status words of the level's one-launch scans
  int64_t chain_stride;             // (kChainJobs slots), zeroed once per call
};

template <class PT>
int32_t parallel_level(const ParLevel& P, hipStream_t s);

}  // namespace hull
