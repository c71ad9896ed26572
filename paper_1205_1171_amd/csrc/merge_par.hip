// Parallel merge strategy for large blocks: the kinetic merge of two movies
// (Sec. 2, the merge step) with only the bridge walk left serial.
//
// In the merge of L and R, a child event matters to the bridge only when it
// changes a link of a current bridge endpoint (nx(u), pv(u), pv(v), nx(v));
// every other child event just passes through or is hidden, depending on
// where the bridge was at its time.  So:
//   1. per-point lists of the child events that change the point's links,
//      in time order (a counting sort by point, then a sort of each short
//      list by event position: a movie is already in time order);
//   2. the bridge walk, one thread per merge: the four bridge moves and the
//      next link change of u and v, earliest first.  Its length is the number
//      of bridge events plus the link changes of the endpoints, not the size
//      of the movies;
//   3. each child event finds, by binary search over the bridge events, the
//      bridge at its time: an L event survives when its point is left of u,
//      an R event when right of v;
//   4. the merged movie is the three time-sorted lists (L survivors, R
//      survivors, bridge events) merged: every element's position is its
//      rank in its own list plus its rank in the two others (prefix sums and
//      binary searches).
// The result is the same movie as the lane-serial merge, event for event.
#include <algorithm>
#include <initializer_list>

#include "common.hpp"
#include "events.hpp"

namespace hull {

// # of events among slots [base, base + len) strictly before X.
template <class PT>
__device__ int count_before(const PT* pts, const Event* ev, int64_t base, int len, const Cand& X,
                            int zs) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    Cand c = cand_of(ev, base + mid);
    if (ev_cmp(pts, c, X, zs) < 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Sort one point's entries by slot (= time order within the child movie),
// then replace each slot by the event's time.
__device__ void sort_entries(Entry* a, int k, const Event* ev) {
  int gap = 1;
  while (gap < k / 3) gap = 3 * gap + 1;
  for (; gap > 0; gap /= 3)
    for (int i = gap; i < k; ++i) {
      Entry x = a[i];
      int j = i;
      while (j >= gap && a[j - gap].key > x.key) {
        a[j] = a[j - gap];
        j -= gap;
      }
      a[j] = x;
    }
  for (int i = 0; i < k; ++i) a[i].key = __float_as_int(ev[a[i].key].t);
}

// Link of p after an event that changes it.
__device__ __forceinline__ int right_after(const Entry& E, int p) {
  return p == E.a ? (E.kind() ? E.w() : E.b) : E.b;
}
__device__ __forceinline__ int left_after(const Entry& E, int p) {
  return p == E.b ? (E.kind() ? E.w() : E.a) : E.a;
}

// A sorted entry as a candidate (its key holds the time).
__device__ __forceinline__ Cand cand_entry(const Entry* e, int j) {
  const Entry E = e[j];
  Cand c;
  c.t = Tri{E.a, E.w(), E.b};
  c.kind = E.kind();
  c.st = (double)__int_as_float(E.key);
  return c;
}

// Position in a point's list of its first change strictly after T.
template <class PT>
__device__ int first_after(const ParRun& R, const Entry* e, int off, int cnt, bool haveT,
                           const Cand& T) {
  if (!haveT) return 0;
  int lo = 0, hi = cnt;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    Cand c = cand_entry(e, off + mid);
    if (ev_cmp((const PT*)R.pts, c, T, R.zs) > 0) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

struct Endpoint {
  int p;       // the point
  int nx, pv;  // its links at the current time
  int cr, cl;  // next unprocessed change in its right / left list
  int oR, nR, oL, nL;
};

template <class PT>
__device__ void lookup(const ParRun& R, Endpoint& X, bool haveT, const Cand& T) {
  int p = X.p;
  // a point no child event touched at this level has empty lists (its
  // counters still hold an earlier level's values)
  const bool hasR = R.claimR[p] == R.stamp, hasL = R.claimL[p] == R.stamp;
  X.oR = hasR ? R.offR[p] : 0;
  X.nR = hasR ? R.cntR[p] : 0;
  X.oL = hasL ? R.offL[p] : 0;
  X.nL = hasL ? R.cntL[p] : 0;
  X.cr = first_after<PT>(R, R.entR, X.oR, X.nR, haveT, T);
  X.cl = first_after<PT>(R, R.entL, X.oL, X.nL, haveT, T);
  X.nx = X.cr > 0 ? right_after(R.entR[X.oR + X.cr - 1], p) : R.nx0[p];
  X.pv = X.cl > 0 ? left_after(R.entL[X.oL + X.cl - 1], p) : R.pv0[p];
}

// One link of p just after T (the right link with `right`), without the rest
// of the endpoint state: the tangent search needs only that.
template <class PT>
__device__ int link_after(const ParRun& R, int p, bool right, bool haveT, const Cand& T) {
  if (right) {
    if (R.claimR[p] != R.stamp) return R.nx0[p];
    const int o = R.offR[p];
    const int c = first_after<PT>(R, R.entR, o, R.cntR[p], haveT, T);
    return c > 0 ? right_after(R.entR[o + c - 1], p) : R.nx0[p];
  }
  if (R.claimL[p] != R.stamp) return R.pv0[p];
  const int o = R.offL[p];
  const int c = first_after<PT>(R, R.entL, o, R.cntL[p], haveT, T);
  return c > 0 ? left_after(R.entL[o + c - 1], p) : R.pv0[p];
}

// Orientation of the rank-ordered triple (a, b, c) just after event T: its
// sign at t = -inf is sign(D), and it flips once, at its own event.
template <class PT>
__device__ int orient_after(const PT* pts, int a, int b, int c, const Cand& T, int zs) {
  const PT A = pts[a], B = pts[b], C = pts[c];
  int ds = d_sign(A, B, C);
  Cand x = make_cand(pts, a, b, c, A, B, C, 0, zs);
  return ev_cmp(pts, x, T, zs) > 0 ? ds : -ds;
}

// Segment i of S of a merge covers the events after boundary b_i up to and
// including b_(i+1), b_0 = -inf, b_S = +inf.  With N = nL + nR child events
// in time order (both movies merged), b_i (0 < i < S) is the one at position
// floor(i * N / S) - 1, so every segment spans the same number of child
// events of the two movies together.  Found by a co-rank search: the number
// jL of left-movie events among the first k = floor(i * N / S) is the first
// j at which L[j] comes after R[k-1-j].  Returns b_i's input-movie slot.
template <class PT>
__device__ int64_t boundary_slot(const ParRun& R, int64_t s, int64_t m, int i, int S) {
  const PT* pts = (const PT*)R.pts;
  const int nL = R.len_in[s], nR = R.len_in[m];
  const int64_t N = (int64_t)nL + nR;
  const int k = (int)((int64_t)i * N / S);
  int lo = k - nR > 0 ? k - nR : 0, hi = k < nL ? k : nL;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ev_cmp(pts, cand_of(R.ev_in, 2 * s + mid), cand_of(R.ev_in, 2 * m + (k - 1 - mid)),
               R.zs) < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int jL = lo, jR = k - lo;
  if (jL == 0) return 2 * m + jR - 1;
  if (jR == 0) return 2 * s + jL - 1;
  const int64_t a = 2 * s + jL - 1, b = 2 * m + jR - 1;
  return ev_cmp(pts, cand_of(R.ev_in, a), cand_of(R.ev_in, b), R.zs) > 0 ? a : b;
}

__device__ __forceinline__ int segments_for(int nL, int nR, int G) {
  int nn = nL > nR ? nL : nR;
  int S = 1 + (nL + nR) / G;
  return S > nn + 1 ? nn + 1 : S;
}

// The bridge walk over one time segment.  Returns the number of bridge
// events in the segment; with `out` set, writes them there (and their
// bridges after each move to `out_uv`).  Segment 0 also reports the -inf
// bridge in `uv0`.
template <class PT>
__device__ int walk_segment(const ParRun& R, Header* h, int64_t s, int64_t m, int64_t e,
                            int64_t b0, int64_t b1, Event* out, int2* out_uv, int cap,
                            int2* uv0, int2* start_uv, bool have_start, Event* keep = nullptr,
                            int2* keep_uv = nullptr, const Event* resume = nullptr) {
  const PT* pts = (const PT*)R.pts;
  const int zs = R.zs;
  bool haveT = false, haveEnd = false;
  Cand T, Tend;
  T.t = Tri{-1, -1, -1};
  T.st = 0.0;
  T.kind = 0;
  Tend = T;
  if (b0 >= 0) {
    T = cand_of(R.ev_in, b0);
    haveT = true;
  }
  if (b1 >= 0) {
    Tend = cand_of(R.ev_in, b1);
    haveEnd = true;
  }
  if (resume) {  // continue after an event this segment already produced
    T = cand_of(resume, 0);
    haveT = true;
  }
  // the bridge at the start of the segment: walk to the lower common tangent
  // of the two chains, from the inner ends of the blocks (each step needs one
  // link of one endpoint); the counting pass leaves it for the writing pass
  int up = (int)m - 1, vp = (int)m;
  if (have_start) {
    up = start_uv->x;
    vp = start_uv->y;
    if (up < s || up >= m || vp < m || vp >= e) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      return 0;
    }
  } else {
    int vnx = link_after<PT>(R, vp, true, haveT, T), upv = link_after<PT>(R, up, false, haveT, T);
    for (int guard = 0;; ++guard) {
      if (guard > 2 * (e - s) + 4) {
        atomicCAS(&h->err, 0, HULL_EINTERNAL);
        return 0;
      }
      if (vnx != kNil) {
        int o = haveT ? orient_after(pts, up, vp, vnx, T, zs) : d_sign(pts[up], pts[vp], pts[vnx]);
        if (o < 0) {
          vp = vnx;
          vnx = link_after<PT>(R, vp, true, haveT, T);
          continue;
        }
      }
      if (upv != kNil) {
        int o = haveT ? orient_after(pts, upv, up, vp, T, zs) : d_sign(pts[upv], pts[up], pts[vp]);
        if (o < 0) {
          up = upv;
          upv = link_after<PT>(R, up, false, haveT, T);
          continue;
        }
      }
      break;
    }
    if (start_uv) *start_uv = make_int2(up, vp);
  }
  Endpoint U{up, 0, 0, 0, 0, 0, 0, 0, 0}, V{vp, 0, 0, 0, 0, 0, 0, 0, 0};
  lookup<PT>(R, U, haveT, T);
  lookup<PT>(R, V, haveT, T);
  if (uv0) *uv0 = make_int2(U.p, V.p);
  PT Pu = pts[U.p], Pv = pts[V.p];
  int nb = 0;
  const int64_t iter_cap = (int64_t)R.len_in[s] + R.len_in[m] + 4 * (e - s) + 16;
  for (int64_t it = 0;; ++it) {
    if (it > iter_cap) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      break;
    }
    // candidates: 0..3 bridge moves (checked against T), 4..7 the next link
    // changes of u and v (after T by construction).  The running best is
    // kept field by field in scalars and every candidate index is a
    // compile-time constant, so the candidates stay in registers.
    int bi = -1, ba = 0, bw = 0, bb = 0, bk = 0;
    double bs = 0.0;
#define HULL_CONSIDER(IDX, CAND)                                                  \
  do {                                                                            \
    const Cand cc_ = (CAND);                                                      \
    bool take_ = !((IDX) < 4 && haveT && ev_cmp(pts, cc_, T, zs) <= 0);           \
    if (take_ && bi >= 0) {                                                       \
      Cand cb_;                                                                   \
      cb_.t = Tri{ba, bw, bb};                                                    \
      cb_.st = bs;                                                                \
      cb_.kind = bk;                                                              \
      take_ = ev_cmp(pts, cc_, cb_, zs) < 0;                                      \
    }                                                                             \
    if (take_) {                                                                  \
      bi = (IDX);                                                                 \
      ba = cc_.t.a;                                                               \
      bw = cc_.t.w;                                                               \
      bb = cc_.t.b;                                                               \
      bs = cc_.st;                                                                \
      bk = cc_.kind;                                                              \
    }                                                                             \
  } while (0)
    if (U.nx != kNil) HULL_CONSIDER(0, make_cand(pts, U.p, U.nx, V.p, Pu, pts[U.nx], Pv, 1, zs));
    if (U.pv != kNil) HULL_CONSIDER(1, make_cand(pts, U.pv, U.p, V.p, pts[U.pv], Pu, Pv, 0, zs));
    if (V.pv != kNil) HULL_CONSIDER(2, make_cand(pts, U.p, V.pv, V.p, Pu, pts[V.pv], Pv, 1, zs));
    if (V.nx != kNil) HULL_CONSIDER(3, make_cand(pts, U.p, V.p, V.nx, Pu, Pv, pts[V.nx], 0, zs));
    if (U.cr < U.nR) HULL_CONSIDER(4, cand_entry(R.entR, U.oR + U.cr));
    if (U.cl < U.nL) HULL_CONSIDER(5, cand_entry(R.entL, U.oL + U.cl));
    if (V.cl < V.nL) HULL_CONSIDER(6, cand_entry(R.entL, V.oL + V.cl));
    if (V.cr < V.nR) HULL_CONSIDER(7, cand_entry(R.entR, V.oR + V.cr));
#undef HULL_CONSIDER
    Cand best;
    best.t = Tri{ba, bw, bb};
    best.st = bs;
    best.kind = bk;
    if (bi < 0) break;
    if (haveEnd && ev_cmp(pts, best, Tend, zs) > 0) break;
    T = best;
    haveT = true;
    if (bi >= 4) {  // a link change of an endpoint
      if (bi == 4) { U.nx = right_after(R.entR[U.oR + U.cr], U.p); ++U.cr; }
      else if (bi == 5) { U.pv = left_after(R.entL[U.oL + U.cl], U.p); ++U.cl; }
      else if (bi == 6) { V.pv = left_after(R.entL[V.oL + V.cl], V.p); ++V.cl; }
      else { V.nx = right_after(R.entR[V.oR + V.cr], V.p); ++V.cr; }
      continue;
    }
    if (bi == 0) U.p = U.nx;
    else if (bi == 1) U.p = U.pv;
    else if (bi == 2) V.p = V.pv;
    else V.p = V.nx;
    if (bi <= 1) {
      Pu = pts[U.p];
      lookup<PT>(R, U, true, T);
    } else {
      Pv = pts[V.p];
      lookup<PT>(R, V, true, T);
    }
    if (out) {
      if (nb >= cap) {
        atomicCAS(&h->err, 0, HULL_EINTERNAL);
        break;
      }
      out[nb] = make_event(T.t.a, T.t.w, T.t.b, T.kind, T.st);
      out_uv[nb] = make_int2(U.p, V.p);
    } else if (keep && nb < kSegKeep) {
      keep[nb] = make_event(T.t.a, T.t.w, T.t.b, T.kind, T.st);
      keep_uv[nb] = make_int2(U.p, V.p);
    }
    ++nb;
  }
  return nb;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

// Per merge: child event count and walk segments; counters reset.
__global__ void __launch_bounds__(256) k_par_prep(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int merges = P.S.moff[P.S.H];
  const int64_t half = int64_t(1) << (P.k - 1);
  GRID_STRIDE(g, (int64_t)merges + 1) {
    if (g == 0) {
      R.ctr[kCtrTouched] = 0;
      R.ctr[kCtrMerges] = merges;
    }
    if (g < merges && !P.h->err) {
      const int2 se = P.S.mlist[g];
      const int nL = R.len_in[se.x], nR = R.len_in[se.x + half];
      R.ecnt[g] = nL + nR;
      R.segS[g] = segments_for(nL, nR, P.seg_events);
    } else {
      R.ecnt[g] = 0;
      R.segS[g] = 0;
    }
    R.nB[g] = 0;
  }
}

// The compact list of child events (slot and merge of each), and the
// link-change counters of their points cleared; then, past the events, the
// segment table: per walk segment its merge and the slot of the child event
// it starts after.
template <class PT>
__global__ void __launch_bounds__(256) k_par_enum(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int merges = R.ctr[kCtrMerges], E = R.ctr[kCtrEvents], Sg = R.ctr[kCtrSegments];
  const int64_t half = int64_t(1) << (P.k - 1);
  const bool err = P.h->err != 0;
  GRID_STRIDE(c, (int64_t)E + Sg) {
    if (c >= E) {
      const int64_t t = c - E;
      const int g = find_owner(R.segBase, merges, t);
      R.segMerge[t] = g;
      const int i = (int)(t - R.segBase[g]);
      const int64_t s = P.S.mlist[g].x;
      R.segB[t] = i == 0 || err ? -1 : (int)boundary_slot<PT>(R, s, s + half, i, R.segS[g]);
      continue;
    }
    const int g = find_owner(R.eoff, merges, c);
    const int2 se = P.S.mlist[g];
    const int64_t s = se.x, m = s + half;
    const int nL = R.len_in[s];
    const int64_t i = c - R.eoff[g];
    const int64_t slot = i < nL ? 2 * s + i : 2 * m + (i - nL);
    R.cslot[c] = (int)slot;
    R.cmerge[c] = g;
    const Event X = R.ev_in[slot];
    R.cntR[X.a] = 0;
    R.curR[X.a] = 0;
    R.cntL[X.b] = 0;
    R.curL[X.b] = 0;
    if (X.kind()) {
      R.cntR[X.w()] = 0;
      R.curR[X.w()] = 0;
      R.cntL[X.w()] = 0;
      R.curL[X.w()] = 0;
    }
  }
}

// Which links an event changes: nx(a) and pv(b); an insertion also sets
// nx(w) and pv(w).
__global__ void __launch_bounds__(256) k_par_count(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  GRID_STRIDE(c, R.ctr[kCtrEvents]) {
    const Event X = R.ev_in[R.cslot[c]];
    atomicAdd(&R.cntR[X.a], 1);
    atomicAdd(&R.cntL[X.b], 1);
    if (X.kind()) {
      atomicAdd(&R.cntR[X.w()], 1);
      atomicAdd(&R.cntL[X.w()], 1);
    }
  }
}

// One list per touched (point, side), allocated by whichever child event
// claims it first at this level (claim stamp = the level).  Pass 1: each
// event claims, and records how many list entries and lists it allocates;
// after exclusive scans of those counts, pass 2 places the lists.  (No
// shared counters: space comes from prefix sums.)
__global__ void __launch_bounds__(256) k_par_claim(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int E = R.ctr[kCtrEvents], st = R.stamp;
  GRID_STRIDE(c, (int64_t)E + 1) {
    if (c == E) {  // the scans read one entry past the last event
      R.aR[c] = R.aL[c] = R.aT[c] = 0;
      continue;
    }
    const Event X = R.ev_in[R.cslot[c]];
    unsigned bits = 0;
    int nR = 0, nL = 0;
    if (atomicExch(&R.claimR[X.a], st) != st) {
      bits |= 1u;
      nR += R.cntR[X.a];
    }
    if (atomicExch(&R.claimL[X.b], st) != st) {
      bits |= 4u;
      nL += R.cntL[X.b];
    }
    if (X.kind()) {
      if (atomicExch(&R.claimR[X.w()], st) != st) {
        bits |= 2u;
        nR += R.cntR[X.w()];
      }
      if (atomicExch(&R.claimL[X.w()], st) != st) {
        bits |= 8u;
        nL += R.cntL[X.w()];
      }
    }
    R.aR[c] = nR;
    R.aL[c] = nL;
    R.aT[c] = __builtin_popcount(bits);
    R.wf[c] = (unsigned char)bits;
  }
}

__global__ void __launch_bounds__(256) k_par_place(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int E = R.ctr[kCtrEvents];
  // capacities: 3n entries per side (one per child event, 2n events, and one
  // more per insertion, n of them: a point is inserted at most once in its
  // block's movie), 2n touched lists (one per point and side)
  const int64_t ent_cap = P.ecap + P.ecap / 2, touched_cap = P.ecap;
  if (R.aR[E] > ent_cap || R.aL[E] > ent_cap || R.aT[E] > touched_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
    return;
  }
  GRID_STRIDE(c, (int64_t)E + 1) {
    if (c == E) {
      R.ctr[kCtrTouched] = R.aT[E];  // touched lists of the level
      continue;
    }
    const unsigned bits = R.wf[c];
    if (!bits) continue;
    const Event X = R.ev_in[R.cslot[c]];
    int bR = R.aR[c], bL = R.aL[c], bT = R.aT[c];
    if (bits & 1u) {
      R.offR[X.a] = bR;
      bR += R.cntR[X.a];
      R.touched[bT++] = X.a << 1;
    }
    if (bits & 2u) {
      R.offR[X.w()] = bR;
      R.touched[bT++] = X.w() << 1;
    }
    if (bits & 4u) {
      R.offL[X.b] = bL;
      bL += R.cntL[X.b];
      R.touched[bT++] = (X.b << 1) | 1;
    }
    if (bits & 8u) {
      R.offL[X.w()] = bL;
      R.touched[bT++] = (X.w() << 1) | 1;
    }
  }
}

// Lists of link changes: every entry is the child event and its slot in the
// input movies (the sort key: a movie is in time order).
__global__ void __launch_bounds__(256) k_par_fill(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts || P.h->err) return;  // after an error the offsets may be stale
  GRID_STRIDE(c, R.ctr[kCtrEvents]) {
    const int q = R.cslot[c];
    const Event E = R.ev_in[q];
    Entry X;
    X.a = E.a;
    X.wk = E.wk;
    X.b = E.b;
    X.key = q;
    int j = R.offR[E.a] + atomicAdd(&R.curR[E.a], 1);
    R.entR[j] = X;
    j = R.offL[E.b] + atomicAdd(&R.curL[E.b], 1);
    R.entL[j] = X;
    if (E.kind()) {
      const int w = E.w();
      j = R.offR[w] + atomicAdd(&R.curR[w], 1);
      R.entR[j] = X;
      j = R.offL[w] + atomicAdd(&R.curL[w], 1);
      R.entL[j] = X;
    }
  }
}

__global__ void __launch_bounds__(256) k_par_sort(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts || P.h->err) return;
  GRID_STRIDE(t, R.ctr[kCtrTouched]) {
    const int x = R.touched[t], p = x >> 1;
    if (x & 1) sort_entries(R.entL + R.offL[p], R.cntL[p], R.ev_in);
    else sort_entries(R.entR + R.offR[p], R.cntR[p], R.ev_in);
  }
}

// Pass 1 counts each segment's bridge events; pass 2 writes them at their
// place in the merge's bridge list.
template <class PT>
__global__ void __launch_bounds__(64) k_par_walk(ParLevel P, int write) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int total = R.ctr[kCtrSegments];
  const int64_t half = int64_t(1) << (P.k - 1);
  GRID_STRIDE(t, (int64_t)total + 1) {
    if (t == total) {  // the scan reads one entry past the last segment
      if (!write) R.segCnt[t] = 0;
      continue;
    }
    const int g = R.segMerge[t];
    const int first = R.segBase[g], S = R.segS[g], i = (int)(t - first);
    const int2 se = P.S.mlist[g];
    const int64_t s = se.x, m = s + half, e = se.y;
    const int64_t b0 = R.segB[t], b1 = i + 1 < S ? R.segB[t + 1] : -1;
    if (P.h->err) {
      if (!write) R.segCnt[t] = 0;
      else if (i == 0) {
        R.nB[g] = 0;
        R.uv0[g] = make_int2(0, 0);
      }
      continue;
    }
    if (!write) {
      R.segCnt[t] = walk_segment<PT>(R, P.h, s, m, e, b0, b1, nullptr, nullptr, 0,
                                 i == 0 ? &R.uv0[g] : nullptr, &R.segUV[t], false,
                                 R.segTmp + (int64_t)t * kSegKeep,
                                 R.segTmpUV + (int64_t)t * kSegKeep);
      continue;
    }
    if (i == 0) R.nB[g] = R.segOff[first + S] - R.segOff[first];
    const int cnt = R.segCnt[t];
    if (cnt == 0) continue;  // nothing to write (the -inf bridge is known)
    const int64_t off = R.segOff[t] - R.segOff[first];
    const int cap = (int)(2 * (e - s) - off);
    // the counting pass kept the first kSegKeep: copy them, and walk on from
    // the last of them only for the rest
    const int kept = cnt < kSegKeep ? cnt : kSegKeep;
    if (cnt > cap) {
      atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
      continue;
    }
    for (int q = 0; q < kept; ++q) {
      R.bev[2 * s + off + q] = R.segTmp[(int64_t)t * kSegKeep + q];
      R.buv[2 * s + off + q] = R.segTmpUV[(int64_t)t * kSegKeep + q];
    }
    if (cnt <= kSegKeep) continue;
    const int64_t last = (int64_t)t * kSegKeep + kSegKeep - 1;
    walk_segment<PT>(R, P.h, s, m, e, b0, b1, R.bev + 2 * s + off + kSegKeep,
                 R.buv + 2 * s + off + kSegKeep, cap - kSegKeep, nullptr, &R.segTmpUV[last],
                 true, nullptr, nullptr, &R.segTmp[last]);
  }
}

// Survival of every child event, and the number of bridge events before it.
template <class PT>
__global__ void __launch_bounds__(256) k_par_classify(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int E = R.ctr[kCtrEvents];
  const int64_t half = int64_t(1) << (P.k - 1);
  const bool err = P.h->err != 0;
  GRID_STRIDE(c, (int64_t)E + 1) {
    if (c == E || err) {
      R.surv[c] = 0;
      continue;
    }
    const int g = R.cmerge[c];
    const int q = R.cslot[c];
    const int64_t s = P.S.mlist[g].x, m = s + half;
    const bool isL = q < 2 * m;
    const Cand x = cand_of(R.ev_in, q);
    const int j = count_before((const PT*)R.pts, R.bev, 2 * s, R.nB[g], x, R.zs);
    const int2 ref = j > 0 ? R.buv[2 * s + j - 1] : R.uv0[g];
    R.surv[c] = isL ? (x.t.w < ref.x) : (x.t.w > ref.y);
    R.jb[c] = j;
  }
}

// Scatter: child survivors, then bridge events, to their places in the
// merged movies; then every merge writes its length and splices its -inf
// chains (no kernel of this level reads the -inf links after the walk).
template <class PT>
__global__ void __launch_bounds__(256) k_par_scatter(ParLevel P) {
  const PT* pts = (const PT*)P.run[blockIdx.y].pts;
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const bool err = P.h->err != 0;
  const int merges = R.ctr[kCtrMerges], E = R.ctr[kCtrEvents], Bt = R.ctr[kCtrBridge];
  const int64_t half = int64_t(1) << (P.k - 1);
  GRID_STRIDE(t, (int64_t)E + Bt + merges) {
    if (t < E) {
      const int64_t c = t;
      if (err || !R.surv[c]) continue;
      const int g = R.cmerge[c];
      const int q = R.cslot[c];
      const int2 se = P.S.mlist[g];
      const int64_t s = se.x, m = s + half, e = se.y;
      const int nL = R.len_in[s], nR = R.len_in[m];
      const int c0 = R.eoff[g], cR = c0 + nL;
      const Cand x = cand_of(R.ev_in, q);
      int64_t pos;
      if (q < 2 * m) {
        const int idx = count_before(pts, R.ev_in, 2 * m, nR, x, R.zs);
        pos = (R.pre[c] - R.pre[c0]) + (R.pre[cR + idx] - R.pre[cR]) + R.jb[c];
      } else {
        const int idx = count_before(pts, R.ev_in, 2 * s, nL, x, R.zs);
        pos = (R.pre[c0 + idx] - R.pre[c0]) + (R.pre[c] - R.pre[cR]) + R.jb[c];
      }
      if (pos >= 2 * (e - s)) {
        atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
        continue;
      }
      R.ev_out[2 * s + pos] = R.ev_in[q];
    } else if (t < (int64_t)E + Bt) {
      if (err) continue;
      const int64_t b = t - E;
      const int g = find_owner(R.boff, merges, b);
      const int j = (int)(b - R.boff[g]);
      const int2 se = P.S.mlist[g];
      const int64_t s = se.x, m = s + half, e = se.y;
      const int nL = R.len_in[s], nR = R.len_in[m];
      const int c0 = R.eoff[g], cR = c0 + nL;
      const Cand x = cand_of(R.bev, 2 * s + j);
      const int iL = count_before(pts, R.ev_in, 2 * s, nL, x, R.zs);
      const int iR = count_before(pts, R.ev_in, 2 * m, nR, x, R.zs);
      const int64_t pos = j + (R.pre[c0 + iL] - R.pre[c0]) + (R.pre[cR + iR] - R.pre[cR]);
      if (pos >= 2 * (e - s)) {
        atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
        continue;
      }
      R.ev_out[2 * s + pos] = R.bev[2 * s + j];
    } else {
      const int g = (int)(t - E - Bt);
      const int2 se = P.S.mlist[g];
      const int64_t s = se.x, e = se.y;
      // every merge writes its length, also after an error (then 0)
      const int cnt = err ? 0 : (R.pre[R.eoff[g + 1]] - R.pre[R.eoff[g]]) + R.nB[g];
      R.len_out[s] = cnt <= 2 * (e - s) ? cnt : 0;
      if (cnt > 2 * (e - s)) atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
      if (!err) {
        const int2 b0 = R.uv0[g];
        R.nx0[b0.x] = b0.y;
        R.pv0[b0.y] = b0.x;
      }
    }
  }
}

// Scans of the same per-run arrays of both runs (and of several arrays) in
// one set of launches.
static ScanJobs jobs_of(const ParLevel& P, std::initializer_list<int> fields, int ctr_index) {
  ScanJobs J{};
  for (int r = 0; r < 2; ++r) {
    const ParRun& R = P.run[r];
    if (!R.pts) continue;
    for (int f : fields) {
      int32_t* a = nullptr;
      switch (f) {
        // the level totals of child events, walk segments and bridge events
        // come from the scans themselves
        case 0: J.j[J.count] = ScanJob{R.ecnt, R.eoff, R.ctr + ctr_index, R.ctr + kCtrEvents}; break;
        case 1:
          J.j[J.count] = ScanJob{R.segS, R.segBase, R.ctr + ctr_index, R.ctr + kCtrSegments};
          break;
        case 2: a = R.aR; J.j[J.count] = ScanJob{a, a, R.ctr + ctr_index, nullptr}; break;
        case 3: a = R.aL; J.j[J.count] = ScanJob{a, a, R.ctr + ctr_index, nullptr}; break;
        case 4: a = R.aT; J.j[J.count] = ScanJob{a, a, R.ctr + ctr_index, nullptr}; break;
        case 5: J.j[J.count] = ScanJob{R.segCnt, R.segOff, R.ctr + ctr_index, nullptr}; break;
        case 6: J.j[J.count] = ScanJob{R.nB, R.boff, R.ctr + ctr_index, R.ctr + kCtrBridge}; break;
        default: J.j[J.count] = ScanJob{R.surv, R.pre, R.ctr + ctr_index, nullptr}; break;
      }
      ++J.count;
    }
  }
  return J;
}

// The level's five scans, one launch each, on job slots of their own; the
// epoch (level and scan) tells their status words from those of earlier
// levels of the call.
static int32_t chained(const ParLevel& P, const ScanJobs& J, int slot, int site, int64_t cap,
                       hipStream_t s) {
  return exclusive_scan_chained(J, 1, cap, P.chain_words + slot * P.chain_stride, P.chain_stride,
                                (unsigned)(P.k * 8 + site), P.h, s);
}

template <class PT>
int32_t parallel_level(const ParLevel& P, hipStream_t s) {
  const dim3 g2(kStrideBlocks, 2), b256(256);
  hipLaunchKernelGGL(k_par_prep, g2, b256, 0, s, P);
  // per merge: child events, walk segments (length: merges + 1)
  int32_t rc = chained(P, jobs_of(P, {0, 1}, kCtrMerges), 0, 1, P.S.mcap + 1, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_par_enum<PT>, g2, b256, 0, s, P);
  hipLaunchKernelGGL(k_par_count, g2, b256, 0, s, P);
  hipLaunchKernelGGL(k_par_claim, g2, b256, 0, s, P);
  // per child event: list entries and lists it allocates (length: events + 1)
  rc = chained(P, jobs_of(P, {2, 3, 4}, kCtrEvents), 4, 2, P.ecap + 1, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_par_place, g2, b256, 0, s, P);
  hipLaunchKernelGGL(k_par_fill, g2, b256, 0, s, P);
  hipLaunchKernelGGL(k_par_sort, g2, b256, 0, s, P);
  const dim3 gw(16384, 2), b64(64);
  hipLaunchKernelGGL(k_par_walk<PT>, gw, b64, 0, s, P, 0);
  rc = chained(P, jobs_of(P, {5}, kCtrSegments), 10, 3, P.seg_cap + 1, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_par_walk<PT>, gw, b64, 0, s, P, 1);
  rc = chained(P, jobs_of(P, {6}, kCtrMerges), 12, 4, P.S.mcap + 1, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_par_classify<PT>, g2, b256, 0, s, P);
  rc = chained(P, jobs_of(P, {7}, kCtrEvents), 14, 5, P.ecap + 1, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_par_scatter<PT>, g2, b256, 0, s, P);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

template int32_t parallel_level<int4>(const ParLevel&, hipStream_t);
template int32_t parallel_level<WPt>(const ParLevel&, hipStream_t);

}  // namespace hull
