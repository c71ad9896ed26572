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

#include "common.hpp"
#include "events.hpp"

namespace hull {

__device__ __forceinline__ int64_t in_block_start(int64_t q, int k) {
  return ((q >> 1) >> (k - 1)) << (k - 1);
}

// # of events among slots [base, base + len) strictly before X.
__device__ int count_before(const int4* pts, const Event* ev, const double* tau, int64_t base,
                            int len, const Cand& X, int zs) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    Cand c = cand_of(ev, tau, base + mid);
    if (ev_cmp(pts, c, X, zs) < 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_par_zero(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P.n;
       p += (int64_t)gridDim.x * blockDim.x) {
    R.cntR[p] = 0;
    R.cntL[p] = 0;
    R.curR[p] = 0;
    R.curL[p] = 0;
  }
}

// Which links an event changes: nx(a) and pv(b); an insertion also sets
// nx(w) and pv(w).
__global__ void __launch_bounds__(256) k_par_count(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts || P.h->err) return;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < 2 * P.n;
       q += (int64_t)gridDim.x * blockDim.x) {
    int64_t sb = in_block_start(q, P.k);
    if (q - 2 * sb >= R.len_in[sb]) continue;
    Event E = R.ev_in[q];
    atomicAdd(&R.cntR[E.a], 1);
    atomicAdd(&R.cntL[E.b], 1);
    if (E.kind) {
      atomicAdd(&R.cntR[E.w], 1);
      atomicAdd(&R.cntL[E.w], 1);
    }
  }
}

// Lists of link changes: every entry is the child event itself (its kind
// field also carries its slot, kind | slot << 1, the sort key) and its time.
__global__ void __launch_bounds__(256) k_par_fill(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts || P.h->err) return;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < 2 * P.n;
       q += (int64_t)gridDim.x * blockDim.x) {
    int64_t sb = in_block_start(q, P.k);
    if (q - 2 * sb >= R.len_in[sb]) continue;
    Event E = R.ev_in[q];
    double t = R.tau_in[q];
    Event X{E.a, E.w, E.b, (int)(q << 1) | E.kind};
    int j = R.offR[E.a] + atomicAdd(&R.curR[E.a], 1);
    R.entR[j] = X;
    R.entRt[j] = t;
    j = R.offL[E.b] + atomicAdd(&R.curL[E.b], 1);
    R.entL[j] = X;
    R.entLt[j] = t;
    if (E.kind) {
      j = R.offR[E.w] + atomicAdd(&R.curR[E.w], 1);
      R.entR[j] = X;
      R.entRt[j] = t;
      j = R.offL[E.w] + atomicAdd(&R.curL[E.w], 1);
      R.entL[j] = X;
      R.entLt[j] = t;
    }
  }
}

// Sort one point's entries by slot (= time order within the child movie).
__device__ void sort_entries(Event* a, double* t, int k) {
  int gap = 1;
  while (gap < k / 3) gap = 3 * gap + 1;
  for (; gap > 0; gap /= 3)
    for (int i = gap; i < k; ++i) {
      Event x = a[i];
      double y = t[i];
      int j = i;
      while (j >= gap && a[j - gap].kind > x.kind) {
        a[j] = a[j - gap];
        t[j] = t[j - gap];
        j -= gap;
      }
      a[j] = x;
      t[j] = y;
    }
}

__global__ void __launch_bounds__(256) k_par_sort(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts || P.h->err) return;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P.n;
       p += (int64_t)gridDim.x * blockDim.x) {
    sort_entries(R.entR + R.offR[p], R.entRt + R.offR[p], R.cntR[p]);
    sort_entries(R.entL + R.offL[p], R.entLt + R.offL[p], R.cntL[p]);
  }
}

// Link of p after an event that changes it.
__device__ __forceinline__ int right_after(const Event& E, int p) {
  return p == E.a ? ((E.kind & 1) ? E.w : E.b) : E.b;
}
__device__ __forceinline__ int left_after(const Event& E, int p) {
  return p == E.b ? ((E.kind & 1) ? E.w : E.a) : E.a;
}

__device__ __forceinline__ Cand cand_entry(const Event* e, const double* t, int j) {
  Event E = e[j];
  Cand c;
  c.t = Tri{E.a, E.w, E.b};
  c.kind = E.kind & 1;
  c.st = t[j];
  return c;
}

// Position in a point's list of its first change strictly after T.
__device__ int first_after(const ParRun& R, const Event* e, const double* t, int off, int cnt,
                           bool haveT, const Cand& T) {
  if (!haveT) return 0;
  int lo = 0, hi = cnt;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    Cand c = cand_entry(e, t, off + mid);
    if (ev_cmp(R.pts, c, T, R.zs) > 0) hi = mid;
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

__device__ void lookup(const ParRun& R, Endpoint& X, bool haveT, const Cand& T) {
  int p = X.p;
  X.oR = R.offR[p];
  X.nR = R.cntR[p];
  X.oL = R.offL[p];
  X.nL = R.cntL[p];
  X.cr = first_after(R, R.entR, R.entRt, X.oR, X.nR, haveT, T);
  X.cl = first_after(R, R.entL, R.entLt, X.oL, X.nL, haveT, T);
  X.nx = X.cr > 0 ? right_after(R.entR[X.oR + X.cr - 1], p) : R.nx0[p];
  X.pv = X.cl > 0 ? left_after(R.entL[X.oL + X.cl - 1], p) : R.pv0[p];
}

// Orientation of the rank-ordered triple (a, b, c) just after event T: its
// sign at t = -inf is sign(D), and it flips once, at its own event.
__device__ int orient_after(const int4* pts, int a, int b, int c, const Cand& T, int zs) {
  int4 A = pts[a], B = pts[b], C = pts[c];
  int ds = d_sign(A, B, C);
  Cand x = make_cand(pts, a, b, c, A, B, C, 0, zs);
  return ev_cmp(pts, x, T, zs) > 0 ? ds : -ds;
}

// Segment i of S of a merge covers the events after boundary b_i up to and
// including b_(i+1), b_0 = -inf, b_S = +inf; b_i (0 < i < S) is the event at
// index floor(i * n / S) of the longer child movie.
__device__ __forceinline__ int64_t boundary_slot(const ParRun& R, int64_t s, int64_t m, int i,
                                                 int S) {
  int nL = R.len_in[s], nR = R.len_in[m];
  int64_t base = nL >= nR ? 2 * s : 2 * m;
  int64_t nn = nL >= nR ? nL : nR;
  return base + (int64_t)i * nn / S;
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
__device__ int walk_segment(const ParRun& R, Header* h, int64_t s, int64_t m, int64_t e, int seg,
                            int S, Event* out, double* out_tau, int2* out_uv, int cap,
                            int2* uv0) {
  const int4* pts = R.pts;
  const int zs = R.zs;
  bool haveT = false, haveEnd = false;
  Cand T, Tend;
  T.t = Tri{-1, -1, -1};
  T.st = 0.0;
  T.kind = 0;
  Tend = T;
  if (seg > 0) {
    T = cand_of(R.ev_in, R.tau_in, boundary_slot(R, s, m, seg, S));
    haveT = true;
  }
  if (seg + 1 < S) {
    Tend = cand_of(R.ev_in, R.tau_in, boundary_slot(R, s, m, seg + 1, S));
    haveEnd = true;
  }
  // the bridge at the start of the segment: walk to the lower common tangent
  // of the two chains, from the inner ends of the blocks
  Endpoint U{(int)m - 1, 0, 0, 0, 0, 0, 0, 0, 0}, V{(int)m, 0, 0, 0, 0, 0, 0, 0, 0};
  lookup(R, U, haveT, T);
  lookup(R, V, haveT, T);
  for (int guard = 0;; ++guard) {
    if (guard > 2 * (e - s) + 4) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      return 0;
    }
    if (V.nx != kNil) {
      int o = haveT ? orient_after(pts, U.p, V.p, V.nx, T, zs)
                    : d_sign(pts[U.p], pts[V.p], pts[V.nx]);
      if (o < 0) {
        V.p = V.nx;
        lookup(R, V, haveT, T);
        continue;
      }
    }
    if (U.pv != kNil) {
      int o = haveT ? orient_after(pts, U.pv, U.p, V.p, T, zs)
                    : d_sign(pts[U.pv], pts[U.p], pts[V.p]);
      if (o < 0) {
        U.p = U.pv;
        lookup(R, U, haveT, T);
        continue;
      }
    }
    break;
  }
  if (uv0) *uv0 = make_int2(U.p, V.p);
  int4 Pu = pts[U.p], Pv = pts[V.p];
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
    if (U.cr < U.nR) HULL_CONSIDER(4, cand_entry(R.entR, R.entRt, U.oR + U.cr));
    if (U.cl < U.nL) HULL_CONSIDER(5, cand_entry(R.entL, R.entLt, U.oL + U.cl));
    if (V.cl < V.nL) HULL_CONSIDER(6, cand_entry(R.entL, R.entLt, V.oL + V.cl));
    if (V.cr < V.nR) HULL_CONSIDER(7, cand_entry(R.entR, R.entRt, V.oR + V.cr));
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
      lookup(R, U, true, T);
    } else {
      Pv = pts[V.p];
      lookup(R, V, true, T);
    }
    if (out) {
      if (nb >= cap) {
        atomicCAS(&h->err, 0, HULL_EINTERNAL);
        break;
      }
      out[nb] = Event{T.t.a, T.t.w, T.t.b, T.kind};
      out_tau[nb] = T.st;
      out_uv[nb] = make_int2(U.p, V.p);
    }
    ++nb;
  }
  return nb;
}

// Segments per merge, from the child movie lengths.
__global__ void __launch_bounds__(256) k_par_segcount(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int64_t width = int64_t(1) << P.k;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g <= P.merges;
       g += (int64_t)gridDim.x * blockDim.x) {
    if (g == P.merges || P.h->err) {
      R.segS[g] = g == P.merges ? 0 : 1;
      continue;
    }
    int64_t s = g * width, m = s + (width >> 1);
    R.segS[g] = segments_for(R.len_in[s], R.len_in[m], P.seg_events);
  }
}

__global__ void __launch_bounds__(256) k_par_segtable(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < P.merges;
       g += (int64_t)gridDim.x * blockDim.x) {
    int b = R.segBase[g], S = R.segS[g];
    for (int i = 0; i < S; ++i) R.segMerge[b + i] = (int)g;
  }
}

// Pass 1 counts each segment's bridge events; pass 2 writes them at their
// place in the merge's bridge list.
__global__ void __launch_bounds__(64) k_par_walk(ParLevel P, int write) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t > P.seg_cap) return;
  const int total = R.segBase[P.merges];
  if (t >= total) {
    if (!write) R.segCnt[t] = 0;
    return;
  }
  const int g = R.segMerge[t];
  const int first = R.segBase[g], S = R.segS[g], i = (int)(t - first);
  const int64_t width = int64_t(1) << P.k;
  const int64_t s = g * width, m = s + (width >> 1), e = std::min(s + width, P.n);
  if (P.h->err) {
    if (!write) R.segCnt[t] = 0;
    else if (i == 0) {
      R.nB[s] = 0;
      R.uv0[s] = make_int2(0, 0);
    }
    return;
  }
  if (!write) {
    R.segCnt[t] = walk_segment(R, P.h, s, m, e, i, S, nullptr, nullptr, nullptr, 0, nullptr);
    return;
  }
  int64_t off = R.segOff[t] - R.segOff[first];
  int cap = (int)(2 * (e - s) - off);
  walk_segment(R, P.h, s, m, e, i, S, R.bev + 2 * s + off, R.btau + 2 * s + off,
               R.buv + 2 * s + off, cap, i == 0 ? &R.uv0[s] : nullptr);
  if (i == 0) R.nB[s] = R.segOff[first + S] - R.segOff[first];
}

// Survival of every child event, and the number of bridge events before it.
__global__ void __launch_bounds__(256) k_par_classify(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const int k = P.k;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q <= 2 * P.n;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q == 2 * P.n || P.h->err) {
      R.surv[q] = 0;
      continue;
    }
    int64_t sb = in_block_start(q, k);
    int64_t g = sb >> k;
    if (g >= P.merges || q - 2 * sb >= R.len_in[sb]) {
      R.surv[q] = 0;
      continue;
    }
    int64_t s = g << k;
    bool isL = sb == s;
    Cand c = cand_of(R.ev_in, R.tau_in, q);
    int nb = R.nB[s];
    int j = count_before(R.pts, R.bev, R.btau, 2 * s, nb, c, R.zs);
    int2 ref = j > 0 ? R.buv[2 * s + j - 1] : R.uv0[s];
    R.surv[q] = isL ? (c.t.w < ref.x) : (c.t.w > ref.y);
    R.jb[q] = j;
  }
}

// Scatter: child survivors (indices [0, 2n)) and bridge events ([2n, 4n))
// to their places in the merged movies.
__global__ void __launch_bounds__(256) k_par_scatter(ParLevel P) {
  const ParRun& R = P.run[blockIdx.y];
  if (!R.pts) return;
  const bool err = P.h->err != 0;
  const int k = P.k;
  const int64_t n = P.n, width = int64_t(1) << k, half = width >> 1;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 4 * n;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t < 2 * n) {
      int64_t q = t;
      if (err || !R.surv[q]) continue;
      int64_t sb = in_block_start(q, k);
      int64_t s = (sb >> k) << k, m = s + half;
      bool isL = sb == s;
      Cand c = cand_of(R.ev_in, R.tau_in, q);
      int64_t pos;
      if (isL) {
        int idx = count_before(R.pts, R.ev_in, R.tau_in, 2 * m, R.len_in[m], c, R.zs);
        pos = (R.pre[q] - R.pre[2 * s]) + (R.pre[2 * m + idx] - R.pre[2 * m]) + R.jb[q];
      } else {
        int idx = count_before(R.pts, R.ev_in, R.tau_in, 2 * s, R.len_in[s], c, R.zs);
        pos = (R.pre[2 * s + idx] - R.pre[2 * s]) + (R.pre[q] - R.pre[2 * m]) + R.jb[q];
      }
      if (pos >= 2 * (std::min(s + width, n) - s)) {
        atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
        continue;
      }
      R.ev_out[2 * s + pos] = R.ev_in[q];
      R.tau_out[2 * s + pos] = c.st;
    } else {
      int64_t q = t - 2 * n;
      int64_t g = (q >> 1) >> k;
      if (g >= P.merges) continue;
      int64_t s = g << k, m = s + half, e = std::min(s + width, n);
      int64_t j = q - 2 * s;
      int nb = R.nB[s];
      if (j == 0) {
        // every merge writes its length, also after an error (then 0)
        int cnt = err ? 0 : (R.pre[2 * e] - R.pre[2 * s]) + nb;
        R.len_out[s] = cnt <= 2 * (e - s) ? cnt : 0;
        if (cnt > 2 * (e - s)) atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
        // splice the -inf chains at the -inf bridge (no kernel of this level
        // reads the -inf links after the walk)
        if (!err) {
          int2 b0 = R.uv0[s];
          R.nx0[b0.x] = b0.y;
          R.pv0[b0.y] = b0.x;
        }
      }
      if (err || j >= nb) continue;
      Cand c = cand_of(R.bev, R.btau, q);
      int iL = count_before(R.pts, R.ev_in, R.tau_in, 2 * s, R.len_in[s], c, R.zs);
      int iR = count_before(R.pts, R.ev_in, R.tau_in, 2 * m, R.len_in[m], c, R.zs);
      int64_t pos = j + (R.pre[2 * s + iL] - R.pre[2 * s]) + (R.pre[2 * m + iR] - R.pre[2 * m]);
      if (pos >= 2 * (e - s)) {
        atomicCAS(&P.h->err, 0, HULL_EINTERNAL);
        continue;
      }
      R.ev_out[2 * s + pos] = R.bev[q];
      R.tau_out[2 * s + pos] = c.st;
    }
  }
}

static unsigned blocks_for(int64_t work, int64_t cap = 8192) {
  int64_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

int32_t parallel_level(const ParLevel& P, int32_t* partials, hipStream_t s) {
  const int64_t n = P.n;
  hipLaunchKernelGGL(k_par_zero, dim3(blocks_for(n), 2), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_par_count, dim3(blocks_for(2 * n), 2), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_par_segcount, dim3(blocks_for(P.merges + 1), 2), dim3(256), 0, s, P);
  for (int r = 0; r < 2; ++r) {
    const ParRun& R = P.run[r];
    if (!R.pts) continue;
    int32_t rc = exclusive_scan_i32(R.cntR, R.offR, n, partials, s);
    if (!rc) rc = exclusive_scan_i32(R.cntL, R.offL, n, partials, s);
    if (!rc) rc = exclusive_scan_i32(R.segS, R.segBase, P.merges + 1, partials, s);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_par_fill, dim3(blocks_for(2 * n), 2), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_par_sort, dim3(blocks_for(n), 2), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_par_segtable, dim3(blocks_for(P.merges), 2), dim3(256), 0, s, P);
  const unsigned wg = (unsigned)((P.seg_cap + 1 + 63) / 64);
  hipLaunchKernelGGL(k_par_walk, dim3(wg, 2), dim3(64), 0, s, P, 0);
  for (int r = 0; r < 2; ++r) {
    const ParRun& R = P.run[r];
    if (!R.pts) continue;
    int32_t rc = exclusive_scan_i32(R.segCnt, R.segOff, P.seg_cap + 1, partials, s);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_par_walk, dim3(wg, 2), dim3(64), 0, s, P, 1);
  hipLaunchKernelGGL(k_par_classify, dim3(blocks_for(2 * n + 1), 2), dim3(256), 0, s, P);
  for (int r = 0; r < 2; ++r) {
    const ParRun& R = P.run[r];
    if (!R.pts) continue;
    int32_t rc = exclusive_scan_i32(R.surv, R.pre, 2 * n + 1, partials, s);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_par_scatter, dim3(blocks_for(4 * n), 2), dim3(256), 0, s, P);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

}  // namespace hull
