// One merge per group of G lanes (G = 8: eight merges per wavefront; G = 64:
// one), for the levels whose merges are long (the merge step of Sec. 2 and
// the kernel of Sec. 3, Fig. "kernel_variables", with the candidates of an
// iteration spread over lanes).
//
// A lane-serial merge runs its whole iteration on one lane, and the 64 lanes
// of a wave, each on its own merge, run in lockstep through the union of
// their branches.  Here a group runs one merge: its lanes 0 and 1 hold the
// next event of the left and right child movie, lanes 2..5 the four bridge
// moves (nx(u) enters, u leaves, pv(v) enters, v leaves), each recomputed by
// its own lane only when its triple changed; the earliest valid candidate is
// found by a reduction over the six lanes with the standard-part filter, and
// by exact comparisons among the candidates the filter cannot tell apart.
// The child movies come through LDS in chunks of G events, loaded by the
// whole group.  Control flow is uniform within a group.
//
// The result is the lane-serial merge's, event for event: both take, at every
// step, the earliest valid candidate in the (time, rank triple) order, which
// is a strict total order on the candidates' distinct triples.
#pragma once
#include "common.hpp"
#include "events.hpp"

#include <type_traits>

namespace hull {

// x of the lane CTRL names, through a data-parallel move (a register
// operation: no LDS round trip); CTRL: quad permutation or half-row mirror.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Minimum over each aligned group of 8 lanes, on all 8 lanes: the quad
// permutations [1,0,3,2] and [2,3,0,1], then the half-row mirror (lane i and
// lane 7 - i), which pairs the two quads.
__device__ inline double min8(double x) {
  x = fmin(x, dpp_f64<0xB1>(x));
  x = fmin(x, dpp_f64<0x4E>(x));
  return fmin(x, dpp_f64<0x141>(x));
}

// x of lane `src` of the caller's group of G lanes (src the same on every lane
// of the group): a lane read into a scalar register when the group is the
// whole wave, else a permute through LDS.
template <int G>
__device__ inline int group_bcast(int x, int src) {
  if constexpr (G == 64) return __builtin_amdgcn_readlane(x, __builtin_amdgcn_readfirstlane(src));
  else return __shfl(x, src, G);
}
template <int G>
__device__ inline double group_bcast(double x, int src) {
  if constexpr (G == 64) {
    const long long b = __double_as_longlong(x);
    const int s = __builtin_amdgcn_readfirstlane(src);
    const int lo = __builtin_amdgcn_readlane((int)b, s), hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  } else {
    return __shfl(x, src, G);
  }
}

// An event with its three ranks lowered by base (the kind bit above the
// middle rank is kept: the rank stays at least base).
__device__ __forceinline__ Event shift_event(Event E, int base) {
  E.a -= base;
  E.wk -= base;
  E.b -= base;
  return E;
}

// MODE 0: the merge's working links in the level's global working array,
// points global.  MODE 1: the working links in LDS as block-local int16 ranks
// (dynamic LDS: 256 / G merges per block x width link pairs of 4 bytes),
// loaded by the group from the -inf links.  MODE 2: links and points in LDS,
// the merge working in block-local ranks (events shifted on the way in and
// out); blocks of 64 lanes, for levels of few, long merges whose iterations
// wait on point loads (dynamic LDS: 64 / G merges x width x (4 + point
// size) bytes).
template <class PT, int G, int MODE>
__global__ void __launch_bounds__(256) k_merge_wave(LevelArgs A) {
  static_assert(G == 8 || G == 16 || G == 32 || G == 64, "lanes per merge");
  static_assert(MODE >= 0 && MODE <= 2, "link and point placement");
  constexpr int NB = MODE == 2 ? 64 : 256;  // lanes per block
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  // per group of the block: G events of each child movie
  __shared__ Event chunk[NB / G][2][G];
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  const int gshift = (threadIdx.x & 63) & ~(G - 1);  // the group's first lane in the wave
  const int64_t g0 = (blockIdx.x * (int64_t)NB + threadIdx.x) / G;
  const RunPtrs& R = A.run[blockIdx.y];
  if (!R.pts || g0 >= A.S.moff[A.S.H]) return;  // the same for every lane of the group
  const int* perm = A.perm[blockIdx.y];
  const int64_t g = perm ? perm[g0] : g0;
  const int2 se = A.S.mlist[g];
  const int64_t s = se.x, m = s + A.half, e = se.y;
  Header* h = A.h;
  if (h->err) {
    if (lane == 0) R.len_out[s] = 0;
    return;
  }
  const int nL = R.len_in[s], nR = R.len_in[m];
  if (nL < 0 || nR < 0 || nL > 2 * (m - s) || nR > 2 * (e - m)) {
    if (lane == 0) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      R.len_out[s] = 0;
    }
    return;
  }
  const int zs = R.zs;
  // ranks inside the loop are global ranks minus base
  const int base = MODE == 2 ? (int)s : 0;
  using LK = typename std::conditional<
      MODE == 2, LdsLinks<short, 1>,
      typename std::conditional<MODE == 1, LdsLinksShifted<short>, GlobalLinks>::type>::type;
  LK lk;
  const PT* pts;
  if constexpr (MODE >= 1) {
    if (e - s > A.width || A.width > 32767) {
      if (lane == 0) {
        atomicCAS(&h->err, 0, HULL_EINTERNAL);
        R.len_out[s] = 0;
      }
      return;
    }
    lk.p = (LinkPair<short>*)dyn_lds + (int64_t)grp * A.width;
    if constexpr (MODE == 2) {
      PT* P = (PT*)((LinkPair<short>*)dyn_lds + (int64_t)(NB / G) * A.width) + (int64_t)grp * A.width;
      const PT* src = (const PT*)R.pts + s;
      for (int j = lane; j < (int)(e - s); j += G) {
        P[j] = src[j];
        const int pv = R.pv0[s + j], nx = R.nx0[s + j];
        lk.set(j, pv == kNil ? kNil : pv - base, nx == kNil ? kNil : nx - base);
      }
      pts = P;
    } else {
      lk.base = (int)s;
      for (int j = lane; j < (int)(e - s); j += G) lk.set((int)s + j, R.pv0[s + j], R.nx0[s + j]);
      pts = (const PT*)R.pts;
    }
    __builtin_amdgcn_wave_barrier();
  } else {
    lk.p = R.lk;
    pts = (const PT*)R.pts;
  }
  const Event* Lev = R.ev_in + 2 * s;
  const Event* Rev = R.ev_in + 2 * m;
  Event* out = R.ev_out + 2 * s;
  const int64_t cap = 2 * (e - s);
  Event* Lc = chunk[grp][0];
  Event* Rc = chunk[grp][1];

  // 1. bridge at t = -inf: every lane takes the same walk (the working links
  // hold the -inf links at the start of the merge)
  int u = (int)(m - base) - 1, v = (int)(m - base);
  {
    PT Pu = pts[u], Pv = pts[v];
    for (int guard = 0;; ++guard) {
      if (guard > 2 * (e - s) + 4) {
        if (lane == 0) {
          atomicCAS(&h->err, 0, HULL_EINTERNAL);
          R.len_out[s] = 0;
        }
        return;
      }
      int w = lk.get(v).y;
      if (w != kNil) {
        const PT Pw = pts[w];
        if (d_sign(Pu, Pv, Pw) < 0) {
          v = w;
          Pv = Pw;
          continue;
        }
      }
      w = lk.get(u).x;
      if (w != kNil) {
        const PT Pw = pts[w];
        if (d_sign(Pw, Pu, Pv) < 0) {
          u = w;
          Pu = Pw;
          continue;
        }
      }
      break;
    }
  }
  const int u0 = u, v0 = v;

  // 2. event loop.  Uniform state: u, v and their working links, the last
  // event T, the child cursors.  Lane state (lanes 0..5): the lane's
  // candidate, whether it exists and is after T.
  int pu, nu, pvv, nv;
  {
    const int2 lu = lk.get(u), lv = lk.get(v);
    pu = lu.x;
    nu = lu.y;
    pvv = lv.x;
    nv = lv.y;
  }
  bool haveT = false;
  Cand T;
  T.t = Tri{-1, -1, -1};
  T.st = 0.0;
  T.kind = 0;
  Cand c;
  c.t = Tri{-1, -1, -1};
  c.st = 0.0;
  c.kind = 0;
  bool valid = false;
  unsigned dirty = 0xF;  // bridge lanes 2..5 whose triple changed
  int i = 0, j = 0, k = 0;
  if (lane < nL) Lc[lane] = shift_event(Lev[lane], base);
  if (lane < nR) Rc[lane] = shift_event(Rev[lane], base);
  __builtin_amdgcn_wave_barrier();
  const int64_t iter_cap = (int64_t)nL + nR + 4 * (e - s) + 16;
  for (int64_t it = 0;; ++it) {
    if (it > iter_cap) {
      if (lane == 0) atomicCAS(&h->err, 0, HULL_EINTERNAL);
      break;
    }
    // the lanes' candidates
    if (lane < 2) {
      const int q = lane == 0 ? i : j;
      valid = q < (lane == 0 ? nL : nR);
      if (valid) {
        const Event E = (lane == 0 ? Lc : Rc)[q % G];
        c.t = Tri{E.a, E.w(), E.b};
        c.kind = E.kind();
        c.st = (double)E.t;
      }
    } else if (lane < 6 && ((dirty >> (lane - 2)) & 1u)) {
      int a, w, b;
      if (lane == 2) { a = u; w = nu; b = v; }
      else if (lane == 3) { a = pu; w = u; b = v; }
      else if (lane == 4) { a = u; w = pvv; b = v; }
      else { a = u; w = v; b = nv; }
      valid = (lane == 2 ? nu : lane == 3 ? pu : lane == 4 ? pvv : nv) != kNil;
      if (valid) {
        c = make_cand(pts, a, w, b, pts[a], pts[w], pts[b], (lane == 2 || lane == 4) ? 1 : 0, zs);
        valid = !haveT || ev_cmp(pts, c, T, zs) > 0;
      }
    }
    dirty = 0;
    // the earliest valid candidate: the filter's minimum when every other
    // valid candidate is known to be later; else exact comparisons
    const bool mine = lane < 6 && valid;
    const bool num = mine && c.st == c.st;
    // (lanes 0..7 of the group hold the minimum; only lanes 0..5 use it)
    const double mn = min8(num ? c.st : __builtin_inf());
    const bool amb = mine && (!num || !(c.st - mn > 0x1p-23 * (fabs(c.st) + fabs(mn))));
    const uint64_t mask = (__ballot(amb) >> gshift) & 0x3Full;
    if (!mask) break;
    int win = __builtin_ctzll(mask);
    if (mask & (mask - 1)) {
      // two or more candidates the filter cannot order: a tournament over
      // them, on every lane alike
      for (uint64_t rest = mask & (mask - 1); rest; rest &= rest - 1) {
        const int x = __builtin_ctzll(rest);
        Cand cx, cw;
        cx.t = Tri{__shfl(c.t.a, x, G), __shfl(c.t.w, x, G), __shfl(c.t.b, x, G)};
        cx.st = __shfl(c.st, x, G);
        cx.kind = __shfl(c.kind, x, G);
        cw.t = Tri{__shfl(c.t.a, win, G), __shfl(c.t.w, win, G), __shfl(c.t.b, win, G)};
        cw.st = __shfl(c.st, win, G);
        cw.kind = __shfl(c.kind, win, G);
        if (ev_cmp(pts, cx, cw, zs) < 0) win = x;
      }
    }
    const int ba = group_bcast<G>(c.t.a, win), bw = group_bcast<G>(c.t.w, win),
              bb = group_bcast<G>(c.t.b, win);
    const int bk = group_bcast<G>(c.kind, win);
    const double bs = group_bcast<G>(c.st, win);
    T.t = Tri{ba, bw, bb};
    T.st = bs;
    T.kind = bk;
    haveT = true;
    bool emit;
    if (win <= 1) {
      emit = win == 0 ? (bw < u) : (bw > v);
      // the child's next event; a new chunk when this one is used up
      const int q = win == 0 ? ++i : ++j;
      const int nq = win == 0 ? nL : nR;
      if (q % G == 0 && q < nq) {
        __builtin_amdgcn_wave_barrier();
        if (q + lane < nq) (win == 0 ? Lc : Rc)[lane] = shift_event((win == 0 ? Lev : Rev)[q + lane], base);
        __builtin_amdgcn_wave_barrier();
      }
      // the event sets nx(a) and pv(b) (and, inserting w, both links of w);
      // every lane stores the same values, so that each lane's later loads
      // follow its own stores
      const int na = bk ? bw : bb, pb = bk ? bw : ba;
      lk.set_nx(ba, na);
      lk.set_pv(bb, pb);
      if (bk) lk.set(bw, ba, bb);
      if (ba == u) { nu = na; dirty |= 1u; }
      if (bb == u) { pu = pb; dirty |= 2u; }
      if (bb == v) { pvv = pb; dirty |= 4u; }
      if (ba == v) { nv = na; dirty |= 8u; }
    } else {
      emit = true;
      if (win == 2 || win == 3) {
        u = win == 2 ? nu : pu;
        const int2 l = lk.get(u);
        pu = l.x;
        nu = l.y;
      } else {
        v = win == 4 ? pvv : nv;
        const int2 l = lk.get(v);
        pvv = l.x;
        nv = l.y;
      }
      dirty = 0xF;
    }
    if (emit) {
      if (k >= cap) {
        if (lane == 0) atomicCAS(&h->err, 0, HULL_EINTERNAL);
        break;
      }
      if (lane == 0) out[k] = make_event(ba + base, bw + base, bb + base, bk, bs);
      ++k;
    }
  }
  // 3. splice the -inf chains
  if (lane == 0) {
    R.nx0[u0 + base] = v0 + base;
    R.pv0[v0 + base] = u0 + base;
    R.len_out[s] = k;
  }
}

}  // namespace hull
