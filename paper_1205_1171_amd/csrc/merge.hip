// Bottom-up merge levels of the kinetic hull (Sec. 2: the movie array and the
// merge step; Sec. 3: Fig. "main_loop_figure", the level loop with ping-pong
// event arrays, and Fig. "kernel_variables", the block offsets of a merge).
//
// Movie of a block [s, e) of ranks: its events, time-ordered, stored at slots
// [2s, 2s + len) of the level's event array (at most 2 events per point, the
// paper's two slots per point).  An event is the face (a, w, b) whose middle
// vertex w enters or leaves the chain, plus the standard part of its time.
//
// Unlike the paper (a movie of bare point indices, with the point's own
// prev/next links replayed and rewound), every event here carries its face.
// The merge then needs no rewind pass: the -inf chains live in their own link
// arrays (pv0/nx0), merging two of them is one splice at the -inf bridge, and
// the working links (pv/nx) of each level start as a copy of them.
//
// Merge of L = [s, m) and R = [m, e) (the kinetic bridge walk):
//   1. bridge at t = -inf: u = m-1, v = m, walk to the lower common tangent of
//      the two xy chains;
//   2. event loop: candidates are the next L event, the next R event and the
//      four bridge moves (nx(u) enters, u leaves, pv(v) enters, v leaves);
//      take the earliest strictly after the last event in (time, rank
//      triple) order; L events left of u and R events right of v go to the
//      output, every child event updates its child's chain, bridge moves are
//      output events of the merged chain;
//   3. splice the -inf chains at the -inf bridge.
#include <stdlib.h>

#include <algorithm>

#include "common.hpp"
#include "events.hpp"
#include "merge_wave.hpp"

namespace hull {

// The merge of blocks [s, m) and [m, e) of the arrays pts and lk (working
// links), whose index i holds the point of rank i + base: base = 0 for the
// global arrays, the block start for a block staged in LDS.  Child events
// (Lev, Rev), the merged movie (out) and the -inf link arrays (pv0, nx0) are
// global and in global ranks.  Returns the merged movie's length, -1 after an
// internal error.  kInline: which comparisons take the mid tier inline rather
// than as a call (0 none, 1 the bridge moves against the last event, 2 all):
// inline costs registers, a call costs the wave a round trip whenever any of
// its lanes meets a tie of the standard parts.
template <int kInline, class PT, class LK>
__device__ __forceinline__ int merge_core(const PT* pts, LK lk, int* pv0, int* nx0, int base,
                          const Event* Lev, int nL, const Event* Rev, int nR, Event* out,
                          Header* h, int64_t s, int64_t m, int64_t e, int zs) {
  const int64_t cap = 2 * (e - s);

  // 1. bridge at t = -inf
  int u = (int)m - 1, v = (int)m;
  PT Pu = pts[u], Pv = pts[v];
  for (int guard = 0;; ++guard) {
    if (guard > 2 * (e - s) + 4) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      return -1;
    }
    int w = nx0[v + base];
    if (w != kNil) {
      w -= base;
      PT Pw = pts[w];
      if (d_sign(Pu, Pv, Pw) < 0) {
        v = w;
        Pv = Pw;
        continue;
      }
    }
    w = pv0[u + base];
    if (w != kNil) {
      w -= base;
      PT Pw = pts[w];
      if (d_sign(Pw, Pu, Pv) < 0) {
        u = w;
        Pu = Pw;
        continue;
      }
    }
    break;
  }
  const int u0 = u, v0 = v;

  // 2. event loop.  Candidates: the next L event, the next R event and the
  // four bridge moves: nx(u) enters (u, nx u, v), u leaves (pv u, u, v),
  // pv(v) enters (u, pv v, v), v leaves (u, v, nx v).  A child event is
  // always later than the last event T (it follows T in its own movie, or T
  // was chosen before it), so only the bridge moves are checked against T.
  // The bridge moves, their validity (strictly after T) and the earliest of
  // them depend only on u, v and the four links, so they are recomputed only
  // when one of those changes; a valid move not taken stays after T, an
  // invalid one stays before it.
  int i = 0, j = 0, k = 0;
  bool haveT = false;
  Cand T;
  T.t = Tri{-1, -1, -1};
  T.st = 0.0;
  T.kind = 0;
  int nu, pu, pvv, nv;
  {
    const int2 lu = lk.get(u), lv = lk.get(v);
    pu = lu.x;
    nu = lu.y;
    pvv = lv.x;
    nv = lv.y;
  }
  // bridge best: slot (2..5, -1 = none) and its standard part
  int bbi = -1;
  double bbs = 0.0;
  double st2 = 0.0, st3 = 0.0, st4 = 0.0, st5 = 0.0;
  bool ok2 = false, ok3 = false, ok4 = false, ok5 = false;
  unsigned dirty = 0xF;
  // the next event of each child, loaded one iteration ahead
  int4 EL = make_int4(0, 0, 0, 0), ER = make_int4(0, 0, 0, 0);
  double tL = 0.0, tR = 0.0;
  // events hold global ranks: shifted to the arrays' indexing
  const int4 shift = make_int4(base, base, base, 0);
  // a child event as (a, w, b, kind) in the arrays' indexing and its time
  auto load_ev = [&](const Event* E, int4& X, double& t) {
    const int4 raw = *(const int4*)E;
    X = make_int4(raw.x - shift.x, (raw.y & 0x7fffffff) - shift.y, raw.z - shift.z,
                  (int)((unsigned)raw.y >> 31));
    t = (double)__int_as_float(raw.w);
  };
  if (nL > 0) load_ev(&Lev[0], EL, tL);
  if (nR > 0) load_ev(&Rev[0], ER, tR);
  const int64_t iter_cap = (int64_t)nL + nR + 4 * (e - s) + 16;
  for (int64_t it = 0;; ++it) {
    if (it > iter_cap) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      break;
    }
    if (dirty) {
#define HULL_SLOT(BIT, OK, ST, LINK, A, W, B, PA, PW, PB, KIND)                  \
  if (dirty & (BIT)) {                                                         \
    OK = (LINK) != kNil;                                                       \
    if (OK) {                                                                  \
      const PT pa_ = (PA), pw_ = (PW), pb_ = (PB);                             \
      const Cand c_ = make_cand(pts, A, W, B, pa_, pw_, pb_, KIND, zs);        \
      ST = c_.st;                                                              \
      OK = !haveT || (kInline >= 1 ? ev_cmp_half(pts, c_, pa_, pw_, pb_, T, zs) \
                                   : ev_cmp(pts, c_, T, zs)) > 0;              \
    }                                                                          \
  }
      HULL_SLOT(1u, ok2, st2, nu, u, nu, v, Pu, pts[nu], Pv, 1)
      HULL_SLOT(2u, ok3, st3, pu, pu, u, v, pts[pu], Pu, Pv, 0)
      HULL_SLOT(4u, ok4, st4, pvv, u, pvv, v, Pu, pts[pvv], Pv, 1)
      HULL_SLOT(8u, ok5, st5, nv, u, v, nv, Pu, Pv, pts[nv], 0)
#undef HULL_SLOT
      // earliest valid bridge move, slots in a fixed order
      bbi = -1;
      int ba = 0, bw = 0, bb = 0, bk = 0;
#define HULL_BRIDGE(IDX, OK, ST, A, W, B, KIND)                            \
  if (OK) {                                                              \
    bool take_ = bbi < 0;                                                \
    if (!take_) {                                                        \
      Cand x_, y_;                                                       \
      x_.t = Tri{A, W, B};                                               \
      x_.st = ST;                                                        \
      x_.kind = KIND;                                                    \
      y_.t = Tri{ba, bw, bb};                                            \
      y_.st = bbs;                                                       \
      y_.kind = bk;                                                      \
      take_ = ev_cmp<(kInline >= 2)>(pts, x_, y_, zs) < 0;                   \
    }                                                                    \
    if (take_) {                                                         \
      bbi = (IDX);                                                       \
      ba = A;                                                            \
      bw = W;                                                            \
      bb = B;                                                            \
      bk = KIND;                                                         \
      bbs = ST;                                                          \
    }                                                                    \
  }
      HULL_BRIDGE(2, ok2, st2, u, nu, v, 1)
      HULL_BRIDGE(3, ok3, st3, pu, u, v, 0)
      HULL_BRIDGE(4, ok4, st4, u, pvv, v, 1)
      HULL_BRIDGE(5, ok5, st5, u, v, nv, 0)
#undef HULL_BRIDGE
      dirty = 0;
    }
    // the bridge best as a candidate
    int bi = -1, ba = 0, bw = 0, bb = 0, bk = 0;
    double bs = bbs;
    if (bbi >= 0) {
      bi = bbi;
      if (bbi == 2) { ba = u; bw = nu; bb = v; bk = 1; }
      else if (bbi == 3) { ba = pu; bw = u; bb = v; bk = 0; }
      else if (bbi == 4) { ba = u; bw = pvv; bb = v; bk = 1; }
      else { ba = u; bw = v; bb = nv; bk = 0; }
    }
#define HULL_CHILD(IDX, E_, T_)                                            \
  {                                                                      \
    bool take_ = bi < 0;                                                 \
    if (!take_) {                                                        \
      Cand x_, y_;                                                       \
      x_.t = Tri{(E_).x, (E_).y, (E_).z};                                \
      x_.st = (T_);                                                      \
      x_.kind = 0;                                                       \
      y_.t = Tri{ba, bw, bb};                                            \
      y_.st = bs;                                                        \
      y_.kind = 0;                                                       \
      take_ = ev_cmp<(kInline >= 2)>(pts, x_, y_, zs) < 0;                   \
    }                                                                    \
    if (take_) {                                                         \
      bi = (IDX);                                                        \
      ba = (E_).x;                                                       \
      bw = (E_).y;                                                       \
      bb = (E_).z;                                                       \
      bs = (T_);                                                         \
    }                                                                    \
  }
    if (i < nL) HULL_CHILD(0, EL, tL)
    if (j < nR) HULL_CHILD(1, ER, tR)
#undef HULL_CHILD
    if (bi < 0) break;
    // the kind of the chosen event, from its source once the choice is made
    // (not carried through the selection: hipcc for gfx950 has dropped the
    // condition on such a carried field, taking the old value for lanes that
    // switch candidates)
    if (bi == 0) bk = EL.w;
    else if (bi == 1) bk = ER.w;
    else bk = (bi == 2 || bi == 4) ? 1 : 0;
    T.t = Tri{ba, bw, bb};
    T.st = bs;
    T.kind = bk;
    haveT = true;
    bool emit = false;
    if (bi <= 1) {
      // the child's next event, issued now so that its latency overlaps the
      // rest of this iteration
      if (bi == 0) {
        if (++i < nL) load_ev(&Lev[i], EL, tL);
      } else {
        if (++j < nR) load_ev(&Rev[j], ER, tR);
      }
      emit = bi == 0 ? (bw < u) : (bw > v);
      // the event sets nx(a) and pv(b) (and, inserting w, both links of w)
      const int na = bk ? bw : bb, pb = bk ? bw : ba;
      lk.set_nx(ba, na);
      lk.set_pv(bb, pb);
      if (bk) lk.set(bw, ba, bb);  // the inserted point's links
      // links of u and v it changed (w is never u or v when inserted)
      unsigned d = 0;
      if (ba == u) { nu = na; d |= 1u; }
      if (bb == u) { pu = pb; d |= 2u; }
      if (bb == v) { pvv = pb; d |= 4u; }
      if (ba == v) { nv = na; d |= 8u; }
      dirty = d;
    } else {
      emit = true;
      if (bi == 2 || bi == 3) {
        u = bi == 2 ? nu : pu;
        Pu = pts[u];
        const int2 l = lk.get(u);
        pu = l.x;
        nu = l.y;
      } else {
        v = bi == 4 ? pvv : nv;
        Pv = pts[v];
        const int2 l = lk.get(v);
        pvv = l.x;
        nv = l.y;
      }
      dirty = 0xF;
    }
    if (emit) {
      if (k >= cap) {
        atomicCAS(&h->err, 0, HULL_EINTERNAL);
        break;
      }
      out[k] = make_event(ba + base, bw + base, bb + base, bk, bs);
      ++k;
    }
  }
  // 3. splice the -inf chains
  nx0[u0 + base] = v0 + base;
  pv0[v0 + base] = u0 + base;
  return k;
}

template <class PT>
__device__ void merge_one(const RunPtrs& R, Header* h, int64_t s, int64_t m, int64_t e) {
  const int nL = R.len_in[s], nR = R.len_in[m];
  if (nL < 0 || nR < 0 || nL > 2 * (m - s) || nR > 2 * (e - m)) {
    atomicCAS(&h->err, 0, HULL_EINTERNAL);
    R.len_out[s] = 0;
    return;
  }
  const int k = merge_core<1>((const PT*)R.pts, GlobalLinks{R.lk}, R.pv0, R.nx0, 0, R.ev_in + 2 * s, nL, R.ev_in + 2 * m, nR,
                           R.ev_out + 2 * s, h, s, m, e, R.zs);
  R.len_out[s] = k < 0 ? 0 : k;
}

template <class PT>
__global__ void __launch_bounds__(256) k_merge_level(LevelArgs A) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const RunPtrs& R = A.run[blockIdx.y];
  if (!R.pts || t >= A.S.moff[A.S.H]) return;
  const int* perm = A.perm[blockIdx.y];
  const int64_t g = perm ? perm[t] : t;
  const int2 se = A.S.mlist[g];
  const int64_t s = se.x, m = s + A.half, e = se.y;
  // After an error the movies are empty, so that every later kernel still
  // reads lengths that were written.
  if (A.h->err) {
    R.len_out[s] = 0;
    return;
  }
  merge_one<PT>(R, A.h, s, m, e);
}

// Lane-serial levels from this one on list their merges in work order; below
// it the merge kernel moves about as many bytes as the memory system serves
// (L2 misses), and the order would only add its own launches.  A level with
// fewer merges than one wave per SIMD (256 CUs x 4 SIMDs x 64 lanes over two
// runs) keeps the plain order: with the waves already spread one to a SIMD,
// packing the longest merges into one wave only adds up their divergent
// branches.
constexpr int kOrderFromLevel = 6;
constexpr int64_t kOrderMinMerges = 32768;
// Lane-group levels of at most this many merges (both runs) hold the merge's
// points in LDS as well as its links.
constexpr int kPtsLdsMerges = 1024;

// Bytes of LDS one workgroup may use on the current device (looked up once
// per device).
static int64_t max_lds_bytes() {
  static int64_t cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 65536;
    cached[dev] = v;
  }
  return cached[dev];
}

// Work order of a level's merges.  The lanes of a wavefront run their merges
// in lockstep, so a wave lasts as long as its longest merge; listing the
// merges by child event count, largest first, gives each wave merges of
// about the same length (and starts the longest first).  A counting sort:
// histogram, scan, placement; the order inside a count is arbitrary and
// changes nothing but timing (every merge writes only its own block).
__device__ __forceinline__ int work_bin(const LevelArgs& A, const RunPtrs& R, int64_t g) {
  const int64_t s = A.S.mlist[g].x;
  int w = R.len_in[s] + R.len_in[s + A.half];
  w = w < 0 ? 0 : (w > kWorkBins - 1 ? kWorkBins - 1 : w);
  return kWorkBins - 1 - w;
}

__global__ void __launch_bounds__(256) k_work_clear(LevelArgs A) {
  if (!A.run[blockIdx.y].pts) return;
  for (int i = threadIdx.x; i < kWorkBins; i += blockDim.x) A.wbins[blockIdx.y][i] = 0;
}

__global__ void __launch_bounds__(256) k_work_hist(LevelArgs A) {
  __shared__ int hist[kWorkBins];
  const RunPtrs& R = A.run[blockIdx.y];
  const int64_t M = A.S.moff[A.S.H];
  if (!R.pts || blockIdx.x * (int64_t)blockDim.x >= M) return;
  for (int i = threadIdx.x; i < kWorkBins; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < M) atomicAdd(&hist[work_bin(A, R, g)], 1);
  __syncthreads();
  int* bins = A.wbins[blockIdx.y];
  for (int i = threadIdx.x; i < kWorkBins; i += blockDim.x)
    if (hist[i]) atomicAdd(&bins[i], hist[i]);
}

// One wavefront per run: the histogram becomes each bin's first position.
__global__ void __launch_bounds__(64) k_work_scan(LevelArgs A) {
  if (!A.run[blockIdx.y].pts) return;
  int* bins = A.wbins[blockIdx.y];
  constexpr int per = kWorkBins / 64;
  int v[per];
  int sum = 0;
#pragma unroll
  for (int j = 0; j < per; ++j) {
    v[j] = bins[threadIdx.x * per + j];
    sum += v[j];
  }
  int incl = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if ((int)threadIdx.x >= o) incl += y;
  }
  int run = incl - sum;
#pragma unroll
  for (int j = 0; j < per; ++j) {
    bins[threadIdx.x * per + j] = run;
    run += v[j];
  }
}

__global__ void __launch_bounds__(256) k_work_place(LevelArgs A) {
  __shared__ int cnt[kWorkBins];
  __shared__ int base[kWorkBins];
  const RunPtrs& R = A.run[blockIdx.y];
  const int64_t M = A.S.moff[A.S.H];
  if (!R.pts || blockIdx.x * (int64_t)blockDim.x >= M) return;
  for (int i = threadIdx.x; i < kWorkBins; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int b = -1, local = 0;
  if (g < M) {
    b = work_bin(A, R, g);
    local = atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  int* cur = A.wbins[blockIdx.y];
  for (int i = threadIdx.x; i < kWorkBins; i += blockDim.x)
    base[i] = cnt[i] ? atomicAdd(&cur[i], cnt[i]) : 0;
  __syncthreads();
  if (b >= 0) A.perm[blockIdx.y][base[b] + local] = (int)g;
}

// The lowest levels with each lane's block (points and working links) staged
// in LDS: the merge's scattered point and link accesses then stay on chip
// (global memory serves only the sequential child events and the output).
// One wavefront per workgroup; a lane touches only its own LDS slice.
template <class PT, int W>
__global__ void __launch_bounds__(64) k_merge_level_lds(LevelArgs A) {
  __shared__ PT sp[64 * W];
  __shared__ int2 sl[64 * W];
  const RunPtrs& R = A.run[blockIdx.y];
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (!R.pts || g >= A.S.moff[A.S.H]) return;
  const int2 se = A.S.mlist[g];
  const int64_t s = se.x, m = s + A.half, e = se.y;
  if (A.h->err || e - s > W) {
    if (!A.h->err) atomicCAS(&A.h->err, 0, HULL_EINTERNAL);
    R.len_out[s] = 0;
    return;
  }
  const int nL = R.len_in[s], nR = R.len_in[m];
  if (nL < 0 || nR < 0 || nL > 2 * (m - s) || nR > 2 * (e - m)) {
    atomicCAS(&A.h->err, 0, HULL_EINTERNAL);
    R.len_out[s] = 0;
    return;
  }
  PT* P = sp + threadIdx.x * W;
  const PT* pts = (const PT*)R.pts;
  int2* K = sl + threadIdx.x * W;
  const int w = (int)(e - s), b = (int)s;
  for (int j = 0; j < w; ++j) {
    P[j] = pts[s + j];
    const int pv = R.pv0[s + j], nx = R.nx0[s + j];
    K[j] = make_int2(pv == kNil ? kNil : pv - b, nx == kNil ? kNil : nx - b);
  }
  const int k = merge_core<2>(P, GlobalLinks{K}, R.pv0, R.nx0, b, R.ev_in + 2 * s, nL, R.ev_in + 2 * m, nR,
                           R.ev_out + 2 * s, A.h, 0, m - s, e - s, R.zs);
  R.len_out[s] = k < 0 ? 0 : k;
}

// Lane-serial levels with each lane's working links in LDS as block-local
// int8 ranks (blocks of up to kLinkLdsLane points, the lanes of a wave
// interleaved): the merge's scattered link reads and writes stay on chip, and
// the level needs no copy of the -inf links into a global working array.
// Points, child events and the merged movie stay in global memory.  Dynamic
// LDS: width x 64 link pairs of 2 bytes.
template <class PT>
__global__ void __launch_bounds__(64) k_merge_level_lk(LevelArgs A) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const RunPtrs& R = A.run[blockIdx.y];
  if (!R.pts || t >= A.S.moff[A.S.H]) return;
  const int* perm = A.perm[blockIdx.y];
  const int64_t g = perm ? perm[t] : t;
  const int2 se = A.S.mlist[g];
  const int64_t s = se.x, m = s + A.half, e = se.y;
  if (A.h->err) {
    R.len_out[s] = 0;
    return;
  }
  const int nL = R.len_in[s], nR = R.len_in[m];
  if (nL < 0 || nR < 0 || nL > 2 * (m - s) || nR > 2 * (e - m) || e - s > A.width ||
      A.width > kLinkLdsLane) {
    atomicCAS(&A.h->err, 0, HULL_EINTERNAL);
    R.len_out[s] = 0;
    return;
  }
  const LdsLinks<signed char, 64> K{(LinkPair<signed char>*)dyn_lds + threadIdx.x};
  const int w = (int)(e - s), b = (int)s;
  auto local = [b](int r) { return r == kNil ? -1 : r - b; };
  int j = 0;
  if ((s & 3) == 0) {  // 16-byte loads of four links at a time
    const int4* p4 = (const int4*)(R.pv0 + s);
    const int4* n4 = (const int4*)(R.nx0 + s);
    for (; j + 4 <= w; j += 4) {
      const int4 pv = p4[j >> 2], nx = n4[j >> 2];
      K.set(j, local(pv.x), local(nx.x));
      K.set(j + 1, local(pv.y), local(nx.y));
      K.set(j + 2, local(pv.z), local(nx.z));
      K.set(j + 3, local(pv.w), local(nx.w));
    }
  }
  for (; j < w; ++j) K.set(j, local(R.pv0[s + j]), local(R.nx0[s + j]));
  const int k = merge_core<1>((const PT*)R.pts + s, K, R.pv0, R.nx0, b, R.ev_in + 2 * s, nL,
                           R.ev_in + 2 * m, nR, R.ev_out + 2 * s, A.h, 0, m - s, e - s, R.zs);
  R.len_out[s] = k < 0 ? 0 : k;
}

// Level 1: the merge of two single points has no events (neither chain has a
// link to move along), so it is the splice of their -inf chains and an empty
// movie.  The same result as the merge loop, without its machinery.
__global__ void __launch_bounds__(256) k_merge_level1(LevelArgs A) {
  const RunPtrs& R = A.run[blockIdx.y];
  if (!R.pts) return;
  const int64_t M = A.S.moff[A.S.H];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < M;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int2 se = A.S.mlist[g];
    const int s = se.x;
    if (A.h->err || se.y - se.x != 2 || R.len_in[s] != 0 || R.len_in[s + 1] != 0) {
      if (!A.h->err) atomicCAS(&A.h->err, 0, HULL_EINTERNAL);
      R.len_out[s] = 0;
      continue;
    }
    R.nx0[s] = s + 1;
    R.pv0[s + 1] = s;
    R.len_out[s] = 0;
  }
}

// The unpaired trailing block of a hull at this level keeps its movie: copy
// it across (a hull already complete keeps its movie where it is).
__global__ void __launch_bounds__(256) k_passthrough(LevelArgs A) {
  const RunPtrs& R = A.run[blockIdx.y];
  if (!R.pts) return;
  const int count = A.S.toff[A.S.H];
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const int64_t s = A.S.tlist[t];
    int len = R.len_in[s];
    if (A.h->err || len < 0 || len > 2 * A.half) len = 0;
    for (int q = threadIdx.x; q < len; q += blockDim.x) R.ev_out[2 * s + q] = R.ev_in[2 * s + q];
    if (threadIdx.x == 0) R.len_out[s] = len;
  }
}

__global__ void __launch_bounds__(256) k_init_links(int* pv0, int* nx0, int* len, int* claimR,
                                                    int* claimL, int64_t n) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    pv0[p] = kNil;
    nx0[p] = kNil;
    len[p] = 0;
    claimR[p] = 0;
    claimL[p] = 0;
  }
}

__global__ void __launch_bounds__(256) k_copy_links(const int* __restrict__ pv0,
                                                    const int* __restrict__ nx0,
                                                    int2* __restrict__ lk, int64_t n) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    lk[p] = make_int2(pv0[p], nx0[p]);
}

__device__ __forceinline__ int dev_levels(int64_t n) {
  int L = 0;
  while ((int64_t(1) << L) < n) ++L;
  return L;
}

// Level schedule: per hull, merges = floor(blocks / 2) and one trailing
// block when the number of blocks is odd and above one.
__global__ void __launch_bounds__(256) k_sched_count(Sched S, int k, int* mcnt, int* tcnt) {
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h <= S.H;
       h += (int64_t)gridDim.x * blockDim.x) {
    if (h == S.H) {
      mcnt[h] = 0;
      tcnt[h] = 0;
      continue;
    }
    const int64_t nh = S.off[h + 1] - S.off[h];
    const int64_t w = int64_t(1) << (k - 1);
    const int64_t nb = (nh + w - 1) >> (k - 1);
    mcnt[h] = (int)(nb >> 1);
    tcnt[h] = (nb > 1 && (nb & 1)) ? 1 : 0;
  }
}

__global__ void __launch_bounds__(256) k_sched_fill(Sched S, int k) {
  const int merges = S.moff[S.H];
  const int64_t width = int64_t(1) << k, w = width >> 1;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < merges;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int h = find_owner(S.moff, (int)S.H, g);
    const int64_t s = S.off[h] + (g - S.moff[h]) * width;
    const int64_t e = s + width < S.off[h + 1] ? s + width : S.off[h + 1];
    S.mlist[g] = make_int2((int)s, (int)e);
  }
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < S.H;
       h += (int64_t)gridDim.x * blockDim.x) {
    if (S.toff[h + 1] > S.toff[h]) {
      const int64_t nh = S.off[h + 1] - S.off[h];
      const int64_t nb = (nh + w - 1) >> (k - 1);
      S.tlist[S.toff[h]] = (int)(S.off[h] + (nb - 1) * w);
    }
  }
}

// The same schedule for a single hull of n points in one launch (no scans:
// merge g covers [g 2^k, min((g + 1) 2^k, n))).
__global__ void __launch_bounds__(256) k_sched_single(Sched S, int k, int64_t n) {
  const int64_t width = int64_t(1) << k, w = width >> 1;
  const int64_t nb = (n + w - 1) >> (k - 1);
  const int64_t merges = nb >> 1;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < merges;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = g * width;
    S.mlist[g] = make_int2((int)s, (int)(s + width < n ? s + width : n));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int t = (nb > 1 && (nb & 1)) ? 1 : 0;
    S.moff[0] = 0;
    S.moff[1] = (int)merges;
    S.toff[0] = 0;
    S.toff[1] = t;
    if (t) S.tlist[0] = (int)((nb - 1) * w);
  }
}

__global__ void k_set_off1(int64_t* off, int64_t n) {
  if (threadIdx.x == 0) {
    off[0] = 0;
    off[1] = n;
  }
}

// Faces: every hull's final movies sit in the buffer of its own last level.
struct ExtractArgs {
  Sched S;
  const Event* ev[2][2];  // [run][buffer]
  const int* len[2][2];
  const void* pts;  // int4 or WPt
  int* fcnt;  // [H + 1], scanned in place into face offsets
  int32_t* faces;
  int64_t cap;
  int64_t* face_off;  // [H + 1] output (may be null)
  int64_t* info;
  const Header* h;
};

__global__ void __launch_bounds__(256) k_face_count(ExtractArgs X) {
  const Sched& S = X.S;
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h <= S.H;
       h += (int64_t)gridDim.x * blockDim.x) {
    int F = 0;
    if (h < S.H) {
      const int64_t o = S.off[h], nh = S.off[h + 1] - o;
      if (nh >= 3) {
        const int b = dev_levels(nh) & 1;
        if (X.ev[0][b]) F += X.len[0][b][o];
        if (X.ev[1][b]) F += X.len[1][b][o];
      }
    }
    if (S.H == 1) {  // offsets [0, F] directly, no scan
      if (h == 0) {
        X.fcnt[0] = 0;
        X.fcnt[1] = F;
      }
    } else {
      X.fcnt[h] = F;
    }
  }
}

// Event (a, w, b) gives the face with the middle vertex w; an insertion has
// D(a, w, b) < 0, a deletion D > 0.  Lower faces need D < 0 for an outward
// orientation, upper faces D > 0.  Indices are the points' own (within their
// hull).
template <class PT>
__global__ void __launch_bounds__(256) k_extract(ExtractArgs X) {
  const PT* pts = (const PT*)X.pts;
  const Sched& S = X.S;
  const int64_t total = X.fcnt[S.H];
  const bool over = total > X.cap || total < 0;
  const int err = X.h->err;
  const int64_t F = (over || err) ? 0 : total;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < F;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int h = find_owner(X.fcnt, (int)S.H, t);
    const int64_t o = S.off[h];
    const int b = dev_levels(S.off[h + 1] - o) & 1;
    int64_t q = t - X.fcnt[h];
    const int nl = X.ev[0][b] ? X.len[0][b][o] : 0;
    const bool lower = q < nl;
    const Event E = lower ? X.ev[0][b][2 * o + q] : X.ev[1][b][2 * o + (q - nl)];
    const bool keep = lower ? E.kind() == 1 : E.kind() == 0;
    const int a = pts[E.a].w, w = pts[E.w()].w, c = pts[E.b].w;
    X.faces[3 * t + 0] = a;
    X.faces[3 * t + 1] = keep ? w : c;
    X.faces[3 * t + 2] = keep ? c : w;
  }
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h <= S.H;
       h += (int64_t)gridDim.x * blockDim.x)
    if (X.face_off) X.face_off[h] = (over || err) ? 0 : X.fcnt[h];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    X.info[0] = err ? err : (over ? HULL_EINTERNAL : 0);
    X.info[1] = F;
  }
}

__global__ void k_info_small(int64_t* info, const Header* h) {
  if (threadIdx.x == 0) {
    info[0] = h ? h->err : 0;
    info[1] = 0;
  }
}

__global__ void __launch_bounds__(256)
    k_export_movies(const Event* __restrict__ ev, const int* __restrict__ len,
                    const int4* __restrict__ pts, int64_t n, int64_t width, int32_t* d_ev,
                    int32_t* d_block_len, int32_t* d_order, const Header* h) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    d_order[p] = pts[p].w;
    bool start = p % width == 0;
    int L = start && !h->err ? len[p] : 0;
    if (L < 0 || L > 2 * std::min(width, n - p)) L = 0;
    d_block_len[p] = L;
  }
  for (int64_t s = 0; s < n; s += width) {
    int L = h->err ? 0 : len[s];
    if (L < 0 || L > 2 * std::min(width, n - s)) L = 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < L;
         q += (int64_t)gridDim.x * blockDim.x) {
      Event E = ev[2 * s + q];
      d_ev[4 * (2 * s + q) + 0] = E.a;
      d_ev[4 * (2 * s + q) + 1] = E.w();
      d_ev[4 * (2 * s + q) + 2] = E.b;
      d_ev[4 * (2 * s + q) + 3] = E.kind();
    }
  }
}

// Lane-serial levels whose blocks (2, 4, 8, 16 points) are staged in LDS.
constexpr int kLdsLevels = 4;
constexpr int kFirstWaveLevel = 4;

static int levels_for(int64_t n) {
  int L = 0;
  while ((int64_t(1) << L) < n) ++L;
  return L;
}

static unsigned grid_for(int64_t work, int64_t cap_blocks = 4096) {
  int64_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return (unsigned)b;
}

static int env_int(const char* name, int dflt) {
  const char* e = getenv(name);
  return (e && *e) ? atoi(e) : dflt;
}

// The merge schedule: which levels run lane-serial and the walk segment
// length.  Unset fields take the environment (HULL_SERIAL_LEVELS,
// HULL_WALK_SEGMENT), then defaults.
struct Opts {
  int serial_max, seg;
  int wave_from;   // first lane-serial level run by lane groups (0: none)
  int wave_lanes;  // lanes per merge at level wave_from (8, 16, 32 or 64), doubling per level
  int wave_lanes_max;  // ... up to this many
  bool lds_links;  // working links in LDS where they fit (HULL_LDS_LINKS=0: global)
  int lds_levels;  // lowest levels with points and links staged in LDS (at most kLdsLevels;
                   // above them, the links alone)
  int order_from;     // lane-serial levels from this one list their merges in work order
  int64_t order_min;  // ... when the level bounds at least this many merges
  int64_t pts_lds_merges;  // lane-group levels of at most this many merges (both runs
                           // together) hold the points in LDS too, where they fit
};

// The first lane-group level when the caller gives none: lane groups pay
// once a level's merges are too few to fill the chip one lane each (they
// then get several lanes), so the fewer points a call has in all, the lower
// the level -- level 4 up to 2^16 points, 5 up to 2^18, one level later per
// doubling, level 8 from 2^21 (measured on cubes and spheres of 2^11..2^20
// points and on the n = 2^24 workload).
static int default_wave_level(int64_t total) {
  const int L = levels_for(total);
  return L <= 16 ? kFirstWaveLevel : std::min(8, std::max(5, L - 13));
}

static Opts resolve(const hull_schedule_t* sc, int64_t total) {
  Opts o;
  o.serial_max = sc && sc->serial_levels >= 0 ? sc->serial_levels : env_int("HULL_SERIAL_LEVELS", 10);
  o.seg = sc && sc->walk_segment > 0 ? sc->walk_segment : env_int("HULL_WALK_SEGMENT", 4);
  if (o.seg < kMinWalkSegment) o.seg = kMinWalkSegment;
  o.lds_levels = std::min(std::max(env_int("HULL_LDS_LEVELS", 3), 0), kLdsLevels);
  const int wf = sc && sc->wave_from != 0 ? sc->wave_from
                                          : env_int("HULL_WAVE_LEVEL", default_wave_level(total));
  // lane groups start above the LDS-staged levels, at level 4 (16 points) at the earliest
  o.wave_from = wf > 0 ? std::max(wf, std::max(o.lds_levels + 1, kFirstWaveLevel)) : 0;
  const int wl = sc && sc->wave_lanes > 0 ? sc->wave_lanes : env_int("HULL_WAVE_LANES", 8);
  o.wave_lanes = wl >= 64 ? 64 : (wl >= 32 ? 32 : (wl >= 16 ? 16 : 8));
  const int wm = sc && sc->wave_lanes_max > 0 ? sc->wave_lanes_max : env_int("HULL_WAVE_LANES_MAX", 64);
  o.wave_lanes_max = std::max(o.wave_lanes, wm >= 64 ? 64 : (wm >= 32 ? 32 : (wm >= 16 ? 16 : 8)));
  o.lds_links = env_int("HULL_LDS_LINKS", 1) != 0;
  o.order_from = env_int("HULL_ORDER_LEVEL", kOrderFromLevel);
  o.order_min = std::max(env_int("HULL_ORDER_MIN", (int)kOrderMinMerges), 0);
  o.pts_lds_merges = std::max(env_int("HULL_PTS_LDS_MERGES", kPtsLdsMerges), 0);
  return o;
}

// Runs `levels` merge levels of the selected runs over the hulls of S.
template <class PT>
static int32_t run_levels(int64_t n, const Sched& S0, char* ws, const Plan& pl, hipStream_t s,
                          bool lower, bool upper, int levels, const Opts& opt,
                          hipEvent_t* events) {
  Header* h = (Header*)(ws + pl.header);
  Sched S = S0;
  S.moff = (int*)(ws + pl.moff);
  S.mlist = (int2*)(ws + pl.mlist);
  S.toff = (int*)(ws + pl.toff);
  S.tlist = (int*)(ws + pl.tlist);
  S.mcap = pl.mcap;
  int* mcnt = (int*)(ws + pl.mcnt);
  int* tcnt = (int*)(ws + pl.tcnt);
  LevelArgs A{};
  A.h = h;
  A.S = S;
  A.n = n;
  ParLevel P{};
  P.h = h;
  P.S = S;
  P.seg_events = opt.seg;
  P.seg_cap = pl.seg_cap;
  P.ecap = 2 * n;
  // the call's one-launch scans tell their status words apart by epoch (the
  // sort cleared the words at the start of the call)
  P.chain_words = (unsigned long long*)(ws + pl.chain_words);
  P.chain_stride = pl.chain_stride;
  for (int r = 0; r < 2; ++r) {
    bool on = r == 0 ? lower : upper;
    RunPtrs& R = A.run[r];
    R.pts = on ? (const void*)(ws + pl.pts) : nullptr;
    R.pv0 = (int*)(ws + pl.pv0[r]);
    R.nx0 = (int*)(ws + pl.nx0[r]);
    R.lk = (int2*)(ws + pl.lk[r]);
    R.zs = r == 0 ? 1 : -1;
    ParRun& Q = P.run[r];
    Q.pts = R.pts;
    Q.pv0 = R.pv0;
    Q.nx0 = R.nx0;
    Q.zs = R.zs;
    Q.cntR = (int*)(ws + pl.cntR[r]);
    Q.cntL = (int*)(ws + pl.cntL[r]);
    Q.offR = (int*)(ws + pl.offR[r]);
    Q.offL = (int*)(ws + pl.offL[r]);
    Q.curR = (int*)(ws + pl.curR[r]);
    Q.curL = (int*)(ws + pl.curL[r]);
    Q.claimR = (int*)(ws + pl.claimR[r]);
    Q.claimL = (int*)(ws + pl.claimL[r]);
    Q.entR = (Entry*)(ws + pl.entR[r]);
    Q.entL = (Entry*)(ws + pl.entL[r]);
    Q.ctr = (int*)(ws + pl.ctr[r]);
    Q.touched = (int*)(ws + pl.touched[r]);
    Q.ecnt = (int*)(ws + pl.ecnt[r]);
    Q.eoff = (int*)(ws + pl.eoff[r]);
    Q.cslot = (int*)(ws + pl.cslot[r]);
    Q.cmerge = (int*)(ws + pl.cmerge[r]);
    Q.segS = (int*)(ws + pl.segS[r]);
    Q.segBase = (int*)(ws + pl.segBase[r]);
    Q.segMerge = (int*)(ws + pl.segMerge[r]);
    Q.segB = (int*)(ws + pl.segB[r]);
    Q.segCnt = (int*)(ws + pl.segCnt[r]);
    Q.segOff = (int*)(ws + pl.segOff[r]);
    Q.segUV = (int2*)(ws + pl.segUV[r]);
    Q.segTmp = (Event*)(ws + pl.segTmp[r]);
    Q.segTmpUV = (int2*)(ws + pl.segTmpUV[r]);
    Q.bev = (Event*)(ws + pl.bev[r]);
    Q.buv = (int2*)(ws + pl.buv[r]);
    Q.nB = (int*)(ws + pl.nB[r]);
    Q.boff = (int*)(ws + pl.boff[r]);
    Q.uv0 = (int2*)(ws + pl.uv0[r]);
    Q.surv = (int*)(ws + pl.surv[r]);
    Q.jb = (int*)(ws + pl.jb[r]);
    Q.pre = (int*)(ws + pl.pre[r]);
    Q.aR = (int*)(ws + pl.aR[r]);
    Q.aL = (int*)(ws + pl.aL[r]);
    Q.aT = (int*)(ws + pl.aT[r]);
    Q.wf = (unsigned char*)(ws + pl.wf[r]);
    if (on)
      hipLaunchKernelGGL(k_init_links, dim3(grid_for(n)), dim3(256), 0, s, R.pv0, R.nx0,
                         (int*)(ws + pl.len[r][0]), Q.claimR, Q.claimL, n);
  }
  int buf = 0;
  const unsigned hgrid = grid_for(S.H + 1, 1024);
  for (int k = 1; k <= levels; ++k) {
    A.width = int64_t(1) << k;
    A.half = A.width >> 1;
    const bool serial = k <= opt.serial_max;
    // lane groups at this level, and where the working links live
    const bool wave = serial && k > opt.lds_levels && opt.wave_from > 0 && k >= opt.wave_from;
    const int lanes =
        wave ? std::min(opt.wave_lanes_max, opt.wave_lanes << std::min(k - opt.wave_from, 3)) : 0;
    const bool lds_lane = serial && k > opt.lds_levels && !wave && opt.lds_links &&
                          A.width <= kLinkLdsLane;
    const int64_t bound = std::min<int64_t>(pl.mcap, n / A.width + S.H + 1);
    // points in LDS as well: levels of few merges (each iteration of a long
    // merge then waits on LDS rather than on a cache), when a block fits
    const bool pts_lds = wave && opt.lds_links && 2 * bound <= opt.pts_lds_merges &&
                         A.width <= 32767 &&
                         (64 / lanes) * A.width * (int64_t)(sizeof(LinkPair<short>) + sizeof(PT)) +
                                 (int64_t)sizeof(Event) * 128 <=
                             max_lds_bytes();
    const bool lds_group = wave && opt.lds_links && !pts_lds &&
                           (256 / lanes) * A.width * (int64_t)sizeof(LinkPair<short>) <=
                               kLinkLdsGroupBytes;
    // the schedule of this level
    int32_t rc = HULL_OK;
    const bool single = S.H == 1;
    if (single) {
      hipLaunchKernelGGL(k_sched_single, dim3(grid_for(n / A.width + 1)), dim3(256), 0, s, S, k,
                         n);
    } else {
      hipLaunchKernelGGL(k_sched_count, dim3(hgrid), dim3(256), 0, s, S, k, mcnt, tcnt);
      rc = scan_chained_i32(mcnt, S.moff, S.H + 1, P.chain_words, P.chain_stride,
                            (unsigned)(8 * k + 6), h, s);
      if (!rc)
        rc = scan_chained_i32(tcnt, S.toff, S.H + 1, P.chain_words, P.chain_stride,
                              (unsigned)(8 * k + 7), h, s);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sched_fill, dim3(grid_for(std::min<int64_t>(pl.mcap, n / A.width + S.H + 1))),
                         dim3(256), 0, s, S, k);
    }
    for (int r = 0; r < 2; ++r) {
      RunPtrs& R = A.run[r];
      R.ev_in = (const Event*)(ws + pl.ev[r][buf]);
      R.len_in = (const int*)(ws + pl.len[r][buf]);
      R.ev_out = (Event*)(ws + pl.ev[r][buf ^ 1]);
      R.len_out = (int*)(ws + pl.len[r][buf ^ 1]);
      ParRun& Q = P.run[r];
      Q.ev_in = R.ev_in;
      Q.len_in = R.len_in;
      Q.ev_out = R.ev_out;
      Q.len_out = R.len_out;
      if (R.pts && serial && k > opt.lds_levels && !lds_lane && !lds_group && !pts_lds)
        hipLaunchKernelGGL(k_copy_links, dim3(grid_for(n)), dim3(256), 0, s, R.pv0, R.nx0, R.lk, n);
    }
    if (events) (void)hipEventRecord(events[2 * k], s);
    if (serial && k == 1) {
      hipLaunchKernelGGL(k_merge_level1, dim3(grid_for(bound), 2), dim3(256), 0, s, A);
    } else if (serial && k <= opt.lds_levels) {
      const dim3 grid((unsigned)((bound + 63) / 64), 2);
      if (k == 1) hipLaunchKernelGGL((k_merge_level_lds<PT, 2>), grid, dim3(64), 0, s, A);
      else if (k == 2) hipLaunchKernelGGL((k_merge_level_lds<PT, 4>), grid, dim3(64), 0, s, A);
      else if (k == 3) hipLaunchKernelGGL((k_merge_level_lds<PT, 8>), grid, dim3(64), 0, s, A);
      else hipLaunchKernelGGL((k_merge_level_lds<PT, 16>), grid, dim3(64), 0, s, A);
    } else if (serial) {
      const dim3 grid((unsigned)((bound + 255) / 256), 2);
      LevelArgs B = A;
      if (k >= opt.order_from && bound >= opt.order_min) {
        for (int r = 0; r < 2; ++r) {
          B.perm[r] = (int*)(ws + pl.perm[r]);
          B.wbins[r] = (int*)(ws + pl.wbins[r]);
        }
        hipLaunchKernelGGL(k_work_clear, dim3(1, 2), dim3(256), 0, s, B);
        hipLaunchKernelGGL(k_work_hist, grid, dim3(256), 0, s, B);
        hipLaunchKernelGGL(k_work_scan, dim3(1, 2), dim3(64), 0, s, B);
        hipLaunchKernelGGL(k_work_place, grid, dim3(256), 0, s, B);
      }
      if (wave) {
        // lanes per merge double with every level (merges halve), so that
        // every lane-group level keeps about the same number of waves
        const int nb = pts_lds ? 64 : 256;  // lanes per block
        const int per = nb / lanes;          // merges per block
        const dim3 wg((unsigned)((bound + per - 1) / per), 2);
        const size_t lds =
            pts_lds ? (size_t)per * A.width * (sizeof(LinkPair<short>) + sizeof(PT))
                    : (lds_group ? (size_t)per * A.width * sizeof(LinkPair<short>) : 0);
#define HULL_WAVE(G)                                                                        \
  if (pts_lds) hipLaunchKernelGGL((k_merge_wave<PT, G, 2>), wg, dim3(64), lds, s, B);         \
  else if (lds_group) hipLaunchKernelGGL((k_merge_wave<PT, G, 1>), wg, dim3(256), lds, s, B); \
  else hipLaunchKernelGGL((k_merge_wave<PT, G, 0>), wg, dim3(256), 0, s, B);
        if (lanes == 64) { HULL_WAVE(64) }
        else if (lanes == 32) { HULL_WAVE(32) }
        else if (lanes == 16) { HULL_WAVE(16) }
        else { HULL_WAVE(8) }
#undef HULL_WAVE
      } else if (lds_lane) {
        const dim3 g64((unsigned)((bound + 63) / 64), 2);
        const size_t lds = (size_t)A.width * 64 * sizeof(LinkPair<signed char>);
        hipLaunchKernelGGL(k_merge_level_lk<PT>, g64, dim3(64), lds, s, B);
      } else
        hipLaunchKernelGGL(k_merge_level<PT>, grid, dim3(256), 0, s, B);
    } else {
      P.k = k;
      P.run[0].stamp = P.run[1].stamp = k;
      rc = parallel_level<PT>(P, s);
      if (rc) return rc;
    }
    if (events) (void)hipEventRecord(events[2 * k + 1], s);
    // a single hull has a trailing block at this level when its block count
    // is odd and above one
    const int64_t nb = (n + A.half - 1) / A.half;
    if (!single || (nb > 1 && (nb & 1)))
      hipLaunchKernelGGL(k_passthrough, dim3((unsigned)std::min<int64_t>(S.H, 4096), 2), dim3(256),
                         0, s, A);
    HULL_LAUNCH_CHECK();
    buf ^= 1;
  }
  return HULL_OK;
}

// Faces of every hull of S after its merges.
template <class PT>
static int32_t extract(const Sched& S, char* ws, const Plan& pl, hipStream_t s, bool lower,
                       bool upper, int32_t* d_faces, int64_t cap, int64_t* d_face_off,
                       int64_t* d_info) {
  ExtractArgs X{};
  X.S = S;
  for (int r = 0; r < 2; ++r)
    for (int b = 0; b < 2; ++b) {
      bool on = r == 0 ? lower : upper;
      X.ev[r][b] = on ? (const Event*)(ws + pl.ev[r][b]) : nullptr;
      X.len[r][b] = (const int*)(ws + pl.len[r][b]);
    }
  X.pts = (const void*)(ws + pl.pts);
  X.fcnt = (int*)(ws + pl.fcnt);
  X.faces = d_faces;
  X.cap = cap;
  X.face_off = d_face_off;
  X.info = d_info;
  X.h = (const Header*)(ws + pl.header);
  hipLaunchKernelGGL(k_face_count, dim3(grid_for(S.H + 1, 1024)), dim3(256), 0, s, X);
  if (S.H > 1) {  // one hull: k_face_count writes the offsets themselves
    int32_t rc = scan_chained_i32(X.fcnt, X.fcnt, S.H + 1, (unsigned long long*)(ws + pl.chain_words),
                                  pl.chain_stride, kChainEpochFaces, (Header*)(ws + pl.header), s);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_extract<PT>, dim3(grid_for(std::max<int64_t>(cap, S.H + 1), 2048)), dim3(256), 0,
                     s, X);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

template <class InT, class PT>
static int32_t hull_runs_t(const InT* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                           int64_t* d_info, void* d_ws, size_t ws_bytes, hipStream_t s, bool lower,
                           bool upper, void* const* events, int32_t nevents) {
  if (n < 0 || n > kMaxN || !d_info || (n > 0 && !d_xyz) || !d_faces || cap < 2 * n || !d_ws)
    return HULL_EINVAL;
  const int L = levels_for(n);
  if (events && nevents < 2 * L + 3) return HULL_EINVAL;
  hipEvent_t* ev = (hipEvent_t*)events;
  const Opts opt = resolve(nullptr, n);
  Plan pl = make_plan(n, 1, opt.seg, (int)sizeof(PT));
  if (ws_bytes < pl.total) return HULL_EWORKSPACE;
  char* ws = (char*)d_ws;
  Header* h = (Header*)(ws + pl.header);
  if (ev) (void)hipEventRecord(ev[0], s);
  init_header(h, s);
  if (n < 3) {
    hipLaunchKernelGGL(k_info_small, dim3(1), dim3(64), 0, s, d_info, h);
    HULL_LAUNCH_CHECK();
    if (ev)
      for (int q = 1; q < 2 * L + 3; ++q) (void)hipEventRecord(ev[q], s);
    return HULL_OK;
  }
  int64_t* off = (int64_t*)(ws + pl.off1);
  hipLaunchKernelGGL(k_set_off1, dim3(1), dim3(64), 0, s, off, n);
  Sched S{};
  S.off = off;
  S.H = 1;
  int32_t rc = sort_points<InT, PT>(d_xyz, n, nullptr, 1, ws, pl, s);
  if (rc) return rc;
  if (ev) (void)hipEventRecord(ev[1], s);
  rc = run_levels<PT>(n, S, ws, pl, s, lower, upper, L, opt, ev);
  if (rc) return rc;
  S.moff = (int*)(ws + pl.moff);
  rc = extract<PT>(S, ws, pl, s, lower, upper, d_faces, cap, nullptr, d_info);
  if (ev) (void)hipEventRecord(ev[2 * L + 2], s);
  return rc;
}

int32_t hull_runs(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, hipStream_t s, bool lower, bool upper,
                  void* const* events, int32_t nevents) {
  return hull_runs_t<int32_t, int4>(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, s, lower,
                                    upper, events, nevents);
}

int32_t hull_runs(const int64_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, hipStream_t s, bool lower, bool upper,
                  void* const* events, int32_t nevents) {
  return hull_runs_t<int64_t, WPt>(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, s, lower, upper,
                                   events, nevents);
}

int32_t batched(const int32_t* d_xyz, const int64_t* d_off, const int64_t* h_off, int64_t H,
                int32_t* d_faces, int64_t cap, int64_t* d_face_off, int64_t* d_info, void* d_ws,
                size_t ws_bytes, const hull_schedule_t* sched, hipStream_t s) {
  if (H < 1 || !d_off || !h_off || !d_info || !d_faces || !d_face_off || !d_ws) return HULL_EINVAL;
  const int64_t n = h_off[H];
  if (h_off[0] != 0 || n < 0 || n > kMaxTotal || (n > 0 && !d_xyz) || cap < 2 * n)
    return HULL_EINVAL;
  const Opts opt = resolve(sched, n);
  int L = 0;
  for (int64_t q = 0; q < H; ++q) {
    const int64_t nh = h_off[q + 1] - h_off[q];
    if (nh < 0 || nh > kMaxN) return HULL_EINVAL;
    L = std::max(L, levels_for(nh));
  }
  Plan pl = make_plan(n, H, opt.seg);
  if (ws_bytes < pl.total) return HULL_EWORKSPACE;
  char* ws = (char*)d_ws;
  Header* h = (Header*)(ws + pl.header);
  init_header(h, s);
  Sched S{};
  S.off = d_off;
  S.H = H;
  if (n > 0) {
    int32_t rc = sort_points<int32_t, int4>(d_xyz, n, d_off, H, ws, pl, s);
    if (rc) return rc;
    rc = run_levels<int4>(n, S, ws, pl, s, true, true, L, opt, nullptr);
    if (rc) return rc;
  } else {
    for (int r = 0; r < 2; ++r)
      hipLaunchKernelGGL(k_init_links, dim3(1), dim3(256), 0, s, (int*)(ws + pl.pv0[r]),
                         (int*)(ws + pl.nx0[r]), (int*)(ws + pl.len[r][0]),
                         (int*)(ws + pl.claimR[r]), (int*)(ws + pl.claimL[r]), int64_t(1));
  }
  return extract<int4>(S, ws, pl, s, true, true, d_faces, cap, d_face_off, d_info);
}

int32_t movies(const int32_t* d_xyz, int64_t n, int32_t run, int32_t level, int32_t* d_ev,
               int32_t* d_block_len, int32_t* d_order, int64_t* d_info, void* d_ws,
               size_t ws_bytes, hipStream_t s) {
  if (n < 1 || n > kMaxN || !d_xyz || !d_ev || !d_block_len || !d_order || !d_info || !d_ws ||
      (run != 0 && run != 1))
    return HULL_EINVAL;
  const Opts opt = resolve(nullptr, n);
  Plan pl = make_plan(n, 1, opt.seg);
  if (ws_bytes < pl.total) return HULL_EWORKSPACE;
  char* ws = (char*)d_ws;
  Header* h = (Header*)(ws + pl.header);
  init_header(h, s);
  int64_t* off = (int64_t*)(ws + pl.off1);
  hipLaunchKernelGGL(k_set_off1, dim3(1), dim3(64), 0, s, off, n);
  Sched S{};
  S.off = off;
  S.H = 1;
  int32_t rc = sort_points<int32_t, int4>(d_xyz, n, nullptr, 1, ws, pl, s);
  if (rc) return rc;
  int L = levels_for(n);
  if (level >= 0 && level < L) L = level;
  rc = run_levels<int4>(n, S, ws, pl, s, run == 0, run == 1, L, opt, nullptr);
  if (rc) return rc;
  hipLaunchKernelGGL(k_export_movies, dim3(grid_for(2 * n, 1024)), dim3(256), 0, s,
                     (const Event*)(ws + pl.ev[run][L & 1]), (const int*)(ws + pl.len[run][L & 1]),
                     (const int4*)(ws + pl.pts), n, int64_t(1) << L, d_ev, d_block_len, d_order,
                     h);
  hipLaunchKernelGGL(k_info_small, dim3(1), dim3(64), 0, s, d_info, h);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

}  // namespace hull

extern "C" {

const char* hull_strerror(int32_t code) {
  switch (code) {
    case HULL_OK: return "ok";
    case HULL_EINVAL: return "invalid argument";
    case HULL_EWORKSPACE: return "workspace too small";
    case HULL_ERANGE: return "coordinate outside the supported range (or not finite)";
    case HULL_EHIP: return "HIP runtime error";
    case HULL_EINTERNAL: return "internal consistency bound exceeded";
    default: return "unknown status";
  }
}

int32_t hull_workspace_bytes(int64_t n, int32_t flags, size_t* bytes) {
  if (!bytes || n < 0 || n > hull::kMaxN) return HULL_EINVAL;
  switch (flags) {
    case HULL_WS_STANDARD: *bytes = hull::make_plan(n, 1, hull::kMinWalkSegment).total; break;
    case HULL_WS_WIDE: *bytes = hull::wide_workspace_bytes(n); break;
    case HULL_WS_F32: *bytes = hull::f32_workspace_bytes(n); break;
    default: return HULL_EINVAL;
  }
  return HULL_OK;
}

int32_t hull_schedule_defaults(hull_schedule_t* out) {
  if (!out) return HULL_EINVAL;
  const hull::Opts o = hull::resolve(nullptr, hull::kMaxN);
  out->serial_levels = o.serial_max;
  out->walk_segment = o.seg;
  out->fused_levels = o.lds_levels;
  out->wave_from = o.wave_from;
  out->wave_lanes = o.wave_lanes;
  out->wave_lanes_max = o.wave_lanes_max;
  return HULL_OK;
}

int32_t hull_workspace_bytes_batched(int64_t total_points, int64_t H, size_t* bytes) {
  if (!bytes || total_points < 0 || total_points > hull::kMaxTotal || H < 1) return HULL_EINVAL;
  *bytes = hull::make_plan(total_points, H, hull::kMinWalkSegment).total;
  return HULL_OK;
}

int32_t hull_lower(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                   void* d_ws, size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         false, nullptr, 0);
}

int32_t hull_full(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         true, nullptr, 0);
}

int32_t hull_full_timed(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                        int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream,
                        void* const* events, int32_t nevents) {
  hull::clear_stale_hip_error();
  if (!events) return HULL_EINVAL;
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         true, events, nevents);
}

int32_t hull_full_batched(const int32_t* d_xyz, const int64_t* d_offsets, const int64_t* h_offsets,
                          int64_t H, int32_t* d_faces, int64_t cap, int64_t* d_face_offsets,
                          int64_t* d_info, void* d_ws, size_t ws_bytes,
                          const hull_schedule_t* schedule, void* stream) {
  hull::clear_stale_hip_error();
  return hull::batched(d_xyz, d_offsets, h_offsets, H, d_faces, cap, d_face_offsets, d_info, d_ws,
                       ws_bytes, schedule, (hipStream_t)stream);
}

int32_t hull_movies(const int32_t* d_xyz, int64_t n, int32_t run, int32_t level, int32_t* d_ev,
                    int32_t* d_block_len, int32_t* d_order, int64_t* d_info, void* d_ws,
                    size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::movies(d_xyz, n, run, level, d_ev, d_block_len, d_order, d_info, d_ws, ws_bytes,
                      (hipStream_t)stream);
}

}  // extern "C"
