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

namespace hull {

__device__ void merge_one(const RunPtrs& R, Header* h, int64_t s, int64_t m, int64_t e) {
  const int4* pts = R.pts;
  int* pv = R.pv;
  int* nx = R.nx;
  const int zs = R.zs;
  const int nL = R.len_in[s], nR = R.len_in[m];
  if (nL < 0 || nR < 0 || nL > 2 * (m - s) || nR > 2 * (e - m)) {
    atomicCAS(&h->err, 0, HULL_EINTERNAL);
    R.len_out[s] = 0;
    return;
  }
  const Event* Lev = R.ev_in + 2 * s;
  const Event* Rev = R.ev_in + 2 * m;
  const double* Ltau = R.tau_in + 2 * s;
  const double* Rtau = R.tau_in + 2 * m;
  Event* out = R.ev_out + 2 * s;
  double* out_tau = R.tau_out + 2 * s;
  const int64_t cap = 2 * (e - s);

  // 1. bridge at t = -inf
  int u = (int)m - 1, v = (int)m;
  int4 Pu = pts[u], Pv = pts[v];
  for (int guard = 0;; ++guard) {
    if (guard > 2 * (e - s) + 4) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      R.len_out[s] = 0;
      return;
    }
    int w = R.nx0[v];
    if (w != kNil) {
      int4 Pw = pts[w];
      if (d_sign(Pu, Pv, Pw) < 0) {
        v = w;
        Pv = Pw;
        continue;
      }
    }
    w = R.pv0[u];
    if (w != kNil) {
      int4 Pw = pts[w];
      if (d_sign(Pw, Pu, Pv) < 0) {
        u = w;
        Pu = Pw;
        continue;
      }
    }
    break;
  }
  const int u0 = u, v0 = v;

  // 2. event loop
  int i = 0, j = 0, k = 0;
  bool haveT = false;
  Cand T;
  T.t = Tri{-1, -1, -1};
  T.st = 0.0;
  T.kind = 0;
  const int64_t iter_cap = (int64_t)nL + nR + 4 * (e - s) + 16;
  for (int64_t it = 0;; ++it) {
    if (it > iter_cap) {
      atomicCAS(&h->err, 0, HULL_EINTERNAL);
      break;
    }
    // candidates: 0 next L event, 1 next R event, 2..5 bridge moves.  The
    // running best is kept field by field in scalars, every candidate index
    // is a compile-time constant: the candidates stay in registers.
    int bi = -1, ba = 0, bw = 0, bb = 0, bk = 0;
    double bs = 0.0;
#define HULL_CONSIDER(IDX, CAND)                                                  \
  do {                                                                            \
    const Cand cc_ = (CAND);                                                      \
    bool take_ = !(haveT && ev_cmp(pts, cc_, T, zs) <= 0);                        \
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
    if (i < nL) {
      Event E = Lev[i];
      Cand c;
      c.t = Tri{E.a, E.w, E.b};
      c.kind = E.kind;
      c.st = Ltau[i];
      HULL_CONSIDER(0, c);
    }
    if (j < nR) {
      Event E = Rev[j];
      Cand c;
      c.t = Tri{E.a, E.w, E.b};
      c.kind = E.kind;
      c.st = Rtau[j];
      HULL_CONSIDER(1, c);
    }
    const int nu = nx[u], pu = pv[u], pvv = pv[v], nv = nx[v];
    if (nu != kNil) HULL_CONSIDER(2, make_cand(pts, u, nu, v, Pu, pts[nu], Pv, 1, zs));
    if (pu != kNil) HULL_CONSIDER(3, make_cand(pts, pu, u, v, pts[pu], Pu, Pv, 0, zs));
    if (pvv != kNil) HULL_CONSIDER(4, make_cand(pts, u, pvv, v, Pu, pts[pvv], Pv, 1, zs));
    if (nv != kNil) HULL_CONSIDER(5, make_cand(pts, u, v, nv, Pu, Pv, pts[nv], 0, zs));
#undef HULL_CONSIDER
    if (bi < 0) break;
    T.t = Tri{ba, bw, bb};
    T.st = bs;
    T.kind = bk;
    haveT = true;
    bool emit = false;
    if (bi <= 1) {
      const Tri& t = T.t;
      emit = bi == 0 ? (t.w < u) : (t.w > v);
      if (T.kind) {  // insertion into the child's chain
        nx[t.a] = t.w;
        pv[t.b] = t.w;
        pv[t.w] = t.a;
        nx[t.w] = t.b;
      } else {  // deletion
        nx[t.a] = t.b;
        pv[t.b] = t.a;
      }
      if (bi == 0) ++i; else ++j;
    } else {
      emit = true;
      if (bi == 2) { u = nu; Pu = pts[u]; }
      else if (bi == 3) { u = pu; Pu = pts[u]; }
      else if (bi == 4) { v = pvv; Pv = pts[v]; }
      else { v = nv; Pv = pts[v]; }
    }
    if (emit) {
      if (k >= cap) {
        atomicCAS(&h->err, 0, HULL_EINTERNAL);
        break;
      }
      out[k] = Event{T.t.a, T.t.w, T.t.b, T.kind};
      out_tau[k] = T.st;
      ++k;
    }
  }
  // 3. splice the -inf chains
  R.nx0[u0] = v0;
  R.pv0[v0] = u0;
  R.len_out[s] = k;
}

__global__ void __launch_bounds__(256) k_merge_level(LevelArgs A) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= 2 * A.merges) return;
  int r = g >= A.merges ? 1 : 0;
  int64_t q = g - r * A.merges;
  if (!A.run[r].pts) return;
  int64_t s = q * A.width, m = s + A.half, e = std::min(s + A.width, A.n);
  // After an error the movies are empty, so that every later kernel still
  // reads lengths that were written.
  if (A.h->err) {
    A.run[r].len_out[s] = 0;
    return;
  }
  merge_one(A.run[r], A.h, s, m, e);
}

// Bottom levels fused in LDS: one workgroup takes a tile of 2^KT consecutive
// ranks (run blockIdx.y) through merge levels 1..KT with the lane-serial
// merge, every array of the tile (points, links, both movie buffers) in LDS.
// Only the tile's final movie and -inf links go back to HBM, in the layout
// the level loop expects after KT levels (block start = tile start).
template <int KT>
__global__ void __launch_bounds__(256) k_merge_tile(LevelArgs A, const int4* __restrict__ gpts,
                                                    int outbuf_is_b) {
  constexpr int TP = 1 << KT;
  __shared__ int4 P[TP];
  __shared__ int pv0[TP], nx0[TP], pv[TP], nx[TP];
  __shared__ Event ev[2][2 * TP];
  __shared__ double tau[2][2 * TP];
  __shared__ int len[2][TP];
  const RunPtrs& G = A.run[blockIdx.y];
  if (!G.pts) return;
  const int64_t base = (int64_t)blockIdx.x * TP;
  const int tn = (int)std::min<int64_t>(TP, A.n - base);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < TP; i += nt) {
    if (i < tn) P[i] = gpts[base + i];
    pv0[i] = kNil;
    nx0[i] = kNil;
    len[0][i] = 0;
  }
  __syncthreads();
  RunPtrs R = G;
  R.pts = P;
  R.pv0 = pv0;
  R.nx0 = nx0;
  R.pv = pv;
  R.nx = nx;
  int buf = 0;
  for (int k = 1; k <= KT; ++k) {
    const int width = 1 << k, half = width >> 1;
    for (int i = tid; i < tn; i += nt) {
      pv[i] = pv0[i];
      nx[i] = nx0[i];
    }
    __syncthreads();
    R.ev_in = ev[buf];
    R.tau_in = tau[buf];
    R.len_in = len[buf];
    R.ev_out = ev[buf ^ 1];
    R.tau_out = tau[buf ^ 1];
    R.len_out = len[buf ^ 1];
    const int blocks = (tn + width - 1) / width;
    for (int b = tid; b < blocks; b += nt) {
      const int s = b * width, m = s + half, e = std::min(s + width, tn);
      if (m >= e) {  // unpaired trailing block: passes through
        int L = R.len_in[s];
        for (int q = 0; q < L; ++q) {
          R.ev_out[2 * s + q] = R.ev_in[2 * s + q];
          R.tau_out[2 * s + q] = R.tau_in[2 * s + q];
        }
        R.len_out[s] = L;
      } else if (A.h->err) {
        R.len_out[s] = 0;
      } else {
        merge_one(R, A.h, s, m, e);
      }
    }
    __syncthreads();
    buf ^= 1;
  }
  // the tile is one block now: its movie, lengths and -inf links to HBM
  const int L = len[buf][0];
  Event* gev = G.ev_out + 2 * base;
  double* gtau = G.tau_out + 2 * base;
  (void)outbuf_is_b;
  for (int q = tid; q < L; q += nt) {
    Event E = ev[buf][q];
    gev[q] = Event{E.a + (int)base, E.w + (int)base, E.b + (int)base, E.kind};
    gtau[q] = tau[buf][q];
  }
  for (int i = tid; i < tn; i += nt) {
    G.pv0[base + i] = pv0[i] == kNil ? kNil : pv0[i] + (int)base;
    G.nx0[base + i] = nx0[i] == kNil ? kNil : nx0[i] + (int)base;
  }
  if (tid == 0) G.len_out[base] = L;
}

// The unpaired trailing block of a level keeps its movie: copy it across.
__global__ void __launch_bounds__(256) k_passthrough(LevelArgs A, int64_t s) {
  int r = blockIdx.y;
  const RunPtrs& R = A.run[r];
  if (!R.pts) return;
  int len = R.len_in[s];
  if (A.h->err || len < 0 || len > 2 * (A.n - s)) len = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < len;
       q += (int64_t)gridDim.x * blockDim.x) {
    R.ev_out[2 * s + q] = R.ev_in[2 * s + q];
    R.tau_out[2 * s + q] = R.tau_in[2 * s + q];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) R.len_out[s] = len;
}

__global__ void __launch_bounds__(256) k_init_links(int* pv0, int* nx0, int* len, int64_t n) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    pv0[p] = kNil;
    nx0[p] = kNil;
    len[p] = 0;
  }
}

__global__ void __launch_bounds__(256) k_copy_links(const int* __restrict__ pv0,
                                                    const int* __restrict__ nx0,
                                                    int* __restrict__ pv, int* __restrict__ nx,
                                                    int64_t n) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    pv[p] = pv0[p];
    nx[p] = nx0[p];
  }
}

// Faces from the final movies: event (a, w, b) gives the face with the
// middle vertex w; an insertion has D(a, w, b) < 0, a deletion D > 0.  Lower
// faces need D < 0 for an outward orientation, upper faces D > 0.
__global__ void __launch_bounds__(256)
    k_extract(const Event* __restrict__ evL, const int* lenL, const Event* __restrict__ evU,
              const int* lenU, const int4* __restrict__ pts, int32_t* __restrict__ faces,
              int64_t cap, int64_t* info, const Header* h) {
  int nL = evL ? *lenL : 0, nU = evU ? *lenU : 0;
  int64_t total = (int64_t)nL + nU;
  const bool over = total > cap;
  if (over || h->err) total = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    bool lower = q < nL;
    Event E = lower ? evL[q] : evU[q - nL];
    bool keep = lower ? E.kind == 1 : E.kind == 0;
    int a = pts[E.a].w, w = pts[E.w].w, b = pts[E.b].w;
    faces[3 * q + 0] = a;
    faces[3 * q + 1] = keep ? w : b;
    faces[3 * q + 2] = keep ? b : w;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    info[0] = h->err ? h->err : (over ? HULL_EINTERNAL : 0);
    info[1] = total;
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
      d_ev[4 * (2 * s + q) + 1] = E.w;
      d_ev[4 * (2 * s + q) + 2] = E.b;
      d_ev[4 * (2 * s + q) + 3] = E.kind;
    }
  }
}

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

// Highest level merged by the lane-serial strategy; higher levels use the
// parallel strategy.  Tunable through HULL_SERIAL_LEVELS (0 = parallel from
// the first level, a large value = lane-serial throughout).
static int serial_levels() {
  const char* e = getenv("HULL_SERIAL_LEVELS");
  if (e && *e) return atoi(e);
  return 10;
}

// Levels fused in LDS at the bottom (7, 8 or 9; 0 = none).  Tunable through
// HULL_FUSED_LEVELS.
static int fused_levels() {
  const char* e = getenv("HULL_FUSED_LEVELS");
  int v = (e && *e) ? atoi(e) : 0;
  if (v <= 0) return 0;
  return v < 7 ? 7 : (v > 9 ? 9 : v);
}

// Child events per time segment of a bridge walk (parallel strategy).
// Tunable through HULL_WALK_SEGMENT.
static int seg_events() {
  const char* e = getenv("HULL_WALK_SEGMENT");
  int v = (e && *e) ? atoi(e) : 16;
  return v < 8 ? 8 : v;
}

// Runs `levels` merge levels of the selected runs; returns the buffer index
// holding the final movies.
static int32_t run_levels(int64_t n, char* ws, const Plan& pl, hipStream_t s, bool lower,
                          bool upper, int levels, int* final_buf, hipEvent_t* events) {
  Header* h = (Header*)(ws + pl.header);
  const int serial_max = serial_levels();
  LevelArgs A{};
  A.h = h;
  A.n = n;
  ParLevel P{};
  P.h = h;
  P.n = n;
  for (int r = 0; r < 2; ++r) {
    bool on = r == 0 ? lower : upper;
    RunPtrs& R = A.run[r];
    R.pts = on ? (const int4*)(ws + pl.pts) : nullptr;
    R.pv0 = (int*)(ws + pl.pv0[r]);
    R.nx0 = (int*)(ws + pl.nx0[r]);
    R.pv = (int*)(ws + pl.pv[r]);
    R.nx = (int*)(ws + pl.nx[r]);
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
    Q.entR = (Event*)(ws + pl.entR[r]);
    Q.entL = (Event*)(ws + pl.entL[r]);
    Q.entRt = (double*)(ws + pl.entRt[r]);
    Q.entLt = (double*)(ws + pl.entLt[r]);
    Q.segS = (int*)(ws + pl.segS[r]);
    Q.segBase = (int*)(ws + pl.segBase[r]);
    Q.segMerge = (int*)(ws + pl.segMerge[r]);
    Q.segCnt = (int*)(ws + pl.segCnt[r]);
    Q.segOff = (int*)(ws + pl.segOff[r]);
    Q.bev = (Event*)(ws + pl.bev[r]);
    Q.btau = (double*)(ws + pl.btau[r]);
    Q.buv = (int2*)(ws + pl.buv[r]);
    Q.nB = (int*)(ws + pl.nB[r]);
    Q.uv0 = (int2*)(ws + pl.uv0[r]);
    Q.surv = (int*)(ws + pl.surv[r]);
    Q.jb = (int*)(ws + pl.jb[r]);
    Q.pre = (int*)(ws + pl.pre[r]);
    if (on)
      hipLaunchKernelGGL(k_init_links, dim3(grid_for(n)), dim3(256), 0, s, R.pv0, R.nx0,
                         (int*)(ws + pl.len[r][0]), n);
  }
  int32_t* partials = (int32_t*)(ws + pl.partials);
  int buf = 0;
  // levels 1..KT fused in LDS, one workgroup per tile of 2^KT ranks
  // (only when at least KT levels are asked for: the kernel runs exactly KT)
  int KT = fused_levels();
  if (KT > levels) KT = 0;
  if (KT > 0) {
    for (int r = 0; r < 2; ++r) {
      RunPtrs& R = A.run[r];
      R.ev_out = (Event*)(ws + pl.ev[r][KT & 1]);
      R.tau_out = (double*)(ws + pl.tau[r][KT & 1]);
      R.len_out = (int*)(ws + pl.len[r][KT & 1]);
    }
    if (events) (void)hipEventRecord(events[2], s);
    const int64_t tiles = (n + (int64_t(1) << KT) - 1) >> KT;
    const int4* gpts = (const int4*)(ws + pl.pts);
    if (KT == 7)
      hipLaunchKernelGGL(k_merge_tile<7>, dim3((unsigned)tiles, 2), dim3(256), 0, s, A, gpts, 0);
    else if (KT == 8)
      hipLaunchKernelGGL(k_merge_tile<8>, dim3((unsigned)tiles, 2), dim3(256), 0, s, A, gpts, 0);
    else
      hipLaunchKernelGGL(k_merge_tile<9>, dim3((unsigned)tiles, 2), dim3(256), 0, s, A, gpts, 0);
    if (events)
      for (int q = 3; q <= 2 * KT + 1; ++q) (void)hipEventRecord(events[q], s);
    HULL_LAUNCH_CHECK();
    buf = KT & 1;
  }
  for (int k = KT + 1; k <= levels; ++k) {
    A.width = int64_t(1) << k;
    A.half = A.width >> 1;
    int64_t blocks = (n + A.width - 1) / A.width;
    int64_t last_s = (blocks - 1) * A.width;
    bool trailing = last_s + A.half >= n;
    A.merges = trailing ? blocks - 1 : blocks;
    const bool serial = k <= serial_max;
    for (int r = 0; r < 2; ++r) {
      RunPtrs& R = A.run[r];
      R.ev_in = (const Event*)(ws + pl.ev[r][buf]);
      R.tau_in = (const double*)(ws + pl.tau[r][buf]);
      R.len_in = (const int*)(ws + pl.len[r][buf]);
      R.ev_out = (Event*)(ws + pl.ev[r][buf ^ 1]);
      R.tau_out = (double*)(ws + pl.tau[r][buf ^ 1]);
      R.len_out = (int*)(ws + pl.len[r][buf ^ 1]);
      ParRun& Q = P.run[r];
      Q.ev_in = R.ev_in;
      Q.tau_in = R.tau_in;
      Q.len_in = R.len_in;
      Q.ev_out = R.ev_out;
      Q.tau_out = R.tau_out;
      Q.len_out = R.len_out;
      if (R.pts && serial)
        hipLaunchKernelGGL(k_copy_links, dim3(grid_for(n)), dim3(256), 0, s, R.pv0, R.nx0, R.pv,
                           R.nx, n);
    }
    if (events) (void)hipEventRecord(events[2 * k], s);
    if (A.merges > 0) {
      if (serial) {
        hipLaunchKernelGGL(k_merge_level, dim3(grid_for(2 * A.merges, int64_t(1) << 30), 1),
                           dim3(256), 0, s, A);
      } else {
        P.k = k;
        P.merges = A.merges;
        P.seg_events = seg_events();
        // sum over merges of 1 + (events)/G, events <= 2 * (points)
        P.seg_cap = std::min<int64_t>(A.merges + (2 * n) / P.seg_events + 1, n);
        int32_t rc = parallel_level(P, partials, s);
        if (rc) return rc;
      }
    }
    if (events) (void)hipEventRecord(events[2 * k + 1], s);
    if (trailing)
      hipLaunchKernelGGL(k_passthrough, dim3(grid_for(2 * (n - last_s), 1024), 2), dim3(256), 0,
                         s, A, last_s);
    HULL_LAUNCH_CHECK();
    buf ^= 1;
  }
  *final_buf = buf;
  return HULL_OK;
}

int32_t hull_runs(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, hipStream_t s, bool lower, bool upper,
                  void* const* events, int32_t nevents) {
  if (n < 0 || n > kMaxN || !d_info || (n > 0 && !d_xyz) || !d_faces || cap < 2 * n || !d_ws)
    return HULL_EINVAL;
  const int L = levels_for(n);
  if (events && nevents < 2 * L + 3) return HULL_EINVAL;
  hipEvent_t* ev = (hipEvent_t*)events;
  Plan pl = make_plan(n);
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
  int32_t rc = sort_points(d_xyz, n, ws, pl, s);
  if (rc) return rc;
  if (ev) (void)hipEventRecord(ev[1], s);
  int buf = 0;
  rc = run_levels(n, ws, pl, s, lower, upper, L, &buf, ev);
  if (rc) return rc;
  const Event* evL = lower ? (const Event*)(ws + pl.ev[0][buf]) : nullptr;
  const Event* evU = upper ? (const Event*)(ws + pl.ev[1][buf]) : nullptr;
  hipLaunchKernelGGL(k_extract, dim3(grid_for(2 * n, 2048)), dim3(256), 0, s, evL,
                     (const int*)(ws + pl.len[0][buf]), evU, (const int*)(ws + pl.len[1][buf]),
                     (const int4*)(ws + pl.pts), d_faces, cap, d_info, h);
  if (ev) (void)hipEventRecord(ev[2 * L + 2], s);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

int32_t movies(const int32_t* d_xyz, int64_t n, int32_t run, int32_t level, int32_t* d_ev,
               int32_t* d_block_len, int32_t* d_order, int64_t* d_info, void* d_ws,
               size_t ws_bytes, hipStream_t s) {
  if (n < 1 || n > kMaxN || !d_xyz || !d_ev || !d_block_len || !d_order || !d_info || !d_ws ||
      (run != 0 && run != 1))
    return HULL_EINVAL;
  Plan pl = make_plan(n);
  if (ws_bytes < pl.total) return HULL_EWORKSPACE;
  char* ws = (char*)d_ws;
  Header* h = (Header*)(ws + pl.header);
  init_header(h, s);
  int32_t rc = sort_points(d_xyz, n, ws, pl, s);
  if (rc) return rc;
  int L = levels_for(n);
  if (level >= 0 && level < L) L = level;
  int buf = 0;
  rc = run_levels(n, ws, pl, s, run == 0, run == 1, L, &buf, nullptr);
  if (rc) return rc;
  hipLaunchKernelGGL(k_export_movies, dim3(grid_for(2 * n, 1024)), dim3(256), 0, s,
                     (const Event*)(ws + pl.ev[run][buf]), (const int*)(ws + pl.len[run][buf]),
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
    case HULL_ERANGE: return "coordinate outside [-2^29, 2^29]";
    case HULL_EHIP: return "HIP runtime error";
    case HULL_EINTERNAL: return "internal consistency bound exceeded";
    default: return "unknown status";
  }
}

int32_t hull_workspace_bytes(int64_t n, int32_t flags, size_t* bytes) {
  (void)flags;
  if (!bytes || n < 0 || n > hull::kMaxN) return HULL_EINVAL;
  *bytes = hull::make_plan(n).total;
  return HULL_OK;
}

int32_t hull_lower(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                   void* d_ws, size_t ws_bytes, void* stream) {
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         false, nullptr, 0);
}

int32_t hull_full(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap, int64_t* d_info,
                  void* d_ws, size_t ws_bytes, void* stream) {
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         true, nullptr, 0);
}

int32_t hull_full_timed(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                        int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream,
                        void* const* events, int32_t nevents) {
  if (!events) return HULL_EINVAL;
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         true, events, nevents);
}

int32_t hull_movies(const int32_t* d_xyz, int64_t n, int32_t run, int32_t level, int32_t* d_ev,
                    int32_t* d_block_len, int32_t* d_order, int64_t* d_info, void* d_ws,
                    size_t ws_bytes, void* stream) {
  return hull::movies(d_xyz, n, run, level, d_ev, d_block_len, d_order, d_info, d_ws, ws_bytes,
                      (hipStream_t)stream);
}

}  // extern "C"
