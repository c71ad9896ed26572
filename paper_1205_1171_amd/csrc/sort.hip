// Presort by x (Sec. 2: the points are sorted by x before the merges), as a
// stable LSD radix sort of the key x - min(x) carrying the input index, so
// that equal x values stay in input order: ranks follow (x, input index),
// the x-order of the perturbed points.  Then a gather writes the points in
// rank order as int4 (x, y, z, i).
#include <algorithm>

#include "common.hpp"
#include "predicates.hpp"

namespace hull {


// ---------------------------------------------------------------------------
// Range check and x extent.
// ---------------------------------------------------------------------------
__global__ void k_header_init(Header* h) {
  if (threadIdx.x == 0) {
    h->err = 0;
    h->minx = 0x7fffffff;
    h->maxx = -0x7fffffff - 1;
    h->nbits = 0;
  }
}

template <class InT>
__global__ void __launch_bounds__(256) k_extent(const InT* __restrict__ xyz, int64_t n,
                                                Header* h) {
  __shared__ int smin[256], smax[256], sbad[256];
  int lo = 0x7fffffff, hi = -0x7fffffff - 1, bad = 0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const InT x = xyz[3 * p], y = xyz[3 * p + 1], z = xyz[3 * p + 2];
    const bool b = pt_out_of_range(x, y, z);
    // x of a row in range fits int32 on either range
    const int xi = b ? 0 : (int)x;
    lo = min(lo, xi);
    hi = max(hi, xi);
    bad |= b;
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMin(&h->minx, smin[0]);
    atomicMax(&h->maxx, smax[0]);
    if (sbad[0]) atomicCAS(&h->err, 0, HULL_ERANGE);
  }
}

__global__ void k_nbits(Header* h) {
  if (threadIdx.x == 0) {
    uint32_t span = (uint32_t)((int64_t)h->maxx - h->minx);
    int b = 0;
    while (b < 32 && (span >> b) != 0) ++b;
    h->nbits = b;
  }
}

// ---------------------------------------------------------------------------
// Radix passes.  The x passes sort the key x - min(x) (value = input index);
// passes whose digit lies above the key's bit length are skipped.  For a
// batch, stable passes on the hull id follow, so the final order is (hull,
// x, input index).  Executed pass e reads buffer (e - 1) & 1 (pass 0 reads
// xyz) and writes buffer e & 1; the buffers are chosen on the device.
// ---------------------------------------------------------------------------
struct RadixBufs {
  uint32_t* keys[2];
  int32_t* vals[2];
};

__device__ __forceinline__ int x_passes(const Header* h) {
  int p = (h->nbits + kRadixBits - 1) / kRadixBits;
  return p < 1 ? 1 : p;
}

// Digit of element p for (kind, d): kind 0 = x digit d, kind 1 = hull digit d.
template <class InT>
__device__ __forceinline__ uint32_t radix_key(const InT* xyz, const RadixBufs& B,
                                              const int32_t* hid, int64_t p, int e, int kind,
                                              int minx, int32_t* val) {
  if (kind == 0) {
    if (e == 0) {
      *val = (int32_t)p;
      return (uint32_t)((int64_t)xyz[3 * p] - minx);
    }
    *val = B.vals[(e - 1) & 1][p];
    return B.keys[(e - 1) & 1][p];
  }
  int v = B.vals[(e - 1) & 1][p];
  *val = v;
  return (uint32_t)hid[v];
}

template <class InT>
__global__ void __launch_bounds__(kSortThreads)
    k_radix_hist(const InT* __restrict__ xyz, RadixBufs B, const int32_t* __restrict__ hid,
                 int64_t n, int kind, int d, int tiles, int32_t* __restrict__ counts,
                 const Header* h) {
  const int xp = x_passes(h);
  if (kind == 0 && d >= xp) return;
  const int e = kind == 0 ? d : xp + d;
  __shared__ int hist[kBuckets];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int minx = h->minx;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int j = 0; j < kSortItems; ++j) {
    int64_t p = base + j * kSortThreads + threadIdx.x;
    if (p < n) {
      int32_t v;
      uint32_t k = radix_key(xyz, B, hid, p, e, kind, minx, &v);
      atomicAdd(&hist[(k >> (d * kRadixBits)) & (kBuckets - 1)], 1);
    }
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * tiles + blockIdx.x] = hist[threadIdx.x];
}

template <class InT>
__global__ void __launch_bounds__(kSortThreads)
    k_radix_scatter(const InT* __restrict__ xyz, RadixBufs B, const int32_t* __restrict__ hid,
                    int64_t n, int kind, int d, int tiles, const int32_t* __restrict__ offsets,
                    const Header* h) {
  const int xp = x_passes(h);
  if (kind == 0 && d >= xp) return;
  const int e = kind == 0 ? d : xp + d;
  constexpr int kWaves = kSortThreads / 64;
  __shared__ int base[kBuckets];
  __shared__ int wcnt[kWaves][kBuckets];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base[tid] = offsets[(int64_t)tid * tiles + blockIdx.x];
  const int minx = h->minx;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tbase = (int64_t)blockIdx.x * kTile;
  uint32_t* kout = B.keys[e & 1];
  int32_t* vout = B.vals[e & 1];
  for (int j = 0; j < kSortItems; ++j) {
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    int64_t p = tbase + j * kSortThreads + tid;
    bool valid = p < n;
    uint32_t k = 0;
    int32_t v = 0;
    if (valid) k = radix_key(xyz, B, hid, p, e, kind, minx, &v);
    int dg = (k >> (d * kRadixBits)) & (kBuckets - 1);
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < kRadixBits; ++b) {
      uint64_t on = __ballot((dg >> b) & 1);
      peers &= ((dg >> b) & 1) ? on : ~on;
    }
    int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][dg] = __popcll(peers);
    __syncthreads();
    int pos = 0;
    if (valid) {
      pos = base[dg] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dg];
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
    base[tid] += add;
    if (valid) {
      if (kind == 0) kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
  }
}

// Hull id of every input point (batches).
__global__ void __launch_bounds__(256) k_hull_ids(const int64_t* __restrict__ off, int64_t H,
                                                  int64_t n, int32_t* __restrict__ hid) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = H;  // largest h with off[h] <= i
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (off[mid] <= i) lo = mid;
      else hi = mid;
    }
    hid[i] = (int32_t)lo;
  }
}

// Gather the points in rank order from the buffer of the last executed pass;
// the index carried with each is the one within the point's hull.
template <class InT, class PT>
__global__ void __launch_bounds__(256)
    k_gather(const InT* __restrict__ xyz, RadixBufs B, const int32_t* __restrict__ hid,
             const int64_t* __restrict__ off, int hull_passes, int64_t n, PT* __restrict__ pts,
             const Header* h) {
  const int e = x_passes(h) + hull_passes - 1;
  const int32_t* v = B.vals[e & 1];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    int i = v[r];
    int local = hid ? (int)(i - off[hid[i]]) : i;
    pts[r] = make_pt(xyz, i, local);
  }
}

// ---------------------------------------------------------------------------
// Exclusive scans of int32 (one launch each: a chained scan).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int block_exclusive_scan(int x, int* lds_wave, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = x;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) lds_wave[wave] = incl;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    int t = lds_wave[w];
    if (w < wave) before += t;
    total += t;
  }
  __syncthreads();
  return before + incl - x;
}

// The length of a scan: read from device memory (+ add, at most cap), or cap
// itself for a length known on the host.
__device__ __forceinline__ int64_t dev_len(const int32_t* d_len, int add, int64_t cap) {
  if (!d_len) return cap;  // a length known on the host: cap itself
  int64_t L = (int64_t)(*d_len) + add;
  return L < 0 ? 0 : (L > cap ? cap : L);
}

// Scans of up to kMaxScanJobs arrays (blockIdx.y = job), one launch.  Tile t
// of a job (blocks stride over the
// tiles) publishes its sum, then finds the sum of all tiles before it by
// looking back over their published words, 64 at a time, until one holds an
// inclusive prefix (a chained scan with decoupled look-back), publishes its
// own inclusive prefix and writes its outputs.  A word packs a flag (bit 62:
// the tile's sum; bit 63: the inclusive prefix through the tile), the scan's
// epoch (bits 32-61; a word of another epoch counts as not yet published) and
// the 32-bit value, so one atomic load sees all three.  The grid (at most
// kScanDevGrid blocks per job) is resident at once and a tile waits only for
// tiles of lower index, which blocks of lower index or earlier strides hold;
// the wait is bounded anyway (kChainSpins re-reads, then HULL_EINTERNAL).
constexpr unsigned long long kChainSum = 1ull << 62, kChainIncl = 1ull << 63;
constexpr unsigned long long kChainEpoch = 0x3fffffffull << 32;
constexpr int kChainSpins = 1 << 22;

__device__ __forceinline__ unsigned long long chain_load(const unsigned long long* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void chain_store(unsigned long long* w, unsigned long long v) {
  __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kSortThreads)
    k_scan_chained(ScanJobs J, int add, int64_t cap, unsigned long long* words, int64_t wstride,
                   unsigned epoch, Header* h) {
  const ScanJob& jb = J.j[blockIdx.y];
  const int64_t len = dev_len(jb.d_len, add, cap);
  const int64_t ntiles = (len + kScanBlock - 1) / kScanBlock;
  unsigned long long* W = words + blockIdx.y * wstride;
  const unsigned long long ep = (unsigned long long)epoch << 32;
  __shared__ int wsum[kSortThreads / 64];
  __shared__ int s_prefix;
  const int lane = threadIdx.x & 63;
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0 && jb.total) *jb.total = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = base + j < len ? jb.in[base + j] : 0;
      sum += v[j];
    }
    int total;
    const int ex = block_exclusive_scan(sum, wsum, total);
    if (threadIdx.x == 0)
      chain_store(&W[tile], (tile == 0 ? kChainIncl : kChainSum) | ep | (unsigned)total);
    if (threadIdx.x < 64) {
      int prefix = 0;
      if (tile > 0) {
        int64_t newest = tile - 1;  // the window: tiles newest - 63 .. newest, lane l on newest - l
        int spins = 0;
        for (;;) {
          const int64_t q = newest - lane;
          unsigned long long w = q >= 0 ? chain_load(&W[q]) : (kChainIncl | ep);
          if ((w & kChainEpoch) != ep) w = 0;
          const uint64_t incl = __ballot((w & kChainIncl) != 0);
          const uint64_t none = __ballot((w & (kChainIncl | kChainSum)) == 0);
          const int stop = incl ? __builtin_ctzll(incl) : 64;  // the nearest inclusive prefix
          const uint64_t upto = stop >= 63 ? ~0ull : ((2ull << stop) - 1);
          if (none & upto) {  // a tile up to it has not published yet
            if (++spins > kChainSpins) {
              if (lane == 0) atomicCAS(&h->err, 0, HULL_EINTERNAL);
              break;
            }
            continue;
          }
          int x = lane <= stop ? (int)(unsigned)(w & 0xffffffffull) : 0;
          for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
          prefix += x;
          if (stop < 64) break;
          newest -= 64;  // 64 sums: the prefix lies further back
        }
      }
      if (threadIdx.x == 0) {
        s_prefix = prefix;
        if (tile > 0) chain_store(&W[tile], kChainIncl | ep | (unsigned)(prefix + total));
      }
    }
    __syncthreads();
    int run = s_prefix + ex;
    for (int j = 0; j < kScanItems; ++j) {
      if (base + j < len) jb.out[base + j] = run;
      run += v[j];
    }
    if (tile == ntiles - 1 && threadIdx.x == 0 && jb.total) *jb.total = s_prefix + total;
    __syncthreads();  // s_prefix is rewritten by the next tile
  }
}

int32_t exclusive_scan_chained(const ScanJobs& J, int add, int64_t cap, unsigned long long* words,
                               int64_t wstride, unsigned epoch, Header* h, hipStream_t s) {
  if (cap <= 0 || J.count <= 0) return HULL_OK;
  const int64_t blocks = (cap + kScanBlock - 1) / kScanBlock;
  if (J.count > kMaxScanJobs || blocks > wstride || epoch == 0 || epoch > 0x3fffffffu)
    return HULL_EINVAL;
  const unsigned grid = (unsigned)(blocks < kScanDevGrid ? blocks : kScanDevGrid);
  hipLaunchKernelGGL(k_scan_chained, dim3(grid, J.count), dim3(kSortThreads), 0, s, J, add, cap,
                     words, wstride, epoch, h);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

int32_t scan_chained_i32(const int32_t* in, int32_t* out, int64_t len, unsigned long long* words,
                         int64_t wstride, unsigned epoch, Header* h, hipStream_t s) {
  if (len <= 0) return HULL_OK;
  ScanJobs J{};
  J.j[0] = ScanJob{in, out, nullptr, nullptr};
  J.count = 1;
  return exclusive_scan_chained(J, 0, len, words, wstride, epoch, h, s);
}

__global__ void __launch_bounds__(256) k_zero_words(unsigned long long* w, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0;
}

void zero_words(unsigned long long* w, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const int64_t b = (count + 255) / 256;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(256), 0, s, w,
                     count);
}

void init_header(Header* h, hipStream_t s) {
  hipLaunchKernelGGL(k_header_init, dim3(1), dim3(64), 0, s, h);
}

template <class InT, class PT>
int32_t sort_points(const InT* d_xyz, int64_t n, const int64_t* hull_off, int64_t H, char* ws,
                    const Plan& pl, hipStream_t s) {
  Header* h = (Header*)(ws + pl.header);
  RadixBufs B;
  B.keys[0] = (uint32_t*)(ws + pl.keys0);
  B.keys[1] = (uint32_t*)(ws + pl.keys1);
  B.vals[0] = (int32_t*)(ws + pl.vals0);
  B.vals[1] = (int32_t*)(ws + pl.vals1);
  int32_t* counts = (int32_t*)(ws + pl.counts);
  int32_t* hid = nullptr;
  int hull_passes = 0;
  if (hull_off && H > 1) {
    hid = (int32_t*)(ws + pl.hid);
    int hb = 0;
    while (hb < 31 && ((H - 1) >> hb) != 0) ++hb;
    hull_passes = (hb + kRadixBits - 1) / kRadixBits;
  }
  const int tiles = (int)pl.tiles;
  // the status words of the call's one-launch scans start from zero here:
  // the sort's passes use epochs 1..8, the merge levels higher ones
  unsigned long long* words = (unsigned long long*)(ws + pl.chain_words);
  zero_words(words, kChainJobs * pl.chain_stride, s);
  unsigned eg = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  if (eg < 1) eg = 1;
  hipLaunchKernelGGL(k_extent<InT>, dim3(eg), dim3(256), 0, s, d_xyz, n, h);
  hipLaunchKernelGGL(k_nbits, dim3(1), dim3(64), 0, s, h);
  if (hid) hipLaunchKernelGGL(k_hull_ids, dim3(eg), dim3(256), 0, s, hull_off, H, n, hid);
  for (int kind = 0; kind < 2; ++kind) {
    const int npass = kind == 0 ? 4 : hull_passes;
    for (int d = 0; d < npass; ++d) {
      hipLaunchKernelGGL(k_radix_hist<InT>, dim3(tiles), dim3(kSortThreads), 0, s, d_xyz, B, hid, n,
                         kind, d, tiles, counts, h);
      int32_t rc = scan_chained_i32(counts, counts, pl.count_len, words, pl.chain_stride,
                                    (unsigned)(1 + kind * 4 + d), h, s);
      if (rc) return rc;
      hipLaunchKernelGGL(k_radix_scatter<InT>, dim3(tiles), dim3(kSortThreads), 0, s, d_xyz, B, hid, n,
                         kind, d, tiles, counts, h);
    }
  }
  hipLaunchKernelGGL((k_gather<InT, PT>), dim3(eg), dim3(256), 0, s, d_xyz, B, hid, hull_off,
                     hull_passes, n, (PT*)(ws + pl.pts), h);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

template int32_t sort_points<int32_t, int4>(const int32_t*, int64_t, const int64_t*, int64_t,
                                            char*, const Plan&, hipStream_t);
template int32_t sort_points<int64_t, WPt>(const int64_t*, int64_t, const int64_t*, int64_t,
                                           char*, const Plan&, hipStream_t);

}  // namespace hull
