// Presort by x (Sec. 2: the points are sorted by x before the merges), as a
// stable LSD radix sort of the key x - min(x) carrying the input index, so
// that equal x values stay in input order: ranks follow (x, input index),
// the x-order of the perturbed points.  Then a gather writes the points in
// rank order as int4 (x, y, z, i).
#include <algorithm>

#include "common.hpp"

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

__global__ void __launch_bounds__(256) k_extent(const int32_t* __restrict__ xyz, int64_t n,
                                                Header* h) {
  __shared__ int smin[256], smax[256], sbad[256];
  int lo = 0x7fffffff, hi = -0x7fffffff - 1, bad = 0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    int x = xyz[3 * p], y = xyz[3 * p + 1], z = xyz[3 * p + 2];
    lo = min(lo, x);
    hi = max(hi, x);
    bad |= (x > kMaxCoord) | (x < -kMaxCoord) | (y > kMaxCoord) | (y < -kMaxCoord) |
           (z > kMaxCoord) | (z < -kMaxCoord);
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
// Radix passes.  Pass 0 reads keys straight from xyz (value = input index);
// later passes ping-pong between (keys0, vals0) and (keys1, vals1).  A pass
// whose digit lies above the key's bit length is skipped.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t load_key(const int32_t* xyz, const uint32_t* keys, int64_t p,
                                             int pass, int minx) {
  return pass == 0 ? (uint32_t)((int64_t)xyz[3 * p] - minx) : keys[p];
}

__global__ void __launch_bounds__(kSortThreads)
    k_radix_hist(const int32_t* __restrict__ xyz, const uint32_t* __restrict__ keys, int64_t n,
                 int pass, int tiles, int32_t* __restrict__ counts, const Header* h) {
  if (pass > 0 && pass * kRadixBits >= h->nbits) return;
  __shared__ int hist[kBuckets];
  hist[threadIdx.x] = 0;
  __syncthreads();
  int minx = h->minx;
  int64_t base = (int64_t)blockIdx.x * kTile;
  for (int j = 0; j < kSortItems; ++j) {
    int64_t p = base + j * kSortThreads + threadIdx.x;
    if (p < n) {
      uint32_t k = load_key(xyz, keys, p, pass, minx);
      atomicAdd(&hist[(k >> (pass * kRadixBits)) & (kBuckets - 1)], 1);
    }
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * tiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads)
    k_radix_scatter(const int32_t* __restrict__ xyz, const uint32_t* __restrict__ keys,
                    const int32_t* __restrict__ vals, int64_t n, int pass, int tiles,
                    const int32_t* __restrict__ offsets, uint32_t* __restrict__ keys_out,
                    int32_t* __restrict__ vals_out, const Header* h) {
  if (pass > 0 && pass * kRadixBits >= h->nbits) return;
  constexpr int kWaves = kSortThreads / 64;
  __shared__ int base[kBuckets];
  __shared__ int wcnt[kWaves][kBuckets];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base[tid] = offsets[(int64_t)tid * tiles + blockIdx.x];
  const int minx = h->minx;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tbase = (int64_t)blockIdx.x * kTile;
  for (int j = 0; j < kSortItems; ++j) {
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    int64_t p = tbase + j * kSortThreads + tid;
    bool valid = p < n;
    uint32_t k = 0;
    int v = 0;
    if (valid) {
      k = load_key(xyz, keys, p, pass, minx);
      v = pass == 0 ? (int)p : vals[p];
    }
    int d = (k >> (pass * kRadixBits)) & (kBuckets - 1);
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < kRadixBits; ++b) {
      uint64_t on = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? on : ~on;
    }
    int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    int pos = 0;
    if (valid) {
      pos = base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
    base[tid] += add;
    if (valid) {
      keys_out[pos] = k;
      vals_out[pos] = v;
    }
    __syncthreads();
  }
}

// Gather the points in rank order; the sorted values sit in the buffer the
// last executed pass wrote.
__global__ void __launch_bounds__(256)
    k_gather(const int32_t* __restrict__ xyz, const int32_t* __restrict__ vals0,
             const int32_t* __restrict__ vals1, int64_t n, int4* __restrict__ pts,
             const Header* h) {
  int passes = (h->nbits + kRadixBits - 1) / kRadixBits;
  if (passes < 1) passes = 1;
  const int32_t* v = (passes & 1) ? vals0 : vals1;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    int i = v[r];
    pts[r] = make_int4(xyz[3 * (int64_t)i], xyz[3 * (int64_t)i + 1], xyz[3 * (int64_t)i + 2], i);
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 (three phases: tile sums, scan of the sums, tiles).
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

__global__ void __launch_bounds__(kSortThreads)
    k_scan_tile_sums(const int32_t* __restrict__ in, int64_t len, int32_t* __restrict__ sums) {
  __shared__ int wsum[kSortThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int s = 0;
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < len) s += in[base + j];
  int total;
  block_exclusive_scan(s, wsum, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kSortThreads) k_scan_sums(int32_t* sums, int64_t nsums) {
  __shared__ int wsum[kSortThreads / 64];
  int carry = 0;
  for (int64_t b = 0; b < nsums; b += kSortThreads) {
    int64_t q = b + threadIdx.x;
    int x = q < nsums ? sums[q] : 0;
    int total;
    int ex = block_exclusive_scan(x, wsum, total);
    if (q < nsums) sums[q] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(kSortThreads)
    k_scan_tiles(const int32_t* __restrict__ in, int64_t len, const int32_t* __restrict__ sums,
                 int32_t* __restrict__ out) {
  __shared__ int wsum[kSortThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < len ? in[base + j] : 0;
    s += v[j];
  }
  int total;
  int run = block_exclusive_scan(s, wsum, total) + sums[blockIdx.x];
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < len) out[base + j] = run;
    run += v[j];
  }
}

int32_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t len, int32_t* partials,
                           hipStream_t s) {
  if (len <= 0) return HULL_OK;
  int64_t blocks = (len + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)blocks), dim3(kSortThreads), 0, s, in, len,
                     partials);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kSortThreads), 0, s, partials, blocks);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)blocks), dim3(kSortThreads), 0, s, in, len,
                     partials, out);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}


void init_header(Header* h, hipStream_t s) {
  hipLaunchKernelGGL(k_header_init, dim3(1), dim3(64), 0, s, h);
}

int32_t sort_points(const int32_t* d_xyz, int64_t n, char* ws, const Plan& pl, hipStream_t s) {
  Header* h = (Header*)(ws + pl.header);
  uint32_t* keys[2] = {(uint32_t*)(ws + pl.keys0), (uint32_t*)(ws + pl.keys1)};
  int32_t* vals[2] = {(int32_t*)(ws + pl.vals0), (int32_t*)(ws + pl.vals1)};
  int32_t* counts = (int32_t*)(ws + pl.counts);
  int32_t* partials = (int32_t*)(ws + pl.partials);
  int tiles = (int)pl.tiles;
  unsigned eg = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  if (eg < 1) eg = 1;
  hipLaunchKernelGGL(k_extent, dim3(eg), dim3(256), 0, s, d_xyz, n, h);
  hipLaunchKernelGGL(k_nbits, dim3(1), dim3(64), 0, s, h);
  for (int pass = 0; pass < 4; ++pass) {
    int src = (pass + 1) & 1, dst = pass & 1;  // pass 0 writes buffer 0
    hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(kSortThreads), 0, s, d_xyz, keys[src], n,
                       pass, tiles, counts, h);
    int32_t rc = exclusive_scan_i32(counts, counts, pl.count_len, partials, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(kSortThreads), 0, s, d_xyz, keys[src],
                       vals[src], n, pass, tiles, counts, keys[dst], vals[dst], h);
  }
  hipLaunchKernelGGL(k_gather, dim3(eg), dim3(256), 0, s, d_xyz, vals[0], vals[1], n,
                     (int4*)(ws + pl.pts), h);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

}  // namespace hull
