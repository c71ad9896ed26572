// Face adjacency of hull surfaces: for every face and each of its three
// directed edges, the face across that edge (the half-edge twin) -- the
// connectivity of an edge-list structure, which the paper names as the
// prerequisite for further algorithms (Sec. "Conclusion", future work; Sec.
// "Introduction" on the missing doubly connected edge list).
//
// A hash table of directed edges in the caller's workspace: every half-edge
// (a -> b) of face f inserts the key (a, b) with the value 3f + k; then every
// half-edge looks up (b, a).  Keys use point indices made global with the
// cloud's point offset, so clouds of a batch never match each other.  Open
// addressing, linear probing, table size a power of two >= 2x the half-edges
// (every probe sequence ends at an empty slot or its key).
#include <algorithm>

#include "common.hpp"

namespace hull {

constexpr unsigned long long kEmptyKey = ~0ull;
// Half-edge ids 3f + k are stored as int32: at most this many faces.
constexpr int64_t kMaxAdjFaces = (int64_t(INT32_MAX) - 2) / 3;

struct __align__(16) EdgeSlot {
  unsigned long long key;
  int val;
  int pad;
};

__device__ __forceinline__ int64_t owner64(const int64_t* off, int64_t count, int64_t x) {
  int64_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t slot_of(unsigned long long key, int bits) {
  return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits);
}

struct AdjArgs {
  const int32_t* faces;
  int64_t F;
  const int64_t* face_off;  // [H + 1] or null (one surface)
  const int64_t* pt_off;    // [H + 1] or null
  int64_t H;
  EdgeSlot* table;
  int bits;
  int32_t* adj;
  int64_t* info;
  int* err;    // device status word (in the workspace)
  int* open;   // half-edges without a twin
};

// The half-edge e = 3f + k as a key (a, b), a and b made global; false when
// an index lies outside its cloud.
__device__ __forceinline__ bool edge_key(const AdjArgs& A, int64_t e, bool reverse,
                                         unsigned long long& key) {
  const int64_t f = e / 3;
  const int k = (int)(e - 3 * f);
  int64_t a = A.faces[3 * f + k], b = A.faces[3 * f + (k == 2 ? 0 : k + 1)];
  if (A.face_off) {
    const int64_t h = owner64(A.face_off, A.H, f);
    const int64_t p0 = A.pt_off[h], np = A.pt_off[h + 1] - p0;
    if (a < 0 || b < 0 || a >= np || b >= np) return false;
    a += p0;
    b += p0;
  } else if (a < 0 || b < 0) {
    return false;
  }
  key = reverse ? ((unsigned long long)b << 32) | (unsigned long long)a
                : ((unsigned long long)a << 32) | (unsigned long long)b;
  return true;
}

__global__ void __launch_bounds__(256) k_adj_clear(AdjArgs A) {
  const int64_t size = int64_t(1) << A.bits;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < size;
       i += (int64_t)gridDim.x * blockDim.x)
    A.table[i].key = kEmptyKey;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *A.err = 0;
    *A.open = 0;
  }
}

__global__ void __launch_bounds__(256) k_adj_insert(AdjArgs A) {
  const int64_t size = int64_t(1) << A.bits, mask = size - 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 3 * A.F;
       e += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long key;
    if (!edge_key(A, e, false, key)) {
      atomicCAS(A.err, 0, HULL_ERANGE);
      continue;
    }
    int64_t i = (int64_t)slot_of(key, A.bits);
    for (int64_t probe = 0; probe < size; ++probe, i = (i + 1) & mask) {
      const unsigned long long prev = atomicCAS(&A.table[i].key, kEmptyKey, key);
      if (prev == kEmptyKey) {
        A.table[i].val = (int)e;
        break;
      }
      if (prev == key) {  // the same directed edge twice: not a 2-manifold
        atomicCAS(A.err, 0, HULL_EINTERNAL);
        break;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_adj_lookup(AdjArgs A) {
  const int64_t size = int64_t(1) << A.bits, mask = size - 1;
  const bool bad = *A.err != 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 3 * A.F;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t twin = -1;
    unsigned long long key;
    if (!bad && edge_key(A, e, true, key)) {
      int64_t i = (int64_t)slot_of(key, A.bits);
      for (int64_t probe = 0; probe < size; ++probe, i = (i + 1) & mask) {
        const unsigned long long k = A.table[i].key;
        if (k == key) {
          twin = A.table[i].val / 3;
          break;
        }
        if (k == kEmptyKey) break;
      }
    }
    A.adj[e] = twin;
    if (twin < 0 && !bad) atomicAdd(A.open, 1);
  }
}

__global__ void k_adj_info(AdjArgs A) {
  if (threadIdx.x == 0) {
    A.info[0] = *A.err;
    A.info[1] = *A.err ? 0 : *A.open;
  }
}

static int table_bits(int64_t F) {
  int bits = 4;
  while ((int64_t(1) << bits) < 6 * F) ++bits;
  return bits;
}

static size_t adj_ws_bytes(int64_t F) { return 256 + (size_t(1) << table_bits(F)) * sizeof(EdgeSlot); }

}  // namespace hull

extern "C" {

int32_t hull_adjacency_workspace_bytes(int64_t F, size_t* bytes) {
  if (!bytes || F < 0 || F > hull::kMaxAdjFaces) return HULL_EINVAL;
  *bytes = hull::adj_ws_bytes(F);
  return HULL_OK;
}

int32_t hull_face_adjacency(const int32_t* d_faces, int64_t F, const int64_t* d_face_off,
                            const int64_t* d_pt_off, int64_t H, int32_t* d_adj, int64_t* d_info,
                            void* d_ws, size_t ws_bytes, void* stream) {
  if (F < 0 || F > hull::kMaxAdjFaces || !d_info || !d_ws || (F > 0 && (!d_faces || !d_adj)) ||
      (d_face_off && (!d_pt_off || H < 1)) || (!d_face_off && d_pt_off))
    return HULL_EINVAL;
  if (ws_bytes < hull::adj_ws_bytes(F)) return HULL_EWORKSPACE;
  hull::clear_stale_hip_error();
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)d_ws;
  hull::AdjArgs A{};
  A.faces = d_faces;
  A.F = F;
  A.face_off = d_face_off;
  A.pt_off = d_pt_off;
  A.H = d_face_off ? H : 1;
  A.err = (int*)ws;
  A.open = (int*)(ws + 64);
  A.table = (hull::EdgeSlot*)(ws + 256);
  A.bits = hull::table_bits(F);
  A.adj = d_adj;
  A.info = d_info;
  const int64_t size = int64_t(1) << A.bits;
  unsigned gt = (unsigned)std::min<int64_t>((size + 255) / 256, 8192);
  unsigned ge = (unsigned)std::max<int64_t>(1, std::min<int64_t>((3 * F + 255) / 256, 8192));
  hipLaunchKernelGGL(hull::k_adj_clear, dim3(gt), dim3(256), 0, s, A);
  hipLaunchKernelGGL(hull::k_adj_insert, dim3(ge), dim3(256), 0, s, A);
  hipLaunchKernelGGL(hull::k_adj_lookup, dim3(ge), dim3(256), 0, s, A);
  hipLaunchKernelGGL(hull::k_adj_info, dim3(1), dim3(64), 0, s, A);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

}  // extern "C"
