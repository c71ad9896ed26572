// Entry points of the wide coordinate range (int64 rows, |x|, |y| <= 2^30,
// |z| <= 2^42) and of float input snapped to a lattice.  The paper keeps the
// points as single-precision floats on the GPU (Sec. 3, Fig.
// "point_datatypes"); here they are mapped exactly onto an integer lattice
// by one power-of-two scale and a round to nearest (ties to even), and the
// hull is the exact perturbed hull of the lattice points.
#include <algorithm>

#include "common.hpp"
#include "predicates.hpp"

namespace hull {

static size_t round256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of the float entry points: the wide hull's plan, then the
// lattice rows (int64 [n, 3]), then one line holding the largest magnitude.
struct F32Layout {
  size_t hull, rows, amax, total;
};

static F32Layout f32_layout(int64_t n) {
  F32Layout L;
  L.hull = round256(make_plan(n, 1, kMinWalkSegment, (int)sizeof(WPt)).total);
  L.rows = round256((size_t)(n > 0 ? n : 1) * 3 * sizeof(int64_t));
  L.amax = 256;
  L.total = L.hull + L.rows + L.amax;
  return L;
}

__global__ void k_amax_init(uint32_t* amax) {
  if (threadIdx.x == 0) amax[0] = 0;
}

// The largest |c| over all 3n coordinates, as the bit pattern of a
// non-negative float (which orders like the float itself); NaN and infinity
// have the all-ones exponent and so compare above every finite value.
__global__ void __launch_bounds__(256) k_amax(const float* __restrict__ xyz, int64_t m,
                                              uint32_t* amax) {
  __shared__ uint32_t red[256];
  uint32_t a = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < m;
       q += (int64_t)gridDim.x * blockDim.x)
    a = max(a, __float_as_uint(xyz[q]) & 0x7fffffffu);
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0]) atomicMax(amax, red[0]);
}

// E: the least integer with amax <= 2^E (0 for amax = 0).
__device__ __forceinline__ int exponent_bound(float amax) {
  if (amax == 0.0f) return 0;
  int e = 0;
  const double m = frexp((double)amax, &e);  // amax = m 2^e, 1/2 <= m < 1
  return m == 0.5 ? e - 1 : e;
}

// Lattice rows: rint(c * 2^(bits - E)).  A non-finite input makes its row
// fall outside the wide range, so that the hull's range check reports
// HULL_ERANGE.
__global__ void __launch_bounds__(256) k_snap(const float* __restrict__ xyz, int64_t n, int bits,
                                              const uint32_t* amax, int64_t* __restrict__ rows) {
  const uint32_t a = amax[0];
  const bool finite = a < 0x7f800000u;
  const int sh = finite ? bits - exponent_bound(__uint_as_float(a)) : 0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    for (int k = 0; k < 3; ++k) {
      const double c = (double)xyz[3 * p + k];
      rows[3 * p + k] = finite ? (int64_t)rint(ldexp(c, sh)) : kMaxWideZ + 1;
    }
  }
}

static int32_t snap_and_hull(const float* d_xyz, int64_t n, int32_t bits, int32_t* d_faces,
                             int64_t cap, int64_t* d_info, void* d_ws, size_t ws_bytes,
                             hipStream_t s, bool upper) {
  if (n < 0 || n > kMaxN || bits < 1 || bits > 30 || !d_info || (n > 0 && !d_xyz) || !d_faces ||
      cap < 2 * n || !d_ws)
    return HULL_EINVAL;
  const F32Layout L = f32_layout(n);
  if (ws_bytes < L.total) return HULL_EWORKSPACE;
  char* ws = (char*)d_ws;
  int64_t* rows = (int64_t*)(ws + L.hull);
  uint32_t* amax = (uint32_t*)(ws + L.hull + L.rows);
  if (n > 0) {
    const unsigned g = (unsigned)std::min<int64_t>((3 * n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_amax_init, dim3(1), dim3(64), 0, s, amax);
    hipLaunchKernelGGL(k_amax, dim3(g), dim3(256), 0, s, d_xyz, 3 * n, amax);
    hipLaunchKernelGGL(k_snap, dim3(std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0, s,
                       d_xyz, n, (int)bits, (const uint32_t*)amax, rows);
    HULL_LAUNCH_CHECK();
  }
  return hull_runs(n > 0 ? rows : (const int64_t*)nullptr, n, d_faces, cap, d_info, d_ws, L.hull,
                   s, true, upper, nullptr, 0);
}

size_t wide_workspace_bytes(int64_t n) {
  return make_plan(n, 1, kMinWalkSegment, (int)sizeof(WPt)).total;
}

size_t f32_workspace_bytes(int64_t n) { return f32_layout(n).total; }

}  // namespace hull

extern "C" {

int32_t hull_lower_wide(const int64_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                        int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         false, nullptr, 0);
}

int32_t hull_full_wide(const int64_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                       int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, d_ws, ws_bytes, (hipStream_t)stream, true,
                         true, nullptr, 0);
}

int32_t hull_full_f32(const float* d_xyz, int64_t n, int32_t bits, int32_t* d_faces, int64_t cap,
                      int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::snap_and_hull(d_xyz, n, bits, d_faces, cap, d_info, d_ws, ws_bytes,
                             (hipStream_t)stream, true);
}

int32_t hull_lower_f32(const float* d_xyz, int64_t n, int32_t bits, int32_t* d_faces, int64_t cap,
                       int64_t* d_info, void* d_ws, size_t ws_bytes, void* stream) {
  hull::clear_stale_hip_error();
  return hull::snap_and_hull(d_xyz, n, bits, d_faces, cap, d_info, d_ws, ws_bytes,
                             (hipStream_t)stream, false);
}

}  // extern "C"
