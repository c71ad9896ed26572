// 2-d Delaunay triangulation by lifting: the lower hull of the points
// (x, y, x^2 + y^2) projects to the Delaunay triangulation of (x, y) (the
// widening of the hull named in the paper's future work; the kinetic merge
// itself is unchanged).  With |x|, |y| <= 2^20 the lifted coordinate is at
// most 2^41, inside the hull's wide range, so the same symbolic perturbation
// decides every cocircular or collinear tie.
#include <algorithm>

#include "common.hpp"

namespace hull {

constexpr int32_t kMaxPlanar = 1 << 20;

// Lifted points as int64 rows; a coordinate out of range becomes a lifted
// value the hull's own range check rejects (HULL_ERANGE in d_info[0]).
__global__ void __launch_bounds__(256) k_lift(const int32_t* __restrict__ xy, int64_t n,
                                              int64_t* __restrict__ xyz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = xy[2 * i], y = xy[2 * i + 1];
    const bool ok = x >= -kMaxPlanar && x <= kMaxPlanar && y >= -kMaxPlanar && y <= kMaxPlanar;
    const int64_t X = ok ? x : 0, Y = ok ? y : 0;
    xyz[3 * i] = X;
    xyz[3 * i + 1] = Y;
    xyz[3 * i + 2] = ok ? X * X + Y * Y : kMaxWideZ + 1;
  }
}

// Lower faces point their normal to -z, so seen from +z they run clockwise:
// swap two corners for counter-clockwise triangles in the plane.
__global__ void __launch_bounds__(256) k_ccw(int32_t* tris, const int64_t* info) {
  const int64_t T = info[0] == 0 ? info[1] : 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < T;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = tris[3 * t + 1];
    tris[3 * t + 1] = tris[3 * t + 2];
    tris[3 * t + 2] = b;
  }
}

static size_t round256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace hull

extern "C" {

int32_t hull_delaunay_workspace_bytes(int64_t n, size_t* bytes) {
  size_t hb = 0;
  int32_t rc = hull_workspace_bytes(n, HULL_WS_WIDE, &hb);
  if (rc || !bytes) return rc ? rc : HULL_EINVAL;
  *bytes = hull::round256(hb) + hull::round256((size_t)(n > 0 ? n : 1) * 24);
  return HULL_OK;
}

int32_t hull_delaunay(const int32_t* d_xy, int64_t n, int32_t* d_tris, int64_t cap, int64_t* d_info,
                      void* d_ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  if (n < 0 || n > hull::kMaxN || !d_info || (n > 0 && !d_xy) || !d_tris || cap < 2 * n || !d_ws)
    return HULL_EINVAL;
  if (hull_delaunay_workspace_bytes(n, &need) || ws_bytes < need) return HULL_EWORKSPACE;
  hull::clear_stale_hip_error();
  hipStream_t s = (hipStream_t)stream;
  size_t hb = 0;
  hull_workspace_bytes(n, HULL_WS_WIDE, &hb);
  const size_t head = hull::round256(hb);
  int64_t* xyz = (int64_t*)((char*)d_ws + head);
  if (n > 0) {
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(hull::k_lift, dim3(g), dim3(256), 0, s, d_xy, n, xyz);
  }
  int32_t rc = hull::hull_runs(n > 0 ? xyz : (const int64_t*)nullptr, n, d_tris, cap, d_info, d_ws, head, s, true,
                               false, nullptr, 0);
  if (rc) return rc;
  hipLaunchKernelGGL(hull::k_ccw, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + 255) / 256, 4096))),
                     dim3(256), 0, s, d_tris, d_info);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

}  // extern "C"
