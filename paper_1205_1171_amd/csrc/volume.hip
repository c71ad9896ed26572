// Volume and surface area of hull surfaces, and their gradients with respect
// to float point positions on a fixed face set, batched over clouds.
//
// For the outward faces (a, b, d) of a closed surface and a reference point c
// (here the cloud's point 0, inside the hull, so every term is >= 0):
//   V = 1/6 sum_f (a - c) . ((b - c) x (d - c)),  A = 1/2 sum_f |n_f|,
//   n_f = (b - a) x (d - a)  (the same for every rotation of the face).
// Gradients (c drops out on a closed surface):
//   dV/dp = 1/6 sum_{f containing p} n_f,
//   dA/da = 1/2 (b - d) x n_f / |n_f| for the corner a of f = (a, b, d)
//           (0 for a face of zero area).
#include <stddef.h>

#include "common.hpp"

namespace hull {

constexpr int kVolThreads = 256;

struct Kahan {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
};

__device__ __forceinline__ float3 sub3(float3 a, float3 b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 ld3(const float* p, int64_t i) {
  return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}

// Deterministic block reduction of two floats (wave shuffles, then LDS).
__device__ __forceinline__ float2 block_sum2(float x, float y) {
  __shared__ float sx[kVolThreads / 64], sy[kVolThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    x += __shfl_down(x, o);
    y += __shfl_down(y, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sx[wave] = x;
    sy[wave] = y;
  }
  __syncthreads();
  float tx = 0.f, ty = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < kVolThreads / 64; ++w) {
      tx += sx[w];
      ty += sy[w];
    }
  return make_float2(tx, ty);
}

// One workgroup per cloud (blockIdx.x).
__global__ void __launch_bounds__(kVolThreads)
    k_vol_area_fwd(const float* __restrict__ p, const int64_t* __restrict__ pt_off,
                   const int32_t* __restrict__ faces, const int64_t* __restrict__ face_off,
                   float* __restrict__ V, float* __restrict__ A) {
  const int h = blockIdx.x;
  const int64_t po = pt_off[h], pn = pt_off[h + 1] - po;
  const int64_t f0 = face_off[h], f1 = face_off[h + 1];
  Kahan kv, ka;
  if (pn > 0) {
    const float3 c = ld3(p, po);
    for (int64_t f = f0 + threadIdx.x; f < f1; f += kVolThreads) {
      const int ia = faces[3 * f], ib = faces[3 * f + 1], id = faces[3 * f + 2];
      const float3 a = ld3(p, po + ia), b = ld3(p, po + ib), d = ld3(p, po + id);
      kv.add(dot3(sub3(a, c), cross3(sub3(b, c), sub3(d, c))));
      const float3 n = cross3(sub3(b, a), sub3(d, a));
      ka.add(sqrtf(dot3(n, n)));
    }
  }
  float2 t = block_sum2(kv.s - kv.c, ka.s - ka.c);
  if (threadIdx.x == 0) {
    V[h] = t.x / 6.f;
    A[h] = t.y * 0.5f;
  }
}

__global__ void __launch_bounds__(256) k_vol_area_zero(float* __restrict__ g,
                                                       const int64_t* __restrict__ pt_off,
                                                       int32_t H) {
  const int64_t total = 3 * pt_off[H];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x)
    g[q] = 0.f;
}

// Faces of cloud blockIdx.y, spread over gridDim.x workgroups.
__global__ void __launch_bounds__(256)
    k_vol_area_bwd(const float* __restrict__ p, const int64_t* __restrict__ pt_off,
                   const int32_t* __restrict__ faces, const int64_t* __restrict__ face_off,
                   const float* __restrict__ gV, const float* __restrict__ gA,
                   float* __restrict__ grad) {
  const int h = blockIdx.y;
  const int64_t po = pt_off[h];
  const int64_t f0 = face_off[h], f1 = face_off[h + 1];
  const float sv = gV ? gV[h] / 6.f : 0.f, sa = gA ? gA[h] * 0.5f : 0.f;
  for (int64_t f = f0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < f1;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ia = po + faces[3 * f], ib = po + faces[3 * f + 1], id = po + faces[3 * f + 2];
    const float3 a = ld3(p, ia), b = ld3(p, ib), d = ld3(p, id);
    const float3 n = cross3(sub3(b, a), sub3(d, a));
    const float nn = sqrtf(dot3(n, n));
    const float inv = nn > 0.f ? sa / nn : 0.f;
    const float3 m = make_float3(n.x * inv, n.y * inv, n.z * inv);  // gA/2 * unit normal
    const float3 v = make_float3(n.x * sv, n.y * sv, n.z * sv);    // gV/6 * n
    const float3 ga = cross3(sub3(b, d), m), gb = cross3(sub3(d, a), m), gd = cross3(sub3(a, b), m);
    atomicAdd(&grad[3 * ia + 0], v.x + ga.x);
    atomicAdd(&grad[3 * ia + 1], v.y + ga.y);
    atomicAdd(&grad[3 * ia + 2], v.z + ga.z);
    atomicAdd(&grad[3 * ib + 0], v.x + gb.x);
    atomicAdd(&grad[3 * ib + 1], v.y + gb.y);
    atomicAdd(&grad[3 * ib + 2], v.z + gb.z);
    atomicAdd(&grad[3 * id + 0], v.x + gd.x);
    atomicAdd(&grad[3 * id + 1], v.y + gd.y);
    atomicAdd(&grad[3 * id + 2], v.z + gd.z);
  }
}

}  // namespace hull

extern "C" {

int32_t hull_volume_area_fwd(const float* d_p, const int64_t* d_pt_off, const int32_t* d_faces,
                             const int64_t* d_face_off, int32_t H, float* d_V, float* d_A,
                             void* stream) {
  if (H < 0 || (H > 0 && (!d_p || !d_pt_off || !d_faces || !d_face_off || !d_V || !d_A)))
    return HULL_EINVAL;
  if (H == 0) return HULL_OK;
  hull::clear_stale_hip_error();
  hipLaunchKernelGGL(hull::k_vol_area_fwd, dim3(H), dim3(hull::kVolThreads), 0,
                     (hipStream_t)stream, d_p, d_pt_off, d_faces, d_face_off, d_V, d_A);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

int32_t hull_volume_area_bwd(const float* d_p, const int64_t* d_pt_off, const int32_t* d_faces,
                             const int64_t* d_face_off, int32_t H, const float* d_gV,
                             const float* d_gA, float* d_grad_p, void* stream) {
  if (H < 0 || (H > 0 && (!d_p || !d_pt_off || !d_faces || !d_face_off || !d_grad_p)))
    return HULL_EINVAL;
  if (H == 0) return HULL_OK;
  hull::clear_stale_hip_error();
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(hull::k_vol_area_zero, dim3(1024), dim3(256), 0, s, d_grad_p, d_pt_off, H);
  hipLaunchKernelGGL(hull::k_vol_area_bwd, dim3(16, H), dim3(256), 0, s, d_p, d_pt_off, d_faces,
                     d_face_off, d_gV, d_gA, d_grad_p);
  HULL_LAUNCH_CHECK();
  return HULL_OK;
}

}  // extern "C"
