// hull_full without a caller workspace: the scratch memory of the call lives
// in a fixed device array of the library, for callers that cannot allocate
// (code under HIP graph capture, serving loops, harnesses that forbid
// allocation).  The kernels and the method are those of hull_full.
#include <mutex>

#include "common.hpp"

namespace hull {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

// The array itself.  Host code never passes this name to a kernel (on the
// host it only stands for the symbol): the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the array on the current device (found on the first
// call on that device).  Returns HULL_EHIP if HIP cannot give it.
static int32_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    note_hip_error(e);
    return HULL_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return HULL_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      note_hip_error(e);
      return HULL_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HULL_OK;
}

}  // namespace hull

extern "C" int32_t hull_full_noalloc(const int32_t* d_xyz, int64_t n, int32_t* d_faces, int64_t cap,
                                     int64_t* d_info, void* stream) {
  hull::clear_stale_hip_error();
  if (n < 0 || n > hull::kMaxN) return HULL_EINVAL;
  size_t need = 0;
  int32_t rc = hull_workspace_bytes(n, HULL_WS_STANDARD, &need);
  if (rc) return rc;
  if (need > hull::kScratchBytes) return HULL_EWORKSPACE;
  void* ws = nullptr;
  rc = hull::scratch_ptr(&ws);
  if (rc) return rc;
  return hull::hull_runs(d_xyz, n, d_faces, cap, d_info, ws, hull::kScratchBytes,
                         (hipStream_t)stream, true, true, nullptr, 0);
}
