// The tree build for callers that cannot allocate device memory: the radix
// sort's workspace (keys and values double-buffered, digit counts, scan block
// totals) lives in one fixed device array of this library instead of a
// caller workspace.  The kernels are the ones of the ordinary tree build.
//
// The array is a file-scope __device__ variable, so each device the library
// runs on holds its own copy, at its own address, from the first call on that
// device until the process ends (kScratchBytes = 67,371,264 bytes).  In host
// code the variable's name is not a device address: the address comes from
// hipGetSymbolAddress, looked up once per device with that device current and
// kept in g_scratch_ptr.  Every call on a device shares that device's array,
// so calls that overlap on one device (different streams, different host
// threads) race on it; nothing in it has to start at zero, because every pass
// writes all the workspace it later reads.
#include <mutex>

#include "fmm2d_internal.h"

namespace fmm2d {

constexpr size_t kScratchBytes = tree_ws::bytes(kNoAllocMaxPoints);
static_assert(kScratchBytes == 67371264, "the size the header states");
static_assert(kNoAllocMaxPoints == FMM2D_NOALLOC_MAX_POINTS, "the limit the header states");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch`.
static int scratch_on_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return set_error(FMM2D_EHIP, "build_tree_noalloc: no usable current device (%d)", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return set_error(FMM2D_EHIP, "build_tree_noalloc: hipGetSymbolAddress failed on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FMM2D_OK;
}

int launch_build_tree_noalloc(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                              uint32_t *domain_flag, hipStream_t s) {
  if (n > kNoAllocMaxPoints || tree_ws::bytes(n) > kScratchBytes)
    return set_error(FMM2D_EWORKSPACE, "fmm2d_build_tree_noalloc: n = %lld exceeds the %lld points its array holds",
                     (long long)n, (long long)kNoAllocMaxPoints);
  void *ws = nullptr;
  const int rc = scratch_on_current_device(&ws);
  if (rc != FMM2D_OK) return rc;
  return launch_build_tree(xy, n, depth, perm, leaf_start, domain_flag, ws, s);
}

}  // namespace fmm2d
