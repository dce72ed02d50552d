// Device-resident scratch of the no-allocation batched raster
// (gsr_raster_batch_noalloc): the raster work-item list and its count live in a
// file-scope device array instead of a caller workspace, so the call allocates
// nothing. Each GPU holds its own copy of the array for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns for
// that device (the array's name in host code is a host-side stand-in).
#include <mutex>

#include "raster_common.h"

namespace gsr {
namespace {

constexpr int64_t kScratchTiles = GSR_NOALLOC_MAX_TILES;  // 32 frames of 1920x1080
constexpr size_t kScratchWords = (size_t)((max_items(kScratchTiles) + 63) / 64 * 64) + 64;  // items, then the count

static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
uint32_t* g_ptr[kMaxDevices] = {};

}  // namespace

int64_t noalloc_max_tiles() { return kScratchTiles; }

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_ptr[device]) return hipSuccess;
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess) return e;
  g_ptr[device] = static_cast<uint32_t*>(p);
  return hipSuccess;
}

uint32_t* noalloc_scratch(int device, size_t* words) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (words) *words = kScratchWords;
  return (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
}

}  // namespace gsr
