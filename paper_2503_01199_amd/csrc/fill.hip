// Fill kernels (used instead of memset nodes so that enqueued work stays
// capturable in a HIP graph).
#include "gsr_internal.h"

namespace gsr {
namespace {

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u32<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
}

void fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_f32<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
}

}  // namespace gsr
