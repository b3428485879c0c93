// Binning and stable sort of one environment's particles with no device
// allocation: the variant of mpm_sort_keys for callers that cannot allocate
// (code under graph capture, serving loops, harnesses that forbid it). Its
// scratch -- the key copy and the ping-pong buffers of the radix sort, and the
// per-block digit counts -- is one file-scope device array, held by every GPU
// the library runs on until the process ends. Calls that overlap on one GPU
// share that array and race; the digit counts are rewritten in full by every
// pass, so nothing in it must start at zero.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mpm.h"
#include "mpm_kernels.h"

namespace {

constexpr int64_t kMax = MPM_SORT_NOALLOC_MAX;   // particles per call
constexpr int64_t kBlocksMax = (kMax + mpmx::RS_TILE - 1) / mpmx::RS_TILE;
// uint32 words: sort keys, key and value ping-pong buffers, digit counts and totals
constexpr int64_t kScratchWords = 3 * kMax + 256 * (kBlocksMax + 1);
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {

std::mutex g_mutex;
uint32_t* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

// the address of this device's copy of the array, looked up once per device
hipError_t scratch_on_current_device(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

// the binning key of mpm_sort_keys for a lone environment: tile * 64 + cell of
// the clamped base node floor(x n - 1/2); written to keys (the output) and to
// sk (the copy the sort permutes); vals = identity
__global__ void __launch_bounds__(256) k_keys_one_env(const float* __restrict__ x, int64_t n, int grid_n,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ sk,
                                                      uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int T = grid_n >> 2;
  int b[3];
  for (int a = 0; a < 3; ++a) {
    const int q = mpmx::base_floor(x[3 * i + a], grid_n);
    b[a] = q < 0 ? 0 : (q > grid_n - 3 ? grid_n - 3 : q);
  }
  const uint32_t tile = (uint32_t)(((b[0] >> 2) * T + (b[1] >> 2)) * T + (b[2] >> 2));
  const uint32_t cell = (uint32_t)(((b[0] & 3) << 4) | ((b[1] & 3) << 2) | (b[2] & 3));
  const uint32_t key = tile * 64u + cell;
  keys[i] = key;
  sk[i] = key;
  vals[i] = (uint32_t)i;
}

}  // namespace

extern "C" int mpm_sort_keys_noalloc(const float* x, int64_t n, int32_t grid_n, uint32_t* keys, uint32_t* perm,
                                     void* stream) {
  if (n < 0 || n > kMax) return MPM_INVALID_ARG;
  if (grid_n < 12 || grid_n % 4 != 0 || grid_n > 1024) return MPM_INVALID_ARG;
  if (n == 0) return MPM_OK;
  if (!x || !keys || !perm) return MPM_INVALID_ARG;
  uint32_t* ptr = nullptr;
  if (scratch_on_current_device(&ptr) != hipSuccess) return MPM_DEVICE_ERROR;
  const hipStream_t s = (hipStream_t)stream;
  uint32_t* sk = ptr;
  uint32_t* k1 = ptr + kMax;
  uint32_t* v1 = ptr + 2 * kMax;
  uint32_t* counts = ptr + 3 * kMax;
  hipLaunchKernelGGL(k_keys_one_env, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, grid_n, keys, sk, perm);
  const int cell_bits = ceil_log2((uint64_t)grid_n * grid_n * grid_n);
  const int which = mpmx::launch_radix_sort(sk, perm, k1, v1, counts, n, cell_bits > 0 ? cell_bits : 1, s);
  if (which && hipMemcpyAsync(perm, v1, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return MPM_DEVICE_ERROR;
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_DEVICE_ERROR;
}
