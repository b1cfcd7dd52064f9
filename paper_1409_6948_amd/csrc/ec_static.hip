// The library's one static device buffer, for the allocation-free sweep entry
// point (ec_sweep_static in ec_api.cpp): the cell lists, chain draws,
// tallies, counters and the device record of one system live here instead of
// a caller workspace.  Each GPU holds its own copy of the array until the
// process ends; host code never uses the array's name as an address, only the
// per-device address that hipGetSymbolAddress returns.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ec_internal.h"

namespace ec {
namespace {

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// Clear [p, p + bytes) (a fill kernel, so that a captured graph holds no
// memset node).
__global__ void k_fill_zero(unsigned long long* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Store the device record (passed by value, so a captured graph keeps its own
// copy) and the number of the first sweep.
__global__ void k_store_record(Dev rec, Dev* dst, int64_t first_sweep) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *dst = rec;
    *rec.sweep_ctr = first_sweep;
  }
}

// Digests of sweeps first .. first + n - 1 (n <= kDigestRing) and the device
// error word, to caller device buffers (either may be null).
__global__ void k_copy_out(const Dev* __restrict__ ds, int64_t first, int64_t n,
                           unsigned long long* digests, int32_t* err) {
  const Dev& d = *ds;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (digests && i < n) digests[i] = d.digest_ring[(first + i) % kDigestRing];
  if (err && i == 0) *err = *d.err;
}

}  // namespace

hipError_t static_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

hipError_t launch_static_setup(const Dev& rec, Dev* dst, unsigned char* base, size_t bytes,
                               int64_t first_sweep, hipStream_t st) {
  const size_t words = (bytes + 7) / 8;
  const unsigned blocks = (unsigned)((words + 255) / 256 < 1024 ? (words + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st,
                     (unsigned long long*)base, words);
  hipLaunchKernelGGL(k_store_record, dim3(1), dim3(64), 0, st, rec, dst, first_sweep);
  return hipGetLastError();
}

hipError_t launch_static_copy_out(const Dev* ds, int64_t first, int64_t n,
                                  unsigned long long* digests, int32_t* err, hipStream_t st) {
  const unsigned blocks = (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1);
  hipLaunchKernelGGL(k_copy_out, dim3(blocks), dim3(256), 0, st, ds, first, n, digests, err);
  return hipGetLastError();
}

}  // namespace ec
