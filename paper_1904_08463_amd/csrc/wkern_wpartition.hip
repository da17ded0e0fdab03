// w-plane partition of visibility records (the first three steps of
// Algorithms 1 and 2): sort the records by (absolute) w, cut the sorted
// sequence into M planes of equal size, take each plane's average or median
// w as the w-term its kernel is generated for.
//
// Sort: the w values become 64-bit keys whose unsigned order is the order of
// the key value (|w| or w), and rocPRIM's stable LSD radix sort carries the
// record indices along.  Plane m holds sorted positions
// [floor(m n / M), floor((m + 1) n / M)).  Statistics read the sorted keys
// back as doubles (the key map is invertible), one workgroup per plane,
// every sum in a fixed order.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include <rocprim/device/device_radix_sort.hpp>

#include "wkern.h"
#include "wkern_internal.h"

namespace {

constexpr uint64_t kSign = 0x8000000000000000ull;
constexpr uint64_t kNanKey = ~0ull;
constexpr int kStatThreads = 1024;
constexpr size_t kAlign = 256;

// Key of a record.  |w|: the IEEE bits of a non-negative double already sort
// as unsigned integers.  Signed w: positives get the sign bit set, negatives
// are bit-inverted (larger magnitude -> smaller key).  -0.0 is keyed as
// +0.0, every NaN as the largest key.
__device__ __forceinline__ uint64_t sort_key(double w, int absolute) {
  if (w != w) return kNanKey;
  const uint64_t b = (uint64_t)__double_as_longlong(w);
  if (absolute) return b & ~kSign;
  if (w == 0.0) return kSign;
  return (b & kSign) ? ~b : (b | kSign);
}

// The key value (|w| or w) back from its key.
__device__ __forceinline__ double key_value(uint64_t k, int absolute) {
  if (k == kNanKey) return __longlong_as_double(0x7FF8000000000000ll);
  if (absolute) return __longlong_as_double((long long)k);
  return __longlong_as_double((long long)((k & kSign) ? (k & ~kSign) : ~k));
}

__global__ void k_wkeys(const double* __restrict__ w, int n, int absolute,
                        uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    keys[i] = sort_key(w[i], absolute);
    idx[i] = i;
  }
}

// One workgroup per plane: start offset, mean (fixed-order sum: a strided
// per-thread sum, then a tree over the threads) or median.
__global__ __launch_bounds__(kStatThreads) void k_wplane_stats(const uint64_t* __restrict__ keys,
                                                               int64_t n, int M, int absolute,
                                                               int stat,
                                                               int64_t* __restrict__ planeStart,
                                                               double* __restrict__ wPlane) {
  __shared__ double sh[kStatThreads];
  const int m = blockIdx.x;
  const int64_t s = (int64_t)m * n / M;
  const int64_t e = (int64_t)(m + 1) * n / M;
  const int t = threadIdx.x;
  if (t == 0) {
    planeStart[m] = s;
    if (m == M - 1) planeStart[M] = n;
  }
  const int64_t c = e - s;
  if (stat == 1) {
    if (t == 0) {
      const int64_t mid = s + c / 2;
      wPlane[m] = (c & 1) ? key_value(keys[mid], absolute)
                          : (key_value(keys[mid - 1], absolute) + key_value(keys[mid], absolute)) /
                                2.0;
    }
    return;
  }
  double acc = 0.0;
  for (int64_t j = s + t; j < e; j += kStatThreads) acc += key_value(keys[j], absolute);
  sh[t] = acc;
  for (int o = kStatThreads / 2; o > 0; o >>= 1) {
    __syncthreads();
    if (t < o) sh[t] += sh[t + o];
  }
  if (t == 0) wPlane[m] = sh[0] / (double)c;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

wkern_status pfail(wkern_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  wkern::set_last_error(buf);
  return s;
}

// Workspace: keys in, keys out, record indices in, rocPRIM temporary storage.
wkern_status sort_storage(int n, hipStream_t s, size_t* tmp) {
  *tmp = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, *tmp, (const uint64_t*)nullptr,
                                           (uint64_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, n, 0, 64, s);
  if (e != hipSuccess) return pfail(WKERN_ERR_DEVICE, "sort storage query: %s", hipGetErrorString(e));
  return WKERN_OK;
}

size_t workspace_total(int n, size_t tmp) {
  return align_up((size_t)n * 8) * 2 + align_up((size_t)n * 4) + align_up(tmp);
}

// Scratch of wkern_wpartition_noalloc: the keys, record indices and sort
// storage of wkern_wpartition's workspace, in a device array that the
// library holds for the life of the process (one copy per device, at its own
// address on each).  Host code never uses the array's name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int64_t kStaticMaxRecords = (int64_t)1 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
wkern_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return pfail(WKERN_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return pfail(WKERN_ERR_UNSUPPORTED, "device %d beyond the %d the static scratch covers", dev,
                 kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return pfail(WKERN_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return WKERN_OK;
}

wkern_status check_partition_args(const double* w, int64_t n_records, int32_t n_planes,
                                  int32_t absolute, int32_t stat, const int32_t* order,
                                  const int64_t* plane_start, const double* w_plane) {
  if (!w || !order || !plane_start || !w_plane) return pfail(WKERN_ERR_INVALID_ARG, "NULL argument");
  if (n_planes < 1 || n_records < n_planes)
    return pfail(WKERN_ERR_INVALID_ARG, "need n_records (%lld) >= n_planes (%d) >= 1",
                 (long long)n_records, n_planes);
  if (n_records > 0x7FFFFFFF)
    return pfail(WKERN_ERR_UNSUPPORTED, "n_records %lld above 2^31 - 1", (long long)n_records);
  if (absolute != 0 && absolute != 1) return pfail(WKERN_ERR_INVALID_ARG, "absolute must be 0 or 1");
  if (stat != WKERN_WSTAT_MEAN && stat != WKERN_WSTAT_MEDIAN)
    return pfail(WKERN_ERR_INVALID_ARG, "stat %d unknown", stat);
  return WKERN_OK;
}

// The partition with its scratch at `base` (256-byte aligned, `bytes` long):
// keys, sort, plane statistics, all on `s`.
wkern_status partition_into(const double* w, int n, int32_t n_planes, int32_t absolute,
                            int32_t stat, char* base, size_t bytes, int32_t* order,
                            int64_t* plane_start, double* w_plane, hipStream_t s) {
  size_t tmp = 0;
  wkern_status st = sort_storage(n, s, &tmp);
  if (st != WKERN_OK) return st;
  const size_t need = workspace_total(n, tmp);
  if (bytes < need) return pfail(WKERN_ERR_INVALID_ARG, "workspace %zu bytes < %zu", bytes, need);
  if ((uintptr_t)base % kAlign)
    return pfail(WKERN_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
  uint64_t* keysIn = (uint64_t*)base;
  uint64_t* keysOut = (uint64_t*)(base + align_up((size_t)n * 8));
  int32_t* idxIn = (int32_t*)(base + 2 * align_up((size_t)n * 8));
  void* sortTmp = base + 2 * align_up((size_t)n * 8) + align_up((size_t)n * 4);

  const int grid = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_wkeys, dim3(grid), dim3(256), 0, s, w, n, absolute, keysIn, idxIn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(WKERN_ERR_DEVICE, "key launch: %s", hipGetErrorString(e));
  e = rocprim::radix_sort_pairs(sortTmp, tmp, keysIn, keysOut, idxIn, order, n, 0, 64, s);
  if (e != hipSuccess) return pfail(WKERN_ERR_DEVICE, "radix sort: %s", hipGetErrorString(e));
  hipLaunchKernelGGL(k_wplane_stats, dim3(n_planes), dim3(kStatThreads), 0, s, keysOut,
                     (int64_t)n, n_planes, absolute, stat, plane_start, w_plane);
  e = hipGetLastError();
  if (e != hipSuccess) return pfail(WKERN_ERR_DEVICE, "plane statistics launch: %s", hipGetErrorString(e));
  return WKERN_OK;
}

}  // namespace

extern "C" {

wkern_status wkern_wpartition_workspace(int64_t n_records, size_t* bytes) {
  wkern::set_last_error("");
  if (!bytes) return pfail(WKERN_ERR_INVALID_ARG, "bytes is NULL");
  if (n_records < 1) return pfail(WKERN_ERR_INVALID_ARG, "n_records %lld < 1", (long long)n_records);
  if (n_records > 0x7FFFFFFF)
    return pfail(WKERN_ERR_UNSUPPORTED, "n_records %lld above 2^31 - 1", (long long)n_records);
  size_t tmp = 0;
  wkern_status st = sort_storage((int)n_records, nullptr, &tmp);
  if (st != WKERN_OK) return st;
  *bytes = workspace_total((int)n_records, tmp);
  return WKERN_OK;
}

wkern_status wkern_wpartition(const double* w, int64_t n_records, int32_t n_planes,
                              int32_t absolute, int32_t stat, void* workspace,
                              size_t workspace_bytes, int32_t* order, int64_t* plane_start,
                              double* w_plane, void* stream) {
  wkern::set_last_error("");
  wkern_status st =
      check_partition_args(w, n_records, n_planes, absolute, stat, order, plane_start, w_plane);
  if (st != WKERN_OK) return st;
  if (!workspace) return pfail(WKERN_ERR_INVALID_ARG, "NULL argument");
  return partition_into(w, (int)n_records, n_planes, absolute, stat, (char*)workspace,
                        workspace_bytes, order, plane_start, w_plane, (hipStream_t)stream);
}

wkern_status wkern_wpartition_noalloc(const double* w, int64_t n_records, int32_t n_planes,
                                      int32_t absolute, int32_t stat, int32_t* order,
                                      int64_t* plane_start, double* w_plane, void* stream) {
  wkern::set_last_error("");
  wkern_status st =
      check_partition_args(w, n_records, n_planes, absolute, stat, order, plane_start, w_plane);
  if (st != WKERN_OK) return st;
  if (n_records > kStaticMaxRecords)
    return pfail(WKERN_ERR_INVALID_ARG,
                 "n_records %lld above %lld, the most the static scratch holds; use "
                 "wkern_wpartition with a workspace",
                 (long long)n_records, (long long)kStaticMaxRecords);
  void* base = nullptr;
  if ((st = static_scratch(&base)) != WKERN_OK) return st;
  return partition_into(w, (int)n_records, n_planes, absolute, stat, (char*)base,
                        kStaticScratchBytes, order, plane_start, w_plane, (hipStream_t)stream);
}

}  // extern "C"
