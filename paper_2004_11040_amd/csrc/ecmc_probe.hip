// ecmc_probe.hip -- memory microbenchmarks behind include/ecmc_probe.h: the
// dependent-load latency and the random-line gather bandwidth that bound the
// event kernel (latency: Little's law over k chains; bandwidth: line-granular
// bytes per lifting).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ecmc_probe.h"

namespace {

constexpr int LINE_U32 = 16;  // 64-byte line = 16 uint32

__device__ unsigned long long probe_out[4];

template <int SCOPE>
__device__ __forceinline__ uint32_t load_u32(const uint32_t *p) {
  if constexpr (SCOPE == 1)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *(const volatile uint32_t *)p;
}
template <int SCOPE>
__device__ __forceinline__ uint64_t load_u64(const uint64_t *p) {
  if constexpr (SCOPE == 1)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *(const volatile uint64_t *)p;
}

// one thread: `hops` warm-up loads, then `hops` timed dependent loads
template <int SCOPE>
__global__ void k_chase(const uint32_t *lines, uint64_t n_lines, int64_t hops) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t q = 0;
  for (int64_t h = 0; h < hops; ++h) q = load_u32<SCOPE>(lines + q * LINE_U32) % n_lines;
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  for (int64_t h = 0; h < hops; ++h) q = load_u32<SCOPE>(lines + q * LINE_U32) % n_lines;
  const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
  probe_out[0] = t1 - t0;
  probe_out[1] = q;  // keeps the chain live
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {  // SplitMix64 finaliser
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// every load's address depends only on (thread, iteration): independent loads
template <int SCOPE>
__global__ void __launch_bounds__(256) k_gather(const uint64_t *lines, uint64_t n_lines, int loads) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t acc = 0;
  for (int it = 0; it < loads; ++it) {
    const uint64_t q = mix64(tid * 0x9e3779b97f4a7c15ull + (uint64_t)it) % n_lines;
    acc += load_u64<SCOPE>(lines + q * (LINE_U32 / 2));
  }
  if (acc == 0x5bd1e995ull) probe_out[2] = acc;  // practically never taken; keeps the loads
}

}  // namespace

extern "C" int ecmc_probe_chase(const void *lines, int64_t n_lines, int64_t hops, int32_t scope,
                                void *stream, double *ns_per_hop) {
  if (!lines || n_lines < 2 || hops < 1 || hops > (1ll << 26) || (scope != 0 && scope != 1) || !ns_per_hop ||
      ((uintptr_t)lines & 255))
    return -1;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t *p = (const uint32_t *)lines;
  if (scope)
    k_chase<1><<<1, 64, 0, st>>>(p, (uint64_t)n_lines, hops);
  else
    k_chase<0><<<1, 64, 0, st>>>(p, (uint64_t)n_lines, hops);
  if (hipGetLastError() != hipSuccess) return -3;
  unsigned long long out[2] = {0, 0};
  if (hipMemcpyFromSymbolAsync(out, HIP_SYMBOL(probe_out), sizeof(out), 0, hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return -3;
  if (hipStreamSynchronize(st) != hipSuccess) return -3;
  *ns_per_hop = (double)out[0] * 10.0 / (double)hops;  // s_memrealtime runs at 100 MHz
  return 0;
}

extern "C" int ecmc_probe_gather(const void *lines, int64_t n_lines, int32_t blocks, int32_t loads_per_thread,
                                 int32_t scope, void *stream, double *gbs) {
  if (!lines || n_lines < 1 || blocks < 1 || blocks > 65536 || loads_per_thread < 1 ||
      loads_per_thread > 4096 || (scope != 0 && scope != 1) || !gbs || ((uintptr_t)lines & 255))
    return -1;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t *p = (const uint64_t *)lines;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -3;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -3;
  }
  int rc = 0;
  // one untimed launch warms the TLB and caches the way the timed one sees them
  for (int rep = 0; rep < 2 && rc == 0; ++rep) {
    if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = -3;
    if (scope)
      k_gather<1><<<blocks, 256, 0, st>>>(p, (uint64_t)n_lines, loads_per_thread);
    else
      k_gather<0><<<blocks, 256, 0, st>>>(p, (uint64_t)n_lines, loads_per_thread);
    if (hipGetLastError() != hipSuccess) rc = -3;
  }
  if (rc == 0 && hipEventRecord(e1, st) != hipSuccess) rc = -3;
  float ms = 0.f;
  if (rc == 0 && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = -3;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const double bytes = (double)blocks * 256.0 * (double)loads_per_thread * 64.0;
  *gbs = ms > 0.f ? bytes / ((double)ms * 1e-3) / 1e9 : 0.0;
  return 0;
}
