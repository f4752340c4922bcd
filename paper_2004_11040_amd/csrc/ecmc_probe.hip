// ecmc_probe.hip -- memory microbenchmarks behind include/ecmc_probe.h: the
// dependent-load latency and the random-line gather bandwidth that bound the
// event kernel (latency: Little's law over k chains; bandwidth: line-granular
// bytes per lifting), and two litmus tests of the ordering discipline the
// kernel relies on.
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

// ---- litmus tests: the event kernel's discipline (relaxed agent-scope
// atomics, order between locations from completion waits)
__device__ __forceinline__ void lit_st(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t lit_ld(uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lit_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

template <bool WAIT>
__global__ void __launch_bounds__(64) k_litmus_mp(uint32_t *data, uint32_t *flag, int iters, int spin) {
  const int pair = blockIdx.x >> 1, role = blockIdx.x & 1;
  const int64_t base = ((int64_t)pair * 64 + threadIdx.x) * iters;
  unsigned long long seen = 0, stale = 0;
  for (int it = 0; it < iters; ++it) {
    const int64_t k = base + it;
    const uint32_t v = (uint32_t)it + 1u;
    if (role == 0) {
      lit_st(&data[k], v);
      if (WAIT) lit_wait();
      lit_st(&flag[k], v);
    } else {
      uint32_t f = 0;
      for (int s = 0; s < spin && f != v; ++s) f = lit_ld(&flag[k]);
      if (f == v) {
        ++seen;
        if (lit_ld(&data[k]) != v) ++stale;
      }
    }
  }
  if (role == 1) {
    atomicAdd(&probe_out[0], seen);
    atomicAdd(&probe_out[1], stale);
  }
}

__global__ void __launch_bounds__(256) k_litmus_cas(uint32_t *tag, uint32_t *counter, int locs, int rounds,
                                                    int tries) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t me = (uint32_t)tid + 1u;
  unsigned long long got = 0;
  for (int r = 0; r < rounds; ++r) {
    const int l = (int)(mix64(tid * 0x9e3779b97f4a7c15ull + (uint64_t)r) % (uint64_t)locs);
    bool done = false;
    for (int t = 0; t < tries && !done; ++t) {
      uint32_t old = 0u;
      if (__hip_atomic_compare_exchange_strong(&tag[l], &old, me, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        lit_wait();  // the claim completes before the reads that depend on it
        const uint32_t v = lit_ld(&counter[l]);
        lit_st(&counter[l], v + 1u);
        lit_wait();  // the data store completes before the release
        lit_st(&tag[l], 0u);
        done = true;
      }
    }
    if (done) ++got;
  }
  atomicAdd(&probe_out[2], got);
}

}  // namespace

extern "C" int ecmc_probe_litmus_mp(void *data, void *flag, int32_t pairs, int32_t iters, int32_t spin,
                                    int32_t waits, void *stream, int64_t *seen, int64_t *stale) {
  if (!data || !flag || pairs < 1 || pairs > 4096 || iters < 1 || iters > 4096 || spin < 1 || spin > 4096 ||
      !seen || !stale)
    return -1;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long zero[3] = {0, 0, 0};
  if (hipMemcpyToSymbolAsync(HIP_SYMBOL(probe_out), zero, sizeof(zero), 0, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return -3;
  if (waits)
    k_litmus_mp<true><<<2 * pairs, 64, 0, st>>>((uint32_t *)data, (uint32_t *)flag, iters, spin);
  else
    k_litmus_mp<false><<<2 * pairs, 64, 0, st>>>((uint32_t *)data, (uint32_t *)flag, iters, spin);
  if (hipGetLastError() != hipSuccess) return -3;
  unsigned long long out[3] = {0, 0, 0};
  if (hipMemcpyFromSymbolAsync(out, HIP_SYMBOL(probe_out), sizeof(out), 0, hipMemcpyDeviceToHost, st) != hipSuccess)
    return -3;
  if (hipStreamSynchronize(st) != hipSuccess) return -3;
  *seen = (int64_t)out[0];
  *stale = (int64_t)out[1];
  return 0;
}

extern "C" int ecmc_probe_litmus_cas(void *tag, void *counter, int32_t locs, int32_t blocks, int32_t rounds,
                                     int32_t tries, void *stream, int64_t *acquired) {
  if (!tag || !counter || locs < 1 || locs > (1 << 20) || blocks < 1 || blocks > 4096 || rounds < 1 ||
      rounds > 4096 || tries < 1 || tries > 4096 || !acquired)
    return -1;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long zero[3] = {0, 0, 0};
  if (hipMemcpyToSymbolAsync(HIP_SYMBOL(probe_out), zero, sizeof(zero), 0, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return -3;
  k_litmus_cas<<<blocks, 256, 0, st>>>((uint32_t *)tag, (uint32_t *)counter, locs, rounds, tries);
  if (hipGetLastError() != hipSuccess) return -3;
  unsigned long long out[3] = {0, 0, 0};
  if (hipMemcpyFromSymbolAsync(out, HIP_SYMBOL(probe_out), sizeof(out), 0, hipMemcpyDeviceToHost, st) != hipSuccess)
    return -3;
  if (hipStreamSynchronize(st) != hipSuccess) return -3;
  *acquired = (int64_t)out[2];
  return 0;
}

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
