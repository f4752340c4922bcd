/*
 * ecmc_probe.h -- C ABI of two memory microbenchmarks (libecmc_probe.so)
 * that give the event kernel's rooflines on the running GPU.
 *
 * The event kernel of libecmc is a chain of dependent shared-memory round
 * trips per lifting (corridor scan, claim, re-read and commit; Alg. 5 and
 * Sec. 2.2), each a gather of scattered records.  Two bounds follow:
 *  - a latency (Little's law) bound: k chains, each needing about three
 *    dependent round trips per lifting of latency l, make at most k / (3 l)
 *    liftings per second.  ecmc_probe_chase measures l;
 *  - a bandwidth bound: the random-line gather bandwidth over a working set of
 *    the kernel's size, divided by the bytes each lifting touches at cache
 *    line granularity.  ecmc_probe_gather measures that bandwidth.
 * The two litmus tests check the ordering the kernel relies on.
 * The chase and the gather use the same load flavour as the kernel when scope = 1 (relaxed
 * agent-scope atomic loads, which bypass the non-coherent per-XCD L2 and are
 * served from the Infinity Cache or HBM), or plain loads when scope = 0.
 *
 * Conventions: device buffers are the caller's; the library allocates no
 * device memory (results go through a small static device array).  stream is
 * a hipStream_t passed as void*; every call synchronises it.  Return 0 on
 * success, -1 for bad arguments, -3 if a HIP call failed.  Not a method of
 * the paper: measurement only.
 */
#ifndef ECMC_PROBE_H
#define ECMC_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pointer chase with one thread over a DEVICE buffer of n_lines 64-byte lines
 * (bytes = 64 * n_lines, 256-byte aligned) whose line q holds, in its first
 * 4 bytes (uint32), the index of the next line; the caller writes a random
 * cyclic permutation there.  Indices are taken modulo n_lines, so any
 * content is safe.  Runs `hops` dependent loads starting at line 0 (after
 * `hops` warm-up loads) and writes the mean latency per load in ns (device
 * clock, 100 MHz) to *ns_per_hop.  n_lines >= 2, 1 <= hops <= 2^26. */
int ecmc_probe_chase(const void *lines, int64_t n_lines, int64_t hops, int32_t scope,
                     void *stream, double *ns_per_hop);

/* Random-line gather: blocks x 256 threads, each issuing loads_per_thread
 * independent 8-byte loads at pseudo-random line-aligned offsets (a hash of
 * thread and iteration) of a DEVICE buffer of n_lines 64-byte lines.  Writes
 * the line-granular bandwidth, loads x 64 B / duration (HIP events), in GB/s
 * to *gbs.  n_lines >= 1, 1 <= blocks <= 65536, 1 <= loads_per_thread <= 4096. */
int ecmc_probe_gather(const void *lines, int64_t n_lines, int32_t blocks, int32_t loads_per_thread,
                      int32_t scope, void *stream, double *gbs);

/* Message-passing litmus test across workgroups (and so across XCDs, which
 * take workgroups in turn), with the event kernel's ordering discipline:
 * relaxed agent-scope atomic stores and loads, ordered by completion waits.
 * Workgroup 2q (64 threads) writes, workgroup 2q + 1 reads: for iteration it
 * of lane l the writer stores data then (after a wait if waits != 0) flag;
 * the reader loads flag up to `spin` times until it sees the value, then
 * loads data.  *seen counts iterations whose flag the reader saw, *stale those
 * among them whose data was not yet visible (a reordering).  data and flag:
 * DEVICE arrays of pairs x 64 x iters uint32, zero on entry.  Every loop is
 * bounded.  1 <= pairs <= 4096, 1 <= iters <= 4096, 1 <= spin <= 4096. */
int ecmc_probe_litmus_mp(void *data, void *flag, int32_t pairs, int32_t iters, int32_t spin, int32_t waits,
                         void *stream, int64_t *seen, int64_t *stale);

/* Compare-and-swap exclusivity litmus test, the claim of the event kernel:
 * blocks x 256 threads each make `rounds` attempts to increment one of `locs`
 * counters under its lock word (CAS 0 -> thread id, wait, load the counter,
 * store it plus one, wait, store 0), with at most `tries` CAS tries per
 * round.  *acquired counts the increments made; with exclusive locks and
 * ordered hand-overs the counters sum to it (the caller checks).  tag and
 * counter: DEVICE arrays of locs uint32, zero on entry.  Every loop is
 * bounded.  1 <= locs <= 2^20, 1 <= blocks <= 4096, 1 <= rounds, tries <= 4096. */
int ecmc_probe_litmus_cas(void *tag, void *counter, int32_t locs, int32_t blocks, int32_t rounds, int32_t tries,
                          void *stream, int64_t *acquired);

#ifdef __cplusplus
}
#endif
#endif /* ECMC_PROBE_H */
