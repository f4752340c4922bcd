/*
 * ecmc.h -- C ABI of the MI355X (gfx950) library for multithreaded
 * event-chain Monte Carlo of hard disks with local times.
 *
 * Method: Li, Todo, Maggs, Krauth, "Multithreaded event-chain Monte Carlo with
 * local times".  Between two breakpoints h and h' (a "leg"), k active disks
 * ("chains") move with one common velocity v (+x, +y, -x or -y).  Each chain advances
 * on its own local time: it finds the next disk it would hit (time of flight
 * tau_ij = forward distance - b_ij, b_ij = sqrt((2 sigma)^2 - dp^2), Sec. 2.2),
 * checks the horizon condition t_i + tau_ij > t_j (Eq. 2) on the nearest disk
 * of each of its three lanes (Sec. 3.1, the out-arrows of the constraint graph
 * G(3)), claims the target with a compare-and-swap on its tag (Alg. 5),
 * re-checks the target's position and local time, and lifts (Eq. 1).  A horizon violation stops
 * every chain; the liftings at or after the earliest time that is not settled
 * (min of the violation times and of the chains' pending event times) are
 * taken back from per-chain undo records and the leg resumes from there
 * (restart strategy 2, Sec. 3.4).  If the same race keeps recurring, a short
 * stretch runs with a tiny bounded lag (chains then commit in global-time
 * order up to near-ties), and as a last resort in global-time order (Alg. 2),
 * which cannot violate.  Without
 * violations the liftings equal those of Alg. 2 (Lemma 2); every path
 * evaluates each lifting from the chain's activation state with the same
 * binary64 operations, so results are bit-identical to global-time order.
 *
 * Conventions
 *  - Every function returns ECMC_OK (0) or a negative ECMC_E* code, except
 *    ecmc_workspace_bytes (bytes, or a negative code), ecmc_last_error and
 *    ecmc_free.  No function aborts the process.
 *  - sigma is the disk RADIUS; disks touch at centre distance d = 2 sigma.
 *  - The box is the periodic square [0, box)^2.
 *  - Device memory is owned by the caller: the library never allocates device
 *    memory.  ecmc_workspace_bytes() tells how much one context needs; the
 *    caller passes a device buffer of at least that size to ecmc_init() and
 *    keeps it alive until ecmc_free().
 *  - "stream" is a hipStream_t passed as void*; every kernel of a context runs
 *    on it.  Calls that return data to the host synchronise that stream.
 *  - Host pointers are read or written during the call only; the caller keeps
 *    ownership.
 *  - A context is not thread safe; use one context per host thread.
 */
#ifndef ECMC_H
#define ECMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define ECMC_OK 0
#define ECMC_EINVAL (-1)   /* bad argument or unsupported parameter set       */
#define ECMC_EOVERLAP (-2) /* input disks overlap (closer than 2 sigma)       */
#define ECMC_EDEVICE (-3)  /* a HIP runtime call failed                        */
#define ECMC_ECELL (-4)    /* more disks in one cell than its 4 slots          */
#define ECMC_EHANG (-5)    /* an event chain exceeded its iteration limit      */
#define ECMC_ESTATE (-6)   /* call order violated (e.g. run before set_active) */

/* ---- flags for ecmc_init ------------------------------------------------ */
#define ECMC_FP64 0u        /* collision search in binary64                    */
#define ECMC_FP32_MIXED 1u  /* collision search in binary32 on cell-relative
                               coordinates, winners and near-ties recomputed in
                               binary64; positions, local times and sums stay
                               binary64 (results identical to ECMC_FP64).  It
                               filters the corridor scan (ECMC_NEIGHBOURS_CELLS);
                               graph candidates are three binary64 times of
                               flight per scan in either form             */

/* ---- options for ecmc_set_option --------------------------------------- */
#define ECMC_OPT_LANES 1          /* lanes per chain: 16, 32 or 64 (default 64) */
#define ECMC_OPT_WAIT_RETRIES 2   /* failed claims on an active target before the
                                     chain moves up to contact (default 64)     */
#define ECMC_OPT_MAX_SPLITS 3     /* consecutive rollbacks that do not move
                                     past the earliest unsettled time before a
                                     short stretch runs with a tiny bounded lag
                                     (default 1; in a batch, before a
                                     global-order stretch, also default 1)      */
#define ECMC_OPT_FORCE_GLOBAL 4   /* 1: run every leg in global-time order      */
#define ECMC_OPT_INJECT_CHAIN 5   /* test hook: chain that reports a horizon    */
#define ECMC_OPT_INJECT_EVENT 6   /*   violation at its given event of the next
                                     leg attempt (-1 disables; host-forced, the
                                     kernel still exits normally)              */
#define ECMC_OPT_KERNEL_TIMING 7  /* 1: time every event-kernel launch with HIP
                                     events recorded on the context's stream
                                     (statistics event_kernel_ms / launches)    */
#define ECMC_OPT_STRICT_ORDER 8   /* 1: add agent-scope acquire/release fences to
                                     the completion waits that order the shared
                                     fields (validation mode; slower)           */
#define ECMC_OPT_WINDOW_MICRO 9   /* bounded lag, in units of 1e-6 sigma: a chain
                                     commits an event only if its time is within
                                     this of the smallest next-event time over
                                     all chains (0: chains run freely).  Pure
                                     scheduling: results do not depend on it.   */
#define ECMC_OPT_FEATURES 10      /* bit set of the ECMC_FEAT_* refinements of the
                                     horizon protocol that are switched on
                                     (contexts: ECMC_FEAT_DEFAULT; batches:
                                     ECMC_FEAT_ALL); each only avoids needless
                                     rollbacks                                  */

/* ---- refinements of the horizon protocol (ECMC_OPT_FEATURES) ------------ */
#define ECMC_FEAT_SCREEN 1u   /* a lane minimum that fails Eq. 2 but is active on
                                 a chain whose activation record shows it at
                                 rest until after the lifting is not a violation */
#define ECMC_FEAT_RESERVE 2u  /* chains reserve their target; a claim for a
                                 later lifting gives the target back           */
#define ECMC_FEAT_REREAD 4u   /* a failure of Eq. 2 is confirmed on a record read
                                 again after a pause (a disk being stopped shows
                                 its new time with its old position for a moment) */
#define ECMC_FEAT_FRESH 8u    /* after a claim, lane minima whose records changed
                                 are checked on the new records (else the new
                                 local time with the scanned position)         */
#define ECMC_FEAT_UNRESERVE 16u /* with RESERVE: a chain takes its reservation
                                 back when it changes target or time, and when
                                 it leaves the attempt                        */
#define ECMC_FEAT_ALL 31u
#define ECMC_FEAT_DEFAULT 30u /* all but SCREEN: at N = 2^20 screening cleared a
                                 few violations per 20 legs, for five stores
                                 per lifting of the activation record that it
                                 reads (about 200 B of HBM writes per lifting)
                                 at no measurable gain in throughput          */
#define ECMC_OPT_GRAPH 11         /* batches: 1 captures the persistent launch
                                     in a hipGraph once and replays it (every
                                     setting travels in the replica descriptors
                                     uploaded before each replay; default 0)    */
#define ECMC_OPT_NEIGHBOURS 13    /* where a chain finds its candidates (contexts
                                     and batches): ECMC_NEIGHBOURS_GRAPH (the
                                     three arrows of the constraint graph G(3),
                                     built at every breakpoint, Sec. 3.1;
                                     default) or ECMC_NEIGHBOURS_CELLS (the
                                     corridor scan over home cells, where the
                                     FP32-mixed form filters in binary32).
                                     Same results.                              */
#define ECMC_NEIGHBOURS_CELLS 0
#define ECMC_NEIGHBOURS_GRAPH 1
#define ECMC_OPT_COOPERATIVE 14   /* contexts: chains wait on each other and
                                     on a clock workgroup, so all workgroups of
                                     an event launch must be resident at once.
                                     0 (default): plain launch; each workgroup
                                     counts itself in when it starts, and a
                                     chain that has waited 1 ms checks the
                                     count: if part of the grid has not started,
                                     the attempt is taken back and run again and
                                     the context switches to 1 for good.
                                     1: cooperative launch, the runtime
                                     guarantees co-residency                    */
#define ECMC_OPT_TEST_NONRESIDENT 15 /* test hook (contexts): a plain launch
                                     expects this many workgroups beyond its
                                     grid (0..4; default 0) and checks at the
                                     first wait, so the fallback runs           */
#define ECMC_OPT_CLOCK_PERIOD_NS 16 /* least time between two recomputations
                                     of H, in ns (0..100000; 0: as often as
                                     possible).  Contexts: a pass of the clock
                                     workgroup that ends early waits before it
                                     loads the next-event times again.
                                     Batches: a replica's waiting chains
                                     recompute H at most once per period (the
                                     one whose compare-and-swap on a time stamp
                                     succeeds).  Pure scheduling: results do
                                     not depend on it.                          */
#define ECMC_OPT_CELL_PCT 12      /* batches: home-cell width in percent of 2 sigma,
                                     100..141 (cells of at most 4 disks), used
                                     where admissible for a replica (else its
                                     own cells); 0: autotune (default)          */

typedef struct ecmc_ctx ecmc_ctx;

typedef struct {
  int64_t events;          /* committed liftings (elements of L)              */
  int64_t legs;            /* legs completed                                  */
  int64_t legs_violated;   /* legs in which a horizon violation was seen      */
  int64_t attempts;        /* event-kernel launches                           */
  int64_t reruns;          /* rollbacks to the earliest unsettled time        */
  int64_t global_legs;     /* legs or stretches run in global-time order       */
  int64_t cas_fail;        /* lock-less lock re-checks that failed            */
  int64_t active_waits;    /* claims that found the target active             */
  int64_t contact_moves;   /* moves up to contact with an active target       */
  int64_t fp32_refines;    /* binary64 recomputations of near-tie candidates  */
  int64_t slots_scanned;   /* cell slots examined by the corridor scans        */
  int64_t overlaps;        /* pairs closer than 2 sigma - 4 ulp(box), last check */
  double sum_b;            /* sum of b_ij over liftings (per chain, then chains) */
  double chain_time;       /* total chain time, k * (sum of leg lengths)       */
  double pressure;         /* 1 + sum_b / chain_time (raw ECMC estimator)      */
  double device_ms;        /* device time spent in ecmc_run (HIP events)       */
  double event_kernel_ms;  /* summed duration of timed event-kernel launches   */
  int64_t event_launches;  /* number of timed event-kernel launches            */
  int64_t timed_events;    /* liftings committed inside the timed launches     */
  int64_t timed_slots;     /* cell slots scanned inside the timed launches     */
  int64_t violations_by_kind[4]; /* horizon violations seen: [0] in the scan,
                                  [1] re-checked after a claim, [2] target at a
                                  breakpoint (stalled or paused), [3] before a
                                  move up to contact                           */
  int32_t last_violation_kind;   /* first violation of the last violating attempt */
  int32_t last_violation_chain;  /*   chain that saw it                           */
  int32_t last_violation_disk;   /*   disk whose local time was too late          */
  int32_t pad_;
  double last_violation_t;       /*   the chain's local time                     */
  double last_violation_tj;      /*   that disk's local time                     */
  double last_violation_tau;     /*   time of flight to that disk                */
  double last_violation_h;       /*   start of the attempt                       */
  int64_t lockstep_runs;         /* stall-breaking stretches with a tiny lag      */
  int64_t violations_screened;   /* failed Eq. 2 checks on a lane minimum that the
                                    activation record of its chain showed harmless */
  int64_t claim_yields;          /* claims given back to an earlier reservation */
  int64_t spin_aborts;           /* attempts a chain aborted after 32768 rounds of
                                    scan and claim without a lifting (the race goes
                                    to the rollback; last_violation_kind 4, and
                                    last_violation_disk then names the retry path:
                                    1 rescan, 2 yield wait, 3 contact check,
                                    4 active target, 5 changed records, 6 yield) */
  int64_t nonresident_launches;  /* plain event launches whose co-residency
                                    handshake timed out (taken back, rerun)   */
  int64_t cooperative;           /* 1 once event launches are cooperative      */
  int64_t clock_iters;           /* passes of the clock workgroup's loop over the
                                    timed event launches (the clock's period is
                                    event_kernel_ms / clock_iters)             */
  int64_t overflow_legs;         /* legs replayed whole in global-time order because
                                    a chain committed more liftings after the last
                                    settled time than its undo records hold (also
                                    counted in global_legs)                    */
} ecmc_stats_t;

/* Bytes of device workspace for a context (the storage of the lifted
 * configuration {C, A} of Sec. 2.1 with the per-leg home cells, local times
 * and tags of Sec. 2.2-2.3).  n disks of radius sigma in a box of
 * side box; cells per side (0: floor(box / (2 sigma)) reduced until the cell is
 * at least 2 sigma wide); max_chains >= the k later passed to ecmc_set_active;
 * log_cap = number of target ids kept per chain (a ring: the last log_cap
 * liftings of each chain).  Negative ECMC_EINVAL for invalid sizes. */
int64_t ecmc_workspace_bytes(int64_t n, double sigma, double box, int32_t cells,
                             int32_t max_chains, int64_t log_cap,
                             uint32_t flags);

/* Create a context (Sec. 2.1, Alg. 1 input C_h).
 * positions_xy: DEVICE pointer, n x 2 doubles, row-major (x0,y0,x1,y1,...),
 *   every coordinate in [0, box).  Copied; the caller may reuse it afterwards.
 * cells: 0 or cells per side with 2 sigma <= box/cells <= 2 sqrt(2) sigma and
 *   cells >= 5 (each cell then holds at most 4 disks).
 * workspace: DEVICE buffer of ws_bytes >= ecmc_workspace_bytes(...), 256-byte
 *   aligned.  stream: hipStream_t.
 * Errors: ECMC_EINVAL (n < 2, sigma <= 0, box <= 0, bad cells, workspace too
 * small or misaligned, coordinates outside [0, box)), ECMC_EOVERLAP (a pair
 * closer than 2 sigma - 4 ulp(box)), ECMC_ECELL, ECMC_EDEVICE.  On error *out
 * is NULL. */
int ecmc_init(ecmc_ctx **out, const double *positions_xy, int64_t n,
              double sigma, double box, int32_t cells, uint32_t flags,
              void *workspace, int64_t ws_bytes, int32_t max_chains,
              int64_t log_cap, void *stream);

/* Active set A_h: chain c moves disk idx[c] (HOST array of k distinct indices
 * in [0, n)).  The active set then evolves with the liftings and persists
 * across legs and runs (Remark on stalled spheres).  Resets the chain logs and
 * per-chain sums.  Errors: ECMC_EINVAL (k < 1, k > max_chains, duplicates,
 * index out of range). */
int ecmc_set_active(ecmc_ctx *ctx, const int32_t *idx, int32_t k);

/* Run chain_time / breakpoint_interval legs (that ratio must be an integer
 * within 1e-9) of length T = breakpoint_interval each.  A leg is the interval
 * between two breakpoints h and h' = h + T: the multithreaded local-time
 * algorithm (Alg. 5 / Alg. 6, Sec. 2.3-2.4) takes the lifted configuration
 * {C_h, A_h} to {C_h', A_h'} and adds the leg's liftings to L; without a
 * horizon violation this is the output of global-time ECMC, Alg. 2 (Lemma 2,
 * Lemma 3), and violations are undone by restarts (Sec. 3.4).
 * direction: 0 +x, 1 +y, 2 -x, 3 -y, 4 alternate +x/+y (the first leg of the
 * context is +x, and the alternation continues across calls).  -x and -y run
 * the leg on the reflected coordinate L - x (or L - y), so a leg followed by
 * the opposite leg of the same length returns the configuration (Remark on
 * time-reversal invariance) up to the rounding of the reflection, a few ulps
 * of the box.
 * n_chains must equal the k given to ecmc_set_active.  T must satisfy
 * 0 <= T <= box - 4 (box/cells) - 2 sigma.  Horizon violations are absorbed by
 * rollbacks and counted in the statistics.  Synchronises the stream once per
 * event-kernel launch (to read the violation flag).  Errors: ECMC_EINVAL, ECMC_ESTATE,
 * ECMC_ECELL, ECMC_EHANG, ECMC_EDEVICE. */
int ecmc_run(ecmc_ctx *ctx, int32_t n_chains, double chain_time,
             double breakpoint_interval, int32_t direction);

/* n_legs legs of length T = breakpoint_interval, leg l along directions[l]
 * (HOST array of n_legs int32: 0 +x, 1 +y, 2 -x, 3 -y).  A production loop
 * changes v between breakpoints (Sec. 2.1: v is fixed within a leg; the
 * constraint graph is rebuilt for each new v, Sec. 3.1 and the closing
 * paragraph of Sec. 3.4 on production codes); the caller draws the
 * directions, so the random numbers of the loop are inputs.  Everything else
 * as ecmc_run with chain_time = n_legs T.  Errors: ECMC_EINVAL (n_legs < 0,
 * directions NULL or T = 0 with n_legs > 0, a direction outside 0..3, and
 * the checks of ecmc_run), ECMC_ESTATE, ECMC_ECELL, ECMC_EHANG,
 * ECMC_EDEVICE. */
int ecmc_run_directions(ecmc_ctx *ctx, int32_t n_chains, double breakpoint_interval, int64_t n_legs,
                        const int32_t *directions);

/* Statistics accumulated since ecmc_set_active.  events counts elements of
 * the lifting set L (Alg. 1 output); sum_b and pressure are the ECMC pressure
 * estimator, beta P / rho = 1 + sum of b_ij over liftings / chain time (the
 * lifting distance b_ij of Sec. 2.2 summed per chain in lifting order, then
 * over chains); the other counters describe the horizon protocol (Eq. 2,
 * Alg. 5) and its restarts (Sec. 3.4).  Synchronises the stream. */
int ecmc_stats(ecmc_ctx *ctx, ecmc_stats_t *out);

/* Copy the current configuration C (Sec. 2.1) to HOST memory: out_xy n x 2
 * doubles, row-major (x0,y0,x1,y1,...).  Synchronises the stream. */
int ecmc_get_positions(ecmc_ctx *ctx, double *out_xy);

/* Local times t_i at the end of the last leg (HOST, n doubles, relative to
 * the leg's breakpoint h; Remark on the meaning of local times: the last time
 * disk i was active, h' for the stalled active disks, Remark on stalled
 * spheres).  Synchronises the stream. */
int ecmc_get_stamps(ecmc_ctx *ctx, double *out);

/* Current active set A (Sec. 2.1; HOST, k int32: disk of chain c).
 * Synchronises the stream. */
int ecmc_get_active(ecmc_ctx *ctx, int32_t *out);

/* Per-chain results since ecmc_set_active (HOST, k entries each; either may
 * be NULL): sum of the lifting distances b_ij (Sec. 2.2) in the chain's
 * lifting order, and its number of liftings.  Synchronises the stream. */
int ecmc_get_chain_sums(ecmc_ctx *ctx, double *sum_b, int64_t *events);

/* Lifting log of one chain: the target disk ids j of its liftings i -> j,
 * in order (the chain's part of the lifting set L output by Alg. 1 and
 * Alg. 2; consecutive entries are the disks the chain moved).
 * Writes min(count, log_cap, cap) most recent entries to the HOST array
 * targets and the chain's total lifting count to *n_out.  ECMC_EINVAL if
 * chain is out of range or cap < min(count, log_cap). */
int ecmc_get_log(ecmc_ctx *ctx, int32_t chain, int32_t *targets, int64_t cap,
                 int64_t *n_out);

/* Count pairs closer than 2 sigma - 4 ulp(box) in the current configuration
 * (binary64, minimum image; zero tolerance beyond rounding of contact
 * positions).  Hard disks may not overlap (Sec. 1, the hard-disk model; a
 * valid run keeps every pair at distance >= 2 sigma, Eq. 1 moves a disk up
 * to contact only).  Writes the count to *count and into the statistics.
 * Synchronises the stream. */
int ecmc_overlaps(ecmc_ctx *ctx, int64_t *count);

/* The count of ecmc_overlaps for callers that cannot allocate device memory
 * (code under graph capture, serving loops, harnesses that forbid it): no
 * context and no workspace.  positions_xy: DEVICE pointer, n x 2 doubles,
 * row-major, every coordinate in [0, box).  The cell list and the counters
 * live in one static device array per GPU of 28.8 MB (cells of at least
 * 2 sigma, at most 1200 per side: box up to about 2400 sigma), held by each
 * GPU the library runs on until the process ends; the call allocates
 * nothing, clears what it uses, and synchronises `stream`.  Calls that
 * overlap in time on one GPU share that array and race.  Errors: ECMC_EINVAL
 * (n < 1, sigma <= 0, box <= 0, fewer than 3 or more than 1200 cells per
 * side, a coordinate outside [0, box)), ECMC_EOVERLAP (five centres in one
 * cell: disks overlap, count not given), ECMC_EDEVICE. */
int ecmc_overlaps_noalloc(const double *positions_xy, int64_t n, double sigma, double box,
                          int64_t *count, void *stream);

/* Constraint graph G(3) of the current configuration for velocity
 * `direction` (0 +x, 1 +y, 2 -x, 3 -y) (Sec. 3.1): for every disk i the disk
 * with the smallest (time of flight, id) in each lane of its corridor,
 * |dp| < sigma, sigma <= dp < 2 sigma and -2 sigma < dp <= -sigma, keeping
 * only arrows with a time of flight below `horizon` (a leg of that length
 * cannot reach further; 0 < horizon <= box - 4 cell - 2 sigma).  Writes
 * arrows[3 i + q] = target disk id, or -1 for an empty lane (HOST array of
 * 3 n int32).  Disks closer than 2 sigma across v cannot pass each other,
 * so the arrows hold for a whole leg; they are the candidates the event
 * kernel uses with ECMC_NEIGHBOURS_GRAPH.  Rebuilds the home cells (call
 * between runs).  Synchronises the stream.  Errors: ECMC_EINVAL, ECMC_ECELL,
 * ECMC_EDEVICE. */
int ecmc_graph(ecmc_ctx *ctx, int32_t direction, double horizon, int32_t *arrows);

/* Tuning and test options (ECMC_OPT_*): scheduling of the horizon protocol
 * (Alg. 5), the necklace retries (Remark on active-sphere necklaces), the
 * restart ladder (Sec. 3.4) and test hooks.  None changes results.
 * ECMC_EINVAL for unknown keys or values. */
int ecmc_set_option(ecmc_ctx *ctx, int32_t key, int64_t value);

/* Static description of the last error on this context (never NULL; the
 * caller must not free it).  Bookkeeping of the C ABI, no paper passage. */
const char *ecmc_last_error(const ecmc_ctx *ctx);

/* Release the context (host memory only; the workspace stays the caller's).
 * Accepts NULL.  Bookkeeping of the C ABI, no paper passage. */
void ecmc_free(ecmc_ctx *ctx);

/* ---- batched replicas -----------------------------------------------------
 * Many independent systems ("replicas"), each the problem of Sec. 2.1 (one
 * lifted configuration advanced leg by leg between breakpoints; running many
 * of them at once is a systems pattern, not part of the paper), each a
 * context set up as usual
 * (ecmc_init, ecmc_set_active), run together in ONE persistent launch: a
 * workgroup claims a replica and runs its next two legs, largest expected
 * remaining time first (a replica moves between workgroups from turn to
 * turn, one at a time), with the breakpoint synchronisation, rollbacks (Sec. 3.4, strategy 2) and the
 * global-order fallback (Alg. 2) done on the device; its chains share the
 * workgroup's compute unit.  Results are read per replica with the
 * per-context calls
 * (ecmc_stats, ecmc_get_positions, ecmc_get_log, ...), and are identical to
 * running each context with ecmc_run and no bounded lag.
 * Requirements: all contexts on one stream, all FP64 or all FP32-mixed,
 * at most 128 chains per replica (4 lanes x 128 = 512 threads).  The chains
 * of a replica share one workgroup, so its shared fields use workgroup-scope
 * atomics. */
typedef struct ecmc_batch ecmc_batch;

typedef struct {
  int32_t lanes;        /* cap on the lanes per chain of the last run: each
                           replica of k chains runs the largest of 4, 8, 16,
                           32 lanes up to the cap with k * lanes <= 512     */
  int32_t graph;        /* 1 if the last run replayed a captured hipGraph   */
  int32_t workgroups;   /* persistent grid of the last launch             */
  int32_t cell_pct;     /* home-cell width of the last run, % of 2 sigma    */
  double device_ms;     /* duration of the last run's main launch (HIP events) */
  int64_t events;       /* liftings committed by the main launch, all replicas */
  int64_t legs;         /* legs run by the last call, all replicas         */
  int64_t rollbacks;    /* rollbacks in the last call, all replicas        */
  int64_t global_runs;  /* global-order stretches in the last call         */
  double tune_events_per_ms[4]; /* autotuner: liftings per replica-ms (per ms
                                   of summed replica device time) in one leg
                                   with a lane cap of 4, 8, 16, 32 (0: not
                                   tried, or the same lanes for every replica
                                   as a smaller cap); a larger cap is chosen
                                   only if 3 % faster than the best smaller
                                   one                                     */
  double tune_cell_events_per_ms[4]; /* autotuner: liftings per replica-ms with cells
                                   of 100, 115, 130, 141 % of 2 sigma at the
                                   chosen cap (0: not tried or no change)  */
  int32_t tune_from_cache;  /* 1 if the last run took its settings from the
                               autotuner cache                            */
  int32_t pad2_;
  double replica_ms_max;  /* longest device time of one replica in the main launch */
  double replica_ms_sum;  /* summed over replicas: with device_ms and workgroups
                             this gives the launch's load balance        */
} ecmc_batch_info_t;

/* Bytes of device scratch for a batch of n_ctx contexts (each replica's
 * descriptor, and its results with the state by which replicas are handed
 * out; bookkeeping of the batch, no paper passage).  Negative ECMC_EINVAL for n_ctx outside
 * [1, 2^20]. */
int64_t ecmc_batch_scratch_bytes(int32_t n_ctx);

/* Group n_ctx distinct contexts (HOST array of handles; the contexts must
 * outlive the batch) with a DEVICE scratch buffer of at least
 * ecmc_batch_scratch_bytes(n_ctx) bytes, 256-byte aligned, owned by the
 * caller.  Each context stays one system of Sec. 2.1; the grouping is
 * bookkeeping of the batch, no paper passage.  Errors: ECMC_EINVAL (sizes,
 * duplicates, mixed streams or forms), ECMC_ESTATE (a context without an
 * active set). */
int ecmc_batch_create(ecmc_batch **out, ecmc_ctx *const *ctxs, int32_t n_ctx,
                      void *scratch, int64_t scratch_bytes);

/* ECMC_OPT_LANES (cap on the lanes per chain: 4, 8, 16, 32; 0: autotune at
 * the first run), ECMC_OPT_CELL_PCT (0: autotune), ECMC_OPT_GRAPH,
 * ECMC_OPT_FEATURES, ECMC_OPT_WAIT_RETRIES, ECMC_OPT_MAX_SPLITS and
 * ECMC_OPT_WINDOW_MICRO (bounded lag between a replica's chains in units of
 * 1e-6 sigma, 0 = free; a chain waiting at the lag takes the replica's H from
 * its chains' next-event times itself), ECMC_OPT_CLOCK_PERIOD_NS (least
 * time between two such recomputations in a replica).  Scheduling and layout of Alg. 5 on
 * the device; results do not depend on them.  Options take effect at the
 * next ecmc_batch_run, also when a captured graph is replayed. */
int ecmc_batch_set_option(ecmc_batch *b, int32_t key, int64_t value);

/* Autotuner cache (host file, JSON, one entry per line): with a path set, a
 * run that has to autotune first looks up this batch's signature (device,
 * form, every replica's size, chains, box, cells and leg length, and the run
 * settings) and uses the stored lane cap and cell width if found; otherwise
 * it tunes and stores its choice.  NULL or "" switches the cache off.  The
 * file is rewritten through a temporary file; concurrent writers are not
 * coordinated.  Bookkeeping of the runtime, no paper passage. */
int ecmc_batch_tune_cache(ecmc_batch *b, const char *path);

/* Run every replica r with legs of length leg_T[r] (HOST arrays of n_ctx)
 * until its committed liftings reach target_events[r], or for at most
 * max_legs legs in this call (0: no limit).  direction as for ecmc_run,
 * continuing each context's alternation.  With lanes or cells on autotune
 * (and no cache entry), the autotuner first runs one leg per replica with
 * each lane cap that changes some replica's lanes, then with each cell width
 * that changes some replica's cells (those legs count), and keeps the
 * fastest.  Each replica runs the legs of ecmc_run: Alg. 5 between
 * breakpoints with restart strategy 2 (Sec. 3.4), on its own.  Synchronises
 * the stream.  Errors: ECMC_EINVAL, ECMC_ECELL, ECMC_EHANG, ECMC_EDEVICE. */
int ecmc_batch_run(ecmc_batch *b, const int64_t *target_events,
                   const double *leg_T, int32_t direction, int32_t max_legs);

/* Details of the last ecmc_batch_run (liftings as for ecmc_stats, restarts
 * of Sec. 3.4, global-order stretches of Alg. 2, and the autotuner's rates). */
int ecmc_batch_info(const ecmc_batch *b, ecmc_batch_info_t *out);

/* Static description of the last error of the batch (never NULL; bookkeeping
 * of the C ABI, no paper passage). */
const char *ecmc_batch_last_error(const ecmc_batch *b);

/* Release the batch (host memory and the captured graph).  Accepts NULL.
 * Bookkeeping of the C ABI, no paper passage. */
void ecmc_batch_free(ecmc_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* ECMC_H */
