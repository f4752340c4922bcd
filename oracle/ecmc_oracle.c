/*
 * ecmc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, double-precision reference for event-chain Monte Carlo (ECMC)
 * of hard disks between two breakpoints, with k active disks ("chains") that
 * share one velocity, in the global-time form of the paper
 * (Li, Todo, Maggs, Krauth, "Multithreaded event-chain Monte Carlo with local
 * times", Sec. 2.1, Algorithms 1 and 2).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's library.  It shares no code, header or constant with the GPU
 * library; the product path never calls it.
 *
 * What is computed (Sec. 2.1, Alg. 2): starting from a lifted configuration
 * {C_h, A_h} at breakpoint h, the next lifting time is the current global time
 * plus the minimum, over active i and static j, of the time of flight tau_ij.
 * Active disks advance to that time (or to h'); at a lifting the active label
 * passes from i to j (Eq. 1: positions unchanged, activity transferred) and the
 * local time of j is set to the lifting time (Alg. 1).  At h' every chain stops
 * ("stalled", Remark on stalled spheres).  Output: the lifted configuration at
 * h' and the set L of liftings.
 *
 * Implementation notes (no reordering of the algorithm, only bookkeeping):
 *  - min over (i in A, j not in A) of tau_ij is min over chains of the chain's
 *    own minimum; each chain caches its own minimum (tau_c, j_c) and the cache
 *    is refreshed exactly when the set of static disks changes in a way that
 *    can alter it (its target became active, or a newly static disk appeared).
 *  - An active disk's stored position is the position at its activation; with
 *    all active disks sharing the velocity, its position at global time t is
 *    the stored one advanced by t - t_c.  This is Alg. 2's "advance all active
 *    disks" written lazily.
 *  - Static disks are kept in a uniform cell grid (cells at least one contact
 *    distance wide) so that the minimum over j is found without visiting all N
 *    disks; a brute-force mode visits all N disks and must give bit-identical
 *    results.
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes):
 *  - sigma is the disk radius; contact at centre distance d = 2 sigma (Sec. 1).
 *  - tau_ij = (forward distance along v from i to j) - b_ij with
 *    b_ij = sqrt(d^2 - dp^2) (Sec. 2.2; the text's "+ b" contradicts the time
 *    of flight used in Alg. 5 and Eq. 3; the minus sign is used).
 *  - periodic box: dp is the minimum image, the forward distance lies in
 *    [0, L), and a computed tau below zero (contact within rounding) is 0.
 *  - a disk is in the corridor iff dp^2 < d^2 (grazing contact: no lifting,
 *    consistent with tau = infinity in the footnote to Alg. 2).
 *  - ties: within a chain the smaller (tau, disk id) wins; between chains the
 *    smaller (event time, chain id) wins (the paper assumes generic times).
 *  - a lifting is admissible iff tau < h' - t_c (Alg. 5: before the breakpoint).
 *
 * Floating point: IEEE binary64, round to nearest, no contraction
 * (compile with -ffp-contract=off), correctly rounded sqrt.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_overlaps(int64_t n, double sigma, double L, const double *x,
                        const double *y, double tol);

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ELOG (-3)

typedef struct {
  int64_t n;
  double sigma, d, d2, L, halfL;
  int axis; /* 0: velocity along x, 1: along y */
  int sign; /* +1 or -1 */
  double *A; /* coordinate along the velocity axis (points into x or y) */
  double *P; /* perpendicular coordinate */
  /* cell grid of static disks (by current position) */
  int32_t nc;
  double cw; /* cell width */
  int32_t *head, *next, *prev, *cell_of;
} Sys;

/* ------------------------------------------------------------------------ */
/* Time of flight (Sec. 2.2, Eq. 2 context; Alg. 5).                          */
/* Returns +inf if j is outside the corridor |dp| < d.  *b_out = b_ij.        */
/* ------------------------------------------------------------------------ */
static double tof(const Sys *s, double ai, double pi, double aj, double pj,
                  double *b_out) {
  double dp = pj - pi;
  if (dp > s->halfL)
    dp = dp - s->L;
  else if (dp < -s->halfL)
    dp = dp + s->L;
  double dp2 = dp * dp;
  if (!(dp2 < s->d2)) return INFINITY;
  double da;
  if (s->sign > 0)
    da = aj - ai;
  else
    da = ai - aj;
  if (da < 0.0) da = da + s->L;
  double b = sqrt(s->d2 - dp2);
  double tau = da - b;
  if (tau < 0.0) tau = 0.0;
  if (b_out) *b_out = b;
  return tau;
}

/* Move a coordinate by distance `dist` along the velocity, wrapped to [0,L). */
static double advance(const Sys *s, double a, double dist) {
  double r;
  if (s->sign > 0) {
    r = a + dist;
    if (r >= s->L) r = r - s->L;
  } else {
    r = a - dist;
    if (r < 0.0) r = r + s->L;
  }
  if (r >= s->L) r = 0.0; /* a tiny negative plus L can round up to L */
  return r;
}

/* ------------------------------------------------------------------------ */
/* Cell grid of static disks                                                  */
/* ------------------------------------------------------------------------ */
static int32_t cell_col(const Sys *s, double v) {
  int32_t c = (int32_t)floor(v / s->cw);
  if (c < 0) c = 0;
  if (c >= s->nc) c = s->nc - 1;
  return c;
}
static int32_t cell_index(const Sys *s, int64_t i) {
  return cell_col(s, s->P[i]) * s->nc + cell_col(s, s->A[i]);
}
static void grid_insert(Sys *s, int64_t i) {
  int32_t c = cell_index(s, i);
  s->cell_of[i] = c;
  s->prev[i] = -1;
  s->next[i] = s->head[c];
  if (s->head[c] >= 0) s->prev[s->head[c]] = (int32_t)i;
  s->head[c] = (int32_t)i;
}
static void grid_remove(Sys *s, int64_t i) {
  int32_t c = s->cell_of[i];
  if (c < 0) return;
  if (s->prev[i] >= 0)
    s->next[s->prev[i]] = s->next[i];
  else
    s->head[c] = s->next[i];
  if (s->next[i] >= 0) s->prev[s->next[i]] = s->prev[i];
  s->cell_of[i] = -1;
  s->next[i] = s->prev[i] = -1;
}

typedef struct {
  double tau; /* +inf if no admissible candidate */
  int32_t j;
  double b;
} Cand;

static int cand_less(double tau1, int32_t j1, double tau2, int32_t j2) {
  if (tau1 < tau2) return 1;
  if (tau1 > tau2) return 0;
  return j1 < j2;
}

/* Minimum over static disks j of (tau_ij, j) for the chain whose disk sat at
 * (ai, pi) when it was activated at time tc, evaluated at global time tnow:
 *  - tau < bound (the chain's remaining time h' - t_c: candidates beyond it
 *    can never be lifted to during this activation);
 *  - tc + tau >= tnow: a static disk whose contact time computed from the
 *    activation position lies in the past came to rest behind the moving disk
 *    after the disk had passed; it is not ahead of it (with h' - h shorter
 *    than L - d the next contact with it, one lap later, is never reached).
 * Cell search: rows covering the corridor, columns walked forward along the
 * velocity until the smallest tau a column can contain exceeds the best one
 * found.  */
static Cand scan_cells(const Sys *s, int64_t self, double ai, double pi,
                       double tc, double tnow, double bound) {
  Cand best = {INFINITY, -1, 0.0};
  const double margin = 1e-7;
  int32_t nc = s->nc;
  /* rows whose span meets [pi - d, pi + d], widened by one row each side */
  int32_t r_lo = (int32_t)floor((pi - s->d) / s->cw) - 1;
  int32_t r_hi = (int32_t)floor((pi + s->d) / s->cw) + 1;
  if (r_hi - r_lo + 1 >= nc) {
    r_lo = 0;
    r_hi = nc - 1;
  }
  int32_t col_i = cell_col(s, ai);
  double f; /* distance from the trailing edge of the own column to ai */
  if (s->sign > 0)
    f = ai - (double)col_i * s->cw;
  else
    f = (double)(col_i + 1) * s->cw - ai;
  for (int32_t m = 0; m < nc; ++m) {
    if (m >= 1) {
      /* every disk in the m-th column ahead is at least m*cw - f away */
      double lb = (double)m * s->cw - f - s->d - margin;
      double lim = best.tau < bound ? best.tau : bound;
      if (lb > lim) break;
    }
    int32_t col = s->sign > 0 ? col_i + m : col_i - m;
    col = ((col % nc) + nc) % nc;
    for (int32_t rr = r_lo; rr <= r_hi; ++rr) {
      int32_t row = ((rr % nc) + nc) % nc;
      for (int32_t j = s->head[row * nc + col]; j >= 0; j = s->next[j]) {
        if (j == self) continue;
        double b;
        double tau = tof(s, ai, pi, s->A[j], s->P[j], &b);
        if (!(tau < bound) || tc + tau < tnow) continue;
        if (cand_less(tau, j, best.tau, best.j)) {
          best.tau = tau;
          best.j = j;
          best.b = b;
        }
      }
    }
  }
  return best;
}

/* Same minimum by visiting every disk (mode 1). */
static Cand scan_all(const Sys *s, const uint8_t *is_active, int64_t self,
                     double ai, double pi, double tc, double tnow,
                     double bound) {
  Cand best = {INFINITY, -1, 0.0};
  for (int64_t j = 0; j < s->n; ++j) {
    if (j == self || is_active[j]) continue;
    double b;
    double tau = tof(s, ai, pi, s->A[j], s->P[j], &b);
    if (!(tau < bound) || tc + tau < tnow) continue;
    if (cand_less(tau, (int32_t)j, best.tau, best.j)) {
      best.tau = tau;
      best.j = (int32_t)j;
      best.b = b;
    }
  }
  return best;
}

/* ------------------------------------------------------------------------ */
/* One leg [0, T] of Alg. 2 with the given direction (leg-relative times).  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t *chain, *from, *to;
  double *time, *b;
  int64_t cap, n;
} Log;

static int run_leg(Sys *s, int32_t k, int32_t *active, double T, int brute,
                   uint8_t *is_active, double *stamp, Log *log, double *sum_b,
                   int64_t *events) {
  int64_t n = s->n;
  double *tc = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
  Cand *cand = (Cand *)malloc(sizeof(Cand) * (size_t)(k > 0 ? k : 1));
  if (!tc || !cand) {
    free(tc);
    free(cand);
    return OR_ENOMEM;
  }
  /* Alg. 1: all local times start at h (= 0 in leg-relative time). */
  for (int64_t i = 0; i < n; ++i) stamp[i] = 0.0;
  memset(is_active, 0, (size_t)n);
  for (int32_t c = 0; c < k; ++c) is_active[active[c]] = 1;
  if (!brute) {
    for (int32_t c = 0; c < s->nc * s->nc; ++c) s->head[c] = -1;
    for (int64_t i = 0; i < n; ++i) {
      s->cell_of[i] = -1;
      s->next[i] = s->prev[i] = -1;
      if (!is_active[i]) grid_insert(s, i);
    }
  }
  for (int32_t c = 0; c < k; ++c) {
    int64_t i = active[c];
    tc[c] = 0.0;
    cand[c] = brute ? scan_all(s, is_active, i, s->A[i], s->P[i], 0.0, 0.0, T)
                    : scan_cells(s, i, s->A[i], s->P[i], 0.0, 0.0, T);
  }
  for (;;) {
    /* next lifting: smallest event time t_c + tau_c over admissible chains */
    int32_t w = -1;
    double ew = INFINITY;
    for (int32_t c = 0; c < k; ++c) {
      if (!(cand[c].tau < T - tc[c])) continue;
      double e = tc[c] + cand[c].tau;
      if (w < 0 || e < ew) {
        w = c;
        ew = e;
      }
    }
    if (w < 0) break;
    int64_t i = active[w];
    int32_t j = cand[w].j;
    double tau = cand[w].tau;
    double bw = cand[w].b;
    /* Eq. 1 and Alg. 1: i stops where it touches j; j takes over. */
    s->A[i] = advance(s, s->A[i], tau);
    stamp[i] = ew;
    stamp[j] = ew;
    is_active[i] = 0;
    is_active[j] = 1;
    if (!brute) {
      grid_insert(s, i);
      grid_remove(s, j);
    }
    if (log->chain) {
      if (log->n >= log->cap) {
        free(tc);
        free(cand);
        return OR_ELOG;
      }
      log->chain[log->n] = w;
      log->from[log->n] = (int32_t)i;
      log->to[log->n] = j;
      log->time[log->n] = ew;
      log->b[log->n] = bw;
    }
    log->n++;
    sum_b[w] += bw;
    (*events)++;
    active[w] = j;
    tc[w] = ew;
    /* refresh the caches that this lifting can change */
    for (int32_t c = 0; c < k; ++c) {
      int64_t ic = active[c];
      double bound = T - tc[c];
      if (c == w || cand[c].j == j) {
        cand[c] = brute ? scan_all(s, is_active, ic, s->A[ic], s->P[ic], tc[c],
                                   ew, bound)
                        : scan_cells(s, ic, s->A[ic], s->P[ic], tc[c], ew,
                                     bound);
      } else {
        double b;
        double t2 = tof(s, s->A[ic], s->P[ic], s->A[i], s->P[i], &b);
        if (t2 < bound && !(tc[c] + t2 < ew) &&
            cand_less(t2, (int32_t)i, cand[c].tau, cand[c].j)) {
          cand[c].tau = t2;
          cand[c].j = (int32_t)i;
          cand[c].b = b;
        }
      }
    }
  }
  /* h' reached: every chain is stalled (Remark on stalled spheres). */
  for (int32_t c = 0; c < k; ++c) {
    int64_t i = active[c];
    s->A[i] = advance(s, s->A[i], T - tc[c]);
    stamp[i] = T;
  }
  free(tc);
  free(cand);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Public entry point.                                                        */
/*                                                                            */
/*  x, y      : positions in [0, L), in/out                                   */
/*  active    : disk of each chain, in/out (distinct)                         */
/*  leg_dir   : per leg 0:+x 1:+y 2:-x 3:-y                                   */
/*  T         : leg length h' - h                                             */
/*  mode      : 0 cell search, 1 visit every disk                             */
/*  logs      : per-lifting records (may be NULL; then only counted)          */
/*  sum_b     : per chain, accumulated (in/out)                               */
/*  stamps    : local times at the end of the last leg (out, may be NULL)     */
/* ------------------------------------------------------------------------ */
int oracle_run(int64_t n, double sigma, double L, double *x, double *y,
               int32_t k, int32_t *active, int32_t n_legs,
               const int32_t *leg_dir, double T, int32_t mode, int64_t log_cap,
               int32_t *log_chain, int32_t *log_from, int32_t *log_to,
               double *log_time, double *log_b, int64_t *n_events,
               double *sum_b, double *stamps) {
  if (n < 1 || !(sigma > 0.0) || !(L > 0.0) || k < 0 || k > n || n_legs < 0 ||
      !(T >= 0.0) || (mode != 0 && mode != 1) || !x || !y ||
      (k > 0 && (!active || !sum_b)) || (n_legs > 0 && !leg_dir))
    return OR_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (!(x[i] >= 0.0 && x[i] < L && y[i] >= 0.0 && y[i] < L))
      return OR_EINVAL;
  /* with several chains, a rescan at a later global time discards disks that
   * came to rest behind the moving disk; that is exact only if no contact one
   * lap later can fall inside the leg (see scan_cells). */
  if (k > 1 && !(T < L - 2.0 * sigma)) return OR_EINVAL;
  /* hard disks may not overlap (contacts computed in earlier legs may sit a
   * few rounding units inside the contact distance) */
  if (oracle_overlaps(n, sigma, L, x, y, 1e-9 * sigma) != 0) return OR_EINVAL;
  Sys s;
  memset(&s, 0, sizeof(s));
  s.n = n;
  s.sigma = sigma;
  s.d = 2.0 * sigma;
  s.d2 = s.d * s.d;
  s.L = L;
  s.halfL = 0.5 * L;
  s.nc = (int32_t)floor(L / s.d);
  if (s.nc < 1) s.nc = 1;
  while (s.nc > 1 && L / (double)s.nc < s.d) s.nc--;
  s.cw = L / (double)s.nc;
  uint8_t *is_active = (uint8_t *)calloc((size_t)n, 1);
  double *stamp = (double *)malloc(sizeof(double) * (size_t)n);
  s.head = (int32_t *)malloc(sizeof(int32_t) * (size_t)s.nc * (size_t)s.nc);
  s.next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  s.prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  s.cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int rc = OR_OK;
  if (!is_active || !stamp || !s.head || !s.next || !s.prev || !s.cell_of) {
    rc = OR_ENOMEM;
    goto done;
  }
  for (int32_t c = 0; c < k; ++c) {
    if (active[c] < 0 || active[c] >= n || is_active[active[c]]) {
      rc = OR_EINVAL;
      goto done;
    }
    is_active[active[c]] = 1;
  }
  for (int64_t i = 0; i < n; ++i) stamp[i] = 0.0;
  Log log = {log_chain, log_from, log_to, log_time, log_b, log_cap, 0};
  if (log_chain && (!log_from || !log_to || !log_time || !log_b)) {
    rc = OR_EINVAL;
    goto done;
  }
  int64_t events = 0;
  for (int32_t leg = 0; leg < n_legs; ++leg) {
    int dcode = leg_dir[leg];
    if (dcode < 0 || dcode > 3) {
      rc = OR_EINVAL;
      goto done;
    }
    s.axis = dcode & 1;
    s.sign = dcode >= 2 ? -1 : 1;
    s.A = s.axis == 0 ? x : y;
    s.P = s.axis == 0 ? y : x;
    rc = run_leg(&s, k, active, T, mode == 1, is_active, stamp, &log, sum_b,
                 &events);
    if (rc != OR_OK) goto done;
  }
  if (n_events) *n_events = events;
  if (stamps)
    for (int64_t i = 0; i < n; ++i) stamps[i] = stamp[i];
done:
  free(is_active);
  free(stamp);
  free(s.head);
  free(s.next);
  free(s.prev);
  free(s.cell_of);
  return rc;
}

/* Number of pairs closer than d - tol (minimum image), by cell search.
 * Used by the tests' no-overlap invariant. */
int64_t oracle_overlaps(int64_t n, double sigma, double L, const double *x,
                        const double *y, double tol) {
  double d = 2.0 * sigma;
  double lim = d - tol;
  double lim2 = lim * lim;
  double halfL = 0.5 * L;
  int32_t nc = (int32_t)floor(L / d);
  while (nc > 1 && L / (double)nc < d) nc--;
  if (nc < 3) nc = 1; /* tiny boxes: one cell holding every disk */
  double cw = L / (double)nc;
  int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc * (size_t)nc);
  int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!head || !next) {
    free(head);
    free(next);
    return -1;
  }
  for (int64_t c = 0; c < (int64_t)nc * nc; ++c) head[c] = -1;
  for (int64_t i = 0; i < n; ++i) {
    int32_t cx = (int32_t)floor(x[i] / cw), cy = (int32_t)floor(y[i] / cw);
    if (cx < 0) cx = 0;
    if (cx >= nc) cx = nc - 1;
    if (cy < 0) cy = 0;
    if (cy >= nc) cy = nc - 1;
    next[i] = head[cy * nc + cx];
    head[cy * nc + cx] = (int32_t)i;
  }
  int64_t count = 0;
  int32_t span = nc >= 3 ? 1 : 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t cx = (int32_t)floor(x[i] / cw), cy = (int32_t)floor(y[i] / cw);
    if (cx >= nc) cx = nc - 1;
    if (cy >= nc) cy = nc - 1;
    if (cx < 0) cx = 0;
    if (cy < 0) cy = 0;
    for (int32_t oy = -span; oy <= span; ++oy)
      for (int32_t ox = -span; ox <= span; ++ox) {
        int32_t qx = ((cx + ox) % nc + nc) % nc, qy = ((cy + oy) % nc + nc) % nc;
        for (int32_t j = head[qy * nc + qx]; j >= 0; j = next[j]) {
          if (j <= i) continue;
          double dx = x[j] - x[i], dy = y[j] - y[i];
          if (dx > halfL) dx -= L;
          else if (dx < -halfL) dx += L;
          if (dy > halfL) dy -= L;
          else if (dy < -halfL) dy += L;
          if (dx * dx + dy * dy < lim2) count++;
        }
      }
  }
  free(head);
  free(next);
  return count;
}
