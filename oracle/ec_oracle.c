/*
 * ec_oracle.c -- TEST INFRASTRUCTURE ONLY (see ec_oracle.h).
 *
 * Plain serial FP64 reference of the parallel event-chain (PEC) Monte Carlo
 * sweep for hard disks.  Written step by step from the paper:
 *   - event chain, straight variant: Sec. 3.2 (a disk moves along d until it
 *     touches another; the rest of ell passes to the hit disk);
 *   - xy / +x directions for a single periodic box: Sec. 3.2;
 *   - PEC sweep: Sec. 3.4, steps 1-7 (shifted square cells, 2x2 blocks, one
 *     colour order per sweep, n_m starts per cell drawn WITH replacement,
 *     other cells frozen);
 *   - reflection at the cell wall and at frozen disks, angle of incidence equal
 *     to angle of reflection: Sec. 3.4 and Fig. 1 (right);
 *   - volume fraction and box: Sec. 2, eta = N pi sigma^2 / (4 L^2).
 * Readings where the paper is silent (ties, direction law, RNG streams, EC
 * pressure with reflections, halo band) follow the written contract of this
 * project and are listed with the design notes.
 *
 * Build with -ffp-contract=off: every fused multiply-add is an explicit fma().
 */
#include "ec_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* pi rounded to the nearest double */
static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its definition.    */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream kinds (second key word). */
enum { KIND_SWEEP = 1, KIND_START = 2, KIND_DIR = 3, KIND_SHUFFLE = 4 };

/* A draw stream: words 0..3 of block 0, then of block 1, ...; the block number
 * is the fourth counter word. */
typedef struct {
  uint64_t key[2];
  uint64_t ctr[4];
  uint64_t buf[4];
  int pos;
} stream_t;

static void stream_init(stream_t* st, uint64_t seed, uint64_t kind, uint64_t c0, uint64_t c1,
                        uint64_t c2) {
  st->key[0] = seed; st->key[1] = kind;
  st->ctr[0] = c0; st->ctr[1] = c1; st->ctr[2] = c2; st->ctr[3] = 0;
  st->pos = 4;
}

static uint64_t stream_next(stream_t* st) {
  if (st->pos == 4) {
    orc_philox4x64_10(st->ctr, st->key, st->buf);
    st->ctr[3] += 1;
    st->pos = 0;
  }
  return st->buf[st->pos++];
}

/* Uniform double in [0,1): top 53 bits times 2^-53. */
static double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* Unbiased integer in [0, n) by Lemire's multiply-shift with rejection. */
static uint64_t draw_index(stream_t* st, uint64_t n) {
  uint64_t x = stream_next(st);
  unsigned __int128 m = (unsigned __int128)x * n;
  uint64_t l = (uint64_t)m;
  if (l < n) {
    uint64_t t = (0 - n) % n;
    while (l < t) {
      x = stream_next(st);
      m = (unsigned __int128)x * n;
      l = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

static uint64_t cell_key(const orc_params* p, int32_t cell) {
  return (uint64_t)(uint32_t)cell | ((uint64_t)p->system << 32);
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */
double orc_box_length(int64_t n, double sigma, double eta) {
  /* eta = N pi sigma^2 / (4 L^2)  =>  L = sigma sqrt(N pi / (4 eta))  (Sec. 2) */
  return sigma * sqrt((double)n * ORC_PI / (4.0 * eta));
}

void orc_lattice(const orc_params* p, double* x, double* y) {
  /* k x k centred-rectangular lattice, spacing a = L/k, odd rows shifted by a/2 */
  int64_t k = (int64_t)llround(sqrt((double)p->n));
  double L = orc_box_length(p->n, p->sigma, p->eta);
  double a = L / (double)k;
  for (int64_t j = 0; j < k; ++j)
    for (int64_t i = 0; i < k; ++i) {
      int64_t id = j * k + i;
      x[id] = ((double)i + ((j & 1) ? 0.75 : 0.25)) * a;
      y[id] = ((double)j + 0.5) * a;
    }
}

/* First contact of a disk moving along unit d with a disk at relative offset r:
 * |r - s d| = sigma with s the smaller root.  With a = r.d and c = r x d this
 * is s = a - sqrt(sigma^2 - c^2), defined when the other disk lies ahead
 * (a > 0) and inside the corridor (sigma^2 - c^2 > 0).  A negative value
 * (disks already in contact) is clamped to zero. */
double orc_collision_distance(double rx, double ry, double dx, double dy, double sigma) {
  double a = fma(rx, dx, ry * dy);
  double c = fma(rx, dy, -(ry * dx));
  double disc = fma(-c, c, sigma * sigma);
  if (a > 0.0 && disc > 0.0) {
    double s = a - sqrt(disc);
    if (s < 0.0) s = 0.0;
    return s;
  }
  return INFINITY;
}

/* ------------------------------------------------------------------------ */
/* Draws of one sweep (step 1 and 3 of the PEC sweep)                        */
/* ------------------------------------------------------------------------ */
static void decode_perm(uint64_t idx, int32_t perm[4]) {
  int32_t avail[4] = {0, 1, 2, 3};
  int navail = 4;
  uint64_t fact[4] = {6, 2, 1, 1};
  for (int pos = 0; pos < 4; ++pos) {
    uint64_t q = idx / fact[pos];
    idx = idx % fact[pos];
    perm[pos] = avail[q];
    for (int t = (int)q; t < navail - 1; ++t) avail[t] = avail[t + 1];
    navail--;
  }
}

void orc_sweep_draws(const orc_params* p, int64_t sweep, double* shift_x, double* shift_y,
                     int32_t perm[4]) {
  double L = orc_box_length(p->n, p->sigma, p->eta);
  double w = L / (double)p->cells;
  stream_t st;
  stream_init(&st, p->seed, KIND_SWEEP, (uint64_t)sweep, (uint64_t)p->system, 0);
  *shift_x = u01(stream_next(&st)) * w;
  *shift_y = u01(stream_next(&st)) * w;
  decode_perm(draw_index(&st, 24), perm);
}

int64_t orc_start_index(const orc_params* p, int64_t sweep, int32_t cell, int64_t chain,
                        int64_t n_c) {
  stream_t st;
  stream_init(&st, p->seed, KIND_START, (uint64_t)sweep, cell_key(p, cell), (uint64_t)chain);
  return (int64_t)draw_index(&st, (uint64_t)n_c);
}

void orc_direction(const orc_params* p, int64_t sweep, int32_t cell, int64_t chain, double* dx,
                   double* dy) {
  if (p->dir_mode == ORC_DIR_X) { *dx = 1.0; *dy = 0.0; return; }
  if (p->dir_mode == ORC_DIR_XY) {
    if ((chain & 1) == 0) { *dx = 1.0; *dy = 0.0; } else { *dx = 0.0; *dy = 1.0; }
    return;
  }
  /* isotropic: uniform point in the unit disk by rejection, then normalised */
  stream_t st;
  stream_init(&st, p->seed, KIND_DIR, (uint64_t)sweep, cell_key(p, cell), (uint64_t)chain);
  double vx, vy, r2;
  for (;;) {
    vx = 2.0 * u01(stream_next(&st)) - 1.0;
    vy = 2.0 * u01(stream_next(&st)) - 1.0;
    r2 = fma(vx, vx, vy * vy);
    if (r2 < 1.0 && r2 >= 0x1p-40) break;
  }
  double r = sqrt(r2);
  *dx = vx / r;
  *dy = vy / r;
}

/* ------------------------------------------------------------------------ */
/* Event log and digest                                                      */
/* ------------------------------------------------------------------------ */
static orc_event* g_log = NULL;
static int64_t g_log_cap = 0, g_log_n = 0, g_chain_no = 0;
/* threads of the phase-parallel mode (1: serial) */
static int g_threads = 1;

void orc_set_log(orc_event* buf, int64_t capacity) {
  g_log = buf; g_log_cap = capacity; g_log_n = 0; g_chain_no = 0;
}
int64_t orc_log_count(void) { return g_log_n; }

/* Event digest (a test device, not part of the method): every event of a
 * cell's phase gets the record r = bits(s) ^ id*K1 ^ kind<<56, and the cell
 * digest is the XOR over its events i = 0, 1, ... of mix(r ^ i*K2), with mix
 * the splitmix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).  The index makes
 * it order-sensitive; the XOR lets a device hash a batch of events at once. */
#define DIGEST_K1 0x9E3779B97F4A7C15ULL
#define DIGEST_K2 0xD6E8FEB86659FD93ULL

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* One event chain                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int periodic;
  int64_t n;              /* N: walls are ids N, N+1; pseudo N+2; end N+3   */
  double L, half_L, w, sigma, cap;
  int64_t n_own;
  double *ox, *oy;        /* movable disks (local coordinates, or global if periodic) */
  const int64_t* ogid;
  int64_t n_halo;
  const double *hx, *hy;  /* frozen disks (local coordinates) */
  const int64_t* hgid;
  int32_t cell;
  double* acc_delta;      /* this cell's accumulators */
  uint64_t* acc_cnt;
  uint64_t digest;
  uint64_t n_events;       /* events of this cell so far in the phase (digest index) */
  int reject;              /* ORC_BOUNDARY_REJECT: a wall or frozen event undoes the chain */
  int64_t u_n, u_cap;      /* undo log of the running chain: disk, position before a move */
  int64_t* u_a;
  double *u_x, *u_y;
} chain_ctx;

static void undo_push(chain_ctx* cx, int64_t a) {
  if (cx->u_n == cx->u_cap) {
    cx->u_cap = cx->u_cap ? 2 * cx->u_cap : 64;
    cx->u_a = (int64_t*)realloc(cx->u_a, sizeof(int64_t) * (size_t)cx->u_cap);
    cx->u_x = (double*)realloc(cx->u_x, sizeof(double) * (size_t)cx->u_cap);
    cx->u_y = (double*)realloc(cx->u_y, sizeof(double) * (size_t)cx->u_cap);
  }
  cx->u_a[cx->u_n] = a;
  cx->u_x[cx->u_n] = cx->ox[a];
  cx->u_y[cx->u_n] = cx->oy[a];
  cx->u_n += 1;
}

static void digest_event(chain_ctx* cx, int kind, int64_t gid, double s) {
  uint64_t sb;
  memcpy(&sb, &s, sizeof sb);
  const uint64_t r = sb ^ ((uint64_t)gid * DIGEST_K1) ^ ((uint64_t)kind << 56);
  cx->digest ^= mix64(r ^ (cx->n_events * DIGEST_K2));
  cx->n_events += 1;
}

static double min_image(double r, const chain_ctx* cx) {
  if (r < -cx->half_L) r += cx->L;
  else if (r >= cx->half_L) r -= cx->L;
  return r;
}

static double wrap_box(double v, const chain_ctx* cx) {
  if (v >= cx->L) v -= cx->L;
  else if (v < 0.0) v += cx->L;
  return v;
}

static void log_event(const chain_ctx* cx, int kind, int64_t gid, int64_t active, double s, double dx,
                      double dy, double ax, double ay, double px, double py) {
  if (!g_log) return;
  if (g_log_n < g_log_cap) {
    orc_event* e = &g_log[g_log_n];
    e->chain = g_chain_no; e->cell = cx->cell; e->kind = kind; e->gid = gid;
    e->active = active; e->s = s; e->dx = dx; e->dy = dy;
    e->ax = ax; e->ay = ay; e->px = px; e->py = py;
  }
  g_log_n++;
}

static void move_by(chain_ctx* cx, int64_t a, double s, double dx, double dy) {
  cx->ox[a] = fma(s, dx, cx->ox[a]);
  cx->oy[a] = fma(s, dy, cx->oy[a]);
  if (cx->periodic) {
    cx->ox[a] = wrap_box(cx->ox[a], cx);
    cx->oy[a] = wrap_box(cx->oy[a], cx);
  }
}

static void run_chain(chain_ctx* cx, int64_t a, double dx, double dy, double ell) {
  double rem = ell;
  double sigma = cx->sigma;
  double idx = (dx != 0.0) ? 1.0 / dx : 0.0;
  double idy = (dy != 0.0) ? 1.0 / dy : 0.0;
  cx->acc_cnt[ORC_CNT_CHAINS] += 1;
  /* rejection variant: the chain's lifts and contact sum count only if it is accepted */
  double chain_delta = 0.0;
  uint64_t chain_lifts = 0;
  cx->u_n = 0;
  for (;;) {
    double ax = cx->ox[a], ay = cx->oy[a];
    /* brute-force search for the first event: key (s, id), lowest id wins ties */
    double best_s = INFINITY;
    int64_t best_gid = INT64_MAX;
    int best_kind = 0;
    int64_t best_j = -1;
    for (int64_t j = 0; j < cx->n_own; ++j) {
      if (j == a) continue;
      double rx = cx->ox[j] - ax, ry = cx->oy[j] - ay;
      if (cx->periodic) { rx = min_image(rx, cx); ry = min_image(ry, cx); }
      double s = orc_collision_distance(rx, ry, dx, dy, sigma);
      if (s < best_s || (s == best_s && s != INFINITY && cx->ogid[j] < best_gid)) {
        best_s = s; best_gid = cx->ogid[j]; best_kind = ORC_EV_LIFT; best_j = j;
      }
    }
    for (int64_t h = 0; h < cx->n_halo; ++h) {
      double rx = cx->hx[h] - ax, ry = cx->hy[h] - ay;
      double s = orc_collision_distance(rx, ry, dx, dy, sigma);
      if (s < best_s || (s == best_s && s != INFINITY && cx->hgid[h] < best_gid)) {
        best_s = s; best_gid = cx->hgid[h]; best_kind = ORC_EV_FROZEN; best_j = h;
      }
    }
    if (!cx->periodic) {
      /* cell walls at local coordinates 0 and w; the centre may not cross them */
      if (dx != 0.0) {
        double t = (dx > 0.0) ? (cx->w - ax) * idx : (0.0 - ax) * idx;
        if (t < 0.0) t = 0.0;
        if (t < best_s || (t == best_s && cx->n + 0 < best_gid)) {
          best_s = t; best_gid = cx->n + 0; best_kind = ORC_EV_WALL_X; best_j = -1;
        }
      }
      if (dy != 0.0) {
        double t = (dy > 0.0) ? (cx->w - ay) * idy : (0.0 - ay) * idy;
        if (t < 0.0) t = 0.0;
        if (t < best_s || (t == best_s && cx->n + 1 < best_gid)) {
          best_s = t; best_gid = cx->n + 1; best_kind = ORC_EV_WALL_Y; best_j = -1;
        }
      }
    } else {
      /* periodic box: nearest images are exact only for flights up to L/2 - sigma */
      double lim = best_s < rem ? best_s : rem;
      if (lim > cx->cap) {
        digest_event(cx, ORC_EV_PSEUDO, cx->n + 2, cx->cap);
        move_by(cx, a, cx->cap, dx, dy);
        log_event(cx, ORC_EV_PSEUDO, cx->n + 2, cx->ogid[a], cx->cap, dx, dy, cx->ox[a], cx->oy[a],
                  NAN, NAN);
        rem = rem - cx->cap;
        cx->acc_cnt[ORC_CNT_PSEUDO] += 1;
        continue;
      }
    }
    if (!(best_s < rem)) {
      /* no event before the displacement is used up: the chain ends */
      digest_event(cx, ORC_EV_END, cx->n + 3, rem);
      move_by(cx, a, rem, dx, dy);
      log_event(cx, ORC_EV_END, cx->n + 3, cx->ogid[a], rem, dx, dy, cx->ox[a], cx->oy[a], NAN,
                NAN);
      if (cx->reject) {  /* accepted */
        cx->acc_delta[0] += chain_delta;
        cx->acc_cnt[ORC_CNT_LIFTS] += chain_lifts;
      }
      break;
    }
    digest_event(cx, best_kind, best_gid, best_s);
    if (cx->reject) undo_push(cx, a);
    move_by(cx, a, best_s, dx, dy);
    rem = rem - best_s;
    ax = cx->ox[a]; ay = cx->oy[a];
    {
      double px = NAN, py = NAN;
      if (best_kind == ORC_EV_LIFT) { px = cx->ox[best_j]; py = cx->oy[best_j]; }
      if (best_kind == ORC_EV_FROZEN) { px = cx->hx[best_j]; py = cx->hy[best_j]; }
      log_event(cx, best_kind, best_gid, cx->ogid[a], best_s, dx, dy, ax, ay, px, py);
    }
    if (cx->reject && best_kind != ORC_EV_LIFT) {
      /* a wall or a frozen disk: the whole chain is rejected -- every move is
       * undone, latest first; the event that caused it is counted */
      cx->acc_cnt[best_kind == ORC_EV_FROZEN ? ORC_CNT_FROZEN : ORC_CNT_WALLS] += 1;
      for (int64_t u = cx->u_n - 1; u >= 0; --u) {
        cx->ox[cx->u_a[u]] = cx->u_x[u];
        cx->oy[cx->u_a[u]] = cx->u_y[u];
      }
      break;
    }
    if (best_kind == ORC_EV_LIFT) {
      /* straight EC: the hit disk continues along the same direction */
      double rx = cx->ox[best_j] - ax, ry = cx->oy[best_j] - ay;
      if (cx->periodic) { rx = min_image(rx, cx); ry = min_image(ry, cx); }
      if (cx->reject) {
        chain_delta = chain_delta + fma(rx, dx, ry * dy);
        chain_lifts += 1;
      } else {
        cx->acc_delta[0] += fma(rx, dx, ry * dy);
        cx->acc_cnt[ORC_CNT_LIFTS] += 1;
      }
      a = best_j;
    } else if (best_kind == ORC_EV_FROZEN) {
      /* specular reflection about the contact normal */
      double rx = cx->hx[best_j] - ax, ry = cx->hy[best_j] - ay;
      cx->acc_delta[0] += fma(rx, dx, ry * dy);
      cx->acc_cnt[ORC_CNT_FROZEN] += 1;
      double nrm = sqrt(fma(rx, rx, ry * ry));
      double nx = rx / nrm, ny = ry / nrm;
      double dn = fma(dx, nx, dy * ny);
      double t = -2.0 * dn;
      double ux = fma(t, nx, dx), uy = fma(t, ny, dy);
      double m = sqrt(fma(ux, ux, uy * uy));
      dx = ux / m;
      dy = uy / m;
      idx = (dx != 0.0) ? 1.0 / dx : 0.0;
      idy = (dy != 0.0) ? 1.0 / dy : 0.0;
    } else if (best_kind == ORC_EV_WALL_X) {
      dx = -dx; idx = -idx;
      cx->acc_cnt[ORC_CNT_WALLS] += 1;
    } else { /* ORC_EV_WALL_Y */
      dy = -dy; idy = -idy;
      cx->acc_cnt[ORC_CNT_WALLS] += 1;
    }
  }
  g_chain_no++;
}

/* ------------------------------------------------------------------------ */
/* Start lists (step 5 of the PEC sweep)                                     */
/* ------------------------------------------------------------------------ */
/* Fill starts[0..n_m) with indices into the cell's id-ordered own list. */
static void make_start_list_(const orc_params* p, int64_t sweep, int32_t cell, int64_t n_c,
                             int64_t n_m, int64_t* starts);
void orc_start_list(const orc_params* p, int64_t sweep, int32_t cell, int64_t n_c, int64_t n_m,
                    int64_t* starts) {
  make_start_list_(p, sweep, cell, n_c, n_m, starts);
}
static void make_start_list_(const orc_params* p, int64_t sweep, int32_t cell, int64_t n_c,
                            int64_t n_m, int64_t* starts) {
  if (p->start_mode == ORC_START_DISTINCT) {
    /* shuffled list of distinct disks (the variant shown to be incorrect) */
    int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_c);
    for (int64_t i = 0; i < n_c; ++i) list[i] = i;
    stream_t st;
    stream_init(&st, p->seed, KIND_SHUFFLE, (uint64_t)sweep, cell_key(p, cell), 0);
    for (int64_t i = 0; i + 1 < n_c; ++i) {
      int64_t j = i + (int64_t)draw_index(&st, (uint64_t)(n_c - i));
      int64_t t = list[i]; list[i] = list[j]; list[j] = t;
    }
    for (int64_t k = 0; k < n_m; ++k) starts[k] = list[k % n_c];
    free(list);
  } else {
    /* drawn with replacement: every start is uniform over all disks of the cell */
    for (int64_t k = 0; k < n_m; ++k) starts[k] = orc_start_index(p, sweep, cell, k, n_c);
  }
}

/* ------------------------------------------------------------------------ */
/* Sweeps                                                                    */
/* ------------------------------------------------------------------------ */
static int check_params(const orc_params* p) {
  if (p->n < 1 || !(p->sigma > 0.0) || !(p->eta > 0.0) || !(p->ell > 0.0)) return -1;
  if (p->eta >= ORC_PI / (2.0 * sqrt(3.0))) return -1;
  if (p->cells < 1) return -1;
  if (p->cells > 1 && (p->cells < 4 || (p->cells & 1))) return -1;
  double L = orc_box_length(p->n, p->sigma, p->eta);
  if (p->boundary == ORC_BOUNDARY_STRIPES) {
    /* stripes wider than 2 sigma (frozen disks come from the two neighbours),
     * a box longer than 2 sigma (nearest images along the stripe), chains
     * along the stripes */
    if (p->cells < 4 || (p->cells & 1) || p->dir_mode != ORC_DIR_XY) return -1;
    if (!(L / (double)p->cells > 2.0 * p->sigma) || !(L > 2.0 * p->sigma)) return -1;
    return 0;
  }
  if (p->cells > 1 && p->dir_mode != ORC_DIR_ISO) return -1;
  if (p->cells == 1 && !(L > 2.0 * p->sigma)) return -1;
  if (p->cells > 1 && !(L / (double)p->cells > p->sigma)) return -1;
  if (p->boundary > ORC_BOUNDARY_REJECT || (p->boundary == ORC_BOUNDARY_REJECT && p->cells == 1)) return -1;
  return 0;
}

static void sweep_periodic(const orc_params* p, double* x, double* y, int64_t sweep,
                           double* acc_delta, uint64_t* acc_cnt, uint64_t* digest_out) {
  chain_ctx cx;
  memset(&cx, 0, sizeof cx);
  cx.periodic = 1;
  cx.n = p->n;
  cx.L = orc_box_length(p->n, p->sigma, p->eta);
  cx.half_L = 0.5 * cx.L;
  cx.sigma = p->sigma;
  cx.cap = cx.half_L - p->sigma;
  cx.n_own = p->n;
  cx.ox = x; cx.oy = y;
  int64_t* gid = (int64_t*)malloc(sizeof(int64_t) * (size_t)p->n);
  for (int64_t i = 0; i < p->n; ++i) gid[i] = i;
  cx.ogid = gid;
  cx.cell = 0;
  cx.acc_delta = &acc_delta[0];
  cx.acc_cnt = &acc_cnt[0];
  cx.digest = 0;
  cx.n_events = 0;
  int64_t n_m = p->chains_per_cell > 0 ? p->chains_per_cell : p->n;
  int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_m > 0 ? n_m : 1));
  make_start_list_(p, sweep, 0, p->n, n_m, starts);
  for (int64_t k = 0; k < n_m; ++k) {
    double dx, dy;
    orc_direction(p, sweep, 0, k, &dx, &dy);
    run_chain(&cx, starts[k], dx, dy, p->ell);
  }
  if (digest_out) *digest_out = cx.digest; /* cell 0: weight 2*0+1 = 1 */
  free(starts);
  free(gid);
}

/* Shifted-frame coordinate and local cell coordinate of a position. */
static double shifted(double pos, double shift, double L) {
  double t = pos - shift;
  if (t < 0.0) t += L;
  return t;
}
static double local_coord(double pos, double shift, double origin, double L, double half_L) {
  double v = shifted(pos, shift, L) - origin;
  if (v < -half_L) v += L;
  else if (v >= half_L) v -= L;
  return v;
}

int orc_assign_cells(const orc_params* p, const double* x, const double* y, int64_t sweep,
                     int32_t* cell_of) {
  if (check_params(p) != 0) return -1;
  int32_t C = p->cells;
  if (C == 1) { for (int64_t i = 0; i < p->n; ++i) cell_of[i] = 0; return 0; }
  double L = orc_box_length(p->n, p->sigma, p->eta);
  double w = L / (double)C;
  double sx, sy;
  int32_t perm[4];
  orc_sweep_draws(p, sweep, &sx, &sy, perm);
  for (int64_t i = 0; i < p->n; ++i) {
    int64_t cxi = (int64_t)floor(shifted(x[i], sx, L) / w);
    int64_t cyi = (int64_t)floor(shifted(y[i], sy, L) / w);
    if (cxi > C - 1) cxi = C - 1;
    if (cyi > C - 1) cyi = C - 1;
    cell_of[i] = (int32_t)(cyi * C + cxi);
  }
  return 0;
}

/* Process one simulation cell of a sweep: stage own and frozen disks, run its
 * chains, write the moved disks back.  start/ids are the id-ordered own lists
 * of all cells (cell c: ids[start[c] .. start[c+1])). */
static void run_cell(const orc_params* p, double* x, double* y, int64_t sweep, int32_t cell,
                     const int64_t* start, const int64_t* ids, double sx, double sy,
                     double* acc_delta, uint64_t* acc_cnt, uint64_t* cell_digest) {
  const int64_t* own_ids = &ids[start[cell]];
  const int64_t n_c = start[cell + 1] - start[cell];
  int32_t C = p->cells;
  double L = orc_box_length(p->n, p->sigma, p->eta);
  double half_L = 0.5 * L;
  double w = L / (double)C;
  double sigma = p->sigma;
  int32_t cxi = cell % C, cyi = cell / C;
  double ox = (double)cxi * w, oy = (double)cyi * w;

  double* vx = (double*)malloc(sizeof(double) * (size_t)(n_c > 0 ? n_c : 1));
  double* vy = (double*)malloc(sizeof(double) * (size_t)(n_c > 0 ? n_c : 1));
  double* vx0 = (double*)malloc(sizeof(double) * (size_t)(n_c > 0 ? n_c : 1));
  double* vy0 = (double*)malloc(sizeof(double) * (size_t)(n_c > 0 ? n_c : 1));
  for (int64_t k = 0; k < n_c; ++k) {
    int64_t i = own_ids[k];
    vx[k] = vx0[k] = local_coord(x[i], sx, ox, L, half_L);
    vy[k] = vy0[k] = local_coord(y[i], sy, oy, L, half_L);
  }
  /* frozen disks: centres of other cells within sigma of this cell (square
   * band).  The cell side exceeds sigma, so every such centre lies in one of
   * the eight neighbouring cells (C >= 4 makes them distinct); only their
   * lists are read, which no cell of the same colour writes. */
  int64_t n_h = 0, cap_h = 64;
  double* hx = (double*)malloc(sizeof(double) * (size_t)cap_h);
  double* hy = (double*)malloc(sizeof(double) * (size_t)cap_h);
  int64_t* hg = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap_h);
  for (int32_t nbh = 0; nbh < 9; ++nbh) {
   if (nbh == 4) continue;
   const int32_t ncx = (cxi + nbh % 3 - 1 + C) % C, ncy = (cyi + nbh / 3 - 1 + C) % C;
   const int32_t nc = ncy * C + ncx;
   for (int64_t t = start[nc]; t < start[nc + 1]; ++t) {
    const int64_t i = ids[t];
    double ux = local_coord(x[i], sx, ox, L, half_L);
    double uy = local_coord(y[i], sy, oy, L, half_L);
    if (ux >= -sigma && ux <= w + sigma && uy >= -sigma && uy <= w + sigma) {
      if (n_h == cap_h) {
        cap_h *= 2;
        hx = (double*)realloc(hx, sizeof(double) * (size_t)cap_h);
        hy = (double*)realloc(hy, sizeof(double) * (size_t)cap_h);
        hg = (int64_t*)realloc(hg, sizeof(int64_t) * (size_t)cap_h);
      }
      hx[n_h] = ux; hy[n_h] = uy; hg[n_h] = i; n_h++;
    }
   }
  }

  chain_ctx cx;
  memset(&cx, 0, sizeof cx);
  cx.periodic = 0;
  cx.n = p->n;
  cx.L = L; cx.half_L = half_L; cx.w = w; cx.sigma = sigma;
  cx.n_own = n_c; cx.ox = vx; cx.oy = vy; cx.ogid = own_ids;
  cx.n_halo = n_h; cx.hx = hx; cx.hy = hy; cx.hgid = hg;
  cx.cell = cell;
  cx.acc_delta = &acc_delta[cell];
  cx.acc_cnt = &acc_cnt[(int64_t)cell * ORC_CNT_NCOL];
  cx.digest = 0;
  cx.n_events = 0;
  cx.reject = p->boundary == ORC_BOUNDARY_REJECT;

  int64_t n_m = 0;
  if (n_c > 0) n_m = p->chains_per_cell > 0 ? p->chains_per_cell : n_c;
  int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_m > 0 ? n_m : 1));
  make_start_list_(p, sweep, cell, n_c, n_m, starts);
  for (int64_t k = 0; k < n_m; ++k) {
    double dx, dy;
    orc_direction(p, sweep, cell, k, &dx, &dy);
    run_chain(&cx, starts[k], dx, dy, p->ell);
  }
  /* write back: new position = old position + local displacement, wrapped */
  for (int64_t k = 0; k < n_c; ++k) {
    int64_t i = own_ids[k];
    double nx = x[i] + (vx[k] - vx0[k]);
    double ny = y[i] + (vy[k] - vy0[k]);
    if (nx < 0.0) nx += L; else if (nx >= L) nx -= L;
    if (ny < 0.0) ny += L; else if (ny >= L) ny -= L;
    x[i] = nx; y[i] = ny;
  }
  *cell_digest = cx.digest;
  free(starts); free(hx); free(hy); free(hg); free(vx); free(vy); free(vx0); free(vy0);
  free(cx.u_a); free(cx.u_x); free(cx.u_y);
}

/* id-ordered own lists of all cells: counting sort of disks by cell. */
static void build_lists(const int32_t* cell_of, int64_t n, int32_t ncells, int64_t* start,
                        int64_t* ids) {
  for (int32_t c = 0; c <= ncells; ++c) start[c] = 0;
  for (int64_t i = 0; i < n; ++i) start[cell_of[i] + 1]++;
  for (int32_t c = 0; c < ncells; ++c) start[c + 1] += start[c];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncells);
  for (int32_t c = 0; c < ncells; ++c) fill[c] = start[c];
  for (int64_t i = 0; i < n; ++i) ids[fill[cell_of[i]]++] = i;
  free(fill);
}

static int cell_colour(int32_t cell, int32_t C) {
  int32_t cxi = cell % C, cyi = cell / C;
  return (cxi & 1) | ((cyi & 1) << 1);
}

static void sweep_cells(const orc_params* p, double* x, double* y, int64_t sweep, int32_t n_phases,
                        const int32_t* only, int32_t n_only, double* acc_delta, uint64_t* acc_cnt,
                        uint64_t* digest_out, uint64_t* only_digest) {
  int32_t C = p->cells, ncells = C * C;
  double sx, sy;
  int32_t perm[4];
  orc_sweep_draws(p, sweep, &sx, &sy, perm);
  int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)p->n);
  orc_assign_cells(p, x, y, sweep, cell_of);
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncells + 1));
  int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)p->n);
  build_lists(cell_of, p->n, ncells, start, ids);
  /* the cells of one colour share nothing (each writes only its own disks and
   * its own accumulators, and reads the lists of neighbours of other
   * colours), so with threads they run in parallel; the sweep digest is a sum
   * over cells and does not depend on their order */
  uint64_t* h = (uint64_t*)calloc((size_t)ncells, sizeof(uint64_t));
  int32_t* todo = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncells > 0 ? ncells : 1));
  const int threads = (g_log == NULL && g_threads > 1) ? g_threads : 1;
  for (int32_t q = 0; q < n_phases; ++q) {
    int colour = perm[q];
    int32_t n_todo = 0;
    for (int32_t c = 0; c < ncells; ++c) {
      if (cell_colour(c, C) != colour) continue;
      if (only) {
        int32_t slot = -1;
        for (int32_t t = 0; t < n_only; ++t) if (only[t] == c) { slot = t; break; }
        if (slot < 0) continue;
      }
      todo[n_todo++] = c;
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) if (threads > 1)
    for (int32_t t = 0; t < n_todo; ++t)
      run_cell(p, x, y, sweep, todo[t], start, ids, sx, sy, acc_delta, acc_cnt, &h[todo[t]]);
  }
  uint64_t total = 0;
  for (int32_t c = 0; c < ncells; ++c) total += h[c] * (2ULL * (uint64_t)c + 1ULL);
  if (only_digest)
    for (int32_t t = 0; t < n_only; ++t)
      only_digest[t] = (only[t] >= 0 && only[t] < ncells) ? h[only[t]] : 0;
  if (digest_out) *digest_out = total;
  free(h); free(todo);
  free(cell_of); free(start); free(ids);
}

void orc_set_threads(int32_t n) { g_threads = n > 1 ? n : 1; }

/* ------------------------------------------------------------------------ */
/* Striped decomposition with rejection (Sec. 3.4, Fig. 3 "stripes"; Sec. 4) */
/* ------------------------------------------------------------------------ */
/* Disks of one stripe move along it: coordinate a (along the stripe, periodic
 * in [0, L)) and v (across it, local to the stripe).  Frozen disks are those
 * of the two neighbouring stripes within sigma of it. */
typedef struct {
  double L, half_L, sigma, cap;
  int64_t n;                         /* N: pseudo event id N+2, chain end N+3 */
  int64_t n_own, n_fr;
  double *oa, *ov;                   /* own disks (a updated in place)        */
  const int64_t* ogid;
  const double *fa, *fv;             /* frozen disks                          */
  const int64_t* fgid;
  double* acc_delta;
  uint64_t* acc_cnt;
  uint64_t digest, n_events;
  int64_t u_n, u_cap, *u_i;          /* undo log of the running chain          */
  double* u_a;
} stripe_ctx;

static void stripe_digest(stripe_ctx* sx, int kind, int64_t gid, double s) {
  uint64_t sb;
  memcpy(&sb, &s, sizeof sb);
  const uint64_t r = sb ^ ((uint64_t)gid * DIGEST_K1) ^ ((uint64_t)kind << 56);
  sx->digest ^= mix64(r ^ (sx->n_events * DIGEST_K2));
  sx->n_events += 1;
}

/* Contact distance along the stripe to a disk at offset (ra, rv): the
 * collision distance of Sec. 3.2 with the direction (1, 0). */
static double stripe_contact(double ra, double rv, double sigma) {
  const double disc = fma(-rv, rv, sigma * sigma);
  if (ra > 0.0 && disc > 0.0) {
    double s = ra - sqrt(disc);
    if (s < 0.0) s = 0.0;
    return s;
  }
  return INFINITY;
}

static double stripe_image(double r, const stripe_ctx* sx) {
  if (r < -sx->half_L) r += sx->L;
  else if (r >= sx->half_L) r -= sx->L;
  return r;
}

/* Move own disk i by s along the stripe in direction sgn (+1 or -1). */
static void stripe_move(stripe_ctx* sx, int64_t i, double s, int sgn) {
  double a = sgn > 0 ? sx->oa[i] + s : sx->oa[i] - s;
  if (a >= sx->L) a -= sx->L;
  else if (a < 0.0) a += sx->L;
  sx->oa[i] = a;
}

/* A chain along the stripe in direction sgn: the chain and its reverse (the
 * opposite direction from the last disk) are proposed alike, and a chain is
 * rejected exactly when its reverse is, so rejection keeps detailed balance. */
static void stripe_chain(stripe_ctx* sx, int64_t a, double ell, int sgn) {
  double rem = ell;
  double chain_delta = 0.0;
  uint64_t chain_lifts = 0;
  sx->u_n = 0;
  sx->acc_cnt[ORC_CNT_CHAINS] += 1;
  for (;;) {
    const double aa = sx->oa[a], av = sx->ov[a];
    double best_s = INFINITY;
    int64_t best_gid = INT64_MAX, best_j = -1;
    int best_kind = 0;
    for (int64_t j = 0; j < sx->n_own; ++j) {
      if (j == a) continue;
      const double ra = stripe_image(sx->oa[j] - aa, sx);
      const double s = stripe_contact(sgn > 0 ? ra : -ra, sx->ov[j] - av, sx->sigma);
      if (s < best_s || (s == best_s && s != INFINITY && sx->ogid[j] < best_gid)) {
        best_s = s; best_gid = sx->ogid[j]; best_j = j; best_kind = ORC_EV_LIFT;
      }
    }
    for (int64_t j = 0; j < sx->n_fr; ++j) {
      const double ra = stripe_image(sx->fa[j] - aa, sx);
      const double s = stripe_contact(sgn > 0 ? ra : -ra, sx->fv[j] - av, sx->sigma);
      if (s < best_s || (s == best_s && s != INFINITY && sx->fgid[j] < best_gid)) {
        best_s = s; best_gid = sx->fgid[j]; best_j = j; best_kind = ORC_EV_FROZEN;
      }
    }
    /* nearest images are exact for flights up to L/2 - sigma only */
    const double lim = best_s < rem ? best_s : rem;
    if (lim > sx->cap) {
      stripe_digest(sx, ORC_EV_PSEUDO, sx->n + 2, sx->cap);
      if (sx->u_n == sx->u_cap) {
        sx->u_cap = sx->u_cap ? 2 * sx->u_cap : 64;
        sx->u_i = (int64_t*)realloc(sx->u_i, sizeof(int64_t) * (size_t)sx->u_cap);
        sx->u_a = (double*)realloc(sx->u_a, sizeof(double) * (size_t)sx->u_cap);
      }
      sx->u_i[sx->u_n] = a; sx->u_a[sx->u_n] = sx->oa[a]; sx->u_n += 1;
      stripe_move(sx, a, sx->cap, sgn);
      rem = rem - sx->cap;
      sx->acc_cnt[ORC_CNT_PSEUDO] += 1;
      continue;
    }
    if (!(best_s < rem)) {
      stripe_digest(sx, ORC_EV_END, sx->n + 3, rem);
      stripe_move(sx, a, rem, sgn);
      sx->acc_delta[0] += chain_delta;  /* accepted */
      sx->acc_cnt[ORC_CNT_LIFTS] += chain_lifts;
      break;
    }
    stripe_digest(sx, best_kind, best_gid, best_s);
    if (sx->u_n == sx->u_cap) {
      sx->u_cap = sx->u_cap ? 2 * sx->u_cap : 64;
      sx->u_i = (int64_t*)realloc(sx->u_i, sizeof(int64_t) * (size_t)sx->u_cap);
      sx->u_a = (double*)realloc(sx->u_a, sizeof(double) * (size_t)sx->u_cap);
    }
    sx->u_i[sx->u_n] = a; sx->u_a[sx->u_n] = sx->oa[a]; sx->u_n += 1;
    stripe_move(sx, a, best_s, sgn);
    rem = rem - best_s;
    if (best_kind == ORC_EV_FROZEN) {
      /* a disk of a neighbouring stripe: the chain is rejected and undone */
      sx->acc_cnt[ORC_CNT_FROZEN] += 1;
      for (int64_t u = sx->u_n - 1; u >= 0; --u) sx->oa[sx->u_i[u]] = sx->u_a[u];
      break;
    }
    const double rd = stripe_image(sx->oa[best_j] - sx->oa[a], sx);
    chain_delta = chain_delta + (sgn > 0 ? rd : -rd);
    chain_lifts += 1;
    a = best_j;
  }
}

static void sweep_stripes(const orc_params* p, double* x, double* y, int64_t sweep,
                          double* acc_delta, uint64_t* acc_cnt, uint64_t* digest_out) {
  const int32_t S = p->cells;
  const double L = orc_box_length(p->n, p->sigma, p->eta), half_L = 0.5 * L;
  const double h = L / (double)S, sigma = p->sigma;
  /* even sweeps: horizontal stripes, chains along +x; odd sweeps: vertical
   * stripes, chains along +y */
  double* along = (sweep & 1) ? y : x;
  const double* across = (sweep & 1) ? x : y;
  /* draws: the shift of the stripes across their direction, and which of
   * the two stripe colours goes first */
  stream_t st;
  stream_init(&st, p->seed, KIND_SWEEP, (uint64_t)sweep, (uint64_t)p->system, 0);
  const double shift = u01(stream_next(&st)) * h;
  const int first = (int)draw_index(&st, 2);
  int32_t* stripe_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)p->n);
  for (int64_t i = 0; i < p->n; ++i) {
    int64_t k = (int64_t)floor(shifted(across[i], shift, L) / h);
    if (k > S - 1) k = S - 1;
    stripe_of[i] = (int32_t)k;
  }
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S + 1));
  int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)p->n);
  build_lists(stripe_of, p->n, S, start, ids);
  uint64_t total = 0;
  for (int32_t q = 0; q < 2; ++q) {
    for (int32_t k = 0; k < S; ++k) {
      if ((k & 1) != (first ^ q)) continue;
      const double origin = (double)k * h;
      const int64_t n_c = start[k + 1] - start[k];
      stripe_ctx sx;
      memset(&sx, 0, sizeof sx);
      sx.L = L; sx.half_L = half_L; sx.sigma = sigma; sx.cap = half_L - sigma; sx.n = p->n;
      sx.n_own = n_c;
      sx.ogid = &ids[start[k]];
      sx.oa = (double*)malloc(sizeof(double) * (size_t)(n_c > 0 ? n_c : 1));
      sx.ov = (double*)malloc(sizeof(double) * (size_t)(n_c > 0 ? n_c : 1));
      for (int64_t t = 0; t < n_c; ++t) {
        const int64_t i = sx.ogid[t];
        sx.oa[t] = along[i];
        sx.ov[t] = local_coord(across[i], shift, origin, L, half_L);
      }
      int64_t cap_f = 64;
      double* fa = (double*)malloc(sizeof(double) * (size_t)cap_f);
      double* fv = (double*)malloc(sizeof(double) * (size_t)cap_f);
      int64_t* fg = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap_f);
      for (int32_t side = -1; side <= 1; side += 2) {
        const int32_t nk = (k + side + S) % S;
        for (int64_t t = start[nk]; t < start[nk + 1]; ++t) {
          const int64_t i = ids[t];
          const double v = local_coord(across[i], shift, origin, L, half_L);
          if (!(v >= -sigma && v <= h + sigma)) continue;
          if (sx.n_fr == cap_f) {
            cap_f *= 2;
            fa = (double*)realloc(fa, sizeof(double) * (size_t)cap_f);
            fv = (double*)realloc(fv, sizeof(double) * (size_t)cap_f);
            fg = (int64_t*)realloc(fg, sizeof(int64_t) * (size_t)cap_f);
          }
          fa[sx.n_fr] = along[i]; fv[sx.n_fr] = v; fg[sx.n_fr] = i; sx.n_fr++;
        }
      }
      sx.fa = fa; sx.fv = fv; sx.fgid = fg;
      sx.acc_delta = &acc_delta[k];
      sx.acc_cnt = &acc_cnt[(int64_t)k * ORC_CNT_NCOL];
      const int64_t n_m = n_c > 0 ? (p->chains_per_cell > 0 ? p->chains_per_cell : n_c) : 0;
      int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_m > 0 ? n_m : 1));
      make_start_list_(p, sweep, k, n_c, n_m, starts);
      for (int64_t c = 0; c < n_m; ++c) {
        /* the sign of chain c: the top bit of the first word of its
         * direction stream (set: against the axis) */
        stream_t ds;
        stream_init(&ds, p->seed, KIND_DIR, (uint64_t)sweep, cell_key(p, k), (uint64_t)c);
        const int sgn = (stream_next(&ds) >> 63) ? -1 : 1;
        stripe_chain(&sx, starts[c], p->ell, sgn);
      }
      for (int64_t t = 0; t < n_c; ++t) along[sx.ogid[t]] = sx.oa[t];
      total += sx.digest * (2ULL * (uint64_t)k + 1ULL);
      free(starts); free(fa); free(fv); free(fg); free(sx.oa); free(sx.ov); free(sx.u_i); free(sx.u_a);
    }
  }
  if (digest_out) *digest_out = total;
  free(stripe_of); free(start); free(ids);
}

int orc_run(const orc_params* p, double* x, double* y, int64_t sweep0, int64_t n_sweeps,
            double* acc_delta, uint64_t* acc_cnt, uint64_t* digests) {
  if (check_params(p) != 0) return -1;
  for (int64_t s = 0; s < n_sweeps; ++s) {
    uint64_t d = 0;
    if (p->cells == 1)
      sweep_periodic(p, x, y, sweep0 + s, acc_delta, acc_cnt, &d);
    else if (p->boundary == ORC_BOUNDARY_STRIPES)
      sweep_stripes(p, x, y, sweep0 + s, acc_delta, acc_cnt, &d);
    else
      sweep_cells(p, x, y, sweep0 + s, 4, NULL, 0, acc_delta, acc_cnt, &d, NULL);
    if (digests) digests[s] = d;
  }
  return 0;
}

int orc_run_cells(const orc_params* p, double* x, double* y, int64_t sweep, int32_t n_phases,
                  const int32_t* cells, int32_t n_cells, double* acc_delta, uint64_t* acc_cnt,
                  uint64_t* cell_digest) {
  if (check_params(p) != 0 || p->cells == 1 || p->boundary == ORC_BOUNDARY_STRIPES) return -1;
  if (n_phases < 1 || n_phases > 4) return -1;
  for (int32_t t = 0; t < n_cells; ++t) cell_digest[t] = 0;
  sweep_cells(p, x, y, sweep, n_phases, cells, n_cells, acc_delta, acc_cnt, NULL, cell_digest);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One walled cell on its own (for exact stationarity checks)               */
/* ------------------------------------------------------------------------ */
int orc_cell_chains(const orc_params* p, double w, int64_t n_own, double* ox, double* oy,
                    int64_t n_frozen, const double* fx, const double* fy, int64_t n_chains,
                    double* trace, double* acc_delta, uint64_t* acc_cnt) {
  if (!(w > 0.0) || n_own < 1 || n_frozen < 0 || n_chains < 0 || !(p->ell > 0.0) ||
      !(p->sigma > 0.0) || p->boundary > ORC_BOUNDARY_REJECT)
    return -1;
  int64_t* ogid = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_own);
  int64_t* hgid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_frozen > 0 ? n_frozen : 1));
  for (int64_t i = 0; i < n_own; ++i) ogid[i] = i;
  for (int64_t i = 0; i < n_frozen; ++i) hgid[i] = n_own + i;
  chain_ctx cx;
  memset(&cx, 0, sizeof cx);
  cx.periodic = 0;
  cx.n = n_own + n_frozen;
  cx.w = w;
  cx.sigma = p->sigma;
  cx.n_own = n_own; cx.ox = ox; cx.oy = oy; cx.ogid = ogid;
  cx.n_halo = n_frozen; cx.hx = fx; cx.hy = fy; cx.hgid = hgid;
  cx.cell = 0;
  cx.acc_delta = acc_delta;
  cx.acc_cnt = acc_cnt;
  cx.reject = p->boundary == ORC_BOUNDARY_REJECT;
  for (int64_t k = 0; k < n_chains; ++k) {
    /* chain k: start drawn with replacement and an isotropic direction, from
     * the streams of sweep k, cell 0, chain 0 */
    const int64_t a = orc_start_index(p, k, 0, 0, n_own);
    double dx, dy;
    orc_direction(p, k, 0, 0, &dx, &dy);
    run_chain(&cx, a, dx, dy, p->ell);
    if (trace)
      for (int64_t i = 0; i < n_own; ++i) {
        trace[(k * n_own + i) * 2] = ox[i];
        trace[(k * n_own + i) * 2 + 1] = oy[i];
      }
  }
  free(ogid); free(hgid); free(cx.u_a); free(cx.u_x); free(cx.u_y);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Smallest pair distance (overlap check)                                   */
/* ------------------------------------------------------------------------ */
double orc_min_pair_distance(int64_t n, double L, const double* x, const double* y, double r_cut,
                             int64_t* i_out, int64_t* j_out) {
  /* grid of g x g squares of side L/g >= r_cut: pairs closer than r_cut lie in
   * the same or neighbouring squares (minimum image) */
  int64_t g = (int64_t)floor(L / r_cut);
  if (g < 3) g = 1;
  if (g > 65536) g = 65536;
  const double side = L / (double)g, half = 0.5 * L;
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g * g));
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* sq = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t c = 0; c < g * g; ++c) head[c] = -1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = (int64_t)floor(x[i] / side), cy = (int64_t)floor(y[i] / side);
    cx = ((cx % g) + g) % g;
    cy = ((cy % g) + g) % g;
    sq[i] = cy * g + cx;
    next[i] = head[sq[i]];
    head[sq[i]] = i;
  }
  double best2 = INFINITY;
  int64_t bi = -1, bj = -1;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t cx = sq[i] % g, cy = sq[i] / g;
    const int64_t reach = g == 1 ? 0 : 1;
    for (int64_t oy = -reach; oy <= reach; ++oy)
      for (int64_t ox = -reach; ox <= reach; ++ox) {
        const int64_t c = (((cy + oy) % g + g) % g) * g + (((cx + ox) % g + g) % g);
        for (int64_t j = head[c]; j >= 0; j = next[j]) {
          if (j <= i) continue;
          double dx = x[j] - x[i], dy = y[j] - y[i];
          if (dx < -half) dx += L; else if (dx >= half) dx -= L;
          if (dy < -half) dy += L; else if (dy >= half) dy -= L;
          const double d2 = dx * dx + dy * dy;
          if (d2 < best2) { best2 = d2; bi = i; bj = j; }
        }
      }
  }
  free(head); free(next); free(sq);
  if (!(best2 < r_cut * r_cut)) { best2 = INFINITY; bi = -1; bj = -1; }
  if (i_out) *i_out = bi;
  if (j_out) *j_out = bj;
  return sqrt(best2);
}

/* ------------------------------------------------------------------------ */
/* Hexatic order parameter (Sec. 2, eq. Psi), cutoff neighbours               */
/* ------------------------------------------------------------------------ */
void orc_psi6_box(int64_t n, double L, const double* x, const double* y, double r_cut,
                  double* re, double* im, double* mean_nb, double* per_disk) {
  const double half = 0.5 * L, rc2 = r_cut * r_cut;
  double sre = 0.0, sim = 0.0, snb = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double kre = 0.0, kim = 0.0;
    int64_t nk = 0;
    for (int64_t l = 0; l < n; ++l) {
      if (l == k) continue;
      double dx = x[l] - x[k], dy = y[l] - y[k];
      if (dx < -half) dx += L; else if (dx >= half) dx -= L;
      if (dy < -half) dy += L; else if (dy >= half) dy -= L;
      const double r2 = dx * dx + dy * dy;
      if (!(r2 < rc2)) continue;
      /* exp(6 i phi) = ((dx + i dy) / r)^6 */
      const double phi = atan2(dy, dx);
      kre += cos(6.0 * phi);
      kim += sin(6.0 * phi);
      nk += 1;
    }
    if (nk > 0) { kre /= (double)nk; kim /= (double)nk; }
    if (per_disk) { per_disk[2 * k] = kre; per_disk[2 * k + 1] = kim; }
    sre += kre;
    sim += kim;
    snb += (double)nk;
  }
  if (re) *re = n > 0 ? sre / (double)n : 0.0;
  if (im) *im = n > 0 ? sim / (double)n : 0.0;
  if (mean_nb) *mean_nb = n > 0 ? snb / (double)n : 0.0;
}

void orc_psi6(const orc_params* p, const double* x, const double* y, double r_cut, double* re,
              double* im, double* mean_nb, double* per_disk) {
  orc_psi6_box(p->n, orc_box_length(p->n, p->sigma, p->eta), x, y, r_cut, re, im, mean_nb,
               per_disk);
}

/* ------------------------------------------------------------------------ */
/* Pair histogram (pressure route of eq. pressure)                          */
/* ------------------------------------------------------------------------ */
void orc_pair_histogram(const orc_params* p, const double* x, const double* y, double r_max,
                        int32_t n_bins, uint64_t* counts, uint64_t* overlaps) {
  const double L = orc_box_length(p->n, p->sigma, p->eta), half = 0.5 * L;
  const double delta = (r_max - p->sigma) / (double)n_bins;
  for (int64_t k = 0; k < p->n; ++k) {
    for (int64_t l = 0; l < p->n; ++l) {
      if (l == k) continue;
      double dx = x[l] - x[k], dy = y[l] - y[k];
      if (dx < -half) dx += L; else if (dx >= half) dx -= L;
      if (dy < -half) dy += L; else if (dy >= half) dy -= L;
      const double d2 = dx * dx + dy * dy;
      if (!(d2 < r_max * r_max)) continue;
      const double dist = sqrt(d2);
      if (dist < p->sigma) {
        if (overlaps) *overlaps += 1;
        continue;
      }
      const double t = floor((dist - p->sigma) / delta);
      if (t < (double)n_bins) counts[(int64_t)t] += 1;
    }
  }
}
