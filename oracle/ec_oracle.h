/*
 * ec_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial FP64 reference of the parallel event-chain (PEC) sweep
 * for two-dimensional hard disks (Kampmann, Boltz, Kierfeld, "Parallelized
 * event chain algorithm for dense hard sphere and polymer systems", Sec. 3.2
 * and Sec. 3.4).  Only the test-suite, the package smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library; the two meet only through the written
 * arithmetic and random-number contract.
 *
 * Every event is found by brute force over all candidate disks, every sum is
 * taken in the order the events happen, and nothing is blocked or reordered.
 */
#ifndef EC_ORACLE_H
#define EC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DIR_XY = 0, ORC_DIR_ISO = 1, ORC_DIR_X = 2 };
enum { ORC_START_REPLACE = 0, ORC_START_DISTINCT = 1 };
/* What a chain does at a cell wall or a frozen disk (walled cells): reflect
 * with equal angles (Sec. 3.4, Fig. 1 right), or reject the whole chain,
 * the variant of Sec. 3.4 attributed to the striped decomposition.
 * ORC_BOUNDARY_STRIPES: the striped decomposition itself (Sec. 3.4, Fig. 3
 * "stripes"; Sec. 4): `cells` stripes spanning the box, chains along the
 * stripes (along x, either sign, in horizontal stripes on even sweeps; along
 * y in vertical stripes on odd sweeps; dir_mode must be ORC_DIR_XY), a chain
 * that hits a disk of a neighbouring stripe rejected and undone. */
enum { ORC_BOUNDARY_REFLECT = 0, ORC_BOUNDARY_REJECT = 1, ORC_BOUNDARY_STRIPES = 2 };

/* Event kinds, also used in the event digest. */
enum { ORC_EV_LIFT = 1, ORC_EV_FROZEN = 2, ORC_EV_WALL_X = 3, ORC_EV_WALL_Y = 4,
       ORC_EV_PSEUDO = 5, ORC_EV_END = 6 };

/* Per-cell accumulator columns (uint64) */
enum { ORC_CNT_LIFTS = 0, ORC_CNT_FROZEN = 1, ORC_CNT_WALLS = 2, ORC_CNT_CHAINS = 3,
       ORC_CNT_PSEUDO = 4, ORC_CNT_NCOL = 5 };

typedef struct {
  int64_t  n;               /* number of disks N                                 */
  double   sigma;           /* disk diameter                                     */
  double   eta;             /* packing fraction N*pi*sigma^2/(4 L^2)             */
  double   ell;             /* total displacement of one event chain             */
  int32_t  cells;           /* C: 1 = one periodic cell; else even and >= 4      */
  int32_t  chains_per_cell; /* <= 0: n_m = disks in the cell; > 0: fixed n_m      */
  int32_t  dir_mode;        /* ORC_DIR_*                                          */
  int32_t  start_mode;      /* ORC_START_*                                        */
  uint64_t seed;
  uint32_t system;          /* index of the system inside a batch (RNG key)      */
  uint32_t boundary;        /* ORC_BOUNDARY_* (walled cells)                      */
} orc_params;

/* Optional event log (small systems only). */
typedef struct {
  int64_t  chain;           /* running chain number within the call            */
  int32_t  cell;
  int32_t  kind;            /* ORC_EV_*                                          */
  int64_t  gid;             /* partner id; N, N+1 walls; N+2 pseudo; N+3 end   */
  int64_t  active;          /* id of the disk that moved in this segment        */
  double   s;               /* length of the segment                            */
  double   dx, dy;          /* direction during the segment                     */
  double   ax, ay;          /* moving disk after the segment (cell-local / box) */
  double   px, py;          /* partner disk (same frame), NaN for walls and ends */
} orc_event;

double   orc_box_length(int64_t n, double sigma, double eta);
void     orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void     orc_lattice(const orc_params* p, double* x, double* y);

/* Random draws of the contract, exposed for statistical pins. */
void     orc_sweep_draws(const orc_params* p, int64_t sweep, double* shift_x, double* shift_y,
                         int32_t perm[4]);
int64_t  orc_start_index(const orc_params* p, int64_t sweep, int32_t cell, int64_t chain, int64_t n_c);
void     orc_direction(const orc_params* p, int64_t sweep, int32_t cell, int64_t chain,
                       double* dx, double* dy);
/* Collision distance of a disk moving along unit d towards a disk at relative
 * position r; returns +inf when the two never touch. */
double   orc_collision_distance(double rx, double ry, double dx, double dy, double sigma);

/* Cell of every disk for a sweep (walled mode); cell index = cy*C + cx. */
int      orc_assign_cells(const orc_params* p, const double* x, const double* y, int64_t sweep,
                          int32_t* cell_of);

/*
 * Run sweeps sweep0 .. sweep0+n_sweeps-1 in place on x, y (disk-id order,
 * coordinates in [0, L)).  acc_delta[C*C] and acc_cnt[C*C*ORC_CNT_NCOL] are
 * per-cell accumulators that are added to; digests[n_sweeps] receives one
 * event digest per sweep (may be NULL).  Returns 0, or a negative code for
 * invalid parameters.
 */
int      orc_run(const orc_params* p, double* x, double* y, int64_t sweep0, int64_t n_sweeps,
                 double* acc_delta, uint64_t* acc_cnt, uint64_t* digests);

/*
 * Run only the cells listed in `cells` of sweep `sweep`, in the colour phase
 * each belongs to, for phases 0 .. n_phases-1 (cells of later phases are
 * skipped).  With n_phases == 1 and positions at the start of the sweep this
 * reproduces those cells exactly, because first-phase cells only see
 * positions from the start of the sweep.  cell_digest[n_cells] receives each
 * listed cell's digest (0 if skipped).
 */
int      orc_run_cells(const orc_params* p, double* x, double* y, int64_t sweep, int32_t n_phases,
                       const int32_t* cells, int32_t n_cells, double* acc_delta, uint64_t* acc_cnt,
                       uint64_t* cell_digest);

/*
 * Hexatic order parameter, eq. (Psi) of Sec. 2: Psi = N^-1 sum_k Psi_k with
 * Psi_k = n_k^-1 sum_l exp(6 i phi_kl), phi_kl the angle of the vector from k
 * to neighbour l against the x axis.  Neighbours: every other disk within
 * r_cut (minimum image in the L x L box of p), in place of the Delaunay
 * neighbours of the paper; a disk without neighbours has Psi_k = 0.  Brute
 * force over all pairs.  per_disk (may be NULL) receives re, im of each
 * Psi_k (2N doubles); mean_nb (may be NULL) the mean neighbour count.
 */
void     orc_psi6(const orc_params* p, const double* x, const double* y, double r_cut,
                  double* re, double* im, double* mean_nb, double* per_disk);
/* The same over positions in an explicit periodic box of side L. */
void     orc_psi6_box(int64_t n, double L, const double* x, const double* y, double r_cut,
                      double* re, double* im, double* mean_nb, double* per_disk);

/*
 * Pair histogram for the pressure route of eq. (pressure), Sec. 2: counts[i]
 * += number of ordered pairs (k, l), k != l, whose minimum-image distance d
 * (d^2 = dx*dx + dy*dy, d = sqrt(d^2)) lies in bin i = floor((d - sigma) /
 * delta), delta = (r_max - sigma) / n_bins, for 0 <= i < n_bins.  Pairs closer
 * than sigma are counted in *overlaps (may be NULL).  Brute force over all pairs.
 */
void     orc_pair_histogram(const orc_params* p, const double* x, const double* y, double r_max,
                            int32_t n_bins, uint64_t* counts, uint64_t* overlaps);

/* The start list of step 5 of the sweep for one cell: starts[k], k < n_m, is
 * the index (into the cell's id-ordered list of n_c disks) where chain k
 * starts; drawn with replacement, or from a shuffled list of distinct disks. */
void     orc_start_list(const orc_params* p, int64_t sweep, int32_t cell, int64_t n_c,
                        int64_t n_m, int64_t* starts);

/*
 * One walled square cell [0, w]^2 on its own: n_own movable disks (ox, oy,
 * updated in place; ids 0..n_own-1) and n_frozen frozen disks (fx, fy; ids
 * n_own..).  Chain k (k < n_chains) starts at a disk drawn with replacement
 * and runs along an isotropic direction (the streams of sweep k, cell 0,
 * chain 0 of the seed in p) for p->ell, reflecting or rejected at the walls
 * and frozen disks as p->boundary says -- the chains of one simulation cell
 * of Sec. 3.4.  trace (may be NULL) receives the movable positions after
 * every chain (n_chains * n_own * 2 doubles); acc_delta[1] and
 * acc_cnt[ORC_CNT_NCOL] are added to.  Returns 0, or -1 for bad arguments.
 */
int      orc_cell_chains(const orc_params* p, double w, int64_t n_own, double* ox, double* oy,
                         int64_t n_frozen, const double* fx, const double* fy, int64_t n_chains,
                         double* trace, double* acc_delta, uint64_t* acc_cnt);

/* Smallest pair distance (minimum image in a periodic L x L box) among the
 * pairs closer than r_cut, and that pair (i_out < j_out; -1 and +inf when no
 * pair is closer than r_cut).  A grid of squares of side >= r_cut. */
double   orc_min_pair_distance(int64_t n, double L, const double* x, const double* y, double r_cut,
                               int64_t* i_out, int64_t* j_out);

/*
 * Phase-parallel mode: the cells of one colour phase run on n OpenMP threads
 * (n <= 1: serial, the default).  Cells of one colour share nothing, each
 * cell's chains run in their own order, and the sweep digest is a sum over
 * cells, so every result is bit-identical to the serial run.  Ignored while
 * an event log is set.
 */
void     orc_set_threads(int32_t n);

/* Event log: set a buffer before orc_run; events beyond capacity are counted but dropped. */
void     orc_set_log(orc_event* buf, int64_t capacity);
int64_t  orc_log_count(void);

#ifdef __cplusplus
}
#endif
#endif
