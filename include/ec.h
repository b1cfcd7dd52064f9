/*
 * ec.h -- C ABI of the MI355X (gfx950) parallel event-chain library for
 * two-dimensional hard disks.
 *
 * The method (Kampmann, Boltz, Kierfeld, "Parallelized event chain algorithm
 * for dense hard sphere and polymer systems"):
 *   - N hard disks of diameter sigma in a periodic L x L box, packing fraction
 *     eta = N pi sigma^2 / (4 L^2)                                  (Sec. 2);
 *   - straight event chains: a disk moves along d until it touches another,
 *     the remaining displacement passes to the hit disk, until a total of ell
 *     is used up                                                    (Sec. 3.2);
 *   - parallel sweep: the box is cut into C x C square simulation cells
 *     shifted by a random vector, grouped in 2 x 2 blocks; one random order
 *     of the four colours per sweep; in each cell n_m start disks are drawn
 *     WITH replacement and one chain is run from each while all other cells
 *     are frozen; chains reflect at cell walls and at frozen disks with equal
 *     angles of incidence and reflection                          (Sec. 3.4,
 *     Fig. 1, Fig. 2).
 *
 * Every call returns ec_status (EC_OK = 0).  No exception crosses the ABI.
 *
 * Memory: the caller allocates one device buffer of ec_workspace_bytes()
 * bytes, 256-byte aligned (for instance a torch uint8 tensor, whose device
 * allocations are), and keeps it alive until ec_destroy.  The library
 * allocates no device memory.  The host handle is created by ec_init_system
 * and freed by ec_destroy.  Host arrays passed to the get/set calls belong to
 * the caller.
 *
 * Streams: every device operation is enqueued on the stream given at init
 * (a hipStream_t passed as void*, NULL = the null stream), in call order.
 * Calls that return host data synchronise that stream.
 *
 * Threading: a handle may be used by one host thread at a time.
 *
 * Determinism: results are a pure function of the parameters, the seed and
 * the number of sweeps done; sweeps may be split over any number of calls.
 * Given the same inputs the device path reproduces the CPU reference bit for
 * bit (same event sequence, same positions).
 */
#ifndef EC_H
#define EC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EC_ABI_VERSION 1u

typedef enum {
  EC_OK = 0,
  EC_E_INVALID = 1,     /* invalid argument; nothing was changed            */
  EC_E_OVERLAP = 2,     /* positions given with two disks closer than sigma  */
  EC_E_HIP = 3,         /* a HIP runtime call failed (see ec_last_error)     */
  EC_E_NOMEM = 4,       /* workspace too small                               */
  EC_E_STATE = 5,       /* a device check failed in a sweep, or wrong handle */
  EC_E_UNSUPPORTED = 6  /* valid request that is not implemented             */
} ec_status;

typedef enum {
  EC_DIR_XY = 0,        /* +x for even chains, +y for odd ones; one periodic cell only (Sec. 3.2) */
  EC_DIR_ISOTROPIC = 1, /* uniform direction on the circle (required with C > 1)                 */
  EC_DIR_X = 2          /* +x only; one periodic cell only                                       */
} ec_dir_mode;

typedef enum {
  EC_PREC_FP64 = 0,        /* every candidate distance in FP64                               */
  EC_PREC_FP32_SCREEN = 1  /* FP32 screening with a guard band, FP64 for the survivors,
                              the winner and every commit; identical events to EC_PREC_FP64 */
} ec_precision;

typedef enum {
  EC_START_REPLACE = 0,  /* starts drawn with replacement: the correct rule (Sec. 3.4, Fig. 2) */
  EC_START_DISTINCT = 1  /* shuffled list of distinct disks: the rule shown to be incorrect
                            for n_m > 1 (Fig. 3); a negative control only                   */
} ec_start_mode;

/* ec_params.flags */
#define EC_FLAG_SCAN_SEARCH 1u  /* walled cells: search every staged disk for each event
                                   instead of the 8x8-bin window (same events, slower)     */
/* Schedule of the walled-cell sweep.  The results are identical either way
 * (same positions, digests and tallies); only the timing differs.
 *   one launch:    all four colour phases in one kernel launch, each cell
 *                  starting once its neighbours of earlier phases are done;
 *                  the default of a system swept alone.
 *   phase launches: one launch per colour phase, the launch boundary
 *                  separating the phases (Sec. 3.4 as written).
 * A batch runs from a device ready queue unless one of these bits selects
 * its initial schedule (EC_SCHEDULE_* below).  Setting both bits is
 * EC_E_INVALID; the systems of a batch share them. */
#define EC_FLAG_PHASE_LAUNCHES 2u
#define EC_FLAG_ONE_LAUNCH 4u
/* Rejection at the cell boundary (walled cells, FP64): a chain that would
 * take a centre across its cell's wall or hit a frozen disk is rejected and
 * every move it made is undone -- the variant Sec. 3.4 attributes to the
 * striped decomposition, instead of the paper's reflection.  Tallies: lifts
 * and the contact sum of accepted chains only; the wall and frozen counts
 * are the rejections they caused; chains counts all.  The EC pressure
 * estimator does not apply (use the pair-correlation route).  A chain may
 * make at most 256 lifts (device error bit 32 beyond).  The systems of a
 * batch share it. */
#define EC_FLAG_REJECT 8u
/* Debug: after every sweep, check every pair of disks in neighbouring cells
 * (all pairs for one periodic cell) for a distance below sigma (1 - 1e-12),
 * the bound rounding may reach on touching disks.  A pair found sets a device
 * error: the next synchronising call returns EC_E_OVERLAP, and ec_last_error
 * names the sweep, the number of such pairs and the first pair (the race and
 * overlap check of the method: disks of two cells run at once never
 * interpenetrate when the colour phases keep neighbouring cells apart,
 * Sec. 3.4 step 4).  Costs one pass over the neighbour pairs per sweep. */
#define EC_FLAG_CHECK_OVERLAP 16u
/* The striped decomposition with rejection, the variant Sec. 3.4 compares
 * against (the stripes of Fig. 3): cells_per_side stripes of width L/C > 2 sigma
 * span the box, horizontal on even sweeps with chains along x, vertical on
 * odd sweeps with chains along y, each with a random sign (dir_mode must be
 * EC_DIR_XY); a random
 * shift across the stripes and a random first colour per sweep; the two
 * colours run one after the other, one wavefront per stripe; a chain that
 * hits a disk of a neighbouring stripe is rejected and undone (at most 1024
 * moves per chain, device error bit 32 beyond).  Tallies as EC_FLAG_REJECT.
 * FP64, no EC_FLAG_REJECT (implied); a stripe's disks must fit one CU's LDS
 * (EC_E_UNSUPPORTED).  Sec. 4 explains why isotropic chains suit stripes
 * badly; this is a comparison variant, not the method. */
#define EC_FLAG_STRIPES 32u

typedef struct {
  uint32_t abi_version;     /* must equal EC_ABI_VERSION                                    */
  uint32_t flags;           /* EC_FLAG_* bits, 0 = default                                  */
  int64_t  n_disks;         /* N; disk i starts on site (i mod k, i div k) of the k x k
                               start lattice, k = ceil(sqrt N); walled cells (C > 1)
                               take N <= 2^29 - 4, one periodic cell N <= 2048
                               (EC_E_UNSUPPORTED above)                                  */
  double   sigma;           /* disk diameter, in [2^-300, 2^300]                            */
  double   eta;             /* 0 < eta < pi/(2 sqrt 3); L = sigma sqrt(N pi / (4 eta))       */
  double   ell;             /* displacement of one chain, > 0                               */
  int32_t  cells_per_side;  /* C: 1 = one periodic cell without walls; else even, >= 4,
                               and cell side L/C > sigma; a walled cell needs a side of at
                               least 3 sigma and its LDS (20 B per bin of side < 0.7 sigma
                               plus lists) within 160 KiB, about 54 sigma at most
                               (EC_E_UNSUPPORTED outside)                                   */
  int32_t  chains_per_cell; /* <= 0: n_m = number of disks in the cell; > 0: fixed n_m      */
  int32_t  dir_mode;        /* ec_dir_mode                                                  */
  int32_t  precision;       /* ec_precision                                                 */
  int32_t  start_mode;      /* ec_start_mode                                                */
  int32_t  cells_per_block; /* schedule only: simulation cells per workgroup (1, 2, 4);     
                               0 = 1 where a colour phase has no more cells than the
                               device has CUs, else 4 when four cells' LDS fits 160 KiB,
                               else 1                                                       */
  double   screen_margin;   /* relative guard band of EC_PREC_FP32_SCREEN, 0 = 1e-5         */
  uint64_t seed;            /* Philox4x64-10 key word                                       */
  uint32_t system;          /* index of the system inside a batch (second key-word part)    */
  uint32_t reserved;
} ec_params;

typedef struct ec_system_s* ec_system;

/* Bytes of device workspace a system with these parameters needs.
 * EC_E_INVALID for invalid parameters (see ec_init_system). */
ec_status ec_workspace_bytes(const ec_params* p, size_t* bytes);

/* Create a system: validates p, lays out the workspace, places the disks on
 * the k x k start lattice (odd rows shifted by half a spacing) and clears the
 * tallies.  dev_workspace: device pointer, 256-byte aligned, ws_bytes >=
 * ec_workspace_bytes().  hip_stream: hipStream_t (borrowed; NULL = null
 * stream).  Errors: EC_E_INVALID (bad parameters, or a workspace that is not
 * 256-byte aligned), EC_E_NOMEM (workspace too small), EC_E_HIP. */
ec_status ec_init_system(const ec_params* p, void* dev_workspace, size_t ws_bytes,
                         void* hip_stream, ec_system* out);

/* Enqueue n_sweeps PEC sweeps (Sec. 3.4 steps 1-7; with C = 1, N chains in
 * the one periodic box).  Asynchronous; advances the sweep counter. */
ec_status ec_sweep(ec_system sys, int64_t n_sweeps);

/* EC pressure over the sweeps since the last reset (the collision-statistics
 * route cited in Sec. 3.4, extended to frozen-disk contacts):
 *   z = beta P / rho = 1 + sum(contact projections) / (n_chains * ell),
 *   beta_p_sigma2 = z * N sigma^2 / L^2.
 * counts (may be NULL) receives 5 uint64: lifts, frozen-disk reflections,
 * wall reflections, chains, periodic free-flight caps.  Synchronises.
 * EC_E_STATE if a device check failed since init (cell or bin capacity, events
 * per chain, draw retries; ec_last_error names the first tripped chain). */
ec_status ec_measure_pressure(ec_system sys, double* z, double* beta_p_sigma2, uint64_t* counts);

/* Hexatic order parameter of the current positions, eq. (Psi) of Sec. 2:
 * Psi = N^-1 sum_k Psi_k, Psi_k = n_k^-1 sum_l exp(6 i phi_kl) with phi_kl the
 * angle of the bond k -> l against the x axis.  Neighbours are all disks
 * within r_cut (minimum image), not the Delaunay neighbours of the paper;
 * r_cut <= 0 selects 1.4 sigma, and r_cut may not exceed the cell side (half
 * the box with C = 1; EC_E_INVALID).  A disk without neighbours has Psi_k = 0.
 * per_disk (may be NULL): 2N doubles, re and im of each Psi_k in disk-id
 * order.  mean_neighbours (may be NULL): mean n_k.  Bond terms are summed per
 * disk in units of 2^-52 and the disks in a fixed order, so results repeat
 * bit for bit.  Synchronises. */
ec_status ec_measure_psi6(ec_system sys, double r_cut, double* psi_re, double* psi_im,
                          double* mean_neighbours, double* per_disk);

/* Psi with Delaunay neighbours, as eq. (Psi, Sec. 2) defines it: l is a
 * neighbour of k iff the bisector of k and l bounds k's Voronoi cell, found
 * on the device among the disks within r_search of k (<= 0: 4 L/sqrt(N), four
 * mean spacings, about 50 candidates at any density, capped at the cell side).  The result is exact when every Voronoi vertex lies
 * within r_search/2 of its disk, which is checked for every disk:
 * EC_E_UNSUPPORTED (with ec_last_error) if some cell is not certified (raise
 * r_search) or a disk has more than 128 candidates (lower it).  On a torus the
 * mean neighbour count is 6.  Outputs as for ec_measure_psi6, plus
 * neighbours[N] (may be NULL): each disk's count.  Configurations with four
 * or more cocircular disks have several triangulations; this returns one.
 * EC_E_INVALID if r_search exceeds the cell side (half the box for one
 * periodic cell).  Synchronises. */
ec_status ec_measure_psi6_delaunay(ec_system sys, double r_search, double* psi_re, double* psi_im,
                                   double* mean_neighbours, double* per_disk, int32_t* neighbours);

/* Autocorrelation of a time series of Psi (eq. tau, Sec. 2), host only:
 * c[dt] = Re(sum_t conj(Psi_t) Psi_(t+dt) / (n - dt)) / (sum_t |Psi_t|^2 / n)
 * for dt = 0..max_lag (c[0] = 1; the mean of Psi is taken as zero, its phase
 * being arbitrary), and tau (may be NULL) from the least-squares fit of
 * ln c[dt] = -dt / tau over dt = 1, 2, ... while c[dt] > e^-2 (NaN if
 * c[1] <= e^-2).  EC_E_INVALID for n < 2, max_lag outside [1, n), a zero
 * series or a NULL input. */
ec_status ec_psi_autocorrelation(const double* psi_re, const double* psi_im, int64_t n,
                                 int32_t max_lag, double* c, double* tau);

/* ---- Pressure from the pair correlation at contact, eq. (pressure) of Sec. 2:
 * beta P sigma^2 = sigma^2 rho (1 + (pi/2) sigma^2 rho g(sigma+)).  Ordered pairs
 * (k, l), k != l, are counted in bins [e_i, e_i+1), e_i = sigma + i delta,
 * delta = (r_max - sigma)/n_bins, by the minimum-image distance
 * d = sqrt(dx*dx + dy*dy), bin floor((d - sigma)/delta); integer counts, so the
 * result does not depend on summation order. */

/* Add the current configuration's pair counts to the system's histogram
 * (asynchronous).  sigma < r_max <= cell side (half the box with C = 1),
 * 1 <= n_bins <= 1024 (EC_E_INVALID).  A call with other r_max or n_bins than
 * the series so far starts a new series. */
ec_status ec_gr_accumulate(ec_system sys, double r_max, int32_t n_bins);

/* Counts of the series (counts[n_bins]), the number of configurations added
 * and the pairs closer than sigma (0 for a valid configuration).  Synchronises. */
ec_status ec_gr_counts(ec_system sys, uint64_t* counts, int64_t* samples, uint64_t* overlaps);

/* Clear the histogram (asynchronous). */
ec_status ec_gr_reset(ec_system sys);

/* Host only (no device call): g(R_i) = counts_i / (samples N rho pi (e_i+1^2 - e_i^2))
 * with rho = N / box^2, at R_i = 2 (e_i+1^3 - e_i^3) / (3 (e_i+1^2 - e_i^2)); the
 * contact value g(sigma+) from a least-squares quadratic in R - sigma over the
 * bins with R_i - sigma < fit_width (at least 3); z = beta P / rho =
 * 1 + (pi/2) sigma^2 rho g(sigma+).  g, R (n_bins each), g_contact, z may be NULL. */
ec_status ec_gr_normalize(int64_t n_disks, double box, double sigma, double r_max, int32_t n_bins,
                          const uint64_t* counts, int64_t samples, double fit_width, double* g,
                          double* R, double* g_contact, double* z);

/* Clear the pressure tallies (asynchronous). */
ec_status ec_reset_tallies(ec_system sys);

/* Copy positions to host arrays x[n], y[n] in disk-id order, coordinates in
 * [0, L).  n must equal N.  Synchronises. */
ec_status ec_get_positions(ec_system sys, double* x, double* y, int64_t n);

/* Replace all positions (host arrays in disk-id order, any real values; they
 * are wrapped into [0, L)).  EC_E_OVERLAP, with nothing changed, if two disks
 * are closer than sigma (periodic minimum image).  Synchronises. */
ec_status ec_set_positions(ec_system sys, const double* x, const double* y, int64_t n);

/* Event digests of the last n sweeps (oldest first; n <= min(sweeps done,
 * 1024)).  Synchronises. */
ec_status ec_get_digests(ec_system sys, uint64_t* out, int64_t n);

/* Per-cell accumulators in cell order (cell = cy*C + cx): delta[C*C] sums of
 * contact projections, counts[C*C*5] as in ec_measure_pressure.  Synchronises. */
ec_status ec_get_cell_tallies(ec_system sys, double* delta, uint64_t* counts);

/* Event digest of every cell (cell order) for the last sweep in which that
 * cell ran; the sweep digest is sum_c digest_c * (2c + 1) mod 2^64.
 * out[C*C].  Synchronises. */
ec_status ec_get_cell_digests(ec_system sys, uint64_t* out);

/* Sweeps done so far. */
ec_status ec_get_sweep_count(ec_system sys, int64_t* sweeps);

/* Timing of the simulation-cell kernels: with on != 0, every later ec_sweep
 * records HIP events on the system's stream around each launch of the
 * simulation-cell kernel (one per sweep by default, four with
 * EC_FLAG_PHASE_LAUNCHES, one for the periodic cell) and around the two
 * rebin kernels (cell of every disk, scatter by cell), without waiting for
 * them: the durations are read when the totals are asked for, or once 64
 * timed sweeps are pending (ec_sweep then synchronises).  Switching on or off
 * clears the totals.  Off by default. */
ec_status ec_set_timing(ec_system sys, int32_t on);
/* Summed simulation-cell kernel milliseconds and number of launches timed.
 * Synchronises. */
ec_status ec_get_timing(ec_system sys, double* phase_ms, int64_t* launches);
/* Summed milliseconds of the two rebin kernels (count: cell of every disk;
 * scatter: ids grouped by cell) over the timed sweeps of a walled system, and
 * the number of sweeps (0 for one periodic cell).  Synchronises. */
ec_status ec_get_rebin_timing(ec_system sys, double* count_ms, double* scatter_ms,
                              int64_t* sweeps);

/* One-launch sweep (walled cells, default schedule): upper limit of one
 * cell's wait for its neighbours of earlier phases, in seconds (default 60).
 * A wait that reaches it sets device error bit 16 and ends the sweep; the
 * next synchronising call reports EC_E_STATE and the system must be
 * initialised again.  0 fails every wait: a test of that error path.  Takes
 * effect from the next sweep.  EC_E_INVALID for a negative or non-finite
 * value; EC_E_STATE for a system of a batch. */
ec_status ec_set_dep_wait_limit(ec_system sys, double seconds);

/* Destroy the handle (does not free the caller's workspace).  Synchronises. */
ec_status ec_destroy(ec_system sys);

const char* ec_status_string(ec_status s);
/* Text of the last error on this handle ("" if none); valid until the next call. */
const char* ec_last_error(ec_system sys);

/* ---- Batched form -------------------------------------------------------
 * Several walled systems (C >= 4) advanced together: every step of a sweep
 * (rebin, draws, the simulation cells of Sec. 3.4) is one launch over all of
 * them, so small systems fill the GPU together.  The schedule (below, with
 * an optional HIP graph per sweep and the cells per workgroup) never changes
 * a trajectory: system i of a batch follows exactly the sweeps of a solo
 * system with the same parameters (its seed and `system` index key its
 * random streams).  Intended callers: ensembles of independent runs, such as
 * a density scan.
 *
 * Schedules of the simulation cells of a batch sweep:
 *   EC_SCHEDULE_READY_QUEUE (default): one persistent launch for every cell
 *     of every system; a cell is appended to a device queue as soon as its
 *     earlier-phase neighbours in its own system are done, and the resident
 *     wavefronts take the queue in order (no wavefront waits while holding a
 *     slot, no system waits for another's slowest cell);
 *   EC_SCHEDULE_ONE_LAUNCH: one launch, each system's cells in phase order
 *     with per-cell dependency waits (the single-system default);
 *   EC_SCHEDULE_PHASE_LAUNCHES: one launch per colour phase.
 * EC_FLAG_ONE_LAUNCH / EC_FLAG_PHASE_LAUNCHES in the parameters select the
 * initial schedule; ec_batch_set_schedule and ec_batch_autotune change it.
 */
#define EC_SCHEDULE_PHASE_LAUNCHES 0
#define EC_SCHEDULE_ONE_LAUNCH 1
#define EC_SCHEDULE_READY_QUEUE 2
typedef struct ec_batch_s* ec_batch;

/* Device bytes for a batch of n_sys systems ps[0..n_sys): their workspaces
 * plus a snapshot area of the same size used by ec_batch_autotune.
 * EC_E_INVALID / EC_E_UNSUPPORTED as ec_workspace_bytes, or for a periodic
 * system (C = 1), or n_sys outside [1, 4096]. */
ec_status ec_batch_workspace_bytes(const ec_params* ps, int32_t n_sys, size_t* bytes);

/* Create the batch in dev_workspace (caller-owned, 256-byte aligned (else
 * EC_E_INVALID), >= ec_batch_workspace_bytes) on hip_stream (borrowed).
 * Each system starts from its lattice as in ec_init_system;
 * ps[i].cells_per_block is ignored (the batch schedule applies, initially
 * 1).  Synchronises. */
ec_status ec_init_batch(const ec_params* ps, int32_t n_sys, void* dev_workspace, size_t ws_bytes,
                        void* hip_stream, ec_batch* out);

/* Enqueue n_sweeps sweeps of every system (asynchronous). */
ec_status ec_sweep_batch(ec_batch b, int64_t n_sweeps);

/* Handle of system i for the queries of a single system (positions,
 * pressure, digests, tallies, timing; ec_sweep advances that system alone).
 * Owned by the batch: ec_destroy on it returns EC_E_STATE. */
ec_status ec_batch_system(ec_batch b, int32_t i, ec_system* out);

/* With on != 0, the first later sweep is captured into a HIP graph (kernels
 * only) and every sweep replays it.  Needs a stream other than the null
 * stream (EC_E_UNSUPPORTED). */
ec_status ec_batch_set_graph(ec_batch b, int32_t on);

/* Simulation cells per workgroup in the phase launches: 1, 2 or 4
 * (EC_E_UNSUPPORTED if the LDS of that many cells exceeds 160 KiB). */
ec_status ec_batch_set_cells_per_block(ec_batch b, int32_t cells_per_block);

/* Schedule of the simulation cells (EC_SCHEDULE_*; EC_E_INVALID otherwise).
 * Synchronises. */
ec_status ec_batch_set_schedule(ec_batch b, int32_t schedule);

/* Time trial_sweeps sweeps for each schedule and each cells-per-workgroup
 * choice (1, 2, 4), each from a snapshot of the current state, keep the
 * fastest pair and put the state back (sweep counts included): the batch
 * continues as if no trial had run.  schedule_out and cpb_out (may be NULL)
 * receive the choice, ms_out[9] (may be NULL) the trial times, index
 * 3 * schedule + (0, 1, 2 for 1, 2, 4 cells), -1 where not allowed.
 * Synchronises. */
ec_status ec_batch_autotune(ec_batch b, int32_t trial_sweeps, int32_t* schedule_out,
                            int32_t* cpb_out, double* ms_out);

/* Text of the last batch-level error ("" if none). */
const char* ec_batch_last_error(ec_batch b);

/* Destroy the batch and its system handles (not the workspace).  Synchronises. */
ec_status ec_destroy_batch(ec_batch b);

/* ---- Sweeps without allocation -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * sweeps as ec_init_system + ec_sweep, with the positions in caller device
 * buffers and every other piece of state (cell lists, chain draws, tallies,
 * counters, the device record) in one static device buffer of the library,
 * 10 MiB per GPU, held until the process ends.
 *
 * x[n], y[n]: device arrays, disk-id order, coordinates in [0, L) of a
 * non-overlapping configuration (not checked; ec_set_positions's checks are
 * the caller's to make), advanced in place by sweeps first_sweep ..
 * first_sweep + n_sweeps - 1 of the system p describes (its seed keys the
 * random streams as in ec_init_system, whose first sweep is number 0).
 * digests (may be NULL): device uint64[n_sweeps], the per-sweep event digests
 * (n_sweeps <= 1024 then).  err (may be NULL): device int32, the device error
 * bits of ec_last_error's message (0 = none) after the last sweep.  Every
 * operation is enqueued on hip_stream (NULL = null stream); nothing is
 * allocated, copied to or from the host, or synchronised.
 *
 * Errors: EC_E_INVALID / EC_E_UNSUPPORTED as ec_init_system; EC_E_NOMEM if
 * the system exceeds the static buffer (N > 262144 disks, or more cells or
 * chains than 10 MiB holds); EC_E_HIP for a failed launch.  Every call on a
 * GPU uses that GPU's one buffer and clears it first: calls that overlap on
 * one GPU (other streams, other host threads) race and corrupt each other. */
ec_status ec_sweep_static(const ec_params* p, double* x, double* y, int64_t first_sweep,
                          int64_t n_sweeps, uint64_t* digests, int32_t* err, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
