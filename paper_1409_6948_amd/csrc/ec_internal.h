// Internal interface between the C ABI (ec_api.cpp) and the gfx950 kernels
// (ec_kernels.hip).  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ec {

// Per-sweep draws written by the prep kernel (shift of the cell grid and the
// order of the four colours, Sec. 3.4 steps 1 and 3).
struct SweepDraws {
  double sx, sy;
  int32_t perm;  // colour of phase q in bits 2q, 2q+1
  int32_t pad;
};

// Column order of the per-cell counters.
enum { CNT_LIFTS = 0, CNT_FROZEN = 1, CNT_WALLS = 2, CNT_CHAINS = 3, CNT_PSEUDO = 4, CNT_NCOL = 5 };

// Device error bits.  Any nonzero value also tells every running wave to stop.
enum {
  ERR_OWN_CAP = 1,     // a cell (own or neighbour) holds more disks than the packing bound
  ERR_BIN_CAP = 2,     // more than four centres in one LDS bin
  ERR_EVENT_CAP = 4,   // a chain exceeded kMaxEventsPerChain events
  ERR_DRAW_CAP = 8,    // a rejection draw exceeded kMaxDrawTries attempts
  ERR_DEP_WAIT = 16,   // a cell waited longer than dep_wait_ticks for a neighbour of an earlier phase
  ERR_UNDO_CAP = 32,   // rejection variant: a chain made more lifts than the undo log holds
  ERR_OVERLAP = 64,    // overlap check (debug flag): two disks closer than sigma after a sweep
  ERR_ABANDONED = 128  // ready-queue batch sweep: left unfinished after another system's error
};

// Ready queue of the batched sweep (one launch runs every cell of every
// system of a batch): header words, then per cell of the batch a task slot,
// its publication flag, and the count of earlier-phase neighbours not yet
// done.  Laid out by the batch in its workspace.
struct ReadyQueue {
  int32_t* hdr;        // [0] tasks claimed, [1] tasks reserved, [2] sweep epoch, [3] abort
  int64_t* tasks;      // [total] system << 32 | cell, in the order cells became ready
  int32_t* flags;      // [total] epoch of the sweep that published the slot
  int32_t* dep;        // [total] earlier-phase neighbours still running or waiting
  const int32_t* base; // [n_sys + 1] first queue index of each system's cells
  int32_t total;       // cells of all systems
  int32_t workers;     // wavefronts of the persistent launch
};
enum { QH_READ = 0, QH_RESERVE = 1, QH_EPOCH = 2, QH_ABORT = 3 };

// Events allowed in one chain before the sweep gives up with ERR_EVENT_CAP.
// Only degenerate input (a closed ring of touching disks, a disk pinned
// between two antipodal frozen contacts) comes near it; every wave then
// leaves its loops and the host reports the error.
constexpr int64_t kMaxEventsPerChain = int64_t(1) << 20;
// Events between two polls of the device error word.
constexpr int64_t kAbortPollEvents = 1024;
static_assert(kMaxEventsPerChain % kAbortPollEvents == 0, "the event cap is tested at polls");
// Attempts of one rejection draw (acceptance 0.785 for directions, > 1 - 2^-50
// for indices); reaching the cap sets ERR_DRAW_CAP.
constexpr int kMaxDrawTries = 256;
// Doubles in the debug snapshot written by the first wave that trips a cap.
constexpr int kDebugWords = 16;

constexpr int kDigestRing = 1024;
// Bins of the pair histogram (pressure route).
constexpr int kMaxGrBins = 1024;
// Events hashed together, one per lane, by the walled-cell kernel's digest
// (event ids then fit in 29 bits: N < 2^29 - 3).
constexpr int kDigestBatch = 64;
// regions of a cell: 3 x 3, r = 3 * ry + rx with rx, ry in {0: first strip,
// 1: middle, 2: last strip}
constexpr int kRegions = 9;
// Rejection variant: lifts of one chain that can be undone (LDS log entries).
constexpr int kUndoCap = 256;

// Everything a kernel needs: device pointers into the caller's workspace and
// the derived constants.  Passed by value.
struct Dev {
  double* x;                        // [N] positions, disk-id order
  double* y;
  int32_t* reg_count;               // [9*C*C] disks per (cell, region)
  int32_t* reg_fill;                // [9*C*C]
  int32_t* cell_start;              // [C*C+1] exclusive prefix sum over cells
  int32_t* reg_start;               // [9*C*C+1] exclusive prefix sum over (cell, region)
  int32_t* cell_of;                 // [N]
  uint8_t* reg_of;                  // [N] region of the disk in its cell (see k_count)
  int32_t* cell_ids;                // [N] ids grouped by cell, by region inside a cell
  double* acc_delta;                // [C*C]
  unsigned long long* acc_cnt;      // [C*C*CNT_NCOL]
  unsigned long long* digest_ring;  // [kDigestRing]
  unsigned long long* cell_digest;  // [C*C] digest of each cell in the last sweep it ran
  SweepDraws* draws;                // [1]
  int32_t* err;                     // [1]
  double* red;                      // [8]: reduced tallies (double sum + counters as bits)
  int32_t* chain_start;             // [max chains per sweep] start index within its cell
  double2* chain_dir;               // [max chains per sweep] direction of each chain
  int32_t* shuffle;                 // [N] per-cell shuffled lists (distinct-start mode)
  double* dbg;                      // [kDebugWords] state of the first wave that tripped a cap
  int64_t* sweep_ctr;               // [1] sweeps done; read by every kernel of a sweep
  double2* psi;                     // [N] per-disk hexatic order Psi_k (re, im)
  double* psi_part;                 // [3 * ceil(N/256)] per-block sums (re, im, neighbours)
  double* psi_red;                  // [3] Psi (re, im) and the mean neighbour count
  int32_t* psi_nb;                  // [N] Delaunay neighbour count of each disk
  unsigned long long* psi_err;      // [2] disks whose Voronoi cell was not certified; candidate overflows
  unsigned long long* gr_counts;    // [kMaxGrBins + 1] pair counts per bin, then pairs < sigma
  int32_t* queue;                   // [1] ticket counter of the one-launch sweep
  int64_t* cell_done;               // [C*C] last sweep + 1 whose write-back the cell has published
  unsigned long long* ovl;          // [4] overlap check: pairs found, first pair (i, j), its sweep

  int64_t n;
  double sigma, sig2, ell, L, half_L, w, cap, b, inv_b, margin;
  // width of the wall strips that split a cell into 3 x 3 regions: sigma plus
  // a margin far above the rounding of cell-local coordinates, so every disk a
  // neighbour stages as frozen lies in the strips that face it
  double strip;
  // FP32 screen (precision 1): error bounds of the FP32 contact terms against
  // the FP64 ones (a, sigma^2 - c^2, distance) and the threshold of
  // sigma^2 - c^2 above which the FP32 distance is within scr_e
  float scr_ea, scr_ed, scr_dg, scr_e;
  int32_t C, nb, gridb, cap_own, chains_per_cell, dir_mode, start_mode, precision;
  int32_t pbins;  // one periodic cell: bins per side of its bin grid, 0 = brute-force search
  int32_t lds_per_cell, cells_per_block;
  int32_t search;                   // 0: 8x8-bin window with guard; 1: scan of every slot
  int64_t dep_wait_ticks;           // one-launch sweep: limit of one wait, 100 MHz clock ticks
  int32_t reject;                   // 1: a chain reaching a wall or a frozen disk is undone
  int32_t check_overlap;            // 1: every sweep ends with a check of all neighbour pairs
  int32_t stripes;                  // 1: striped decomposition, C stripes of width w, rejection
  int32_t stripe_cap_own, stripe_cap_frozen, stripe_undo;  // LDS capacities of one stripe
  uint64_t seed;
  uint32_t system;
};

// LDS layout of one simulation cell in the walled-cell kernel: a grid of
// gridb x gridb square bins of side b < sigma/sqrt(2), one slot each (FP64
// position, 32-bit meta word: own index, or frozen id | top bit); the cell's
// id-ordered list and the slot of each own disk; one sink slot per lane (a
// target for the lanes that do not store when one or two lanes write).
struct CellLds {
  int32_t off_pos, off_meta, off_own_gid, off_own_loc, off_sink, off_undo, bytes;
};

// reject: an undo log of kUndoCap entries (slots and old position, 32 B each).
__host__ __device__ inline CellLds cell_lds_layout(int gridb, int cap_own, bool reject) {
  CellLds l;
  int slots = gridb * gridb;
  int o = 0;
  l.off_pos = o;      o += 16 * slots;
  l.off_meta = o;     o += 4 * slots;
  o = (o + 15) & ~15;
  l.off_own_gid = o;  o += 4 * cap_own;
  l.off_own_loc = o;  o += 4 * cap_own;
  o = (o + 15) & ~15;
  l.off_sink = o;     o += 16 * 64;
  l.off_undo = o;     o += reject ? 32 * kUndoCap : 0;
  l.bytes = (o + 15) & ~15;
  return l;
}

// LDS of the binned periodic cell: pbins x pbins slots (FP64 position, 32-bit
// disk id), the slot of every disk, the shuffled start list, one sink slot
// per lane.
struct PeriodicLds {
  int32_t off_pos, off_meta, off_slot_of, off_tmp, off_sink, bytes;
};
__host__ __device__ inline PeriodicLds periodic_lds_layout(int pbins, int n) {
  PeriodicLds l;
  const int slots = pbins * pbins;
  int o = 0;
  l.off_pos = o;      o += 16 * slots;
  l.off_meta = o;     o += 4 * slots;
  l.off_slot_of = o;  o += 4 * n;
  l.off_tmp = o;      o += 4 * n;
  o = (o + 15) & ~15;
  l.off_sink = o;     o += 16 * 64;
  l.bytes = o;
  return l;
}

// LDS of one stripe in the striped-decomposition kernel: own disks (position
// along and across the stripe, id, and a staging word), frozen disks
// (along, across, id), and the undo log (disk, old position along).
__host__ __device__ inline int stripe_lds_bytes(int cap_own, int cap_frozen, int undo) {
  return 24 * cap_own + 20 * cap_frozen + 16 * undo + 64;
}

// Largest N the one-periodic-cell kernel keeps in LDS.
constexpr int64_t kPeriodicMaxN = 2048;

// Extents of one launch over n_sys systems whose Dev records are in device
// memory (ds[0..n_sys)): maxima over the systems, and the shared schedule.
struct LaunchShape {
  int32_t n_sys;
  bool periodic;            // one periodic cell (single system only)
  bool any_distinct;        // some system uses the distinct-start control
  bool fp32_screen;         // the FP32-screened phase kernel (same for all)
  bool one_launch;          // all four phases in one launch (k_sweep_cells), else one per phase
  bool ready_queue;         // a batch: every cell of every system in one launch fed by a ready queue
  ReadyQueue queue;         // (ready_queue only)
  bool reject;              // rejection at the cell boundary (same for all)
  bool check_overlap;       // some system checks for overlaps after every sweep
  bool stripes;             // striped decomposition (same for all)
  int64_t max_n;            // disks
  int64_t max_chains;       // chains per sweep
  int32_t max_cells;        // C * C
  int32_t max_cells_side;   // C (stripes: the number of stripes)
  int32_t pbins;            // one periodic cell: bins per side (0: brute-force kernel)
  int32_t max_active;       // C * C / 4
  int32_t cpb;              // simulation cells per workgroup (same for all)
  int32_t max_lds_per_cell; // bytes
};

// Optional HIP events recorded around every phase launch (begin[q], end[q]);
// the one-launch sweep and the periodic cell use begin[0], end[0] only.
// rebin[0..1] bracket the count kernel, rebin[2..3] the scatter kernel
// (walled cells).
struct PhaseEvents {
  hipEvent_t begin[4], end[4];
  hipEvent_t rebin[4];
};

hipError_t launch_lattice(const Dev* ds, int64_t n, int64_t k, double a, hipStream_t st);
// One sweep of every system in ds: rebin, draws, four colour phases (or the
// periodic kernel), then the sweep counters advance.  Kernels only (no memset
// or copy), so the sequence can be captured in a HIP graph and replayed.
hipError_t launch_sweep(const Dev* ds, const LaunchShape& sh, hipStream_t st,
                        const PhaseEvents* ev = nullptr);
hipError_t launch_reduce(const Dev* ds, hipStream_t st);
// Allow the phase kernel up to `bytes` of dynamic LDS per workgroup.
hipError_t set_phase_lds_limit(int bytes);
// Wavefronts of the ready-queue launch that fit on the device at once with
// this much LDS per cell and cells per workgroup (resident workgroups per CU
// times CUs times cells per workgroup).
hipError_t ready_queue_workers(int lds_per_cell, int cpb, int fp32, int reject, int* workers);
hipError_t launch_zero_tallies(const Dev* ds, int32_t n_cells, hipStream_t st);
// Hexatic order parameter of one system (cutoff neighbours within r_cut,
// r_cut <= cell side): rebin of the current sweep, per-disk Psi_k, and a
// fixed-order reduction into psi_red.
// Cell lists of the current grid (sweep draws, count, offsets, scatter), for
// the observables of ec_observe.hip; one walled system.
hipError_t launch_rebin(const Dev* ds, const LaunchShape& sh, hipStream_t st);
hipError_t launch_psi6(const Dev* ds, const LaunchShape& sh, double r_cut, hipStream_t st);
// Add the current configuration's ordered-pair counts (bins of width delta =
// (r_max - sigma)/n_bins from sigma; r_max <= cell side) to gr_counts.
// Psi with Delaunay neighbours: candidates within r_search, Voronoi cells
// certified within r_search / 2.
hipError_t launch_psi6_delaunay(const Dev* ds, const LaunchShape& sh, double r_search, hipStream_t st);
hipError_t launch_gr(const Dev* ds, const LaunchShape& sh, double r_max, double delta, int n_bins,
                     hipStream_t st);
// Allocation-free sweeps (ec_sweep_static): bytes of the library's static
// device buffer (one per GPU) and the largest system it holds.
constexpr size_t kStaticScratchBytes = size_t(10) << 20;
constexpr int64_t kStaticMaxDisks = int64_t(1) << 18;
// Address of this GPU's static buffer (looked up once per device).
hipError_t static_scratch(void** ptr);
// Clear [base, base + bytes) with a kernel, then store rec at dst and the
// number of the first sweep in rec.sweep_ctr.
hipError_t launch_static_setup(const Dev& rec, Dev* dst, unsigned char* base, size_t bytes,
                               int64_t first_sweep, hipStream_t st);
// Digests of sweeps first .. first + n - 1 and the device error word into
// caller device buffers (either may be null).
hipError_t launch_static_copy_out(const Dev* ds, int64_t first, int64_t n,
                                  unsigned long long* digests, int32_t* err, hipStream_t st);

// Debug check after a sweep: every pair of disks in neighbouring cells of the
// sweep's grid (all pairs for one periodic cell) closer than sigma (1 - 1e-12)
// is counted in ovl and sets ERR_OVERLAP.  Systems without check_overlap skip it.
hipError_t launch_check_overlap(const Dev* ds, const LaunchShape& sh, hipStream_t st);

}  // namespace ec
