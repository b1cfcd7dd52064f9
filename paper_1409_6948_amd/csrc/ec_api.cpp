// C ABI of the gfx950 parallel event-chain library (declared in include/ec.h):
// parameter checks, workspace layout, launch order, host/device copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ec.h"
#include "ec_internal.h"

namespace {

// pi rounded to the nearest double
constexpr double kPi = 3.14159265358979323846;

struct Layout {
  size_t dev, sweep_ctr, x, y, cell_of, reg_of, cell_ids, reg_count, reg_fill, cell_start, reg_start,
      acc_delta, acc_cnt,
      ring, cell_digest, draws, err, red, chain_start, chain_dir, shuffle, dbg, psi, psi_part, psi_red,
      gr, queue, cell_done, psi_nb, psi_err, ovl, total;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// One-launch sweep: default limit of one dependency wait, 60 s of the 100 MHz
// device clock.
constexpr int64_t kDefaultDepWaitTicks = int64_t(60) * 100000000;

// sweep_only: no positions (the caller's) and no observables, for the
// allocation-free entry point whose state lives in the static scratch.
Layout make_layout(int64_t n, int32_t C, int32_t chains_per_cell, bool sweep_only = false) {
  Layout l;
  size_t o = 0;
  size_t nc = (size_t)C * (size_t)C;
  const size_t no = sweep_only ? 0 : (size_t)n;  // disks of the per-disk arrays left out
  size_t max_chains = chains_per_cell > 0 ? nc * (size_t)chains_per_cell : (size_t)n;
  if (C == 1) max_chains = 0;  // the periodic kernel draws its chains itself
  l.dev = o;        o = align256(o + sizeof(ec::Dev));
  l.sweep_ctr = o;  o = align256(o + 8);
  l.x = o;          o = align256(o + 8 * no);
  l.y = o;          o = align256(o + 8 * no);
  const size_t nr = (size_t)ec::kRegions * nc;
  l.cell_of = o;    o = align256(o + 4 * (size_t)n);
  l.reg_of = o;     o = align256(o + (size_t)n);
  l.cell_ids = o;   o = align256(o + 4 * (size_t)n);
  l.reg_count = o;  o = align256(o + 4 * nr);
  l.reg_fill = o;   o = align256(o + 4 * nr);
  l.cell_start = o; o = align256(o + 4 * (nc + 1));
  l.reg_start = o;  o = align256(o + 4 * (nr + 1));
  l.acc_delta = o;  o = align256(o + 8 * nc);
  l.acc_cnt = o;    o = align256(o + 8 * ec::CNT_NCOL * nc);
  l.ring = o;       o = align256(o + 8 * (size_t)ec::kDigestRing);
  l.cell_digest = o; o = align256(o + 8 * nc);
  l.draws = o;      o = align256(o + sizeof(ec::SweepDraws));
  l.err = o;        o = align256(o + 8);
  l.red = o;        o = align256(o + 64);
  l.chain_start = o; o = align256(o + 4 * max_chains);
  l.chain_dir = o;  o = align256(o + 16 * max_chains);
  l.shuffle = o;    o = align256(o + (C == 1 ? 0 : 4 * (size_t)n));
  l.dbg = o;        o = align256(o + 8 * ec::kDebugWords);
  l.psi = o;        o = align256(o + 16 * no);
  l.psi_part = o;   o = align256(o + 24 * ((no + 255) / 256));
  l.psi_red = o;    o = align256(o + (sweep_only ? 0 : 32));
  l.gr = o;         o = align256(o + (sweep_only ? 0 : 8 * (size_t)(ec::kMaxGrBins + 1)));
  l.queue = o;      o = align256(o + 8);
  l.cell_done = o;  o = align256(o + 8 * nc);
  l.psi_nb = o;     o = align256(o + 4 * no);
  l.psi_err = o;    o = align256(o + (sweep_only ? 0 : 16));
  l.ovl = o;        o = align256(o + 32);
  l.total = o;
  return l;
}

struct Derived {
  double L, w;
  int32_t nb, cap_own, cpb, lds_per_cell;
  int32_t pbins;  // one periodic cell: bins per side of its grid, 0 = brute force
  int32_t stripe_cap_own, stripe_cap_frozen, stripe_undo;  // striped decomposition only
};

// Oler's bound for a rectangle a x b: at most (2/sqrt 3) A/s^2 + P/(2s) + 1
// points with mutual distance >= s.
int32_t rect_capacity(double a, double b, double sigma) {
  const double u = a / sigma + 1e-6, v = b / sigma + 1e-6;
  const double bound = (2.0 / std::sqrt(3.0)) * u * v + (u + v) + 1.0;
  return ((int32_t)std::ceil(bound) + 63) & ~63;
}
// Lifts of one chain the striped kernel can undo.
constexpr int32_t kStripeUndo = 1024;

// Oler's bound: at most (2/sqrt 3) A/s^2 + P/(2s) + 1 points with mutual
// distance >= s fit in a convex region of area A and perimeter P.
int32_t own_capacity(double w, double sigma) {
  double u = w / sigma + 1e-6;
  double bound = (2.0 / std::sqrt(3.0)) * u * u + 2.0 * u + 1.0;
  int32_t cap = (int32_t)std::ceil(bound);
  return (cap + 63) & ~63;
}

ec_status validate(const ec_params* p, Derived* out, std::string* why) {
  *out = Derived{};
  if (!p) { *why = "null parameters"; return EC_E_INVALID; }
  if (p->abi_version != EC_ABI_VERSION) { *why = "abi_version mismatch"; return EC_E_INVALID; }
  if (p->n_disks < 1 || p->n_disks > 0x7FFFFFF0LL) { *why = "n_disks out of range"; return EC_E_INVALID; }
  if (!(p->sigma >= 0x1p-300) || !(p->sigma <= 0x1p300)) {
    *why = "sigma must be in [2^-300, 2^300]"; return EC_E_INVALID;
  }
  if ((p->flags & EC_FLAG_REJECT) &&
      (p->cells_per_side == 1 || p->precision != EC_PREC_FP64)) {
    *why = "EC_FLAG_REJECT needs walled cells and FP64"; return EC_E_UNSUPPORTED;
  }
  if ((p->flags & EC_FLAG_STRIPES) &&
      (p->cells_per_side == 1 || p->precision != EC_PREC_FP64 || (p->flags & EC_FLAG_REJECT))) {
    *why = "EC_FLAG_STRIPES needs C >= 4 stripes and FP64 (it implies rejection)";
    return EC_E_UNSUPPORTED;
  }
  if ((p->flags & EC_FLAG_PHASE_LAUNCHES) && (p->flags & EC_FLAG_ONE_LAUNCH)) {
    *why = "EC_FLAG_PHASE_LAUNCHES and EC_FLAG_ONE_LAUNCH exclude each other"; return EC_E_INVALID;
  }
  if (!(p->eta > 0.0) || !(p->eta < kPi / (2.0 * std::sqrt(3.0)))) {
    *why = "eta must lie in (0, pi/(2 sqrt 3))"; return EC_E_INVALID;
  }
  if (!(p->ell > 0.0) || !std::isfinite(p->ell)) { *why = "ell must be > 0"; return EC_E_INVALID; }
  if (p->dir_mode < 0 || p->dir_mode > 2) { *why = "bad dir_mode"; return EC_E_INVALID; }
  if (p->start_mode < 0 || p->start_mode > 1) { *why = "bad start_mode"; return EC_E_INVALID; }
  if (p->precision < 0 || p->precision > 1) { *why = "bad precision"; return EC_E_INVALID; }
  const int32_t C = p->cells_per_side;
  double L = p->sigma * std::sqrt((double)p->n_disks * kPi / (4.0 * p->eta));
  out->L = L;
  if (C == 1) {
    if (!(L > 2.0 * p->sigma)) { *why = "one periodic cell needs L > 2 sigma"; return EC_E_INVALID; }
    if (p->n_disks > ec::kPeriodicMaxN) {
      *why = "one periodic cell supports at most 2048 disks"; return EC_E_UNSUPPORTED;
    }
    out->w = L; out->nb = 0; out->cap_own = 0; out->cpb = 1; out->lds_per_cell = 0;
    // The bin grid of the periodic cell: bins below 0.7 sigma (one centre
    // each), at least 12 per side (the 8 x 8 window never meets itself), the
    // window's reach 5b - sigma below the free-flight cap L/2 - sigma (a window
    // event is then never a pseudo event), and the grid within 160 KiB of LDS;
    // otherwise the brute-force search.
    {
      const double pb_side = 0.7 * p->sigma;
      const double nbd = std::floor(L / pb_side) + 1.0;
      const int32_t pb = nbd < 1000.0 ? (int32_t)nbd : 1000;
      const double b = L / (double)pb;
      const bool fits = pb >= 12 && pb <= 100 && b < pb_side && 2.0 * b > p->sigma &&
                        5.0 * b < 0.5 * L &&
                        ec::periodic_lds_layout(pb, (int)p->n_disks).bytes <= 160 * 1024;
      out->pbins = fits ? pb : 0;
    }
  } else if (p->flags & EC_FLAG_STRIPES) {
    if (C < 4 || (C & 1)) { *why = "the number of stripes must be even and >= 4"; return EC_E_INVALID; }
    if (p->dir_mode != EC_DIR_XY) {
      *why = "stripes need chains along them (dir_mode EC_DIR_XY)"; return EC_E_INVALID;
    }
    const double w = L / (double)C;
    if (!(w > 2.0 * p->sigma)) { *why = "stripe width must exceed 2 sigma"; return EC_E_INVALID; }
    if (p->n_disks > (int64_t(1) << 29) - 4) {
      *why = "at most 2^29 - 4 disks"; return EC_E_UNSUPPORTED;
    }
    out->w = w;
    out->nb = 0;
    out->cap_own = 0;
    out->cpb = 1;
    out->stripe_cap_own = rect_capacity(L, w, p->sigma);
    out->stripe_cap_frozen = 2 * rect_capacity(L, p->sigma, p->sigma);
    out->stripe_undo = kStripeUndo;
    out->lds_per_cell = ec::stripe_lds_bytes(out->stripe_cap_own, out->stripe_cap_frozen, kStripeUndo);
    if (out->lds_per_cell > 160 * 1024) {
      *why = "a stripe's disks exceed the LDS of one CU (fewer disks or more stripes)";
      return EC_E_UNSUPPORTED;
    }
  } else {
    if (C < 4 || (C & 1)) { *why = "cells_per_side must be 1 or even and >= 4"; return EC_E_INVALID; }
    if (p->dir_mode != EC_DIR_ISOTROPIC) {
      *why = "walled cells need isotropic directions"; return EC_E_INVALID;
    }
    double w = L / (double)C;
    if (!(w > p->sigma)) { *why = "cell side must exceed sigma"; return EC_E_INVALID; }
    if (std::floor(w / p->sigma) < 3) {
      *why = "cell side below 3 sigma is not supported"; return EC_E_UNSUPPORTED;
    }
    // nb x nb bins of side b = w / nb < 0.7 sigma (< sigma / sqrt 2, so a bin
    // holds at most one centre) and, as w >= 3 sigma, b > 0.56 sigma (two
    // rings of bins outside the cell hold the sigma-wide frozen band)
    const int32_t nb = (int32_t)std::floor(w / (0.7 * p->sigma)) + 1;
    const double b = w / (double)nb;
    if (!(b < 0.7 * p->sigma) || !(2.0 * b > p->sigma)) {
      *why = "internal: bin side out of range"; return EC_E_UNSUPPORTED;
    }
    if (p->n_disks > (int64_t(1) << 29) - 4) {
      *why = "walled cells support at most 2^29 - 4 disks"; return EC_E_UNSUPPORTED;
    }
    if (nb + 4 > 100) {  // the kernel's slot-to-bin division is exact up to here (the
                         // LDS limit below is met first: about 87 bins per side)
      *why = "internal: more than 100 bins per side"; return EC_E_UNSUPPORTED;
    }
    out->w = w;
    out->nb = nb;
    out->cap_own = own_capacity(w, p->sigma);
    out->lds_per_cell =
        ec::cell_lds_layout(nb + 4, out->cap_own, (p->flags & EC_FLAG_REJECT) != 0).bytes;
    if (4 * out->cap_own > 16 * (nb + 4) * (nb + 4)) {  // the staging ids live in the slots
      *why = "internal: staging buffer"; return EC_E_UNSUPPORTED;
    }
    // Default: four cells (four waves) per workgroup when their LDS fits one CU.
    // The waves of one workgroup go to the four SIMDs of one CU; one-wave
    // workgroups leave the SIMD choice to the dispatcher, which has been
    // measured to put two waves on one SIMD for part of a launch (both then
    // run about 25 % slower while another SIMD idles).
    int32_t cpb = p->cells_per_block;
    if (cpb == 0) cpb = (size_t)4 * out->lds_per_cell <= 160 * 1024 ? 4 : 1;
    if (cpb != 1 && cpb != 2 && cpb != 4) { *why = "cells_per_block must be 0, 1, 2 or 4"; return EC_E_INVALID; }
    out->cpb = cpb;
    if ((size_t)cpb * out->lds_per_cell > 160 * 1024) {
      *why = "LDS per workgroup exceeds 160 KiB"; return EC_E_UNSUPPORTED;
    }
  }
  if (p->precision == EC_PREC_FP32_SCREEN && C == 1) {
    *why = "FP32 screening is built for walled cells"; return EC_E_UNSUPPORTED;
  }
  if (!(p->screen_margin >= 0.0) || p->screen_margin > 1e-2) {
    *why = "screen_margin must be in [0, 1e-2]"; return EC_E_INVALID;
  }
  // lattice start: k = ceil(sqrt(N)) columns, spacing L/k must exceed sigma
  int64_t k = (int64_t)std::ceil(std::sqrt((double)p->n_disks));
  while (k * k < p->n_disks) ++k;
  if (!(L / (double)k > p->sigma)) { *why = "start lattice spacing below sigma"; return EC_E_INVALID; }
  return EC_OK;
}

}  // namespace

struct ec_system_s {
  ec_params p;
  Derived dv;
  Layout lay;
  ec::Dev dev;           // host copy of the record kernels read from dev_d
  ec::Dev* dev_d;        // device copy (in the workspace)
  ec::LaunchShape shape; // this system alone
  bool in_batch;         // owned by a batch (ec_destroy refuses it)
  hipStream_t stream;
  int64_t sweeps;
  std::string last_error;
  // optional kernel timing: a pool of event sets, one per sweep, read when
  // the pool is full or the totals are asked for
  bool timing;
  std::vector<ec::PhaseEvents> ev;
  int pending;
  double phase_ms, count_ms, scatter_ms;
  int64_t phase_launches, rebin_launches;
  // pair histogram series (pressure route)
  double gr_rmax;
  int32_t gr_bins;
  int64_t gr_samples;
};

namespace {

ec_status hip_fail(ec_system s, hipError_t e, const char* what) {
  if (s) {
    s->last_error = std::string(what) + ": " + hipGetErrorString(e);
  }
  return EC_E_HIP;
}

#define EC_HIP(sys, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(sys, e_, #call); \
  } while (0)

}  // namespace

extern "C" {

const char* ec_status_string(ec_status s) {
  switch (s) {
    case EC_OK: return "ok";
    case EC_E_INVALID: return "invalid argument";
    case EC_E_OVERLAP: return "overlapping disks";
    case EC_E_HIP: return "HIP runtime error";
    case EC_E_NOMEM: return "workspace too small";
    case EC_E_STATE: return "device capacity check failed";
    case EC_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* ec_last_error(ec_system sys) { return sys ? sys->last_error.c_str() : ""; }

ec_status ec_workspace_bytes(const ec_params* p, size_t* bytes) {
  Derived dv;
  std::string why;
  ec_status st = validate(p, &dv, &why);
  if (st != EC_OK) return st;
  if (!bytes) return EC_E_INVALID;
  *bytes = make_layout(p->n_disks, p->cells_per_side, p->chains_per_cell).total;
  return EC_OK;
}

}  // extern "C"

namespace {

// Largest dynamic LDS the phase kernel may request (MI355X: 160 KiB per CU);
// set once, outside any stream capture.
hipError_t prepare_kernels() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = ec::set_phase_lds_limit(160 * 1024);
  if (e == hipSuccess) done = true;
  return e;
}

ec::LaunchShape shape_of(const ec::Dev& d, const ec_params& p) {
  ec::LaunchShape sh;
  sh.n_sys = 1;
  sh.periodic = d.C == 1;
  sh.any_distinct = d.start_mode == 1;
  sh.fp32_screen = d.precision == EC_PREC_FP32_SCREEN;
  sh.max_n = d.n;
  sh.max_chains = d.chains_per_cell > 0 ? (int64_t)d.C * d.C * d.chains_per_cell : d.n;
  sh.max_cells = d.C * d.C;
  sh.max_cells_side = d.C;
  sh.pbins = d.C == 1 ? d.pbins : 0;
  sh.max_active = (d.C / 2) * (d.C / 2);
  sh.cpb = d.cells_per_block;
  sh.max_lds_per_cell = d.lds_per_cell;
  sh.one_launch = d.C > 1 && !(p.flags & EC_FLAG_PHASE_LAUNCHES);  // a system swept alone
  sh.reject = d.reject != 0;
  sh.check_overlap = d.check_overlap != 0;
  sh.stripes = d.stripes != 0;
  if (sh.stripes) sh.one_launch = false;
  return sh;
}

// Error bounds of the FP32 screen.  With u = 2^-24, coordinates of staged
// disks bounded by X = w + 2 sigma and window offsets by R = 9b (an 8 x 8-bin
// window reaches at most 6 bins along each axis from the moving disk), the FP32
// offsets are within u (2X + R) of the exact ones, so a = r.d and c = r x d
// are within Ea = u (4X + 8R) (also covering the FP64 values), sigma^2 - c^2
// within Ed = 2 (sigma + Ea) Ea + 4 u sigma^2, and where the FP32
// sigma^2 - c^2 exceeds Dg = sigma^2 / 64 its square root is within
// Ed / sqrt(Dg - Ed) + 2 u sigma.  Each bound is doubled; the caller's
// relative margin (times sigma) is added to the distance bound.
void screen_bounds(ec::Dev* d) {
  const double u = std::ldexp(1.0, -24);
  const double sg = d->sigma, X = d->w + 2.0 * sg, R = 9.0 * d->b;
  const double ea = 2.0 * u * (4.0 * X + 8.0 * R);
  const double ed = 2.0 * (2.0 * (sg + ea) * ea + 4.0 * u * sg * sg);
  const double dg = sg * sg / 64.0;
  const double es = 2.0 * (ed / std::sqrt(dg - ed) + 2.0 * u * sg);
  const double e = ea + es + 4.0 * u * (R + sg) + d->margin * sg;
  d->scr_ea = (float)ea;
  d->scr_ed = (float)ed;
  d->scr_dg = (float)dg;
  d->scr_e = (float)e;
}

// The device record of a system whose workspace region starts at b.
void fill_record(ec::Dev* out, const ec_params* p, const Derived& dv, unsigned char* b,
                 const Layout& lay) {
  ec::Dev& d = *out;
  std::memset(&d, 0, sizeof d);
  d.x = (double*)(b + lay.x);
  d.y = (double*)(b + lay.y);
  d.cell_of = (int32_t*)(b + lay.cell_of);
  d.cell_ids = (int32_t*)(b + lay.cell_ids);
  d.reg_count = (int32_t*)(b + lay.reg_count);
  d.reg_fill = (int32_t*)(b + lay.reg_fill);
  d.reg_start = (int32_t*)(b + lay.reg_start);
  d.reg_of = (uint8_t*)(b + lay.reg_of);
  d.cell_start = (int32_t*)(b + lay.cell_start);
  d.acc_delta = (double*)(b + lay.acc_delta);
  d.acc_cnt = (unsigned long long*)(b + lay.acc_cnt);
  d.digest_ring = (unsigned long long*)(b + lay.ring);
  d.cell_digest = (unsigned long long*)(b + lay.cell_digest);
  d.draws = (ec::SweepDraws*)(b + lay.draws);
  d.err = (int32_t*)(b + lay.err);
  d.red = (double*)(b + lay.red);
  d.chain_start = (int32_t*)(b + lay.chain_start);
  d.chain_dir = (double2*)(b + lay.chain_dir);
  d.shuffle = (int32_t*)(b + lay.shuffle);
  d.dbg = (double*)(b + lay.dbg);
  d.sweep_ctr = (int64_t*)(b + lay.sweep_ctr);
  d.psi = (double2*)(b + lay.psi);
  d.psi_part = (double*)(b + lay.psi_part);
  d.psi_red = (double*)(b + lay.psi_red);
  d.gr_counts = (unsigned long long*)(b + lay.gr);
  d.queue = (int32_t*)(b + lay.queue);
  d.cell_done = (int64_t*)(b + lay.cell_done);
  d.psi_nb = (int32_t*)(b + lay.psi_nb);
  d.psi_err = (unsigned long long*)(b + lay.psi_err);
  d.ovl = (unsigned long long*)(b + lay.ovl);
  d.check_overlap = (p->flags & EC_FLAG_CHECK_OVERLAP) ? 1 : 0;
  d.stripes = (p->flags & EC_FLAG_STRIPES) ? 1 : 0;
  d.stripe_cap_own = dv.stripe_cap_own;
  d.stripe_cap_frozen = dv.stripe_cap_frozen;
  d.stripe_undo = dv.stripe_undo;
  d.dep_wait_ticks = kDefaultDepWaitTicks;
  d.reject = (p->flags & EC_FLAG_REJECT) ? 1 : 0;
  d.search = (p->flags & EC_FLAG_SCAN_SEARCH) ? 1 : 0;
  d.n = p->n_disks;
  d.sigma = p->sigma;
  d.sig2 = p->sigma * p->sigma;
  d.ell = p->ell;
  d.L = dv.L;
  d.half_L = 0.5 * dv.L;
  d.w = dv.w;
  d.cap = 0.5 * dv.L - p->sigma;
  d.C = p->cells_per_side;
  d.nb = dv.nb;
  d.gridb = dv.nb + 4;  // own bins 2..nb+1, two rings of frozen-band bins around them
  d.pbins = dv.pbins;
  d.b = dv.nb > 0 ? dv.w / (double)dv.nb : 0.0;
  d.inv_b = dv.nb > 0 ? 1.0 / d.b : 0.0;
  // the cell's wall strips: sigma plus 1e-9 L, far above the few ulps of L by
  // which two cells' local coordinates of one disk can disagree (w >= 3 sigma
  // keeps the strips apart)
  d.strip = p->sigma + 1e-9 * dv.L;
  d.margin = p->screen_margin > 0.0 ? p->screen_margin : 1e-5;  // relative to sigma
  d.cap_own = dv.cap_own;
  d.chains_per_cell = p->chains_per_cell;
  d.dir_mode = p->dir_mode;
  d.start_mode = p->start_mode;
  d.precision = p->precision;
  if (p->precision == EC_PREC_FP32_SCREEN) screen_bounds(&d);
  d.lds_per_cell = dv.lds_per_cell;
  d.cells_per_block = dv.cpb;
  d.seed = p->seed;
  d.system = p->system;
}

// Default cells per workgroup of a system swept alone, on the current device:
// where a colour phase has no more cells than the device has CUs, one cell
// per workgroup, so that each wavefront has a CU of its own (measured about
// 2 % faster at 64 cells per phase than four wavefronts sharing a CU); else
// the choice of validate().  An explicit cells_per_block is kept.
static void default_cells_per_block(const ec_params* p, Derived* dv) {
  if (p->cells_per_block != 0 || p->cells_per_side <= 1 || (p->flags & EC_FLAG_STRIPES)) return;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return;
  const int64_t half = p->cells_per_side / 2;
  if (half * half <= (int64_t)n_cu) dv->cpb = 1;
}

// Create a system in a workspace region (validated parameters); with a
// batch owner the handle is a view that the batch destroys.
ec_status init_system_at(const ec_params* p, const Derived& dv, unsigned char* b, size_t ws_bytes,
                         hipStream_t stream, bool in_batch, ec_system* out) {
  Layout lay = make_layout(p->n_disks, p->cells_per_side, p->chains_per_cell);
  if (ws_bytes < lay.total) return EC_E_NOMEM;
  ec_system s = new (std::nothrow) ec_system_s();
  if (!s) return EC_E_NOMEM;
  s->p = *p;
  s->dv = dv;
  if (!in_batch) default_cells_per_block(p, &s->dv);
  s->lay = lay;
  s->stream = stream;
  s->in_batch = in_batch;
  s->sweeps = 0;
  s->timing = false;
  s->pending = 0;
  s->phase_ms = s->count_ms = s->scatter_ms = 0.0;
  s->phase_launches = s->rebin_launches = 0;
  s->gr_rmax = 0.0;
  s->gr_bins = 0;
  s->gr_samples = 0;
  fill_record(&s->dev, p, s->dv, b, lay);
  ec::Dev& d = s->dev;
  s->dev_d = (ec::Dev*)(b + lay.dev);
  s->shape = shape_of(d, *p);

  int64_t k = (int64_t)std::ceil(std::sqrt((double)p->n_disks));
  while (k * k < p->n_disks) ++k;
  double a = dv.L / (double)k;
  hipError_t e = prepare_kernels();
  if (e == hipSuccess) e = hipMemcpyAsync(s->dev_d, &s->dev, sizeof(ec::Dev), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.sweep_ctr, 0, 8, stream);
  if (e == hipSuccess) e = ec::launch_lattice(s->dev_d, d.n, k, a, stream);
  if (e == hipSuccess) e = ec::launch_zero_tallies(s->dev_d, d.C * d.C, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.err, 0, 8, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.dbg, 0, 8 * ec::kDebugWords, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.digest_ring, 0, 8 * ec::kDigestRing, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.cell_digest, 0, 8 * (size_t)d.C * (size_t)d.C, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.cell_done, 0, 8 * (size_t)d.C * (size_t)d.C, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.queue, 0, 8, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.ovl, 0, 32, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.gr_counts, 0, 8 * (size_t)(ec::kMaxGrBins + 1), stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the host record is copied by now
  if (e != hipSuccess) {
    ec_status r = hip_fail(s, e, "init");
    delete s;
    return r;
  }
  *out = s;
  return EC_OK;
}

}  // namespace

extern "C" {

ec_status ec_init_system(const ec_params* p, void* ws, size_t ws_bytes, void* stream,
                         ec_system* out) {
  if (!out || !ws) return EC_E_INVALID;
  if (((uintptr_t)ws & 255) != 0) return EC_E_INVALID;  // the layout's arrays are 256-byte aligned
  *out = nullptr;
  Derived dv;
  std::string why;
  ec_status st = validate(p, &dv, &why);
  if (st != EC_OK) return st;
  return init_system_at(p, dv, (unsigned char*)ws, ws_bytes, (hipStream_t)stream, false, out);
}

// Read the durations of the timed sweeps still held in the event pool.
static ec_status resolve_timing(ec_system s) {
  if (!s->timing || s->pending == 0) return EC_OK;
  EC_HIP(s, hipStreamSynchronize(s->stream));
  const int nq = (s->shape.periodic || s->shape.one_launch) ? 1 : (s->shape.stripes ? 2 : 4);
  for (int k = 0; k < s->pending; ++k) {
    const ec::PhaseEvents& ev = s->ev[(size_t)k];
    for (int q = 0; q < nq; ++q) {
      float ms = 0.f;
      EC_HIP(s, hipEventElapsedTime(&ms, ev.begin[q], ev.end[q]));
      s->phase_ms += ms;
      s->phase_launches += 1;
    }
    if (!s->shape.periodic) {
      float m0 = 0.f, m1 = 0.f;
      EC_HIP(s, hipEventElapsedTime(&m0, ev.rebin[0], ev.rebin[1]));
      EC_HIP(s, hipEventElapsedTime(&m1, ev.rebin[2], ev.rebin[3]));
      s->count_ms += m0;
      s->scatter_ms += m1;
      s->rebin_launches += 1;
    }
  }
  s->pending = 0;
  return EC_OK;
}

ec_status ec_sweep(ec_system s, int64_t n_sweeps) {
  if (!s || n_sweeps < 0) return EC_E_INVALID;
  for (int64_t i = 0; i < n_sweeps; ++i) {
    if (s->timing) {
      if (s->pending == (int)s->ev.size()) {
        ec_status st = resolve_timing(s);
        if (st != EC_OK) return st;
      }
      EC_HIP(s, ec::launch_sweep(s->dev_d, s->shape, s->stream, &s->ev[(size_t)s->pending]));
      s->pending += 1;
    } else {
      EC_HIP(s, ec::launch_sweep(s->dev_d, s->shape, s->stream));
    }
    s->sweeps += 1;
  }
  return EC_OK;
}

// Sweeps whose kernel events the pool holds before ec_sweep reads them.
constexpr int kTimingPool = 64;

static void destroy_events(ec_system s) {
  for (auto& ev : s->ev) {
    for (int q = 0; q < 4; ++q) {
      if (ev.begin[q]) (void)hipEventDestroy(ev.begin[q]);  // cleanup: failures ignored
      if (ev.end[q]) (void)hipEventDestroy(ev.end[q]);
      if (ev.rebin[q]) (void)hipEventDestroy(ev.rebin[q]);
    }
  }
  s->ev.clear();
}

ec_status ec_set_timing(ec_system s, int32_t on) {
  if (!s) return EC_E_INVALID;
  if (on && !s->timing) {
    s->ev.assign(kTimingPool, ec::PhaseEvents{});
    for (auto& ev : s->ev) {
      for (int q = 0; q < 4; ++q) {
        hipError_t e = hipEventCreate(&ev.begin[q]);
        if (e == hipSuccess) e = hipEventCreate(&ev.end[q]);
        if (e == hipSuccess) e = hipEventCreate(&ev.rebin[q]);
        if (e != hipSuccess) {
          destroy_events(s);
          return hip_fail(s, e, "hipEventCreate");
        }
      }
    }
    s->timing = true;
  }
  if (!on && s->timing) {
    EC_HIP(s, hipStreamSynchronize(s->stream));
    destroy_events(s);
    s->timing = false;
  }
  s->pending = 0;
  s->phase_ms = s->count_ms = s->scatter_ms = 0.0;
  s->phase_launches = s->rebin_launches = 0;
  return EC_OK;
}

ec_status ec_get_timing(ec_system s, double* phase_ms, int64_t* launches) {
  if (!s || !phase_ms || !launches) return EC_E_INVALID;
  ec_status st = resolve_timing(s);
  if (st != EC_OK) return st;
  *phase_ms = s->phase_ms;
  *launches = s->phase_launches;
  return EC_OK;
}

ec_status ec_get_rebin_timing(ec_system s, double* count_ms, double* scatter_ms,
                              int64_t* sweeps) {
  if (!s || !count_ms || !scatter_ms || !sweeps) return EC_E_INVALID;
  ec_status st = resolve_timing(s);
  if (st != EC_OK) return st;
  *count_ms = s->count_ms;
  *scatter_ms = s->scatter_ms;
  *sweeps = s->rebin_launches;
  return EC_OK;
}

ec_status ec_set_dep_wait_limit(ec_system s, double seconds) {
  if (!s || !(seconds >= 0.0) || !std::isfinite(seconds)) return EC_E_INVALID;
  if (s->in_batch) return EC_E_STATE;
  const double ticks = seconds * 1e8;
  s->dev.dep_wait_ticks = ticks >= 9.0e18 ? INT64_MAX : (int64_t)ticks;
  EC_HIP(s, hipMemcpyAsync(s->dev_d, &s->dev, sizeof(ec::Dev), hipMemcpyHostToDevice, s->stream));
  EC_HIP(s, hipStreamSynchronize(s->stream));  // the host record may change again at once
  return EC_OK;
}

static ec_status check_err(ec_system s) {
  int32_t err[2] = {0, 0};
  double dbg[ec::kDebugWords];
  unsigned long long ovl[4] = {0, 0, 0, 0};
  EC_HIP(s, hipMemcpyAsync(err, s->dev.err, 8, hipMemcpyDeviceToHost, s->stream));
  EC_HIP(s, hipMemcpyAsync(dbg, s->dev.dbg, sizeof dbg, hipMemcpyDeviceToHost, s->stream));
  EC_HIP(s, hipMemcpyAsync(ovl, s->dev.ovl, sizeof ovl, hipMemcpyDeviceToHost, s->stream));
  EC_HIP(s, hipStreamSynchronize(s->stream));
  if (err[0] == ec::ERR_OVERLAP) {
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "overlap check: %llu pairs closer than sigma after sweep %llu; first pair: "
                  "disks %llu and %llu",
                  ovl[0], ovl[3], ovl[1], ovl[2]);
    s->last_error = buf;
    return EC_E_OVERLAP;
  }
  if (err[0] != 0) {
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "device check failed (bits 0x%x: 1 cell capacity, 2 bin capacity, 4 events per "
                  "chain, 8 draw retries, 16 dependency wait, 32 undo log, 64 overlap, 128 batch "
                  "sweep abandoned after another system's error); first "
                  "tripped chain: "
                  "cell %.0f "
                  "chain %.0f sweep %.0f "
                  "phase %.0f pos (%.17g, %.17g) dir (%.17g, %.17g) rem %.17g slot %.0f id %.0f "
                  "n_own %.0f",
                  err[0], dbg[0], dbg[1], dbg[2], dbg[3], dbg[4], dbg[5], dbg[6], dbg[7], dbg[8],
                  dbg[9], dbg[10], dbg[11]);
    s->last_error = buf;
    return EC_E_STATE;
  }
  return EC_OK;
}

ec_status ec_measure_pressure(ec_system s, double* z, double* bp, uint64_t* counts) {
  if (!s) return EC_E_INVALID;
  EC_HIP(s, ec::launch_reduce(s->dev_d, s->stream));
  double red[8];
  EC_HIP(s, hipMemcpyAsync(red, s->dev.red, sizeof red, hipMemcpyDeviceToHost, s->stream));
  ec_status st = check_err(s);
  if (st != EC_OK) return st;
  uint64_t cnt[ec::CNT_NCOL];
  for (int k = 0; k < ec::CNT_NCOL; ++k) std::memcpy(&cnt[k], &red[1 + k], 8);
  double chains = (double)cnt[ec::CNT_CHAINS];
  double zz = chains > 0 ? 1.0 + red[0] / (chains * s->p.ell) : 1.0;
  if (z) *z = zz;
  if (bp) *bp = zz * (double)s->p.n_disks * s->p.sigma * s->p.sigma / (s->dv.L * s->dv.L);
  if (counts) for (int k = 0; k < ec::CNT_NCOL; ++k) counts[k] = cnt[k];
  return EC_OK;
}

ec_status ec_measure_psi6(ec_system s, double r_cut, double* psi_re, double* psi_im,
                          double* mean_neighbours, double* per_disk) {
  if (!s) return EC_E_INVALID;
  const double rc = r_cut > 0.0 ? r_cut : 1.4 * s->p.sigma;
  const double limit = s->p.cells_per_side == 1 ? 0.5 * s->dv.L : s->dv.w;
  if (!(rc <= limit)) {
    s->last_error = "r_cut must not exceed the cell side (half the box for one periodic cell)";
    return EC_E_INVALID;
  }
  EC_HIP(s, ec::launch_psi6(s->dev_d, s->shape, rc, s->stream));
  double red[3];
  EC_HIP(s, hipMemcpyAsync(red, s->dev.psi_red, sizeof red, hipMemcpyDeviceToHost, s->stream));
  if (per_disk)
    EC_HIP(s, hipMemcpyAsync(per_disk, s->dev.psi, 16 * (size_t)s->p.n_disks, hipMemcpyDeviceToHost,
                             s->stream));
  ec_status st = check_err(s);
  if (st != EC_OK) return st;
  if (psi_re) *psi_re = red[0];
  if (psi_im) *psi_im = red[1];
  if (mean_neighbours) *mean_neighbours = red[2];
  return EC_OK;
}

ec_status ec_measure_psi6_delaunay(ec_system s, double r_search, double* psi_re, double* psi_im,
                                   double* mean_neighbours, double* per_disk, int32_t* neighbours) {
  if (!s || !std::isfinite(r_search)) return EC_E_INVALID;
  const double spacing = s->dv.L / std::sqrt((double)s->p.n_disks);
  const double rs = r_search > 0.0 ? r_search : std::min(4.0 * spacing, s->p.cells_per_side == 1 ? 0.5 * s->dv.L : s->dv.w);
  const double limit = s->p.cells_per_side == 1 ? 0.5 * s->dv.L : s->dv.w;
  if (!(rs <= limit) || s->p.n_disks < 3) {
    s->last_error = "r_search must not exceed the cell side (half the box for one periodic cell)";
    return EC_E_INVALID;
  }
  EC_HIP(s, ec::launch_psi6_delaunay(s->dev_d, s->shape, rs, s->stream));
  double red[3];
  unsigned long long bad[2];
  EC_HIP(s, hipMemcpyAsync(red, s->dev.psi_red, sizeof red, hipMemcpyDeviceToHost, s->stream));
  EC_HIP(s, hipMemcpyAsync(bad, s->dev.psi_err, sizeof bad, hipMemcpyDeviceToHost, s->stream));
  if (per_disk)
    EC_HIP(s, hipMemcpyAsync(per_disk, s->dev.psi, 16 * (size_t)s->p.n_disks, hipMemcpyDeviceToHost,
                             s->stream));
  if (neighbours)
    EC_HIP(s, hipMemcpyAsync(neighbours, s->dev.psi_nb, 4 * (size_t)s->p.n_disks,
                             hipMemcpyDeviceToHost, s->stream));
  ec_status st = check_err(s);
  if (st != EC_OK) return st;
  if (bad[0] || bad[1]) {
    char buf[256];
    std::string why = "Delaunay neighbours not certified at r_search = ";
    std::snprintf(buf, sizeof buf, "%.6g:", rs);
    why += buf;
    if (bad[0]) {
      std::snprintf(buf, sizeof buf, " %llu disks with a Voronoi vertex beyond r_search/2 (raise r_search);", bad[0]);
      why += buf;
    }
    if (bad[1]) {
      std::snprintf(buf, sizeof buf, " %llu disks with more than 128 candidates (lower r_search);", bad[1]);
      why += buf;
    }
    s->last_error = why;
    return EC_E_UNSUPPORTED;
  }
  if (psi_re) *psi_re = red[0];
  if (psi_im) *psi_im = red[1];
  if (mean_neighbours) *mean_neighbours = red[2];
  return EC_OK;
}

ec_status ec_psi_autocorrelation(const double* psi_re, const double* psi_im, int64_t n,
                                 int32_t max_lag, double* c, double* tau) {
  if (!psi_re || !psi_im || !c || n < 2 || max_lag < 1 || max_lag >= n) return EC_E_INVALID;
  // eq. (tau): C(dt) = Re <Psi*(t) Psi(t + dt)>_t / <|Psi(t)|^2>_t
  double den = 0.0;
  for (int64_t t = 0; t < n; ++t) den += psi_re[t] * psi_re[t] + psi_im[t] * psi_im[t];
  den /= (double)n;
  if (!(den > 0.0)) return EC_E_INVALID;
  for (int32_t lag = 0; lag <= max_lag; ++lag) {
    double acc = 0.0;
    for (int64_t t = 0; t + lag < n; ++t)  // Re(conj(a) b) = ar br + ai bi
      acc += psi_re[t] * psi_re[t + lag] + psi_im[t] * psi_im[t + lag];
    c[lag] = acc / (double)(n - lag) / den;
  }
  if (tau) {
    // ln C(dt) = -dt / tau by least squares through the origin, dt = 1, 2, ...
    // while C(dt) > e^-2
    double sdd = 0.0, sdl = 0.0;
    for (int32_t lag = 1; lag <= max_lag; ++lag) {
      if (!(c[lag] > std::exp(-2.0))) break;
      sdd += (double)lag * (double)lag;
      sdl += (double)lag * std::log(c[lag]);
    }
    *tau = sdd > 0.0 ? -sdd / sdl : std::nan("");
  }
  return EC_OK;
}

ec_status ec_gr_reset(ec_system s) {
  if (!s) return EC_E_INVALID;
  EC_HIP(s, hipMemsetAsync(s->dev.gr_counts, 0, 8 * (size_t)(ec::kMaxGrBins + 1), s->stream));
  s->gr_samples = 0;
  s->gr_bins = 0;
  s->gr_rmax = 0.0;
  return EC_OK;
}

ec_status ec_gr_accumulate(ec_system s, double r_max, int32_t n_bins) {
  if (!s) return EC_E_INVALID;
  const double limit = s->p.cells_per_side == 1 ? 0.5 * s->dv.L : s->dv.w;
  if (!(r_max > s->p.sigma) || !(r_max <= limit) || n_bins < 1 || n_bins > ec::kMaxGrBins) {
    s->last_error = "need sigma < r_max <= cell side (half the box for one cell), 1 <= n_bins <= 1024";
    return EC_E_INVALID;
  }
  if (s->gr_samples == 0 || r_max != s->gr_rmax || n_bins != s->gr_bins) {
    ec_status st = ec_gr_reset(s);  // a new series starts from zero counts
    if (st != EC_OK) return st;
  }
  s->gr_rmax = r_max;
  s->gr_bins = n_bins;
  const double delta = (r_max - s->p.sigma) / (double)n_bins;
  EC_HIP(s, ec::launch_gr(s->dev_d, s->shape, r_max, delta, n_bins, s->stream));
  s->gr_samples += 1;
  return EC_OK;
}

ec_status ec_gr_counts(ec_system s, uint64_t* counts, int64_t* samples, uint64_t* overlaps) {
  if (!s || !counts) return EC_E_INVALID;
  std::vector<uint64_t> h((size_t)ec::kMaxGrBins + 1);
  EC_HIP(s, hipMemcpyAsync(h.data(), s->dev.gr_counts, 8 * h.size(), hipMemcpyDeviceToHost, s->stream));
  ec_status st = check_err(s);
  if (st != EC_OK) return st;
  for (int32_t i = 0; i < s->gr_bins; ++i) counts[i] = h[(size_t)i];
  if (samples) *samples = s->gr_samples;
  if (overlaps) *overlaps = h[(size_t)s->gr_bins];
  return EC_OK;
}

ec_status ec_gr_normalize(int64_t n_disks, double box, double sigma, double r_max, int32_t n_bins,
                          const uint64_t* counts, int64_t samples, double fit_width, double* g,
                          double* R, double* g_contact, double* z) {
  if (n_disks < 2 || !(box > 0.0) || !(sigma > 0.0) || !(r_max > sigma) || n_bins < 1 || !counts ||
      samples < 1 || !(fit_width > 0.0))
    return EC_E_INVALID;
  const double rho = (double)n_disks / (box * box);
  const double delta = (r_max - sigma) / (double)n_bins;
  // least-squares quadratic in x = R - sigma over the bins with x < fit_width
  double sx[5] = {0, 0, 0, 0, 0}, sy[3] = {0, 0, 0};
  int used = 0;
  for (int32_t i = 0; i < n_bins; ++i) {
    const double e0 = sigma + delta * i, e1 = sigma + delta * (i + 1);
    const double area = kPi * (e1 * e1 - e0 * e0);
    const double gi = (double)counts[i] / ((double)samples * (double)n_disks * rho * area);
    const double Ri = 2.0 * (e1 * e1 * e1 - e0 * e0 * e0) / (3.0 * (e1 * e1 - e0 * e0));
    if (g) g[i] = gi;
    if (R) R[i] = Ri;
    const double x = Ri - sigma;
    if (x < fit_width) {
      double p = 1.0;
      for (int k = 0; k < 5; ++k) { sx[k] += p; if (k < 3) sy[k] += p * gi; p *= x; }
      ++used;
    }
  }
  if (used < 3) return EC_E_INVALID;
  // normal equations [sx0 sx1 sx2; sx1 sx2 sx3; sx2 sx3 sx4] c = sy, Cramer's rule for c0
  const double a00 = sx[0], a01 = sx[1], a02 = sx[2], a11 = sx[2], a12 = sx[3], a22 = sx[4];
  const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) +
                     a02 * (a01 * a12 - a11 * a02);
  if (!(std::fabs(det) > 0.0)) return EC_E_INVALID;
  const double det0 = sy[0] * (a11 * a22 - a12 * a12) - a01 * (sy[1] * a22 - a12 * sy[2]) +
                      a02 * (sy[1] * a12 - a11 * sy[2]);
  const double gc = det0 / det;
  if (g_contact) *g_contact = gc;
  // eq. (pressure): beta P / rho = 1 + (pi/2) sigma^2 rho g(sigma+)
  if (z) *z = 1.0 + 0.5 * kPi * sigma * sigma * rho * gc;
  return EC_OK;
}

ec_status ec_reset_tallies(ec_system s) {
  if (!s) return EC_E_INVALID;
  EC_HIP(s, ec::launch_zero_tallies(s->dev_d, s->p.cells_per_side * s->p.cells_per_side, s->stream));
  return EC_OK;
}

ec_status ec_get_positions(ec_system s, double* x, double* y, int64_t n) {
  if (!s || !x || !y || n != s->p.n_disks) return EC_E_INVALID;
  EC_HIP(s, hipMemcpyAsync(x, s->dev.x, 8 * (size_t)n, hipMemcpyDeviceToHost, s->stream));
  EC_HIP(s, hipMemcpyAsync(y, s->dev.y, 8 * (size_t)n, hipMemcpyDeviceToHost, s->stream));
  return check_err(s);
}

ec_status ec_set_positions(ec_system s, const double* x, const double* y, int64_t n) {
  if (!s || !x || !y || n != s->p.n_disks) return EC_E_INVALID;
  const double L = s->dv.L, sigma = s->p.sigma;
  std::vector<double> hx((size_t)n), hy((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(x[i]) || !std::isfinite(y[i])) return EC_E_INVALID;
    double vx = std::fmod(x[i], L), vy = std::fmod(y[i], L);
    if (vx < 0.0) vx += L;
    if (vy < 0.0) vy += L;
    if (vx >= L) vx -= L;
    if (vy >= L) vy -= L;
    hx[(size_t)i] = vx;
    hy[(size_t)i] = vy;
  }
  // overlap check with a grid of side >= sigma (minimum image)
  int64_t g = (int64_t)std::floor(L / sigma);
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  double gs = L / (double)g;
  std::vector<int64_t> head((size_t)(g * g), -1), next((size_t)n, -1);
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = std::min<int64_t>((int64_t)(hx[(size_t)i] / gs), g - 1);
    int64_t cy = std::min<int64_t>((int64_t)(hy[(size_t)i] / gs), g - 1);
    next[(size_t)i] = head[(size_t)(cy * g + cx)];
    head[(size_t)(cy * g + cx)] = i;
  }
  const double s2 = sigma * sigma;
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = std::min<int64_t>((int64_t)(hx[(size_t)i] / gs), g - 1);
    int64_t cy = std::min<int64_t>((int64_t)(hy[(size_t)i] / gs), g - 1);
    for (int64_t oy = -1; oy <= 1; ++oy)
      for (int64_t ox = -1; ox <= 1; ++ox) {
        int64_t nx = ((cx + ox) % g + g) % g, ny = ((cy + oy) % g + g) % g;
        for (int64_t j = head[(size_t)(ny * g + nx)]; j >= 0; j = next[(size_t)j]) {
          if (j <= i) continue;
          double dx = hx[(size_t)j] - hx[(size_t)i], dy = hy[(size_t)j] - hy[(size_t)i];
          dx -= L * std::nearbyint(dx / L);
          dy -= L * std::nearbyint(dy / L);
          if (dx * dx + dy * dy < s2) {
            s->last_error = "disks " + std::to_string(i) + " and " + std::to_string(j) + " overlap";
            return EC_E_OVERLAP;
          }
        }
        if (g < 3 && (ox != 0 || oy != 0)) { /* small grids revisit cells; harmless */ }
      }
  }
  EC_HIP(s, hipMemcpyAsync(s->dev.x, hx.data(), 8 * (size_t)n, hipMemcpyHostToDevice, s->stream));
  EC_HIP(s, hipMemcpyAsync(s->dev.y, hy.data(), 8 * (size_t)n, hipMemcpyHostToDevice, s->stream));
  EC_HIP(s, hipStreamSynchronize(s->stream));
  return EC_OK;
}

ec_status ec_get_digests(ec_system s, uint64_t* out, int64_t n) {
  if (!s || !out || n < 0 || n > s->sweeps || n > ec::kDigestRing) return EC_E_INVALID;
  std::vector<uint64_t> ring(ec::kDigestRing);
  EC_HIP(s, hipMemcpyAsync(ring.data(), s->dev.digest_ring, 8 * ring.size(), hipMemcpyDeviceToHost,
                           s->stream));
  ec_status st = check_err(s);
  if (st != EC_OK) return st;
  for (int64_t i = 0; i < n; ++i) {
    int64_t sw = s->sweeps - n + i;
    out[i] = ring[(size_t)(sw % ec::kDigestRing)];
  }
  return EC_OK;
}

ec_status ec_get_cell_tallies(ec_system s, double* delta, uint64_t* counts) {
  if (!s || !delta || !counts) return EC_E_INVALID;
  size_t nc = (size_t)s->p.cells_per_side * (size_t)s->p.cells_per_side;
  EC_HIP(s, hipMemcpyAsync(delta, s->dev.acc_delta, 8 * nc, hipMemcpyDeviceToHost, s->stream));
  EC_HIP(s, hipMemcpyAsync(counts, s->dev.acc_cnt, 8 * ec::CNT_NCOL * nc, hipMemcpyDeviceToHost,
                           s->stream));
  return check_err(s);
}

ec_status ec_get_cell_digests(ec_system s, uint64_t* out) {
  if (!s || !out) return EC_E_INVALID;
  size_t nc = (size_t)s->p.cells_per_side * (size_t)s->p.cells_per_side;
  EC_HIP(s, hipMemcpyAsync(out, s->dev.cell_digest, 8 * nc, hipMemcpyDeviceToHost, s->stream));
  return check_err(s);
}

ec_status ec_get_sweep_count(ec_system s, int64_t* sweeps) {
  if (!s || !sweeps) return EC_E_INVALID;
  *sweeps = s->sweeps;
  return EC_OK;
}

ec_status ec_destroy(ec_system s) {
  if (!s) return EC_E_INVALID;
  if (s->in_batch) return EC_E_STATE;  // views are destroyed with their batch
  if (s->timing) (void)ec_set_timing(s, 0);  // cleanup: its failure is reported below
  hipError_t e = hipStreamSynchronize(s->stream);
  delete s;
  return e == hipSuccess ? EC_OK : EC_E_HIP;
}

// ---------------------------------------------------------------------------
// Batched form: several walled systems advanced by shared launches
// ---------------------------------------------------------------------------
}  // extern "C"

struct ec_batch_s {
  std::vector<ec_system> sys;
  std::vector<size_t> off;      // byte offset of each system's region
  int32_t schedule;             // EC_SCHEDULE_*
  unsigned char* ws;
  size_t sys_bytes;             // bytes of all system regions (snapshot size)
  ec::Dev* devs_d;              // device array of the systems' records
  ec::LaunchShape shape;
  hipStream_t stream;
  bool use_graph;
  bool graph_ready;
  hipGraph_t graph;
  hipGraphExec_t exec;
  std::string last_error;
};

namespace {

constexpr int32_t kMaxBatch = 4096;

struct BatchLayout {
  size_t devs, q_hdr, q_tasks, q_flags, q_dep, q_base, systems, snapshot, total;
  int32_t cells;                // cells of all systems (ready-queue slots)
  std::vector<size_t> off;
  std::vector<int32_t> base;    // first queue index of each system's cells, then the total
};

ec_status batch_layout(const ec_params* ps, int32_t n, BatchLayout* bl, std::vector<Derived>* dvs,
                       std::string* why) {
  if (!ps || n < 1 || n > kMaxBatch) { *why = "batch size out of range"; return EC_E_INVALID; }
  size_t o = 0;
  bl->devs = o;
  o = align256(o + sizeof(ec::Dev) * (size_t)n);
  bl->base.assign((size_t)n + 1, 0);
  int64_t cells = 0;
  for (int32_t i = 0; i < n; ++i) {
    bl->base[(size_t)i] = (int32_t)cells;
    cells += (int64_t)ps[i].cells_per_side * ps[i].cells_per_side;
    if (cells > (int64_t(1) << 30)) { *why = "too many cells in the batch"; return EC_E_INVALID; }
  }
  bl->base[(size_t)n] = (int32_t)cells;
  bl->cells = (int32_t)cells;
  bl->q_hdr = o;   o = align256(o + 16);
  bl->q_tasks = o; o = align256(o + 8 * (size_t)cells);
  bl->q_flags = o; o = align256(o + 4 * (size_t)cells);
  bl->q_dep = o;   o = align256(o + 4 * (size_t)cells);
  bl->q_base = o;  o = align256(o + 4 * ((size_t)n + 1));
  bl->systems = o;
  bl->off.resize((size_t)n);
  dvs->resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    ec_status st = validate(&ps[i], &(*dvs)[(size_t)i], why);
    if (st != EC_OK) return st;
    if (ps[i].cells_per_side == 1) { *why = "batches hold walled systems (C >= 4) only"; return EC_E_UNSUPPORTED; }
    if (ps[i].precision != ps[0].precision) {
      *why = "the systems of a batch share one precision"; return EC_E_UNSUPPORTED;
    }
    if ((ps[i].flags ^ ps[0].flags) &
        (EC_FLAG_PHASE_LAUNCHES | EC_FLAG_ONE_LAUNCH | EC_FLAG_REJECT | EC_FLAG_STRIPES)) {
      *why = "the systems of a batch share one schedule"; return EC_E_UNSUPPORTED;
    }
    bl->off[(size_t)i] = o;
    o = align256(o + make_layout(ps[i].n_disks, ps[i].cells_per_side, ps[i].chains_per_cell).total);
  }
  size_t sys_bytes = o - bl->systems;
  bl->snapshot = o;
  o = align256(o + sys_bytes);
  bl->total = o;
  return EC_OK;
}

// The launch shape of the batch's schedule (ready queue: as many persistent
// wavefronts as fit on the device, at most one per cell).
ec_status batch_apply_schedule(ec_batch b) {
  ec::LaunchShape& sh = b->shape;
  // (the striped decomposition has its own two phase launches)
  sh.one_launch = b->schedule == EC_SCHEDULE_ONE_LAUNCH && !sh.stripes;
  sh.ready_queue = b->schedule == EC_SCHEDULE_READY_QUEUE && !sh.stripes;
  if (sh.ready_queue) {
    int workers = 0;
    hipError_t e = ec::ready_queue_workers(sh.max_lds_per_cell, sh.cpb, sh.fp32_screen ? 1 : 0,
                                           sh.reject ? 1 : 0, &workers);
    if (e != hipSuccess) {
      b->last_error = std::string("ready-queue occupancy: ") + hipGetErrorString(e);
      return EC_E_HIP;
    }
    sh.queue.workers = std::max(1, std::min(workers, sh.queue.total));
  }
  return EC_OK;
}

// Upload the records with the batch's schedule and drop any captured graph.
ec_status batch_sync_records(ec_batch b) {
  ec_status st0 = batch_apply_schedule(b);
  if (st0 != EC_OK) return st0;
  std::vector<ec::Dev> h(b->sys.size());
  for (size_t i = 0; i < b->sys.size(); ++i) {
    b->sys[i]->dev.cells_per_block = b->shape.cpb;
    b->sys[i]->shape.cpb = b->shape.cpb;
    h[i] = b->sys[i]->dev;
  }
  hipError_t e = hipMemcpyAsync(b->devs_d, h.data(), sizeof(ec::Dev) * h.size(), hipMemcpyHostToDevice,
                                b->stream);
  for (size_t i = 0; i < b->sys.size() && e == hipSuccess; ++i)
    e = hipMemcpyAsync(b->sys[i]->dev_d, &h[i], sizeof(ec::Dev), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // h is a local
  if (b->graph_ready) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->graph_ready = false;
  }
  if (e != hipSuccess) {
    b->last_error = std::string("batch records: ") + hipGetErrorString(e);
    return EC_E_HIP;
  }
  return EC_OK;
}

ec_status batch_fail(ec_batch b, hipError_t e, const char* what) {
  b->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return EC_E_HIP;
}

ec_status batch_sweeps(ec_batch b, int64_t n) {
  if (b->use_graph) {
    if (!b->graph_ready) {
      hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return batch_fail(b, e, "begin capture");
      hipError_t el = ec::launch_sweep(b->devs_d, b->shape, b->stream);
      e = hipStreamEndCapture(b->stream, &b->graph);
      if (el != hipSuccess) return batch_fail(b, el, "captured sweep");
      if (e != hipSuccess) return batch_fail(b, e, "end capture");
      e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(b->graph);
        return batch_fail(b, e, "instantiate");
      }
      b->graph_ready = true;
    }
    for (int64_t i = 0; i < n; ++i) {
      hipError_t e = hipGraphLaunch(b->exec, b->stream);
      if (e != hipSuccess) return batch_fail(b, e, "graph launch");
    }
  } else {
    for (int64_t i = 0; i < n; ++i) {
      hipError_t e = ec::launch_sweep(b->devs_d, b->shape, b->stream);
      if (e != hipSuccess) return batch_fail(b, e, "sweep");
    }
  }
  for (auto* s : b->sys) s->sweeps += n;
  return EC_OK;
}

}  // namespace

extern "C" {

ec_status ec_batch_workspace_bytes(const ec_params* ps, int32_t n_sys, size_t* bytes) {
  if (!bytes) return EC_E_INVALID;
  BatchLayout bl;
  std::vector<Derived> dvs;
  std::string why;
  ec_status st = batch_layout(ps, n_sys, &bl, &dvs, &why);
  if (st != EC_OK) return st;
  *bytes = bl.total;
  return EC_OK;
}

ec_status ec_init_batch(const ec_params* ps, int32_t n_sys, void* ws, size_t ws_bytes, void* stream,
                        ec_batch* out) {
  if (!out || !ws) return EC_E_INVALID;
  if (((uintptr_t)ws & 255) != 0) return EC_E_INVALID;  // the layout's arrays are 256-byte aligned
  *out = nullptr;
  BatchLayout bl;
  std::vector<Derived> dvs;
  std::string why;
  ec_status st = batch_layout(ps, n_sys, &bl, &dvs, &why);
  if (st != EC_OK) return st;
  if (ws_bytes < bl.total) return EC_E_NOMEM;
  ec_batch b = new (std::nothrow) ec_batch_s();
  if (!b) return EC_E_NOMEM;
  b->ws = (unsigned char*)ws;
  b->off = bl.off;
  b->sys_bytes = bl.snapshot - bl.systems;
  b->devs_d = (ec::Dev*)(b->ws + bl.devs);
  b->stream = (hipStream_t)stream;
  b->use_graph = false;
  b->graph_ready = false;
  // schedule: the ready queue unless a schedule flag asks for another
  b->schedule = (ps[0].flags & EC_FLAG_ONE_LAUNCH)       ? EC_SCHEDULE_ONE_LAUNCH
                : (ps[0].flags & EC_FLAG_PHASE_LAUNCHES) ? EC_SCHEDULE_PHASE_LAUNCHES
                                                         : EC_SCHEDULE_READY_QUEUE;
  ec::LaunchShape& sh = b->shape;
  std::memset(&sh, 0, sizeof sh);
  sh.n_sys = n_sys;
  sh.periodic = false;
  sh.fp32_screen = ps[0].precision == EC_PREC_FP32_SCREEN;
  sh.reject = (ps[0].flags & EC_FLAG_REJECT) != 0;
  sh.stripes = (ps[0].flags & EC_FLAG_STRIPES) != 0;
  sh.cpb = 1;
  sh.queue.hdr = (int32_t*)(b->ws + bl.q_hdr);
  sh.queue.tasks = (int64_t*)(b->ws + bl.q_tasks);
  sh.queue.flags = (int32_t*)(b->ws + bl.q_flags);
  sh.queue.dep = (int32_t*)(b->ws + bl.q_dep);
  sh.queue.base = (const int32_t*)(b->ws + bl.q_base);
  sh.queue.total = bl.cells;
  sh.queue.workers = 1;
  {
    // queue header, flags and per-system bases (init synchronises below)
    hipError_t e = hipMemsetAsync(b->ws + bl.q_hdr, 0, 16, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->ws + bl.q_flags, 0, 4 * (size_t)bl.cells, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->ws + bl.q_base, bl.base.data(), 4 * bl.base.size(), hipMemcpyHostToDevice,
                         b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // bl.base is a local
    if (e != hipSuccess) {
      delete b;
      return EC_E_HIP;
    }
  }
  for (int32_t i = 0; i < n_sys; ++i) {
    ec_params p = ps[i];
    p.cells_per_block = 1;
    ec_system s = nullptr;
    size_t region = (i + 1 < n_sys ? bl.off[(size_t)i + 1] : bl.snapshot) - bl.off[(size_t)i];
    st = init_system_at(&p, dvs[(size_t)i], b->ws + bl.off[(size_t)i], region, b->stream, true, &s);
    if (st != EC_OK) {
      b->last_error = "system " + std::to_string(i) + ": init failed";
      for (auto* v : b->sys) delete v;
      delete b;
      return st;
    }
    b->sys.push_back(s);
    const ec::LaunchShape& one = s->shape;
    sh.any_distinct = sh.any_distinct || one.any_distinct;
    sh.check_overlap = sh.check_overlap || one.check_overlap;
    sh.max_n = std::max(sh.max_n, one.max_n);
    sh.max_chains = std::max(sh.max_chains, one.max_chains);
    sh.max_cells = std::max(sh.max_cells, one.max_cells);
    sh.max_cells_side = std::max(sh.max_cells_side, one.max_cells_side);
    sh.max_active = std::max(sh.max_active, one.max_active);
    sh.max_lds_per_cell = std::max(sh.max_lds_per_cell, one.max_lds_per_cell);
  }
  st = batch_sync_records(b);
  if (st != EC_OK) {
    for (auto* v : b->sys) delete v;
    delete b;
    return st;
  }
  *out = b;
  return EC_OK;
}

ec_status ec_sweep_batch(ec_batch b, int64_t n_sweeps) {
  if (!b || n_sweeps < 0) return EC_E_INVALID;
  return batch_sweeps(b, n_sweeps);
}

ec_status ec_batch_system(ec_batch b, int32_t i, ec_system* out) {
  if (!b || !out || i < 0 || i >= (int32_t)b->sys.size()) return EC_E_INVALID;
  *out = b->sys[(size_t)i];
  return EC_OK;
}

ec_status ec_batch_set_graph(ec_batch b, int32_t on) {
  if (!b) return EC_E_INVALID;
  if (on && b->stream == nullptr) {
    b->last_error = "graph capture needs a stream other than the null stream";
    return EC_E_UNSUPPORTED;
  }
  b->use_graph = on != 0;
  return EC_OK;
}

ec_status ec_batch_set_cells_per_block(ec_batch b, int32_t cpb) {
  if (!b) return EC_E_INVALID;
  if (cpb != 1 && cpb != 2 && cpb != 4) return EC_E_INVALID;
  if ((size_t)cpb * (size_t)b->shape.max_lds_per_cell > 160 * 1024) return EC_E_UNSUPPORTED;
  b->shape.cpb = cpb;
  return batch_sync_records(b);
}

ec_status ec_batch_set_schedule(ec_batch b, int32_t schedule) {
  if (!b) return EC_E_INVALID;
  if (schedule < EC_SCHEDULE_PHASE_LAUNCHES || schedule > EC_SCHEDULE_READY_QUEUE) return EC_E_INVALID;
  b->schedule = schedule;
  return batch_sync_records(b);
}

ec_status ec_batch_autotune(ec_batch b, int32_t trial_sweeps, int32_t* schedule_out,
                            int32_t* cpb_out, double* ms_out) {
  if (!b || trial_sweeps < 1) return EC_E_INVALID;
  // the trials run from a snapshot of every system's state, which is put back
  // afterwards: the schedule changes timing only, never the trajectory
  unsigned char* sys0 = b->ws + b->off[0];
  unsigned char* snap = sys0 + b->sys_bytes;
  std::vector<int64_t> sweeps0;
  for (auto* s : b->sys) sweeps0.push_back(s->sweeps);
  hipError_t e = hipMemcpyAsync(snap, sys0, b->sys_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return batch_fail(b, e, "snapshot");
  hipEvent_t t0, t1;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return batch_fail(b, e, "event");
  if ((e = hipEventCreate(&t1)) != hipSuccess) { (void)hipEventDestroy(t0); return batch_fail(b, e, "event"); }
  const int32_t cands[3] = {1, 2, 4};
  int32_t best = b->shape.cpb, best_sched = b->schedule;
  double best_ms = 0.0;
  ec_status st = EC_OK;
  for (int sc = EC_SCHEDULE_PHASE_LAUNCHES; sc <= EC_SCHEDULE_READY_QUEUE && st == EC_OK; ++sc) {
    for (int c = 0; c < 3 && st == EC_OK; ++c) {
      double ms_c = -1.0;
      if ((size_t)cands[c] * (size_t)b->shape.max_lds_per_cell <= 160 * 1024) {
        b->schedule = sc;
        b->shape.cpb = cands[c];
        st = batch_sync_records(b);
        if (st != EC_OK) break;
        e = hipMemcpyAsync(sys0, snap, b->sys_bytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) st = batch_sweeps(b, 1);  // warm-up (graph capture, caches)
        if (e == hipSuccess && st == EC_OK) e = hipMemcpyAsync(sys0, snap, b->sys_bytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess && st == EC_OK) e = hipEventRecord(t0, b->stream);
        if (e == hipSuccess && st == EC_OK) st = batch_sweeps(b, trial_sweeps);
        if (e == hipSuccess && st == EC_OK) e = hipEventRecord(t1, b->stream);
        if (e == hipSuccess && st == EC_OK) e = hipEventSynchronize(t1);
        float ms = 0.f;
        if (e == hipSuccess && st == EC_OK) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) { st = batch_fail(b, e, "autotune trial"); break; }
        ms_c = ms;
        if (best_ms == 0.0 || ms < best_ms) { best_ms = ms; best = cands[c]; best_sched = sc; }
      }
      if (ms_out) ms_out[3 * sc + c] = ms_c;
    }
  }
  (void)hipEventDestroy(t0);  // cleanup: failures ignored
  (void)hipEventDestroy(t1);
  // back to the snapshot with the chosen schedule
  e = hipMemcpyAsync(sys0, snap, b->sys_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess && st == EC_OK) st = batch_fail(b, e, "restore");
  for (size_t i = 0; i < b->sys.size(); ++i) b->sys[i]->sweeps = sweeps0[i];
  b->shape.cpb = best;
  b->schedule = best_sched;
  ec_status st2 = batch_sync_records(b);
  if (st == EC_OK) st = st2;
  if (cpb_out) *cpb_out = best;
  if (schedule_out) *schedule_out = best_sched;
  return st;
}

const char* ec_batch_last_error(ec_batch b) { return b ? b->last_error.c_str() : ""; }

// ---------------------------------------------------------------------------
// Allocation-free sweeps: the state of ec_sweep lives in the static buffer
// ---------------------------------------------------------------------------
ec_status ec_sweep_static(const ec_params* p, double* x, double* y, int64_t first_sweep,
                          int64_t n_sweeps, uint64_t* digests, int32_t* err, void* stream) {
  if (!x || !y || first_sweep < 0 || n_sweeps < 0) return EC_E_INVALID;
  if (digests && n_sweeps > ec::kDigestRing) return EC_E_INVALID;
  Derived dv;
  std::string why;
  ec_status st = validate(p, &dv, &why);
  if (st != EC_OK) return st;
  default_cells_per_block(p, &dv);
  if (p->n_disks > ec::kStaticMaxDisks) return EC_E_NOMEM;
  const Layout lay = make_layout(p->n_disks, p->cells_per_side, p->chains_per_cell, true);
  if (lay.total > ec::kStaticScratchBytes) return EC_E_NOMEM;
  void* base = nullptr;
  if (ec::static_scratch(&base) != hipSuccess) return EC_E_HIP;
  if (prepare_kernels() != hipSuccess) return EC_E_HIP;
  unsigned char* b = (unsigned char*)base;
  ec::Dev d;
  fill_record(&d, p, dv, b, lay);
  d.x = x;  // the caller's positions; no observables in this form
  d.y = y;
  d.psi = nullptr;
  d.psi_part = nullptr;
  d.psi_red = nullptr;
  d.psi_nb = nullptr;
  d.psi_err = nullptr;
  d.gr_counts = nullptr;
  ec::Dev* dd = (ec::Dev*)(b + lay.dev);
  const ec::LaunchShape sh = shape_of(d, *p);
  const hipStream_t hs = (hipStream_t)stream;
  hipError_t e = ec::launch_static_setup(d, dd, b, lay.total, first_sweep, hs);
  for (int64_t i = 0; i < n_sweeps && e == hipSuccess; ++i) e = ec::launch_sweep(dd, sh, hs);
  if (e == hipSuccess)
    e = ec::launch_static_copy_out(dd, first_sweep, digests ? n_sweeps : 0,
                                   (unsigned long long*)digests, err, hs);
  return e == hipSuccess ? EC_OK : EC_E_HIP;
}

ec_status ec_destroy_batch(ec_batch b) {
  if (!b) return EC_E_INVALID;
  hipError_t e = hipStreamSynchronize(b->stream);
  if (b->graph_ready) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
  }
  for (auto* s : b->sys) {
    if (s->timing) { s->in_batch = false; (void)ec_set_timing(s, 0); }
    delete s;
  }
  delete b;
  return e == hipSuccess ? EC_OK : EC_E_HIP;
}

}  // extern "C"
