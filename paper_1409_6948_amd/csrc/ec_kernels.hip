// gfx950 kernels of the parallel event-chain (PEC) sweep for 2D hard disks.
//
// Method: Kampmann, Boltz, Kierfeld, "Parallelized event chain algorithm for
// dense hard sphere and polymer systems" -- event chains Sec. 3.2, the
// parallel sweep Sec. 3.4 (steps 1-7), boundary reflection Fig. 1 (right),
// starts with replacement Fig. 2.
//
// Mapping to CDNA4: one wavefront (64 lanes) per active simulation cell.  A
// cell's own disks and its frozen neighbours (centres within sigma outside
// the cell) are staged in LDS in a grid of square bins of side b <
// sigma/sqrt(2); such a bin holds at most one centre of a configuration
// without overlaps, so one slot per bin suffices and a cell takes about 20 KB
// (eight cells, two wavefronts per SIMD, per CU).  One event search reads an
// 8 x 8 window of bins around the moving disk, one slot per lane, computes
// the contact distance of every slot in FP64, and takes a wave-wide minimum
// of the key (distance, disk id).  A geometric guard proves that no disk
// outside the window can be hit first; when it cannot (long free flights),
// the search is repeated over all slots of the cell.  The event found is
// therefore exactly the minimum over all candidate disks, in the same
// arithmetic as a plain serial search.
//
// Arithmetic contract (shared in writing with the CPU reference, no code
// shared): FP64 with no contraction (-ffp-contract=off) and explicit fma();
// correctly rounded sqrt and division; Philox4x64-10 streams keyed by
// (seed, kind) with counters (sweep, cell | system << 32, chain, block).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ec_internal.h"

namespace ec {
namespace {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

enum : uint64_t { kKindSweep = 1, kKindStart = 2, kKindDir = 3, kKindShuffle = 4 };

struct Block4 {
  uint64_t v0, v1, v2, v3;
};

__device__ __forceinline__ Block4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                         uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += kW0; k1 += kW1; }
    uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return Block4{c0, c1, c2, c3};
}

// Words 0..3 of counter block 0, then block 1, ...
struct Stream {
  uint64_t k0, k1, c0, c1, c2, blk;
  Block4 b;
  int pos;
  __device__ Stream(uint64_t seed, uint64_t kind, uint64_t a, uint64_t bb, uint64_t c)
      : k0(seed), k1(kind), c0(a), c1(bb), c2(c), blk(0), b{0, 0, 0, 0}, pos(4) {}
  __device__ uint64_t next() {
    if (pos == 4) {
      b = philox(c0, c1, c2, blk, k0, k1);
      blk += 1;
      pos = 0;
    }
    uint64_t w = (pos == 0) ? b.v0 : (pos == 1) ? b.v1 : (pos == 2) ? b.v2 : b.v3;
    pos += 1;
    return w;
  }
};

__device__ __forceinline__ double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// Lemire's multiply-shift with rejection: exactly uniform on [0, n).
__device__ uint64_t draw_index(Stream& st, uint64_t n) {
  uint64_t x = st.next();
  uint64_t hi = __umul64hi(x, n), lo = x * n;
  if (lo < n) {
    uint64_t t = (0ull - n) % n;
    while (lo < t) {
      x = st.next();
      hi = __umul64hi(x, n);
      lo = x * n;
    }
  }
  return hi;
}

__device__ __forceinline__ uint64_t cell_key(const Dev& d, int cell) {
  return (uint64_t)(uint32_t)cell | ((uint64_t)d.system << 32);
}

// Direction of chain k of a cell in a sweep.
__device__ void chain_direction(const Dev& d, int64_t sweep, int cell, int64_t k, double& dx,
                                double& dy) {
  if (d.dir_mode == 2) { dx = 1.0; dy = 0.0; return; }          // +x only
  if (d.dir_mode == 0) {                                         // +x / +y alternating
    if ((k & 1) == 0) { dx = 1.0; dy = 0.0; } else { dx = 0.0; dy = 1.0; }
    return;
  }
  // isotropic: uniform in the unit disk by rejection, then normalised
  Stream st(d.seed, kKindDir, (uint64_t)sweep, cell_key(d, cell), (uint64_t)k);
  double vx, vy, r2;
  for (;;) {
    vx = 2.0 * u01(st.next()) - 1.0;
    vy = 2.0 * u01(st.next()) - 1.0;
    r2 = fma(vx, vx, vy * vy);
    if (r2 < 1.0 && r2 >= 0x1p-40) break;
  }
  double r = sqrt(r2);
  dx = vx / r;
  dy = vy / r;
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ unsigned umin_(unsigned a, unsigned b) { return a < b ? a : b; }

// Minimum of a 32-bit value over the 64 lanes as a scalar: DPP steps within
// rows of 16, then the row broadcasts of lane 15 into rows 1 and 3 and of
// lane 31 into rows 2 and 3, which leave the minimum in lane 63.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));
  // rows outside a broadcast's mask may take any value: only rows 1 and 3
  // (then row 3) are read afterwards
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x142, 0xA, 0xF, false));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x143, 0xC, 0xF, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(v), lane));
}
__device__ __forceinline__ int readlane_i32(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
// Make a value that is equal in all lanes visibly wave-uniform, so that the
// branches on it are scalar branches.  The event dispatch below relies on
// this: compiled as a divergent if/else chain on a vector register, one of
// its arms (the y-wall reflection) lost its direction update.
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Lane `lane` of a, b, c replaced by the wave-uniform values va, vb, vc
// (v_writelane, lane select in M0: no compare and no change of the execution
// mask)
__device__ __forceinline__ void writelane3(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t va,
                                           uint32_t vb, uint32_t vc, int lane) {
  asm("v_writelane_b32 %0, %3, m0\n\t"
      "v_writelane_b32 %1, %4, m0\n\t"
      "v_writelane_b32 %2, %5, m0"
      : "+v"(a), "+v"(b), "+v"(c)
      : "s"(uniform_i32((int)va)), "s"(uniform_i32((int)vb)), "s"(uniform_i32((int)vc)),
        "{m0}"(lane));
}

// Lane holding the smallest key (s, id) among lanes with valid = true, where
// s >= 0 so that its bit pattern orders like its value.  -1 if none.
__device__ __forceinline__ int wave_argmin(double s, uint32_t id, bool valid) {
  uint64_t sb = (uint64_t)__double_as_longlong(s);
  unsigned hi = valid ? (unsigned)(sb >> 32) : 0xFFFFFFFFu;
  unsigned m = wave_min_u32(hi);
  if (m == 0xFFFFFFFFu) return -1;
  uint64_t mask = __ballot(valid && hi == m);
  int wl = __ffsll((unsigned long long)mask) - 1;
  mask &= mask - 1;
  if (mask) {  // equal high words: resolve on the full key
    uint64_t bs = readlane_u64(sb, wl);
    uint32_t bi = (uint32_t)readlane_i32((int)id, wl);
    while (mask) {
      int l = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      uint64_t ls = readlane_u64(sb, l);
      uint32_t li = (uint32_t)readlane_i32((int)id, l);
      if (ls < bs || (ls == bs && li < bi)) { bs = ls; bi = li; wl = l; }
    }
  }
  return wl;
}

// Minimum of a 32-bit value over the 64 lanes, left in every lane: DPP steps
// within rows of 16, then the gfx950 row-pair and half-wave swaps (no trip
// through a scalar register).
__device__ __forceinline__ unsigned wave_min_all(unsigned v) {
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));
  v = umin_(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));
  const auto r16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = umin_((unsigned)r16[0], (unsigned)r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return umin_((unsigned)r32[0], (unsigned)r32[1]);
}

// As wave_argmin, with the minimum of the high words kept in every lane.
// The argmin in two steps: argmin_key is the lane's key (the high word of s
// on valid lanes, all ones elsewhere); its wave minimum m is all ones exactly
// when no lane is valid, since a valid lane's high word (a non-negative
// distance) never is.  Given m below all ones, argmin_lane returns the lane.
__device__ __forceinline__ unsigned argmin_key(double s, bool valid) {
  return valid ? (unsigned)((uint64_t)__double_as_longlong(s) >> 32) : 0xFFFFFFFFu;
}
__device__ __forceinline__ int argmin_lane(double s, uint32_t id, unsigned hi, unsigned m) {
  const uint64_t sb = (uint64_t)__double_as_longlong(s);
  uint64_t mask = __builtin_amdgcn_ballot_w64(hi == m);  // not empty: some lane holds m
  int wl = __builtin_ctzll(mask);
  if (__builtin_expect(mask != (1ull << wl), 0)) {  // equal high words: resolve on the full key
    mask &= mask - 1;
    uint64_t bs = readlane_u64(sb, wl);
    uint32_t bi = (uint32_t)readlane_i32((int)id, wl);
    while (mask) {
      const int l = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const uint64_t ls = readlane_u64(sb, l);
      const uint32_t li = (uint32_t)readlane_i32((int)id, l);
      if (ls < bs || (ls == bs && li < bi)) { bs = ls; bi = li; wl = l; }
    }
  }
  return wl;
}
__device__ __forceinline__ int wave_argmin_all(double s, uint32_t id, bool valid) {
  const unsigned hi = argmin_key(s, valid);
  const unsigned m = wave_min_u32(hi);
  if (m == 0xFFFFFFFFu) return -1;
  return argmin_lane(s, id, hi, m);
}

// Event digest (a test device, not part of the method).  Event i of a cell's
// phase has the record r = bits(s) ^ id*K1 ^ kind<<56; the cell digest is the
// XOR over i of mix(r ^ i*K2), mix being the splitmix64 finaliser (Steele,
// Lea, Flood, OOPSLA 2014).  The XOR lets a wave hash 64 events at once.
constexpr uint64_t kDigestK1 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kDigestK2 = 0xD6E8FEB86659FD93ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t digest_term(int kind, uint64_t gid, double s, uint64_t i) {
  const uint64_t r = (uint64_t)__double_as_longlong(s) ^ (gid * kDigestK1) ^ ((uint64_t)kind << 56);
  return mix64(r ^ (i * kDigestK2));
}

// XOR of a 32-bit value over the 64 lanes, left in every lane.
__device__ __forceinline__ unsigned wave_xor_all(unsigned v) {
  v ^= (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
  v ^= (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
  v ^= (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);
  v ^= (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true);
  const auto r16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = (unsigned)r16[0] ^ (unsigned)r16[1];
  const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (unsigned)r32[0] ^ (unsigned)r32[1];
}

// Digest terms of the first `count` event records held one per lane (lane k:
// record of event first + k, in three 32-bit registers: the step's bits and
// kind << 29 | id, where a lift (kind 1) names its disk by the index into the
// cell's id-ordered list own_gid), XOR-ed over the wave.
__device__ __forceinline__ uint64_t digest_batch(uint32_t rec_lo, uint32_t rec_hi, uint32_t rec_tag,
                                                 int lane, int count, uint64_t first,
                                                 const int32_t* own_gid) {
  uint64_t t = 0;
  if (lane < count) {
    const uint64_t sb = ((uint64_t)rec_hi << 32) | rec_lo;
    const int kind = (int)(rec_tag >> 29);
    uint32_t id = rec_tag & 0x1FFFFFFFu;
    if (kind == 1) id = (uint32_t)own_gid[id];
    t = digest_term(kind, id, __longlong_as_double((long long)sb), first + (uint64_t)lane);
  }
  const uint32_t lo = (uint32_t)uniform_i32((int)wave_xor_all((uint32_t)t));
  const uint32_t hi = (uint32_t)uniform_i32((int)wave_xor_all((uint32_t)(t >> 32)));
  return ((uint64_t)hi << 32) | lo;
}

// The same hash of records whose ids are the disks' own (no index to turn
// into an id): the periodic cell's records.
__device__ __forceinline__ uint64_t digest_batch_ids(uint32_t rec_lo, uint32_t rec_hi, uint32_t rec_tag,
                                                     int lane, int count, uint64_t first) {
  uint64_t t = 0;
  if (lane < count) {
    const uint64_t sb = ((uint64_t)rec_hi << 32) | rec_lo;
    t = digest_term((int)(rec_tag >> 29), rec_tag & 0x1FFFFFFFu,
                    __longlong_as_double((long long)sb), first + (uint64_t)lane);
  }
  const uint32_t lo = (uint32_t)uniform_i32((int)wave_xor_all((uint32_t)t));
  const uint32_t hi = (uint32_t)uniform_i32((int)wave_xor_all((uint32_t)(t >> 32)));
  return ((uint64_t)hi << 32) | lo;
}

enum { EV_LIFT = 1, EV_FROZEN = 2, EV_WALL_X = 3, EV_WALL_Y = 4, EV_PSEUDO = 5, EV_END = 6 };

// Lifts among the first count event records held in the lanes.
__device__ __forceinline__ uint32_t count_lifts(uint32_t rec_tag, int lane, int count) {
  const bool is_lift = lane < count && (rec_tag >> 29) == (uint32_t)EV_LIFT;
  return (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(is_lift));
}

// Contact distance of a disk moving along unit d towards a disk at offset r:
// s = a - sqrt(sigma^2 - c^2) with a = r.d, c = r x d, for a > 0 and
// sigma^2 - c^2 > 0; negative values (touching disks) become 0.
// Correctly rounded square root of x in [2^-767, 2^1000] (Markstein's
// method: the hardware reciprocal square root estimate, one Newton step on
// (g, h) = (x y, y/2), then two corrections with the exact residual x - g^2
// from a fused multiply-add; P. Markstein, IBM J. Res. Dev. 34 (1990) 111).
// The general sqrt() adds range scaling and special-value selects; the
// contact term's argument sigma^2 - c^2, where positive, is at least about
// 2^-106 sigma^2, and sigma is limited to [2^-300, 2^300], so x stays in range.
__device__ __forceinline__ double sqrt_contact(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double dd = fma(-g, g, x);
  g = fma(dd, h, g);
  dd = fma(-g, g, x);
  return fma(dd, h, g);
}

__device__ __forceinline__ bool contact(double rx, double ry, double dx, double dy, double sig2,
                                        double& s) {
  double a = fma(rx, dx, ry * dy);
  double c = fma(rx, dy, -(ry * dx));
  double disc = fma(-c, c, sig2);
  // computed in every lane and selected (no branch): where disc <= 0 the
  // root is NaN or infinite and the lane is not a candidate
  const bool ok = a > 0.0 && disc > 0.0;
  const double t = a - sqrt_contact(disc);
  s = ok ? ((t < 0.0) ? 0.0 : t) : s;
  return ok;
}

// Shifted-frame coordinate in [0, L] and cell-local coordinate.
__device__ __forceinline__ double shifted(double p, double shift, double L) {
  double t = p - shift;
  if (t < 0.0) t += L;
  return t;
}
__device__ __forceinline__ double local_coord(double p, double shift, double origin, double L,
                                              double half_L) {
  double v = shifted(p, shift, L) - origin;
  if (v < -half_L) v += L;
  else if (v >= half_L) v -= L;
  return v;
}

// ---------------------------------------------------------------------------
// Start lattice
// ---------------------------------------------------------------------------
__global__ void k_lattice(const Dev* __restrict__ ds, int64_t k, double a) {
  const Dev& d = ds[blockIdx.y];
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= d.n) return;
  int64_t j = id / k, i = id % k;
  d.x[id] = ((double)i + ((j & 1) ? 0.75 : 0.25)) * a;
  d.y[id] = ((double)j + 0.5) * a;
}

// ---------------------------------------------------------------------------
// Rebin: sweep draws, cell of every disk, counting sort by cell
// ---------------------------------------------------------------------------
// Permutation number idx in [0, 24) decoded in the factorial base: the
// colour of phase q lands in bits 2q, 2q+1 of the result.  The colours not
// yet taken are kept in order as 2-bit fields of `avail`.
__device__ int32_t decode_perm(uint64_t idx) {
  uint32_t avail = 0 | (1u << 2) | (2u << 4) | (3u << 6);
  const uint32_t fact[4] = {6, 2, 1, 1};
  int32_t out = 0;
  uint32_t r = (uint32_t)idx;
#pragma unroll
  for (int pos = 0; pos < 4; ++pos) {
    const uint32_t q = r / fact[pos];
    r = r % fact[pos];
    out |= (int32_t)(((avail >> (2 * q)) & 3u) << (2 * pos));
    // drop field q: the fields above it move down by one
    const uint32_t low = avail & ((1u << (2 * q)) - 1u);
    avail = low | ((avail >> (2 * q + 2)) << (2 * q));
  }
  return out;
}

// squares = 0: the sweep's own decomposition (stripes for a striped system);
// 1: the square cells that the observables' rebin always uses.
__global__ void k_prep(const Dev* __restrict__ ds, int squares) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  const int nreg = kRegions * d.C * d.C;
  for (int c = threadIdx.x; c < nreg; c += blockDim.x) {
    d.reg_count[c] = 0;
    d.reg_fill[c] = 0;
  }
  if (threadIdx.x == 0) {
    Stream st(d.seed, kKindSweep, (uint64_t)sweep, (uint64_t)d.system, 0);
    SweepDraws dr;
    if (d.stripes && !squares) {
      // stripes: shift across them, and which of the two colours goes first
      dr.sx = u01(st.next()) * d.w;
      dr.sy = 0.0;
      dr.perm = (int32_t)draw_index(st, 2);
    } else {
      dr.sx = u01(st.next()) * d.w;
      dr.sy = u01(st.next()) * d.w;
      dr.perm = decode_perm(draw_index(st, 24));
    }
    dr.pad = 0;
    *d.draws = dr;
    d.digest_ring[sweep % kDigestRing] = 0;
    *d.queue = 0;  // ticket counter of the one-launch sweep
  }
}

__device__ __forceinline__ int cell_of_pos(const Dev& d, double px, double py, double sx,
                                           double sy) {
  int cx = (int)floor(shifted(px, sx, d.L) / d.w);
  int cy = (int)floor(shifted(py, sy, d.L) / d.w);
  if (cx > d.C - 1) cx = d.C - 1;
  if (cy > d.C - 1) cy = d.C - 1;
  return cy * d.C + cx;
}

// Region of a cell-local coordinate along one axis: 0 within the strip at the
// cell's low wall, 2 within the strip at its high wall, 1 between.
__device__ __forceinline__ int strip_of(double v, double w, double strip) {
  return v < strip ? 0 : (v >= w - strip ? 2 : 1);
}

__global__ void k_count(const Dev* __restrict__ ds, int squares) {
  const Dev& d = ds[blockIdx.y];
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  SweepDraws dr = *d.draws;
  int c, r = 0;  // cell and region (stripes and one periodic cell: region 0)
  if (d.stripes && !squares) {
    // stripe index from the coordinate across the stripes: horizontal stripes
    // (across = y) on even sweeps, vertical ones (across = x) on odd sweeps
    const double across = (*d.sweep_ctr & 1) ? d.x[i] : d.y[i];
    c = (int)floor(shifted(across, dr.sx, d.L) / d.w);
    if (c > d.C - 1) c = d.C - 1;
  } else {
    c = cell_of_pos(d, d.x[i], d.y[i], dr.sx, dr.sy);
    if (d.C > 1) {
      // the disk's region in its cell, from its cell-local coordinates (the
      // wall strips are what neighbouring cells stage as their frozen band)
      const int cx = c % d.C, cy = c / d.C;
      const double vx = shifted(d.x[i], dr.sx, d.L) - (double)cx * d.w;
      const double vy = shifted(d.y[i], dr.sy, d.L) - (double)cy * d.w;
      r = 3 * strip_of(vy, d.w, d.strip) + strip_of(vx, d.w, d.strip);
    }
  }
  d.cell_of[i] = c;
  d.reg_of[i] = (uint8_t)r;
  // one atomic per distinct (cell, region) of the wavefront: consecutive ids
  // are mostly neighbours in space, so a wave's disks fall into a few cells
  const int key = kRegions * c + r;
  uint64_t todo = __builtin_amdgcn_ballot_w64(true);
  while (todo) {
    const int leader = (int)__builtin_ctzll(todo);
    const int lk = __builtin_amdgcn_readlane(key, leader);
    const uint64_t same = __builtin_amdgcn_ballot_w64(key == lk) & todo;
    if ((threadIdx.x & 63) == (unsigned)leader) atomicAdd(&d.reg_count[lk], (int)__builtin_popcountll(same));
    todo &= ~same;
  }
}

// Exclusive prefix sum of the (cell, region) counts, one workgroup of 1024
// threads; a cell's start is that of its first region.  The counts are
// taken in tiles of 4,096, four consecutive counts per thread in one 16-byte
// access (the count and start arrays are 256-byte aligned), summed in the
// thread, then over the wave and over the 16 waves; the next tile's counts
// are loaded while the current one is summed.
__global__ void __launch_bounds__(1024) k_scan(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  constexpr int kTile = 4096;
  __shared__ int32_t wsum[16];
  const int ncell = d.C * d.C;
  const int nreg = kRegions * ncell;
  const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
  const int32_t* __restrict__ cnt = d.reg_count;
  int32_t* __restrict__ start = d.reg_start;
  auto load = [&](int base) __attribute__((always_inline)) {
    const int i0 = base + 4 * t;
    int4 v;
    if (i0 + 3 < nreg) {
      v = *(const int4*)(cnt + i0);
    } else {
      v.x = (i0 < nreg) ? cnt[i0] : 0;
      v.y = (i0 + 1 < nreg) ? cnt[i0 + 1] : 0;
      v.z = (i0 + 2 < nreg) ? cnt[i0 + 2] : 0;
      v.w = 0;
    }
    return v;
  };
  int4 v = load(0);
  int carry = 0;
  for (int base = 0; base < nreg; base += kTile) {
    const int4 cur = v;
    if (base + kTile < nreg) v = load(base + kTile);  // the next tile, in flight meanwhile
    const int tot = cur.x + cur.y + cur.z + cur.w;
    // inclusive sum of the thread totals over the wave
    int x = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int woff = 0, tile_total = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const int sw = wsum[w];
      woff += (w < wave) ? sw : 0;
      tile_total += sw;
    }
    const int e0 = carry + woff + (x - tot);
    const int4 out = make_int4(e0, e0 + cur.x, e0 + cur.x + cur.y, e0 + cur.x + cur.y + cur.z);
    const int i0 = base + 4 * t;
    if (i0 + 3 < nreg) {
      *(int4*)(start + i0) = out;
    } else {
      if (i0 < nreg) start[i0] = out.x;
      if (i0 + 1 < nreg) start[i0 + 1] = out.y;
      if (i0 + 2 < nreg) start[i0 + 2] = out.z;
    }
    // the cell starts: the one multiple of kRegions among the four, if any
    const int r0 = i0 % kRegions;
    const int k = (r0 == 0) ? 0 : kRegions - r0;
    if (k < 4 && i0 + k < nreg) {
      const int sv = (k == 0) ? out.x : ((k == 1) ? out.y : ((k == 2) ? out.z : out.w));
      d.cell_start[(i0 + k) / kRegions] = sv;
    }
    carry += tile_total;
    __syncthreads();  // every thread has read wsum before the next tile writes it
  }
  if (t == 0) {
    start[nreg] = carry;
    d.cell_start[ncell] = carry;
  }
}

__global__ void k_scatter(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int k = kRegions * d.cell_of[i] + (int)d.reg_of[i];
  // one atomic per distinct (cell, region) of the wavefront; each lane's slot
  // is the group's base plus its rank among the group's lanes (the order
  // inside a region is free: staging sorts a cell's ids)
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t todo = __builtin_amdgcn_ballot_w64(true);
  int slot = 0;
  while (todo) {
    const int leader = (int)__builtin_ctzll(todo);
    const int lk = __builtin_amdgcn_readlane(k, leader);
    const uint64_t same = __builtin_amdgcn_ballot_w64(k == lk) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(&d.reg_fill[lk], (int)__builtin_popcountll(same));
    base = __builtin_amdgcn_readlane(base, leader);
    if (k == lk) slot = base + (int)__builtin_popcountll(same & below);
    todo &= ~same;
  }
  d.cell_ids[d.reg_start[k] + slot] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Chain draws of a sweep (Sec. 3.4 step 5): one thread per chain computes the
// start index, drawn with replacement among the cell's n_c disks, and the
// isotropic direction.  Rejection loops are capped (kMaxDrawTries).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t chains_of(const Dev& d, int n_c) {
  if (n_c <= 0) return 0;
  return d.chains_per_cell > 0 ? d.chains_per_cell : n_c;
}
__device__ __forceinline__ int64_t chain_base(const Dev& d, int cell) {
  return d.chains_per_cell > 0 ? (int64_t)cell * d.chains_per_cell : (int64_t)d.cell_start[cell];
}

__device__ bool draw_index_capped(Stream& st, uint64_t n, uint64_t& out) {
  uint64_t x = st.next();
  uint64_t hi = __umul64hi(x, n), lo = x * n;
  if (lo < n) {
    uint64_t t = (0ull - n) % n;
    int tries = 0;
    while (lo < t) {
      if (++tries > kMaxDrawTries) return false;
      x = st.next();
      hi = __umul64hi(x, n);
      lo = x * n;
    }
  }
  out = hi;
  return true;
}

__device__ bool iso_direction_capped(const Dev& d, int64_t sweep, int cell, int64_t k, double& dx,
                                     double& dy) {
  Stream st(d.seed, kKindDir, (uint64_t)sweep, cell_key(d, cell), (uint64_t)k);
  for (int tries = 0; tries < kMaxDrawTries; ++tries) {
    double vx = 2.0 * u01(st.next()) - 1.0;
    double vy = 2.0 * u01(st.next()) - 1.0;
    double r2 = fma(vx, vx, vy * vy);
    if (r2 < 1.0 && r2 >= 0x1p-40) {
      double r = sqrt(r2);
      dx = vx / r;
      dy = vy / r;
      return true;
    }
  }
  dx = 1.0;
  dy = 0.0;
  return false;
}

// Cell whose range [cell_start[c], cell_start[c+1]) holds chain slot i.
__device__ __forceinline__ int cell_of_slot(const Dev& d, int64_t i) {
  int lo = 0, hi = d.C * d.C - 1;
  while (lo < hi) {  // largest c with cell_start[c] <= i
    int mid = (lo + hi + 1) >> 1;
    if ((int64_t)d.cell_start[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_draws(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  const int64_t total = d.chains_per_cell > 0 ? (int64_t)d.C * d.C * d.chains_per_cell : d.n;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int cell;
  int64_t k;
  if (d.chains_per_cell > 0) {
    cell = (int)(i / d.chains_per_cell);
    k = i % d.chains_per_cell;
  } else {
    cell = cell_of_slot(d, i);
    k = i - d.cell_start[cell];
  }
  int n_c = d.cell_start[cell + 1] - d.cell_start[cell];
  double dx, dy;
  bool ok = iso_direction_capped(d, sweep, cell, k, dx, dy);
  d.chain_dir[i] = make_double2(dx, dy);
  int32_t start = 0;
  if (n_c > 0 && d.start_mode == 0) {
    Stream st(d.seed, kKindStart, (uint64_t)sweep, cell_key(d, cell), (uint64_t)k);
    uint64_t v = 0;
    if (!draw_index_capped(st, (uint64_t)n_c, v)) ok = false;
    start = (int32_t)v;
  }
  if (d.start_mode == 0) d.chain_start[i] = start;
  if (!ok) atomicOr(d.err, ERR_DRAW_CAP);
}

// Distinct-start negative control: one thread per cell shuffles [0, n_c)
// (Fisher-Yates) and chain k starts at list[k mod n_c].
__global__ void k_shuffle(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  if (d.start_mode != 1) return;
  const int64_t sweep = *d.sweep_ctr;
  int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= d.C * d.C) return;
  int s0 = d.cell_start[cell];
  int n_c = d.cell_start[cell + 1] - s0;
  if (n_c <= 0) return;
  int32_t* list = d.shuffle + s0;
  for (int i = 0; i < n_c; ++i) list[i] = i;
  Stream st(d.seed, kKindShuffle, (uint64_t)sweep, cell_key(d, cell), 0);
  bool ok = true;
  for (int i = 0; i + 1 < n_c; ++i) {
    uint64_t v = 0;
    if (!draw_index_capped(st, (uint64_t)(n_c - i), v)) ok = false;
    int j = i + (int)v;
    int t = list[i]; list[i] = list[j]; list[j] = t;
  }
  int64_t n_m = chains_of(d, n_c);
  int64_t base = chain_base(d, cell);
  for (int64_t k = 0; k < n_m; ++k) d.chain_start[base + k] = list[k % n_c];
  if (!ok) atomicOr(d.err, ERR_DRAW_CAP);
}

// ---------------------------------------------------------------------------
// Walled simulation cells: one wavefront per active cell of colour perm[q]
// ---------------------------------------------------------------------------
// Meta word of a slot: an own disk's index into the cell's id-ordered list,
// or a frozen disk's id with the top bit set; all ones while staging finds
// the slot empty.
constexpr uint32_t kFrozenBit = 0x80000000u;
constexpr uint32_t kEmptySlot = 0xFFFFFFFFu;

// Lane of the smallest key (s, id) among the window's candidates, given the
// wave minimum mn of their high words hi (as argmin_lane); the ids are taken
// only on the rare path of equal high words: a frozen disk's from its meta
// word, an own disk's from the cell's id list.
__device__ __forceinline__ int argmin_lane_slots(double s, uint32_t m, const int32_t* own_gid,
                                                 unsigned hi, unsigned mn) {
  const uint64_t sb = (uint64_t)__double_as_longlong(s);
  uint64_t mask = __builtin_amdgcn_ballot_w64(hi == mn);  // not empty: some lane holds mn
  int wl = __builtin_ctzll(mask);
  if (__builtin_expect(mask != (1ull << wl), 0)) {  // equal high words: resolve on the full key
    uint32_t id = 0;
    if (hi == mn) id = (m & kFrozenBit) ? (m & ~kFrozenBit) : (uint32_t)own_gid[m];
    mask &= mask - 1;
    uint64_t bs = readlane_u64(sb, wl);
    uint32_t bi = (uint32_t)readlane_i32((int)id, wl);
    while (mask) {
      const int l = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const uint64_t ls = readlane_u64(sb, l);
      const uint32_t li = (uint32_t)readlane_i32((int)id, l);
      if (ls < bs || (ls == bs && li < bi)) { bs = ls; bi = li; wl = l; }
    }
  }
  return wl;
}

__device__ __forceinline__ int32_t load_err(const Dev& d) {
  return __hip_atomic_load(d.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// PREC 0: FP64 contact distances; PREC 1: FP32 screen, FP64 for the survivors.
// One active cell of colour phase q (Sec. 3.4, steps 3-6): stage the own
// disks and the frozen band into LDS, run the cell's chains, write back.  One
// wavefront; base is its LDS region.  Returns early, with d.err set, when a
// capacity check fails.  REJ 1: a chain that reaches a wall or a frozen disk
// is rejected and undone (the rejection variant of Sec. 3.4); every event then
// takes the general path, which logs each lift for the undo.
template <int PREC, int REJ>
__device__ __forceinline__ void phase_cell(const Dev& d, const int64_t sweep, const SweepDraws& dr,
                                           const int q, const int blk, unsigned char* const base,
                                           const int lane) {
  const int half = d.C >> 1;
  const int colour = (dr.perm >> (2 * (q & 3))) & 3;
  const int cx = 2 * (blk % half) + (colour & 1);
  const int cy = 2 * (blk / half) + (colour >> 1);
  const int cell = cy * d.C + cx;
  const double ox = (double)cx * d.w, oy = (double)cy * d.w;
  const double L = d.L, half_L = d.half_L, w = d.w, sigma = d.sigma, sig2 = d.sig2;
  const int gridb = d.gridb, nb = d.nb;
  const int nslots = gridb * gridb;  // one slot per bin
  // bin coordinates of a slot: by = floor(slot / gridb) as (slot * m) >> 20
  // with m = ceil(2^20 / gridb), exact for slot < gridb^2 when gridb^3 < 2^20
  // (the host limits gridb to 100)
  const uint32_t inv_g20 = ((1u << 20) + (uint32_t)gridb - 1u) / (uint32_t)gridb;
  auto slot_bin = [&](int slot, int& bx, int& by) __attribute__((always_inline)) {
    by = (int)(((uint32_t)slot * inv_g20) >> 20);
    bx = slot - by * gridb;
  };

  const CellLds lay = cell_lds_layout(gridb, d.cap_own, REJ == 1);
  double2* pos = (double2*)(base + lay.off_pos);
  uint32_t* meta = (uint32_t*)(base + lay.off_meta);
  int32_t* own_gid = (int32_t*)(base + lay.off_own_gid);
  int32_t* own_loc = (int32_t*)(base + lay.off_own_loc);
  // the id staging buffer of the rank sort lies in the position slots, which
  // are filled only after the sort
  int32_t* tmp = (int32_t*)(base + lay.off_pos);
  // per-lane sink slots: lanes that have nothing to store write here, so a
  // store by one or two lanes needs no change of the execution mask
  double2* const sink = (double2*)(base + lay.off_sink) + lane;
  uint32_t* const sink32 = (uint32_t*)sink;
  // REJ 1 only: per logged lift the old position, then (slot before, slot after)
  double2* undo_pos = (double2*)(base + lay.off_undo);
  int2* undo_slot = (int2*)(undo_pos + kUndoCap);

  // ---- stage: own disks, sorted by id -----------------------------------
  const int start = d.cell_start[cell];
  const int n_own = d.cell_start[cell + 1] - start;
  if (n_own < 0 || n_own > d.cap_own || start < 0 || (int64_t)start + n_own > d.n) {
    if (lane == 0) atomicOr(d.err, ERR_OWN_CAP);
    return;
  }
  for (int i = lane; i < n_own; i += 64) tmp[i] = d.cell_ids[start + i];
  wave_sync();
  for (int i = lane; i < n_own; i += 64) {
    int v = tmp[i];
    int r = 0;
    for (int j = 0; j < n_own; ++j) r += (tmp[j] < v) ? 1 : 0;
    own_gid[r] = v;
  }
  wave_sync();
  const double2 nan2 = make_double2(__builtin_nan(""), __builtin_nan(""));
  for (int s = lane; s < nslots; s += 64) {
    pos[s] = nan2;
    meta[s] = kEmptySlot;
  }
  wave_sync();

  // own disks into bins 2..nb+1: a bin's diagonal is below sigma, so it holds
  // at most one centre of a configuration without overlaps (a second one is
  // reported as a capacity error)
  for (int k = lane; k < n_own; k += 64) {
    int g = own_gid[k];
    double vx = local_coord(d.x[g], dr.sx, ox, L, half_L);
    double vy = local_coord(d.y[g], dr.sy, oy, L, half_L);
    int bx = (int)floor(vx * d.inv_b) + 2, by = (int)floor(vy * d.inv_b) + 2;
    bx = bx < 2 ? 2 : (bx > nb + 1 ? nb + 1 : bx);
    by = by < 2 ? 2 : (by > nb + 1 ? nb + 1 : by);
    const int s = by * gridb + bx;
    if (atomicCAS(&meta[s], kEmptySlot, (uint32_t)k) != kEmptySlot) {
      atomicOr(d.err, ERR_BIN_CAP);
      continue;
    }
    pos[s] = make_double2(vx, vy);
    own_loc[k] = s;
  }
  // frozen disks: centres of the 8 neighbouring cells within sigma of this
  // cell, in the two outer rings of bins.  Only a neighbour's regions that
  // face this cell are read (its wall strips are wider than sigma, so they
  // hold every such centre): the strip along the shared wall of an edge
  // neighbour, the corner region of a diagonal one.  A region row is one
  // range of the list, a region column three.
  for (int nbh = 0; nbh < 9; ++nbh) {
    if (nbh == 4) continue;
    const int ox_ = nbh % 3 - 1, oy_ = nbh / 3 - 1;  // neighbour at (cx + ox_, cy + oy_)
    int ncx = (cx + ox_ + d.C) % d.C;
    int ncy = (cy + oy_ + d.C) % d.C;
    int nc = ncy * d.C + ncx;
    // its strips facing this cell: the low strip of a neighbour above or to
    // the right, the high strip of one below or to the left, all three
    // across an edge it shares
    const int rx0 = ox_ > 0 ? 0 : (ox_ < 0 ? 2 : 0), rx1 = ox_ > 0 ? 0 : 2;
    const int ry0 = oy_ > 0 ? 0 : (oy_ < 0 ? 2 : 0), ry1 = oy_ > 0 ? 0 : 2;
    for (int ry = ry0; ry <= ry1; ++ry) {
    const int k0 = kRegions * nc + 3 * ry;
    int s0 = d.reg_start[k0 + rx0], s1 = d.reg_start[k0 + rx1 + 1];
    if (s0 < 0 || s1 < s0 || s1 - s0 > d.cap_own || (int64_t)s1 > d.n) {
      if (lane == 0) atomicOr(d.err, ERR_OWN_CAP);
      return;
    }
    for (int i = s0 + lane; i < s1; i += 64) {
      int g = d.cell_ids[i];
      double vx = local_coord(d.x[g], dr.sx, ox, L, half_L);
      double vy = local_coord(d.y[g], dr.sy, oy, L, half_L);
      if (vx >= -sigma && vx <= w + sigma && vy >= -sigma && vy <= w + sigma) {
        int bx = (int)floor(vx * d.inv_b) + 2, by = (int)floor(vy * d.inv_b) + 2;
        bx = bx < 0 ? 0 : (bx > nb + 3 ? nb + 3 : bx);
        by = by < 0 ? 0 : (by > nb + 3 ? nb + 3 : by);
        const int s = by * gridb + bx;
        if (atomicCAS(&meta[s], kEmptySlot, (uint32_t)g | kFrozenBit) != kEmptySlot) {
          atomicOr(d.err, ERR_BIN_CAP);
          continue;
        }
        pos[s] = make_double2(vx, vy);
      }
    }
    }  // region rows
  }
  wave_sync();
  if (load_err(d) != 0) return;  // a capacity check failed somewhere: do not run chains

  // ---- chains --------------------------------------------------------------
  const int64_t n_m = chains_of(d, n_own);
  const int64_t cbase = chain_base(d, cell);
  double acc = d.acc_delta[cell];
  uint32_t n_lift = 0, n_frozen = 0, n_wall = 0;
  uint64_t h = 0;
  int n_ring = 0;            // event records held in the lanes (lane k: record k)
  uint64_t ring_first = 0;    // digest index of record 0
  uint32_t rec_lo = 0, rec_hi = 0, rec_tag = 0;
  // lane = lx + 8 ly: one bin of an 8 x 8 window per lane, a window row in 8
  // neighbouring lanes
  const int lx = lane & 7, ly = lane >> 3;
  const int loff = ly * gridb + lx;  // this lane's slot inside a window
  const double inv_b = d.inv_b;
  // A window of 8 x 8 bins reaches 2 bins behind the moving disk's bin and 5
  // ahead of it along each axis (clamped windows only add room, since nothing
  // is staged beyond the outer bins).  With sigma/2 < b < sigma/sqrt(2), the
  // 2b behind cover sigma, and a move of length t keeps its
  // sigma-neighbourhood inside the window whenever t * max(|dx|, |dy|) <=
  // 5b - sigma - eps: then no disk outside the window can be hit first, and
  // the event found in the window is exact.
  const double eps = 1e-9 * sigma;
  const double reach = 5.0 * d.b - sigma - eps;
  // a plain lift keeps the moved centre in [wlo, whi] on both axes (see there)
  const double wlo = eps, whi = w - eps;
  const bool use_window = d.search == 0;
  const uint64_t wall_x_id = (uint64_t)d.n, wall_y_id = (uint64_t)d.n + 1, end_id = (uint64_t)d.n + 3;
  int aborted = 0;
  int stop = 0;  // nonzero once a poll sees the device error word set

  // draws of chain 0; later, those of chain k + 1 and the device error word
  // are loaded while chain k runs (their latency is then hidden)
  int32_t nxt_start = n_m > 0 ? d.chain_start[cbase] : 0;
  double2 nxt_dir = n_m > 0 ? d.chain_dir[cbase] : make_double2(1.0, 0.0);
  int32_t nxt_err = load_err(d);
  for (int64_t k = 0; k < n_m && aborted == 0; ++k) {
    int j = uniform_i32(nxt_start);
    if (j < 0 || j >= n_own) j = 0;  // guarded: the draw kernel writes indices below n_own
    const double2 dir = nxt_dir;
    double dx = dir.x, dy = dir.y;
    stop = uniform_i32(nxt_err);
    if (k + 1 < n_m) {
      nxt_start = d.chain_start[cbase + k + 1];
      nxt_dir = d.chain_dir[cbase + k + 1];
    }
    nxt_err = load_err(d);
    // per-direction constants
    double idx, idy, wallx, wally, idxw, idyw, dsafe;
    int xneg, yneg;
#define EC_SET_DIRECTION()                                                          \
    do {                                                                            \
      idx = (dx != 0.0) ? 1.0 / dx : 0.0;                                           \
      idy = (dy != 0.0) ? 1.0 / dy : 0.0;                                           \
      wallx = (dx > 0.0) ? w : ((dx < 0.0) ? 0.0 : INFINITY);                       \
      wally = (dy > 0.0) ? w : ((dy < 0.0) ? 0.0 : INFINITY);                       \
      idxw = (dx != 0.0) ? idx : 1.0;                                               \
      idyw = (dy != 0.0) ? idy : 1.0;                                               \
      /* reach / max(|dx|, |dy|) as reach * min(|1/dx|, |1/dy|) (a 0 component    */ \
      /* has a factor 1, and then the other is +-1); a few ulps off, far below     */ \
      /* the eps the reach keeps in hand, and only ever a guard                     */ \
      dsafe = use_window ? reach * fmin(fabs(idxw), fabs(idyw)) : -1.0;             \
      xneg = uniform_i32(dx < 0.0 ? 1 : 0);                                         \
      yneg = uniform_i32(dy < 0.0 ? 1 : 0);                                         \
    } while (0)
    // origin bin of the 8 x 8-bin window around bin (bx, by): two bins behind
    // the disk and five ahead of it along each axis, clamped to the grid
#define EC_WINDOW(bx, by, xn, yn)                                                   \
    do {                                                                            \
      wx0 = (bx) - 2 - 3 * (xn);                                                    \
      wy0 = (by) - 2 - 3 * (yn);                                                    \
      wx0 = max(min(wx0, gridb - 8), 0);                                            \
      wy0 = max(min(wy0, gridb - 8), 0);                                            \
      wbase = wy0 * gridb + wx0;                                                    \
    } while (0)
    EC_SET_DIRECTION();
    int a_loc = uniform_i32(own_loc[j]);
    int a_lidx = j;
    const double2 ap = pos[a_loc];
    double ax = ap.x, ay = ap.y;
    double rem = d.ell;
    // event cap and abort polling, both at the digest flush (every 64 events
    // of the cell): the error word loaded at the previous flush (or chain
    // start) is read, the next load is issued, and the chain's event count,
    // ring_first - ev0 at a flush, is held against the cap (so a chain makes
    // at most kMaxEventsPerChain + 63 events)
    const uint64_t ev0 = ring_first + (uint64_t)n_ring;
    int capped = 0;
#define EC_POLL()                                                                   \
    do {                                                                            \
      stop |= uniform_i32(nxt_err);                                                 \
      nxt_err = load_err(d);                                                        \
      capped = (ring_first - ev0 >= (uint64_t)kMaxEventsPerChain) ? 1 : 0;          \
    } while (0)
    // REJ 1: the chain's undo log, contact sum and lifts (counted once accepted)
    int n_undo = 0;
    double chain_acc = 0.0;
    uint32_t chain_lifts = 0;
    int wx0, wy0, wbase;
    {
      int bx0, by0;
      slot_bin(a_loc, bx0, by0);
      EC_WINDOW(bx0, by0, xneg, yneg);
    }
    int widx = wbase + loff;  // this lane's slot in the window
    double2 p = pos[widx];
    uint32_t m = meta[widx];
    int ended = 0;  // the chain length is used up

    while (ended == 0 && stop == 0 && capped == 0) {
      // the event found, and the decision (also read by the general path)
      double tx, ty, best_s, wpx, wpy, e, step, nax, nay;
      uint32_t wm;  // meta word of the nearest disk: own index, or id | frozen bit
      int w_bx, w_by, w_slot, packed;
      // (a disk can be hit exactly when best_s is finite)
      // Plain lifts run in this inner loop, where the direction and its
      // derived constants do not change: the general path, which can change
      // them, sits outside it, so the common event needs no register copies
      // where the two paths would otherwise join.  The loop leaves as soon as
      // an event is not a plain lift, or after a poll that stops the chain.
      // distances to the walls of the cell ahead: (wall - v) / d with 1/d
      // precomputed, clamped at 0
#define EC_WALLS()                                                                  \
      do {                                                                          \
        tx = (wallx - ax) * idxw;                                                   \
        tx = (tx < 0.0) ? 0.0 : tx;                                                 \
        ty = (wally - ay) * idyw;                                                   \
        ty = (ty < 0.0) ? 0.0 : ty;                                                 \
      } while (0)
      // One plain-lift event; false on any other event (left to the general
      // path) and after a poll that stops the chain.  The loop runs two per
      // pass, so that the common event takes a taken branch only every other
      // time; every return is a constant, so each exit is a plain branch.
      auto plain_event = [&]() __attribute__((always_inline)) -> bool {

      // -- contact distance of the disk in this lane's window slot
      double s = 0.0;
      bool valid;
      if (PREC == 0) {
        valid = contact(p.x - ax, p.y - ay, dx, dy, sig2, s);
      } else {
        // FP32 screen: lanes whose FP32 terms prove the FP64 test fails drop
        // out; lanes whose FP32 distance is certain to within scr_e of the
        // FP64 one drop out when they cannot be the minimum; the rest (the
        // survivors) get the FP64 distance.  The minimum over the survivors
        // is then the FP64 minimum over the window.
        // the FP32 coordinates are those of the FP64 slot position, rounded
        const float rx = (float)p.x - (float)ax, ry = (float)p.y - (float)ay;
        const float dx32 = (float)dx, dy32 = (float)dy;
        const float a32 = fmaf(rx, dx32, ry * dy32);
        const float c32 = fmaf(rx, dy32, -(ry * dx32));
        const float disc32 = fmaf(-c32, c32, (float)sig2);
        const bool maybe = a32 > -d.scr_ea && disc32 > -d.scr_ed;
        const bool sure = a32 > d.scr_ea && disc32 > d.scr_dg;
        const float s32 = fmaxf(a32 - __builtin_amdgcn_sqrtf(disc32), 0.0f);
        const float hi = sure ? s32 + d.scr_e : INFINITY;
        const float bound = __uint_as_float(wave_min_all(__float_as_uint(hi)));
        const bool survivor = maybe && (!sure || s32 - d.scr_e <= bound);
        valid = false;
        if (survivor) valid = contact(p.x - ax, p.y - ay, dx, dy, sig2, s);
      }
      // The plain-lift test (the conditions are listed where its result is
      // read) made by every lane on its own candidate while the wave minimum
      // forms, so that it fills the DPP hazard slots; only the winning lane's
      // result is used, computed with the winner's own values.  The lane also
      // forms the slot of the moved centre's bin.
      int plain_l, nslot_l;
      {
        const double nxl = fma(s, dx, ax), nyl = fma(s, dy, ay);
        const int bxl = (int)(nxl * inv_b) + 2, byl = (int)(nyl * inv_b) + 2;
        plain_l = (int)((m & kFrozenBit) == 0) & (int)(s < rem) & (int)(s <= dsafe) &
                  (int)(nxl >= wlo) & (int)(nxl <= whi) & (int)(nyl >= wlo) & (int)(nyl <= whi);
        nslot_l = byl * gridb + bxl;
        asm volatile("" : : "v"(plain_l));  // keep it here, beside the wave minimum
      }
      const unsigned key = argmin_key(s, valid);
      const unsigned key_min = wave_min_u32(key);
      if (__builtin_expect(key_min == 0xFFFFFFFFu, 0)) {
        // no disk in the window: the general path decides (a wall, the chain
        // end, or, where the window cannot vouch, a search of every slot);
        // the nearest disk's other values are read there only for a disk
        best_s = INFINITY;
        wm = kFrozenBit;
        return false;
      }
      {
      // the nearest disk
      const int wls = argmin_lane_slots(s, m, own_gid, key, key_min);
      best_s = readlane_f64(s, wls);
      wm = (uint32_t)readlane_i32((int)m, wls);
      wpx = readlane_f64(p.x, wls);
      wpy = readlane_f64(p.y, wls);
      w_bx = wx0 + (wls & 7);
      w_by = wy0 + (wls >> 3);
      w_slot = readlane_i32(widx, wls);

      // the decision, made in vector registers and moved to the scalar unit once
#define EC_DECIDE(CHECK_WINDOW)                                                     \
      do {                                                                          \
        int kd = (best_s < INFINITY) ? ((wm & kFrozenBit) ? EV_FROZEN : EV_LIFT) : 0; \
        e = best_s;                                                                 \
        if (tx < e) { e = tx; kd = EV_WALL_X; }                                     \
        if (ty < e) { e = ty; kd = EV_WALL_Y; }                                     \
        const bool en = !(e < rem);                                                 \
        step = en ? rem : e;                                                        \
        nax = fma(step, dx, ax);                                                    \
        nay = fma(step, dy, ay);                                                    \
        /* bin of the moved centre, unclamped: a centre lies in [0, w], where    */ \
        /* truncation gives bins 2..nb+1, and nb + 2 only on the far wall (or    */ \
        /* one rounding past it); that case counts as a bin change and the      */ \
        /* general path clamps it                                               */ \
        const int bx_ = (int)(nax * inv_b) + 2;                                     \
        const int by_ = (int)(nay * inv_b) + 2;                                     \
        bool ok_ = true;                                                            \
        if (CHECK_WINDOW) ok_ = step <= dsafe;                                      \
        const int cr_ = (bx_ != abx || by_ != aby) ? 1 : 0;                          \
        packed = uniform_i32(bx_ | (by_ << 8) | (kd << 16) | ((en ? 1 : 0) << 20) | \
                             ((ok_ ? 1 : 0) << 21) | (cr_ << 22));                  \
      } while (0)
      // The common event, a plain lift: the nearest disk (not frozen) is hit
      // within the remaining chain length, the window vouches for the move,
      // and the moved centre stays inside the cell by the margin wmargin on
      // both axes, so neither wall comes first (with the wall distance
      // (wall - v) / d rounded as the full decision rounds it, a centre that
      // stops wmargin short of the wall leaves the wall farther by far more
      // than the rounding); the centre may change bin.  This is exactly the
      // full decision (EC_DECIDE) finding such a lift; the general path makes
      // the full decision for every other event.
      nax = fma(best_s, dx, ax);
      nay = fma(best_s, dy, ay);
      const int nslot = readlane_i32(nslot_l, wls);
      // any other event goes to the general path
      if (__builtin_expect(REJ == 1 || readlane_i32(plain_l, wls) == 0, 0)) return false;
      {
        {
          const uint64_t sb = (uint64_t)__double_as_longlong(best_s);
          // (the disk of a plain lift is not frozen: its meta word is its own
          // index, turned into its id when the records are hashed)
          const uint32_t tag = ((uint32_t)EV_LIFT << 29) | wm;
          writelane3(rec_lo, rec_hi, rec_tag, (uint32_t)sb, (uint32_t)(sb >> 32), tag, n_ring);
        }
        {
          double2* const dst = (lane == 0) ? pos + a_loc : sink;
          *dst = make_double2(nax, nay);
        }
        if (__builtin_expect(nslot != a_loc, 0)) {
          // the moved centre crossed into another bin, which is empty (a bin
          // holds one centre): lane 0 empties the old slot (over the store
          // above: LDS stores of a wave land in order), lane 1 fills the new
          // one, then lane 0 moves the meta word and lane 1 the slot index
          double2* const dst = (lane == 0) ? pos + a_loc : ((lane == 1) ? pos + nslot : sink);
          *dst = (lane == 0) ? nan2 : make_double2(nax, nay);
          uint32_t* const dm = (lane == 0) ? meta + nslot : ((lane == 1) ? (uint32_t*)own_loc + a_lidx : sink32);
          *dm = (lane == 0) ? (uint32_t)a_lidx : (uint32_t)nslot;
        }
        __builtin_amdgcn_wave_barrier();
        acc = acc + fma(wpx - nax, dx, (wpy - nay) * dy);
        rem = rem - best_s;
        a_loc = w_slot;
        a_lidx = (int)wm;
        ax = wpx;
        ay = wpy;
        EC_WINDOW(w_bx, w_by, xneg, yneg);
        widx = wbase + loff;
        p = pos[widx];
        m = meta[widx];
        if (__builtin_expect(++n_ring == kDigestBatch, 0)) {
          h ^= digest_batch(rec_lo, rec_hi, rec_tag, lane, kDigestBatch, ring_first, own_gid);
          if (REJ == 0) n_lift += count_lifts(rec_tag, lane, kDigestBatch);
          ring_first += kDigestBatch;
          n_ring = 0;
          EC_POLL();
          if (stop != 0 || capped != 0) return false;
        }
      }
      }  // a disk in the window
      return true;
      };
      for (;;) {
        if (__builtin_expect(!plain_event(), 0)) break;
        if (__builtin_expect(!plain_event(), 0)) break;
      }  // plain lifts
      if (stop != 0 || capped != 0) continue;  // leaves the event loop
      {
      // the mover's bin (the plain-lift loop carries only its slot)
      int abx, aby;
      slot_bin(a_loc, abx, aby);
      EC_WALLS();
      EC_DECIDE(true);
      if (__builtin_expect(((packed >> 21) & 1) == 0, 0)) {
        // the window cannot vouch for this event: exact search over every slot
        double ls = INFINITY;
        uint32_t lid = 0xFFFFFFFFu;
        int lslot = -1;
        for (int sl = lane; sl < nslots; sl += 64) {
          const double2 q2 = pos[sl];
          double s2;
          if (contact(q2.x - ax, q2.y - ay, dx, dy, sig2, s2)) {
            const uint32_t m2 = meta[sl];
            const uint32_t i2 = (m2 & kFrozenBit) ? (m2 & ~kFrozenBit) : (uint32_t)own_gid[m2];
            if (s2 < ls || (s2 == ls && i2 < lid)) { ls = s2; lid = i2; lslot = sl; }
          }
        }
        const int fl = wave_argmin_all(ls, lid, lslot >= 0);
        best_s = INFINITY;
        wm = kFrozenBit;
        if (fl >= 0) {
          best_s = readlane_f64(ls, fl);
          w_slot = readlane_i32(lslot, fl);
          wm = (uint32_t)uniform_i32((int)meta[w_slot]);
          w_bx = w_slot % gridb;
          w_by = w_slot / gridb;
          // read into scalar registers here, so no load is left in flight
          // where this rare path rejoins the event path
          const double2 q2 = pos[w_slot];
          wpx = readlane_f64(q2.x, 0);
          wpy = readlane_f64(q2.y, 0);
        }
        EC_DECIDE(false);
      }
#undef EC_DECIDE
#undef EC_WALLS
      const int kind = (packed >> 16) & 7;
      const bool ends = ((packed >> 20) & 1) != 0;
      const int nbx = min(packed & 0xFF, nb + 1), nby = min((packed >> 8) & 0xFF, nb + 1);
      // REJ 1: a wall or a frozen disk rejects the chain
      const bool rejected = REJ == 1 && !ends && kind != EV_LIFT;
      const double pax = ax, pay = ay;  // position before this event's move
      ax = nax;
      ay = nay;
      // event record for the digest: bits of the step, kind << 29 | id (an own
      // disk by its own index, turned into its id when the records are hashed)
      const uint32_t eid = ends ? (uint32_t)end_id
                                : (kind == EV_WALL_X ? (uint32_t)wall_x_id
                                                     : (kind == EV_WALL_Y ? (uint32_t)wall_y_id
                                                                          : (wm & ~kFrozenBit)));
      {
        // lane n_ring keeps this event's record (lane writes, no change of
        // the execution mask)
        const uint64_t sb = (uint64_t)__double_as_longlong(step);
        const uint32_t tag = ((uint32_t)(ends ? EV_END : kind) << 29) | eid;
        writelane3(rec_lo, rec_hi, rec_tag, (uint32_t)sb, (uint32_t)(sb >> 32), tag, n_ring);
      }
      if (REJ == 1 && !rejected && !ends) {
        // log the lift's move: slot before it and old position (the slot after
        // it is known below); a full log stops the sweep with an error
        if (n_undo == kUndoCap) {
          if (lane == 0) atomicOr(d.err, ERR_UNDO_CAP);
          stop = 1;
        } else if (lane == 0) {
          undo_pos[n_undo] = make_double2(pax, pay);
          undo_slot[n_undo] = make_int2(a_loc, a_loc);
        }
      }
      if (rejected) {
        // undo every logged lift, latest first: each disk goes back to the
        // slot it left (a slot vacated in between was refilled only by moves
        // that are undone before it) and to its old position
        if (lane == 0) {
          for (int u = n_undo - 1; u >= 0; --u) {
            const int2 sl = undo_slot[u];
            const double2 old = undo_pos[u];
            if (sl.y != sl.x) {
              const uint32_t mv = meta[sl.y];
              pos[sl.y] = nan2;
              meta[sl.x] = mv;
              own_loc[(int)mv] = sl.x;
            }
            pos[sl.x] = old;
          }
        }
        n_undo = 0;
        if (kind == EV_FROZEN) n_frozen += 1;
        else n_wall += 1;
      } else
      // store the moved disk; move it to another bin if it crossed a bin edge
      if (nbx == abx && nby == aby) {
        double2* const dst = (lane == 0) ? pos + a_loc : sink;
        *dst = make_double2(ax, ay);
      } else {
        const int ns = nby * gridb + nbx;
        const bool free_ = __builtin_isnan(readlane_f64(pos[ns].x, 0));
        if (__builtin_expect(!free_, 0)) {
          if (lane == 0) {
            atomicOr(d.err, ERR_BIN_CAP);
            pos[a_loc] = make_double2(ax, ay);
          }
        } else {
          if (lane == 0) {
            pos[a_loc] = nan2;
            pos[ns] = make_double2(ax, ay);
            meta[ns] = (uint32_t)a_lidx;
            own_loc[a_lidx] = ns;
          }
          a_loc = ns;
          abx = nbx;
          aby = nby;
        }
      }
      if (REJ == 1 && !rejected && !ends && stop == 0) {
        if (lane == 0) undo_slot[n_undo].y = a_loc;  // the slot the disk now holds
        n_undo += 1;
      }
      __builtin_amdgcn_wave_barrier();
      if (__builtin_expect(++n_ring == kDigestBatch, 0)) {
        h ^= digest_batch(rec_lo, rec_hi, rec_tag, lane, kDigestBatch, ring_first, own_gid);
          if (REJ == 0) n_lift += count_lifts(rec_tag, lane, kDigestBatch);
        ring_first += kDigestBatch;
        n_ring = 0;
        EC_POLL();
      }
      if (rejected) {
        ended = 1;
      } else if (!ends && kind == EV_LIFT) {
        // straight chain: the hit disk goes on in the same direction
        if (REJ == 1) {
          chain_acc = chain_acc + fma(wpx - ax, dx, (wpy - ay) * dy);
          chain_lifts += 1;
        } else {
          acc = acc + fma(wpx - ax, dx, (wpy - ay) * dy);
        }
        rem = rem - e;
        a_loc = w_slot;
        a_lidx = (int)wm;
        abx = w_bx;
        aby = w_by;
        ax = wpx;
        ay = wpy;
      } else if (__builtin_expect(ends, 0)) {
        ended = 1;
        if (REJ == 1) {  // accepted: its contact sum and lifts count
          acc = acc + chain_acc;
          n_lift += chain_lifts;
        }
      } else {
        rem = rem - e;
        if (__builtin_expect(kind == EV_FROZEN, 1)) {
          // mirror the direction about the contact normal
          const double rx = wpx - ax, ry = wpy - ay;
          acc = acc + fma(rx, dx, ry * dy);
          n_frozen += 1;
          // (both square roots are correctly rounded; their arguments, about
          // sigma^2 and 1, lie in the range of sqrt_contact)
          const double nrm = sqrt_contact(fma(rx, rx, ry * ry));
          const double nx = rx / nrm, ny = ry / nrm;
          const double dn = fma(dx, nx, dy * ny);
          const double tt = -2.0 * dn;
          const double ux = fma(tt, nx, dx), uy = fma(tt, ny, dy);
          const double mm = sqrt_contact(fma(ux, ux, uy * uy));
          dx = ux / mm;
          dy = uy / mm;
          EC_SET_DIRECTION();
        } else {
          // a wall: reverse the normal component of the direction
          n_wall += 1;
          if (kind == EV_WALL_X) {
            dx = -dx; idx = -idx; idxw = -idxw; wallx = w - wallx; xneg ^= 1;
          } else {
            dy = -dy; idy = -idy; idyw = -idyw; wally = w - wally; yneg ^= 1;
          }
        }
      }
      // window of the next event (the stores above are seen: LDS operations
      // of one wave complete in order)
      EC_WINDOW(abx, aby, xneg, yneg);
      widx = wbase + loff;
      p = pos[widx];
      m = meta[widx];
      }
    }
#undef EC_POLL
    if (ended == 0) {
      // stopped by another wave's error, or this chain reached the event cap
      if (stop == 0 && lane == 0) {
        atomicOr(d.err, ERR_EVENT_CAP);
        if (atomicAdd(d.err + 1, 1) == 0) {
          double* g = d.dbg;
          g[0] = (double)cell; g[1] = (double)k; g[2] = (double)sweep; g[3] = (double)q;
          g[4] = ax; g[5] = ay; g[6] = dx; g[7] = dy; g[8] = rem; g[9] = (double)a_loc;
          g[10] = (double)own_gid[a_lidx]; g[11] = (double)n_own;
        }
      }
      aborted = 1;
    }
#undef EC_WINDOW
#undef EC_SET_DIRECTION
  }

  // ---- write back: old position + local displacement, wrapped --------------
  wave_sync();
  h ^= digest_batch(rec_lo, rec_hi, rec_tag, lane, n_ring, ring_first, own_gid);
  if (REJ == 0) n_lift += count_lifts(rec_tag, lane, n_ring);
  // The cell's id list is sorted again by the regions of the moved disks:
  // the neighbours of later colour phases stage their frozen band from the
  // regions that face them.  The list keeps its range [start, start + n_own)
  // (disks stay in their cell), and the region starts are rewritten; both
  // are published with the positions.  LDS: the meta words are free now and
  // hold the 9 region counts and the 9 fill cursors; own_loc takes each
  // disk's region once its slot has been read.
  uint32_t* const rcnt = meta;
  if (lane < 2 * kRegions) rcnt[lane] = 0u;
  wave_sync();
  for (int k = lane; k < n_own; k += 64) {
    int g = own_gid[k];
    double2 v = pos[own_loc[k]];
    double px = d.x[g], py = d.y[g];
    double v0x = local_coord(px, dr.sx, ox, L, half_L);
    double v0y = local_coord(py, dr.sy, oy, L, half_L);
    double nx = px + (v.x - v0x);
    double ny = py + (v.y - v0y);
    if (nx < 0.0) nx += L; else if (nx >= L) nx -= L;
    if (ny < 0.0) ny += L; else if (ny >= L) ny -= L;
    d.x[g] = nx;
    d.y[g] = ny;
    // (from the cell-local position, which differs from the one a neighbour
    // computes from (nx, ny) by a few ulps of L, far inside the strip margin)
    const int r = 3 * strip_of(v.y, w, d.strip) + strip_of(v.x, w, d.strip);
    own_loc[k] = r;
    atomicAdd(&rcnt[r], 1u);
  }
  wave_sync();
  if (lane == 0) {
    uint32_t run = (uint32_t)start;
    for (int r = 0; r < kRegions; ++r) {
      d.reg_start[kRegions * cell + r] = (int32_t)run;
      rcnt[kRegions + r] = run;
      run += rcnt[r];
    }
  }
  wave_sync();
  for (int k = lane; k < n_own; k += 64) {
    const uint32_t at = atomicAdd(&rcnt[kRegions + own_loc[k]], 1u);
    d.cell_ids[at] = own_gid[k];
  }
  if (lane == 0) {
    d.acc_delta[cell] = acc;
    unsigned long long* c = d.acc_cnt + (size_t)cell * CNT_NCOL;
    c[CNT_LIFTS] += n_lift;
    c[CNT_FROZEN] += n_frozen;
    c[CNT_WALLS] += n_wall;
    c[CNT_CHAINS] += (uint64_t)n_m;
    d.cell_digest[cell] = h;
    atomicAdd(&d.digest_ring[sweep % kDigestRing], h * (2ull * (uint64_t)cell + 1ull));
  }
}

// Colour phase q of a sweep: one launch per phase, one wavefront per active
// cell; the launch boundary separates the phases.
template <int PREC, int REJ>
__global__ void __launch_bounds__(256) k_phase(const Dev* __restrict__ ds, int q) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = d.C >> 1;
  const int blk = blockIdx.x * d.cells_per_block + wave;
  if (blk >= half * half) return;  // the whole wave leaves; no workgroup barrier follows
  const SweepDraws dr = *d.draws;
  phase_cell<PREC, REJ>(d, sweep, dr, q, blk, lds_raw + (size_t)wave * d.lds_per_cell, lane);
}

// All four colour phases of a sweep in one launch.  The phases order only
// neighbouring cells: a cell of phase q reads the disks of its eight
// neighbours (frozen band) and writes its own, so it must follow the
// neighbours of earlier phases and precede those of later ones, while cells
// farther apart share nothing.  Each wavefront takes tickets from a counter
// in phase order (ticket = q * C^2/4 + block), waits until the neighbours of
// earlier phases have published this sweep's epoch, runs the cell and
// publishes its own epoch.  Every cell then reads exactly the positions the
// phase-by-phase schedule gives it, so the results are identical; a cell no
// longer waits for the slowest cell of the previous phase anywhere in the
// system.
//
// Progress: a wave waits only for cells with smaller tickets, which were
// taken by waves already running, so by induction over tickets every wait
// ends.  Every wait is also bounded by d.dep_wait_ticks (100 MHz clock) and
// abandoned when any wave has set d.err: on either, the wave sets or sees the
// error and leaves, and the sweep reports it.
template <int PREC, int REJ>
__global__ void __launch_bounds__(256) k_sweep_cells(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  unsigned char* const base = lds_raw + (size_t)wave * d.lds_per_cell;
  const SweepDraws dr = *d.draws;
  const int half = d.C >> 1;
  const int per_phase = half * half;
  // as many workers as one phase has cells (a batch launches for its largest system)
  if (blockIdx.x * d.cells_per_block + wave >= per_phase) return;
  const int64_t epoch = sweep + 1;
  // phase of each colour, two bits per colour
  int phase_of = 0;
  for (int q = 0; q < 4; ++q) phase_of |= q << (2 * ((dr.perm >> (2 * q)) & 3));

  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(d.queue, 1);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= 4 * per_phase) break;
    const int q = t / per_phase;
    const int blk = t - q * per_phase;
    const int colour = (dr.perm >> (2 * q)) & 3;
    const int cx = 2 * (blk % half) + (colour & 1);
    const int cy = 2 * (blk / half) + (colour >> 1);
    if (q > 0) {
      // lanes 0-7 watch the eight neighbours; those of earlier phases count
      bool need = false;
      int nc = 0;
      if (lane < 8) {
        const int k = lane < 4 ? lane : lane + 1;  // the 3 x 3 block without its centre
        const int ncx = (cx + (k % 3) - 1 + d.C) % d.C;
        const int ncy = (cy + (k / 3) - 1 + d.C) % d.C;
        nc = ncy * d.C + ncx;
        need = ((phase_of >> (2 * ((ncx & 1) | ((ncy & 1) << 1)))) & 3) < q;
      }
      const uint64_t t0 = wall_clock64();
      bool ok = true;
      for (;;) {
        // the limit is tested first, so a limit of 0 fails every wait
        if (wall_clock64() - t0 >= (uint64_t)d.dep_wait_ticks) {
          if (lane == 0) atomicOr(d.err, ERR_DEP_WAIT);
          ok = false;
          break;
        }
        const bool ready =
            !need || __hip_atomic_load(d.cell_done + nc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
        if (__builtin_amdgcn_ballot_w64(!ready) == 0) break;
        if (__builtin_amdgcn_readfirstlane(load_err(d)) != 0) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
      if (!ok) break;
      // the neighbours' write-backs are visible to the staging loads below
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    phase_cell<PREC, REJ>(d, sweep, dr, q, blk, base, lane);
    // this cell's write-back before its flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0)
      __hip_atomic_store(d.cell_done + (cy * d.C + cx), epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane(load_err(d)) != 0) break;
    wave_sync();  // LDS reads of this cell before the next cell's staging writes
  }
}

// ---------------------------------------------------------------------------
// Batched sweep with a ready queue: one launch runs every cell of every
// system of a batch.  A cell is ready once its earlier-phase neighbours in its
// own system are done (the only order the colour phases impose, Sec. 3.4 step
// 4); ready cells are appended to a queue, and persistent wavefronts take
// them in order, so no wavefront holds a slot while it waits for a
// neighbour, and no system waits for the slowest cell of another.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_phase(int phase_of, int C, int cell) {
  const int cx = cell % C, cy = cell / C;
  return (phase_of >> (2 * ((cx & 1) | ((cy & 1) << 1)))) & 3;
}
__device__ __forceinline__ int phase_map(int perm) {  // phase of each colour, two bits per colour
  int phase_of = 0;
  for (int q = 0; q < 4; ++q) phase_of |= q << (2 * ((perm >> (2 * q)) & 3));
  return phase_of;
}

__device__ __forceinline__ void queue_push(const ReadyQueue& rq, int32_t epoch, int64_t task) {
  const int r = atomicAdd(rq.hdr + QH_RESERVE, 1);
  rq.tasks[r] = task;
  // the task word before its flag
  __hip_atomic_store(rq.flags + r, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// New sweep: counters cleared, epoch advanced (one thread).
__global__ void k_queue_reset(ReadyQueue rq) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    rq.hdr[QH_READ] = 0;
    rq.hdr[QH_RESERVE] = 0;
    rq.hdr[QH_EPOCH] += 1;
    rq.hdr[QH_ABORT] = 0;
  }
}

// Count every cell's earlier-phase neighbours; cells with none (the first
// phase) are ready at once.  One thread per cell, grid y = system.
__global__ void k_queue_prep(const Dev* __restrict__ ds, ReadyQueue rq) {
  const Dev& d = ds[blockIdx.y];
  const int ncell = d.C * d.C;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int phase_of = phase_map(d.draws->perm);
  const int q = cell_phase(phase_of, d.C, c);
  const int cx = c % d.C, cy = c / d.C;
  int n = 0;
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    const int nc = ((cy + k / 3 - 1 + d.C) % d.C) * d.C + (cx + k % 3 - 1 + d.C) % d.C;
    n += cell_phase(phase_of, d.C, nc) < q ? 1 : 0;
  }
  const int g = rq.base[blockIdx.y] + c;
  rq.dep[g] = n;
  if (n == 0) queue_push(rq, rq.hdr[QH_EPOCH], ((int64_t)blockIdx.y << 32) | (uint32_t)c);
}

// Persistent wavefronts: take the next queue slot, wait until it is
// published, run that cell, then count it off at its later-phase neighbours
// and append those that become ready.  Every slot below the cell total is
// published eventually: if every wave waited, every published cell would be
// done, and the not-done cell of smallest phase would have all its
// earlier-phase neighbours done, hence be published -- a contradiction.  Each
// wait is also bounded (the first system's dep_wait_ticks) and given up once
// any wave has flagged an abort.
template <int PREC, int REJ>
__global__ void __launch_bounds__(256) k_queue_cells(const Dev* __restrict__ ds, ReadyQueue rq,
                                                     int lds_stride) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // the waves of a workgroup take cells of any system: regions of the largest size
  unsigned char* const base = lds_raw + (size_t)wave * lds_stride;
  const int32_t epoch = __hip_atomic_load(rq.hdr + QH_EPOCH, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t limit = (uint64_t)ds[0].dep_wait_ticks;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(rq.hdr + QH_READ, 1);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= rq.total) break;
    const uint64_t t0 = wall_clock64();
    bool ok = true;
    for (;;) {
      int f = 0, ab = 0;
      if (lane == 0) {
        f = __hip_atomic_load(rq.flags + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ab = __hip_atomic_load(rq.hdr + QH_ABORT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      f = __builtin_amdgcn_readfirstlane(f);
      ab = __builtin_amdgcn_readfirstlane(ab);
      if (f == epoch) break;
      if (ab != 0) { ok = false; break; }
      if (wall_clock64() - t0 >= limit) {
        if (lane == 0) {
          atomicOr(ds[0].err, ERR_DEP_WAIT);
          atomicExch(rq.hdr + QH_ABORT, 1);
        }
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    if (!ok) break;
    // the slot, and the write-backs of the cell's earlier-phase neighbours,
    // are visible to the loads below
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int64_t task = rq.tasks[t];
    const int sys = (int)(task >> 32), cell = (int)(uint32_t)task;
    const Dev& d = ds[sys];
    const int64_t sweep = *d.sweep_ctr;
    const SweepDraws dr = *d.draws;
    const int phase_of = phase_map(dr.perm);
    const int q = cell_phase(phase_of, d.C, cell);
    const int cx = cell % d.C, cy = cell / d.C;
    const int blk = (cy >> 1) * (d.C >> 1) + (cx >> 1);
    phase_cell<PREC, REJ>(d, sweep, dr, q, blk, base, lane);
    if (__builtin_amdgcn_readfirstlane(load_err(d)) != 0) {
      if (lane == 0) atomicExch(rq.hdr + QH_ABORT, 1);
      break;
    }
    // this cell's write-back before its neighbours count it off
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane < 8) {
      const int k = lane < 4 ? lane : lane + 1;  // the 3 x 3 block without its centre
      const int nc = ((cy + k / 3 - 1 + d.C) % d.C) * d.C + (cx + k % 3 - 1 + d.C) % d.C;
      if (cell_phase(phase_of, d.C, nc) > q) {
        const int g = rq.base[sys] + nc;
        const int left = __hip_atomic_fetch_add(rq.dep + g, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == 1) queue_push(rq, epoch, ((int64_t)sys << 32) | (uint32_t)nc);
      }
    }
    wave_sync();  // LDS reads of this cell before the next cell's staging writes
  }
}

// After the launch: if a wave gave up (an error in some system, or a wait
// limit), mark every system of the batch, since their sweeps are unfinished.
__global__ void k_queue_check(const Dev* __restrict__ ds, ReadyQueue rq) {
  const Dev& d = ds[blockIdx.y];
  if (threadIdx.x == 0 && rq.hdr[QH_ABORT] != 0) atomicOr(d.err, ERR_ABANDONED);
}

// ---------------------------------------------------------------------------
// Striped decomposition with rejection (Sec. 3.4, Fig. 3 "stripes"; Sec. 4):
// C stripes of width w span the box; on even sweeps they are horizontal and
// chains run along x, on odd sweeps vertical with chains along y, each chain
// with a random sign (a chain and its reverse are proposed alike, and a chain
// is rejected exactly when its reverse is).  Colour phase q runs every stripe
// k with (k & 1) == first ^ q, one wavefront each; a chain that hits a disk
// of a neighbouring stripe is rejected and undone.
// The search is a brute-force minimum over the stripe's disks and the frozen
// disks of its two neighbours within sigma of it (nearest image along the
// stripe, flights capped at L/2 - sigma as in one periodic box).
// ---------------------------------------------------------------------------
template <int DUMMY>
__global__ void __launch_bounds__(64) k_stripe_phase(const Dev* __restrict__ ds, int q) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  const SweepDraws dr = *d.draws;
  const int k = 2 * (int)blockIdx.x + ((dr.perm ^ q) & 1);
  if (k >= d.C) return;  // the whole wave leaves
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x;
  const int cap_own = d.stripe_cap_own, cap_fr = d.stripe_cap_frozen, cap_undo = d.stripe_undo;
  double* own_a = (double*)lds_raw;
  double* own_v = own_a + cap_own;
  double* fr_a = own_v + cap_own;
  double* fr_v = fr_a + cap_fr;
  double* undo_a = fr_v + cap_fr;
  int32_t* own_gid = (int32_t*)(undo_a + cap_undo);
  int32_t* tmp = own_gid + cap_own;
  int32_t* fr_gid = tmp + cap_own;
  int32_t* undo_i = fr_gid + cap_fr;
  int32_t* n_fr_sh = undo_i + cap_undo;

  double* const along = (sweep & 1) ? d.y : d.x;
  const double* const across = (sweep & 1) ? d.x : d.y;
  const double L = d.L, half_L = d.half_L, sigma = d.sigma, sig2 = d.sig2, cap = d.cap;
  const double origin = (double)k * d.w;

  // ---- stage: own disks in id order, frozen disks of the two neighbours
  const int start = d.cell_start[k];
  const int n_own = d.cell_start[k + 1] - start;
  if (n_own < 0 || n_own > cap_own) {
    if (lane == 0) atomicOr(d.err, ERR_OWN_CAP);
    return;
  }
  for (int i = lane; i < n_own; i += 64) tmp[i] = d.cell_ids[start + i];
  if (lane == 0) *n_fr_sh = 0;
  wave_sync();
  for (int i = lane; i < n_own; i += 64) {
    const int v = tmp[i];
    int r = 0;
    for (int j = 0; j < n_own; ++j) r += (tmp[j] < v) ? 1 : 0;
    own_gid[r] = v;
  }
  wave_sync();
  for (int i = lane; i < n_own; i += 64) {
    const int g = own_gid[i];
    own_a[i] = along[g];
    own_v[i] = local_coord(across[g], dr.sx, origin, L, half_L);
  }
  for (int side = -1; side <= 1; side += 2) {
    const int nk = (k + side + d.C) % d.C;
    const int s0 = d.cell_start[nk], s1 = d.cell_start[nk + 1];
    for (int t = s0 + lane; t < s1; t += 64) {
      const int g = d.cell_ids[t];
      const double v = local_coord(across[g], dr.sx, origin, L, half_L);
      if (v >= -sigma && v <= d.w + sigma) {
        const int slot = atomicAdd(n_fr_sh, 1);
        if (slot < cap_fr) {
          fr_a[slot] = along[g];
          fr_v[slot] = v;
          fr_gid[slot] = g;
        } else {
          atomicOr(d.err, ERR_OWN_CAP);
        }
      }
    }
  }
  wave_sync();
  const int n_fr = min(*n_fr_sh, cap_fr);
  if (__builtin_amdgcn_readfirstlane(load_err(d)) != 0) return;

  // ---- chains
  const int64_t n_m = chains_of(d, n_own);
  const int64_t cbase = chain_base(d, k);
  double acc = d.acc_delta[k];
  uint64_t n_lift = 0, n_frozen = 0, n_pseudo = 0, h = 0, n_ev = 0;
  bool stop = false;
  for (int64_t c = 0; c < n_m && !stop; ++c) {
    int a = uniform_i32(d.chain_start[cbase + c]);
    if (a < 0 || a >= n_own) a = 0;  // guarded: the draw kernel writes indices below n_own
    // the chain's sign: the top bit of the first word of its direction stream
    Stream ss(d.seed, kKindDir, (uint64_t)sweep, cell_key(d, k), (uint64_t)c);
    const bool neg = (ss.next() >> 63) != 0;
    double rem = d.ell, chain_acc = 0.0;
    uint64_t chain_lifts = 0;
    int n_undo = 0;
    int64_t events = 0;
    for (;;) {
      if (++events > kMaxEventsPerChain || (events % kAbortPollEvents) == 0) {
        if (events > kMaxEventsPerChain) {
          if (lane == 0) atomicOr(d.err, ERR_EVENT_CAP);
          stop = true;
          break;
        }
        if (uniform_i32(load_err(d)) != 0) { stop = true; break; }
      }
      const double aa = own_a[a], av = own_v[a];
      double ls = INFINITY;
      uint32_t lid = 0xFFFFFFFFu;
      int lj = -1;  // own index, or cap_own + frozen index
      for (int j = lane; j < n_own + n_fr; j += 64) {
        if (j == a) continue;
        const bool own = j < n_own;
        const int f = j - n_own;
        double ra = (own ? own_a[j] : fr_a[f]) - aa;
        if (ra < -half_L) ra += L; else if (ra >= half_L) ra -= L;
        if (neg) ra = -ra;
        const double rv = (own ? own_v[j] : fr_v[f]) - av;
        const double disc = fma(-rv, rv, sig2);
        if (ra > 0.0 && disc > 0.0) {
          double s = ra - sqrt(disc);
          if (s < 0.0) s = 0.0;
          const uint32_t gid = (uint32_t)(own ? own_gid[j] : fr_gid[f]);
          if (s < ls || (s == ls && gid < lid)) { ls = s; lid = gid; lj = j; }
        }
      }
      const int wl = wave_argmin(ls, lid, lj >= 0);
      double best_s = INFINITY;
      int bj = -1;
      uint32_t bgid = 0;
      if (wl >= 0) {
        best_s = readlane_f64(ls, wl);
        bj = readlane_i32(lj, wl);
        bgid = (uint32_t)readlane_i32((int)lid, wl);
      }
      const double lim = best_s < rem ? best_s : rem;
      if (lim > cap) {
        // a free flight beyond the nearest-image range: moved in pieces
        h ^= digest_term(EV_PSEUDO, (uint64_t)d.n + 2, cap, n_ev++);
        if (n_undo == cap_undo) {
          if (lane == 0) atomicOr(d.err, ERR_UNDO_CAP);
          stop = true;
          break;
        }
        if (lane == 0) { undo_i[n_undo] = a; undo_a[n_undo] = aa; }
        n_undo += 1;
        double na = neg ? aa - cap : aa + cap;
        if (na >= L) na -= L; else if (na < 0.0) na += L;
        if (lane == 0) own_a[a] = na;
        wave_sync();
        rem = rem - cap;
        n_pseudo += 1;
        continue;
      }
      if (!(best_s < rem)) {
        h ^= digest_term(EV_END, (uint64_t)d.n + 3, rem, n_ev++);
        double na = neg ? aa - rem : aa + rem;
        if (na >= L) na -= L; else if (na < 0.0) na += L;
        if (lane == 0) own_a[a] = na;
        wave_sync();
        acc = acc + chain_acc;  // accepted
        n_lift += chain_lifts;
        break;
      }
      const bool frozen = bj >= n_own;
      h ^= digest_term(frozen ? EV_FROZEN : EV_LIFT, bgid, best_s, n_ev++);
      if (n_undo == cap_undo) {
        if (lane == 0) atomicOr(d.err, ERR_UNDO_CAP);
        stop = true;
        break;
      }
      if (lane == 0) { undo_i[n_undo] = a; undo_a[n_undo] = aa; }
      n_undo += 1;
      double na = neg ? aa - best_s : aa + best_s;
      if (na >= L) na -= L; else if (na < 0.0) na += L;
      if (lane == 0) own_a[a] = na;
      wave_sync();
      rem = rem - best_s;
      if (frozen) {
        // a disk of a neighbouring stripe: the chain is rejected and undone
        n_frozen += 1;
        if (lane == 0)
          for (int u = n_undo - 1; u >= 0; --u) own_a[undo_i[u]] = undo_a[u];
        wave_sync();
        break;
      }
      double r = own_a[bj] - na;
      if (r < -half_L) r += L; else if (r >= half_L) r -= L;
      chain_acc = chain_acc + (neg ? -r : r);
      chain_lifts += 1;
      a = bj;
    }
  }
  wave_sync();
  for (int i = lane; i < n_own; i += 64) along[own_gid[i]] = own_a[i];
  if (lane == 0) {
    d.acc_delta[k] = acc;
    unsigned long long* cn = d.acc_cnt + (size_t)k * CNT_NCOL;
    cn[CNT_LIFTS] += n_lift;
    cn[CNT_FROZEN] += n_frozen;
    cn[CNT_CHAINS] += (uint64_t)n_m;
    cn[CNT_PSEUDO] += n_pseudo;
    d.cell_digest[k] = h;
    atomicAdd(&d.digest_ring[sweep % kDigestRing], h * (2ull * (uint64_t)k + 1ull));
  }
}

// ---------------------------------------------------------------------------
// One periodic cell (C = 1): all N disks in LDS, brute-force search with the
// minimum image; flights longer than L/2 - sigma are split (free-flight cap).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_periodic(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x;
  const int n = (int)d.n;
  double* px = (double*)lds_raw;
  double* py = px + n;
  int32_t* tmp = (int32_t*)(py + n);
  const double L = d.L, half_L = d.half_L, sig2 = d.sig2, cap = d.cap;
  for (int i = lane; i < n; i += 64) { px[i] = d.x[i]; py[i] = d.y[i]; }
  int64_t n_m = d.chains_per_cell > 0 ? d.chains_per_cell : n;
  if (d.start_mode == 1) {
    wave_sync();
    if (lane == 0) {
      for (int i = 0; i < n; ++i) tmp[i] = i;
      Stream st(d.seed, kKindShuffle, (uint64_t)sweep, cell_key(d, 0), 0);
      for (int i = 0; i + 1 < n; ++i) {
        int j = i + (int)draw_index(st, (uint64_t)(n - i));
        int t = tmp[i]; tmp[i] = tmp[j]; tmp[j] = t;
      }
    }
  }
  wave_sync();
  double acc = d.acc_delta[0];
  uint64_t n_lift = 0, n_pseudo = 0, h = 0, n_ev = 0;

  for (int64_t k = 0; k < n_m; ++k) {
    int a;
    if (d.start_mode == 1) {
      a = tmp[k % n];
    } else {
      Stream st(d.seed, kKindStart, (uint64_t)sweep, cell_key(d, 0), (uint64_t)k);
      a = (int)draw_index(st, (uint64_t)n);
    }
    double dx, dy;
    chain_direction(d, sweep, 0, k, dx, dy);
    double rem = d.ell;
    double ax = px[a], ay = py[a];
    int64_t n_events = 0;
    for (;;) {
      if (++n_events > kMaxEventsPerChain) {
        if (lane == 0) atomicOr(d.err, ERR_EVENT_CAP);
        break;
      }
      double ls = INFINITY;
      int lj = -1;
      for (int j = lane; j < n; j += 64) {
        if (j == a) continue;
        double rx = px[j] - ax, ry = py[j] - ay;
        if (rx < -half_L) rx += L; else if (rx >= half_L) rx -= L;
        if (ry < -half_L) ry += L; else if (ry >= half_L) ry -= L;
        double s;
        if (contact(rx, ry, dx, dy, sig2, s)) {
          if (s < ls) { ls = s; lj = j; }  // j rises with the loop: lowest id kept on ties
        }
      }
      int wl = wave_argmin(ls, (uint32_t)lj, lj >= 0);
      double best_s = INFINITY;
      int bj = -1;
      if (wl >= 0) { best_s = readlane_f64(ls, wl); bj = readlane_i32(lj, wl); }
      double lim = best_s < rem ? best_s : rem;
      double step;
      int kind;
      if (lim > cap) {
        step = cap; kind = EV_PSEUDO;
        h ^= digest_term(EV_PSEUDO, (uint64_t)d.n + 2, cap, n_ev++);
      } else if (!(best_s < rem)) {
        step = rem; kind = EV_END;
        h ^= digest_term(EV_END, (uint64_t)d.n + 3, rem, n_ev++);
      } else {
        step = best_s; kind = EV_LIFT;
        h ^= digest_term(EV_LIFT, (uint64_t)bj, best_s, n_ev++);
      }
      ax = fma(step, dx, ax);
      ay = fma(step, dy, ay);
      if (ax >= L) ax -= L; else if (ax < 0.0) ax += L;
      if (ay >= L) ay -= L; else if (ay < 0.0) ay += L;
      if (lane == 0) { px[a] = ax; py[a] = ay; }
      wave_sync();
      if (kind == EV_END) break;
      if (kind == EV_PSEUDO) { rem = rem - cap; n_pseudo += 1; continue; }
      rem = rem - best_s;
      double rx = px[bj] - ax, ry = py[bj] - ay;
      if (rx < -half_L) rx += L; else if (rx >= half_L) rx -= L;
      if (ry < -half_L) ry += L; else if (ry >= half_L) ry -= L;
      acc = acc + fma(rx, dx, ry * dy);
      n_lift += 1;
      a = bj;
      ax = px[a];
      ay = py[a];
    }
  }
  wave_sync();
  for (int i = lane; i < n; i += 64) { d.x[i] = px[i]; d.y[i] = py[i]; }
  if (lane == 0) {
    d.acc_delta[0] = acc;
    d.acc_cnt[CNT_LIFTS] += n_lift;
    d.acc_cnt[CNT_CHAINS] += (uint64_t)n_m;
    d.acc_cnt[CNT_PSEUDO] += n_pseudo;
    d.digest_ring[sweep % kDigestRing] = h;
    d.cell_digest[0] = h;
  }
}

// ---------------------------------------------------------------------------
// Tallies
// ---------------------------------------------------------------------------
__global__ void k_reduce(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int ncell = d.C * d.C;
  double s = 0.0;
  uint64_t c[CNT_NCOL] = {0, 0, 0, 0, 0};
  for (int i = 0; i < ncell; ++i) {
    s = s + d.acc_delta[i];
    for (int k = 0; k < CNT_NCOL; ++k) c[k] += d.acc_cnt[(size_t)i * CNT_NCOL + k];
  }
  d.red[0] = s;
  for (int k = 0; k < CNT_NCOL; ++k) d.red[1 + k] = __longlong_as_double((long long)c[k]);
}

__global__ void k_zero_tallies(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  int ncell = d.C * d.C;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x) {
    d.acc_delta[i] = 0.0;
    for (int k = 0; k < CNT_NCOL; ++k) d.acc_cnt[(size_t)i * CNT_NCOL + k] = 0;
  }
}

// ---------------------------------------------------------------------------
// One periodic cell (C = 1) with a bin grid: the same events as k_periodic,
// found in an 8 x 8-bin window around the moving disk as in the walled cells.
// Bins of side b = L / pbins < 0.7 sigma hold one disk each (a slot: FP64
// position, NaN when empty, and the disk's id); the window wraps around the
// box, and each lane forms its disk's offset with the minimum image exactly
// as k_periodic does, so the contact distances are the same numbers.  The
// window reaches 2 bins behind the moving disk and 5 ahead along each axis,
// so a move of length t with t max(|dx|, |dy|) <= 5b - sigma - eps keeps its
// sigma-neighbourhood inside it; the host takes this kernel only where that
// reach is below the free-flight cap L/2 - sigma, so a window event is never
// a pseudo event.  Every other event (a longer flight, the chain end, the
// cap) is decided as in k_periodic, over every slot when the window cannot
// vouch.  Plain lifts (the nearest disk in the window hit within the
// remaining length, the cap and the window's reach) run in an inner loop, as
// in the walled cells.  Event records are kept in the lanes and hashed 64 at
// a time; the lifts are counted from them.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_periodic_bins(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  const int64_t sweep = *d.sweep_ctr;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x;
  const int n = (int)d.n;
  const int nb = d.pbins;
  const PeriodicLds lay = periodic_lds_layout(nb, n);
  double2* const pos = (double2*)(lds_raw + lay.off_pos);
  uint32_t* const meta = (uint32_t*)(lds_raw + lay.off_meta);
  int32_t* const slot_of = (int32_t*)(lds_raw + lay.off_slot_of);
  int32_t* const tmp = (int32_t*)(lds_raw + lay.off_tmp);
  double2* const sink = (double2*)(lds_raw + lay.off_sink) + lane;
  uint32_t* const sink32 = (uint32_t*)sink;
  const int nslots = nb * nb;
  const double L = d.L, half_L = d.half_L, sig2 = d.sig2, cap = d.cap, sigma = d.sigma;
  const double b = L / (double)nb, inv_b = 1.0 / b;
  const double2 nan2 = make_double2(__builtin_nan(""), __builtin_nan(""));
  // bin coordinates of a slot: by = floor(slot / nb) as (slot * m) >> 20 with
  // m = ceil(2^20 / nb), exact for slot < nb^2 when nb^3 < 2^20 (nb <= 100)
  const uint32_t inv_n20 = ((1u << 20) + (uint32_t)nb - 1u) / (uint32_t)nb;
  // the minimum image of an offset, as k_periodic forms it (v + L below
  // -L/2, v - L from L/2 on), written as selects so that no lane branches
  auto min_image = [&](double v) __attribute__((always_inline)) {
    const double vp = v + L, vm = v - L;
    return v < -half_L ? vp : (v >= half_L ? vm : v);
  };
  auto bin_of = [&](double v) __attribute__((always_inline)) {
    int k = (int)(v * inv_b);
    return k > nb - 1 ? nb - 1 : (k < 0 ? 0 : k);
  };

  for (int sl = lane; sl < nslots; sl += 64) {
    pos[sl] = nan2;
    meta[sl] = kEmptySlot;
  }
  wave_sync();
  for (int i = lane; i < n; i += 64) {
    const double x = d.x[i], y = d.y[i];
    const int sl = bin_of(y) * nb + bin_of(x);
    if (atomicCAS(&meta[sl], kEmptySlot, (uint32_t)i) != kEmptySlot) {
      atomicOr(d.err, ERR_BIN_CAP);
      continue;
    }
    pos[sl] = make_double2(x, y);
    slot_of[i] = sl;
  }
  const int64_t n_m = d.chains_per_cell > 0 ? d.chains_per_cell : n;
  if (d.start_mode == 1) {
    wave_sync();
    if (lane == 0) {
      for (int i = 0; i < n; ++i) tmp[i] = i;
      Stream st(d.seed, kKindShuffle, (uint64_t)sweep, cell_key(d, 0), 0);
      for (int i = 0; i + 1 < n; ++i) {
        int j = i + (int)draw_index(st, (uint64_t)(n - i));
        int t = tmp[i]; tmp[i] = tmp[j]; tmp[j] = t;
      }
    }
  }
  wave_sync();
  if (load_err(d) != 0) return;  // two disks in one bin: an overlap

  double acc = d.acc_delta[0];
  uint64_t n_lift = 0, n_pseudo = 0, h = 0;
  int n_ring = 0;           // event records held in the lanes (lane k: record k)
  uint64_t ring_first = 0;  // event index of record 0
  uint32_t rec_lo = 0, rec_hi = 0, rec_tag = 0;
  const int lx = lane & 7, ly = lane >> 3;
  const double eps = 1e-9 * sigma;
  const double reach = 5.0 * b - sigma - eps;
  const uint32_t pseudo_id = (uint32_t)d.n + 2, end_id = (uint32_t)d.n + 3;
  // the records are hashed 64 at a time; lifts are counted from the records
  auto flush = [&]() __attribute__((always_inline)) {
    h ^= digest_batch_ids(rec_lo, rec_hi, rec_tag, lane, kDigestBatch, ring_first);
    n_lift += count_lifts(rec_tag, lane, kDigestBatch);
    ring_first += kDigestBatch;
    n_ring = 0;
  };
  // a coordinate moved across the box edge comes back from the other side
  // (both candidates formed first, so that no lane branches)
  auto wrap_box = [&](double v) __attribute__((always_inline)) {
    const double vm = v - L, vp = v + L;
    return v >= L ? vm : (v < 0.0 ? vp : v);
  };

  for (int64_t k = 0; k < n_m; ++k) {
    int a;
    if (d.start_mode == 1) {
      a = tmp[k % n];
    } else {
      Stream st(d.seed, kKindStart, (uint64_t)sweep, cell_key(d, 0), (uint64_t)k);
      a = (int)draw_index(st, (uint64_t)n);
    }
    // every lane draws the same values; read them as one (scalar) value so
    // that every decision below is a uniform branch
    a = uniform_i32(a);
    double dx, dy;
    chain_direction(d, sweep, 0, k, dx, dy);
    dx = readlane_f64(dx, 0);
    dy = readlane_f64(dy, 0);
    // reach / max(|dx|, |dy|) from the reciprocals (a 0 component has a factor 1)
    const double rx_ = dx != 0.0 ? 1.0 / dx : 1.0, ry_ = dy != 0.0 ? 1.0 / dy : 1.0;
    const double dsafe = reach * fmin(fabs(rx_), fabs(ry_));
    const int offx = dx < 0.0 ? -5 : -2, offy = dy < 0.0 ? -5 : -2;  // window origin
    // this lane's slot in the 8 x 8-bin window around the bin of `slot`,
    // wrapped around the box
    auto window_slot = [&](int slot) __attribute__((always_inline)) {
      const int by = (int)(((uint32_t)slot * inv_n20) >> 20);
      const int bx = slot - by * nb;
      int wx = bx + offx + lx, wy = by + offy + ly;
      wx += wx < 0 ? nb : 0;
      wx -= wx >= nb ? nb : 0;
      wy += wy < 0 ? nb : 0;
      wy -= wy >= nb ? nb : 0;
      return wy * nb + wx;
    };
    double rem = d.ell;
    int a_slot = uniform_i32(slot_of[a]);
    double ax = pos[a_slot].x, ay = pos[a_slot].y;
    // the event cap is held at the digest flushes: ring_first - ev0 is the
    // chain's event count there, so a chain makes at most
    // kMaxEventsPerChain + 63 events before it stops with the error
    const uint64_t ev0 = ring_first + (uint64_t)n_ring;
    int capped = 0;
    int wsl = window_slot(a_slot);
    double2 p = pos[wsl];
    uint32_t m = meta[wsl];
    for (;;) {
      // One plain lift: the nearest disk in the window is hit within the
      // remaining length, within the flight cap and within the reach the
      // window vouches for.  That is exactly the full decision below finding
      // a lift; every other event (no disk in the window, the chain end, a
      // pseudo event, a flight the window cannot vouch for) is left to it,
      // with nothing changed.  Every lane makes the test, moves the mover
      // onto its own candidate and forms that move's pressure term while
      // the wave minimum forms; the winner's values are the event's.  False
      // on any other event, and at a flush that finds the event cap reached.
      auto plain_event = [&]() __attribute__((always_inline)) -> bool {
        const double rx = min_image(p.x - ax), ry = min_image(p.y - ay);
        double s = 0.0;
        const bool valid = contact(rx, ry, dx, dy, sig2, s);  // the mover's own slot: no contact
        double nxl, nyl;
        int plain_l, ns_l;
        {
          nxl = wrap_box(fma(s, dx, ax));
          nyl = wrap_box(fma(s, dy, ay));
          ns_l = bin_of(nyl) * nb + bin_of(nxl);
          plain_l = (int)(s <= dsafe) & (int)(s < rem) & (int)(s <= cap);
          // keep them here, beside the wave minimum
          asm volatile("" : : "v"(plain_l), "v"(ns_l));
        }
        const unsigned key = argmin_key(s, valid);
        const unsigned key_min = wave_min_u32(key);
        if (__builtin_expect(key_min == 0xFFFFFFFFu, 0)) return false;
        const int wl = argmin_lane(s, m, key, key_min);
        if (__builtin_expect(readlane_i32(plain_l, wl) == 0, 0)) return false;
        const double best_s = readlane_f64(s, wl);
        const int bj = readlane_i32((int)m, wl);
        const int bslot = readlane_i32(wsl, wl);
        const double wpx = readlane_f64(p.x, wl), wpy = readlane_f64(p.y, wl);
        const int ns = readlane_i32(ns_l, wl);
        {
          const uint64_t sb = (uint64_t)__double_as_longlong(best_s);
          writelane3(rec_lo, rec_hi, rec_tag, (uint32_t)sb, (uint32_t)(sb >> 32),
                     ((uint32_t)EV_LIFT << 29) | (uint32_t)bj, n_ring);
        }
        // the winning lane stores the moved centre
        {
          double2* const dst = (lane == wl) ? pos + a_slot : sink;
          *dst = make_double2(nxl, nyl);
        }
        if (__builtin_expect(ns != a_slot, 0)) {
          // the centre crossed into another bin, which is empty (a bin holds
          // one centre): the winning lane stores it there, another lane
          // empties the old slot (over the store above: LDS stores of a wave
          // land in order), and lanes 0, 1, 2 move the meta words and the
          // disk's slot in one store
          const int other = wl == 0 ? 1 : 0;
          double2* const dst = (lane == wl) ? pos + ns : ((lane == other) ? pos + a_slot : sink);
          *dst = (lane == wl) ? make_double2(nxl, nyl) : nan2;
          uint32_t* const dm = (lane == 0) ? meta + a_slot
                                           : ((lane == 1) ? meta + ns
                                                          : ((lane == 2) ? (uint32_t*)(slot_of + a) : sink32));
          *dm = (lane == 0) ? kEmptySlot : ((lane == 1) ? (uint32_t)a : (uint32_t)ns);
        }
        __builtin_amdgcn_wave_barrier();
        // the next window is read while the pressure term forms (from the
        // lane's own disk and moved centre, the values of this window)
        const double ox = p.x, oy = p.y;
        wsl = window_slot(bslot);
        p = pos[wsl];
        m = meta[wsl];
        const double tx = min_image(ox - nxl), ty = min_image(oy - nyl);
        acc = acc + readlane_f64(fma(tx, dx, ty * dy), wl);
        rem = rem - best_s;
        a = bj;
        a_slot = bslot;
        ax = wpx;
        ay = wpy;
        if (__builtin_expect(++n_ring == kDigestBatch, 0)) {
          flush();
          capped = (ring_first - ev0 >= (uint64_t)kMaxEventsPerChain) ? 1 : 0;
          if (capped != 0) return false;
        }
        return true;
      };
      for (;;) {
        if (__builtin_expect(!plain_event(), 0)) break;
        if (__builtin_expect(!plain_event(), 0)) break;
      }  // plain lifts
      if (capped != 0) {
        if (lane == 0) atomicOr(d.err, ERR_EVENT_CAP);
        break;
      }
      // the full decision, on the window already read
      const double rx = min_image(p.x - ax), ry = min_image(p.y - ay);
      double s = 0.0;
      const bool valid = contact(rx, ry, dx, dy, sig2, s);  // the mover's own slot: no contact
      const unsigned key = argmin_key(s, valid);
      const unsigned key_min = wave_min_u32(key);
      double best_s = INFINITY, wpx = 0.0, wpy = 0.0;
      int bj = -1, bslot = -1;
      if (key_min != 0xFFFFFFFFu) {
        const int wl = argmin_lane(s, m, key, key_min);
        best_s = readlane_f64(s, wl);
        bj = readlane_i32((int)m, wl);
        bslot = readlane_i32(wsl, wl);
        wpx = readlane_f64(p.x, wl);
        wpy = readlane_f64(p.y, wl);
      }
      if (uniform_i32(best_s <= dsafe ? 0 : 1) != 0) {
        // the window cannot vouch: the nearest contact over every slot
        double ls = INFINITY;
        uint32_t lid = 0xFFFFFFFFu;
        int lsl = -1;
        for (int sl = lane; sl < nslots; sl += 64) {
          const double2 q = pos[sl];
          const double qx = min_image(q.x - ax), qy = min_image(q.y - ay);
          double s2;
          if (contact(qx, qy, dx, dy, sig2, s2)) {
            const uint32_t i2 = meta[sl];
            if (s2 < ls || (s2 == ls && i2 < lid)) { ls = s2; lid = i2; lsl = sl; }
          }
        }
        const int fl = wave_argmin_all(ls, lid, lsl >= 0);
        best_s = INFINITY;
        bj = -1;
        if (fl >= 0) {
          best_s = readlane_f64(ls, fl);
          bj = readlane_i32((int)lid, fl);
          bslot = readlane_i32(lsl, fl);
          const double2 q = pos[bslot];
          wpx = readlane_f64(q.x, 0);
          wpy = readlane_f64(q.y, 0);
        }
      }
      // the event, in the order k_periodic decides it (one scalar value)
      const double lim = best_s < rem ? best_s : rem;
      const int kind = uniform_i32(lim > cap ? EV_PSEUDO : (!(best_s < rem) ? EV_END : EV_LIFT));
      const double step = kind == EV_PSEUDO ? cap : (kind == EV_END ? rem : best_s);
      {
        const uint32_t id = kind == EV_PSEUDO ? pseudo_id : (kind == EV_END ? end_id : (uint32_t)bj);
        const uint64_t sb = (uint64_t)__double_as_longlong(step);
        writelane3(rec_lo, rec_hi, rec_tag, (uint32_t)sb, (uint32_t)(sb >> 32),
                   ((uint32_t)kind << 29) | id, n_ring);
      }
      const double nax = wrap_box(fma(step, dx, ax)), nay = wrap_box(fma(step, dy, ay));
      // store the moved disk (lane 0) and move it to another bin if it crossed
      // one (lane 0 empties the old slot, lane 1 fills the new one, which is
      // empty: a bin holds one centre)
      const int ns = uniform_i32(bin_of(nay) * nb + bin_of(nax));
      {
        double2* const dst = (lane == 0) ? pos + a_slot : sink;
        *dst = make_double2(nax, nay);
      }
      if (ns != a_slot) {
        double2* const dst = (lane == 0) ? pos + a_slot : ((lane == 1) ? pos + ns : sink);
        *dst = (lane == 0) ? nan2 : make_double2(nax, nay);
        uint32_t* const dm = (lane == 0) ? meta + a_slot : ((lane == 1) ? meta + ns : sink32);
        *dm = (lane == 0) ? kEmptySlot : (uint32_t)a;
        if (lane == 0) slot_of[a] = ns;
        a_slot = ns;
      }
      wave_sync();
      if (++n_ring == kDigestBatch) {
        flush();
        capped = (ring_first - ev0 >= (uint64_t)kMaxEventsPerChain) ? 1 : 0;
      }
      if (kind == EV_END) break;
      if (kind == EV_PSEUDO) {
        rem = rem - cap;
        n_pseudo += 1;
        ax = nax;
        ay = nay;
      } else {
        rem = rem - best_s;
        const double tx = min_image(wpx - nax), ty = min_image(wpy - nay);
        acc = acc + fma(tx, dx, ty * dy);
        a = bj;
        a_slot = bslot;
        ax = wpx;
        ay = wpy;
      }
      if (capped != 0) {
        if (lane == 0) atomicOr(d.err, ERR_EVENT_CAP);
        break;
      }
      wsl = window_slot(a_slot);
      p = pos[wsl];
      m = meta[wsl];
    }
  }
  wave_sync();
  h ^= digest_batch_ids(rec_lo, rec_hi, rec_tag, lane, n_ring, ring_first);
  n_lift += count_lifts(rec_tag, lane, n_ring);
  for (int i = lane; i < n; i += 64) {
    const double2 v = pos[slot_of[i]];
    d.x[i] = v.x;
    d.y[i] = v.y;
  }
  if (lane == 0) {
    d.acc_delta[0] = acc;
    d.acc_cnt[CNT_LIFTS] += n_lift;
    d.acc_cnt[CNT_CHAINS] += (uint64_t)n_m;
    d.acc_cnt[CNT_PSEUDO] += n_pseudo;
    d.digest_ring[sweep % kDigestRing] = h;
    d.cell_digest[0] = h;
  }
}

// The sweep counter every kernel of the next sweep reads (one thread per system).
__global__ void k_sweep_done(const Dev* __restrict__ ds) {
  if (threadIdx.x == 0) *ds[blockIdx.y].sweep_ctr += 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Grid x-extents are the maxima over the systems of a launch (gridDim.y =
// systems); blocks beyond a system's own extent leave at once.
// ---------------------------------------------------------------------------
hipError_t launch_lattice(const Dev* ds, int64_t n, int64_t k, double a, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_lattice, dim3((unsigned)blocks), dim3(256), 0, st, ds, k, a);
  return hipGetLastError();
}

hipError_t launch_zero_tallies(const Dev* ds, int32_t n_cells, hipStream_t st) {
  int blocks = (n_cells + 255) / 256;
  hipLaunchKernelGGL(k_zero_tallies, dim3(blocks), dim3(256), 0, st, ds);
  return hipGetLastError();
}

hipError_t set_phase_lds_limit(int bytes) {
  const void* fns[11] = {(const void*)k_phase<0, 0>,       (const void*)k_phase<1, 0>,
                         (const void*)k_phase<0, 1>,       (const void*)k_sweep_cells<0, 0>,
                         (const void*)k_sweep_cells<1, 0>, (const void*)k_sweep_cells<0, 1>,
                         (const void*)k_queue_cells<0, 0>, (const void*)k_queue_cells<1, 0>,
                         (const void*)k_queue_cells<0, 1>, (const void*)k_stripe_phase<0>,
                         (const void*)k_periodic_bins};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t ready_queue_workers(int lds_per_cell, int cpb, int fp32, int reject, int* workers) {
  const void* f = fp32 ? (const void*)k_queue_cells<1, 0>
                       : (reject ? (const void*)k_queue_cells<0, 1> : (const void*)k_queue_cells<0, 0>);
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64 * cpb,
                                                              (size_t)cpb * lds_per_cell);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *workers = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1) * cpb;
  return hipSuccess;
}

hipError_t launch_reduce(const Dev* ds, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(64), 0, st, ds);
  return hipGetLastError();
}

hipError_t launch_sweep(const Dev* ds, const LaunchShape& sh, hipStream_t st,
                        const PhaseEvents* ev) {
  const unsigned ns = (unsigned)sh.n_sys;
  if (sh.periodic) {
    if (ev) (void)hipEventRecord(ev->begin[0], st);
    if (sh.pbins > 0) {
      const size_t lds = (size_t)periodic_lds_layout(sh.pbins, (int)sh.max_n).bytes;
      hipLaunchKernelGGL(k_periodic_bins, dim3(1, ns), dim3(64), lds, st, ds);
    } else {
      const size_t lds = (size_t)sh.max_n * 16 + (size_t)sh.max_n * 4;
      hipLaunchKernelGGL(k_periodic, dim3(1, ns), dim3(64), lds, st, ds);
    }
    if (ev) (void)hipEventRecord(ev->end[0], st);
    hipError_t e = launch_check_overlap(ds, sh, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_done, dim3(1, ns), dim3(64), 0, st, ds);
    return hipGetLastError();
  }
  const unsigned nblk = (unsigned)((sh.max_n + 255) / 256);
  hipLaunchKernelGGL(k_prep, dim3(1, ns), dim3(1024), 0, st, ds, 0);
  if (ev) (void)hipEventRecord(ev->rebin[0], st);
  hipLaunchKernelGGL(k_count, dim3(nblk, ns), dim3(256), 0, st, ds, 0);
  if (ev) (void)hipEventRecord(ev->rebin[1], st);
  hipLaunchKernelGGL(k_scan, dim3(1, ns), dim3(1024), 0, st, ds);
  if (ev) (void)hipEventRecord(ev->rebin[2], st);
  hipLaunchKernelGGL(k_scatter, dim3(nblk, ns), dim3(256), 0, st, ds);
  if (ev) (void)hipEventRecord(ev->rebin[3], st);
  hipLaunchKernelGGL(k_draws, dim3((unsigned)((sh.max_chains + 255) / 256), ns), dim3(256), 0, st,
                     ds);
  if (sh.any_distinct)
    hipLaunchKernelGGL(k_shuffle, dim3((unsigned)((sh.max_cells + 63) / 64), ns), dim3(64), 0, st,
                       ds);
  if (sh.stripes) {
    // two colour phases of C/2 stripes each, one wavefront per stripe
    const unsigned sgrid = (unsigned)((sh.max_cells_side + 1) / 2);
    for (int q = 0; q < 2; ++q) {
      if (ev) (void)hipEventRecord(ev->begin[q], st);
      hipLaunchKernelGGL(k_stripe_phase<0>, dim3(sgrid, ns), dim3(64), (size_t)sh.max_lds_per_cell, st,
                         ds, q);
      if (ev) (void)hipEventRecord(ev->end[q], st);
    }
    hipError_t e = launch_check_overlap(ds, sh, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_done, dim3(1, ns), dim3(64), 0, st, ds);
    return hipGetLastError();
  }
  const int cpb = sh.cpb;
  const unsigned grid = (unsigned)((sh.max_active + cpb - 1) / cpb);
  const size_t lds = (size_t)cpb * sh.max_lds_per_cell;
  if (sh.ready_queue) {
    const ReadyQueue& rq = sh.queue;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, rq);
    hipLaunchKernelGGL(k_queue_prep, dim3((unsigned)((sh.max_cells + 255) / 256), ns), dim3(256), 0,
                       st, ds, rq);
    const unsigned qgrid = (unsigned)((rq.workers + cpb - 1) / cpb);
    if (ev) (void)hipEventRecord(ev->begin[0], st);
    if (sh.fp32_screen)
      hipLaunchKernelGGL((k_queue_cells<1, 0>), dim3(qgrid), dim3(64 * cpb), lds, st, ds, rq,
                         sh.max_lds_per_cell);
    else if (sh.reject)
      hipLaunchKernelGGL((k_queue_cells<0, 1>), dim3(qgrid), dim3(64 * cpb), lds, st, ds, rq,
                         sh.max_lds_per_cell);
    else
      hipLaunchKernelGGL((k_queue_cells<0, 0>), dim3(qgrid), dim3(64 * cpb), lds, st, ds, rq,
                         sh.max_lds_per_cell);
    if (ev) (void)hipEventRecord(ev->end[0], st);
    hipLaunchKernelGGL(k_queue_check, dim3(1, ns), dim3(64), 0, st, ds, rq);
    hipError_t e = launch_check_overlap(ds, sh, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_done, dim3(1, ns), dim3(64), 0, st, ds);
    return hipGetLastError();
  }
  if (sh.one_launch) {
    // as many wavefronts as one phase has cells; each takes cells of all phases
    if (ev) (void)hipEventRecord(ev->begin[0], st);
    if (sh.fp32_screen)
      hipLaunchKernelGGL((k_sweep_cells<1, 0>), dim3(grid, ns), dim3(64 * cpb), lds, st, ds);
    else if (sh.reject)
      hipLaunchKernelGGL((k_sweep_cells<0, 1>), dim3(grid, ns), dim3(64 * cpb), lds, st, ds);
    else
      hipLaunchKernelGGL((k_sweep_cells<0, 0>), dim3(grid, ns), dim3(64 * cpb), lds, st, ds);
    if (ev) (void)hipEventRecord(ev->end[0], st);
    hipError_t e = launch_check_overlap(ds, sh, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_done, dim3(1, ns), dim3(64), 0, st, ds);
    return hipGetLastError();
  }
  for (int q = 0; q < 4; ++q) {
    if (ev) (void)hipEventRecord(ev->begin[q], st);
    if (sh.fp32_screen)
      hipLaunchKernelGGL((k_phase<1, 0>), dim3(grid, ns), dim3(64 * cpb), lds, st, ds, q);
    else if (sh.reject)
      hipLaunchKernelGGL((k_phase<0, 1>), dim3(grid, ns), dim3(64 * cpb), lds, st, ds, q);
    else
      hipLaunchKernelGGL((k_phase<0, 0>), dim3(grid, ns), dim3(64 * cpb), lds, st, ds, q);
    if (ev) (void)hipEventRecord(ev->end[q], st);
  }
  hipError_t e = launch_check_overlap(ds, sh, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sweep_done, dim3(1, ns), dim3(64), 0, st, ds);
  return hipGetLastError();
}

hipError_t launch_rebin(const Dev* ds, const LaunchShape& sh, hipStream_t st) {
  const unsigned nblk = (unsigned)((sh.max_n + 255) / 256);
  hipLaunchKernelGGL(k_prep, dim3(1, 1), dim3(1024), 0, st, ds, 1);
  hipLaunchKernelGGL(k_count, dim3(nblk, 1), dim3(256), 0, st, ds, 1);
  hipLaunchKernelGGL(k_scan, dim3(1, 1), dim3(1024), 0, st, ds);
  hipLaunchKernelGGL(k_scatter, dim3(nblk, 1), dim3(256), 0, st, ds);
  return hipGetLastError();
}

}  // namespace ec
