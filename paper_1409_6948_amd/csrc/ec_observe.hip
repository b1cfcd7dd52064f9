// gfx950 kernels of the observables measured on a configuration between
// sweeps: the hexatic order parameter Psi (eq. Psi, Sec. 2) with cutoff or
// Delaunay neighbours, and the pair histogram of the pressure route
// (eq. pressure, Sec. 2).  Both read the
// positions and the cell lists of the current grid, which launch_rebin (the
// sweep's own rebin kernels) builds first for walled systems.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ec_internal.h"

namespace ec {
namespace {

// ---------------------------------------------------------------------------
// Hexatic order parameter (Sec. 2, eq. Psi) with cutoff neighbours.  One
// thread per disk scans the 3 x 3 cells around its own (cutoff <= cell side,
// so every neighbour is there), minimum image; exp(6 i phi) is computed as
// ((dx + i dy)^2 / r^2)^3 with complex products and summed per disk in fixed
// point.  Sums per block in a fixed order, then one block adds the block
// sums in order: results repeat bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bond6(double dx, double dy, double r2, double& re, double& im) {
  const double u = (dx * dx - dy * dy) / r2, v = (2.0 * dx * dy) / r2;
  re = u * (u * u - 3.0 * v * v);
  im = v * (3.0 * u * u - v * v);
}

__device__ __forceinline__ void psi6_block_sum(double re, double im, double nb, double* part) {
  __shared__ double sh[3][256];
  const int t = threadIdx.x;
  sh[0][t] = re;
  sh[1][t] = im;
  sh[2][t] = nb;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      sh[0][t] = sh[0][t] + sh[0][t + off];
      sh[1][t] = sh[1][t] + sh[1][t + off];
      sh[2][t] = sh[2][t] + sh[2][t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[3 * blockIdx.x] = sh[0][0];
    part[3 * blockIdx.x + 1] = sh[1][0];
    part[3 * blockIdx.x + 2] = sh[2][0];
  }
}

__global__ void __launch_bounds__(256) k_psi6(const Dev* __restrict__ ds, double rc2) {
  const Dev& d = ds[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double re = 0.0, im = 0.0;
  int nb = 0;
  // bond terms in units of 2^-52 (|term| <= 1): integer sums do not depend on
  // the order of the cell lists, which the atomic rebin leaves unspecified
  long long fre = 0, fim = 0;
  if (k < d.n) {
    const double xk = d.x[k], yk = d.y[k];
    const double L = d.L, half_L = d.half_L;
    const int C = d.C;
    const bool one_cell = C == 1;
    const int c = one_cell ? 0 : d.cell_of[k];
    const int cx = c % C, cy = c / C;
    const int span = one_cell ? 0 : 1;
    for (int oy = -span; oy <= span; ++oy) {
      for (int ox = -span; ox <= span; ++ox) {
        const int nc = ((cy + oy + C) % C) * C + (cx + ox + C) % C;
        const int i0 = one_cell ? 0 : d.cell_start[nc];
        const int i1 = one_cell ? (int)d.n : d.cell_start[nc + 1];
        for (int i = i0; i < i1; ++i) {
          const int l = one_cell ? i : d.cell_ids[i];
          if (l == k) continue;
          double dx = d.x[l] - xk, dy = d.y[l] - yk;
          if (dx < -half_L) dx += L; else if (dx >= half_L) dx -= L;
          if (dy < -half_L) dy += L; else if (dy >= half_L) dy -= L;
          const double r2 = dx * dx + dy * dy;
          if (r2 < rc2) {
            double br, bi;
            bond6(dx, dy, r2, br, bi);
            fre += __double2ll_rn(br * 0x1p52);
            fim += __double2ll_rn(bi * 0x1p52);
            nb += 1;
          }
        }
      }
    }
    if (nb > 0) {
      re = ((double)fre * 0x1p-52) / (double)nb;
      im = ((double)fim * 0x1p-52) / (double)nb;
    }
    d.psi[k] = make_double2(re, im);
  }
  psi6_block_sum(re, im, (double)nb, d.psi_part);
}

__global__ void __launch_bounds__(1024) k_psi6_final(const Dev* __restrict__ ds, int nblocks) {
  const Dev& d = ds[blockIdx.y];
  __shared__ double sh[3][1024];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = t; i < nblocks; i += 1024) {
    a = a + d.psi_part[3 * i];
    b = b + d.psi_part[3 * i + 1];
    c = c + d.psi_part[3 * i + 2];
  }
  sh[0][t] = a;
  sh[1][t] = b;
  sh[2][t] = c;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) {
      sh[0][t] = sh[0][t] + sh[0][t + off];
      sh[1][t] = sh[1][t] + sh[1][t + off];
      sh[2][t] = sh[2][t] + sh[2][t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double n = (double)d.n;
    d.psi_red[0] = sh[0][0] / n;
    d.psi_red[1] = sh[1][0] / n;
    d.psi_red[2] = sh[2][0] / n;
  }
}

// ---------------------------------------------------------------------------
// Hexatic order parameter with Delaunay neighbours (eq. Psi, Sec. 2, as the
// paper defines it).  Disk l is a Delaunay neighbour of k iff the bisector of
// k and l keeps a segment of k's Voronoi cell.  With k at the origin and the
// candidates r_m, the cell is {p : p.r_m <= |r_m|^2 / 2 for all m}; on the
// bisector of l, p = r_l / 2 + t e with e = (-r_ly, r_lx), each other m bounds
// t from one side, and l is a neighbour iff the largest lower bound stays
// below the smallest upper bound (a one-dimensional linear program).
// Candidates are the disks within r_search; the answer is exact when every
// vertex of the cell found lies within r_search / 2 of k (no disk farther
// away can cut it), which is checked: a disk that fails, or that has more
// than kMaxCand candidates, is counted in psi_err and the host reports it.
//
// One wavefront per disk, up to two candidates per lane; each wave takes 64
// consecutive disks in order, so the block sums repeat bit for bit.
// ---------------------------------------------------------------------------
constexpr int kMaxCand = 128;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Candidate j of the wave's list: does its bisector keep a segment of the
// cell, is that segment within the certified radius, and its bond term.
__device__ __forceinline__ void delaunay_edge(const double2* cand, int ncand, int j, double vmax2,
                                              bool& edge, bool& outside, long long& fre,
                                              long long& fim) {
  const double2 rl = cand[j];
  const double ex = -rl.y, ey = rl.x;
  double lo = -INFINITY, hi = INFINITY;
  for (int q = 0; q < ncand; ++q) {
    if (q == j) continue;
    const double2 rm = cand[q];
    const double den = ex * rm.x + ey * rm.y;
    const double rhs = 0.5 * (rm.x * (rm.x - rl.x) + rm.y * (rm.y - rl.y));
    if (den > 0.0) hi = fmin(hi, rhs / den);
    else if (den < 0.0) lo = fmax(lo, rhs / den);
    else if (rhs < 0.0) lo = INFINITY;  // parallel and in front: no segment
  }
  edge = lo < hi;
  outside = false;
  fre = fim = 0;
  if (edge) {
    const double ax = 0.5 * rl.x + lo * ex, ay = 0.5 * rl.y + lo * ey;
    const double bx = 0.5 * rl.x + hi * ex, by = 0.5 * rl.y + hi * ey;
    outside = !(ax * ax + ay * ay <= vmax2) || !(bx * bx + by * by <= vmax2);
    // exp(6 i phi) = ((x + i y)^2 / r^2)^3, in units of 2^-52 (|term| <= 1)
    const double r2 = rl.x * rl.x + rl.y * rl.y;
    const double u = (rl.x * rl.x - rl.y * rl.y) / r2, v = (2.0 * rl.x * rl.y) / r2;
    fre = __double2ll_rn((u * (u * u - 3.0 * v * v)) * 0x1p52);
    fim = __double2ll_rn((v * (3.0 * u * u - v * v)) * 0x1p52);
  }
}

__global__ void k_psi6_delaunay_clear(const Dev* __restrict__ ds) {
  if (threadIdx.x < 2) ds[blockIdx.y].psi_err[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_psi6_delaunay(const Dev* __restrict__ ds, double rs2,
                                                       double vmax2) {
  const Dev& d = ds[blockIdx.y];
  __shared__ double2 cand[4][kMaxCand];
  __shared__ double wsum[4][3];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const double L = d.L, half_L = d.half_L;
  const int C = d.C;
  const bool one_cell = C == 1;
  const int span = one_cell ? 0 : 1;
  double sre = 0.0, sim = 0.0, snb = 0.0;  // this wave's sums, in disk order
  const int64_t k0 = (int64_t)blockIdx.x * 256 + (int64_t)wave * 64;
  for (int j = 0; j < 64; ++j) {
    const int64_t k = k0 + j;
    if (k >= d.n) break;
    wave_fence();  // the previous disk's candidate reads before this disk's writes
    const double xk = d.x[k], yk = d.y[k];
    const int c = one_cell ? 0 : d.cell_of[k];
    const int cx = c % C, cy = c / C;
    int ncand = 0;
    for (int oy = -span; oy <= span; ++oy) {
      for (int ox = -span; ox <= span; ++ox) {
        const int nc = ((cy + oy + C) % C) * C + (cx + ox + C) % C;
        const int i0 = one_cell ? 0 : d.cell_start[nc];
        const int i1 = one_cell ? (int)d.n : d.cell_start[nc + 1];
        for (int i = i0; i < i1; i += 64) {
          const int ii = i + lane;
          bool keep = false;
          double dx = 0.0, dy = 0.0;
          if (ii < i1) {
            const int l = one_cell ? ii : d.cell_ids[ii];
            if (l != k) {
              dx = d.x[l] - xk;
              dy = d.y[l] - yk;
              if (dx < -half_L) dx += L; else if (dx >= half_L) dx -= L;
              if (dy < -half_L) dy += L; else if (dy >= half_L) dy -= L;
              keep = dx * dx + dy * dy < rs2;
            }
          }
          const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
          if (keep) {
            const int slot = ncand + (int)__builtin_amdgcn_mbcnt_hi(
                                         (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (slot < kMaxCand) cand[wave][slot] = make_double2(dx, dy);
          }
          ncand += __popcll(m);
        }
      }
    }
    wave_fence();
    double re = 0.0, im = 0.0;
    int nb = 0;
    if (ncand > kMaxCand) {
      if (lane == 0) atomicAdd(&d.psi_err[1], 1ull);
    } else {
      bool e0 = false, e1 = false, o0 = false, o1 = false;
      long long fre = 0, fim = 0, r1 = 0, i1 = 0;
      if (lane < ncand) delaunay_edge(cand[wave], ncand, lane, vmax2, e0, o0, fre, fim);
      if (lane + 64 < ncand) delaunay_edge(cand[wave], ncand, lane + 64, vmax2, e1, o1, r1, i1);
      if (__builtin_amdgcn_ballot_w64(o0 || o1) != 0 && lane == 0) atomicAdd(&d.psi_err[0], 1ull);
      nb = __popcll(__builtin_amdgcn_ballot_w64(e0)) + __popcll(__builtin_amdgcn_ballot_w64(e1));
      fre = wave_sum_i64(fre + r1);
      fim = wave_sum_i64(fim + i1);
      if (nb > 0) {
        re = ((double)fre * 0x1p-52) / (double)nb;
        im = ((double)fim * 0x1p-52) / (double)nb;
      }
    }
    if (lane == 0) {
      d.psi[k] = make_double2(re, im);
      d.psi_nb[k] = nb;
    }
    sre = sre + re;
    sim = sim + im;
    snb = snb + (double)nb;
  }
  if (lane == 0) {
    wsum[wave][0] = sre;
    wsum[wave][1] = sim;
    wsum[wave][2] = snb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, e = 0.0;
    for (int w = 0; w < 4; ++w) {
      a = a + wsum[w][0];
      b = b + wsum[w][1];
      e = e + wsum[w][2];
    }
    d.psi_part[3 * blockIdx.x] = a;
    d.psi_part[3 * blockIdx.x + 1] = b;
    d.psi_part[3 * blockIdx.x + 2] = e;
  }
}

// ---------------------------------------------------------------------------
// Pair histogram for the pressure route of eq. (pressure), Sec. 2: one thread
// per disk scans the 3 x 3 cells around its own (r_max <= cell side), minimum
// image, bin = floor((sqrt(dx*dx + dy*dy) - sigma) / delta).  Counts go to a
// per-block LDS histogram, then to the global one (integers: exact and
// independent of order).  Pairs closer than sigma are counted apart.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gr(const Dev* __restrict__ ds, double r_max, double delta,
                                            int n_bins) {
  const Dev& d = ds[blockIdx.y];
  __shared__ unsigned int hist[kMaxGrBins + 1];
  for (int i = threadIdx.x; i <= n_bins; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < d.n) {
    const double xk = d.x[k], yk = d.y[k];
    const double L = d.L, half_L = d.half_L, r2max = r_max * r_max, sigma = d.sigma;
    const int C = d.C;
    const bool one_cell = C == 1;
    const int c = one_cell ? 0 : d.cell_of[k];
    const int cx = c % C, cy = c / C;
    const int span = one_cell ? 0 : 1;
    for (int oy = -span; oy <= span; ++oy) {
      for (int ox = -span; ox <= span; ++ox) {
        const int nc = ((cy + oy + C) % C) * C + (cx + ox + C) % C;
        const int i0 = one_cell ? 0 : d.cell_start[nc];
        const int i1 = one_cell ? (int)d.n : d.cell_start[nc + 1];
        for (int i = i0; i < i1; ++i) {
          const int l = one_cell ? i : d.cell_ids[i];
          if (l == k) continue;
          double dx = d.x[l] - xk, dy = d.y[l] - yk;
          if (dx < -half_L) dx += L; else if (dx >= half_L) dx -= L;
          if (dy < -half_L) dy += L; else if (dy >= half_L) dy -= L;
          const double d2 = dx * dx + dy * dy;
          if (!(d2 < r2max)) continue;
          const double dist = sqrt(d2);
          if (dist < sigma) {
            atomicAdd(&hist[n_bins], 1u);
            continue;
          }
          const double t = floor((dist - sigma) / delta);
          if (t < (double)n_bins) atomicAdd(&hist[(int)t], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= n_bins; i += blockDim.x)
    if (hist[i]) atomicAdd(&d.gr_counts[i], (unsigned long long)hist[i]);
}

// ---------------------------------------------------------------------------
// Overlap check (debug): one thread per disk counts the disks j > i closer
// than sigma (1 - 1e-12), minimum image, among the 3 x 3 cells of the
// sweep's grid around its own (a pair closer than sigma < cell side lies in
// neighbouring cells; disks stay in their cells during a sweep), or among all
// disks for one periodic cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void report_overlap(const Dev& d, int64_t i, int64_t j, int64_t sweep) {
  if (atomicAdd(d.ovl, 1ull) == 0ull) {
    d.ovl[1] = (unsigned long long)i;
    d.ovl[2] = (unsigned long long)j;
    d.ovl[3] = (unsigned long long)sweep;
  }
  atomicOr(d.err, ERR_OVERLAP);
}

__global__ void __launch_bounds__(256) k_check_overlap(const Dev* __restrict__ ds) {
  const Dev& d = ds[blockIdx.y];
  if (!d.check_overlap) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const double L = d.L, half = d.half_L;
  const double thr = d.sigma * (1.0 - 1e-12), thr2 = thr * thr;
  const double xi = d.x[i], yi = d.y[i];
  const int64_t sweep = *d.sweep_ctr;
  auto test = [&](int64_t j) {
    if (j <= i) return;
    double dx = d.x[j] - xi, dy = d.y[j] - yi;
    if (dx < -half) dx += L; else if (dx >= half) dx -= L;
    if (dy < -half) dy += L; else if (dy >= half) dy -= L;
    if (dx * dx + dy * dy < thr2) report_overlap(d, i, j, sweep);
  };
  if (d.C == 1) {
    for (int64_t j = i + 1; j < d.n; ++j) test(j);
    return;
  }
  const int c = d.cell_of[i];
  if (d.stripes) {  // the sweep's lists are stripes; a pair closer than sigma lies in neighbouring ones
    for (int side = -1; side <= 1; ++side) {
      const int nk = (c + side + d.C) % d.C;
      if (side == 1 && nk == (c - 1 + d.C) % d.C) continue;  // two stripes only
      for (int t = d.cell_start[nk]; t < d.cell_start[nk + 1]; ++t) test(d.cell_ids[t]);
    }
    return;
  }
  const int cx = c % d.C, cy = c / d.C;
  for (int nb = 0; nb < 9; ++nb) {
    const int ncx = (cx + nb % 3 - 1 + d.C) % d.C, ncy = (cy + nb / 3 - 1 + d.C) % d.C;
    const int nc = ncy * d.C + ncx;
    for (int t = d.cell_start[nc]; t < d.cell_start[nc + 1]; ++t) test(d.cell_ids[t]);
  }
}

}  // namespace

hipError_t launch_psi6(const Dev* ds, const LaunchShape& sh, double r_cut, hipStream_t st) {
  const unsigned nblk = (unsigned)((sh.max_n + 255) / 256);
  if (!sh.periodic) {
    // cell lists of the current sweep's grid (the next sweep builds the same ones)
    hipError_t e = launch_rebin(ds, sh, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_psi6, dim3(nblk, 1), dim3(256), 0, st, ds, r_cut * r_cut);
  hipLaunchKernelGGL(k_psi6_final, dim3(1, 1), dim3(1024), 0, st, ds, (int)nblk);
  return hipGetLastError();
}

hipError_t launch_psi6_delaunay(const Dev* ds, const LaunchShape& sh, double r_search, hipStream_t st) {
  const unsigned nblk = (unsigned)((sh.max_n + 255) / 256);
  hipLaunchKernelGGL(k_psi6_delaunay_clear, dim3(1, 1), dim3(64), 0, st, ds);
  if (!sh.periodic) {
    hipError_t e = launch_rebin(ds, sh, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_psi6_delaunay, dim3(nblk, 1), dim3(256), 0, st, ds, r_search * r_search,
                     0.25 * r_search * r_search);
  hipLaunchKernelGGL(k_psi6_final, dim3(1, 1), dim3(1024), 0, st, ds, (int)nblk);
  return hipGetLastError();
}

hipError_t launch_gr(const Dev* ds, const LaunchShape& sh, double r_max, double delta, int n_bins,
                     hipStream_t st) {
  const unsigned nblk = (unsigned)((sh.max_n + 255) / 256);
  if (!sh.periodic) {
    // cell lists of the current sweep's grid (the next sweep builds the same ones)
    hipError_t e = launch_rebin(ds, sh, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gr, dim3(nblk, 1), dim3(256), 0, st, ds, r_max, delta, n_bins);
  return hipGetLastError();
}

hipError_t launch_check_overlap(const Dev* ds, const LaunchShape& sh, hipStream_t st) {
  if (!sh.check_overlap) return hipSuccess;
  const unsigned nblk = (unsigned)((sh.max_n + 255) / 256);
  hipLaunchKernelGGL(k_check_overlap, dim3(nblk, (unsigned)sh.n_sys), dim3(256), 0, st, ds);
  return hipGetLastError();
}

}  // namespace ec
