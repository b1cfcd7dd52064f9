"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests
and the benchmark.  This module holds parameter sets and initial
configurations only; none of the method's arithmetic lives here.

The workloads are synthetic hard-disk systems of the kind the paper studies
(N = 64^2 ... 256^2 disks near the liquid-hexatic transition, eta 0.70-0.72,
square box with periodic boundaries, square simulation cells).  Every system
starts from the k x k lattice unless a test supplies its own positions.
"""
import math

import numpy as np

# Headline and parity workloads: (name, N, eta, cells per side, ell, sweeps)
WORKLOADS = {
    # one periodic cell, +x/+y alternating chains
    "serial_256": dict(n=256, eta=0.70, cells=1, ell=20.0, dir_mode=0, sweeps=200, seed=1,
                       label="N=256 eta=0.70, one periodic cell"),
    # 16 x 16 simulation cells, isotropic chains
    "pec_65k": dict(n=65536, eta=0.70, cells=16, ell=20.0, dir_mode=1, sweeps=1000, seed=1,
                    label="N=65536 eta=0.70"),
    # headline: 64 x 64 cells, one million disks
    "pec_1m": dict(n=1048576, eta=0.72, cells=64, ell=20.0, dir_mode=1, sweeps=500, seed=1,
                   label="N=1M eta=0.72"),
    # 256 x 256 cells, 16.7 million disks; FP32 screening with FP64 commits,
    # pressure and Psi on the device
    "pec_16m": dict(n=16777216, eta=0.716, cells=256, ell=30.0, dir_mode=1, sweeps=100, seed=1,
                    precision="fp32-screen", psi6=True, label="N=16.7M eta=0.716"),
}


def box_length(n, eta, sigma=1.0):
    return sigma * math.sqrt(n * math.pi / (4.0 * eta))


def separated_points(n, L, min_dist, seed, max_tries=200000):
    """Random sequential addition in a periodic L x L box (uniform, seeded)."""
    rng = np.random.default_rng(seed)
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place points")
        p = rng.uniform(0.0, L, size=2)
        ok = True
        for q in pts:
            d = p - q
            d -= L * np.round(d / L)
            if d @ d < min_dist * min_dist:
                ok = False
                break
        if ok:
            pts.append(p)
    a = np.array(pts)
    return np.ascontiguousarray(a[:, 0]), np.ascontiguousarray(a[:, 1])


def batch_systems(n_sys=64, seed=0):
    """Meta-draws of the batched workload: N log-uniform in [4096, 262144]
    rounded to an even square, eta uniform in [0.30, 0.72], about 64 disks per
    cell (even cell count with cell side above one diameter)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_sys):
        n = math.exp(rng.uniform(math.log(4096), math.log(262144)))
        k = max(2, int(round(math.sqrt(n) / 2.0)) * 2)
        n = k * k
        eta = rng.uniform(0.30, 0.72)
        c = max(4, int(round(math.sqrt(n / 64.0) / 2.0)) * 2)
        L = box_length(n, eta)
        while c > 4 and L / c <= 3.0:
            c -= 2
        out.append(dict(n=n, eta=eta, cells=c, ell=20.0, dir_mode=1, seed=i + 1))
    return out


def rods_on_a_ring(n, L, seed):
    """n unit-diameter disks on the row y = L/2 with random free gaps (uniform
    on the simplex of total length L - n)."""
    rng = np.random.default_rng(seed)
    g = rng.dirichlet(np.ones(n)) * (L - n)
    x = np.cumsum(g + 1.0) - g[0] - 1.0 + 0.1
    x = np.mod(x, L)
    return np.ascontiguousarray(x), np.full(n, L / 2)
