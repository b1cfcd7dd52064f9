"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  The product (the HIP library and its
Python binding) never calls it.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

DIR_XY, DIR_ISO, DIR_X = 0, 1, 2
START_REPLACE, START_DISTINCT = 0, 1
BOUNDARY_REFLECT, BOUNDARY_REJECT, BOUNDARY_STRIPES = 0, 1, 2
EV_LIFT, EV_FROZEN, EV_WALL_X, EV_WALL_Y, EV_PSEUDO, EV_END = 1, 2, 3, 4, 5, 6
CNT_LIFTS, CNT_FROZEN, CNT_WALLS, CNT_CHAINS, CNT_PSEUDO, CNT_NCOL = 0, 1, 2, 3, 4, 5


class Params(C.Structure):
    _fields_ = [("n", C.c_int64), ("sigma", C.c_double), ("eta", C.c_double),
                ("ell", C.c_double), ("cells", C.c_int32), ("chains_per_cell", C.c_int32),
                ("dir_mode", C.c_int32), ("start_mode", C.c_int32), ("seed", C.c_uint64),
                ("system", C.c_uint32), ("boundary", C.c_uint32)]


class Event(C.Structure):
    _fields_ = [("chain", C.c_int64), ("cell", C.c_int32), ("kind", C.c_int32),
                ("gid", C.c_int64), ("active", C.c_int64), ("s", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("ax", C.c_double),
                ("ay", C.c_double), ("px", C.c_double), ("py", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        src = os.path.join(os.path.dirname(path), "ec_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = C.CDLL(path)
        dp, u64p, i32p, i64p = (C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                C.POINTER(C.c_int32), C.POINTER(C.c_int64))
        pp = C.POINTER(Params)
        L.orc_box_length.restype = C.c_double
        L.orc_box_length.argtypes = [C.c_int64, C.c_double, C.c_double]
        L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.orc_lattice.argtypes = [pp, dp, dp]
        L.orc_sweep_draws.argtypes = [pp, C.c_int64, dp, dp, i32p]
        L.orc_start_index.restype = C.c_int64
        L.orc_start_index.argtypes = [pp, C.c_int64, C.c_int32, C.c_int64, C.c_int64]
        L.orc_direction.argtypes = [pp, C.c_int64, C.c_int32, C.c_int64, dp, dp]
        L.orc_collision_distance.restype = C.c_double
        L.orc_collision_distance.argtypes = [C.c_double] * 5
        L.orc_assign_cells.restype = C.c_int
        L.orc_assign_cells.argtypes = [pp, dp, dp, C.c_int64, i32p]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [pp, dp, dp, C.c_int64, C.c_int64, dp, u64p, u64p]
        L.orc_run_cells.restype = C.c_int
        L.orc_run_cells.argtypes = [pp, dp, dp, C.c_int64, C.c_int32, i32p, C.c_int32, dp, u64p,
                                    u64p]
        L.orc_psi6.argtypes = [pp, dp, dp, C.c_double, dp, dp, dp, dp]
        L.orc_psi6_box.argtypes = [C.c_int64, C.c_double, dp, dp, C.c_double, dp, dp, dp, dp]
        L.orc_pair_histogram.argtypes = [pp, dp, dp, C.c_double, C.c_int32, u64p, u64p]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_start_list.argtypes = [pp, C.c_int64, C.c_int32, C.c_int64, C.c_int64, i64p]
        L.orc_cell_chains.restype = C.c_int
        L.orc_cell_chains.argtypes = [pp, C.c_double, C.c_int64, dp, dp, C.c_int64, dp, dp,
                                      C.c_int64, dp, dp, u64p]
        L.orc_min_pair_distance.restype = C.c_double
        L.orc_min_pair_distance.argtypes = [C.c_int64, C.c_double, dp, dp, C.c_double, i64p, i64p]
        L.orc_set_log.argtypes = [C.POINTER(Event), C.c_int64]
        L.orc_log_count.restype = C.c_int64
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def params(n, eta, ell, cells, dir_mode=DIR_ISO, seed=1, sigma=1.0, chains_per_cell=0,
           start_mode=START_REPLACE, system=0, boundary=BOUNDARY_REFLECT):
    return Params(int(n), float(sigma), float(eta), float(ell), int(cells), int(chains_per_cell),
                  int(dir_mode), int(start_mode), int(seed), int(system), int(boundary))


def set_threads(n):
    """Threads of the phase-parallel mode (1 = serial); results are identical."""
    lib().orc_set_threads(int(n))


def box_length(n, sigma, eta):
    return lib().orc_box_length(int(n), float(sigma), float(eta))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def lattice(p):
    """The k x k start lattice (k = ceil(sqrt(N)); spacing a = L/k, odd rows
    shifted by a/2).  Its nearest neighbours lie a apart, so it overlaps when
    a < sigma (eta > pi/4 for N = k^2); such a start is refused, as the
    library refuses it, since no chain could then make progress."""
    k = int(math.ceil(math.sqrt(p.n)))
    while k * k < p.n:
        k += 1
    if not box_length(p.n, p.sigma, p.eta) / k > p.sigma:
        raise ValueError("start lattice spacing below sigma (eta > pi/4): the start would overlap")
    x = np.zeros(p.n, dtype=np.float64)
    y = np.zeros(p.n, dtype=np.float64)
    lib().orc_lattice(C.byref(p), _ptr(x, C.c_double), _ptr(y, C.c_double))
    return x, y


def sweep_draws(p, sweep):
    sx, sy = C.c_double(), C.c_double()
    perm = np.zeros(4, dtype=np.int32)
    lib().orc_sweep_draws(C.byref(p), int(sweep), C.byref(sx), C.byref(sy), _ptr(perm, C.c_int32))
    return sx.value, sy.value, perm


def start_index(p, sweep, cell, chain, n_c):
    return lib().orc_start_index(C.byref(p), int(sweep), int(cell), int(chain), int(n_c))


def direction(p, sweep, cell, chain):
    dx, dy = C.c_double(), C.c_double()
    lib().orc_direction(C.byref(p), int(sweep), int(cell), int(chain), C.byref(dx), C.byref(dy))
    return dx.value, dy.value


def collision_distance(rx, ry, dx, dy, sigma=1.0):
    return lib().orc_collision_distance(rx, ry, dx, dy, sigma)


def start_list(p, sweep, cell, n_c, n_m):
    """Start indices of the n_m chains of a cell with n_c disks (step 5)."""
    out = np.zeros(max(int(n_m), 1), dtype=np.int64)
    lib().orc_start_list(C.byref(p), int(sweep), int(cell), int(n_c), int(n_m), _ptr(out, C.c_int64))
    return out[:int(n_m)]


def cell_chains(p, w, own_x, own_y, frozen_x=(), frozen_y=(), n_chains=1, trace=True):
    """Chains of one walled cell [0, w]^2 (see orc_cell_chains): returns the
    final positions, the trace (n_chains, n_own, 2) or None, the contact sum
    and the counts."""
    ox = np.ascontiguousarray(own_x, dtype=np.float64).copy()
    oy = np.ascontiguousarray(own_y, dtype=np.float64).copy()
    fx = np.ascontiguousarray(frozen_x, dtype=np.float64)
    fy = np.ascontiguousarray(frozen_y, dtype=np.float64)
    n_own, n_fr = len(ox), len(fx)
    tr = np.zeros((int(n_chains), n_own, 2)) if trace else None
    acc = np.zeros(1)
    cnt = np.zeros(CNT_NCOL, dtype=np.uint64)
    dp = C.POINTER(C.c_double)
    rc = lib().orc_cell_chains(C.byref(p), float(w), n_own, _ptr(ox, C.c_double), _ptr(oy, C.c_double),
                               n_fr, fx.ctypes.data_as(dp) if n_fr else None,
                               fy.ctypes.data_as(dp) if n_fr else None, int(n_chains),
                               tr.ctypes.data_as(dp) if trace else None, _ptr(acc, C.c_double),
                               _ptr(cnt, C.c_uint64))
    if rc != 0:
        raise ValueError("invalid arguments")
    return ox, oy, tr, float(acc[0]), cnt


def min_pair_distance(x, y, L, r_cut=1.0):
    """(smallest minimum-image pair distance below r_cut or inf, i, j)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    i, j = C.c_int64(), C.c_int64()
    d = lib().orc_min_pair_distance(len(x), float(L), _ptr(x, C.c_double), _ptr(y, C.c_double),
                                    float(r_cut), C.byref(i), C.byref(j))
    return d, i.value, j.value


def assign_cells(p, x, y, sweep):
    cell_of = np.zeros(p.n, dtype=np.int32)
    rc = lib().orc_assign_cells(C.byref(p), _ptr(x, C.c_double), _ptr(y, C.c_double), int(sweep),
                                _ptr(cell_of, C.c_int32))
    if rc != 0:
        raise ValueError("invalid parameters")
    return cell_of


class State:
    """Positions plus per-cell accumulators, advanced in place by the oracle."""

    def __init__(self, p, x=None, y=None):
        self.p = p
        if x is None:
            x, y = lattice(p)
        self.x = np.ascontiguousarray(x, dtype=np.float64).copy()
        self.y = np.ascontiguousarray(y, dtype=np.float64).copy()
        nc = p.cells * p.cells
        self.acc_delta = np.zeros(nc, dtype=np.float64)
        self.acc_cnt = np.zeros((nc, CNT_NCOL), dtype=np.uint64)
        self.sweep = 0
        self.digests = []

    def run(self, n_sweeps):
        d = np.zeros(max(int(n_sweeps), 1), dtype=np.uint64)
        rc = lib().orc_run(C.byref(self.p), _ptr(self.x, C.c_double), _ptr(self.y, C.c_double),
                           self.sweep, int(n_sweeps), _ptr(self.acc_delta, C.c_double),
                           _ptr(self.acc_cnt, C.c_uint64), _ptr(d, C.c_uint64))
        if rc != 0:
            raise ValueError("invalid parameters")
        self.sweep += int(n_sweeps)
        self.digests.extend(int(v) for v in d[:int(n_sweeps)])
        return d[:int(n_sweeps)]

    def run_cells(self, sweep, cells, n_phases=1):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        dig = np.zeros(len(cells), dtype=np.uint64)
        rc = lib().orc_run_cells(C.byref(self.p), _ptr(self.x, C.c_double),
                                 _ptr(self.y, C.c_double), int(sweep), int(n_phases),
                                 _ptr(cells, C.c_int32), len(cells),
                                 _ptr(self.acc_delta, C.c_double), _ptr(self.acc_cnt, C.c_uint64),
                                 _ptr(dig, C.c_uint64))
        if rc != 0:
            raise ValueError("invalid parameters")
        return dig

    def tallies(self):
        """(sum of contact projections, lifts, frozen, walls, chains, pseudo) in cell order."""
        s = 0.0
        for v in self.acc_delta:  # fixed cell order
            s += float(v)
        cnt = self.acc_cnt.sum(axis=0)
        return s, [int(v) for v in cnt]

    def pressure(self):
        """Z = beta P / rho = 1 + sum(contact projections) / (chains * ell)."""
        s, cnt = self.tallies()
        chains = cnt[CNT_CHAINS]
        z = 1.0 + s / (chains * self.p.ell)
        L = box_length(self.p.n, self.p.sigma, self.p.eta)
        return z, z * self.p.n * self.p.sigma ** 2 / (L * L)


def psi6_box(n, L, x, y, r_cut=1.4):
    """Hexatic order parameter (Sec. 2, eq. Psi) with cutoff neighbours in a
    periodic L x L box: returns (Psi as complex, mean neighbour count,
    per-disk Psi_k as a complex array)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    re, im, nb = C.c_double(), C.c_double(), C.c_double()
    per = np.zeros(2 * int(n), dtype=np.float64)
    dp = C.POINTER(C.c_double)
    lib().orc_psi6_box(int(n), float(L), x.ctypes.data_as(dp), y.ctypes.data_as(dp), float(r_cut),
                       C.byref(re), C.byref(im), C.byref(nb), per.ctypes.data_as(dp))
    return complex(re.value, im.value), nb.value, per[0::2] + 1j * per[1::2]


def psi6(p, x, y, r_cut=1.4):
    """psi6_box in the box of the parameters p."""
    return psi6_box(p.n, box_length(p.n, p.sigma, p.eta), x, y, r_cut)


def pair_histogram(p, x, y, r_max, n_bins):
    """Ordered-pair counts in bins [sigma + i delta, sigma + (i+1) delta),
    delta = (r_max - sigma)/n_bins, and the number of pairs closer than sigma."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    counts = np.zeros(int(n_bins), dtype=np.uint64)
    ov = C.c_uint64(0)
    dp = C.POINTER(C.c_double)
    lib().orc_pair_histogram(C.byref(p), x.ctypes.data_as(dp), y.ctypes.data_as(dp), float(r_max),
                             int(n_bins), counts.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(ov))
    return counts, ov.value


def run_logged(p, x, y, sweep0, n_sweeps, capacity=1 << 20):
    """Run with the event log on; returns (x, y, events array)."""
    st = State(p, x, y)
    st.sweep = sweep0
    buf = (Event * capacity)()
    lib().orc_set_log(buf, capacity)
    try:
        st.run(n_sweeps)
        n = lib().orc_log_count()
    finally:
        lib().orc_set_log(None, 0)
    if n > capacity:
        raise RuntimeError("event log overflow")
    ev = np.ctypeslib.as_array(buf)[:n].copy()
    return st, ev
