"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Positions are compared bit for bit, and so are the event digests, the
per-cell pressure sums and the event counts: both sides follow the same
arithmetic and random-number contract, so the trajectories are identical.
Small systems are compared over whole runs here; the full-size workloads are
compared in test_gpu_full_size.py.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from tests import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_6948_amd as P
    P.load_library()
    return P


def _gpu_system(P, n, eta, ell, cells, dir_mode, seed=1, chains_per_cell=0, start_mode=0,
                cells_per_block=0, flags=0, precision=0):
    p = P.make_params(n, eta, ell, cells, dir_mode=dir_mode, seed=seed,
                      chains_per_cell=chains_per_cell, start_mode=start_mode,
                      cells_per_block=cells_per_block, flags=flags, precision=precision)
    return P.System(p)


def _oracle_state(n, eta, ell, cells, dir_mode, seed=1, chains_per_cell=0, start_mode=0, x=None,
                  y=None, boundary=0):
    p = O.params(n, eta, ell, cells, dir_mode=dir_mode, seed=seed,
                 chains_per_cell=chains_per_cell, start_mode=start_mode, boundary=boundary)
    return O.State(p, x, y)


def _compare_full(P, n, eta, ell, cells, dir_mode, sweeps, seed=1, chains_per_cell=0,
                  start_mode=0, x=None, y=None, cells_per_block=0, flags=0, precision=0):
    _say(f"[parity] n={n} eta={eta} ell={ell} C={cells} dir={dir_mode} sweeps={sweeps} "
         f"seed={seed} n_m={chains_per_cell} start={start_mode} cpb={cells_per_block} "
         f"flags={flags} precision={precision}")
    boundary = 1 if flags & P.EC_FLAG_REJECT else 0
    st = _oracle_state(n, eta, ell, cells, dir_mode, seed, chains_per_cell, start_mode, x, y, boundary)
    g = _gpu_system(P, n, eta, ell, cells, dir_mode, seed, chains_per_cell, start_mode,
                    cells_per_block, flags, precision)
    gx, gy = g.get_positions()
    if x is None:
        np.testing.assert_array_equal(gx, st.x)  # the two start lattices agree bit for bit
        np.testing.assert_array_equal(gy, st.y)
    else:
        g.set_positions(st.x, st.y)
    st.run(sweeps)
    g.sweep(sweeps)
    gx, gy = g.get_positions()
    dig = g.get_digests(sweeps)
    delta, cnt = g.get_cell_tallies()
    np.testing.assert_array_equal(dig, np.array(st.digests[-sweeps:], dtype=np.uint64))
    np.testing.assert_array_equal(gx, st.x)
    np.testing.assert_array_equal(gy, st.y)
    np.testing.assert_array_equal(delta, st.acc_delta)
    np.testing.assert_array_equal(cnt, st.acc_cnt)
    z, bp, counts = g.measure_pressure()
    oz, obp = st.pressure()
    assert z == oz and bp == obp
    return g, st


def test_serial_256_xy_lattice(P):
    """One periodic cell, +x/+y chains from the lattice (exact distance ties),
    over the configuration's whole run of 200 sweeps."""
    w = inputs.WORKLOADS["serial_256"]
    _compare_full(P, w["n"], w["eta"], w["ell"], 1, 0, w["sweeps"])


def test_periodic_isotropic_small(P):
    _compare_full(P, 400, 0.60, 7.0, 1, 1, 6, seed=3)


def test_two_disks_free_flight_cap(P):
    L = 4.0
    eta = 2 * math.pi / (4 * L * L)
    _compare_full(P, 2, eta, 3.0, 1, 1, 300, seed=17, x=np.array([0.5, 2.5]),
                  y=np.array([0.5, 0.5]))


def test_rods_on_a_ring(P):
    n, L = 16, 32.0
    x, y = inputs.rods_on_a_ring(n, L, seed=5)
    _compare_full(P, n, n * math.pi / (4 * L * L), 10.0, 1, 2, 40, seed=23, x=x, y=y)


def test_walled_scan_search(P):
    """Walled cells with the search over every staged disk (no bin window)."""
    _compare_full(P, 1024, 0.60, 5.0, 4, 1, 2, seed=3, flags=1)


@pytest.mark.parametrize("n,eta,cells,ell,sweeps", [
    (1024, 0.60, 4, 5.0, 2),      # small, window search
    (4096, 0.72, 8, 20.0, 3),     # small cells (9.5 sigma), dense
    (4096, 0.30, 8, 20.0, 3),     # dilute: long flights, the window guard falls back often
    (2304, 0.65, 6, 12.0, 3),     # 3 x 3 blocks per colour, ragged
    (4096, 0.70, 4, 20.0, 2),     # large cells (17 sigma)
    (576, 0.70, 8, 5.0, 3),       # 3 bins per cell side: all but the middle bin border a wall
    (1024, 0.70, 8, 5.0, 3),      # 4 bins per cell side
])
def test_walled_cells(P, n, eta, cells, ell, sweeps):
    _compare_full(P, n, eta, ell, cells, 1, sweeps, seed=7)


@pytest.mark.parametrize("chains_per_cell", [0, 3])
def test_walled_cells_with_empty_cells(P, chains_per_cell):
    """N = 16 in 4 x 4 cells at eta = 0.05 (one disk per cell on average): on
    the shifted grids of later sweeps some cells hold no disk and run no chain,
    with n_m = n_c and with a fixed n_m = 3 alike (Sec. 3.4, step 5 draws
    from the cell's own disks)."""
    _compare_full(P, 16, 0.05, 5.0, 4, 1, 3, seed=7, chains_per_cell=chains_per_cell)
    # the case does exercise empty cells (per-sweep chain tallies of the oracle)
    st = O.State(O.params(16, 0.05, 5.0, 4, dir_mode=O.DIR_ISO, seed=7,
                          chains_per_cell=chains_per_cell))
    empty = 0
    for _ in range(3):
        before = st.acc_cnt[:, O.CNT_CHAINS].copy()
        st.run(1)
        empty += int(((st.acc_cnt[:, O.CNT_CHAINS] - before) == 0).sum())
    assert empty > 0


def test_tiny_chain_length(P):
    """ell = 1e-7 sigma from the lattice at eta = 0.60: every chain is one
    event, its end (a move of ell, no lift, no contact)."""
    g, st = _compare_full(P, 1024, 0.60, 1e-7, 4, 1, 2, seed=7)
    cnt = st.acc_cnt.sum(axis=0)
    assert cnt[O.CNT_LIFTS] == 0 and cnt[O.CNT_FROZEN] == 0 and cnt[O.CNT_CHAINS] == 2 * 1024


def test_near_jammed_lattice(P):
    """eta = 0.78, just below pi/4, where the start lattice would overlap:
    neighbours 0.35 % of sigma apart, about a thousand events per chain of
    20 sigma: the densest start the lattice allows."""
    _compare_full(P, 1024, 0.78, 20.0, 4, 1, 2, seed=7)


@pytest.mark.parametrize("cpb", [1, 2, 4])
def test_walled_cells_per_workgroup(P, cpb):
    _compare_full(P, 4096, 0.72, 20.0, 8, 1, 2, seed=8, cells_per_block=cpb)


@pytest.mark.parametrize("n,eta,cells,ell,sweeps,cpb", [
    (4096, 0.72, 8, 20.0, 3, 0),
    (2304, 0.65, 6, 12.0, 3, 1),
])
def test_walled_cells_phase_launches(P, n, eta, cells, ell, sweeps, cpb):
    """One launch per colour phase (the launch boundary as the barrier) gives
    the same positions, digests and tallies as the default one-launch sweep."""
    _compare_full(P, n, eta, ell, cells, 1, sweeps, seed=7, cells_per_block=cpb,
                  flags=P.EC_FLAG_PHASE_LAUNCHES)


def test_schedules_agree_at_full_size(P):
    """N = 1,048,576, eta = 0.72, 64 x 64 cells, ell = 20 sigma, 3 sweeps: the
    one-launch sweep of the bench equals the phase-by-phase sweep bit for bit."""
    _say("[parity] pec_1m: one-launch vs phase launches, 3 sweeps")
    out = []
    for flags in (0, P.EC_FLAG_PHASE_LAUNCHES):
        g = _gpu_system(P, 1048576, 0.72, 20.0, 64, 1, seed=1, flags=flags)
        g.sweep(3)
        out.append(g.get_positions() + (g.get_digests(3),) + g.get_cell_tallies())
        g.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)


def test_dependency_wait_limit(P):
    """A wait limit of 0 fails every wait of the one-launch sweep: the sweep
    ends with device error bit 16, reported by the next synchronising call.
    The phase-launch schedule has no waits and ignores the limit."""
    import paper_1409_6948_amd.ec as E
    g = _gpu_system(P, 4096, 0.70, 10.0, 8, 1, seed=5)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(E.ECError) as ei:
            g.set_dep_wait_limit(bad)
        assert ei.value.status == E.EC_E_INVALID
    g.set_dep_wait_limit(0.0)
    _say("[parity] wait limit 0: expecting device error bit 16")
    with pytest.raises(E.ECError) as ei:
        g.sweep(1)
        g.get_positions()
    assert ei.value.status == E.EC_E_STATE
    assert "bits 0x10" in str(ei.value)
    h = _gpu_system(P, 4096, 0.70, 10.0, 8, 1, seed=5, flags=P.EC_FLAG_PHASE_LAUNCHES)
    h.set_dep_wait_limit(0.0)
    h.sweep(1)
    h.get_positions()


@pytest.mark.parametrize("n,eta,cells,ell,sweeps,flags", [
    (1024, 0.55, 4, 1.0, 3, 0),
    (4096, 0.70, 8, 2.0, 3, 0),
    (4096, 0.30, 8, 3.0, 2, 0),           # dilute: long flights, full-cell searches
    (2304, 0.65, 6, 2.0, 2, 2),           # one launch per phase
    (1024, 0.30, 4, 100.0, 2, 0),         # every chain longer than the cell: all undone
    (576, 0.70, 8, 1.0, 3, 0),            # 3 bins per cell side
])
def test_rejection_variant(P, n, eta, cells, ell, sweeps, flags):
    """Rejection at the cell boundary against the oracle bit for bit."""
    _compare_full(P, n, eta, ell, cells, 1, sweeps, seed=5, flags=flags | P.EC_FLAG_REJECT)


def test_rejection_identity_and_counts(P):
    """ell far above the cell: every chain is rejected and the configuration
    keeps its bits; the wall and frozen counts are the rejections."""
    g = _gpu_system(P, 1024, 0.30, 100.0, 4, 1, seed=6, flags=P.EC_FLAG_REJECT)
    x0, y0 = g.get_positions()
    g.sweep(2)
    x1, y1 = g.get_positions()
    np.testing.assert_array_equal(x0, x1)
    np.testing.assert_array_equal(y0, y1)
    _, _, c = g.measure_pressure()
    assert c["lifts"] == 0 and c["walls"] + c["frozen"] == c["chains"] == 2048


def test_fixed_chains_per_cell(P):
    _compare_full(P, 1024, 0.60, 5.0, 4, 1, 4, seed=9, chains_per_cell=7)


def test_distinct_start_negative_control(P):
    _compare_full(P, 1024, 0.60, 5.0, 4, 1, 3, seed=4, chains_per_cell=50, start_mode=1)


def test_resume_split_calls(P):
    g1 = _gpu_system(P, 4096, 0.70, 10.0, 8, 1, seed=12)
    g1.sweep(3)
    g2 = _gpu_system(P, 4096, 0.70, 10.0, 8, 1, seed=12)
    g2.sweep(1)
    g2.sweep(2)
    a, b = g1.get_positions(), g2.get_positions()
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(g1.get_digests(3), g2.get_digests(3))


def test_set_positions_rejects_overlap(P):
    import paper_1409_6948_amd.ec as E
    g = _gpu_system(P, 1024, 0.5, 5.0, 4, 1)
    x0, y0 = g.get_positions()
    x, y = x0.copy(), y0.copy()
    x[5] = x[6] + 0.3
    y[5] = y[6]
    with pytest.raises(E.ECError) as ei:
        g.set_positions(x, y)
    assert ei.value.status == E.EC_E_OVERLAP
    x1, y1 = g.get_positions()
    np.testing.assert_array_equal(x1, x0)
    small = np.zeros(3)
    ptr = small.ctypes.data_as(E.C.POINTER(E.C.c_double))
    assert E.load_library().ec_get_positions(g.h, ptr, ptr, 3) == E.EC_E_INVALID


# ---------------------------------------------------------------------------
# FP32-screened form: the same events as the FP64 form, hence as the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,eta,cells,ell,sweeps", [
    (4096, 0.72, 8, 20.0, 3),
    (4096, 0.30, 8, 20.0, 3),
    (2304, 0.65, 6, 12.0, 2),
    (576, 0.70, 8, 5.0, 3),       # 3 bins per cell side
])
def test_fp32_screen_matches_oracle(P, n, eta, cells, ell, sweeps):
    _compare_full(P, n, eta, ell, cells, 1, sweeps, precision=1)


def test_fp32_screen_equals_fp64_at_full_size(P):
    """1M disks, eta 0.72, 64 x 64 cells: positions and per-sweep digests of the
    screened form equal those of the FP64 form over 100 sweeps (about 2.6e10
    events, each screened)."""
    w = inputs.WORKLOADS["pec_1m"]
    sweeps = 100
    _say(f"[fp32] pec_1m: {sweeps} sweeps in each precision")
    out = []
    for prec in (0, 1):
        g = _gpu_system(P, w["n"], w["eta"], w["ell"], w["cells"], 1, seed=w["seed"],
                        precision=prec)
        g.sweep(sweeps)
        x, y = g.get_positions()
        out.append((x, y, g.get_digests(sweeps), g.measure_pressure()[2]))
        g.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])
    assert out[0][3] == out[1][3]
