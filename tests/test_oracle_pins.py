"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a published
known-answer (numpy's Philox4x64-10), closed-form geometry, exact small-system
results, invariants of the event chain, and the hard-disk virial series.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import cones, inputs

SIG = 1.0


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def _numpy_philox_block(ctr, key):
    """Block for counter `ctr` from numpy's Philox4x64-10, which increments its
    counter (with carry) before producing a block."""
    c = [int(v) for v in ctr]
    # counter one step before ctr, with borrow across words
    prev = list(c)
    for i in range(4):
        if prev[i] > 0:
            prev[i] -= 1
            break
        prev[i] = (1 << 64) - 1
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(prev, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [1, 2]),
    ([5, 123, 7, 0], [1, 3]),
    ([0, 1 << 40, 3, 2], [42, 2]),
    ([(1 << 64) - 1] * 4, [(1 << 64) - 1] * 2),
])
def test_philox_matches_numpy(ctr, key):
    assert [int(v) for v in O.philox(ctr, key)] == _numpy_philox_block(ctr, key)


def test_philox_random_counters_match_numpy():
    rng = np.random.default_rng(7)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(0, 1 << 63, size=4)]
        key = [int(v) for v in rng.integers(0, 1 << 63, size=2)]
        assert [int(v) for v in O.philox(ctr, key)] == _numpy_philox_block(ctr, key)


def test_start_index_uniform_chi2():
    """Starts are drawn with replacement, uniformly over the cell's disks."""
    p = O.params(4096, 0.7, 1.0, 8)
    n_c = 37
    counts = np.zeros(n_c)
    for k in range(n_c * 400):
        counts[O.start_index(p, 3, 5, k, n_c)] += 1
    expected = counts.sum() / n_c
    chi2 = ((counts - expected) ** 2 / expected).sum()
    # 36 degrees of freedom: P(chi2 > 70) ~ 6e-4
    assert chi2 < 70.0


def test_directions_unit_and_isotropic():
    p = O.params(4096, 0.7, 1.0, 8)
    ang = []
    for k in range(20000):
        dx, dy = O.direction(p, 1, 2, k)
        assert abs(math.hypot(dx, dy) - 1.0) < 4e-16
        ang.append(math.atan2(dy, dx))
    hist, _ = np.histogram(ang, bins=24, range=(-math.pi, math.pi))
    e = len(ang) / 24
    chi2 = ((hist - e) ** 2 / e).sum()
    assert chi2 < 55.0  # 23 dof, P ~ 2e-4


def test_xy_and_x_directions():
    p = O.params(256, 0.7, 1.0, 1, dir_mode=O.DIR_XY)
    assert O.direction(p, 0, 0, 0) == (1.0, 0.0)
    assert O.direction(p, 0, 0, 1) == (0.0, 1.0)
    p = O.params(256, 0.7, 1.0, 1, dir_mode=O.DIR_X)
    assert O.direction(p, 0, 0, 1) == (1.0, 0.0)


def test_sweep_draws_shift_and_colour_order():
    p = O.params(65536, 0.7, 20.0, 16)
    w = O.box_length(p.n, 1.0, 0.7) / 16
    perms = {}
    sx_all = []
    for s in range(2400):
        sx, sy, perm = O.sweep_draws(p, s)
        assert 0.0 <= sx <= w and 0.0 <= sy <= w
        assert sorted(perm.tolist()) == [0, 1, 2, 3]
        perms[tuple(perm)] = perms.get(tuple(perm), 0) + 1
        sx_all.append(sx / w)
    assert len(perms) == 24
    cnt = np.array(list(perms.values()))
    chi2 = ((cnt - 100.0) ** 2 / 100.0).sum()
    assert chi2 < 55.0
    hist, _ = np.histogram(sx_all, bins=10, range=(0, 1))
    assert ((hist - 240.0) ** 2 / 240.0).sum() < 30.0


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------
def _contact_by_bisection(rx, ry, dx, dy, sigma):
    """First s >= 0 with |r - s d| = sigma, found by bisection on the distance
    function (an independent method from the closed form)."""
    f = lambda s: math.hypot(rx - s * dx, ry - s * dy) - sigma
    if f(0.0) <= 0.0:
        a = rx * dx + ry * dy
        return 0.0 if a > 0 else math.inf
    # closest approach
    s_min = rx * dx + ry * dy
    if s_min <= 0.0 or f(s_min) >= 0.0:
        return math.inf
    lo, hi = 0.0, s_min
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_collision_distance_closed_cases():
    assert O.collision_distance(3.0, 0.0, 1.0, 0.0) == 2.0           # head-on
    assert O.collision_distance(-3.0, 0.0, 1.0, 0.0) == math.inf     # behind
    assert O.collision_distance(3.0, 1.0, 1.0, 0.0) == math.inf      # grazing miss |c| = sigma
    assert O.collision_distance(3.0, 1.5, 1.0, 0.0) == math.inf      # miss
    assert O.collision_distance(0.0, 2.0, 0.0, 1.0) == 1.0           # along y
    assert O.collision_distance(1.0, 0.0, 1.0, 0.0) == 0.0           # touching ahead
    assert O.collision_distance(0.9, 0.0, 1.0, 0.0) == 0.0           # overlap ahead -> 0
    assert O.collision_distance(0.0, 1.0, 1.0, 0.0) == math.inf      # touching beside (a = 0)
    # 3-4-5 triangle: r = (4, 0.6), d = x: s = 4 - sqrt(1 - 0.36) = 3.2
    assert abs(O.collision_distance(4.0, 0.6, 1.0, 0.0) - 3.2) < 1e-15


def test_collision_distance_vs_bisection():
    rng = np.random.default_rng(3)
    for _ in range(3000):
        r = rng.uniform(-4, 4, size=2)
        if r @ r < 1.0:
            continue
        t = rng.uniform(0, 2 * math.pi)
        d = (math.cos(t), math.sin(t))
        s1 = O.collision_distance(r[0], r[1], d[0], d[1])
        s2 = _contact_by_bisection(r[0], r[1], d[0], d[1], SIG)
        if math.isinf(s2):
            # the closed form may only disagree on numerically grazing rays
            c = abs(r[0] * d[1] - r[1] * d[0])
            assert math.isinf(s1) or c > 1.0 - 1e-9
        else:
            assert abs(s1 - s2) < 1e-9 * max(1.0, s2) + 1e-7 * (1.0 if abs(
                abs(r[0] * d[1] - r[1] * d[0]) - 1.0) < 1e-6 else 0.0)


def test_box_length_and_lattice():
    for n, eta in [(256, 0.70), (65536, 0.70), (1048576, 0.72), (16, 0.05)]:
        L = O.box_length(n, 1.0, eta)
        assert abs(n * math.pi / (4 * L * L) - eta) < 1e-14
        if n <= 65536:
            p = O.params(n, eta, 1.0, 1)
            x, y = O.lattice(p)
            k = int(round(math.sqrt(n)))
            a = L / k
            assert x.min() >= 0 and x.max() < L and y.min() >= 0 and y.max() < L
            if n <= 4096:
                dxm = x[:, None] - x[None, :]
                dym = y[:, None] - y[None, :]
                dxm -= L * np.round(dxm / L)
                dym -= L * np.round(dym / L)
                d2 = dxm ** 2 + dym ** 2
                np.fill_diagonal(d2, np.inf)
                assert abs(math.sqrt(d2.min()) - a) < 1e-12
            assert a > 1.0


# --------------------------------------------------------------------------
# Invariants of event chains
# --------------------------------------------------------------------------
def _min_pair_distance(x, y, L):
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    dx -= L * np.round(dx / L)
    dy -= L * np.round(dy / L)
    d2 = dx * dx + dy * dy
    np.fill_diagonal(d2, np.inf)
    return math.sqrt(d2.min())


def test_periodic_xy_invariants():
    """Single periodic cell, +x/+y chains: every chain moves the disks by a
    total of exactly ell along its direction, contacts are at distance sigma,
    and no two disks ever overlap."""
    # two chains per sweep (+x then +y) with 2 ell < L/2, so per-disk net
    # displacements over a sweep are unambiguous under the minimum image
    p = O.params(256, 0.60, 2.9, 1, dir_mode=O.DIR_XY, seed=11, chains_per_cell=2)
    L = O.box_length(256, 1.0, 0.60)
    assert 2 * p.ell < L / 2
    st = O.State(p)
    n_lifts = 0
    for sweep in range(40):
        xb, yb = st.x.copy(), st.y.copy()
        st2, ev = O.run_logged(p, xb, yb, sweep, 1)
        for ch in np.unique(ev["chain"]):
            e = ev[ev["chain"] == ch]
            assert abs(e["s"].sum() - p.ell) < 1e-12 * len(e) + 1e-12
            lifts = e[e["kind"] == O.EV_LIFT]
            n_lifts += len(lifts)
            if len(lifts):
                r = np.hypot((lifts["px"] - lifts["ax"] + L / 2) % L - L / 2,
                             (lifts["py"] - lifts["ay"] + L / 2) % L - L / 2)
                assert np.all(np.abs(r - 1.0) < 1e-12)
            assert e["kind"][-1] == O.EV_END
        ddx = (st2.x - xb + L / 2) % L - L / 2
        ddy = (st2.y - yb + L / 2) % L - L / 2
        assert abs(ddx.sum() - p.ell) < 1e-11
        assert abs(ddy.sum() - p.ell) < 1e-11
        assert _min_pair_distance(st2.x, st2.y, L) > 1.0 - 1e-12
        st.run(1)
        np.testing.assert_array_equal(st.x, st2.x)
        np.testing.assert_array_equal(st.y, st2.y)
    assert n_lifts > 100


def test_walled_invariants():
    """Shifted square cells: disks stay inside their cell during a sweep, every
    lift and frozen event is a contact at distance sigma, a wall event puts the
    centre on the wall, one chain per disk per sweep, no overlaps."""
    n, eta, C = 1024, 0.55, 4
    p = O.params(n, eta, 6.0, C, seed=5)
    L = O.box_length(n, 1.0, eta)
    w = L / C
    st = O.State(p)
    for sweep in range(4):
        x0, y0 = st.x.copy(), st.y.copy()
        cell_of = O.assign_cells(p, x0, y0, sweep)
        sx, sy, perm = O.sweep_draws(p, sweep)
        st2, ev = O.run_logged(p, x0, y0, sweep, 1)
        assert st2.acc_cnt[:, O.CNT_CHAINS].sum() == n
        for k in (O.EV_LIFT, O.EV_FROZEN):
            e = ev[ev["kind"] == k]
            r = np.hypot(e["px"] - e["ax"], e["py"] - e["ay"])
            assert np.all(np.abs(r - 1.0) < 1e-12), k
        ew = ev[ev["kind"] == O.EV_WALL_X]
        assert np.all(np.minimum(np.abs(ew["ax"]), np.abs(ew["ax"] - w)) < 1e-12)
        ew = ev[ev["kind"] == O.EV_WALL_Y]
        assert np.all(np.minimum(np.abs(ew["ay"]), np.abs(ew["ay"] - w)) < 1e-12)
        assert np.all(ev["ax"] > -1e-12) and np.all(ev["ax"] < w + 1e-12)
        assert np.all(ev["ay"] > -1e-12) and np.all(ev["ay"] < w + 1e-12)
        for ch in np.unique(ev["chain"]):
            e = ev[ev["chain"] == ch]
            assert abs(e["s"].sum() - p.ell) < 1e-12 * len(e) + 1e-12
        # every disk is still inside the cell it started the sweep in
        ux = (st2.x - sx) % L
        uy = (st2.y - sy) % L
        cx, cy = cell_of % C, cell_of // C
        tol = 1e-9
        inside_x = (ux >= cx * w - tol) & (ux <= (cx + 1) * w + tol) | ((cx == C - 1) & (ux < tol))
        inside_y = (uy >= cy * w - tol) & (uy <= (cy + 1) * w + tol) | ((cy == C - 1) & (uy < tol))
        assert inside_x.all() and inside_y.all()
        assert _min_pair_distance(st2.x, st2.y, L) > 1.0 - 1e-12
        st.run(1)
        np.testing.assert_array_equal(st.x, st2.x)


def test_rejection_undoes_every_chain_longer_than_the_cell():
    """Rejection variant (Sec. 3.4): a straight chain's front advances by at
    least ell along its direction, so with ell far above the cell's diagonal
    every chain reaches a wall or a frozen disk and is undone: the
    configuration and the contact sums stay exactly as they were."""
    n, eta, C = 1024, 0.30, 4
    p = O.params(n, eta, 100.0, C, seed=6, boundary=O.BOUNDARY_REJECT)
    st = O.State(p)
    x0, y0 = st.x.copy(), st.y.copy()
    st.run(2)
    np.testing.assert_array_equal(st.x, x0)
    np.testing.assert_array_equal(st.y, y0)
    cnt = st.acc_cnt.sum(axis=0)
    assert cnt[O.CNT_LIFTS] == 0 and np.all(st.acc_delta == 0.0)
    assert cnt[O.CNT_WALLS] + cnt[O.CNT_FROZEN] == cnt[O.CNT_CHAINS] == 2 * n


def test_rejection_invariants():
    """Rejection variant at a chain length that lets some chains finish:
    every chain either ends with its full displacement or is rejected at a
    wall or frozen disk and leaves its disks where they were; disks stay in
    their cells; no overlaps; the counts add up."""
    n, eta, C = 1024, 0.55, 4
    p = O.params(n, eta, 1.0, C, seed=5, boundary=O.BOUNDARY_REJECT)
    L = O.box_length(n, 1.0, eta)
    w = L / C
    st = O.State(p)
    for sweep in range(3):
        x0, y0 = st.x.copy(), st.y.copy()
        cell_of = O.assign_cells(p, x0, y0, sweep)
        sx, sy, _ = O.sweep_draws(p, sweep)
        st2, ev = O.run_logged(p, x0, y0, sweep, 1)
        cnt = st2.acc_cnt.sum(axis=0)
        accepted = rejected = 0
        for ch in np.unique(ev["chain"]):
            e = ev[ev["chain"] == ch]
            last = e["kind"][-1]
            if last == O.EV_END:
                accepted += 1
                assert abs(e["s"].sum() - p.ell) < 1e-12 * len(e) + 1e-12
                assert np.all(np.isin(e["kind"][:-1], [O.EV_LIFT]))
            else:
                rejected += 1
                assert last in (O.EV_WALL_X, O.EV_WALL_Y, O.EV_FROZEN)
                assert np.all(np.isin(e["kind"][:-1], [O.EV_LIFT]))
        assert accepted > 0 and rejected > 0
        assert accepted + rejected == cnt[O.CNT_CHAINS] == n
        assert cnt[O.CNT_WALLS] + cnt[O.CNT_FROZEN] == rejected
        assert cnt[O.CNT_LIFTS] <= (ev["kind"] == O.EV_LIFT).sum()
        ux = (st2.x - sx) % L
        uy = (st2.y - sy) % L
        cx, cy = cell_of % C, cell_of // C
        tol = 1e-9
        inside_x = (ux >= cx * w - tol) & (ux <= (cx + 1) * w + tol) | ((cx == C - 1) & (ux < tol))
        inside_y = (uy >= cy * w - tol) & (uy <= (cy + 1) * w + tol) | ((cy == C - 1) & (uy < tol))
        assert inside_x.all() and inside_y.all()
        assert _min_pair_distance(st2.x, st2.y, L) > 1.0 - 1e-12
        st.run(1)
        np.testing.assert_array_equal(st.x, st2.x)


def test_rejected_chains_leave_no_trace():
    """Rejection variant, one cell's phase replayed by hand: undoing a chain
    restores the configuration bit for bit, so removing the rejected chains'
    events from the log leaves, chain by chain, the moves of the accepted
    ones; in particular a disk whose every chain was rejected keeps its bits."""
    n, eta, C = 1024, 0.55, 4
    p = O.params(n, eta, 1.5, C, seed=9, boundary=O.BOUNDARY_REJECT)
    st = O.State(p)
    x0, y0 = st.x.copy(), st.y.copy()
    st2, ev = O.run_logged(p, x0, y0, 0, 1)
    moved_by_accepted = set()
    for ch in np.unique(ev["chain"]):
        e = ev[ev["chain"] == ch]
        if e["kind"][-1] == O.EV_END:
            moved_by_accepted.update(int(a) for a in e["active"])
    untouched = np.setdiff1d(np.arange(n), np.array(sorted(moved_by_accepted), dtype=np.int64))
    np.testing.assert_array_equal(st2.x[untouched], x0[untouched])
    np.testing.assert_array_equal(st2.y[untouched], y0[untouched])


def test_frozen_reflection_is_specular():
    """After a contact with a frozen disk the direction is mirrored about the
    contact normal: angle of incidence equals angle of reflection."""
    n, eta, C = 1024, 0.62, 4
    p = O.params(n, eta, 8.0, C, seed=9)
    st, ev = O.run_logged(p, None, None, 0, 2)
    count = 0
    for i in np.nonzero(ev["kind"] == O.EV_FROZEN)[0]:
        if i + 1 >= len(ev) or ev["chain"][i + 1] != ev["chain"][i]:
            continue
        e, nxt = ev[i], ev[i + 1]
        nvec = np.array([e["px"] - e["ax"], e["py"] - e["ay"]])
        nvec /= np.linalg.norm(nvec)
        d = np.array([e["dx"], e["dy"]])
        d2 = np.array([nxt["dx"], nxt["dy"]])
        assert abs(np.linalg.norm(d2) - 1.0) < 1e-14
        # tangential component kept, normal component reversed
        t = np.array([-nvec[1], nvec[0]])
        assert abs(d2 @ t - d @ t) < 1e-12
        assert abs(d2 @ nvec + d @ nvec) < 1e-12
        assert d @ nvec > 0  # it was moving towards the frozen disk
        count += 1
    assert count > 20


def test_single_disk_folds_at_walls():
    """One disk alone in a walled cell: after a chain its local position is
    the straight-line end point folded back at the walls."""
    L = 40.0
    eta = math.pi / (4.0 * L * L)
    p = O.params(1, eta, 37.3, 4, seed=21)
    assert abs(O.box_length(1, 1.0, eta) - L) < 1e-12
    w = O.box_length(1, 1.0, eta) / 4
    L = O.box_length(1, 1.0, eta)
    st = O.State(p, np.array([13.7]), np.array([27.1]))

    def fold(t):
        u = t % (2 * w)
        return u if u <= w else 2 * w - u

    for sweep in range(20):
        x0, y0 = st.x[0], st.y[0]
        cell = int(O.assign_cells(p, st.x, st.y, sweep)[0])
        sx, sy, _ = O.sweep_draws(p, sweep)
        cx, cy = cell % 4, cell // 4
        vx = (x0 - sx) % L - cx * w
        vy = (y0 - sy) % L - cy * w
        dx, dy = O.direction(p, sweep, cell, 0)
        ex, ey = fold(vx + p.ell * dx), fold(vy + p.ell * dy)
        st.run(1)
        gx = (st.x[0] - sx) % L - cx * w
        gy = (st.y[0] - sy) % L - cy * w
        assert abs(gx - ex) < 1e-11 and abs(gy - ey) < 1e-11


def test_resume_is_bit_exact():
    p = O.params(1024, 0.65, 5.0, 4, seed=3)
    a = O.State(p)
    a.run(6)
    b = O.State(p)
    b.run(2)
    b.run(4)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.acc_delta, b.acc_delta)
    assert a.digests == b.digests


def test_run_cells_reproduces_first_phase():
    """First-phase cells only see positions from the start of the sweep, so the
    single-cell entry reproduces them exactly."""
    p = O.params(4096, 0.70, 10.0, 8, seed=2)
    full = O.State(p)
    full.run(1)
    _, _, perm = O.sweep_draws(p, 0)
    C = 8
    first = [c for c in range(C * C) if ((c % C) & 1) | (((c // C) & 1) << 1) == perm[0]]
    part = O.State(p)
    part.run_cells(0, first[:5], n_phases=1)
    cell_of = O.assign_cells(p, *O.lattice(p), 0)
    mask = np.isin(cell_of, first[:5])
    np.testing.assert_array_equal(part.x[mask], full.x[mask])
    np.testing.assert_array_equal(part.y[mask], full.y[mask])
    for c in first[:5]:
        assert part.acc_delta[c] == full.acc_delta[c]


# --------------------------------------------------------------------------
# Statistical pins: exact small systems and the virial series
# --------------------------------------------------------------------------
def _batch_mean_err(vals, nb=20):
    vals = np.asarray(vals)
    m = len(vals) // nb
    b = vals[: m * nb].reshape(nb, m).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nb)


def _two_disk_cdf(r, L, s=1.0):
    """CDF of the separation of two disks uniform on an L x L torus, excluded
    core of radius s, for s <= r <= L/sqrt(2)."""
    def area(r):
        if r <= L / 2:
            return math.pi * r * r
        h = L / 2
        return math.pi * r * r - 4 * (r * r * math.acos(h / r) - h * math.sqrt(r * r - h * h))
    return (area(r) - math.pi * s * s) / (L * L - math.pi * s * s)


def test_two_disks_periodic_exact():
    """Two disks in a periodic L x L box, L = 4 sigma: the separation is
    uniform over the torus minus the excluded disk and the EC pressure is
    Z = 1 + pi sigma^2 / (2 (L^2 - pi sigma^2))."""
    L = 4.0
    eta = 2 * math.pi / (4 * L * L)
    p = O.params(2, eta, 3.0, 1, dir_mode=O.DIR_ISO, seed=17)
    st = O.State(p, np.array([0.5, 2.5]), np.array([0.5, 0.5]))
    seps = []
    zs = []
    prev_delta, prev_chains = 0.0, 0
    for _ in range(400):
        st.run(500)
        d = np.array([st.x[1] - st.x[0], st.y[1] - st.y[0]])
        d -= L * np.round(d / L)
        seps.append(float(np.hypot(*d)))
        s, cnt = st.tallies()
        zs.append((s - prev_delta) / ((cnt[O.CNT_CHAINS] - prev_chains) * p.ell))
        prev_delta, prev_chains = s, cnt[O.CNT_CHAINS]
    z_exact = 1.0 + math.pi / (2 * (L * L - math.pi))
    m, e = _batch_mean_err(zs)
    assert abs(1.0 + m - z_exact) < 4 * e + 1e-3, (1 + m, z_exact, e)
    assert e < 0.01
    assert st.acc_cnt[0, O.CNT_PSEUDO] > 0
    # KS test of the separation distribution
    seps = np.sort(seps)
    F = np.array([_two_disk_cdf(r, L) for r in seps])
    emp = np.arange(1, len(seps) + 1) / len(seps)
    ks = max(np.abs(F - emp).max(), np.abs(F - (emp - 1.0 / len(seps))).max())
    assert ks < 1.63 / math.sqrt(len(seps)) * 1.2  # ~1% level


def test_tonks_gas_pressure():
    """Hard rods on a ring (disks on one row, +x chains only).  For N rods of
    length sigma on a ring of length L the free gaps are uniform on the
    simplex, each gap is (L - N sigma) Beta(1, N-1), and the contact density
    gives Z = 1 + (N-1) sigma / (L - N sigma) (-> 1/(1 - N sigma/L) for large N).
    The start has random gaps: from equal gaps and an integer ell the +x
    dynamics would stay on a lattice of gap values."""
    n = 16
    L = 32.0
    eta = n * math.pi / (4 * L * L)
    p = O.params(n, eta, 10.0, 1, dir_mode=O.DIR_X, seed=23)
    x, y = inputs.rods_on_a_ring(n, L, seed=5)
    st = O.State(p, x, y)
    st.run(200)
    st.acc_delta[:] = 0
    st.acc_cnt[:] = 0
    zs = []
    prev = (0.0, 0)
    gaps = []
    for _ in range(400):
        st.run(25)
        s, cnt = st.tallies()
        zs.append((s - prev[0]) / ((cnt[O.CNT_CHAINS] - prev[1]) * p.ell))
        prev = (s, cnt[O.CNT_CHAINS])
        ahead = (st.x - st.x[0]) % L  # gap in front of rod 0
        ahead[0] = np.inf
        gaps.append(ahead.min() - 1.0)
    assert np.all(st.y == y[0])
    m, e = _batch_mean_err(zs)
    z_exact = 1.0 + (n - 1) / (L - n)
    assert abs(1.0 + m - z_exact) < 4 * e + 1e-3, (1 + m, z_exact, e)
    # KS test of the gap in front of one rod against (L - N sigma) Beta(1, N-1)
    gaps = np.sort(np.array(gaps))
    F = 1.0 - (1.0 - gaps / (L - n)) ** (n - 1)
    emp = np.arange(1, len(gaps) + 1) / len(gaps)
    ks = max(np.abs(F - emp).max(), np.abs(F - (emp - 1.0 / len(gaps))).max())
    assert ks < 1.63 / math.sqrt(len(gaps))


@pytest.mark.parametrize("cells", [1, 4])
def test_low_density_virial_series(cells):
    """At eta = 0.08 the EC pressure matches the hard-disk virial series
    Z = 1 + 2 eta + 3.12802 eta^2 + 4.25785 eta^3 + 5.3369 eta^4 (the
    coefficients are B3/B2^2 = 4/3 - sqrt(3)/pi and
    B4/B2^3 = 2 - 9 sqrt(3)/(2 pi) + 10/pi^2 in units of 2 eta), both in one
    periodic cell and with walled cells and frozen neighbours."""
    eta = 0.08
    n, per = (256, 20) if cells == 1 else (1024, 10)
    b3 = 4.0 * (4.0 / 3.0 - math.sqrt(3.0) / math.pi)
    b4 = 8.0 * (2.0 - 9.0 * math.sqrt(3.0) / (2.0 * math.pi) + 10.0 / math.pi ** 2)
    z_series = 1 + 2 * eta + b3 * eta ** 2 + b4 * eta ** 3 + 5.3369 * eta ** 4
    z_series -= 2 * eta / n  # finite-N second virial correction
    p = O.params(n, eta, 30.0, cells, dir_mode=O.DIR_ISO, seed=31)
    st = O.State(p)
    st.run(20)  # melt the lattice
    st.acc_delta[:] = 0
    st.acc_cnt[:] = 0
    zs = []
    prev = (0.0, 0)
    for _ in range(40):
        st.run(per)
        s, cnt = st.tallies()
        zs.append(1.0 + (s - prev[0]) / ((cnt[O.CNT_CHAINS] - prev[1]) * p.ell))
        prev = (s, cnt[O.CNT_CHAINS])
    m, e = _batch_mean_err(zs)
    # the eta^5 term (~2e-5) and O(eta^2/N) corrections are below the tolerance
    assert abs(m - z_series) < 4 * e + 3e-4, (m, z_series, e)
    assert e < 3e-4
    if cells > 1:
        assert st.acc_cnt[:, O.CNT_FROZEN].sum() > 0.02 * st.acc_cnt[:, O.CNT_LIFTS].sum()


# ---------------------------------------------------------------------------
# Hexatic order parameter (Sec. 2, eq. Psi) with cutoff neighbours
# ---------------------------------------------------------------------------
def test_psi6_start_lattice_closed_form():
    """Centred-rectangular start lattice (spacing a, odd rows shifted a/2):
    every disk has 2 neighbours at 0 and 180 degrees and 4 at +-atan2(1, 1/2)
    (+180), all within 1.4 sigma, so Psi_k = (2 + 4 cos(6 atan2(1, 1/2))) / 6."""
    p = O.params(4096, 0.72, 20.0, 8)
    x, y = O.lattice(p)
    psi, nb, per = O.psi6(p, x, y, 1.4)
    want = (2.0 + 4.0 * math.cos(6.0 * math.atan2(1.0, 0.5))) / 6.0
    assert nb == 6.0
    assert abs(psi - want) < 1e-12
    assert np.max(np.abs(per - want)) < 1e-12


@pytest.mark.parametrize("theta", [0.0, 0.1, 0.37, -0.8])
def test_psi6_rotated_triangular_patch(theta):
    """Interior disks of a triangular patch rotated by theta: Psi_k = exp(6 i theta)."""
    a = 1.1
    pts = []
    for j in range(-4, 5):
        for i in range(-4, 5):
            px, py = (i + 0.5 * j) * a, j * a * math.sqrt(3.0) / 2.0
            pts.append((px * math.cos(theta) - py * math.sin(theta) + 50.0,
                        px * math.sin(theta) + py * math.cos(theta) + 50.0))
    pts = np.array(pts)
    _, _, per = O.psi6_box(len(pts), 100.0, pts[:, 0], pts[:, 1], 1.4)
    centre = 4 * 9 + 4
    assert abs(per[centre] - complex(math.cos(6 * theta), math.sin(6 * theta))) < 1e-12
    inner = [j * 9 + i for j in range(2, 7) for i in range(2, 7)]
    assert np.max(np.abs(per[inner] - complex(math.cos(6 * theta), math.sin(6 * theta)))) < 1e-12


def test_psi6_pair_isolated_disk_and_periodic_image():
    """A pair at angle alpha: both disks have Psi_k = exp(6 i alpha) (the bond
    reversed adds 6 pi); a lone disk has Psi_k = 0; a pair across the periodic
    boundary is found through the minimum image."""
    alpha = 0.3
    L = 20.0
    x = np.array([5.0, 5.0 + 1.2 * math.cos(alpha), 15.0])
    y = np.array([5.0, 5.0 + 1.2 * math.sin(alpha), 15.0])
    psi, nb, per = O.psi6_box(3, L, x, y, 1.4)
    e = complex(math.cos(6 * alpha), math.sin(6 * alpha))
    assert abs(per[0] - e) < 1e-14 and abs(per[1] - e) < 1e-14 and per[2] == 0
    assert abs(psi - 2 * e / 3) < 1e-14 and abs(nb - 2 / 3) < 1e-14
    x2 = np.array([0.3, L - 0.5])
    y2 = np.array([7.0, 7.0])
    _, nb2, per2 = O.psi6_box(2, L, x2, y2, 1.4)
    assert nb2 == 1.0 and abs(per2[0] - 1.0) < 1e-14 and abs(per2[1] - 1.0) < 1e-14


# ---------------------------------------------------------------------------
# Pair histogram of the pressure route (eq. pressure)
# ---------------------------------------------------------------------------
def test_pair_histogram_start_lattice():
    """Start lattice: every disk has 2 neighbours at distance a and 4 at
    a sqrt(5)/2 inside 1.5 sigma, so the ordered-pair counts are 2N and 4N in
    the bins holding those distances and 0 elsewhere."""
    p = O.params(4096, 0.72, 20.0, 8)
    x, y = O.lattice(p)
    a = O.box_length(4096, 1.0, 0.72) / 64
    counts, ov = O.pair_histogram(p, x, y, 1.5, 100)
    d = 0.5 / 100
    want = np.zeros(100, dtype=np.uint64)
    want[int((a - 1.0) // d)] += 2 * 4096
    want[int((a * math.sqrt(1.25) - 1.0) // d)] += 4 * 4096
    np.testing.assert_array_equal(counts, want)
    assert ov == 0


def test_pair_histogram_single_pair_and_overlap():
    p = O.params(4, 0.01, 20.0, 1)  # box of side ~17.7
    L = O.box_length(4, 1.0, 0.01)
    x = np.array([1.0, 2.2345, 9.0, 9.5])  # a pair at 1.2345: well inside bin 23
    y = np.array([1.0, 1.0, 9.0, 9.0])
    counts, ov = O.pair_histogram(p, x, y, 1.5, 50)
    assert counts.sum() == 2 and counts[23] == 2
    assert ov == 2  # the pair at distance 0.5, both orders
    assert L > 10


# ---- Delaunay Psi and its autocorrelation time (eq. Psi, eq. tau) --------------------------


def _periodic_empty_circle_neighbours(x, y, L):
    """Periodic Delaunay neighbours by definition: triangles of the 3 x 3 image
    set with an empty circumcircle and at least one vertex in the box."""
    from oracle import delaunay as D
    n = len(x)
    px = np.concatenate([x + sx * L for sx in (-1, 0, 1) for sy in (-1, 0, 1)])
    py = np.concatenate([y + sy * L for sx in (-1, 0, 1) for sy in (-1, 0, 1)])
    base = 4 * n  # (sx, sy) = (0, 0) comes fifth
    p = np.stack([px, py], axis=1)
    m = len(p)
    nbrs = [set() for _ in range(n)]
    for i in range(base, base + n):
        for j in range(m):
            if j == i:
                continue
            for k in range(j + 1, m):
                if k == i:
                    continue
                a, b, c = p[i], p[j], p[k]
                d = 2.0 * (a[0] * (b[1] - c[1]) + b[0] * (c[1] - a[1]) + c[0] * (a[1] - b[1]))
                if abs(d) < 1e-12:
                    continue
                ux = ((a @ a) * (b[1] - c[1]) + (b @ b) * (c[1] - a[1]) + (c @ c) * (a[1] - b[1])) / d
                uy = ((a @ a) * (c[0] - b[0]) + (b @ b) * (a[0] - c[0]) + (c @ c) * (b[0] - a[0])) / d
                r2 = (a[0] - ux) ** 2 + (a[1] - uy) ** 2
                if r2 > (0.5 * L) ** 2:
                    continue  # a circle wider than the box is no triangle of the torus
                dist2 = (p[:, 0] - ux) ** 2 + (p[:, 1] - uy) ** 2
                dist2[[i, j, k]] = np.inf
                if np.all(dist2 > r2):
                    for q in (j, k):
                        v = p[q] - p[i]
                        nbrs[i - base].add((q % n, round(v[0], 9), round(v[1], 9)))
    return nbrs


def test_delaunay_library_step_matches_empty_circles():
    """scipy's triangulation against the definition, plane and torus."""
    from oracle import delaunay as D
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(11)
    pts = rng.random((30, 2)) * 10.0
    tri = Delaunay(pts)
    lib = set()
    for s in tri.simplices:
        for a in range(3):
            for b in range(a + 1, 3):
                lib.add(tuple(sorted((int(s[a]), int(s[b])))))
    assert lib == D.empty_circle_edges(pts[:, 0], pts[:, 1])
    # periodic: 12 disks in a 6 x 6 box
    L = 6.0
    q = rng.random((12, 2)) * L
    offsets, ids = D.delaunay_neighbours(q[:, 0], q[:, 1], L, L, margin=L)
    got = [{(int(i), round(v[0], 9), round(v[1], 9)) for i, v in zip(idk, off)}
           for idk, off in zip(ids, offsets)]
    assert got == _periodic_empty_circle_neighbours(q[:, 0], q[:, 1], L)


def test_delaunay_psi6_triangular_lattice():
    """A periodic triangular lattice: six neighbours each, Psi_k = 1."""
    from oracle import delaunay as D
    nx, ny, a = 12, 14, 1.1
    h = a * math.sqrt(3.0) / 2.0
    x = np.array([(i + 0.5 * (j & 1)) * a for j in range(ny) for i in range(nx)])
    y = np.array([j * h for j in range(ny) for i in range(nx)])
    psi, per, counts = D.psi6_delaunay(x, y, nx * a, ny * h)
    assert np.all(counts == 6)
    np.testing.assert_allclose(per, 1.0, atol=1e-12)
    assert abs(psi - 1.0) < 1e-12


def test_delaunay_psi6_start_lattice_closed_form():
    """The system's start lattice (rows offset by a/2) has a unique
    triangulation: neighbours at (+-a, 0) and (+-a/2, +-a), so every
    Psi_k = (2 + 4 cos(6 atan2(1, 1/2))) / 6, as with the cutoff neighbours."""
    from oracle import delaunay as D
    p = O.params(1024, 0.70, 20.0, 4)
    x, y = O.lattice(p)
    L = O.box_length(1024, 1.0, 0.70)
    psi, per, counts = D.psi6_delaunay(x, y, L, L)
    want = (2.0 + 4.0 * math.cos(6.0 * math.atan2(1.0, 0.5))) / 6.0
    assert np.all(counts == 6)
    np.testing.assert_allclose(per.real, want, atol=1e-12)
    np.testing.assert_allclose(per.imag, 0.0, atol=1e-12)


def test_delaunay_mean_degree_is_six_on_the_torus():
    """Euler's relation on the torus (V - E + F = 0, 3F = 2E): mean degree 6."""
    from oracle import delaunay as D
    rng = np.random.default_rng(5)
    for n, L in ((200, 14.0), (500, 22.0)):
        q = rng.random((n, 2)) * L
        _, _, counts = D.psi6_delaunay(q[:, 0], q[:, 1], L, L)
        assert int(counts.sum()) == 6 * n


def test_autocorrelation_closed_forms():
    """Psi(t) = exp(i w t): C(dt) = cos(w dt); an exactly exponential C
    returns its tau; an AR(1) series Psi(t+1) = a Psi(t) + noise has
    C(dt) = a^dt, tau = -1 / ln a."""
    from oracle import delaunay as D
    w = 0.3
    t = np.arange(400)
    c = D.autocorrelation(np.exp(1j * w * t), 20)
    np.testing.assert_allclose(c, np.cos(w * np.arange(21)), atol=1e-12)
    assert abs(D.tau_fit(np.exp(-np.arange(30) / 4.5)) - 4.5) < 1e-12
    rng = np.random.default_rng(3)
    a, n = 0.9, 200000
    noise = rng.normal(size=n) + 1j * rng.normal(size=n)
    psi = np.empty(n, dtype=np.complex128)
    psi[0] = noise[0]
    for i in range(1, n):
        psi[i] = a * psi[i - 1] + noise[i]
    tau = D.tau_fit(D.autocorrelation(psi, 40))
    assert abs(tau - (-1.0 / math.log(a))) / (-1.0 / math.log(a)) < 0.05


def test_delaunay_planar_patch_equals_periodic():
    """Neighbours of sampled disks from a planar patch equal those of the
    periodic triangulation."""
    from oracle import delaunay as D
    rng = np.random.default_rng(8)
    L, n = 30.0, 700
    q = rng.random((n, 2)) * L
    offsets, _ = D.delaunay_neighbours(q[:, 0], q[:, 1], L, L)
    for k in (0, 17, 333):
        dx = q[:, 0] - q[k, 0]
        dy = q[:, 1] - q[k, 1]
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        sel = np.nonzero(dx * dx + dy * dy < 8.0 ** 2)[0]
        centre = int(np.nonzero(sel == k)[0][0])
        got = D.planar_neighbours(dx[sel], dy[sel], centre)
        a = sorted(map(tuple, np.round(got, 9)))
        b = sorted(map(tuple, np.round(offsets[k], 9)))
        assert a == b


def test_mean_free_path_at_eta_071_matches_the_paper():
    """The paper prints the mean free path at eta = 0.71 (tests/golden/
    mean_free_path.json).  Measured as ell / (disk contacts per chain) over
    sweeps 3-4 of a 4096-disk system (4 x 4 cells, ell = 20 sigma) from the
    lattice: within the printed precision."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mean_free_path.json")))
    p = O.params(4096, gold["eta"], 20.0, 4, seed=2)
    st = O.State(p)
    st.run(2)
    c0 = st.acc_cnt.sum(axis=0).astype(float)
    st.run(2)
    d = st.acc_cnt.sum(axis=0).astype(float) - c0
    lam = p.ell * d[O.CNT_CHAINS] / (d[O.CNT_LIFTS] + d[O.CNT_FROZEN])
    assert abs(lam - gold["lambda0_over_sigma"]) <= 0.005, lam


# --------------------------------------------------------------------------
# Phase-parallel oracle mode (same bits as the serial run)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,eta,cells,ell,sweeps,kw", [
    (4096, 0.72, 8, 20.0, 2, {}),
    (2304, 0.65, 6, 12.0, 2, {}),
    (1024, 0.60, 4, 5.0, 3, dict(chains_per_cell=50, start_mode=O.START_DISTINCT)),
    (1024, 0.55, 4, 1.0, 3, dict(boundary=O.BOUNDARY_REJECT)),
])
def test_phase_parallel_equals_serial(n, eta, cells, ell, sweeps, kw):
    """Cells of one colour share nothing (Sec. 3.4, step 4), so running them on
    several threads must give every bit of the serial run."""
    p = O.params(n, eta, ell, cells, **kw)
    out = []
    for threads in (1, 4):
        O.set_threads(threads)
        try:
            st = O.State(p)
            st.run(sweeps)
        finally:
            O.set_threads(1)
        out.append(st)
    a, b = out
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.acc_delta, b.acc_delta)
    np.testing.assert_array_equal(a.acc_cnt, b.acc_cnt)
    assert a.digests == b.digests


# --------------------------------------------------------------------------
# Start lists: index mapping and the distinct-start shuffle
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bits", [1, 3, 8, 20])
def test_start_index_power_of_two_is_top_bits(bits):
    """For n = 2^b the multiply-shift index map never rejects and returns the
    top b bits of the first Philox word of the stream (key (seed, 2),
    counter (sweep, cell, chain, 0)), taken from numpy's generator."""
    p = O.params(4096, 0.7, 1.0, 8, seed=9)
    n = 1 << bits
    for sweep, cell, chain in [(0, 0, 0), (3, 5, 7), (11, 63, 1000), (2, 17, 99)]:
        word = _numpy_philox_block([sweep, cell, chain, 0], [9, 2])[0]
        assert O.start_index(p, sweep, cell, chain, n) == word >> (64 - bits)


def test_distinct_start_shuffle_uniform_over_permutations():
    """The distinct-start control (Fig. 2-3) uses a shuffled list of the cell's
    disks: for a cell of 4 disks every one of the 24 orders must be equally
    likely (an off-by-one shuffle reaches only some of them, or not evenly)."""
    import itertools
    p = O.params(4096, 0.7, 1.0, 8, start_mode=O.START_DISTINCT, seed=5)
    perms = {q: i for i, q in enumerate(itertools.permutations(range(4)))}
    counts = np.zeros(24)
    draws = 24 * 500
    for s in range(draws):
        lst = tuple(int(v) for v in O.start_list(p, s, 3, 4, 4))
        counts[perms[lst]] += 1  # KeyError if not a permutation of 0..3
    e = draws / 24
    chi2 = ((counts - e) ** 2 / e).sum()
    assert counts.min() > 0
    assert chi2 < 55.0  # 23 dof, P ~ 2e-4
    # with n_m > n_c the list repeats: chain k starts at list[k mod n_c]
    lst = O.start_list(p, 7, 3, 4, 10)
    np.testing.assert_array_equal(lst[4:8], lst[:4])
    np.testing.assert_array_equal(lst[8:], lst[:2])


def test_replacement_start_list_uses_independent_draws():
    """With replacement (Fig. 2) chain k's start is the index draw of stream k."""
    p = O.params(4096, 0.7, 1.0, 8, seed=5)
    lst = O.start_list(p, 2, 9, 37, 50)
    assert [int(v) for v in lst] == [O.start_index(p, 2, 9, k, 37) for k in range(50)]


# --------------------------------------------------------------------------
# Exact stationary laws of one walled cell (Sec. 3.4, Fig. 1 right)
# --------------------------------------------------------------------------
def _bin_mass(w, nb, weight, res=1500):
    """Integral of weight(X, Y) over each of nb x nb bins of [0, w]^2 (midpoint
    rule on res x res points per bin), normalised to total 1."""
    h = w / nb
    t = (np.arange(res) + 0.5) / res * h
    P = np.zeros((nb, nb))
    for i in range(nb):
        for j in range(nb):
            X, Y = np.meshgrid(i * h + t, j * h + t, indexing="ij")
            P[i, j] = weight(X, Y).mean()
    return P / P.sum()


def _batch_z(samples, hist, P, batches=50):
    """z-scores of the bin frequencies against P, with batch-means errors (the
    chain samples are correlated); bins with P = 0 must stay empty."""
    m = len(samples) // batches
    f = np.array([hist(samples[b * m:(b + 1) * m]) for b in range(batches)])
    mean = f.mean(0)
    se = f.std(0, ddof=1) / math.sqrt(batches)
    assert np.all(mean[P == 0] == 0)
    k = P > 0
    return (mean[k] - P[k]) / se[k]


def test_one_disk_beside_a_frozen_disk_is_uniform():
    """One movable disk in a walled cell [0, 3]^2 next to one frozen disk (in
    the band left of the cell): chains reflect at the walls and, with equal
    angles, at the frozen disk.  The stationary law is uniform over the cell
    minus the disk of radius sigma around the frozen centre (the billiard flow
    keeps the uniform measure; each chain restarts with a uniform direction)."""
    w, nb, F = 3.0, 6, (-0.4, 1.3)
    p = O.params(1, 0.5, 7.0, 4, seed=11)
    _, _, tr, _, cnt = O.cell_chains(p, w, [2.0], [1.5], [F[0]], [F[1]], n_chains=200000)
    assert cnt[O.CNT_FROZEN] > 50000 and cnt[O.CNT_WALLS] > 200000
    assert np.all((tr[:, 0, 0] - F[0]) ** 2 + (tr[:, 0, 1] - F[1]) ** 2 >= 1.0 - 1e-12)
    P = _bin_mass(w, nb, lambda X, Y: ((X - F[0]) ** 2 + (Y - F[1]) ** 2 >= 1.0).astype(float))

    def hist(s):
        H, _, _ = np.histogram2d(s[:, 0, 0], s[:, 0, 1], bins=nb, range=[[0, w], [0, w]])
        return H / len(s)

    z = _batch_z(tr, hist, P)
    # about 33 bins; batch-means z are t-distributed with 49 dof
    assert np.abs(z).max() < 4.5
    assert (z ** 2).sum() < len(z) + 5.0 * math.sqrt(2 * len(z)) + 10.0


def test_two_disks_in_a_walled_cell_separation_law():
    """Two movable disks in a walled cell [0, 3]^2 with lifts between them and
    reflections at the walls: the stationary law is uniform over the allowed
    pairs, so the separation r = r1 - r2 has density proportional to
    (w - |r_x|)(w - |r_y|) on |r| >= sigma."""
    w, nb = 3.0, 6
    p = O.params(2, 0.5, 7.0, 4, seed=12)
    _, _, tr, _, cnt = O.cell_chains(p, w, [0.7, 2.2], [0.7, 2.2], n_chains=200000)
    assert cnt[O.CNT_LIFTS] > 100000 and cnt[O.CNT_WALLS] > 200000
    P = _bin_mass(w, nb, lambda X, Y: (w - X) * (w - Y) * (X * X + Y * Y >= 1.0))

    def hist(s):
        r = np.abs(s[:, 0, :] - s[:, 1, :])
        H, _, _ = np.histogram2d(r[:, 0], r[:, 1], bins=nb, range=[[0, w], [0, w]])
        return H / len(s)

    z = _batch_z(tr, hist, P)
    assert np.abs(z).max() < 4.5
    assert (z ** 2).sum() < len(z) + 5.0 * math.sqrt(2 * len(z)) + 10.0


# --------------------------------------------------------------------------
# Overlap check used on the full-size workloads
# --------------------------------------------------------------------------
def test_min_pair_distance_against_brute_force():
    rng = np.random.default_rng(3)
    for n, L, rc in [(300, 20.0, 1.0), (50, 5.0, 1.0), (400, 30.0, 2.5), (2, 4.0, 1.9)]:
        x = rng.uniform(0, L, n)
        y = rng.uniform(0, L, n)
        dx = x[None, :] - x[:, None]
        dy = y[None, :] - y[:, None]
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        d = np.sqrt(dx * dx + dy * dy)
        d[np.arange(n), np.arange(n)] = np.inf
        ref = d.min()
        got, i, j = O.min_pair_distance(x, y, L, rc)
        if ref < rc:
            assert abs(got - ref) <= 1e-12 * L and abs(d[i, j] - ref) <= 1e-12 * L
        else:
            assert got == math.inf and i == -1 and j == -1


# --------------------------------------------------------------------------
# Dependency cones: a cell of a later phase replayed from the sweep start
# --------------------------------------------------------------------------
def test_dependency_cone_replays_later_phases():
    """A cell of colour phase q reads the disks its earlier-phase neighbours
    have moved (Sec. 3.4, steps 4-6).  Running only the cells of its cone of
    earlier-phase neighbours (recursively) from the sweep start must give the
    cell exactly what the full sweep gives it."""
    p = O.params(4096, 0.70, 10.0, 8, seed=4)
    full = O.State(p)
    full.run(2)
    x0, y0 = O.lattice(p)
    one = O.State(p)
    one.run(1)
    for sweep, (sx, sy) in ((0, (x0, y0)), (1, (one.x, one.y))):
        for target in (9, 18, 27, 36, 45, 54):
            cells = cones.dependency_cone(p.cells, O.sweep_draws(p, sweep)[2], target)
            st = O.State(p, sx, sy)
            if sweep == 1:
                st.acc_delta[:] = one.acc_delta
                st.acc_cnt[:] = one.acc_cnt
            dig = st.run_cells(sweep, sorted(cells), n_phases=4)
            ref = full if sweep == 1 else one
            cell_of = O.assign_cells(p, sx, sy, sweep)
            mask = np.isin(cell_of, sorted(cells))
            np.testing.assert_array_equal(st.x[mask], ref.x[mask])
            np.testing.assert_array_equal(st.y[mask], ref.y[mask])
            for c in cells:
                assert st.acc_delta[c] == ref.acc_delta[c]
                np.testing.assert_array_equal(st.acc_cnt[c], ref.acc_cnt[c])
            assert len(dig) == len(cells)


# --------------------------------------------------------------------------
# Striped decomposition with rejection (Sec. 3.4, the stripes variant of Fig. 3; Sec. 4)
# --------------------------------------------------------------------------
def _image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("n,eta,stripes,ell,kw", [
    (4096, 0.70, 8, 0.3, {}),
    (1024, 0.30, 4, 3.0, {}),
    (64, 0.10, 4, 30.0, {}),   # flights beyond the nearest-image range: pseudo events
    (1024, 0.60, 4, 0.5, dict(chains_per_cell=50, start_mode=O.START_DISTINCT)),
])
def test_stripes_invariants(n, eta, stripes, ell, kw):
    """Chains run along the stripes: on even sweeps every y keeps its bits and
    the x displacements of all disks add up to ell times a sum of signs, one
    +-1 per accepted chain (odd sweeps: the same with x and y exchanged), so
    the total over ell is an integer of the parity of the accepted count;
    rejected chains leave no trace; no two disks overlap."""
    p = O.params(n, eta, ell, stripes, dir_mode=O.DIR_XY, boundary=O.BOUNDARY_STRIPES, seed=3, **kw)
    L = O.box_length(n, 1.0, eta)
    st = O.State(p)
    for sweep in range(4):
        x0, y0 = st.x.copy(), st.y.copy()
        cnt0 = st.acc_cnt.sum(axis=0).copy()
        st.run(1)
        cnt = st.acc_cnt.sum(axis=0) - cnt0
        along0, along1, across0, across1 = ((x0, st.x, y0, st.y) if sweep % 2 == 0
                                            else (y0, st.y, x0, st.x))
        np.testing.assert_array_equal(across1, across0)
        accepted = int(cnt[O.CNT_CHAINS]) - int(cnt[O.CNT_FROZEN])
        assert cnt[O.CNT_WALLS] == 0
        assert int(cnt[O.CNT_CHAINS]) == (n if not kw else 50 * stripes)
        if 4 * ell < L / 2:  # a disk's net move stays below L/2, so nearest images add up
            m = _image(along1 - along0, L).sum() / ell
            assert abs(m - round(m)) < 1e-9 * max(1.0, accepted)
            assert abs(round(m)) <= accepted and (round(m) - accepted) % 2 == 0
        d, _, _ = O.min_pair_distance(st.x, st.y, L, r_cut=1.0 - 1e-12)
        assert d == math.inf
    if eta == 0.10:
        assert st.acc_cnt[:, O.CNT_PSEUDO].sum() > 0


def test_stripes_two_disks_periodic_exact():
    """Two disks in a periodic L x L box swept by the striped decomposition
    (4 stripes, rejection at the stripe boundaries, starts with replacement):
    the stationary law makes the separation uniform on the torus minus the
    disk of radius sigma, so P(|r| < R) = pi (R^2 - sigma^2) / (L^2 - pi sigma^2)
    for R <= L/2."""
    L = 8.8
    eta = 2 * math.pi / (4 * L * L)
    p = O.params(2, eta, 1.5, 4, dir_mode=O.DIR_XY, boundary=O.BOUNDARY_STRIPES, seed=8)
    st = O.State(p, np.array([1.0, 5.0]), np.array([1.0, 3.0]))
    sweeps = 40000
    rs = np.empty(sweeps)
    for t in range(sweeps // 1000):
        for k in range(1000):
            st.run(1)
            rs[t * 1000 + k] = math.hypot(_image(st.x[1] - st.x[0], L), _image(st.y[1] - st.y[0], L))
    assert rs.min() >= 1.0 - 1e-12
    edges = np.array([1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 4.4])
    exact = np.diff(math.pi * (edges ** 2 - 1.0) / (L * L - math.pi))
    B = 40
    m = sweeps // B
    f = np.array([np.histogram(rs[b * m:(b + 1) * m], bins=edges)[0] / m for b in range(B)])
    z = (f.mean(0) - exact) / (f.std(0, ddof=1) / math.sqrt(B))
    assert np.abs(z).max() < 4.5, z


def test_start_lattice_nearest_neighbours_and_refusal():
    """The start lattice (k x k sites, spacing a = L/k, odd rows shifted by
    a/2) has its nearest neighbours exactly a apart: brute force over all
    pairs with the minimum image, in numpy.  a = sigma sqrt(pi / (4 eta))
    falls below sigma above eta = pi/4, and the oracle then refuses the start
    (the library refuses it too), since the disks would overlap."""
    n = 256
    for eta in (0.50, 0.78):
        p = O.params(n, eta, 1.0, 4)
        x, y = O.lattice(p)
        L = O.box_length(n, 1.0, eta)
        dx = x[:, None] - x[None, :]
        dy = y[:, None] - y[None, :]
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        r = np.sqrt(dx * dx + dy * dy)
        np.fill_diagonal(r, np.inf)
        a = L / 16
        assert abs(r.min() - a) < 1e-12 * L
        assert abs(a - math.sqrt(math.pi / (4.0 * eta))) < 1e-12
        assert r.min() > 1.0
    with pytest.raises(ValueError):
        O.lattice(O.params(n, 0.80, 1.0, 4))
