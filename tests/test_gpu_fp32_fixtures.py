"""Adversarial inputs for the FP32-screened form, against the oracle bit for bit.

The FP32 screen drops a candidate only when its FP32 terms prove that it
cannot be the nearest one; everything else is recomputed in FP64.  The cases
where that proof is hardest are planted in front of the first chain of every
first-phase cell (its start disk and direction follow from the seed, so the
oracle predicts them):

* grazing partners at |c| = sigma (1 - k 2^-24) (a contact, barely) and at
  |c| = sigma (1 + k 2^-24) (a miss, barely), where sigma^2 - c^2 is at the
  level of FP32 rounding;
* two partners mirrored about the line of motion, so their contact distances
  agree to the last few FP64 bits (a near tie decided in FP64);
* a partner touching the moving disk (contact distance about 2^-40 sigma).

Each configuration is swept once by the FP32-screened form and by the FP64
form on the device and by the oracle; positions, digests and tallies must be
identical.  The oracle's event log confirms that each planted partner is the
first event of its chain where the geometry says it must be.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

N, ETA, CELLS, ELL = 1024, 0.20, 4, 6.0
U24 = 2.0 ** -24
KINDS = {
    "graze_in_1": [(0.3, 1.0 - U24)],
    "graze_in_4": [(0.3, 1.0 - 4 * U24)],
    "graze_out_1": [(0.3, 1.0 + U24)],
    "graze_out_4": [(0.3, 1.0 + 4 * U24)],
    "near_tie": [(0.9, 0.6), (0.9, -0.6)],
    "touch": [(1.0 + 2.0 ** -40, 0.0)],
}


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


def _plant(p, kinds):
    """Lattice start with partners planted in front of chain 0 of each
    first-phase cell; returns (x, y, [(cell, kind, start id, partner ids)])."""
    x, y = O.lattice(p)
    L = O.box_length(p.n, 1.0, p.eta)
    C = p.cells
    _, _, perm = O.sweep_draws(p, 0)
    cell_of = O.assign_cells(p, x, y, 0)
    first = [c for c in range(C * C) if ((c % C) & 1) | (((c // C) & 1) << 1) == perm[0]]
    planted = []
    for c, kind in zip(first, kinds):
        ids = sorted(int(i) for i in np.nonzero(cell_of == c)[0])
        a = ids[O.start_index(p, 0, c, 0, len(ids))]
        dx, dy = O.direction(p, 0, c, 0)
        offs = KINDS[kind]
        movers = [i for i in ids if i != a][-len(offs):]
        save = [(m, x[m], y[m]) for m in movers]
        for (al, ac), m in zip(offs, movers):
            # r = al d + ac d_perp with d_perp = (-dy, dx): r . d = al, r x d = -ac
            x[m] = math.fmod(x[a] + al * dx - ac * dy + L, L)
            y[m] = math.fmod(y[a] + al * dy + ac * dx + L, L)
        same_cells = np.array_equal(O.assign_cells(p, x, y, 0), cell_of)
        d, _, _ = O.min_pair_distance(x, y, L, r_cut=1.0)
        if same_cells and d == math.inf:
            planted.append((c, kind, a, movers))
        else:  # the plant would overlap a lattice disk or change a cell: undo it
            for m, mx, my in save:
                x[m], y[m] = mx, my
    return x, y, planted


def test_fp32_screen_adversarial_fixtures(P):
    names = list(KINDS)
    hits = {k: 0 for k in names}
    confirmed = {k: 0 for k in names}
    for seed in range(1, 13):
        kinds = [names[(seed * 4 + t) % len(names)] for t in range(4)]
        p = O.params(N, ETA, ELL, CELLS, dir_mode=O.DIR_ISO, seed=seed)
        x, y, planted = _plant(p, kinds)
        if not planted:
            continue
        _say(f"[fp32 fixtures] seed {seed}: " + ", ".join(f"{k}@{c}" for c, k, _, _ in planted))
        st, ev = O.run_logged(p, x, y, 0, 1)
        for c, kind, a, movers in planted:
            hits[kind] += 1
            e = ev[ev["cell"] == c][0]  # first event of chain 0 of the cell
            assert e["active"] == a
            if kind.startswith("graze_in") or kind == "touch":
                assert e["kind"] == O.EV_LIFT and e["gid"] == movers[0], (kind, e)
                if kind == "touch":
                    assert e["s"] < 1e-10
                confirmed[kind] += 1
            elif kind == "near_tie":
                assert e["kind"] == O.EV_LIFT and e["gid"] in movers
                confirmed[kind] += 1
            else:  # a miss by 2^-24 sigma: the planted disk is not hit first
                if e["gid"] not in movers:
                    confirmed[kind] += 1
        res = []
        for prec in (P.EC_PREC_FP32_SCREEN, P.EC_PREC_FP64):
            g = P.System(P.make_params(N, ETA, ELL, CELLS, seed=seed, precision=prec))
            g.set_positions(x, y)
            g.sweep(1)
            gx, gy = g.get_positions()
            delta, cnt = g.get_cell_tallies()
            res.append((gx, gy, g.get_digests(1), delta, cnt))
            g.close()
        for gx, gy, dig, delta, cnt in res:
            np.testing.assert_array_equal(gx, st.x)
            np.testing.assert_array_equal(gy, st.y)
            assert int(dig[0]) == st.digests[0]
            np.testing.assert_array_equal(delta, st.acc_delta)
            np.testing.assert_array_equal(cnt, st.acc_cnt)
    _say(f"[fp32 fixtures] planted {hits}, confirmed by the oracle's log {confirmed}")
    for k in names:
        assert hits[k] >= 2, (k, hits)
        assert confirmed[k] >= 2, (k, confirmed)
