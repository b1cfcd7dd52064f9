"""Hexatic order parameter with Delaunay neighbours on the device (eq. Psi,
Sec. 2) against the oracle's periodic triangulation: the neighbour count of
every disk equal, Psi_k within 1e-12 (the device forms exp(6 i phi) by
complex products, the oracle by atan2/cos/sin); at the start lattice the
closed form; at 1M disks Euler's relation on the torus (mean degree exactly
6) and a sample of disks against planar patches; the error paths of the
certification."""
import math
import sys

import numpy as np
import pytest

from oracle import delaunay as D
from oracle import oracle as O
from tests import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


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


@pytest.mark.parametrize("n,eta,cells,dir_mode", [(4096, 0.72, 8, 1), (256, 0.70, 1, 0)])
def test_delaunay_psi6_start_lattice(P, n, eta, cells, dir_mode):
    _say(f"[psi6-delaunay] start lattice n={n} C={cells}")
    g = P.System(P.make_params(n, eta, 20.0, cells, dir_mode=dir_mode))
    psi, nb, per, cnt = g.measure_psi6_delaunay(0.0, per_disk=True)
    want = (2.0 + 4.0 * math.cos(6.0 * math.atan2(1.0, 0.5))) / 6.0
    assert np.all(cnt == 6) and nb == 6.0
    assert np.max(np.abs(per - want)) < TOL
    assert abs(psi - want) < TOL


@pytest.mark.parametrize("n,eta,cells,dir_mode,sweeps", [
    (4096, 0.70, 8, 1, 4),
    (4096, 0.40, 8, 1, 2),     # dilute: larger Voronoi cells (default radius 4 spacings)
    (256, 0.70, 1, 0, 2),      # one periodic cell
    (65536, 0.70, 16, 1, 1),   # the 65k workload's geometry
])
def test_delaunay_psi6_matches_oracle(P, n, eta, cells, dir_mode, sweeps):
    _say(f"[psi6-delaunay] n={n} eta={eta} C={cells} after {sweeps} sweeps")
    g = P.System(P.make_params(n, eta, 20.0, cells, dir_mode=dir_mode, seed=3))
    g.sweep(sweeps)
    psi, nb, per, cnt = g.measure_psi6_delaunay(0.0, per_disk=True)
    x, y = g.get_positions()
    L = O.box_length(n, 1.0, eta)
    opsi, oper, ocnt = D.psi6_delaunay(x, y, L, L)
    np.testing.assert_array_equal(cnt, ocnt)
    assert np.max(np.abs(per - oper)) < TOL
    assert abs(psi - opsi) < TOL
    assert nb == 6.0  # Euler's relation on the torus
    # bit-repeatable
    psi2, nb2, per2, cnt2 = g.measure_psi6_delaunay(0.0, per_disk=True)
    assert psi2 == psi and np.array_equal(per2, per) and np.array_equal(cnt2, cnt)


def test_delaunay_psi6_full_size_1m(P):
    """pec_1m after one sweep: mean degree exactly 6; 64 sampled disks equal
    the oracle's triangulation of a planar patch of radius 8 sigma around each."""
    w = inputs.WORKLOADS["pec_1m"]
    _say("[psi6-delaunay] pec_1m, 1 sweep")
    g = P.System(P.make_params(w["n"], w["eta"], w["ell"], w["cells"], dir_mode=w["dir_mode"],
                               seed=w["seed"]))
    g.sweep(1)
    psi, nb, per, cnt = g.measure_psi6_delaunay(0.0, per_disk=True)
    assert nb == 6.0
    assert int(cnt.sum()) == 6 * w["n"]
    x, y = g.get_positions()
    L = O.box_length(w["n"], 1.0, w["eta"])
    rng = np.random.default_rng(9)
    for k in rng.choice(w["n"], 64, replace=False):
        dx = x - x[k]
        dy = y - y[k]
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        sel = np.nonzero(dx * dx + dy * dy < 64.0)[0]
        centre = int(np.nonzero(sel == k)[0][0])
        v = D.planar_neighbours(dx[sel], dy[sel], centre)
        assert len(v) == cnt[k]
        phi = np.arctan2(v[:, 1], v[:, 0])
        want = np.mean(np.cos(6.0 * phi) + 1j * np.sin(6.0 * phi))
        assert abs(per[k] - want) < TOL


def test_delaunay_psi6_certification_errors(P):
    import paper_1409_6948_amd.ec as E
    g = P.System(P.make_params(4096, 0.70, 20.0, 8, seed=2))
    g.sweep(1)
    L = O.box_length(4096, 1.0, 0.70)
    with pytest.raises(E.ECError) as ei:  # beyond the cell side
        g.measure_psi6_delaunay(L / 8 + 0.1)
    assert ei.value.status == E.EC_E_INVALID
    with pytest.raises(E.ECError) as ei:  # Voronoi vertices beyond r_search / 2
        g.measure_psi6_delaunay(1.2)
    assert ei.value.status == E.EC_E_UNSUPPORTED and "raise r_search" in str(ei.value)
    assert "more than 128" not in str(ei.value)
    with pytest.raises(E.ECError) as ei:  # more than 128 candidates
        g.measure_psi6_delaunay(L / 8)
    assert ei.value.status == E.EC_E_UNSUPPORTED and "more than 128" in str(ei.value)
    assert "raise r_search" not in str(ei.value)
    psi, nb = g.measure_psi6_delaunay(0.0)  # the system is untouched
    assert nb == 6.0
