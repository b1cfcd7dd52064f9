"""Hexatic order parameter on the device (Sec. 2, eq. Psi; cutoff neighbours
within 1.4 sigma) against the CPU oracle's brute force: at the start lattice
(closed form), after sweeps of small systems (every disk), and at the
16.7M-disk workload after one sweep (a sample of disks, each recomputed on
the CPU from the full position arrays).  The device forms exp(6 i phi) by
complex products, the oracle by atan2/cos/sin, so values agree to rounding:
the bound used is 1e-12 per disk."""
import math
import sys

import numpy as np
import pytest

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
def test_psi6_start_lattice(P, n, eta, cells, dir_mode):
    g = P.System(P.make_params(n, eta, 20.0, cells, dir_mode=dir_mode))
    psi, nb, per = g.measure_psi6(1.4, per_disk=True)
    want = (2.0 + 4.0 * math.cos(6.0 * math.atan2(1.0, 0.5))) / 6.0
    assert nb == 6.0
    assert abs(psi - want) < TOL and np.max(np.abs(per - want)) < TOL


@pytest.mark.parametrize("n,eta,cells,dir_mode,sweeps", [(4096, 0.72, 8, 1, 2),
                                                          (4096, 0.45, 8, 1, 2),
                                                          (256, 0.70, 1, 0, 3)])
def test_psi6_after_sweeps_matches_oracle(P, n, eta, cells, dir_mode, sweeps):
    _say(f"[psi6] n={n} eta={eta} C={cells}: {sweeps} sweeps")
    p = P.make_params(n, eta, 20.0, cells, dir_mode=dir_mode)
    g = P.System(p)
    g.sweep(sweeps)
    x, y = g.get_positions()
    psi, nb, per = g.measure_psi6(1.4, per_disk=True)
    psi2, nb2 = g.measure_psi6(1.4)
    assert psi2 == psi and nb2 == nb  # fixed-order sums repeat bit for bit
    opsi, onb, oper = O.psi6(O.params(n, eta, 20.0, cells, dir_mode=dir_mode), x, y, 1.4)
    assert nb == onb
    assert abs(psi - opsi) < TOL
    assert np.max(np.abs(per - oper)) < TOL


def _psi6_sample(x, y, L, ks, rc=1.4):
    """Psi_k of the disks ks from the full position arrays (grid of side >= rc)."""
    g = int(L // rc)
    s = L / g
    cx = np.minimum((x / s).astype(np.int64), g - 1)
    cy = np.minimum((y / s).astype(np.int64), g - 1)
    key = cy * g + cx
    order = np.argsort(key, kind="stable")
    skey = key[order]
    out = []
    for k in ks:
        acc, cnt = 0j, 0
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                kk = ((cy[k] + oy) % g) * g + (cx[k] + ox) % g
                lo, hi = np.searchsorted(skey, [kk, kk + 1])
                for l in order[lo:hi]:
                    if l == k:
                        continue
                    dx = x[l] - x[k]
                    dy = y[l] - y[k]
                    dx -= L * round(dx / L)
                    dy -= L * round(dy / L)
                    if dx * dx + dy * dy < rc * rc:
                        ph = math.atan2(dy, dx)
                        acc += complex(math.cos(6 * ph), math.sin(6 * ph))
                        cnt += 1
        out.append(acc / cnt if cnt else 0j)
    return np.array(out)


def test_psi6_full_size_16m(P):
    w = inputs.WORKLOADS["pec_16m"]
    n = w["n"]
    _say(f"[psi6] pec_16m: one sweep, then Psi on the device")
    g = P.System(P.make_params(n, w["eta"], w["ell"], w["cells"], seed=w["seed"]))
    g.sweep(1)
    psi, nb, per = g.measure_psi6(1.4, per_disk=True)
    x, y = g.get_positions()
    L = O.box_length(n, 1.0, w["eta"])
    rng = np.random.default_rng(0)
    ks = rng.choice(n, size=64, replace=False)
    ref = _psi6_sample(x, y, L, ks)
    assert np.max(np.abs(per[ks] - ref)) < TOL
    assert abs(psi - per.mean()) < 1e-9
    assert 0.0 <= abs(psi) <= 1.0 and 5.0 < nb < 7.0
    _say(f"[psi6] pec_16m: Psi = {psi}, mean neighbours {nb}")
