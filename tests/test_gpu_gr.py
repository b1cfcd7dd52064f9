"""Pressure from the pair correlation at contact (eq. pressure, Sec. 2) on
the device: ordered-pair counts per bin against the oracle's brute force
(integers, bit for bit), and the contact pressure against the EC pressure
estimator of the same run (an independent route to the same quantity)."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O

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


@pytest.mark.parametrize("n,eta,cells,dir_mode,sweeps", [(4096, 0.72, 8, 1, 0),
                                                          (4096, 0.70, 8, 1, 2),
                                                          (4096, 0.40, 8, 1, 2),
                                                          (256, 0.70, 1, 0, 2)])
def test_pair_counts_match_oracle(P, n, eta, cells, dir_mode, sweeps):
    _say(f"[gr] n={n} eta={eta} C={cells}: {sweeps} sweeps")
    g = P.System(P.make_params(n, eta, 20.0, cells, dir_mode=dir_mode))
    g.sweep(sweeps)
    x, y = g.get_positions()
    g.gr_accumulate(1.5, 200)
    g.gr_accumulate(1.5, 200)
    counts, samples, ov = g.gr_counts()
    oc, oov = O.pair_histogram(O.params(n, eta, 20.0, cells, dir_mode=dir_mode), x, y, 1.5, 200)
    assert samples == 2 and ov == 0 and oov == 0
    np.testing.assert_array_equal(counts, 2 * oc)


def test_contact_pressure_agrees_with_ec_pressure(P):
    """N = 16384, eta = 0.70, 16 x 16 cells: after 10 sweeps, 30 sweeps with the
    pair counts taken after each; Z from g(sigma+) and Z from the lift tallies
    agree within 3 % (statistics and the contact extrapolation)."""
    n, eta, C = 16384, 0.70, 16
    g = P.System(P.make_params(n, eta, 20.0, C, seed=3))
    g.sweep(10)
    g.reset_tallies()
    for _ in range(30):
        g.sweep(1)
        g.gr_accumulate(1.5, 100)
    z_ec, _, _ = g.measure_pressure()
    counts, samples, ov = g.gr_counts()
    L = O.box_length(n, 1.0, eta)
    _, _, gc, z_gr = P.gr_normalize(n, L, 1.0, 1.5, counts, samples, 0.05)
    _say(f"[gr] eta {eta}: Z(EC) = {z_ec:.4f}, Z(g contact) = {z_gr:.4f}, g(sigma+) = {gc:.4f}")
    assert ov == 0
    assert abs(z_gr - z_ec) / z_ec < 0.03
