"""The device overlap check (EC_FLAG_CHECK_OVERLAP): it changes no result,
and it reports a pair of disks closer than sigma."""
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("n,eta,cells,ell,dm", [
    (65536, 0.70, 16, 20.0, 1),
    (4096, 0.72, 8, 20.0, 1),
    (256, 0.70, 1, 20.0, 0),   # one periodic cell: all pairs
])
def test_check_changes_nothing(P, n, eta, cells, ell, dm):
    _say(f"[overlap] n={n} C={cells}: 2 sweeps with and without the check")
    out = []
    for flags in (0, P.EC_FLAG_CHECK_OVERLAP):
        g = P.System(P.make_params(n, eta, ell, cells, dir_mode=dm, seed=3, flags=flags))
        g.sweep(2)
        out.append(g.get_positions() + (g.get_digests(2),) + g.get_cell_tallies())
        g.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)
