"""The allocation-free entry point (ec_sweep_static) against the workspace
entry points (ec_init_system + ec_sweep): the same sweeps give the same
positions and per-sweep digests bit for bit, on consecutive calls that share
the static buffer, the second with a smaller system."""
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


def _reference(P, p, first, sweeps):
    """Positions before sweep `first`, after it + sweeps, and the digests of
    those sweeps, from the workspace entry points."""
    g = P.System(p)
    g.sweep(first)
    x0, y0 = g.get_positions()
    g.sweep(sweeps)
    x1, y1 = g.get_positions()
    dig = g.get_digests(sweeps)
    g.close()
    return (x0, y0), (x1, y1), dig


@pytest.mark.parametrize("order", ["large_first"])
def test_static_sweeps_equal_workspace_sweeps(P, order):
    import torch
    cases = [  # (N, eta, ell, C, dir, first sweep, sweeps): each call smaller than the one before
        (65536, 0.70, 20.0, 16, P.EC_DIR_ISOTROPIC, 0, 3),
        (16384, 0.72, 10.0, 8, P.EC_DIR_ISOTROPIC, 2, 2),
        (256, 0.70, 20.0, 1, P.EC_DIR_XY, 1, 3),
    ]
    for n, eta, ell, C, dm, first, sweeps in cases:
        _say(f"[no-alloc] n={n} eta={eta} C={C} first sweep {first}, {sweeps} sweeps")
        p = P.make_params(n, eta, ell, C, dir_mode=dm, seed=21)
        (x0, y0), (x1, y1), dig = _reference(P, p, first, sweeps)
        dx = torch.tensor(x0, dtype=torch.float64, device="cuda")
        dy = torch.tensor(y0, dtype=torch.float64, device="cuda")
        ddig = torch.full((sweeps,), -1, dtype=torch.int64, device="cuda")
        derr = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        P.ec.sweep_static(p, dx, dy, first, sweeps, ddig, derr)
        torch.cuda.synchronize()
        assert int(derr.cpu()[0]) == 0
        np.testing.assert_array_equal(dx.cpu().numpy(), x1)
        np.testing.assert_array_equal(dy.cpu().numpy(), y1)
        np.testing.assert_array_equal(ddig.cpu().numpy().view(np.uint64), dig)


def test_static_sweeps_reject_systems_beyond_the_buffer(P):
    import torch
    import paper_1409_6948_amd.ec as E
    n = 514 * 514  # above 262144 disks
    p = P.make_params(n, 0.70, 20.0, 32)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(E.ECError) as ei:
        P.ec.sweep_static(p, x, x.clone(), 0, 1)
    assert ei.value.status == E.EC_E_NOMEM
