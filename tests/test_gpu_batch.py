"""Batched form: several walled systems advanced by shared launches.

The batch only changes the schedule (one launch per sweep step for all
systems, an optional HIP graph per sweep, cells per workgroup), so every
system must follow exactly the sweeps of a solo run with the same parameters:
positions, digests and tallies are compared bit for bit.  The smallest
systems are also checked against the CPU oracle.  Workload: the meta-draws of
the 64-system ensemble (N log-uniform in [4096, 262144], eta uniform in
[0.30, 0.72], about 64 disks per cell).
"""
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


def _params(P, cfgs):
    return [P.make_params(c["n"], c["eta"], c["ell"], c["cells"], dir_mode=c["dir_mode"],
                          seed=c["seed"], system=i) for i, c in enumerate(cfgs)]


def _state(sys_handle):
    x, y = sys_handle.get_positions()
    delta, cnt = sys_handle.get_cell_tallies()
    return x, y, delta, cnt


def _solo_states(P, ps, sweeps):
    out = []
    for p in ps:
        s = P.System(p)
        s.sweep(sweeps)
        out.append(_state(s) + (s.get_digests(sweeps),))
        s.close()
    return out


def _assert_same(batch, solos, sweeps):
    for i, (s, ref) in enumerate(zip(batch.systems, solos)):
        x, y, delta, cnt = _state(s)
        np.testing.assert_array_equal(x, ref[0], err_msg=f"system {i} x")
        np.testing.assert_array_equal(y, ref[1], err_msg=f"system {i} y")
        np.testing.assert_array_equal(delta, ref[2], err_msg=f"system {i} tallies")
        np.testing.assert_array_equal(cnt, ref[3], err_msg=f"system {i} counts")
        np.testing.assert_array_equal(s.get_digests(sweeps), ref[4], err_msg=f"system {i} digests")


def test_batch_of_64_equals_solo_runs(P):
    cfgs = inputs.batch_systems(64, seed=0)
    ps = _params(P, cfgs)
    sweeps = 2
    _say(f"[batch] 64 systems, sum N = {sum(c['n'] for c in cfgs)}, {sweeps} sweeps")
    solos = _solo_states(P, ps, sweeps)
    b = P.Batch(ps)
    b.sweep(sweeps)
    b.stream.synchronize()
    _assert_same(b, solos, sweeps)
    b.close()


@pytest.mark.parametrize("schedule,cpb", [("ready-queue", 1), ("ready-queue", 2), ("ready-queue", 4),
                                          ("phase-launches", 1), ("phase-launches", 4),
                                          ("one-launch", 2)])
def test_batch_graph_and_schedule_keep_trajectories(P, schedule, cpb):
    cfgs = inputs.batch_systems(64, seed=0)[:12]
    ps = _params(P, cfgs)
    sweeps = 3
    _say(f"[batch] graph replay, schedule {schedule}, cells per workgroup {cpb}")
    solos = _solo_states(P, ps, sweeps)
    b = P.Batch(ps)
    b.set_schedule(schedule)
    b.set_cells_per_block(cpb)
    b.set_graph(True)
    b.sweep(1)
    b.sweep(sweeps - 1)  # replays of the captured sweep
    b.stream.synchronize()
    _assert_same(b, solos, sweeps)
    b.close()


def test_batch_one_launch_equals_solo_runs(P):
    """The one-launch schedule forced on a batch (the batch default is one
    launch per phase) follows the solo trajectories; systems smaller than the
    largest leave their surplus wavefronts idle."""
    cfgs = inputs.batch_systems(64, seed=0)[:12]
    ps = _params(P, cfgs)
    sweeps = 2
    _say("[batch] one-launch schedule against solo runs")
    solos = _solo_states(P, ps, sweeps)
    for p in ps:
        p.flags |= P.EC_FLAG_ONE_LAUNCH
    b = P.Batch(ps)
    b.set_graph(True)
    b.sweep(sweeps)
    b.stream.synchronize()
    _assert_same(b, solos, sweeps)
    b.close()


def test_batch_rejection_variant_equals_solo_runs(P):
    """Rejection at the cell boundary (ell = 3 sigma) in a batch follows the
    solo trajectories."""
    cfgs = inputs.batch_systems(64, seed=0)[:12]
    ps = [P.make_params(c["n"], c["eta"], 3.0, c["cells"], dir_mode=c["dir_mode"], seed=c["seed"],
                        system=i, flags=P.EC_FLAG_REJECT) for i, c in enumerate(cfgs)]
    sweeps = 2
    _say("[batch] rejection variant against solo runs")
    solos = _solo_states(P, ps, sweeps)
    b = P.Batch(ps)
    b.set_graph(True)
    b.sweep(sweeps)
    b.stream.synchronize()
    _assert_same(b, solos, sweeps)
    b.close()


def test_autotune_leaves_the_state_untouched(P):
    cfgs = inputs.batch_systems(64, seed=0)[:12]
    ps = _params(P, cfgs)
    solos = _solo_states(P, ps, 3)
    b = P.Batch(ps)
    b.sweep(1)
    sched, cpb, ms = b.autotune(trial_sweeps=1)
    _say(f"[batch] autotune chose {sched} with {cpb} cells per workgroup, trials {ms}")
    assert cpb in (1, 2, 4) and sched in ("phase-launches", "one-launch", "ready-queue")
    assert all(b.systems[i].sweep_count() == 1 for i in range(len(ps)))
    b.set_graph(True)
    b.sweep(2)
    b.stream.synchronize()
    _assert_same(b, solos, 3)
    b.close()


def test_smallest_batch_systems_match_the_oracle(P):
    cfgs = inputs.batch_systems(64, seed=0)
    order = sorted(range(len(cfgs)), key=lambda i: cfgs[i]["n"])[:2]
    ps = _params(P, cfgs)
    b = P.Batch(ps)
    sweeps = 2
    b.sweep(sweeps)
    b.stream.synchronize()
    for i in order:
        c = cfgs[i]
        _say(f"[batch] oracle check of system {i}: N={c['n']} eta={c['eta']:.3f} C={c['cells']}")
        st = O.State(O.params(c["n"], c["eta"], c["ell"], c["cells"], dir_mode=c["dir_mode"],
                              seed=c["seed"], system=i))
        st.run(sweeps)
        x, y = b.systems[i].get_positions()
        np.testing.assert_array_equal(x, st.x)
        np.testing.assert_array_equal(y, st.y)
        np.testing.assert_array_equal(b.systems[i].get_digests(sweeps),
                                      np.array(st.digests[-sweeps:], dtype=np.uint64))
    b.close()


def test_batch_fp32_screen_equals_solo_fp64(P):
    """The FP32-screened batch (the batched workload's form) follows the FP64
    solo trajectories bit for bit."""
    cfgs = inputs.batch_systems(64, seed=0)[:16]
    ps = _params(P, cfgs)
    sweeps = 2
    _say("[batch] FP32-screened batch against FP64 solo runs")
    solos = _solo_states(P, ps, sweeps)
    for p in ps:
        p.precision = P.EC_PREC_FP32_SCREEN
    b = P.Batch(ps)
    b.set_graph(True)
    b.sweep(sweeps)
    b.stream.synchronize()
    _assert_same(b, solos, sweeps)
    b.close()
