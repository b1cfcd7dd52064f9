"""PEC against serial EC at eta = 0.70 (statistical parity of the whole method).

Both sample the hard-disk measure (Sec. 3.4: the parallel scheme with starts
drawn with replacement keeps detailed balance, Fig. 2-3), so the pressure of
the same system must agree within the combined errors: N = 256 disks at
eta = 0.70, serial EC with isotropic chains in one periodic box against PEC
in 4 x 4 walled cells, 8 seeds each, from the lattice.  Fixed seeds make the
outcome a deterministic function of the code.  The EC estimator is the
collision route of Sec. 3.4; for PEC the contact value of g(r) (eq. pressure)
is checked as well.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N, ETA, ELL, SEEDS = 256, 0.70, 20.0, 8
WARM, SWEEPS = 150, 300


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


def _stats(v):
    m = sum(v) / len(v)
    return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))


def test_pec_pressure_equals_serial_ec(P):
    import torch
    box = math.sqrt(N * math.pi / (4.0 * ETA))
    _say(f"[pec-vs-serial] serial EC: {SEEDS} periodic systems, {WARM} + {SWEEPS} sweeps")
    serial = []
    for sd in range(SEEDS):
        st = torch.cuda.Stream()
        serial.append(P.System(P.make_params(N, ETA, ELL, 1, dir_mode=P.EC_DIR_ISOTROPIC,
                                             seed=100 + sd), stream=st))
    for g in serial:
        g.sweep(WARM)
    torch.cuda.synchronize()
    for g in serial:
        g.reset_tallies()
    for t in range(SWEEPS // 50):
        for g in serial:
            g.sweep(50)
        torch.cuda.synchronize()
        _say(f"[pec-vs-serial] serial: {(t + 1) * 50} sweeps")
    z_serial = [g.measure_pressure()[0] for g in serial]
    for g in serial:
        g.close()
    _say(f"[pec-vs-serial] PEC: {SEEDS} systems of 4 x 4 cells, batched")
    b = P.Batch([P.make_params(N, ETA, ELL, 4, seed=100 + sd, system=sd) for sd in range(SEEDS)])
    b.sweep(WARM)
    b.stream.synchronize()
    for s in b.systems:
        s.reset_tallies()
        s.gr_reset()
    for _ in range(SWEEPS):
        b.sweep(1)
        for s in b.systems:
            s.gr_accumulate(1.5, 100)
    b.stream.synchronize()
    z_pec = [s.measure_pressure()[0] for s in b.systems]
    z_gr = []
    for s in b.systems:
        counts, samples, overlaps = s.gr_counts()
        assert overlaps == 0
        z_gr.append(P.gr_normalize(N, box, 1.0, 1.5, counts, samples, 0.05)[3])
    b.close()
    ms, ss = _stats(z_serial)
    mp, sp = _stats(z_pec)
    mg, sg = _stats(z_gr)
    _say(f"[pec-vs-serial] Z serial {ms:.4f} +- {ss:.4f}, PEC {mp:.4f} +- {sp:.4f} (EC route), "
         f"{mg:.4f} +- {sg:.4f} (g route)")
    assert abs(mp - ms) < 3.0 * math.hypot(sp, ss)
    assert abs(mg - ms) < 3.0 * math.hypot(sg, ss) + 0.02  # + the contact fit's bias
    # a sanity band: hexatic-region pressure of hard disks near eta = 0.70
    assert 8.5 < ms < 11.0
