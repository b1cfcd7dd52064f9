"""Statistical checks on the device with fixed seeds: the start rules and the
boundary rules against each other (Sec. 3.4, Fig. 3), and the mean free path
the paper prints.

Negative control of the start rule (Sec. 3.4, Fig. 2 and 3): with n_m > 1
chains per cell, start disks drawn with replacement give one pressure by
both routes (lift tallies, eq. EC pressure; g(r) at contact, eq. pressure),
while a shuffled list of distinct start disks gives a pressure that differs
from it far beyond the statistical error.

The run is deterministic (fixed seeds, a path bit-exact with the oracle), so
the statistical margins below are fixed numbers of this trajectory, not a
flaky draw: 8 systems per rule, N = 16384, eta = 0.70, 16 x 16 cells,
ell = 20 sigma, 20 + 60 sweeps."""
import math
import sys

import pytest

pytestmark = pytest.mark.gpu

N, ETA, CELLS, ELL = 16384, 0.70, 16, 20.0
R_MAX, BINS, FIT = 1.5, 100, 0.05
SEEDS = 8


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


def _mean_se(v):
    m = sum(v) / len(v)
    return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))


def test_distinct_starts_bias_the_pressure(P):
    box = math.sqrt(N * math.pi / (4.0 * ETA))
    ps = []
    for rule in (P.EC_START_REPLACE, P.EC_START_DISTINCT):
        for seed in range(1, SEEDS + 1):
            ps.append(P.make_params(N, ETA, ELL, CELLS, seed=seed, start_mode=rule, system=len(ps)))
    _say(f"[start-rules] {len(ps)} systems, N={N} eta={ETA} C={CELLS}")
    b = P.Batch(ps)
    try:
        b.sweep(20)
        for s in b.systems:
            s.reset_tallies()
            s.gr_reset()
        for _ in range(60):
            b.sweep(1)
            for s in b.systems:
                s.gr_accumulate(R_MAX, BINS)
        z_ec, z_gr = [], []
        for s in b.systems:
            z_ec.append(s.measure_pressure()[0])
            counts, samples, ov = s.gr_counts()
            assert ov == 0 and samples == 60
            z_gr.append(P.gr_normalize(N, box, 1.0, R_MAX, counts, samples, FIT)[3])
    finally:
        b.close()
    ec_r, ec_d = _mean_se(z_ec[:SEEDS]), _mean_se(z_ec[SEEDS:])
    gr_r, gr_d = _mean_se(z_gr[:SEEDS]), _mean_se(z_gr[SEEDS:])
    _say(f"[start-rules] replacement: Z(EC) {ec_r[0]:.4f}+-{ec_r[1]:.4f}, "
         f"Z(g) {gr_r[0]:.4f}+-{gr_r[1]:.4f}")
    _say(f"[start-rules] distinct:    Z(EC) {ec_d[0]:.4f}+-{ec_d[1]:.4f}, "
         f"Z(g) {gr_d[0]:.4f}+-{gr_d[1]:.4f}")
    # the correct rule: both routes give one pressure within the errors
    assert abs(ec_r[0] - gr_r[0]) < 3.0 * math.hypot(ec_r[1], gr_r[1])
    # the shuffled rule: the contact pressure lies far from the correct one
    assert gr_r[0] - gr_d[0] > 5.0 * math.hypot(gr_r[1], gr_d[1])
    assert ec_r[0] - ec_d[0] > 4.0 * math.hypot(ec_r[1], ec_d[1])


def test_rejection_at_the_boundary_samples_the_same_pressure(P):
    """Rejection at the cell boundary (Sec. 3.4) with starts drawn with
    replacement gives the contact pressure of the paper's reflection; with
    shuffled distinct starts both boundary rules are far off (Fig. 3).
    N = 16384, eta = 0.70, 16 x 16 cells, ell = 0.2 sigma, 8 seeds per case,
    1500 + 1500 sweeps, g(r) every 10 sweeps."""
    box = math.sqrt(N * math.pi / (4.0 * ETA))
    z = {}
    for bname, bflag in (("reflect", 0), ("reject", P.EC_FLAG_REJECT)):
        ps = []
        for rule in (P.EC_START_REPLACE, P.EC_START_DISTINCT):
            for seed in range(1, SEEDS + 1):
                ps.append(P.make_params(N, ETA, 0.2, CELLS, seed=seed, start_mode=rule, system=len(ps),
                                        flags=bflag))
        _say(f"[boundary-rules] {bname}: {len(ps)} systems")
        b = P.Batch(ps)
        try:
            b.set_graph(True)
            b.sweep(1500)
            for s in b.systems:
                s.gr_reset()
            for _ in range(150):
                b.sweep(10)
                for s in b.systems:
                    s.gr_accumulate(R_MAX, BINS)
            zs = []
            for s in b.systems:
                counts, samples, ov = s.gr_counts()
                assert ov == 0
                zs.append(P.gr_normalize(N, box, 1.0, R_MAX, counts, samples, FIT)[3])
        finally:
            b.close()
        z[(bname, "replacement")] = _mean_se(zs[:SEEDS])
        z[(bname, "distinct")] = _mean_se(zs[SEEDS:])
    for k, v in z.items():
        _say(f"[boundary-rules] {k}: Z(g) {v[0]:.4f} +- {v[1]:.4f}")
    ref = z[("reflect", "replacement")]
    rej = z[("reject", "replacement")]
    assert abs(rej[0] - ref[0]) < 3.0 * math.hypot(rej[1], ref[1])
    for bname in ("reflect", "reject"):
        dist = z[(bname, "distinct")]
        assert ref[0] - dist[0] > 10.0 * math.hypot(ref[1], dist[1])


def test_mean_free_path_at_eta_071_matches_the_paper(P):
    """The mean free path the paper prints for eta = 0.71 (tests/golden/
    mean_free_path.json), on the device: N = 65536, 16 x 16 cells,
    ell = 20 sigma, sweeps 6-15 from the lattice."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mean_free_path.json")))
    g = P.System(P.make_params(65536, gold["eta"], 20.0, 16, seed=4))
    g.sweep(5)
    g.reset_tallies()
    g.sweep(10)
    _, _, c = g.measure_pressure()
    lam = 20.0 * c["chains"] / (c["lifts"] + c["frozen"])
    _say(f"[mean-free-path] eta {gold['eta']}: lambda = {lam:.4f} sigma")
    assert abs(lam - gold["lambda0_over_sigma"]) <= 0.005
