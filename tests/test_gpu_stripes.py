"""The striped decomposition with rejection (EC_FLAG_STRIPES; Sec. 3.4, Fig. 3
"stripes"; Sec. 4): bit for bit against the oracle, and the statistics of
Fig. 3 -- with starts drawn with replacement the stripes sample the pressure
of the checkerboard with reflection; with shuffled distinct starts they do
not.  The statistical run is deterministic (fixed seeds), so its margins are
fixed numbers of this trajectory."""
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


@pytest.mark.parametrize("n,eta,stripes,ell,sweeps,kw", [
    (16384, 0.70, 16, 0.2, 2, {}),
    (4096, 0.50, 8, 1.0, 3, {}),
    (1024, 0.30, 4, 3.0, 3, {}),
    (64, 0.10, 4, 30.0, 4, {}),   # flights beyond the nearest-image range (pseudo events)
    (1024, 0.60, 4, 0.5, 3, dict(chains_per_cell=50, start_mode=1)),
])
def test_stripes_match_the_oracle(P, n, eta, stripes, ell, sweeps, kw):
    _say(f"[stripes] n={n} eta={eta} S={stripes} ell={ell} sweeps={sweeps} {kw}")
    p = O.params(n, eta, ell, stripes, dir_mode=O.DIR_XY, boundary=O.BOUNDARY_STRIPES, seed=5, **kw)
    st = O.State(p)
    st.run(sweeps)
    g = P.System(P.make_params(n, eta, ell, stripes, dir_mode=P.EC_DIR_XY, seed=5,
                               flags=P.EC_FLAG_STRIPES | P.EC_FLAG_CHECK_OVERLAP, **kw))
    g.sweep(sweeps)
    gx, gy = g.get_positions()
    delta, cnt = g.get_cell_tallies()
    np.testing.assert_array_equal(g.get_digests(sweeps), np.array(st.digests, dtype=np.uint64))
    np.testing.assert_array_equal(gx, st.x)
    np.testing.assert_array_equal(gy, st.y)
    np.testing.assert_array_equal(delta, st.acc_delta)
    np.testing.assert_array_equal(cnt, st.acc_cnt)
    if eta == 0.10:
        assert cnt[:, O.CNT_PSEUDO].sum() > 0
    g.close()


def _mean_se(v):
    m = sum(v) / len(v)
    return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))


def test_stripes_sample_the_checkerboard_pressure(P):
    """N = 16384, eta = 0.70, 16 stripes against 16 x 16 square cells with
    reflection, ell = 0.2 sigma, 8 seeds per case, 1000 + 1000 sweeps, g(r)
    every 10 sweeps: the contact pressure of stripes with replacement agrees
    with the checkerboard's; with shuffled distinct starts it lies far off."""
    N, ETA, C, ELL, SEEDS = 16384, 0.70, 16, 0.2, 8
    R_MAX, BINS, FIT = 1.5, 100, 0.05
    box = math.sqrt(N * math.pi / (4.0 * ETA))
    z = {}
    cases = (("squares", 0, P.EC_DIR_ISOTROPIC, (P.EC_START_REPLACE,)),
             ("stripes", P.EC_FLAG_STRIPES, P.EC_DIR_XY, (P.EC_START_REPLACE, P.EC_START_DISTINCT)))
    for name, flags, dm, rules in cases:
        ps = []
        for rule in rules:
            for seed in range(1, SEEDS + 1):
                ps.append(P.make_params(N, ETA, ELL, C, dir_mode=dm, seed=seed, start_mode=rule,
                                        system=len(ps), flags=flags))
        _say(f"[stripes-stats] {name}: {len(ps)} systems")
        b = P.Batch(ps)
        try:
            b.set_graph(True)
            b.sweep(1000)
            for s in b.systems:
                s.gr_reset()
            for t in range(100):
                b.sweep(10)
                for s in b.systems:
                    s.gr_accumulate(R_MAX, BINS)
                if t % 25 == 24:
                    b.stream.synchronize()
                    _say(f"[stripes-stats] {name}: {(t + 1) * 10} sweeps measured")
            zs = []
            for s in b.systems:
                counts, samples, ov = s.gr_counts()
                assert ov == 0
                zs.append(P.gr_normalize(N, box, 1.0, R_MAX, counts, samples, FIT)[3])
        finally:
            b.close()
        for r, rule in enumerate(rules):
            z[(name, rule)] = _mean_se(zs[r * SEEDS:(r + 1) * SEEDS])
    for k, v in z.items():
        _say(f"[stripes-stats] {k}: Z(g) {v[0]:.4f} +- {v[1]:.4f}")
    ref = z[("squares", P.EC_START_REPLACE)]
    rep = z[("stripes", P.EC_START_REPLACE)]
    dis = z[("stripes", P.EC_START_DISTINCT)]
    assert abs(rep[0] - ref[0]) < 3.0 * math.hypot(rep[1], ref[1])
    assert abs(dis[0] - ref[0]) > 10.0 * math.hypot(dis[1], ref[1])
