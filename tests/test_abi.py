"""Host-side checks of the C ABI: the library loads, exports every symbol
declared in include/ec.h, and rejects invalid parameters (no GPU needed)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import paper_1409_6948_amd as P
from paper_1409_6948_amd import ec as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ec.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ec_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    names = _declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(E.EXPORTED)


def test_status_strings():
    lib = P.load_library()
    for s in range(7):
        assert lib.ec_status_string(s)
    assert lib.ec_last_error(None) == b""


def _ws(**kw):
    base = dict(n=65536, eta=0.70, ell=20.0, cells=16)
    base.update(kw)
    return P.workspace_bytes(P.make_params(**base))


def test_workspace_sizes_scale_with_n():
    a = _ws()
    b = P.workspace_bytes(P.make_params(1048576, 0.72, 20.0, 64))
    assert a >= 65536 * 24 and b >= 1048576 * 24 and b > 10 * a


@pytest.mark.parametrize("kw,status", [
    (dict(n=0), E.EC_E_INVALID),
    (dict(eta=0.0), E.EC_E_INVALID),
    (dict(eta=0.91), E.EC_E_INVALID),
    (dict(eta=0.80), E.EC_E_INVALID),                  # the start lattice overlaps above pi/4
    (dict(ell=0.0), E.EC_E_INVALID),
    (dict(cells=3), E.EC_E_INVALID),
    (dict(cells=2), E.EC_E_INVALID),
    (dict(cells=15), E.EC_E_INVALID),
    (dict(dir_mode=E.EC_DIR_XY), E.EC_E_INVALID),      # xy chains need periodic boundaries
    (dict(cells=128), E.EC_E_UNSUPPORTED),             # cell side 2.1 sigma < 3 sigma
    (dict(cells=1, n=4096), E.EC_E_UNSUPPORTED),       # one periodic cell holds <= 2048 disks
    (dict(cells_per_block=3), E.EC_E_INVALID),
    (dict(flags=E.EC_FLAG_PHASE_LAUNCHES | E.EC_FLAG_ONE_LAUNCH), E.EC_E_INVALID),
    (dict(flags=E.EC_FLAG_REJECT, cells=1, n=1024), E.EC_E_UNSUPPORTED),   # walled cells only
    (dict(flags=E.EC_FLAG_REJECT, precision=E.EC_PREC_FP32_SCREEN), E.EC_E_UNSUPPORTED),
])
def test_invalid_parameters_rejected(kw, status):
    with pytest.raises(E.ECError) as ei:
        _ws(**kw)
    assert ei.value.status == status


def test_walled_cell_side_limits():
    """A walled cell's LDS (one 20-byte slot per bin of side < 0.7 sigma, plus
    its lists) must fit 160 KiB: N = 68^2 in 4 x 4 cells is accepted at a
    side of 54.3 sigma (eta = 0.077) and refused at 67.4 sigma (eta = 0.050)."""
    import math
    n, cells = 68 * 68, 4
    for eta, ok in ((0.077, True), (0.050, False)):
        w = math.sqrt(n * math.pi / (4.0 * eta)) / cells
        assert (w < 55.0) == ok
        if ok:
            assert _ws(n=n, eta=eta, cells=cells) > 0
        else:
            with pytest.raises(E.ECError) as ei:
                _ws(n=n, eta=eta, cells=cells)
            assert ei.value.status == E.EC_E_UNSUPPORTED


def test_abi_version_checked():
    p = P.make_params(65536, 0.70, 20.0, 16)
    p.abi_version = 99
    with pytest.raises(E.ECError):
        P.workspace_bytes(p)


def test_init_rejects_small_workspace_without_touching_gpu():
    lib = P.load_library()
    p = P.make_params(65536, 0.70, 20.0, 16)
    h = C.c_void_p()
    st = lib.ec_init_system(C.byref(p), C.c_void_p(0x1000), 16, None, C.byref(h))
    assert st == E.EC_E_NOMEM and not h.value
    st = lib.ec_init_system(C.byref(p), None, 1 << 30, None, C.byref(h))
    assert st == E.EC_E_INVALID
    # the workspace's arrays are laid out 256-byte aligned from its start
    st = lib.ec_init_system(C.byref(p), C.c_void_p(0x1010), 1 << 30, None, C.byref(h))
    assert st == E.EC_E_INVALID and not h.value
    ps = (E.Params * 2)(P.make_params(4096, 0.70, 20.0, 8), P.make_params(4096, 0.60, 20.0, 8))
    b = C.c_void_p()
    st = lib.ec_init_batch(ps, 2, C.c_void_p(0x1010), 1 << 30, None, C.byref(b))
    assert st == E.EC_E_INVALID and not b.value


def test_batch_workspace_is_systems_plus_snapshot():
    """The batch holds every system's workspace, a snapshot of them (for the
    autotuner) and the ready queue: 16 bytes per cell of all systems."""
    from tests import inputs
    cfgs = inputs.batch_systems(64, seed=0)
    ps = [P.make_params(c["n"], c["eta"], c["ell"], c["cells"], seed=c["seed"], system=i)
          for i, c in enumerate(cfgs)]
    solo = sum(P.workspace_bytes(p) for p in ps)
    cells = sum(c["cells"] ** 2 for c in cfgs)
    total = P.batch_workspace_bytes(ps)
    queue = 16 * cells
    assert 2 * solo + queue <= total <= 2 * solo + queue + 64 * 2 * 256 + 64 * 1024 + 8192


def test_batch_rejects_periodic_systems_and_empty_batches():
    good = P.make_params(65536, 0.70, 20.0, 16)
    with pytest.raises(E.ECError) as ei:
        P.batch_workspace_bytes([good, P.make_params(256, 0.70, 20.0, 1, dir_mode=E.EC_DIR_XY)])
    assert ei.value.status == E.EC_E_UNSUPPORTED
    lib = P.load_library()
    n = C.c_size_t()
    assert lib.ec_batch_workspace_bytes(C.byref(good), 0, C.byref(n)) == E.EC_E_INVALID
    with pytest.raises(E.ECError) as ei:  # one schedule per batch
        P.batch_workspace_bytes([good, P.make_params(65536, 0.70, 20.0, 16,
                                                     flags=E.EC_FLAG_PHASE_LAUNCHES)])
    assert ei.value.status == E.EC_E_UNSUPPORTED


def test_batch_init_rejects_small_workspace_without_touching_gpu():
    lib = P.load_library()
    ps = (E.Params * 2)(P.make_params(65536, 0.70, 20.0, 16), P.make_params(4096, 0.5, 20.0, 8))
    h = C.c_void_p()
    st = lib.ec_init_batch(ps, 2, C.c_void_p(0x1000), 16, None, C.byref(h))
    assert st == E.EC_E_NOMEM and not h.value


def test_gr_normalize_recovers_a_quadratic_contact_value():
    """Host-only normalisation (no GPU): counts built from a known g(R) near
    contact give back g at contact and z = 1 + (pi/2) sigma^2 rho g(sigma+)."""
    import math
    import numpy as np
    N, L, s, rmax, nb, samples = 4096, 80.0, 1.0, 1.5, 100, 10 ** 9
    rho = N / L ** 2
    e = s + (rmax - s) / nb * np.arange(nb + 1)
    R = 2 * (e[1:] ** 3 - e[:-1] ** 3) / (3 * (e[1:] ** 2 - e[:-1] ** 2))
    gtrue = 5.0 - 30.0 * (R - s) + 120.0 * (R - s) ** 2
    counts = np.round(gtrue * samples * N * rho * math.pi * (e[1:] ** 2 - e[:-1] ** 2))
    g, RR, gc, z = P.gr_normalize(N, L, s, rmax, counts.astype(np.uint64), samples, 0.05)
    np.testing.assert_allclose(RR, R, rtol=1e-12)  # e^3 differences cancel: ~1e-14
    np.testing.assert_allclose(g, gtrue, rtol=1e-9)
    assert abs(gc - 5.0) < 1e-8
    assert abs(z - (1 + math.pi / 2 * rho * gc)) < 1e-12


def test_gr_normalize_rejects_bad_arguments():
    import numpy as np
    c = np.ones(10, dtype=np.uint64)
    with pytest.raises(E.ECError):
        P.gr_normalize(4096, 80.0, 1.0, 0.9, c, 1)       # r_max <= sigma
    with pytest.raises(E.ECError):
        P.gr_normalize(4096, 80.0, 1.0, 1.5, c, 0)       # no samples
    with pytest.raises(E.ECError):
        P.gr_normalize(4096, 80.0, 1.0, 1.5, c, 1, 0.01)  # fewer than 3 bins in the fit


def test_psi_autocorrelation_matches_oracle():
    """ec_psi_autocorrelation against the oracle's eq. (tau) on an AR(1)
    series, the closed form cos(w dt) of a rotating phase, and rejections."""
    from oracle import delaunay as D
    rng = np.random.default_rng(4)
    n, a = 20000, 0.8
    noise = rng.normal(size=n) + 1j * rng.normal(size=n)
    psi = np.empty(n, dtype=np.complex128)
    psi[0] = noise[0]
    for i in range(1, n):
        psi[i] = a * psi[i - 1] + noise[i]
    c, tau = P.psi_autocorrelation(psi, 30)
    np.testing.assert_allclose(c, D.autocorrelation(psi, 30), rtol=1e-12, atol=1e-12)
    assert abs(tau - D.tau_fit(D.autocorrelation(psi, 30))) < 1e-9
    c2, _ = P.psi_autocorrelation(np.exp(0.3j * np.arange(500)), 10)
    np.testing.assert_allclose(c2, np.cos(0.3 * np.arange(11)), atol=1e-12)
    _, tau3 = P.psi_autocorrelation(rng.normal(size=1000) + 0j, 5)  # white noise: no decay time
    assert math.isnan(tau3)
    for bad in ((psi[:1], 1), (psi, 0), (psi[:10], 10), (np.zeros(10, complex), 3)):
        with pytest.raises(E.ECError) as ei:
            P.psi_autocorrelation(*bad)
        assert ei.value.status == E.EC_E_INVALID
