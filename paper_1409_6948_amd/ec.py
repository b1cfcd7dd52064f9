"""ctypes binding of the C ABI in include/ec.h (argument marshalling only).

Every step of the sweep runs in the HIP kernels of libec_hip.so.  PyTorch is
used for the device workspace and the stream, nothing else.  If the library
is missing, loading fails loudly; there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libec_hip.so"

EC_OK, EC_E_INVALID, EC_E_OVERLAP, EC_E_HIP, EC_E_NOMEM, EC_E_STATE, EC_E_UNSUPPORTED = range(7)
EC_DIR_XY, EC_DIR_ISOTROPIC, EC_DIR_X = 0, 1, 2
EC_PREC_FP64, EC_PREC_FP32_SCREEN = 0, 1
EC_START_REPLACE, EC_START_DISTINCT = 0, 1
EC_FLAG_SCAN_SEARCH = 1
EC_FLAG_PHASE_LAUNCHES = 2
EC_FLAG_ONE_LAUNCH = 4
EC_FLAG_REJECT = 8
EC_FLAG_CHECK_OVERLAP = 16
EC_FLAG_STRIPES = 32
EC_SCHEDULE_PHASE_LAUNCHES, EC_SCHEDULE_ONE_LAUNCH, EC_SCHEDULE_READY_QUEUE = 0, 1, 2
SCHEDULE_NAMES = ("phase-launches", "one-launch", "ready-queue")
EC_ABI_VERSION = 1
COUNT_NAMES = ("lifts", "frozen", "walls", "chains", "pseudo")

# every symbol declared in include/ec.h
EXPORTED = ("ec_workspace_bytes", "ec_init_system", "ec_sweep", "ec_measure_pressure",
            "ec_reset_tallies", "ec_get_positions", "ec_set_positions", "ec_get_digests",
            "ec_get_cell_tallies", "ec_get_cell_digests", "ec_get_sweep_count",
            "ec_set_timing", "ec_get_timing", "ec_get_rebin_timing", "ec_set_dep_wait_limit", "ec_destroy", "ec_status_string",
            "ec_last_error", "ec_batch_workspace_bytes", "ec_init_batch", "ec_sweep_batch",
            "ec_batch_system", "ec_batch_set_graph", "ec_batch_set_cells_per_block",
            "ec_batch_autotune", "ec_batch_set_schedule", "ec_batch_last_error", "ec_destroy_batch", "ec_measure_psi6",
            "ec_measure_psi6_delaunay", "ec_psi_autocorrelation",
            "ec_gr_accumulate", "ec_gr_counts", "ec_gr_reset", "ec_gr_normalize",
            "ec_sweep_static")


class ECError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("flags", C.c_uint32), ("n_disks", C.c_int64),
                ("sigma", C.c_double), ("eta", C.c_double), ("ell", C.c_double),
                ("cells_per_side", C.c_int32), ("chains_per_cell", C.c_int32),
                ("dir_mode", C.c_int32), ("precision", C.c_int32), ("start_mode", C.c_int32),
                ("cells_per_block", C.c_int32), ("screen_margin", C.c_double),
                ("seed", C.c_uint64), ("system", C.c_uint32), ("reserved", C.c_uint32)]


_lib = None


def lib_path():
    return os.path.join(HERE, _LIB_NAME)


def load_library():
    """Load libec_hip.so (built by build.py); raises if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1409_6948_amd/build.py")
    L = C.CDLL(path)
    P = C.POINTER(Params)
    vp, dp, u64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)
    sigs = {
        "ec_workspace_bytes": [P, C.POINTER(C.c_size_t)],
        "ec_init_system": [P, vp, C.c_size_t, vp, C.POINTER(vp)],
        "ec_sweep": [vp, C.c_int64],
        "ec_measure_pressure": [vp, dp, dp, u64p],
        "ec_measure_psi6": [vp, C.c_double, dp, dp, dp, dp],
        "ec_measure_psi6_delaunay": [vp, C.c_double, dp, dp, dp, dp, C.POINTER(C.c_int32)],
        "ec_psi_autocorrelation": [dp, dp, C.c_int64, C.c_int32, dp, dp],
        "ec_gr_accumulate": [vp, C.c_double, C.c_int32],
        "ec_gr_counts": [vp, u64p, C.POINTER(C.c_int64), u64p],
        "ec_gr_reset": [vp],
        "ec_gr_normalize": [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int32, u64p,
                            C.c_int64, C.c_double, dp, dp, dp, dp],
        "ec_reset_tallies": [vp],
        "ec_get_positions": [vp, dp, dp, C.c_int64],
        "ec_set_positions": [vp, dp, dp, C.c_int64],
        "ec_get_digests": [vp, u64p, C.c_int64],
        "ec_get_cell_tallies": [vp, dp, u64p],
        "ec_get_cell_digests": [vp, u64p],
        "ec_get_sweep_count": [vp, C.POINTER(C.c_int64)],
        "ec_set_timing": [vp, C.c_int32],
        "ec_get_timing": [vp, dp, C.POINTER(C.c_int64)],
        "ec_get_rebin_timing": [vp, dp, dp, C.POINTER(C.c_int64)],
        "ec_set_dep_wait_limit": [vp, C.c_double],
        "ec_destroy": [vp],
        "ec_batch_workspace_bytes": [P, C.c_int32, C.POINTER(C.c_size_t)],
        "ec_init_batch": [P, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)],
        "ec_sweep_batch": [vp, C.c_int64],
        "ec_batch_system": [vp, C.c_int32, C.POINTER(vp)],
        "ec_batch_set_graph": [vp, C.c_int32],
        "ec_batch_set_cells_per_block": [vp, C.c_int32],
        "ec_batch_autotune": [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp],
        "ec_batch_set_schedule": [vp, C.c_int32],
        "ec_destroy_batch": [vp],
        "ec_sweep_static": [P, vp, vp, C.c_int64, C.c_int64, vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.ec_status_string.argtypes = [C.c_int]
    L.ec_status_string.restype = C.c_char_p
    L.ec_last_error.argtypes = [vp]
    L.ec_last_error.restype = C.c_char_p
    L.ec_batch_last_error.argtypes = [vp]
    L.ec_batch_last_error.restype = C.c_char_p
    _lib = L
    return L


def make_params(n, eta, ell, cells, dir_mode=EC_DIR_ISOTROPIC, seed=1, sigma=1.0,
                chains_per_cell=0, precision=EC_PREC_FP64, start_mode=EC_START_REPLACE,
                cells_per_block=0, screen_margin=0.0, system=0, flags=0):
    return Params(EC_ABI_VERSION, int(flags), int(n), float(sigma), float(eta), float(ell), int(cells),
                  int(chains_per_cell), int(dir_mode), int(precision), int(start_mode),
                  int(cells_per_block), float(screen_margin), int(seed), int(system), 0)


def _check(status, handle=None, what="", batch=False):
    if status != EC_OK:
        L = load_library()
        msg = L.ec_status_string(status).decode()
        if handle:
            extra = (L.ec_batch_last_error if batch else L.ec_last_error)(handle).decode()
            if extra:
                msg += ": " + extra
        raise ECError(status, f"{what}: {msg}")


def workspace_bytes(p):
    n = C.c_size_t()
    _check(load_library().ec_workspace_bytes(C.byref(p), C.byref(n)), what="ec_workspace_bytes")
    return n.value


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class System:
    """One hard-disk system on the current GPU.

    The workspace is a torch uint8 tensor on the device; the stream is torch's
    current stream unless one is given.
    """

    def __init__(self, p, device="cuda", stream=None, _view=None):
        self._lib = load_library()
        self.p = p
        self.n = int(p.n_disks)
        if _view is not None:  # a system of a Batch (the batch owns handle and memory)
            self.h, self.stream, self.workspace, self._owned = _view[0], _view[1], None, False
            return
        import torch
        self._owned = True
        self.workspace = torch.empty(workspace_bytes(p), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        h = C.c_void_p()
        st = self._lib.ec_init_system(C.byref(p), C.c_void_p(self.workspace.data_ptr()),
                                      self.workspace.numel(), C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h))
        _check(st, None, "ec_init_system")
        self.h = h

    def sweep(self, n_sweeps=1):
        _check(self._lib.ec_sweep(self.h, int(n_sweeps)), self.h, "ec_sweep")

    def measure_pressure(self):
        z, bp = C.c_double(), C.c_double()
        cnt = np.zeros(5, dtype=np.uint64)
        _check(self._lib.ec_measure_pressure(self.h, C.byref(z), C.byref(bp),
                                             cnt.ctypes.data_as(C.POINTER(C.c_uint64))),
               self.h, "ec_measure_pressure")
        return z.value, bp.value, dict(zip(COUNT_NAMES, (int(v) for v in cnt)))

    def measure_psi6(self, r_cut=0.0, per_disk=False):
        """Hexatic order parameter with cutoff neighbours: (Psi, mean neighbour
        count[, per-disk Psi_k as a complex array])."""
        re, im, nb = C.c_double(), C.c_double(), C.c_double()
        per = np.zeros(2 * self.n, dtype=np.float64) if per_disk else None
        _check(self._lib.ec_measure_psi6(self.h, float(r_cut), C.byref(re), C.byref(im), C.byref(nb),
                                         _dptr(per) if per_disk else None),
               self.h, "ec_measure_psi6")
        out = (complex(re.value, im.value), nb.value)
        return out + (per[0::2] + 1j * per[1::2],) if per_disk else out

    def measure_psi6_delaunay(self, r_search=0.0, per_disk=False):
        """Hexatic order parameter with Delaunay neighbours: (Psi, mean neighbour
        count[, per-disk Psi_k as a complex array, per-disk neighbour counts])."""
        re, im, nb = C.c_double(), C.c_double(), C.c_double()
        per = np.zeros(2 * self.n, dtype=np.float64) if per_disk else None
        cnt = np.zeros(self.n, dtype=np.int32) if per_disk else None
        _check(self._lib.ec_measure_psi6_delaunay(
            self.h, float(r_search), C.byref(re), C.byref(im), C.byref(nb),
            _dptr(per) if per_disk else None,
            cnt.ctypes.data_as(C.POINTER(C.c_int32)) if per_disk else None),
            self.h, "ec_measure_psi6_delaunay")
        out = (complex(re.value, im.value), nb.value)
        return out + (per[0::2] + 1j * per[1::2], cnt) if per_disk else out

    def gr_accumulate(self, r_max, n_bins):
        """Add the current configuration's ordered-pair counts to the histogram."""
        self._gr = (float(r_max), int(n_bins))
        _check(self._lib.ec_gr_accumulate(self.h, float(r_max), int(n_bins)), self.h,
               "ec_gr_accumulate")

    def gr_counts(self):
        """(counts[n_bins], configurations added, pairs closer than sigma)."""
        n_bins = self._gr[1]
        counts = np.zeros(n_bins, dtype=np.uint64)
        samples, ov = C.c_int64(), C.c_uint64()
        _check(self._lib.ec_gr_counts(self.h, counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                                      C.byref(samples), C.byref(ov)), self.h, "ec_gr_counts")
        return counts, samples.value, ov.value

    def gr_reset(self):
        _check(self._lib.ec_gr_reset(self.h), self.h, "ec_gr_reset")

    def reset_tallies(self):
        _check(self._lib.ec_reset_tallies(self.h), self.h, "ec_reset_tallies")

    def get_positions(self):
        x = np.empty(self.n, dtype=np.float64)
        y = np.empty(self.n, dtype=np.float64)
        _check(self._lib.ec_get_positions(self.h, _dptr(x), _dptr(y), self.n), self.h,
               "ec_get_positions")
        return x, y

    def set_positions(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        _check(self._lib.ec_set_positions(self.h, _dptr(x), _dptr(y), self.n), self.h,
               "ec_set_positions")

    def get_digests(self, n):
        out = np.zeros(int(n), dtype=np.uint64)
        _check(self._lib.ec_get_digests(self.h, out.ctypes.data_as(C.POINTER(C.c_uint64)), int(n)),
               self.h, "ec_get_digests")
        return out

    def get_cell_tallies(self):
        nc = int(self.p.cells_per_side) ** 2
        delta = np.zeros(nc, dtype=np.float64)
        cnt = np.zeros((nc, 5), dtype=np.uint64)
        _check(self._lib.ec_get_cell_tallies(self.h, _dptr(delta),
                                             cnt.ctypes.data_as(C.POINTER(C.c_uint64))),
               self.h, "ec_get_cell_tallies")
        return delta, cnt

    def get_cell_digests(self):
        nc = int(self.p.cells_per_side) ** 2
        out = np.zeros(nc, dtype=np.uint64)
        _check(self._lib.ec_get_cell_digests(self.h, out.ctypes.data_as(C.POINTER(C.c_uint64))),
               self.h, "ec_get_cell_digests")
        return out

    def set_dep_wait_limit(self, seconds):
        """Limit of one cell's wait for its earlier-phase neighbours (one-launch sweep)."""
        _check(self._lib.ec_set_dep_wait_limit(self.h, float(seconds)), self.h, "ec_set_dep_wait_limit")

    def set_timing(self, on):
        _check(self._lib.ec_set_timing(self.h, 1 if on else 0), self.h, "ec_set_timing")

    def get_timing(self):
        ms, n = C.c_double(), C.c_int64()
        _check(self._lib.ec_get_timing(self.h, C.byref(ms), C.byref(n)), self.h, "ec_get_timing")
        return ms.value, n.value

    def get_rebin_timing(self):
        """(count kernel ms, scatter kernel ms, sweeps) summed over the timed sweeps."""
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        _check(self._lib.ec_get_rebin_timing(self.h, C.byref(a), C.byref(b), C.byref(n)), self.h,
               "ec_get_rebin_timing")
        return a.value, b.value, n.value

    def sweep_count(self):
        v = C.c_int64()
        _check(self._lib.ec_get_sweep_count(self.h, C.byref(v)), self.h, "ec_get_sweep_count")
        return v.value

    def close(self):
        if getattr(self, "h", None) and getattr(self, "_owned", True):
            self._lib.ec_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(ps):
    arr = (Params * len(ps))(*ps)
    n = C.c_size_t()
    _check(load_library().ec_batch_workspace_bytes(arr, len(ps), C.byref(n)),
           what="ec_batch_workspace_bytes")
    return n.value


class Batch:
    """Several walled systems advanced by shared launches (one per sweep step).

    systems[i] is a System view for per-system queries; the batch owns the
    workspace (torch uint8 tensor) and, unless given, a stream of its own (a
    HIP graph cannot be captured on the null stream).
    """

    def __init__(self, ps, device="cuda", stream=None):
        import torch
        self._lib = load_library()
        self.ps = list(ps)
        self._arr = (Params * len(self.ps))(*self.ps)
        self.workspace = torch.empty(batch_workspace_bytes(self.ps), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.workspace.device)
        h = C.c_void_p()
        _check(self._lib.ec_init_batch(self._arr, len(self.ps), C.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h)), None, "ec_init_batch")
        self.h = h
        self.systems = []
        for i, p in enumerate(self.ps):
            v = C.c_void_p()
            _check(self._lib.ec_batch_system(self.h, i, C.byref(v)), self.h, "ec_batch_system", True)
            self.systems.append(System(p, _view=(v, self.stream)))

    def sweep(self, n_sweeps=1):
        _check(self._lib.ec_sweep_batch(self.h, int(n_sweeps)), self.h, "ec_sweep_batch", True)

    def set_graph(self, on):
        _check(self._lib.ec_batch_set_graph(self.h, 1 if on else 0), self.h, "ec_batch_set_graph", True)

    def set_cells_per_block(self, cpb):
        _check(self._lib.ec_batch_set_cells_per_block(self.h, int(cpb)), self.h,
               "ec_batch_set_cells_per_block", True)

    def set_schedule(self, schedule):
        """EC_SCHEDULE_* or its name ('phase-launches', 'one-launch', 'ready-queue')."""
        if isinstance(schedule, str):
            schedule = SCHEDULE_NAMES.index(schedule)
        _check(self._lib.ec_batch_set_schedule(self.h, int(schedule)), self.h,
               "ec_batch_set_schedule", True)

    def autotune(self, trial_sweeps=2):
        """Time every schedule and cells-per-workgroup choice from a snapshot and
        keep the fastest: returns (schedule name, cells per workgroup,
        {(schedule name, cells): ms})"""
        sched, cpb = C.c_int32(), C.c_int32()
        ms = (C.c_double * 9)()
        _check(self._lib.ec_batch_autotune(self.h, int(trial_sweeps), C.byref(sched), C.byref(cpb), ms),
               self.h, "ec_batch_autotune", True)
        trials = {f"{SCHEDULE_NAMES[k // 3]}/{(1, 2, 4)[k % 3]}": ms[k] for k in range(9)}
        return SCHEDULE_NAMES[sched.value], cpb.value, trials

    def close(self):
        if getattr(self, "h", None):
            for s in getattr(self, "systems", []):
                s.h = None
            self._lib.ec_destroy_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep_static(p, x, y, first_sweep, n_sweeps, digests=None, err=None, stream=None):
    """ec_sweep_static: sweeps of device-resident positions (torch float64
    tensors on the GPU, advanced in place) with the library's static buffer;
    digests (torch int64[n_sweeps]) and err (torch int32[1]) are optional
    device outputs.  Enqueued on `stream` (default: torch's current stream)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    for t in (x, y):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != p.n_disks:
            raise ValueError("x and y must be contiguous float64 CUDA tensors of n_disks elements")
    _check(load_library().ec_sweep_static(
        C.byref(p), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), int(first_sweep),
        int(n_sweeps), C.c_void_p(digests.data_ptr()) if digests is not None else None,
        C.c_void_p(err.data_ptr()) if err is not None else None, C.c_void_p(st.cuda_stream)),
        what="ec_sweep_static")


def psi_autocorrelation(psi, max_lag):
    """C(dt) for dt = 0..max_lag and the fitted decay time tau of a complex
    time series of Psi (ec_psi_autocorrelation, eq. tau)."""
    psi = np.asarray(psi, dtype=np.complex128)
    re = np.ascontiguousarray(psi.real)
    im = np.ascontiguousarray(psi.imag)
    c = np.zeros(int(max_lag) + 1)
    tau = C.c_double()
    _check(load_library().ec_psi_autocorrelation(_dptr(re), _dptr(im), len(psi), int(max_lag),
                                                 _dptr(c), C.byref(tau)),
           what="ec_psi_autocorrelation")
    return c, tau.value


def gr_normalize(n_disks, box, sigma, r_max, counts, samples, fit_width=0.05):
    """Host-only normalisation of pair counts (ec_gr_normalize): returns
    (g[n_bins], R[n_bins], g at contact, z = beta P / rho)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    n = len(counts)
    g = np.zeros(n)
    R = np.zeros(n)
    gc, z = C.c_double(), C.c_double()
    _check(load_library().ec_gr_normalize(int(n_disks), float(box), float(sigma), float(r_max), n,
                                          counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                                          int(samples), float(fit_width), _dptr(g), _dptr(R),
                                          C.byref(gc), C.byref(z)), what="ec_gr_normalize")
    return g, R, gc.value, z.value
