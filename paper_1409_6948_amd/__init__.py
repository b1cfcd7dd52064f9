"""MI355X (gfx950) parallel event-chain Monte Carlo for 2D hard disks.

The hot path runs in the HIP library ``libec_hip.so`` behind the C ABI of
``include/ec.h``; :mod:`paper_1409_6948_amd.ec` is a thin ctypes binding with
the same names.  There is no CPU fallback: importing the binding without the
built library raises.
"""
from .ec import (EC_DIR_ISOTROPIC, EC_DIR_X, EC_DIR_XY, EC_FLAG_ONE_LAUNCH, EC_FLAG_PHASE_LAUNCHES,
                 EC_FLAG_CHECK_OVERLAP, EC_FLAG_REJECT, EC_FLAG_SCAN_SEARCH, EC_FLAG_STRIPES, EC_PREC_FP32_SCREEN, EC_PREC_FP64, EC_START_DISTINCT, EC_START_REPLACE, Batch, ECError, System, batch_workspace_bytes,
                 gr_normalize, lib_path, load_library, make_params, psi_autocorrelation,
                 workspace_bytes)

__all__ = ["EC_DIR_ISOTROPIC", "EC_DIR_X", "EC_DIR_XY", "EC_FLAG_ONE_LAUNCH", "EC_FLAG_PHASE_LAUNCHES",
           "EC_FLAG_CHECK_OVERLAP", "EC_FLAG_REJECT", "EC_FLAG_SCAN_SEARCH", "EC_FLAG_STRIPES", "EC_PREC_FP32_SCREEN", "EC_PREC_FP64", "EC_START_DISTINCT", "EC_START_REPLACE", "Batch", "ECError", "System",
           "batch_workspace_bytes", "gr_normalize", "lib_path", "load_library", "make_params",
           "psi_autocorrelation", "workspace_bytes"]
