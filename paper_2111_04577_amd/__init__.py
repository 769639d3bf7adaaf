"""drpf: dual-resolution phase-field step for AMD MI355X.

A thin ctypes binding over the C-ABI library ``libdrpf.so`` (declared in include/drpf.h):
argument marshalling only, every step of the path runs in the library's HIP kernels.
PyTorch provides device memory and the current stream. Importing this package does not
load the library; the first call that needs it does, and fails loudly if it is missing.
"""
from .binding import (  # noqa: F401
    DRPF_OK, DRPF_EINVAL, DRPF_EWORKSPACE, DRPF_EHIP, DRPF_ENONFINITE, DRPF_EUNSUPPORTED,
    LOCATIONS, BCS, OBSERVABLES, DrpfError, Params, State, Grid, DeviceState, lib, lib_path,
)
