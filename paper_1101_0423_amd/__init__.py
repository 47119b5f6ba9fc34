"""MI355X (gfx950) domain-wall fermion CG solver: Python binding of libdwf.

Argument marshalling only: every step of the operator and the solver runs in
the HIP kernels of ``libdwf.so`` (built by ``paper_1101_0423_amd/build.py``).
Importing the package loads the library and raises if it has not been built.
"""
from .binding import (  # noqa: F401
    DWF_EBUSY, DWF_EDEVICE, DWF_EINVAL, DWF_ENOCONV, DWF_ENOMEM, DWF_ENOTFOUND, DWF_OK, DWF_PENDING,
    OP_C, OP_CCDAG, OP_CDAG, OP_D, OP_DDAG, OP_DW, OP_HOP_EO, OP_HOP_OE, OP_M5, OP_M5T,
    PREC_FP16, PREC_FP32, PREC_FP64, SYSTEM_CCDAG, SYSTEM_D, Context, DwfError, SolveParams, SolveStats,
    ServerStats, LINKS_12, LINKS_18, LINKS_AUTO, SU3_TOL,
    check_device_spinors, check_host_spinors, default_params, odwf_weights, gauge_shape, gauge_su3_deviation, lib, lib_path,
    poll, server_stats, spinor_shape, stream_copy, EXPORTED,
)
