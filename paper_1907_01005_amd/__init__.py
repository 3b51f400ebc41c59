"""MI355X-native matrix-free FE Hamiltonian on BCSR sparse multivectors.

Python side of libmfbcsr (include/mfbcsr.h): the C library plans meshes
and BCSR layouts on the host and runs the apply / overlap kernels on the GPU;
this package only marshals arguments and lends torch device memory.
"""

from .api import (  # noqa: F401
    FP32,
    FP32_MFMA,
    FP64,
    FP64_MFMA,
    OP_H,
    OP_M,
    PREC_NAMES,
    Layout,
    Mesh,
    apply_H,
    apply_H_acc,
    apply_H_tuned,
    apply_op,
    energy,
    mmult,
    mv_axpy,
    mv_dot,
    mv_scale_columns,
    mv_update,
    mv_zero,
    tmmult,
    tmmult_tuned,
)
from ._native import MfbError, lib  # noqa: F401
