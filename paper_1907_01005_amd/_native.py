"""ctypes declarations of the C ABI in include/mfbcsr.h (names kept 1:1)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfbcsr.so")

MFB_OK, MFB_EINVAL, MFB_EUNSUPPORTED, MFB_EPATTERN, MFB_ENOMEM, MFB_EHIP, MFB_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
MFB_FP64, MFB_FP64_MFMA, MFB_FP32_MFMA, MFB_FP32 = 0, 1, 2, 3
MFB_OP_H, MFB_OP_M = 0, 1
STATUS_NAMES = {0: "MFB_OK", -1: "MFB_EINVAL", -2: "MFB_EUNSUPPORTED", -3: "MFB_EPATTERN",
                -4: "MFB_ENOMEM", -5: "MFB_EHIP", -6: "MFB_ESTATE"}


class MeshDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double),
                ("degree", C.c_int32), ("dirichlet_faces", C.c_uint32), ("order", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("ndofs", C.c_int64), ("ncells", C.c_int64), ("nbatches", C.c_int32),
                ("degree", C.c_int32), ("qp_per_cell", C.c_int32),
                ("nodes_per_batch", C.c_int32), ("meta_bytes", C.c_size_t)]


class MvDesc(C.Structure):
    _fields_ = [("M", C.c_int32), ("centers", C.POINTER(C.c_double)),
                ("radius", C.POINTER(C.c_double)), ("radius_count", C.c_int32),
                ("ncolblocks", C.c_int32), ("colblock_sizes", C.POINTER(C.c_int32)),
                ("B", C.c_int32), ("col_order", C.c_int32)]


class MvInfo(C.Structure):
    _fields_ = [("M", C.c_int32), ("nrowblocks", C.c_int32), ("ncolblocks", C.c_int32),
                ("nblocks", C.c_int64), ("nvalues", C.c_int64), ("meta_bytes", C.c_size_t),
                ("work_bytes", C.c_size_t), ("apply_items", C.c_int64),
                ("apply_pairs", C.c_int64), ("apply_pairs_own", C.c_int64),
                ("tm_units", C.c_int64), ("s_pairs", C.c_int64), ("tm_tasks", C.c_int64),
                ("apply_items_own", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("rows_mean", C.c_double), ("rows_std", C.c_double),
                ("cols_mean", C.c_double), ("cols_std", C.c_double),
                ("blocks_per_row_mean", C.c_double),
                ("colblocks_per_cell_mean", C.c_double), ("colblocks_per_cell_std", C.c_double),
                ("colblocks_per_cell_sum", C.c_int64)]


class PatternView(C.Structure):
    _fields_ = [("rowptr", C.POINTER(C.c_int64)), ("colidx", C.POINTER(C.c_int32)),
                ("row_block_start", C.POINTER(C.c_int64)),
                ("col_block_start", C.POINTER(C.c_int32)),
                ("dof_perm", C.POINTER(C.c_int64)), ("col_perm", C.POINTER(C.c_int32)),
                ("block_offset", C.POINTER(C.c_int64)), ("batch_order", C.POINTER(C.c_int32))]


class Tune(C.Structure):
    _fields_ = [("prec", C.c_int32), ("kernel", C.c_int32), ("grid", C.c_int32),
                ("reserved", C.c_int32)]


class TmTune(C.Structure):
    _fields_ = [("unit_steps", C.c_int32), ("long_steps", C.c_int32),
                ("reserved", C.c_int32 * 2)]


VP = C.c_void_p
PI64 = C.POINTER(C.c_int64)
PI32 = C.POINTER(C.c_int32)
PD = C.POINTER(C.c_double)

SIGNATURES = {
    "mfb_last_error": (C.c_char_p, []),
    "mfb_create_mesh": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(VP)]),
    "mfb_mesh_get_info": (C.c_int, [VP, C.POINTER(MeshInfo)]),
    "mfb_mesh_cells": (C.c_int, [VP, PI32]),
    "mfb_mesh_qp_points": (C.c_int, [VP, PD]),
    "mfb_mesh_set_potential": (C.c_int, [VP, PD]),
    "mfb_mesh_set_nodes": (C.c_int, [VP, PD]),
    "mfb_mesh_node_points": (C.c_int, [VP, PD]),
    "mfb_mesh_bind": (C.c_int, [VP, VP, VP]),
    "mfb_destroy_mesh": (None, [VP]),
    "mfb_create_bcsr_multivector": (C.c_int, [VP, C.POINTER(MvDesc), C.POINTER(VP)]),
    "mfb_mv_get_info": (C.c_int, [VP, C.POINTER(MvInfo)]),
    "mfb_query_stats": (C.c_int, [VP, C.POINTER(Stats)]),
    "mfb_mv_pattern": (C.c_int, [VP, C.POINTER(PatternView)]),
    "mfb_mv_pack": (C.c_int, [VP, C.c_int64, PI64, PI32, PD, PD]),
    "mfb_mv_entry_coords": (C.c_int, [VP, PI64, PI32]),
    "mfb_create_like": (C.c_int, [VP, C.POINTER(VP)]),
    "mfb_mv_sizes": (C.c_int, [VP, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "mfb_mv_set_global": (C.c_int, [VP, C.c_int64, PI64, PI32, PD, VP, VP]),
    "mfb_mv_get_global": (C.c_int, [VP, VP, PI64, PI32, PD, VP]),
    "mfb_mv_bind": (C.c_int, [VP, VP, VP]),
    "mfb_destroy_mv": (None, [VP]),
    "mfb_apply_H": (C.c_int, [VP, VP, VP, VP, C.c_int, VP]),
    "mfb_apply_H_acc": (C.c_int, [VP, VP, VP, VP, C.c_int, VP]),
    "mfb_mv_zero": (C.c_int, [VP, VP, VP]),
    "mfb_apply_H_tuned": (C.c_int, [VP, VP, VP, VP, C.POINTER(Tune), VP, VP]),
    "mfb_tmmult": (C.c_int, [VP, VP, VP, VP, VP, VP, VP]),
    "mfb_tmmult_tuned": (C.c_int, [VP, VP, VP, VP, VP, VP, C.POINTER(TmTune), VP]),
    "mfb_tmmult_noalloc": (C.c_int, [VP, VP, VP, VP, VP, VP]),
    "mfb_mv_update": (C.c_int, [VP, VP, VP, VP, VP, C.c_double, VP]),
    "mfb_probe_fp64_fma": (C.c_int, [VP, C.c_int64, C.c_int32, VP]),
    "mfb_create_closure": (C.c_int, [VP, C.POINTER(VP)]),
    "mfb_apply_op": (C.c_int, [VP, VP, VP, C.c_int, VP, VP, C.c_int, VP]),
    "mfb_energy": (C.c_int, [C.c_int32, VP, VP, VP, VP, VP]),
    "mfb_mmult": (C.c_int, [VP, VP, VP, VP, C.c_double, C.c_double, VP, C.c_int, VP]),
    "mfb_mv_axpy": (C.c_int, [VP, C.c_double, VP, VP, VP]),
    "mfb_mv_dot": (C.c_int, [VP, VP, VP, VP, VP, VP]),
    "mfb_mv_scale_columns": (C.c_int, [VP, VP, VP, VP]),
}


class MfbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libmfbcsr.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1907_01005_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(rc: int) -> None:
    if rc != MFB_OK:
        msg = lib().mfb_last_error().decode(errors="replace")
        raise MfbError(rc, msg)
