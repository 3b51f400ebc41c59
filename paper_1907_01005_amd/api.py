"""Thin Python binding over the C ABI: marshalling only.

Device memory comes from torch (the caller owns it); every computation runs
in the library's HIP kernels.  Names follow include/mfbcsr.h.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _native as N
from ._native import check, lib

FP64, FP64_MFMA, FP32_MFMA, FP32 = N.MFB_FP64, N.MFB_FP64_MFMA, N.MFB_FP32_MFMA, N.MFB_FP32
OP_H, OP_M = N.MFB_OP_H, N.MFB_OP_M
PREC_NAMES = {FP64: "fp64", FP64_MFMA: "fp64-mfma", FP32_MFMA: "fp32-mfma", FP32: "fp32"}


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream(stream) -> C.c_void_p:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _dev(t, name: str, nbytes: int, dtype=None) -> C.c_void_p:
    """Pointer of a contiguous GPU tensor of at least nbytes bytes (and the
    given dtype); a mismatch raises ValueError before the library is called,
    so no kernel ever reads past the end of a caller's buffer."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must live on a GPU, not {t.device}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: must be {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{name}: {have} bytes, needs at least {nbytes}")
    return C.c_void_p(t.data_ptr())


def _f64(t, name: str, count: int) -> C.c_void_p:
    import torch
    return _dev(t, name, 8 * max(int(count), 1), torch.float64)


class Mesh:
    """mfb_create_mesh: a box of Q_p cells grouped in Hilbert-ordered 2x2x2 batches."""

    def __init__(self, nx: int, ny: int, nz: int, L: Sequence[float], degree: int,
                 dirichlet: int = 0x3F, order: int = 0):
        d = N.MeshDesc(nx, ny, nz, float(L[0]), float(L[1]), float(L[2]), degree, dirichlet, order)
        h = C.c_void_p()
        check(lib().mfb_create_mesh(C.byref(d), C.byref(h)))
        self._h = h
        info = N.MeshInfo()
        check(lib().mfb_mesh_get_info(h, C.byref(info)))
        self.ndofs = info.ndofs
        self.ncells = info.ncells
        self.nbatches = info.nbatches
        self.degree = info.degree
        self.qp_per_cell = info.qp_per_cell
        self.nodes_per_batch = info.nodes_per_batch
        self.meta_bytes = info.meta_bytes
        self.cells_shape = (nx, ny, nz)
        self.L = tuple(float(x) for x in L)
        self.dirichlet = dirichlet
        self.curved = False
        self._meta = None

    @property
    def handle(self):
        return self._h

    def cells(self) -> np.ndarray:
        out = np.empty((self.ncells, 3), dtype=np.int32)
        check(lib().mfb_mesh_cells(self._h, _ptr(out, C.c_int32)))
        return out

    def qp_points(self) -> np.ndarray:
        out = np.empty((self.ncells, self.qp_per_cell, 3), dtype=np.float64)
        check(lib().mfb_mesh_qp_points(self._h, _ptr(out, C.c_double)))
        return out

    def node_points(self) -> np.ndarray:
        """mfb_mesh_node_points: node positions [ndofs][3]."""
        out = np.empty((self.ndofs, 3), dtype=np.float64)
        check(lib().mfb_mesh_node_points(self._h, _ptr(out, C.c_double)))
        return out

    def set_nodes(self, xyz: np.ndarray) -> None:
        """mfb_mesh_set_nodes: curved cells from node positions [ndofs][3]
        (global lexicographic order); before set_potential."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(self.ndofs, 3)
        check(lib().mfb_mesh_set_nodes(self._h, _ptr(x, C.c_double)))
        info = N.MeshInfo()
        check(lib().mfb_mesh_get_info(self._h, C.byref(info)))
        self.meta_bytes = info.meta_bytes
        self.curved = True

    def set_potential(self, v_qp: np.ndarray) -> None:
        v = np.ascontiguousarray(v_qp, dtype=np.float64).reshape(self.ncells, self.qp_per_cell)
        check(lib().mfb_mesh_set_potential(self._h, _ptr(v, C.c_double)))

    def bind(self, device="cuda", stream=None) -> None:
        import torch
        self._meta = torch.empty(max(self.meta_bytes, 256), dtype=torch.uint8, device=device)
        check(lib().mfb_mesh_bind(self._h, _dev(self._meta, "meta", self.meta_bytes),
                                  _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().mfb_destroy_mesh(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Layout:
    """mfb_create_bcsr_multivector: the BCSR pattern and device plan of X (and Y)."""

    def __init__(self, mesh: Mesh, centers: np.ndarray, radius, colblock_sizes=None, B: int = 8,
                 col_order: int = 0):
        self.mesh = mesh
        cen = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        rad = np.ascontiguousarray(np.atleast_1d(radius), dtype=np.float64)
        M = len(cen)
        sizes = None if colblock_sizes is None else \
            np.ascontiguousarray(colblock_sizes, dtype=np.int32)
        d = N.MvDesc(M, _ptr(cen, C.c_double), _ptr(rad, C.c_double), len(rad),
                     0 if sizes is None else len(sizes),
                     None if sizes is None else _ptr(sizes, C.c_int32), B, col_order)
        h = C.c_void_p()
        check(lib().mfb_create_bcsr_multivector(mesh.handle, C.byref(d), C.byref(h)))
        self.source = None
        self._keep = (cen, rad, sizes)
        self._finish(h)

    def _finish(self, h) -> None:
        self._h = h
        info = N.MvInfo()
        check(lib().mfb_mv_get_info(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in N.MvInfo._fields_}
        self.M = info.M
        self.nvalues = info.nvalues
        self.meta_bytes = info.meta_bytes
        self.work_bytes = info.work_bytes
        self._meta = None

    def closure(self) -> "Layout":
        """mfb_create_closure: the destination layout that holds H X and M X
        entirely.  It keeps this layout alive."""
        h = C.c_void_p()
        check(lib().mfb_create_closure(self._h, C.byref(h)))
        out = Layout.__new__(Layout)
        out.mesh = self.mesh
        out.source = self
        out._keep = None
        out._finish(h)
        return out

    def like(self) -> "Layout":
        """mfb_create_like: a second handle with this layout's pattern (it
        keeps this layout's mesh alive)."""
        h = C.c_void_p()
        check(lib().mfb_create_like(self._h, C.byref(h)))
        out = Layout.__new__(Layout)
        out.mesh = self.mesh
        out.source = self.source
        out._keep = self
        out._finish(h)
        return out

    def sizes(self):
        """mfb_mv_sizes: (value bytes of one multivector, device plan bytes)."""
        vb, mb = C.c_size_t(), C.c_size_t()
        check(lib().mfb_mv_sizes(self._h, C.byref(vb), C.byref(mb)))
        return vb.value, mb.value

    def set_global(self, node, orb, val, values, stream=None) -> None:
        """mfb_mv_set_global: COO triplets (global node, original orbital,
        value) into the device value tensor `values` of this layout."""
        node = np.ascontiguousarray(node, dtype=np.int64)
        orb = np.ascontiguousarray(orb, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        if not (len(node) == len(orb) == len(val)):
            raise ValueError("node, orb and val must have the same length")
        check(lib().mfb_mv_set_global(self._h, len(node), _ptr(node, C.c_int64),
                                      _ptr(orb, C.c_int32), _ptr(val, C.c_double),
                                      _f64(values, "values", self.nvalues), _stream(stream)))

    def get_global(self, values, stream=None):
        """mfb_mv_get_global: (node, orb, val) of every stored position."""
        node = np.empty(self.nvalues, dtype=np.int64)
        orb = np.empty(self.nvalues, dtype=np.int32)
        val = np.empty(self.nvalues, dtype=np.float64)
        check(lib().mfb_mv_get_global(self._h, _f64(values, "values", self.nvalues),
                                      _ptr(node, C.c_int64), _ptr(orb, C.c_int32),
                                      _ptr(val, C.c_double), _stream(stream)))
        return node, orb, val

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = N.Stats()
        check(lib().mfb_query_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in N.Stats._fields_}

    def pattern(self) -> dict:
        v = N.PatternView()
        check(lib().mfb_mv_pattern(self._h, C.byref(v)))
        nrb, ncb = self.info["nrowblocks"], self.info["ncolblocks"]
        nb = self.info["nblocks"]

        def cp(p, n):
            return np.ctypeslib.as_array(p, shape=(n,)).copy() if n > 0 else np.zeros(0, np.int64)
        return {
            "rowptr": cp(v.rowptr, nrb + 1),
            "colidx": cp(v.colidx, nb),
            "row_block_start": cp(v.row_block_start, nrb + 1),
            "col_block_start": cp(v.col_block_start, ncb + 1),
            "dof_perm": cp(v.dof_perm, self.mesh.ndofs),
            "col_perm": cp(v.col_perm, self.M),
            "block_offset": cp(v.block_offset, nb + 1),
            "batch_order": cp(v.batch_order, nrb),
        }

    def pack(self, node, orb, val) -> np.ndarray:
        node = np.ascontiguousarray(node, dtype=np.int64)
        orb = np.ascontiguousarray(orb, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        out = np.empty(self.nvalues, dtype=np.float64)
        check(lib().mfb_mv_pack(self._h, len(node), _ptr(node, C.c_int64), _ptr(orb, C.c_int32),
                                _ptr(val, C.c_double), _ptr(out, C.c_double)))
        return out

    def entry_coords(self):
        node = np.empty(self.nvalues, dtype=np.int64)
        orb = np.empty(self.nvalues, dtype=np.int32)
        check(lib().mfb_mv_entry_coords(self._h, _ptr(node, C.c_int64), _ptr(orb, C.c_int32)))
        return node, orb

    def bind(self, device="cuda", stream=None) -> None:
        import torch
        self._meta = torch.empty(max(self.meta_bytes, 256), dtype=torch.uint8, device=device)
        check(lib().mfb_mv_bind(self._h, _dev(self._meta, "meta", self.meta_bytes),
                                _stream(stream)))

    def new_values(self, device="cuda"):
        import torch
        return torch.zeros(max(self.nvalues, 1), dtype=torch.float64, device=device)

    def new_work(self, device="cuda"):
        import torch
        return torch.zeros(max(self.work_bytes, 256), dtype=torch.uint8, device=device)

    def close(self):
        if getattr(self, "_h", None):
            lib().mfb_destroy_mv(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_H(mesh: Mesh, layout: Layout, X, Y, prec: int = FP64, stream=None) -> None:
    """mfb_apply_H: Y = mask(H X) on the caller's stream (asynchronous)."""
    n = layout.nvalues
    check(lib().mfb_apply_H(mesh.handle, layout.handle, _f64(X, "X", n), _f64(Y, "Y", n),
                            int(prec), _stream(stream)))


def apply_H_acc(mesh: Mesh, layout: Layout, X, Y, prec: int = FP64, stream=None) -> None:
    """mfb_apply_H_acc: Y += mask(H X) (no zero fill) on the caller's stream."""
    n = layout.nvalues
    check(lib().mfb_apply_H_acc(mesh.handle, layout.handle, _f64(X, "X", n), _f64(Y, "Y", n),
                                int(prec), _stream(stream)))


def mv_zero(layout: Layout, Y, stream=None) -> None:
    """mfb_mv_zero: Y <- 0 on the layout's stored entries."""
    check(lib().mfb_mv_zero(layout.handle, _f64(Y, "Y", layout.nvalues), _stream(stream)))


def apply_H_tuned(mesh: Mesh, layout: Layout, X, Y, work, prec: int = FP64, kernel: int = 0,
                  grid: int = 0, stream=None) -> None:
    """mfb_apply_H_tuned: the same result through an explicit kernel configuration."""
    t = N.Tune(int(prec), int(kernel), int(grid), 0)
    n = layout.nvalues
    check(lib().mfb_apply_H_tuned(mesh.handle, layout.handle, _f64(X, "X", n), _f64(Y, "Y", n),
                                  C.byref(t), _dev(work, "work", layout.work_bytes),
                                  _stream(stream)))


def tmmult(layout: Layout, X, Y, S, trace, work, stream=None) -> None:
    """mfb_tmmult: S = X^T Y (M x M, library column order) and trace."""
    nx = layout.source.nvalues if layout.source is not None else layout.nvalues
    M = layout.M
    check(lib().mfb_tmmult(layout.handle, _f64(X, "X", nx), _f64(Y, "Y", layout.nvalues),
                           _f64(S, "S", M * M), _f64(trace, "trace", 1),
                           _dev(work, "work", layout.work_bytes), _stream(stream)))


def tmmult_tuned(layout: Layout, X, Y, S, trace, work, unit_steps: int = 0, long_steps: int = 0,
                 stream=None) -> None:
    """mfb_tmmult_tuned: the same S and trace with chosen row steps per wave."""
    nx = layout.source.nvalues if layout.source is not None else layout.nvalues
    M = layout.M
    t = N.TmTune(int(unit_steps), int(long_steps))
    check(lib().mfb_tmmult_tuned(layout.handle, _f64(X, "X", nx), _f64(Y, "Y", layout.nvalues),
                                 _f64(S, "S", M * M), _f64(trace, "trace", 1),
                                 _dev(work, "work", layout.work_bytes), C.byref(t), _stream(stream)))


def mv_update(layout: Layout, X, Y, S, S2, tau: float, stream=None) -> None:
    """mfb_mv_update: X <- X - tau (Y - X diag(S)/diag(S2)) on the stored entries."""
    n, M = layout.nvalues, layout.M
    check(lib().mfb_mv_update(layout.handle, _f64(X, "X", n), _f64(Y, "Y", n),
                              _f64(S, "S", M * M), _f64(S2, "S2", M * M), float(tau),
                              _stream(stream)))


def probe_fp64_fma(out, blocks: int, iters: int, stream=None) -> int:
    """mfb_probe_fp64_fma: blocks x 256 threads of 16 x iters fp64 FMAs; returns
    the flop count of the launch (the caller times it)."""
    check(lib().mfb_probe_fp64_fma(_f64(out, "out", 1), int(blocks), int(iters), _stream(stream)))
    return int(blocks) * 256 * 32 * int(iters)


def apply_op(mesh: Mesh, x: Layout, y: Layout, op: int, X, Y, prec: int = FP64,
             stream=None) -> None:
    """mfb_apply_op: Y = mask_y(op X), op = OP_H or OP_M; y is x or x.closure()."""
    check(lib().mfb_apply_op(mesh.handle, x.handle, y.handle, int(op), _f64(X, "X", x.nvalues),
                             _f64(Y, "Y", y.nvalues), int(prec), _stream(stream)))


def energy_work_bytes(M: int) -> int:
    """Scratch of mfb_energy: one double per 32x32 tile of the M x M matrices."""
    t = (int(M) + 31) // 32
    return 8 * t * t


def energy(M: int, Mbar, Hbar, E, work, stream=None) -> None:
    """mfb_energy: E = tr((2 I - Mbar) Hbar) into the one-element tensor E."""
    M = int(M)
    check(lib().mfb_energy(M, _f64(Mbar, "Mbar", M * M), _f64(Hbar, "Hbar", M * M),
                           _f64(E, "E", 1), _dev(work, "work", energy_work_bytes(M)),
                           _stream(stream)))


def mmult(a: Layout, c: Layout, A, B, alpha: float, beta: float, Cv, accumulate: bool = False,
          stream=None) -> None:
    """mfb_mmult (Alg. 7 with truncation): Cv = [Cv +] mask_c(A (alpha B + beta I))."""
    M = a.M
    check(lib().mfb_mmult(a.handle, c.handle, _f64(A, "A", a.nvalues), _f64(B, "B", M * M),
                          float(alpha), float(beta), _f64(Cv, "C", c.nvalues),
                          int(bool(accumulate)), _stream(stream)))


def mv_axpy(layout: Layout, alpha: float, X, Y, stream=None) -> None:
    """mfb_mv_axpy: Y += alpha X over the stored values."""
    n = layout.nvalues
    check(lib().mfb_mv_axpy(layout.handle, float(alpha), _f64(X, "X", n), _f64(Y, "Y", n),
                            _stream(stream)))


DOT_WORK_DOUBLES = 1024


def mv_dot(layout: Layout, X, Y, out, work, stream=None) -> None:
    """mfb_mv_dot: out = tr(X^T Y) over the stored entries (fixed order)."""
    n = layout.nvalues
    check(lib().mfb_mv_dot(layout.handle, _f64(X, "X", n), _f64(Y, "Y", n), _f64(out, "out", 1),
                           _f64(work, "work", DOT_WORK_DOUBLES), _stream(stream)))


def mv_scale_columns(layout: Layout, scale, X, stream=None) -> None:
    """mfb_mv_scale_columns: X[:, c] *= scale[c] (library column order)."""
    check(lib().mfb_mv_scale_columns(layout.handle, _f64(scale, "scale", layout.M),
                                     _f64(X, "X", layout.nvalues), _stream(stream)))
