"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments with the documented status codes (host-only calls, no GPU)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1907_01005_amd import Layout, MfbError, Mesh, lib
from paper_1907_01005_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mfbcsr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mfb_[A-Za-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    h = lib()
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(h, name), name
    assert set(names) == set(N.SIGNATURES), set(names) ^ set(N.SIGNATURES)


def test_mesh_errors():
    with pytest.raises(MfbError) as e:
        Mesh(3, 4, 4, (1, 1, 1), 2)
    assert e.value.code == N.MFB_EINVAL
    with pytest.raises(MfbError) as e:
        Mesh(4, 4, 4, (1, 1, 1), 7)
    assert e.value.code == N.MFB_EUNSUPPORTED
    with pytest.raises(MfbError) as e:
        Mesh(4, 4, 4, (1, 1, 1), 0)
    assert e.value.code == N.MFB_EUNSUPPORTED
    with pytest.raises(MfbError) as e:
        Mesh(4, 4, 4, (1, -1, 1), 2)
    assert e.value.code == N.MFB_EINVAL
    h = C.c_void_p()
    assert lib().mfb_create_mesh(None, C.byref(h)) == N.MFB_EINVAL
    assert b"null" in lib().mfb_last_error()


def test_layout_errors():
    m = Mesh(4, 4, 4, (4, 4, 4), 2)
    c = np.random.default_rng(0).random((10, 3)) * 4
    with pytest.raises(MfbError) as e:
        Layout(m, c, 1.5, colblock_sizes=[5, 4])      # does not sum to M
    assert e.value.code == N.MFB_EINVAL
    with pytest.raises(MfbError) as e:
        Layout(m, c, -1.0)
    assert e.value.code == N.MFB_EINVAL
    with pytest.raises(MfbError) as e:
        Layout(m, c, 1.5, colblock_sizes=[5, 0, 5])
    assert e.value.code == N.MFB_EINVAL
    lay = Layout(m, c, 1.5, colblock_sizes=[10])      # width 10 is fine
    assert lay.info["ncolblocks"] == 1


def test_layout_width_limit_and_pattern_errors():
    m = Mesh(4, 4, 4, (4, 4, 4), 2)
    c = np.random.default_rng(0).random((20, 3)) * 4
    with pytest.raises(MfbError) as e:
        Layout(m, c, 1.5, colblock_sizes=[20])
    assert e.value.code == N.MFB_EUNSUPPORTED
    lay = Layout(m, c, 1.5, colblock_sizes=[10, 10])
    node, orb = lay.entry_coords()
    stored = set(zip(node.tolist(), orb.tolist()))
    out = next((g, a) for g in range(m.ndofs) for a in range(20) if (g, a) not in stored)
    with pytest.raises(MfbError) as e:
        lay.pack([out[0]], [out[1]], [1.0])
    assert e.value.code == N.MFB_EPATTERN
    with pytest.raises(MfbError) as e:
        lay.pack([m.ndofs], [0], [1.0])
    assert e.value.code == N.MFB_EINVAL


def test_compute_calls_reject_unbound_handles():
    """Argument and state checks run before any HIP call."""
    m = Mesh(4, 4, 4, (4, 4, 4), 2)
    lay = Layout(m, np.full((8, 3), 2.0), 3.0)
    fake = C.c_void_p(4096)
    rc = lib().mfb_apply_H(m.handle, lay.handle, fake, C.c_void_p(8192), 0, None)
    assert rc == N.MFB_ESTATE
    rc = lib().mfb_apply_H(m.handle, lay.handle, fake, fake, 0, None)
    assert rc in (N.MFB_ESTATE, N.MFB_EINVAL)
    m2 = Mesh(4, 4, 4, (4, 4, 4), 2)
    rc = lib().mfb_apply_H(m2.handle, lay.handle, fake, C.c_void_p(8192), 0, None)
    assert rc == N.MFB_EPATTERN
    rc = lib().mfb_tmmult(lay.handle, fake, fake, fake, fake, fake, None)
    assert rc == N.MFB_ESTATE
    rc = lib().mfb_mesh_bind(m.handle, C.c_void_p(4096), None)
    assert rc == N.MFB_ESTATE                         # no potential yet
    rc = lib().mfb_mv_bind(lay.handle, C.c_void_p(4097), None)
    assert rc == N.MFB_EINVAL                         # misaligned


def test_closure_and_operator_argument_checks():
    """Closure layouts are destinations only; mfb_apply_op checks the pairing
    of source and destination; mfb_energy checks its size (no GPU call)."""
    m = Mesh(4, 4, 4, (4, 4, 4), 2)
    lay = Layout(m, np.full((8, 3), 1.0), 0.5)       # only the corner batch is stored
    clo = lay.closure()
    assert clo.nvalues > lay.nvalues and clo.info["apply_items"] == 0
    h = C.c_void_p()
    assert lib().mfb_create_closure(clo.handle, C.byref(h)) == N.MFB_EINVAL   # closure of a closure
    assert lib().mfb_create_closure(None, C.byref(h)) == N.MFB_EINVAL
    fake, fake2 = C.c_void_p(4096), C.c_void_p(8192)
    # a closure is never a source
    assert lib().mfb_apply_H(m.handle, clo.handle, fake, fake2, 0, None) == N.MFB_EINVAL
    assert lib().mfb_apply_op(m.handle, clo.handle, clo.handle, 0, fake, fake2, 0, None) == N.MFB_EINVAL
    assert lib().mfb_mv_update(clo.handle, fake, fake2, fake, fake, 0.1, None) == N.MFB_EINVAL
    # unbound handles, then a destination that is neither x nor its closure
    assert lib().mfb_apply_op(m.handle, lay.handle, clo.handle, 0, fake, fake2, 0, None) == N.MFB_ESTATE
    other = Layout(m, np.full((8, 3), 1.0), 0.5)
    rc = lib().mfb_apply_op(m.handle, lay.handle, other.handle, 0, fake, fake2, 0, None)
    assert rc in (N.MFB_ESTATE, N.MFB_EPATTERN)
    assert lib().mfb_energy(0, fake, fake, fake, fake, None) == N.MFB_EINVAL
    assert lib().mfb_energy(4, None, fake, fake, fake, None) == N.MFB_EINVAL
    assert lib().mfb_energy(4, fake, fake, fake, None, None) == N.MFB_EINVAL


def test_curved_mesh_errors():
    m = Mesh(4, 2, 2, (4.0, 2.0, 2.0), 2)
    x = m.node_points()
    with pytest.raises(MfbError) as e:
        m.set_nodes(np.where(np.arange(x.size).reshape(x.shape) == 7, np.nan, x))
    assert e.value.code == N.MFB_EINVAL
    with pytest.raises(MfbError) as e:
        m.set_nodes(np.zeros_like(x))                    # every cell collapsed
    assert e.value.code == N.MFB_EINVAL
    m.set_nodes(x + 0.01 * np.sin(x[:, ::-1]))
    m.set_potential(np.zeros((m.ncells, m.qp_per_cell)))
    with pytest.raises(MfbError) as e:
        m.set_nodes(x)                                   # after the potential
    assert e.value.code == N.MFB_ESTATE


def test_create_like_sizes_and_global_marshalling_errors():
    """mfb_create_like gives a handle with the same pattern (and the same
    sizes); mfb_mv_sizes reports 8 nvalues and the plan bytes; a triplet
    outside the pattern or out of range is refused by mfb_mv_set_global before
    the device buffer is touched (a fake device pointer is never used)."""
    m = Mesh(4, 4, 4, (4, 4, 4), 2)
    c = np.random.default_rng(3).random((12, 3)) * 4
    lay = Layout(m, c, 1.5, colblock_sizes=[5, 7])
    like = lay.like()
    assert like.info == lay.info
    assert like.pattern()["colidx"].tolist() == lay.pattern()["colidx"].tolist()
    vb, mb = lay.sizes()
    assert vb == 8 * lay.nvalues and mb == lay.meta_bytes
    assert like.sizes() == (vb, mb)
    clo = lay.closure()
    clo_like = clo.like()
    assert clo_like.info == clo.info and clo_like.nvalues > lay.nvalues
    # a destination like x is accepted by the pairing check of mfb_apply_op
    # (the call then stops at the unbound metadata, before any HIP call)
    fake, fake2 = C.c_void_p(4096), C.c_void_p(8192)
    assert lib().mfb_apply_op(m.handle, lay.handle, like.handle, 0, fake, fake2, 0, None) == \
        N.MFB_ESTATE
    other = Layout(m, c, 1.5, colblock_sizes=[5, 7])   # same inputs, another pattern id
    node, orb = lay.entry_coords()
    stored = set(zip(node.tolist(), orb.tolist()))
    out = next((g, a) for g in range(m.ndofs) for a in range(12) if (g, a) not in stored)
    n64 = np.array([out[0]], dtype=np.int64)
    o32 = np.array([out[1]], dtype=np.int32)
    v = np.array([1.0])
    P64, P32, PD = C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
    rc = lib().mfb_mv_set_global(lay.handle, 1, n64.ctypes.data_as(P64), o32.ctypes.data_as(P32),
                                 v.ctypes.data_as(PD), fake, None)
    assert rc == N.MFB_EPATTERN
    n64[0] = m.ndofs
    rc = lib().mfb_mv_set_global(lay.handle, 1, n64.ctypes.data_as(P64), o32.ctypes.data_as(P32),
                                 v.ctypes.data_as(PD), fake, None)
    assert rc == N.MFB_EINVAL
    assert lib().mfb_mv_set_global(lay.handle, 0, None, None, None, None, None) == N.MFB_EINVAL
    val = np.zeros(lay.nvalues)
    nd = np.zeros(lay.nvalues, dtype=np.int64)
    # node without orb
    rc = lib().mfb_mv_get_global(lay.handle, fake, nd.ctypes.data_as(P64), None,
                                 val.ctypes.data_as(PD), None)
    assert rc == N.MFB_EINVAL
    h = C.c_void_p()
    assert lib().mfb_create_like(None, C.byref(h)) == N.MFB_EINVAL
    vs, ms = C.c_size_t(), C.c_size_t()
    assert lib().mfb_mv_sizes(lay.handle, None, C.byref(ms)) == N.MFB_EINVAL
    del other
