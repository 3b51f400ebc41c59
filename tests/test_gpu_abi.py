"""GPU tests of the boundary itself: the global-coordinate marshalling calls,
a layout created like another, and refused calls that leave every device
buffer as it was (arguments are checked before anything is enqueued)."""

import ctypes as C

import numpy as np
import pytest

import synth
from helpers import device_problem, gpu_available, say
from oracle.workload import OracleProblem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.fail("GPU tests need a visible GPU (run with -m 'not gpu' on CPU)")


def _small(degree=2, bend=0.0):
    ms = synth.MeshSpec(8, 6, 4, (8.0, 6.0, 4.0), degree, bend=bend)
    wl = synth.custom_workload(ms, 29, 2.2, 11, potential="wells")
    wl.colblock_sizes = np.asarray([8, 5, 12, 4], dtype=np.int32)
    return wl


def test_set_get_global_round_trip_and_like_layout():
    import torch
    from paper_1907_01005_amd import FP64, OP_H, apply_op
    wl = _small()
    say("set/get global, like layout")
    op = OracleProblem(wl, values="generic", value_seed=21)
    dp = device_problem(wl)
    dp.layout.set_global(op.node, op.orb, op.val, dp.X)
    torch.cuda.synchronize()
    packed = dp.layout.pack(op.node, op.orb, op.val)
    assert np.array_equal(dp.X.cpu().numpy()[:dp.nvalues], packed)
    node, orb, val = dp.layout.get_global(dp.X)
    n2, o2 = dp.layout.entry_coords()
    assert np.array_equal(node, n2) and np.array_equal(orb, o2)
    assert np.array_equal(val, packed)
    # every triplet comes back at its own coordinates
    got = dict(zip(zip(node.tolist(), orb.tolist()), val.tolist()))
    for g, a, v in zip(op.node.tolist(), op.orb.tolist(), op.val.tolist()):
        assert got[(g, a)] == v
    # Y through a destination layout created like X's equals mfb_apply_H's Y
    dp.apply(FP64)
    torch.cuda.synchronize()
    Y_ref = dp.Y.clone()
    like = dp.layout.like()
    like.bind()
    Y2 = like.new_values()
    apply_op(dp.mesh, dp.layout, like, OP_H, dp.X, Y2, FP64)
    torch.cuda.synchronize()
    scale = Y_ref.abs().max().item()
    assert (Y2 - Y_ref).abs().max().item() <= 1e-14 * scale


def test_refused_calls_leave_buffers_untouched():
    """A refused call returns its status and enqueues nothing: Y keeps the
    sentinel it held (the apply's first kernel would otherwise zero it)."""
    import torch
    import paper_1907_01005_amd._native as N
    from paper_1907_01005_amd import FP64, MfbError, OP_H, apply_H, apply_H_tuned, apply_op
    lib = N.lib()
    for bend in (0.0, 0.3):
        wl = _small(bend=bend)
        say(f"refused calls, bend {bend}")
        op = OracleProblem(wl)
        dp = device_problem(wl)
        dp.set_X_coo(op.node, op.orb, op.val)
        sentinel = torch.full_like(dp.Y, 7.25)
        dp.Y.copy_(sentinel)
        torch.cuda.synchronize()
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        X, Y = C.c_void_p(dp.X.data_ptr()), C.c_void_p(dp.Y.data_ptr())
        for prec in (-1, 4, 9):
            assert lib.mfb_apply_H(dp.mesh.handle, dp.layout.handle, X, Y, prec, st) == N.MFB_EINVAL
        assert lib.mfb_apply_op(dp.mesh.handle, dp.layout.handle, dp.layout.handle, 5, X, Y, 0,
                                st) == N.MFB_EINVAL
        assert lib.mfb_apply_op(dp.mesh.handle, dp.layout.handle, dp.layout.handle, 0, X, Y, 7,
                                st) == N.MFB_EINVAL
        for kernel, grid in ((10, 0), (-1, 0), (0, 3), (0, 128)):
            with pytest.raises(MfbError) as e:
                apply_H_tuned(dp.mesh, dp.layout, dp.X, dp.Y, dp.work, FP64, kernel, grid)
            assert e.value.code == N.MFB_EINVAL
        if bend:
            for kernel in (1, 3, 4, 5, 6, 8, 9):
                with pytest.raises(MfbError) as e:
                    apply_H_tuned(dp.mesh, dp.layout, dp.X, dp.Y, dp.work, FP64, kernel, 0)
                assert e.value.code == N.MFB_EUNSUPPORTED
        # a destination of another pattern, a too-short or wrong-typed tensor
        other = dp.layout.__class__(dp.mesh, wl.centres, wl.radius, wl.colblock_sizes)
        other.bind()
        with pytest.raises(MfbError) as e:
            apply_op(dp.mesh, dp.layout, other, OP_H, dp.X, dp.Y[:other.nvalues], FP64)
        assert e.value.code == N.MFB_EPATTERN
        with pytest.raises(ValueError):
            apply_H(dp.mesh, dp.layout, dp.X, dp.Y[:dp.nvalues - 1], FP64)
        with pytest.raises(ValueError):
            apply_H(dp.mesh, dp.layout, dp.X.float(), dp.Y, FP64)
        with pytest.raises(ValueError):
            apply_H(dp.mesh, dp.layout, dp.X, dp.Y.cpu(), FP64)
        torch.cuda.synchronize()
        assert torch.equal(dp.Y, sentinel)
        # and an accepted call does overwrite it
        apply_H(dp.mesh, dp.layout, dp.X, dp.Y, FP64)
        torch.cuda.synchronize()
        assert not torch.equal(dp.Y, sentinel)


def test_fp64_fma_probe():
    """The measurement probe runs, leaves its output untouched (the chains
    never reach the sentinel) and reports a rate between a tenth of the
    rated fp64 peak and the peak itself; bad arguments are refused."""
    import torch
    from paper_1907_01005_amd import _native as N
    from paper_1907_01005_amd import MfbError
    from paper_1907_01005_amd.api import probe_fp64_fma
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    probe_fp64_fma(out, 8 * cus, 2000)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    flops = probe_fp64_fma(out, 8 * cus, 20000)
    b.record()
    torch.cuda.synchronize()
    tfs = flops / (a.elapsed_time(b) * 1e-3) / 1e12
    say(f"fp64 FMA probe: {tfs:.1f} TFLOP/s on {cus} CUs")
    assert out.item() == 0.0
    assert 0.1 * 78.6 * cus / 256 < tfs <= 1.02 * 78.6 * cus / 256
    for blocks, iters in ((0, 10), (4, 0)):
        with pytest.raises(MfbError) as e:
            probe_fp64_fma(out, blocks, iters)
        assert e.value.code == N.MFB_EINVAL
