"""The allocation-free overlap entry point (mfb_tmmult_noalloc) against
mfb_tmmult with a caller workspace, through the C ABI: two calls in a row,
the second on a smaller layout (the shared scratch keeps the first call's
partial products), each bitwise equal to the workspace form's S and trace.
A layout whose workspace exceeds the fixed scratch is refused before
anything is enqueued."""

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


def _problem(cells, degree, M, radius, seed, sizes):
    ms = synth.MeshSpec(*cells, tuple(float(c) for c in cells), degree)
    wl = synth.custom_workload(ms, M, radius, seed, potential="wells")
    wl.colblock_sizes = np.asarray(sizes, dtype=np.int32)
    op = OracleProblem(wl, values="generic", value_seed=seed)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    return dp


def test_tmmult_noalloc_matches_workspace_form():
    import torch
    import paper_1907_01005_amd._native as N
    from paper_1907_01005_amd import FP64
    lib = N.lib()
    cases = [((16, 12, 8), 2, 61, 3.0, 7, [8, 5, 12, 4, 8, 8, 16]),   # larger first
             ((8, 6, 4), 2, 29, 2.2, 11, [8, 5, 12, 4])]             # then smaller
    for cells, deg, M, r, seed, sizes in cases:
        say(f"noalloc overlap {cells} Q{deg} M={M}")
        dp = _problem(cells, deg, M, r, seed, sizes)
        assert dp.layout.work_bytes <= 64 << 20
        dp.apply(FP64)
        dp.overlap()
        torch.cuda.synchronize()
        S_ref, t_ref = dp.S.clone(), dp.trace.clone()
        S = torch.full_like(dp.S, np.nan)
        t = torch.full_like(dp.trace, np.nan)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.mfb_tmmult_noalloc(dp.layout.handle, C.c_void_p(dp.X.data_ptr()),
                                    C.c_void_p(dp.Y.data_ptr()), C.c_void_p(S.data_ptr()),
                                    C.c_void_p(t.data_ptr()), st)
        assert rc == N.MFB_OK, lib.mfb_last_error()
        torch.cuda.synchronize()
        say(f"noalloc: max |S - S_ref| {float((S - S_ref).abs().max()):.3e}, "
            f"trace {float(t[0]):.17g} vs {float(t_ref[0]):.17g}")
        assert torch.equal(S, S_ref) and torch.equal(t, t_ref)


def test_tmmult_noalloc_refuses_oversize_workspace():
    """A layout whose overlap workspace exceeds the 64 MiB scratch: EINVAL,
    and S is not touched."""
    import torch
    import paper_1907_01005_amd._native as N
    from paper_1907_01005_amd import Layout, Mesh
    lib = N.lib()
    m = Mesh(8, 8, 8, (8.0, 8.0, 8.0), 2)
    c = np.random.default_rng(1).random((640, 3)) * 8
    lay = Layout(m, c, 30.0, colblock_sizes=[8] * 80)   # every block stored: about 210 MB of partials
    assert lay.work_bytes > 64 << 20
    say(f"oversize workspace {lay.work_bytes} bytes")
    S = torch.full((640, 640), 3.5, dtype=torch.float64, device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    X = torch.zeros(lay.nvalues, dtype=torch.float64, device="cuda")
    rc = lib.mfb_tmmult_noalloc(lay.handle, C.c_void_p(X.data_ptr()), C.c_void_p(X.data_ptr()),
                                C.c_void_p(S.data_ptr()), C.c_void_p(t.data_ptr()), None)
    assert rc == N.MFB_EINVAL and b"scratch" in lib.mfb_last_error()
    torch.cuda.synchronize()
    assert bool((S == 3.5).all())
