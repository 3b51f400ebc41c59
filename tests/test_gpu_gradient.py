"""GPU tests of Alg. 7 (post-multiplication with truncation), the gradient of
eq. gradient and a steepest-descent step of the orbital minimisation, against
the oracle; a central-difference check of the gradient at full size."""

import numpy as np
import pytest

import synth
from helpers import device_problem, gpu_available, rel_fro, say
from oracle.apply import block_mask, mmult as o_mmult
from oracle.workload import OracleProblem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.fail("GPU tests need a visible GPU (run with -m 'not gpu' on CPU)")


def _small(degree):
    ms = synth.MeshSpec(8, 6, 4, (8.0, 6.0, 4.0), degree)
    wl = synth.custom_workload(ms, 29, 2.2, 11, potential="wells", name=f"8x6x4-Q{degree}-M29")
    wl.colblock_sizes = np.asarray([8, 5, 12, 4], dtype=np.int32)
    return wl


def _at_entries(dense, node, orb):
    return dense[node, orb]


def _values_dense(layout, values, N, M):
    node, orb = layout.entry_coords()
    D = np.zeros((N, M))
    D[node, orb] = values[:layout.nvalues]
    return D


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_mmult_truncation_against_oracle(degree):
    import torch
    from paper_1907_01005_amd import mmult
    wl = _small(degree)
    say(f"mmult Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=6)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    dp.enable_closure()
    rng = np.random.default_rng(12)
    M, N = wl.M, op.mesh.ndofs
    perm = dp.layout.pattern()["col_perm"]
    B = rng.standard_normal((M, M))
    B_lib = torch.from_numpy(np.ascontiguousarray(B[np.ix_(perm, perm)])).cuda()
    xmask = block_mask(op.pattern, np.arange(M))
    node, orb = dp.layout.entry_coords()
    for src_name, src, Av in (("closure", dp.closure, None), ("x", dp.layout, None)):
        A = torch.from_numpy(rng.standard_normal(src.nvalues)).cuda()
        Ad = _values_dense(src, A.cpu().numpy(), N, M)
        for alpha, beta in ((1.0, 0.0), (-2.0, 4.0)):
            mmult(src, dp.layout, A, B_lib, alpha, beta, dp.Y)
            torch.cuda.synchronize()
            got = dp.Y.cpu().numpy()[:dp.nvalues]
            ref = _at_entries(o_mmult(Ad, alpha * B + beta * np.eye(M), xmask), node, orb)
            e = rel_fro(got, ref)
            say(f"mmult Q{degree} from {src_name} alpha={alpha} beta={beta}: rel {e:.2e}")
            assert e <= 1e-13
    # accumulate form and bitwise repeat
    A = torch.from_numpy(rng.standard_normal(dp.closure.nvalues)).cuda()
    mmult(dp.closure, dp.layout, A, B_lib, 1.0, 0.0, dp.Y)
    mmult(dp.closure, dp.layout, A, B_lib, 1.0, 0.0, dp.Y, True)
    torch.cuda.synchronize()
    twice = dp.Y.cpu().numpy()[:dp.nvalues].copy()
    mmult(dp.closure, dp.layout, A, B_lib, 2.0, 0.0, dp.Y)
    torch.cuda.synchronize()
    assert np.abs(twice - dp.Y.cpu().numpy()[:dp.nvalues]).max() <= 1e-13 * np.abs(twice).max()


def _check_gradient(wl, op, dp, prec, tol):
    import torch
    dp.gradient(prec)
    torch.cuda.synchronize()
    G, E = op.gradient_dense()
    node, orb = dp.layout.entry_coords()
    got = dp.G.cpu().numpy()[:dp.nvalues]
    ref = G[node, orb]
    e = rel_fro(got, ref)
    eE = abs(float(dp.E.cpu()[0]) - E) / abs(E)
    say(f"{wl.name} prec={prec}: gradient rel {e:.2e}, energy rel {eE:.2e}")
    assert e <= tol and eE <= tol


def test_gradient_config1():
    wl = synth.make_workload(1)
    say("gradient config1")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_gradient(wl, op, dp, 0, 1e-12)
    _check_gradient(wl, op, dp, 2, 1e-5)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_gradient_generic_ragged(degree):
    wl = _small(degree)
    say(f"gradient generic Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=2)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_gradient(wl, op, dp, 0, 1e-12)


def test_descent_steps_lower_the_energy():
    """Five steepest-descent steps on config 1: E decreases every step, and
    after the first step it equals the oracle's energy at X - tau G."""
    import torch
    wl = synth.make_workload(1)
    say("descent config1")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    tau = 2e-3
    G0, E0 = op.gradient_dense()
    energies = []
    for k in range(5):
        dp.descent_step(tau)
        torch.cuda.synchronize()
        energies.append(float(dp.E.cpu()[0]))
        if k == 0:
            gg = float(dp.dots.cpu()[0])
            assert abs(gg - np.sum(G0 * G0)) <= 1e-12 * gg
    dp.energy()
    torch.cuda.synchronize()
    energies.append(float(dp.E.cpu()[0]))
    say(f"descent energies: {energies}")
    assert all(b < a for a, b in zip(energies, energies[1:]))
    X1 = op.X_columns(np.arange(op.M)) - tau * G0
    q = OracleProblem.__new__(OracleProblem)
    q.__dict__.update(op.__dict__)
    node, orb = np.nonzero(X1)
    q.node, q.orb, q.val = node, orb.astype(np.int32), X1[node, orb]
    assert abs(energies[1] - q.gradient_dense()[1]) <= 1e-11 * abs(energies[1])


def test_gradient_central_difference_full_size():
    """box-64x40x40-Q2: tr(G^T G) against (E(X + hG) - E(X - hG)) / 2h, all
    on the GPU (the directional derivative of eq. G_ops4 along G)."""
    import torch
    from paper_1907_01005_amd import mv_axpy
    wl = synth.make_workload(2)
    say("gradient full size")
    node, orb, val = synth.orbital_values(wl)
    dp = device_problem(wl)
    dp.set_X_coo(node, orb, val)
    dp.descent_step(0.0)                     # E, G and tr(G^T G) at X; X unchanged
    torch.cuda.synchronize()
    gg = float(dp.dots.cpu()[0])
    G = dp.G.clone()
    X0 = dp.X.clone()
    h = 1e-3 * float(X0.norm()) / np.sqrt(gg)
    ev = []
    for s in (1.0, -1.0):
        dp.X.copy_(X0)
        mv_axpy(dp.layout, s * h, G, dp.X)
        dp.energy()
        torch.cuda.synchronize()
        ev.append(float(dp.E.cpu()[0]))
    fd = (ev[0] - ev[1]) / (2 * h)
    say(f"full size: tr(G^T G) {gg:.6e}, central difference {fd:.6e}")
    assert abs(fd - gg) <= 1e-5 * gg


def test_scale_columns():
    import torch
    from paper_1907_01005_amd import mv_scale_columns
    wl = _small(2)
    say("scale columns")
    op = OracleProblem(wl, values="generic", value_seed=1)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    X0 = dp.X.cpu().numpy()[:dp.nvalues].copy()
    sc = np.random.default_rng(3).uniform(0.5, 2.0, wl.M)          # library column order
    mv_scale_columns(dp.layout, torch.from_numpy(sc).cuda(), dp.X)
    torch.cuda.synchronize()
    node, orb = dp.layout.entry_coords()
    pos = dp.layout.pattern()["col_perm"]
    col_of_orb = np.empty(wl.M, dtype=np.int64)
    col_of_orb[pos] = np.arange(wl.M)
    assert np.array_equal(dp.X.cpu().numpy()[:dp.nvalues], X0 * sc[col_of_orb[orb]])
