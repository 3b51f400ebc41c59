"""GPU tests of the closure destination, the mass operator and the energy:
H X and M X onto the closure of X's pattern against the oracle, the projected
matrices Hbar = X^T H X and Mbar = X^T M X (symmetric, exact), and
E = tr((2 I - Mbar) Hbar) of eq. energy."""

import numpy as np
import pytest

import synth
from helpers import device_problem, gpu_available, rel_fro, say
from oracle.pattern import entry_coords
from oracle.workload import OracleProblem

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.fail("GPU tests need a visible GPU (run with -m 'not gpu' on CPU)")


def _small(degree, values="orbitals", bend=0.0):
    ms = synth.MeshSpec(8, 6, 4, (8.0, 6.0, 4.0), degree, bend=bend)
    wl = synth.custom_workload(ms, 29, 2.2, 11, potential="wells",
                               name=f"8x6x4-Q{degree}-M29")
    wl.colblock_sizes = np.asarray([8, 5, 12, 4], dtype=np.int32)
    return wl


def _closure_values_oracle(op, closure_layout, what):
    """Oracle H X or M X at every stored entry of the library's closure layout."""
    node, orb = closure_layout.entry_coords()
    out = np.zeros(len(node))
    for C in range(op.pattern.ncb):
        orbs = op.block_orbitals(C)
        Y = op.Y_columns(orbs, what, "closure")
        col = {int(a): j for j, a in enumerate(orbs)}
        sel = np.isin(orb, orbs)
        out[sel] = Y[node[sel], [col[int(a)] for a in orb[sel]]]
    return out


def _check(wl, op, dp, prec, tol, full_values=True):
    import torch
    dp.energy(prec)
    torch.cuda.synchronize()
    clo = dp.closure
    if full_values:
        for what, buf in (("H", dp.YH), ("M", dp.YM)):
            Yg = buf.cpu().numpy()[:clo.nvalues]
            Yo = _closure_values_oracle(op, clo, what)
            e = rel_fro(Yg, Yo)
            say(f"{wl.name} prec={prec} {what}X on closure: rel {e:.2e}")
            assert e <= tol
    if not hasattr(op, "_projected"):
        op._projected = op.projected()
    Mo, Ho, Eo = op._projected
    Hg, Mg = dp.original_order(dp.Hbar), dp.original_order(dp.Mbar)
    Eg = float(dp.E.cpu()[0])
    eH, eM, eE = rel_fro(Hg, Ho), rel_fro(Mg, Mo), abs(Eg - Eo) / abs(Eo)
    asym = np.abs(Hg - Hg.T).max() / np.abs(Hg).max()
    say(f"{wl.name} prec={prec}: relHbar {eH:.2e} relMbar {eM:.2e} relE {eE:.2e} asym(Hbar) {asym:.2e}")
    assert eH <= tol and eM <= tol and eE <= tol
    assert asym <= (1e-13 if prec == 0 else 1e-6)
    return Hg, Mg, Eg


def test_config1_closure_energy():
    wl = synth.make_workload(1)
    say("config1 closure")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    for prec, tol in ((0, TOL64), (2, TOL32), (3, TOL32)):
        _check(wl, op, dp, prec, tol)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_closure_generic_values_ragged_blocks(degree):
    wl = _small(degree)
    say(f"closure generic Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=5)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check(wl, op, dp, 0, TOL64)
    _check(wl, op, dp, 2, TOL32)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_mass_on_the_pattern_of_x(degree):
    """mfb_apply_op with y = x: M X and H X kept on X's own pattern, as
    mfb_apply_H keeps H X."""
    import torch
    from paper_1907_01005_amd import OP_H, OP_M, apply_op
    wl = _small(degree)
    say(f"mass on x pattern Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=8)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    node, orb = dp.layout.entry_coords()
    dp.apply(0)
    torch.cuda.synchronize()
    YH = dp.Y.cpu().numpy()[:dp.nvalues].copy()
    for which, code in (("M", OP_M), ("H", OP_H)):
        apply_op(dp.mesh, dp.layout, dp.layout, code, dp.X, dp.Y, 0)
        torch.cuda.synchronize()
        Yg = dp.Y.cpu().numpy()[:dp.nvalues]
        Yo = np.zeros(len(node))
        for C in range(op.pattern.ncb):
            orbs = op.block_orbitals(C)
            Y = op.Y_columns(orbs, which, "x")
            col = {int(a): j for j, a in enumerate(orbs)}
            sel = np.isin(orb, orbs)
            Yo[sel] = Y[node[sel], [col[int(a)] for a in orb[sel]]]
        e = rel_fro(Yg, Yo)
        say(f"{which}X on x pattern Q{degree}: rel {e:.2e}")
        assert e <= TOL64
        if which == "H":
            assert np.abs(Yg - YH).max() <= 1e-14 * np.abs(YH).max()


@pytest.mark.parametrize("cfg", [2, 3])
def test_paper_scale_closure_energy(cfg):
    """Full-size box-64x40x40-Q2 / box-32x20x20-Q4: Hbar, Mbar and E against
    the oracle; Hbar symmetric; Mbar positive definite; the overlap on the
    closure repeatable bit for bit."""
    import torch
    wl = synth.make_workload(cfg)
    say(f"config{cfg} closure full size")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    Hg, Mg, Eg = _check(wl, op, dp, 0, TOL64, full_values=False)
    _check(wl, op, dp, 2, TOL32, full_values=False)
    # Mbar is symmetric positive definite
    np.linalg.cholesky(0.5 * (Mg + Mg.T))
    # repeatable bit for bit (fixed-order overlap and energy on equal inputs)
    Y1 = dp.YH.clone()
    dp.Hbar.zero_()
    from paper_1907_01005_amd import tmmult
    tmmult(dp.closure, dp.X, Y1, dp.Hbar, dp.tr_c[0:1], dp.work_c)
    torch.cuda.synchronize()
    Ha = dp.Hbar.cpu().numpy().copy()
    tmmult(dp.closure, dp.X, Y1, dp.Hbar, dp.tr_c[0:1], dp.work_c)
    torch.cuda.synchronize()
    assert np.array_equal(Ha, dp.Hbar.cpu().numpy())
    from paper_1907_01005_amd import energy
    E1 = dp.E.clone()
    energy(dp.M, dp.Mbar, dp.Hbar, dp.E, dp.work_e)
    e1 = float(dp.E.cpu()[0])
    energy(dp.M, dp.Mbar, dp.Hbar, dp.E, dp.work_e)
    assert e1 == float(dp.E.cpu()[0]) and np.isfinite(float(E1.cpu()[0]))


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_curved_closure_energy(degree):
    """Bent cells: H X and M X on the closure (per-cell metric and JxW),
    Hbar, Mbar and the energy against the oracle."""
    wl = _small(degree, bend=0.3)
    say(f"curved closure Q{degree}")
    op = OracleProblem(wl)
    assert op.mesh.curved
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    for prec, tol in ((0, TOL64), (2, TOL32)):
        _check(wl, op, dp, prec, tol)


def test_dense_closure_energy():
    """Closure with densely populated row blocks: the overlap X^T (H X) onto
    the closure runs most row blocks as tasks whose two sides differ in width."""
    sizes = [8, 5, 12, 4, 16, 7, 9, 3, 11, 6, 10, 9, 14, 2, 13, 11]
    ms = synth.MeshSpec(8, 6, 4, (8.0, 6.0, 4.0), 2)
    wl = synth.custom_workload(ms, sum(sizes), 2.0, 5, potential="wells", name="8x6x4-Q2-dense")
    wl.colblock_sizes = np.asarray(sizes, dtype=np.int32)
    say("dense closure")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    dp.enable_closure()
    assert dp.closure.info["tm_tasks"] > 0
    _check(wl, op, dp, 0, TOL64)


@pytest.mark.parametrize("degree", [5, 6])
def test_high_degree_closure_and_mass(degree):
    """p = 5, 6: H X and M X onto the closure, Hbar, Mbar and E, and M X, H X
    on X's own pattern, in the fp64 and fp32 vector forms against the oracle."""
    import torch
    from paper_1907_01005_amd import OP_H, OP_M, apply_op
    ms = synth.MeshSpec(4, 4, 2, (4.0, 3.5, 2.0), degree, 0b100101)
    wl = synth.custom_workload(ms, 21, 1.6, 40 + degree, potential="wells",
                               name=f"4x4x2-Q{degree}-M21")
    wl.colblock_sizes = np.asarray([8, 5, 4, 4], dtype=np.int32)
    say(f"closure Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=9)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check(wl, op, dp, 0, TOL64)
    _check(wl, op, dp, 3, TOL32)
    node, orb = dp.layout.entry_coords()
    for which, code in (("M", OP_M), ("H", OP_H)):
        apply_op(dp.mesh, dp.layout, dp.layout, code, dp.X, dp.Y, 0)
        torch.cuda.synchronize()
        Yg = dp.Y.cpu().numpy()[:dp.nvalues]
        Yo = np.zeros(len(node))
        for C in range(op.pattern.ncb):
            orbs = op.block_orbitals(C)
            Y = op.Y_columns(orbs, which, "x")
            col = {int(a): j for j, a in enumerate(orbs)}
            sel = np.isin(orb, orbs)
            Yo[sel] = Y[node[sel], [col[int(a)] for a in orb[sel]]]
        e = rel_fro(Yg, Yo)
        say(f"{which}X on x pattern Q{degree}: rel {e:.2e}")
        assert e <= TOL64
