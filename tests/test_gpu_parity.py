"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: the float64 forms (vector and matrix cores) within 1e-12, the float32
forms within 1e-5, each as relative Frobenius error and as max|diff| /
max|oracle| (Y, S; relative error of the trace); BCSR indices bit-exact
(checked on the CPU in test_pattern_parity.py).
"""

import numpy as np
import pytest

import synth
from helpers import device_problem, gate, gpu_available, oracle_full, rel_fro, say
from oracle.workload import OracleProblem

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.fail("GPU tests need a visible GPU (run with -m 'not gpu' on CPU)")


def _run(dp, prec, tuned=None):
    import torch
    if tuned is None:
        dp.apply(prec)
    elif isinstance(tuned, tuple):
        dp.apply_tuned(prec, kernel=tuned[0], grid=tuned[1])
    else:
        dp.apply_tuned(prec, kernel=tuned)
    dp.overlap()
    torch.cuda.synchronize()
    return dp.Y.cpu().numpy()[:dp.nvalues], dp.S_original_order(), float(dp.trace.cpu()[0])


def _check_full(wl, op, dp, prec, tol, tuned=None, ref=None):
    """Y at every stored entry, S and the trace against the oracle; ref: the
    oracle's (Y at the entry coordinates, S, trace) if already computed."""
    Yg, S, tr = _run(dp, prec, tuned)
    if ref is None:
        node, orb = dp.layout.entry_coords()
        ref = oracle_full(op, node, orb)
    Yo, So, tro = ref
    tag = f"{wl.name} prec={prec} tuned={tuned}"
    gate(Yg, Yo, tol, tag + " Y")
    gate(S, So, tol, tag + " S")
    et = abs(tr - tro) / max(abs(tro), 1e-300)
    say(f"{tag} trace rel {et:.2e}")
    assert et <= tol
    return Yg


PRECS = ((0, TOL64), (1, TOL64), (3, TOL32), (2, TOL32))


def _small(cfg_cells, degree, M, radius, seed, sizes=None, dirichlet=0x3F, potential="wells",
           L=None, bend=0.0):
    nx, ny, nz = cfg_cells
    L = L or (float(nx), float(ny), float(nz))
    ms = synth.MeshSpec(nx, ny, nz, L, degree, dirichlet, bend=bend)
    wl = synth.custom_workload(ms, M, radius, seed, potential=potential,
                               name=f"{nx}x{ny}x{nz}-Q{degree}-M{M}")
    if sizes is not None:
        wl.colblock_sizes = np.asarray(sizes, dtype=np.int32)
    return wl


@pytest.mark.parametrize("prec,tol", list(PRECS))
def test_config1_full(prec, tol):
    wl = synth.make_workload(1)
    say(f"config1 prec={prec}")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_full(wl, op, dp, prec, tol)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_generic_values_ragged_blocks(degree):
    """Values at every stored entry (shell items do work) and ragged column blocks."""
    wl = _small((8, 6, 4), degree, 29, 2.2, 11, sizes=[8, 5, 12, 4])
    say(f"generic values Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=3)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    node, orb = dp.layout.entry_coords()
    ref = oracle_full(op, node, orb)
    for prec, tol in PRECS:
        _check_full(wl, op, dp, prec, tol, ref=ref)
    for kernel in range(1, 8):
        _check_full(wl, op, dp, 0, TOL64, tuned=kernel, ref=ref)
        _check_full(wl, op, dp, 1, TOL64, tuned=kernel, ref=ref)
        _check_full(wl, op, dp, 2, TOL32, tuned=kernel, ref=ref)
    if degree >= 2:   # the line kernel (a workgroup per cell): vector-ALU forms
        _check_full(wl, op, dp, 0, TOL64, tuned=9, ref=ref)
        _check_full(wl, op, dp, 3, TOL32, tuned=9, ref=ref)
    if degree <= 2:   # register-resident waves: vector-ALU forms at p <= 2
        _check_full(wl, op, dp, 0, TOL64, tuned=8, ref=ref)
        _check_full(wl, op, dp, 3, TOL32, tuned=8, ref=ref)
    else:
        from paper_1907_01005_amd import MfbError
        import paper_1907_01005_amd._native as N
        with pytest.raises(MfbError) as e:
            dp.apply_tuned(0, kernel=8)
        assert e.value.code == N.MFB_EUNSUPPORTED
    for spw in (1, 4, 64):
        _check_full(wl, op, dp, 0, TOL64, tuned=(0, spw), ref=ref)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_few_nonzero_shell_items(degree):
    """Orbital values plus a few values at stored entries off the supports:
    only some shell items of a checked group hold non-zeros."""
    from oracle.pattern import entry_coords
    wl = _small((8, 6, 4), degree, 29, 2.2, 11, sizes=[8, 5, 12, 4])
    say(f"few non-zero shell items Q{degree}")
    op = OracleProblem(wl)
    node, orb = entry_coords(op.pattern)
    dmask = op.mesh.dirichlet_mask()
    n_all = int(op.mesh.ndofs)
    on_support = np.zeros(n_all * wl.M, dtype=bool)
    on_support[op.node.astype(np.int64) * wl.M + op.orb] = True
    free = np.flatnonzero(~on_support[node.astype(np.int64) * wl.M + orb] & ~dmask[node])
    rng = np.random.default_rng(17)
    pick = rng.choice(free, size=min(12, len(free)), replace=False)
    op.node = np.concatenate([op.node, node[pick]])
    op.orb = np.concatenate([op.orb, orb[pick].astype(op.orb.dtype)])
    op.val = np.concatenate([op.val, rng.standard_normal(len(pick))])
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_full(wl, op, dp, 0, TOL64)
    for spw in (1, 2, 8, 64):
        _check_full(wl, op, dp, 0, TOL64, tuned=(0, spw))
    _check_full(wl, op, dp, 2, TOL32, tuned=(0, 4))
    _check_full(wl, op, dp, 0, TOL64, tuned=1)
    if degree >= 2:
        _check_full(wl, op, dp, 0, TOL64, tuned=9)
    if degree <= 2:
        _check_full(wl, op, dp, 0, TOL64, tuned=8)


def test_natural_bc_lexicographic_free_faces():
    wl = _small((4, 6, 8), 2, 12, 3.0, 5, sizes=[7, 5], dirichlet=0b010110)
    say("mixed Dirichlet faces")
    op = OracleProblem(wl, values="generic", value_seed=9)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_full(wl, op, dp, 0, TOL64)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_closed_form_through_library(degree):
    """V = 1, natural BCs, full support: S = X^T H X hits closed-form integrals."""
    from oracle.fe1d import gll_nodes
    nx, ny, nz = 4, 2, 6
    L = (1.0, 0.5, 1.5)
    ms = synth.MeshSpec(nx, ny, nz, L, degree, 0)
    wl = synth.custom_workload(ms, 4, 100.0, 1, potential="one")
    wl.colblock_sizes = np.asarray([4], dtype=np.int32)
    say(f"closed form Q{degree}")
    dp = device_problem(wl)
    na = [degree * c + 1 for c in (nx, ny, nz)]
    xi = gll_nodes(degree)
    pos = []
    for d, c in enumerate((nx, ny, nz)):
        X = np.arange(na[d])
        cell = np.minimum(X // degree, c - 1)
        pos.append((cell + xi[X - degree * cell]) * (L[d] / c))
    g = np.arange(na[0] * na[1] * na[2])
    x = pos[0][g % na[0]]
    y = pos[1][(g // na[0]) % na[1]]
    cols = [np.ones_like(x), x, y, x * y]
    node = np.concatenate([g] * 4)
    orb = np.repeat(np.arange(4), len(g)).astype(np.int32)
    dp.set_X_coo(node, orb, np.concatenate(cols))
    _, S, tr = _run(dp, 0)
    Lx, Ly, Lz = L
    vol = Lx * Ly * Lz
    exact = {
        (0, 0): vol,
        (1, 1): 0.5 * vol + Lx ** 3 / 3 * Ly * Lz,
        (2, 2): 0.5 * vol + Ly ** 3 / 3 * Lx * Lz,
        (3, 3): 0.5 * (Ly ** 3 / 3 * Lx * Lz + Lx ** 3 / 3 * Ly * Lz) + Lx ** 3 / 3 * Ly ** 3 / 3 * Lz,
        (0, 1): Lx ** 2 / 2 * Ly * Lz,
    }
    for (a, b), v in exact.items():
        assert abs(S[a, b] - v) <= 1e-12 * max(1.0, abs(v)), (a, b, S[a, b], v)
    assert abs(S[1, 0] - exact[(0, 1)]) <= 1e-12
    assert abs(tr - sum(exact[(k, k)] for k in range(4))) <= 1e-11


def test_empty_and_degenerate_layouts():
    """No stored block at all, and an orbital set whose blocks miss some rows."""
    import torch
    wl = _small((4, 4, 4), 2, 8, 0.0, 2)      # no batch centre within radius 0
    say("empty layout")
    dp = device_problem(wl)
    assert dp.nvalues == 0
    dp.apply(0)
    dp.overlap()
    torch.cuda.synchronize()
    assert float(dp.trace.cpu()[0]) == 0.0
    assert not dp.S.abs().max().item()


def test_repeat_determinism_and_queue_kernel():
    wl = synth.make_workload(1)
    say("determinism")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    Y1, S1, _ = _run(dp, 0)
    Y2, S2, _ = _run(dp, 0)
    scale = np.abs(Y1).max()
    assert np.abs(Y1 - Y2).max() <= 1e-14 * scale
    for kernel in range(1, 9):
        Y3, S3, _ = _run(dp, 0, tuned=kernel)
        assert np.abs(Y1 - Y3).max() <= 1e-14 * scale, kernel
    # the overlap reduction has a fixed order: bitwise repeatable for equal inputs
    dp.Y.copy_(torch_from(Y1, dp))
    dp.overlap()
    Sa = dp.S.cpu().numpy().copy()
    dp.overlap()
    assert np.array_equal(Sa, dp.S.cpu().numpy())


def torch_from(a, dp):
    import torch
    t = torch.zeros_like(dp.Y)
    t[:len(a)] = torch.from_numpy(a).to(t.device)
    return t


@pytest.mark.parametrize("cfg", [2, 3])
def test_paper_scale_full(cfg):
    """Full-size configurations (846369 DoFs, 320 orbitals, Q2 / Q4): every
    stored entry of Y in all 40 column blocks, all of S and the trace, in
    every precision form, against one oracle pass."""
    wl = synth.make_workload(cfg)
    say(f"config{cfg} full size")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    node, orb = dp.layout.entry_coords()
    ref = oracle_full(op, node, orb)
    say(f"config{cfg}: oracle done, {len(node)} stored entries")
    for prec, tol in PRECS:
        _check_full(wl, op, dp, prec, tol, ref=ref)
    if wl.mesh.degree <= 2:
        _check_full(wl, op, dp, 0, TOL64, tuned=8, ref=ref)
        _check_full(wl, op, dp, 3, TOL32, tuned=8, ref=ref)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_curved_cells(degree):
    """Bent cells (isoparametric map, the metric coupling all three gradients):
    generic values with ragged blocks, the default and the fused tuned
    kernels in every precision; other tuned kernels are refused."""
    from paper_1907_01005_amd import MfbError
    import paper_1907_01005_amd._native as N
    wl = _small((8, 6, 4), degree, 29, 2.2, 11, sizes=[8, 5, 12, 4], bend=0.3)
    say(f"curved cells Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=5)
    assert op.mesh.curved
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    for prec, tol in ((0, TOL64), (3, TOL32), (2, TOL32)):
        _check_full(wl, op, dp, prec, tol)
    for kernel in (2, 7):
        _check_full(wl, op, dp, 0, TOL64, tuned=kernel)
    with pytest.raises(MfbError) as e:
        dp.apply_tuned(0, kernel=1)
    assert e.value.code == N.MFB_EUNSUPPORTED


DENSE_SIZES = [8, 5, 12, 4, 16, 7, 9, 3, 11, 6, 10, 9, 14, 2, 13, 11]


@pytest.mark.parametrize("degree,cells,radius", [(1, (8, 6, 4), 2.0), (2, (8, 6, 4), 2.0),
                                                 (3, (6, 4, 4), 2.5), (4, (4, 4, 4), 2.0)])
def test_dense_row_blocks(degree, cells, radius):
    """Row blocks with many stored blocks: at Q1 and Q2 their overlap products
    run as one task each (all three width classes; rows in one chunk at Q1,
    up to 7 chunks at Q2, ragged), beside units for sparse rows and for rows
    wider than a task.  At Q3 and Q4 the row blocks are longer than a task
    takes and every product is a unit.  S = X^T (H X) against the oracle,
    then S = X^T Z for generic Z on X's pattern against the oracle's X^T Z."""
    import scipy.sparse as sp
    import torch
    from oracle.apply import overlap as oracle_overlap
    wl = _small(cells, degree, sum(DENSE_SIZES), radius, 5, sizes=DENSE_SIZES)
    say(f"dense row blocks Q{degree} {cells} r={radius}")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    assert (dp.layout.info["tm_tasks"] > 0) == (degree <= 2)
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_full(wl, op, dp, 0, TOL64)
    node, orb = dp.layout.entry_coords()
    z = np.random.default_rng(17).standard_normal(len(node))
    dp.Y[:dp.nvalues].copy_(torch.from_numpy(dp.layout.pack(node, orb, z)))
    dp.overlap()
    torch.cuda.synchronize()
    So = oracle_overlap(op.X_sparse(), sp.csc_matrix((z, (node, orb)), shape=op.X_sparse().shape))
    eS = rel_fro(dp.S_original_order(), So)
    et = abs(float(dp.trace.cpu()[0]) - np.trace(So)) / abs(np.trace(So))
    say(f"dense Q{degree}: X^T Z rel {eS:.2e}, trace rel {et:.2e}")
    assert eS <= TOL64 and et <= TOL64


def test_dense_runs_of_row_blocks():
    """Runs of dense row blocks merged into one task (Q1, 16x12x8 cells, 96
    orbitals in ragged blocks, support radius 6 cells): about 80 tasks, most
    over two to four row blocks, many with blocks that one member does not
    store (zero rows) and a few union pairs that meet in no member (dropped).
    S = X^T Z for generic Z on X's pattern against the oracle's X^T Z."""
    import scipy.sparse as sp
    import torch
    from oracle.apply import overlap as oracle_overlap
    sizes = [8, 5, 12, 4, 16, 7, 9, 3, 11, 6, 10, 5]
    wl = _small((16, 12, 8), 1, sum(sizes), 6.0, 5, sizes=sizes)
    say("dense runs Q1 16x12x8 r=6")
    op = OracleProblem(wl)
    dp = device_problem(wl)
    pat = dp.layout.pattern()
    ka = np.diff(pat["rowptr"])
    qualifying = int(((ka * ka >= 16) & (ka * ka <= 512)).sum())
    assert 0 < dp.layout.info["tm_tasks"] < qualifying
    dp.set_X_coo(op.node, op.orb, op.val)
    _check_full(wl, op, dp, 0, TOL64)
    node, orb = dp.layout.entry_coords()
    z = np.random.default_rng(23).standard_normal(len(node))
    dp.Y[:dp.nvalues].copy_(torch.from_numpy(dp.layout.pack(node, orb, z)))
    dp.overlap()
    torch.cuda.synchronize()
    So = oracle_overlap(op.X_sparse(), sp.csc_matrix((z, (node, orb)), shape=op.X_sparse().shape))
    eS = rel_fro(dp.S_original_order(), So)
    say(f"dense runs: X^T Z rel {eS:.2e}")
    assert eS <= TOL64


@pytest.mark.parametrize("degree", [5, 6])
def test_high_degree(degree):
    """p = 5, 6 (one workgroup per cell, a thread per line): generic values at
    every stored entry with ragged column blocks, and orbital values with
    shell items, in the fp64 and fp32 vector forms against the oracle: all of
    Y, S and the trace.  The matrix-core forms, the other kernels and curved
    cells are refused at these degrees."""
    from paper_1907_01005_amd import MfbError
    import paper_1907_01005_amd._native as N
    wl = _small((4, 4, 2), degree, 21, 1.6, 40 + degree, sizes=[8, 5, 4, 4], dirichlet=0b100101)
    say(f"high degree Q{degree}")
    for values in ("generic", "orbitals"):
        op = OracleProblem(wl, values=values, value_seed=7) if values == "generic" else OracleProblem(wl)
        dp = device_problem(wl)
        dp.set_X_coo(op.node, op.orb, op.val)
        node, orb = dp.layout.entry_coords()
        ref = oracle_full(op, node, orb)
        _check_full(wl, op, dp, 0, TOL64, ref=ref)
        _check_full(wl, op, dp, 3, TOL32, ref=ref)
        _check_full(wl, op, dp, 0, TOL64, tuned=0, ref=ref)
        _check_full(wl, op, dp, 3, TOL32, tuned=9, ref=ref)
    for prec in (1, 2):
        with pytest.raises(MfbError) as e:
            dp.apply(prec)
        assert e.value.code == N.MFB_EUNSUPPORTED
    for kernel in (1, 2, 7, 8):
        with pytest.raises(MfbError) as e:
            dp.apply_tuned(0, kernel=kernel)
        assert e.value.code == N.MFB_EUNSUPPORTED


@pytest.mark.parametrize("degree", [2, 4])
def test_overlap_shapes(degree):
    """mfb_tmmult_tuned: every row-step shape of the two block-product classes
    gives the oracle's S and trace (generic values and ragged column blocks, so
    that 8x8 products, narrower ones and wider ones all occur), and a shape the
    library does not have is refused."""
    import torch
    import paper_1907_01005_amd._native as N
    from paper_1907_01005_amd import MfbError
    wl = _small((8, 6, 4), degree, 29, 2.2, 11, sizes=[8, 5, 12, 4])
    say(f"overlap shapes Q{degree}")
    op = OracleProblem(wl, values="generic", value_seed=3)
    dp = device_problem(wl)
    dp.set_X_coo(op.node, op.orb, op.val)
    node, orb = dp.layout.entry_coords()
    _, So, tro = oracle_full(op, node, orb)
    dp.apply(0)
    for u in (4, 8, 16):
        for lng in (4, 8, 16):
            dp.S.fill_(7.25)
            dp.trace.fill_(7.25)
            dp.overlap_tuned(u, lng)
            torch.cuda.synchronize()
            tag = f"{wl.name} overlap steps {u}/{lng}"
            gate(dp.S_original_order(), So, TOL64, tag + " S")
            tr = float(dp.trace.cpu()[0])
            et = abs(tr - tro) / max(abs(tro), 1e-300)
            say(f"{tag} trace rel {et:.2e}")
            assert et <= TOL64
    for bad in ((5, 4), (4, 32)):
        with pytest.raises(MfbError) as e:
            dp.overlap_tuned(*bad)
        assert e.value.code == N.MFB_EINVAL
