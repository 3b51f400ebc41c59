"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check is independent of the oracle's own formulas: closed forms,
invariants, textbook special cases, brute force on tiny meshes and the sizes
printed in the paper's tables (tests/golden/paper_tables.json).
"""

import itertools
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import apply as oapply
from oracle import element, fe1d
from oracle.hilbert import bits_for, hilbert_index
from oracle.mesh import BoxMesh
from oracle.pattern import batch_nodes, build_pattern, order_batches

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- 1D basis
def test_gll_nodes_closed_form():
    assert np.allclose(fe1d.gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-15)
    s = np.sqrt(3.0 / 7.0)
    assert np.allclose(fe1d.gll_nodes(4), [0.0, (1 - s) / 2, 0.5, (1 + s) / 2, 1.0], atol=1e-15)


def test_gauss_rule_closed_form_and_exactness():
    x, w = fe1d.gauss_rule(3)
    s = np.sqrt(3.0 / 5.0)
    assert np.allclose(x, [(1 - s) / 2, 0.5, (1 + s) / 2], atol=1e-15)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)
    for n in (3, 5):
        x, w = fe1d.gauss_rule(n)
        for m in range(2 * n):             # exact up to degree 2n-1
            assert abs(w @ x ** m - 1.0 / (m + 1)) < 1e-14
        assert abs(w @ x ** (2 * n) - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_lagrange_tables(p):
    nodes = fe1d.gll_nodes(p)
    assert np.allclose(fe1d.lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-14)
    x = np.linspace(0, 1, 7)
    # reproduces monomials up to degree p, and their derivatives
    for m in range(p + 1):
        assert np.allclose(fe1d.lagrange_values(nodes, x) @ nodes ** m, x ** m, atol=1e-13)
        dm = m * x ** (m - 1) if m > 0 else np.zeros_like(x)
        assert np.allclose(fe1d.lagrange_derivatives(nodes, x) @ nodes ** m, dm, atol=1e-12)


# ---------------------------------------------------------------- Hilbert
@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_is_a_continuous_bijection(bits):
    n = 1 << bits
    pts = list(itertools.product(range(n), repeat=3))
    idx = {p: hilbert_index(p, bits) for p in pts}
    assert sorted(idx.values()) == list(range(n ** 3))
    walk = sorted(pts, key=idx.get)
    assert walk[0] == (0, 0, 0)
    for a, b in zip(walk, walk[1:]):
        assert sum(abs(u - v) for u, v in zip(a, b)) == 1
    # a Hilbert curve also visits each octant in one contiguous run
    octant = [tuple(c >= n // 2 for c in p) for p in walk]
    runs = sum(1 for a, b in zip(octant, octant[1:]) if a != b)
    assert runs == 7


def test_hilbert_bits():
    assert bits_for(1) == 1 and bits_for(2) == 1 and bits_for(3) == 2 and bits_for(32) == 5
    with pytest.raises(ValueError):
        hilbert_index((2, 0, 0), 1)


# ---------------------------------------------------------------- element matrices
ANISO = dict(nx=2, ny=3, nz=1, L=(1.0, 2.0, 0.5))


def _mesh(p, dirichlet=0, **kw):
    a = dict(ANISO)
    a.update(kw)
    return BoxMesh(a["nx"], a["ny"], a["nz"], a["L"], p, dirichlet)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_symmetry(p):
    m = _mesh(p)
    rng = np.random.default_rng(0)
    v = rng.standard_normal((m.ncells, (p + 1) ** 3))
    H = oapply.assemble(m, v)
    x, y = rng.standard_normal((2, m.ndofs))
    assert abs(x @ H @ y - y @ H @ x) < 1e-12 * np.abs(H).max() * m.ndofs


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_laplacian_kills_constants_and_linears(p):
    m = _mesh(p, nz=2 if p == 1 else 1)  # Q1 needs two cells along z for interior nodes
    K = oapply.assemble(m, which="K")
    pts = m.node_points()
    one = np.ones(m.ndofs)
    assert np.abs(K @ one).max() < 1e-12
    nc = m.node_coords()
    a = m.nodes_per_axis
    interior = np.all((nc > 0) & (nc < np.array(a) - 1), axis=1)
    for lin in (pts[:, 0], pts[:, 1], pts[:, 2], 2 * pts[:, 0] - 3 * pts[:, 1] + pts[:, 2] + 1):
        r = K @ lin
        assert np.abs(r[interior]).max() < 1e-12
        assert np.abs(r[~interior]).max() > 1e-6     # the boundary term is not zero


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_closed_form_integrals(p):
    m = _mesh(p)
    Lx, Ly, Lz = m.L
    vol = Lx * Ly * Lz
    pts = m.node_points()
    x, y = pts[:, 0], pts[:, 1]
    K = oapply.assemble(m, which="K")
    M = oapply.assemble(m, which="M")
    H1 = oapply.assemble(m, np.ones((m.ncells, (p + 1) ** 3)), which="H")
    one = np.ones(m.ndofs)
    assert abs(one @ M @ one - vol) < 1e-12
    assert abs(one @ H1 @ one - vol) < 1e-12
    assert abs(x @ K @ x - 0.5 * vol) < 1e-12
    assert abs(y @ K @ y - 0.5 * vol) < 1e-12
    assert abs(x @ M @ x - Lx ** 3 / 3 * Ly * Lz) < 1e-12
    assert abs(y @ M @ y - Ly ** 3 / 3 * Lx * Lz) < 1e-12
    assert abs(x @ H1 @ x - (0.5 * vol + Lx ** 3 / 3 * Ly * Lz)) < 1e-12
    xy = x * y     # in Q_p, interpolated exactly
    grad2 = (Ly ** 3 / 3) * Lx * Lz + (Lx ** 3 / 3) * Ly * Lz
    assert abs(xy @ K @ xy - 0.5 * grad2) < 1e-11


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_potential_quadrature_exact_for_linear_V(p):
    m = _mesh(p)
    qp = m.qp_points()
    qp3 = m.qp_points(nq=p + 3)
    f = lambda P: 0.3 + P[..., 0] - 2.0 * P[..., 1] + 0.5 * P[..., 2]
    A = element.potential_matrices(p, m.h, f(qp))
    B = element.potential_matrices(p, m.h, f(qp3), nq=p + 3)
    assert np.abs(A - B).max() < 1e-13
    g = lambda P: P[..., 0] ** (2 * p)      # not integrated exactly: the check has teeth
    A = element.potential_matrices(p, m.h, g(qp))
    B = element.potential_matrices(p, m.h, g(qp3), nq=p + 3)
    assert np.abs(A - B).max() > 1e-10


def _first_eigs(m, k=3):
    K = oapply.assemble(m, which="K")
    M = oapply.assemble(m, which="M")
    free = ~m.dirichlet_mask()
    w = sla.eigh(K[np.ix_(free, free)], M[np.ix_(free, free)], eigvals_only=True)
    return w[:k]


@pytest.mark.parametrize("p,ns,rate", [(1, (4, 8, 16), 2.0), (2, (2, 4, 8), 4.0),
                                        (3, (2, 4, 8), 6.0), (4, (2, 4, 8), 8.0)])
def test_1d_box_dirichlet_eigenvalues_converge_at_2p(p, ns, rate):
    """Dirichlet at x=0 and x=L only: lambda_k = pi^2 k^2 / (2 L^2)."""
    L = 1.5
    errs = []
    for nx in ns:
        m = BoxMesh(nx, 1, 1, (L, 0.7, 0.4), p, dirichlet=0b11)
        lam = _first_eigs(m, 2)
        exact = np.pi ** 2 * np.array([1, 4]) / (2 * L ** 2)
        errs.append(np.abs(lam - exact) / exact)
        assert np.all(lam >= exact * (1 - 1e-12))     # conforming: from above
    errs = np.array(errs)
    obs = np.log2(errs[:-1, 0] / errs[1:, 0])
    assert np.all(np.abs(obs - rate) < 0.6), obs


def test_1d_box_dirichlet_eigenvalues_converge_at_2p_degree5():
    """p = 5: the rate 2p = 10 from meshes of 1, 2, 3 and 4 cells (the
    errors reach 1e-11 at 4 cells, so the halving sequence above would sit
    at the eigensolver's floor)."""
    L = 1.5
    ns = np.array([1, 2, 3, 4])
    errs = []
    for nx in ns:
        m = BoxMesh(int(nx), 1, 1, (L, 0.7, 0.4), 5, dirichlet=0b11)
        lam = _first_eigs(m, 1)[0]
        exact = np.pi ** 2 / (2 * L ** 2)
        assert lam >= exact * (1 - 1e-12)
        errs.append((lam - exact) / exact)
    errs = np.array(errs)
    obs = np.log(errs[:-1] / errs[1:]) / np.log(ns[1:] / ns[:-1])
    assert np.all(np.abs(obs - 10.0) < 1.0), obs


def test_3d_box_dirichlet_eigenvalue():
    """All faces Dirichlet: lambda = pi^2/2 * sum_d 1/L_d^2 (first mode)."""
    L = (1.0, 1.3, 0.8)
    m = BoxMesh(4, 4, 4, L, 2, dirichlet=0x3F)
    lam = _first_eigs(m, 1)[0]
    exact = np.pi ** 2 / 2 * sum(1 / l ** 2 for l in L)
    assert exact < lam < exact * (1 + 2e-3)


# ---------------------------------------------------------------- cell-wise apply
@pytest.mark.parametrize("p,cells", [(1, (4, 2, 2)), (2, (2, 2, 2)), (2, (4, 4, 2)), (3, (2, 2, 2)),
                                     (4, (4, 2, 2)), (5, (2, 2, 2)), (6, (2, 2, 2))])
def test_cellwise_apply_equals_dense_assembled(p, cells):
    m = BoxMesh(*cells, (1.0, 0.8, 0.6), p, dirichlet=0x3F)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((m.ncells, (p + 1) ** 3))
    centres = rng.random((6, 3)) * np.array(m.L)
    pat = build_pattern(m, centres, 0.45, [4, 2])
    X = rng.standard_normal((m.ndofs, 6))
    X[~oapply.block_mask(pat, np.arange(6))] = 0.0
    Y = oapply.masked_apply(pat, v, X, np.arange(6))
    H = oapply.assemble(m, v)
    free = ~m.dirichlet_mask()
    Xi = np.where(free[:, None], X, 0.0)
    ref = np.where(free[:, None], H @ Xi, 0.0)
    ref = np.where(oapply.block_mask(pat, np.arange(6)), ref, 0.0)
    assert np.abs(Y - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    assert np.abs(Y[~free]).max() == 0.0


def test_overlap_symmetric_with_full_support():
    """With every block stored and no mask loss, S = X^T H X is symmetric."""
    m = BoxMesh(2, 2, 2, (1.0, 1.0, 1.0), 2, dirichlet=0x3F)
    rng = np.random.default_rng(5)
    v = rng.standard_normal((m.ncells, 27))
    pat = build_pattern(m, rng.random((4, 3)), 10.0, [4])
    assert pat.stored.all()
    X = rng.standard_normal((m.ndofs, 4))
    X[m.dirichlet_mask()] = 0
    Y = oapply.masked_apply(pat, v, X, np.arange(4))
    import scipy.sparse as sp
    S = oapply.overlap(sp.csc_matrix(X), sp.csc_matrix(Y))
    assert np.abs(S - S.T).max() < 1e-12 * np.abs(S).max()
    assert abs(oapply.trace(S) - np.sum(X * Y)) < 1e-12 * abs(np.sum(X * Y))


# ---------------------------------------------------------------- pattern
def test_row_blocks_first_encounter_brute_force():
    m = BoxMesh(4, 6, 2, (1.0, 1.5, 0.5), 2)
    pat = build_pattern(m, np.array([[0.5, 0.7, 0.2]]), 0.3, [1])
    seen = set()
    for r, b in enumerate(pat.batch_order):
        nodes = set(batch_nodes(m, int(b)).tolist())
        rows = pat.dof_perm[pat.rb_start[r]:pat.rb_start[r + 1]].tolist()
        assert rows == sorted(nodes - seen)
        seen |= nodes
    assert len(seen) == m.ndofs
    assert sorted(pat.dof_perm.tolist()) == list(range(m.ndofs))


def test_batch_order_is_hilbert_walk():
    m = BoxMesh(8, 8, 8, (1.0, 1.0, 1.0), 2)
    order = order_batches(m)
    nb = 4
    coords = [(b % nb, (b // nb) % nb, b // (nb * nb)) for b in order]
    for a, b in zip(coords, coords[1:]):
        assert sum(abs(u - v) for u, v in zip(a, b)) == 1


def test_paper_table_sizes():
    """Mesh and blocking sizes printed in Tables 1 and 3."""
    with open(os.path.join(GOLDEN, "paper_tables.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        m = BoxMesh(*case["cells"], tuple(case["L"]), case["degree"])
        assert m.ncells == case["ncells"]
        assert m.ndofs == case["dofs"]
        assert (m.p + 1) ** 3 == case["dofs_per_cell"]
        nrb = m.ncells // 8
        assert nrb == case["row_blocks"]
        assert abs(m.ndofs / nrb - case["row_block_mean"]) < 1e-3


def test_pattern_invariants_config1():
    import synth
    wl = synth.make_workload(1)
    ms = wl.mesh
    m = BoxMesh(ms.nx, ms.ny, ms.nz, ms.L, ms.degree, ms.dirichlet)
    pat = build_pattern(m, wl.centres, wl.radius, wl.colblock_sizes)
    assert pat.rb_start[-1] == m.ndofs
    for r in range(pat.nrb):
        c = pat.colidx[pat.rowptr[r]:pat.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    # every support value of the synthetic orbitals lies in a stored block
    node, orb, _ = synth.orbital_values(wl)
    assert pat.stored[pat.node_rb[node], pat.orb_cb[orb]].all()


@pytest.mark.slow
def test_row_block_spread_at_paper_density():
    """Soft: Table 1 reports 66.1 +- 18.1 rows per block for the Q2 mesh."""
    m = BoxMesh(64, 40, 40, (64.0, 40.0, 40.0), 2)
    order = order_batches(m)
    from oracle.pattern import row_blocks
    rb_start, _, _, _ = row_blocks(m, order)
    sizes = np.diff(rb_start)
    assert abs(sizes.mean() - 66.1226) < 1e-3
    assert 8.0 < sizes.std() < 30.0


# ---------------------------------------------------------------- closure and energy
def _dense_free(m, which, v=None):
    """Dense assembled matrix restricted to the non-Dirichlet nodes (zero rows
    and columns on the Dirichlet faces)."""
    A = oapply.assemble(m, v, which=which)
    free = (~m.dirichlet_mask()).astype(float)
    return A * free[:, None] * free[None, :]


@pytest.mark.parametrize("p,cells,radius", [(2, (4, 4, 2), 1.6), (4, (6, 4, 2), 1.6)])
def test_closure_holds_operator_results_brute_force(p, cells, radius):
    """Dense H X and M X vanish outside the closure blocks, and the cell-wise
    applies onto the closure equal them: X^T H X and X^T M X by brute force."""
    from oracle.pattern import closure_pattern, entry_coords
    m = BoxMesh(*cells, tuple(float(c) for c in cells), p, 0x3F)
    rng = np.random.default_rng(3)
    M = 6
    centres = rng.uniform(0, 1, (M, 3)) * np.array(m.L)
    pat = build_pattern(m, centres, radius, [2, 3, 1])
    clo = closure_pattern(pat)
    assert (clo.stored | ~pat.stored).all() and clo.nvalues > pat.nvalues
    node, orb = entry_coords(pat)
    keep = ~m.dirichlet_mask()[node]
    X = np.zeros((m.ndofs, M))
    X[node[keep], orb[keep]] = rng.standard_normal(keep.sum())
    v = rng.uniform(-1, 1, (m.ncells, (p + 1) ** 3))
    orbs = np.arange(M)
    inside = oapply.block_mask(clo, orbs)
    for which, op in (("H", "H"), ("M", "M")):
        A = _dense_free(m, which, v if which == "H" else None)
        Yd = A @ X
        assert not np.any(Yd[~inside])
        Yo = oapply.masked_apply(clo, v, X, orbs, op=op)
        assert np.abs(Yo - Yd).max() <= 1e-13 * np.abs(Yd).max()
        S = X.T @ Yo
        assert np.abs(S - X.T @ A @ X).max() <= 1e-12 * np.abs(S).max()
        assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    # on the pattern of X itself some of H X is dropped (the reading of the text)
    Yx = oapply.masked_apply(pat, v, X, orbs)
    assert np.abs(X.T @ Yx - X.T @ _dense_free(m, "H", v) @ X).max() > 1e-6


def _full_support_problem(p, cells, M):
    m = BoxMesh(*cells, tuple(float(c) for c in cells), p, 0x3F)
    centres = np.full((M, 3), 0.5) * np.array(m.L)
    pat = build_pattern(m, centres, 1e3, [M // 2, M - M // 2])
    assert pat.stored.all()
    return m, pat


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_energy_at_generalized_eigenvectors(p):
    """Phi = the M lowest M-orthonormal eigenvectors of H u = lambda M u:
    Mbar = I, Hbar = diag(lambda), E = tr((2I - Mbar) Hbar) = sum lambda."""
    from oracle.pattern import closure_pattern
    # Q1 on 4x2x2 cells has only 3 interior nodes: take 4x4x4 there
    m, pat = _full_support_problem(p, (4, 4, 4) if p == 1 else (4, 2, 2), 4)
    v = np.random.default_rng(1).uniform(0, 2, (m.ncells, (p + 1) ** 3))
    free = ~m.dirichlet_mask()
    H = oapply.assemble(m, v, which="H")[np.ix_(free, free)]
    Mm = oapply.assemble(m, which="M")[np.ix_(free, free)]
    lam, U = sla.eigh(H, Mm)
    X = np.zeros((m.ndofs, 4))
    X[free] = U[:, :4]
    clo = closure_pattern(pat)
    orbs = np.arange(4)
    Hbar = X.T @ oapply.masked_apply(clo, v, X, orbs, op="H")
    Mbar = X.T @ oapply.masked_apply(clo, v, X, orbs, op="M")
    assert np.abs(Mbar - np.eye(4)).max() <= 1e-11
    assert np.abs(Hbar - np.diag(lam[:4])).max() <= 1e-10 * lam[3]
    assert abs(oapply.energy(Mbar, Hbar) - lam[:4].sum()) <= 1e-10 * lam[:4].sum()


def test_energy_invariant_under_orthogonal_mixing():
    """E(Phi Q) = E(Phi) for orthogonal Q (eq. energy is a trace of products
    of projected matrices); a transposed or dropped factor breaks it."""
    from oracle.pattern import closure_pattern
    m, pat = _full_support_problem(2, (4, 4, 2), 6)
    rng = np.random.default_rng(7)
    v = rng.uniform(-1, 1, (m.ncells, 27))
    free = ~m.dirichlet_mask()
    X = np.zeros((m.ndofs, 6))
    X[free] = 0.05 * rng.standard_normal((free.sum(), 6))
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    clo = closure_pattern(pat)
    orbs = np.arange(6)

    def E(Xc):
        Hbar = Xc.T @ oapply.masked_apply(clo, v, Xc, orbs, op="H")
        Mbar = Xc.T @ oapply.masked_apply(clo, v, Xc, orbs, op="M")
        return oapply.energy(Mbar, Hbar), Mbar, Hbar

    e1, Mb, Hb = E(X)
    e2, _, _ = E(X @ Q)
    assert abs(e1 - e2) <= 1e-12 * abs(e1)
    assert abs(e1 - (2 * np.trace(Hb) - np.sum(Mb * Hb.T))) <= 1e-12 * abs(e1)


# ---------------------------------------------------------------- gradient (eq. gradient) and Alg. 7
def test_gradient_matches_central_differences_of_the_energy():
    """tr(D^T G) = dE(X + eps D)/d eps for D on the pattern of X (the line-search
    derivative of the text), by central differences of the closure energy."""
    import synth
    from oracle.apply import block_mask
    from oracle.workload import OracleProblem
    ms = synth.MeshSpec(4, 4, 2, (4.0, 4.0, 2.0), 2)
    wl = synth.custom_workload(ms, 6, 1.8, 2, potential="wells", B=3)
    op = OracleProblem(wl, values="generic", value_seed=4)
    op.val = 0.05 * op.val
    G, E0 = op.gradient_dense()
    rng = np.random.default_rng(9)
    mask = block_mask(op.pattern, np.arange(op.M)) & ~op.mesh.dirichlet_mask()[:, None]
    D = np.where(mask, rng.standard_normal(mask.shape), 0.0)
    node, orb = np.nonzero(mask)

    def E_at(eps):
        X = op.X_columns(np.arange(op.M)) + eps * D
        q = OracleProblem.__new__(OracleProblem)
        q.__dict__.update(op.__dict__)
        q.node, q.orb, q.val = node, orb.astype(np.int32), X[node, orb]
        return q.gradient_dense()[1]

    h = 1e-4
    fd = (E_at(h) - E_at(-h)) / (2 * h)
    an = float(np.sum(D * G))
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (fd, an)
    assert abs(E_at(0.0) - E0) <= 1e-12 * abs(E0)


def test_mmult_truncation_brute_force():
    """Alg. 7: entries outside the destination pattern are discarded, entries
    inside equal the full product, element by element."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((40, 9))
    B = rng.standard_normal((9, 9))
    mask = rng.random((40, 9)) < 0.4
    C = oapply.mmult(A, B, mask)
    for i in range(40):
        for j in range(9):
            ref = sum(A[i, k] * B[k, j] for k in range(9)) if mask[i, j] else 0.0
            assert abs(C[i, j] - ref) <= 1e-12 * (1 + abs(ref))


# ---------------------------------------------------------------- curved cells
# Cells given by node positions (isoparametric map).  None of these checks
# restates the element formula: the identity map must reproduce the box
# path, a rigid motion must keep the spectrum (a J^{-1} / J^{-T} mix-up
# changes it by about 15%), an affine shear must keep volumes and kill
# linear functions exactly, and a boundary-preserving interior deformation
# must keep the order-2p convergence of the 1D-box eigenvalues.
def _with_nodes(m, x):
    return BoxMesh(m.nx, m.ny, m.nz, m.L, m.p, m.dirichlet, nodes=x)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_curved_path_on_the_identity_map_equals_box_path(p):
    m = BoxMesh(2, 3, 2, (1.0, 2.0, 0.5), p, 0)
    mc = _with_nodes(m, m.node_points())
    v = np.random.default_rng(2).random((m.ncells, (p + 1) ** 3))
    for which in ("K", "M", "H"):
        a, b = oapply.assemble(m, v, which), oapply.assemble(mc, v, which)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), which
    assert np.abs(m.qp_points() - mc.qp_points()).max() <= 1e-14


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rigid_motion_keeps_the_box_spectrum(p):
    m = BoxMesh(3, 2, 2, (1.0, 1.6, 0.7), p, 0x3F)
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))
    mr = _with_nodes(m, m.node_points() @ Q.T + np.array([0.3, -1.0, 2.0]))
    a, b = _first_eigs(m, 6), _first_eigs(mr, 6)
    assert np.abs(a - b).max() <= 1e-10 * a.max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_affine_shear_keeps_volume_and_kills_linears(p):
    A = np.array([[1.0, 0.3, 0.1], [0.0, 1.0, 0.2], [0.0, 0.0, 1.0]]) * np.array([1.0, 1.0, 1.3])
    m = BoxMesh(2, 3, 2, (1.0, 2.0, 0.5), p, 0)
    ms = _with_nodes(m, m.node_points() @ A.T)
    one = np.ones(ms.ndofs)
    vol = one @ oapply.assemble(ms, which="M") @ one
    assert abs(vol - np.linalg.det(A) * 1.0 * 2.0 * 0.5) <= 1e-13
    K = oapply.assemble(ms, which="K")
    assert np.abs(K @ one).max() < 1e-12
    nc = ms.node_coords()
    interior = np.all((nc > 0) & (nc < np.array(ms.nodes_per_axis) - 1), axis=1)
    x = ms.node_points()
    r = K @ (2 * x[:, 0] - x[:, 1] + 3 * x[:, 2] + 1)
    assert np.abs(r[interior]).max() < 1e-12
    assert np.abs(r[~interior]).max() > 1e-6


@pytest.mark.parametrize("p,ns,rate", [(1, (4, 8, 16), 2.0), (2, (8, 16, 32), 4.0),
                                       (3, (4, 8, 16), 6.0)])
def test_curved_1d_box_eigenvalues_converge_at_2p(p, ns, rate):
    """Dirichlet at x=0 and x=L: the cells are bent along x (x + a sin(2 pi x / L))
    and the cross-section sheared; the domain and the eigenfunctions sin(k pi x / L)
    are unchanged, so lambda_k = pi^2 k^2 / (2 L^2) still holds."""
    L = 1.5
    errs = []
    for nx in ns:
        m = BoxMesh(nx, 1, 1, (L, 0.7, 0.4), p, dirichlet=0b11)
        x = m.node_points().copy()
        x[:, 0] += 0.02 * L * np.sin(2 * np.pi * x[:, 0] / L)
        x[:, 1] += 0.1 * x[:, 2]
        lam = _first_eigs(_with_nodes(m, x), 2)
        exact = np.pi ** 2 * np.array([1, 4]) / (2 * L ** 2)
        errs.append(np.abs(lam - exact) / exact)
    errs = np.array(errs)
    obs = np.log2(errs[:-1, 0] / errs[1:, 0])
    assert np.all(np.abs(obs - rate) < 0.6), obs
