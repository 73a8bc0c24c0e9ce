"""Pins of the adaptive-spacetree oracle (oracle/adaptive.py) to things other than itself.

- A tree refined everywhere is the uniform hierarchy, and the cycle reduces to the uniform
  oracle cycle.
- The level-wise cycle (leaf residuals, bottom-up accumulation, corrections, top-down
  prolongation) equals eq. (adaFACx) written over the generating system with dense matrices.
  Those matrices are built from the hat functions of every level, evaluated at the composite
  vertices.
- The fixed point is the direct solve of the composite system C^T A^leaf C.
- The level diagonals are a(phi, phi) of the level hats in the composite space.
- Hanging values reproduce d-linear functions.
"""
import numpy as np
import pytest

import adafac_inputs as inp
from oracle import adaptive, cycle, hierarchy


def disk_tree(L=4, lu=2, eps=None, d=2, radius=0.2, transfer="dlinear"):
    ref = inp.refine_ball(d, L, lu, (0.5,) * d if d == 2 else (0.45, 0.5, 0.55), radius)
    return adaptive.AdaptiveTree(d, L, 1, lu, ref, eps, transfer=transfer)


@pytest.mark.parametrize("d,L,k", [(2, 3, 0), (2, 3, 1), (3, 2, 1)])
def test_uniform_tree_is_the_uniform_cycle(d, L, k):
    eps = inp.eps_blocks(d, k, 2.0, seed=3) if k else None
    T = adaptive.AdaptiveTree(d, L, 1, L, {}, eps)
    f = inp.rhs(d, L, seed=4)
    U, hist = adaptive.solve(T, f, 6)
    H = hierarchy.Hierarchy(d, L, 1, eps)
    u, ho = cycle.solve(H, H.rhs(f), 6)
    assert np.abs(U[L].ravel() - u).max() <= 1e-14 * np.abs(u).max()
    for a, b in zip(hist, ho):
        assert abs(a[0] - b[0]) <= 1e-14 * ho[0][0]


@pytest.mark.parametrize("d,L,k", [(2, 3, 1), (2, 3, 2), (3, 2, 1), (3, 2, 2)])
def test_uniform_tree_with_boxmg_is_the_uniform_boxmg_cycle(d, L, k):
    """A tree refined everywhere with operator-dependent transfers is the uniform BoxMG
    hierarchy (Sec. 2.5), whose transfers and Galerkin operators are pinned on their own."""
    eps = inp.eps_blocks(d, k, 3.0, seed=12 + k)
    T = adaptive.AdaptiveTree(d, L, 1, L, {}, eps, transfer="boxmg")
    f = inp.rhs(d, L, seed=14)
    U, hist = adaptive.solve(T, f, 6)
    H = hierarchy.Hierarchy(d, L, 1, eps, "boxmg")
    u, ho = cycle.solve(H, H.rhs(f), 6)
    assert np.abs(U[L].ravel() - u).max() <= 1e-12 * np.abs(u).max()
    for a, b in zip(hist, ho):
        assert abs(a[0] - b[0]) <= 1e-12 * ho[0][0]
    # with blocks on level k = 2 the level-1 cells straddle blocks and the transfers differ from
    # d-linear (the d-linear tree gives another iterate); with k = 1 (= l_min) they coincide
    Td = adaptive.AdaptiveTree(d, L, 1, L, {}, eps)
    Ud, _ = adaptive.solve(Td, f, 6)
    gap = np.abs(Ud[L] - U[L]).max()
    if k > 1:
        assert gap > 1e-6 * np.abs(u).max()
    else:
        assert gap <= 1e-12 * np.abs(u).max()


def test_boxmg_disk_tree_transfers_differ_from_dlinear_only_below_the_blocks():
    """On the 2D disk tree with 9 x 9 coefficient blocks, the level-1 cells straddle blocks, so
    the BoxMG prolongation into level 2 is not d-linear; above level 2 every coarse cell lies in
    one block and the two coincide."""
    eps = inp.eps_blocks(2, 2, 3.0, seed=15)
    Tb = disk_tree(L=4, lu=2, eps=eps, transfer="boxmg")
    Td = disk_tree(L=4, lu=2, eps=eps)
    rng = np.random.default_rng(16)
    for l in range(2, 5):
        x = rng.standard_normal(Tb.shape(l - 1)).ravel()
        diff = np.abs(Tb.P[l](x) - Td.P[l](x)).max()
        if l == 2:
            assert diff > 1e-3
        else:
            assert diff == 0.0


def test_tree_classes():
    T = disk_tree()
    for l in range(T.lmin, T.L + 1):
        assert not np.any(T.dof[l] & T.hang[l])
        assert np.all(T.comp[l] <= T.dof[l])
    # uniform levels have no hanging vertices, refined ones do
    assert T.hang[2].sum() == 0 and T.hang[3].sum() > 0 and T.hang[4].sum() > 0
    # every composite dof appears once: positions are distinct
    pos = set()
    for l, i in T.composite_index():
        v = np.array(np.unravel_index(i, T.shape(l))) * 3 ** (T.L - l)
        pos.add(tuple(v))
    assert len(pos) == len(T.composite_index())


@pytest.mark.parametrize("d", [2, 3])
def test_hanging_values_reproduce_dlinear_functions(d):
    T = disk_tree(L=4 if d == 2 else 3, d=d, radius=0.2 if d == 2 else 0.15)
    coef = np.array([0.3, -1.2, 0.7][:d])

    def g(l):
        idx = np.indices(T.shape(l)).astype(float) * 3.0 ** -l        # axis a is coordinate d-1-a
        return 1.0 + sum(coef[d - 1 - a] * idx[a] for a in range(d))

    U = {l: np.where(T.comp[l], g(l), 0.0) for l in range(T.lmin, T.L + 1)}
    U = T.spread(U)
    for l in range(T.lmin, T.L + 1):
        have = T.dof[l] | T.hang[l]
        assert np.abs(U[l][have] - g(l)[have]).max() < 1e-13


@pytest.mark.parametrize("d,L,k", [(2, 3, 0), (2, 3, 2), (3, 2, 1)])
def test_uniform_tree_pi_is_the_uniform_pi_cycle(d, L, k):
    """adAFAC-PI on a tree refined everywhere is the uniform PI cycle (c~_l = P I c_l)."""
    eps = inp.eps_blocks(d, k, 2.0, seed=17) if k else None
    T = adaptive.AdaptiveTree(d, L, 1, L, {}, eps)
    f = inp.rhs(d, L, seed=18)
    U, hist = adaptive.solve(T, f, 6, damping="pi")
    H = hierarchy.Hierarchy(d, L, 1, eps)
    u, ho = cycle.solve(H, H.rhs(f), 6, damping="pi")
    assert np.abs(U[L].ravel() - u).max() <= 1e-13 * np.abs(u).max()
    for a, b in zip(hist, ho):
        assert abs(a[0] - b[0]) <= 1e-13 * ho[0][0]


@pytest.mark.parametrize("d,damping,transfer", [
    (2, "jac", "dlinear"), (2, "none", "dlinear"), (2, "pi", "dlinear"), (2, "jac", "boxmg"), (2, "pi", "boxmg"),
    (3, "jac", "dlinear"), (3, "none", "boxmg"), (3, "pi", "boxmg")])
def test_cycle_equals_dense_generating_system_form(d, damping, transfer):
    if d == 2:
        eps = inp.eps_blocks(2, 2, 2.0, seed=5)
        T = disk_tree(L=4, lu=2, eps=eps, transfer=transfer)
    else:
        T = disk_tree(L=3, lu=2, d=3, radius=0.15, eps=inp.eps_blocks(3, 1, 2.0, seed=6), transfer=transfer)
    f = inp.rhs(d, T.L, seed=7)
    A, b, pos, lev, Psi, C = adaptive.dense_system(T, f)
    bleaf = T.load(f)
    U = {l: np.zeros(T.shape(l)) for l in range(T.lmin, T.L + 1)}
    u = np.zeros(len(b))
    for it in range(4):
        U, nr = adaptive.cycle(T, U, bleaf, damping=damping)
        u, nd = adaptive.dense_cycle(T, A, b, lev, Psi, u, damping=damping)
        uc = adaptive.to_composite(T, U)
        assert np.abs(uc - u).max() <= 1e-12 * np.abs(u).max(), it
        assert abs(nr[0] - nd[0]) <= 1e-12 * nd[0] and abs(nr[1] - nd[1]) <= 1e-12 * nd[1]


@pytest.mark.parametrize("transfer", ["dlinear", "boxmg"])
def test_level_diagonals_are_hat_energies(transfer):
    T = disk_tree(eps=inp.eps_blocks(2, 2, 2.0, seed=8), transfer=transfer)
    A, b, pos, lev, Psi, C = adaptive.dense_system(T, inp.rhs(2, 4, seed=9))
    for l in range(T.lmin, T.L + 1):
        D = T.D[l].ravel()[np.flatnonzero(T.dof[l].ravel())]
        E = np.einsum("ij,ij->j", Psi[l], A @ Psi[l])
        assert np.abs(D - E).max() <= 1e-12 * D.max(), l


def test_fixed_point_is_the_composite_direct_solve():
    T = disk_tree(eps=inp.eps_blocks(2, 2, 1.0, seed=10))
    f = inp.rhs(2, 4, seed=11)
    A, b, pos, lev, Psi, C = adaptive.dense_system(T, f)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A)[0] > 0
    ustar = np.linalg.solve(A, b)
    U, hist = adaptive.solve(T, f, 400, tol=1e-13)
    u = adaptive.to_composite(T, U)
    assert hist[-1][0] / hist[0][0] <= 1e-13
    assert np.linalg.norm(u - ustar) <= 1e-9 * np.linalg.norm(ustar)


def test_finest_values_are_the_composite_function():
    T = disk_tree()
    U, _ = adaptive.solve(T, inp.rhs(2, 4, seed=12), 3)
    F = adaptive.finest_values(T, U)
    # at every composite dof the finest-lattice value is the dof's value
    for l, i in T.composite_index():
        v = np.array(np.unravel_index(i, T.shape(l))) * 3 ** (T.L - l)
        assert F[tuple(v)] == U[l].ravel()[i]


def test_transfer_keeps_the_composite_function_where_both_trees_resolve_it():
    T1 = disk_tree()
    ref2 = inp.refine_ball(2, 4, 2, (0.6, 0.45), 0.2)
    T2 = adaptive.AdaptiveTree(2, 4, 1, 2, ref2)
    U1, _ = adaptive.solve(T1, inp.rhs(2, 4, seed=13), 3)
    U2 = adaptive.transfer(T1, U1, T2)
    F1, F2 = adaptive.finest_values(T1, U1), adaptive.finest_values(T2, U2)
    # vertices that are composite dofs of both trees on the same level keep their value
    for l in range(T2.lmin, T2.L + 1):
        both = T1.comp[l] & T2.comp[l]
        assert np.array_equal(U2[l][both], U1[l][both])
    # the transferred function is the old one sampled at the new dofs and interpolated between
    # them: wherever the new tree is at least as fine as the old one, the two agree
    fine_both = T1.dof[4] & T2.dof[4]
    assert np.abs(F1[fine_both] - F2[fine_both]).max() == 0.0


@pytest.mark.parametrize("d", [2, 3])
def test_defect_correction_with_fp64_inner_cycles_is_the_plain_iteration(d):
    # the cycle is linear in (u, b): k cycles on A e = r from e = 0 added to u give the k-th
    # iterate of the plain iteration started at u
    T = disk_tree(eps=inp.eps_blocks(2, 2, 2.0, seed=14)) if d == 2 else \
        disk_tree(L=3, lu=2, d=3, radius=0.15, eps=inp.eps_blocks(3, 1, 2.0, seed=15))
    f = inp.rhs(d, T.L, seed=16)
    k, steps = 3, 4
    its = []
    U, hist = adaptive.defect_correction(T, f, k, 0.0, steps, inner_dtype=np.float64, iterates=its)
    Up, hp = adaptive.solve(T, f, k * steps + 1)
    assert len(hist) == steps + 1
    for n in range(steps + 1):
        assert abs(hist[n][0] - hp[n * k][0]) <= 1e-11 * hp[0][0], n
    Fd, Fp = adaptive.finest_values(T, U), adaptive.finest_values(T, adaptive.solve(T, f, k * steps)[0])
    assert np.abs(Fd - Fp).max() <= 1e-11 * np.abs(Fp).max()


def test_defect_correction_with_fp32_inner_cycles_reaches_fp64_accuracy():
    T = disk_tree(eps=inp.eps_blocks(2, 2, 1.0, seed=17))
    f = inp.rhs(2, 4, seed=18)
    A, b, pos, lev, Psi, C = adaptive.dense_system(T, f)
    ustar = np.linalg.solve(A, b)
    U, hist = adaptive.defect_correction(T, f, 4, 1e-12, 100, inner_dtype=np.float32)
    assert hist[-1][0] / hist[0][0] <= 1e-12          # far below FP32 resolution
    u = adaptive.to_composite(T, U)
    assert np.linalg.norm(u - ustar) <= 1e-9 * np.linalg.norm(ustar)
    # the inner arrays really are FP32: a single outer step is off from FP64 by FP32 rounding
    _, h32 = adaptive.defect_correction(T, f, 4, 0.0, 1, inner_dtype=np.float32)
    _, h64 = adaptive.defect_correction(T, f, 4, 0.0, 1, inner_dtype=np.float64)
    gap = abs(h32[1][0] - h64[1][0]) / h64[0][0]
    assert 1e-10 < gap < 1e-4


# --- the lumped load and the composite discretisation at refinement interfaces -------------

@pytest.mark.parametrize("d", [2, 3])
def test_load_of_unit_source_is_the_integral_of_each_composite_hat(d):
    """With f = 1 the lumped load of a composite dof is the integral of its composite hat (on a
    leaf cell K every corner hat integrates to |K| / 2^d, hanging corners included through
    their interpolation weights).  The integral is taken independently of the load: the hat is
    spread to the finest lattice, where it is d-linear on every finest cell, so the trapezoidal
    rule h_L^d sum_v phi(v) is exact."""
    T = disk_tree(L=4, lu=2) if d == 2 else disk_tree(L=3, lu=2, d=3, radius=0.15)
    rh, _ = adaptive.composite_residual(
        T, {l: np.zeros(T.shape(l)) for l in range(T.lmin, T.L + 1)}, T.load(np.ones(T.shape(T.L))))
    hL = 3.0 ** -T.L
    idx = T.composite_index()
    # every composite dof near a refinement interface, and a sample of the others
    near = [j for j, (l, i) in enumerate(idx) if l < T.L]
    pick = sorted(set(near + list(range(0, len(idx), max(1, len(idx) // 50)))))
    for j in pick:
        l, i = idx[j]
        U = {m: np.zeros(T.shape(m)) for m in range(T.lmin, T.L + 1)}
        U[l].ravel()[i] = 1.0
        phi = adaptive.finest_values(T, T.spread(U))
        integral = hL ** d * phi.sum()
        assert abs(rh[l].ravel()[i] - integral) <= 1e-14 * 3.0 ** (-l * d), (l, i)


def _sparse_composite_system(T, f):
    """A_h = sum_l C_l^T A^leaf_l C_l and b_h = sum_l C_l^T b^leaf_l with sparse C_l, built
    level by level: dof rows select the composite dof at that position, hanging rows take the
    d-linear interpolation of the coarser level's rows (Sec. 2.1)."""
    import scipy.sparse as sp
    from oracle import fem, transfer
    d, L = T.d, T.L
    idx = T.composite_index()
    n = len(idx)
    where = {}
    for j, (l, i) in enumerate(idx):
        v = np.array(np.unravel_index(i, T.shape(l))) * 3 ** (L - l)
        where[tuple(v)] = j
    C = {}
    for l in range(T.lmin, L + 1):
        N = int(np.prod(T.shape(l)))
        dofs = np.flatnonzero(T.dof[l].ravel())
        cols = [where[tuple(np.array(np.unravel_index(i, T.shape(l))) * 3 ** (L - l))] for i in dofs]
        Cl = sp.csr_matrix((np.ones(len(dofs)), (dofs, cols)), shape=(N, n))
        if l > T.lmin:
            hang = sp.diags(T.hang[l].ravel().astype(float))
            Cl = Cl + hang @ transfer.dlinear_prolongation(d, l) @ C[l - 1]
        C[l] = Cl.tocsr()
    bleaf = T.load(f)
    A = sp.csr_matrix((n, n))
    b = np.zeros(n)
    for l in range(T.lmin, L + 1):
        if np.any(T.leaf_eps[l]):
            A = A + C[l].T @ fem.assemble(T.leaf_eps[l]) @ C[l]
        b += C[l].T @ bleaf[l].ravel()
    pos = np.array([np.array(np.unravel_index(i, T.shape(l)))[::-1] * 3.0 ** -l for l, i in idx])
    return A.tocsr(), b, pos


def test_sparse_composite_system_is_the_dense_one():
    T = disk_tree(eps=inp.eps_blocks(2, 2, 1.0, seed=19))
    f = inp.rhs(2, 4, seed=20)
    A, b, pos, lev, Psi, C = adaptive.dense_system(T, f)
    As, bs, ps = _sparse_composite_system(T, f)
    assert np.abs(As.toarray() - A).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(bs - b).max() <= 1e-15 * np.abs(b).max()
    assert np.array_equal(ps, pos)


def test_manufactured_solution_converges_at_second_order_on_disk_trees():
    """u* = sin(pi x) sin(pi y), f = 2 pi^2 u*, on trees uniform to level lu and refined around
    a disk two levels further: the composite solution's maximum error at the dofs falls by
    about 3^2 per level (second order in the coarsest mesh width; a load that is wrong at the
    refinement interfaces would leave a first-order error there)."""
    import scipy.sparse.linalg as spla
    errs = []
    for lu in (2, 3, 4):
        L = lu + 2
        ref = inp.refine_ball(2, L, lu, (0.5, 0.5), 0.25)
        T = adaptive.AdaptiveTree(2, L, 1, lu, ref)
        n = 3 ** L
        y, x = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n, indexing="ij")
        f = 2 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y)
        A, b, pos = _sparse_composite_system(T, f)
        u = spla.spsolve(A.tocsc(), b)
        ustar = np.sin(np.pi * pos[:, 0]) * np.sin(np.pi * pos[:, 1])
        errs.append(np.abs(u - ustar).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(6.0 < r < 13.0 for r in ratios), (errs, ratios)


# --- inhomogeneous Dirichlet data on adaptive trees (the set-ups of Sec. 5) -------------------

def _bilinear(d, L):
    """A harmonic d-linear function on the finest lattice (x fastest): x y + 2x - y + 1/2 in 2D,
    x y z + x - z + 1/4 in 3D."""
    x = np.linspace(0.0, 1.0, 3 ** L + 1)
    if d == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        return X * Y + 2 * X - Y + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X * Y * Z + X - Z + 0.25


@pytest.mark.parametrize("d,L,lu", [(2, 4, 2), (3, 3, 1)])
def test_dirichlet_bilinear_data_is_reproduced_on_refined_trees(d, L, lu):
    """f = 0 with the boundary values of a harmonic d-linear p: p lies in the composite space
    (continuous Q1 on the leaf cells; hanging vertices interpolate d-linearly), so the discrete
    solution is p itself at every dof, whatever the tree."""
    p = _bilinear(d, L)
    ref = inp.refine_ball(d, L, lu, (0.5,) * d if d == 2 else (0.45, 0.5, 0.55), 0.2)
    T = adaptive.AdaptiveTree(d, L, 1, lu, ref, g=p)
    U, hist = adaptive.solve(T, np.zeros_like(p), 400, tol=1e-13)
    assert hist[-1][0] / hist[0][0] <= 1e-13
    for l in range(1, L + 1):
        pl = p[tuple(slice(None, None, 3 ** (L - l)) for _ in range(d))]
        m = T.dof[l] | T.hang[l] | T.bnd[l]
        assert np.abs(U[l][m] - pl[m]).max() <= 1e-10, l
    # the finest-lattice composite function is p wherever the tree has cells
    F = adaptive.finest_values(T, U)
    assert np.abs(F - p).max() <= 1e-10


@pytest.mark.parametrize("d,L,field", [(2, 3, "split"), (2, 3, "homogeneous"), (3, 2, "homogeneous")])
def test_dirichlet_uniform_tree_is_the_lifted_uniform_cycle(d, L, field):
    """A tree refined everywhere with the Sec. 5 boundary data (u = 1 on x_2 = 0) runs the
    uniform cycle on the lifted problem, A u_0 = b - A G, with u = u_0 + G."""
    g = inp.paper_boundary(d, L)
    eps = None if field == "homogeneous" else inp.eps_blocks(d, 1, 2.0, seed=9)
    T = adaptive.AdaptiveTree(d, L, 1, L, {}, eps, g=g)
    U, hist = adaptive.solve(T, np.zeros_like(g), 8)
    H = hierarchy.Hierarchy(d, L, 1, eps)
    u0, ho = cycle.solve(H, H.rhs(np.zeros_like(g), g=g), 8)
    from oracle import fem
    u = fem.with_boundary(u0, g)
    assert np.abs(U[L] - u).max() <= 1e-13 * np.abs(u).max()
    for a, b in zip(hist, ho):
        assert abs(a[0] - b[0]) <= 1e-13 * ho[0][0]


def test_dirichlet_defect_correction_with_fp64_inner_cycles_is_the_plain_iteration():
    """The inner cycles solve the correction equation with zero boundary values: with FP64 inner
    cycles, k inner cycles per outer step equal k plain cycles on u."""
    d, L = 2, 4
    g = inp.paper_boundary(d, L)
    T = disk_tree(L=L)
    T = adaptive.AdaptiveTree(d, L, 1, 2, inp.refine_ball(d, L, 2, (0.5, 0.5), 0.2), g=g)
    its = []
    U, h = adaptive.defect_correction(T, np.zeros_like(g), 3, 0.0, 2, inner_dtype=np.float64, iterates=its)
    Up, hp = adaptive.solve(T, np.zeros_like(g), 6)
    assert abs(h[0][0] - hp[0][0]) <= 1e-13 * hp[0][0]
    for l in range(1, L + 1):
        assert np.abs(U[l] - Up[l]).max() <= 1e-12 * max(1.0, np.abs(Up[l]).max())


def test_upsample_reproduces_dlinear_functions():
    """The whole-lattice d-linear interpolation used for boundary traces is exact on d-linear
    functions, boundary included."""
    for d, L in ((2, 2), (3, 2)):
        p_c = _bilinear(d, L - 1)
        p_f = _bilinear(d, L)
        assert np.abs(adaptive._upsample(p_c) - p_f).max() <= 1e-14
