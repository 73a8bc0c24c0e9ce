"""Pins of the FP64 oracle to facts outside itself.

Each test checks the oracle against something the paper or the mathematics
fixes: closed-form element matrices and stencils, the paper's printed
smoothed-operator table, the defining equations of BoxMG, the Galerkin
identity, the cycle written as the explicit sum of eq. (adaFACx) with dense
matrix powers, textbook reductions (one level = damped Jacobi, no damping =
eq. (additive-mg)), the direct solve as fixed point, the asymptotic rate as
the spectral radius of the iteration matrix, and the O(h^2) error of a
manufactured solution.
"""
import itertools
import os

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import cycle, dense, fem, hierarchy, transfer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- Q1 elements and stencils (Sec. 2.1) -------------------------------------

def test_ref_stiffness_closed_form_2d():
    # textbook bilinear element on the unit square: 2/3 diagonal, -1/6 across an edge, -1/3 across the diagonal
    K = fem.ref_stiffness(2)
    for i, j in itertools.product(range(4), repeat=2):
        nd = bin(i ^ j).count("1")
        assert K[i, j] == pytest.approx({0: 2 / 3, 1: -1 / 6, 2: -1 / 3}[nd], abs=1e-15)


def test_ref_stiffness_closed_form_3d():
    # trilinear element on the unit cube: 1/3 diagonal, 0 along an edge, -1/12 face and body diagonals
    K = fem.ref_stiffness(3)
    for i, j in itertools.product(range(8), repeat=2):
        nd = bin(i ^ j).count("1")
        assert K[i, j] == pytest.approx({0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[nd], abs=1e-15)


@pytest.mark.parametrize("level,eps", [(2, 1.0), (3, 7.5)])
def test_assembled_stencil_2d(level, eps):
    A = fem.assemble(np.full((3 ** level,) * 2, eps))
    n = 3 ** level
    c = (n // 2, n // 2)
    row = A.getrow(np.ravel_multi_index(c, (n + 1,) * 2)).toarray().reshape((n + 1,) * 2)
    st = row[c[0] - 1:c[0] + 2, c[1] - 1:c[1] + 2]
    expect = eps / 3.0 * np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]])
    assert np.allclose(st, expect, rtol=0, atol=1e-14 * eps)


@pytest.mark.parametrize("level,eps", [(2, 1.0), (3, 0.25)])
def test_assembled_stencil_3d(level, eps):
    A = fem.assemble(np.full((3 ** level,) * 3, eps))
    n = 3 ** level
    h = 1.0 / n
    c = (n // 2,) * 3
    row = A.getrow(np.ravel_multi_index(c, (n + 1,) * 3)).toarray().reshape((n + 1,) * 3)
    st = row[tuple(slice(x - 1, x + 2) for x in c)]
    for o in itertools.product((-1, 0, 1), repeat=3):
        nz = sum(1 for x in o if x)
        want = eps * h * {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[nz]
        assert st[tuple(x + 1 for x in o)] == pytest.approx(want, abs=1e-15)


@pytest.mark.parametrize("d,level", [(2, 3), (3, 2)])
def test_assembled_interior_rows_sum_to_exactly_zero(d, level):
    """A constant is in the kernel of the Q1 operator away from the boundary; with correctly
    rounded element entries the assembled interior rows of the Poisson operator sum to zero in
    exact arithmetic on the stored doubles (no artificial zero-order term)."""
    import math
    A = fem.assemble(np.ones((3 ** level,) * d)).tocsr()
    m = fem.interior_mask(d, level)
    far = np.zeros_like(m)
    far[(slice(2, -2),) * d] = True
    for i in np.flatnonzero(far.ravel()):
        row = A.data[A.indptr[i]:A.indptr[i + 1]]
        assert math.fsum(row) == 0.0, i


@pytest.mark.parametrize("d,L,k", [(2, 3, 2), (3, 2, 1), (3, 2, 2)])
def test_matrix_free_equals_assembled(d, L, k):
    eps = fem.cell_eps_from_blocks(inp.eps_blocks(d, k, 3.0, seed=3), L)
    A = fem.assemble(eps)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((3 ** L + 1,) * d) * fem.interior_mask(d, L)
    assert np.allclose(fem.apply_matrix_free(u, eps).ravel(), A @ u.ravel(), rtol=0, atol=1e-12)


def test_lumped_rhs_uniform():
    f = inp.rhs(3, 2, seed=5)
    b = fem.lumped_rhs(f, 2)
    m = fem.interior_mask(3, 2)
    assert np.allclose(b[m], (1 / 9) ** 3 * f[m], rtol=1e-15)
    assert np.all(b[~m] == 0)


# --- transfers (Sec. 2.5) ----------------------------------------------------

@pytest.mark.parametrize("d,l", [(2, 3), (3, 2)])
def test_dlinear_reproduces_multilinear(d, l):
    P = transfer.dlinear_prolongation(d, l)
    nc = 3 ** (l - 1)
    xc = np.indices((nc + 1,) * d) / nc
    xf = np.indices((3 * nc + 1,) * d) / (3 * nc)
    g = lambda x: 1.0 + np.sum([(a + 1) * x[a] for a in range(d)], axis=0) + np.prod(x, axis=0)
    fine = (P @ (g(xc) * fem.interior_mask(d, l - 1)).ravel()).reshape(xf.shape[1:])
    # fine vertices whose coarse cell has only interior corners
    ok = np.all((xf * nc >= 1) & (xf * nc <= nc - 1), axis=0)
    assert ok.sum() > 0
    assert np.allclose(fine[ok], g(xf)[ok], rtol=1e-14)


@pytest.mark.parametrize("d,l", [(2, 3), (3, 2)])
def test_boxmg_constant_eps_is_dlinear(d, l):
    # Sec. 5.1: BoxMG gives bilinear transfers for Poisson
    A = fem.assemble(np.full((3 ** l,) * d, 4.0))
    Pb = transfer.boxmg_prolongation(A, d, l)
    Pd = transfer.dlinear_prolongation(d, l)
    assert abs(Pb - Pd).max() < 1e-14


@pytest.mark.parametrize("d,l,k", [(2, 4, 2), (2, 3, 2), (3, 3, 2)])
def test_boxmg_is_dlinear_where_coarse_cells_lie_in_one_block(d, l, k):
    # eps constant on every coarse cell and along every coarse face: the collapsed 1D/2D problems
    # and the cell-interior problem have the d-linear interpolant as their solution
    eps = fem.cell_eps_from_blocks(inp.eps_blocks(d, k, 4.0, seed=17), l)
    Pb = transfer.boxmg_prolongation(fem.assemble(eps), d, l)
    assert abs(Pb - transfer.dlinear_prolongation(d, l)).max() < 1e-13


def _boxmg_equations_hold(d, l, eps_cells):
    """Check the defining equations of Sec. 2.5 on every column of P."""
    A = fem.assemble(eps_cells).tocsr()
    P = transfer.boxmg_prolongation(A, d, l).toarray()
    nf = 3 ** l
    fshape = (nf + 1,) * d
    fm = fem.interior_mask(d, l)
    cm = fem.interior_mask(d, l - 1)
    Ad = A.toarray()
    worst = 0.0
    for ci in np.flatnonzero(cm.ravel()):
        col = P[:, ci].reshape(fshape)
        cv = np.unravel_index(ci, cm.shape)
        for g in zip(*np.nonzero(fm)):
            res = [x % 3 for x in g]
            free = [a for a in range(d) if res[a] != 0]
            if not free:          # c-point: identity
                want = 1.0 if tuple(x // 3 for x in g) == cv else 0.0
                worst = max(worst, abs(col[g] - want))
                continue
            # only points inside the support of this coarse vertex's cells
            if any(abs(g[a] - 3 * cv[a]) >= 3 for a in range(d)):
                assert col[g] == 0.0
                continue
            row = Ad[np.ravel_multi_index(g, fshape)].reshape(fshape)
            s = 0.0
            for o in itertools.product((-1, 0, 1), repeat=d):
                w = tuple(g[a] + o[a] for a in range(d))
                if any(x < 0 or x > nf for x in w):
                    continue
                # collapsed equation: lump the normal directions, i.e. the neighbour's value is
                # taken at the point's own coordinate along every fixed (normal) axis
                q = tuple(w[a] if a in free else g[a] for a in range(d))
                s += row[w] * col[q]
            worst = max(worst, abs(s) / np.abs(row).sum())
    return worst


def test_boxmg_defining_equations_2d():
    eps = fem.cell_eps_from_blocks(inp.eps_blocks(2, 2, 3.0, seed=7), 2)
    assert _boxmg_equations_hold(2, 2, eps) < 1e-13


@pytest.mark.slow
def test_boxmg_defining_equations_3d():
    eps = fem.cell_eps_from_blocks(inp.eps_blocks(3, 2, 4.0, seed=8), 2)
    assert _boxmg_equations_hold(3, 2, eps) < 1e-12


def test_boxmg_rows_sum_to_one_away_from_boundary():
    # constants lie in the kernel of interior stencils, so interpolation reproduces them
    d, l = 2, 3
    eps = fem.cell_eps_from_blocks(inp.eps_blocks(2, 2, 3.0, seed=2), l)
    P = transfer.boxmg_prolongation(fem.assemble(eps), d, l)
    nc = 3 ** (l - 1)
    rows = np.asarray(P.sum(axis=1)).reshape((3 * nc + 1,) * d)
    x = np.indices(rows.shape)
    ok = np.all((x >= 3) & (x <= 3 * nc - 3), axis=0)
    assert np.allclose(rows[ok], 1.0, atol=1e-13)


@pytest.mark.parametrize("d,lf", [(2, 3), (3, 2)])
def test_galerkin_of_constant_eps_is_rediscretisation(d, lf):
    # Sec. 5.1: Ritz-Galerkin gives the rediscretised operator for Poisson (3D: proportional to h)
    A = fem.assemble(np.ones((3 ** lf,) * d))
    P = transfer.dlinear_prolongation(d, lf)
    Ac = (P.T @ A @ P).toarray()
    Ar = fem.assemble(np.ones((3 ** (lf - 1),) * d)).toarray()
    assert np.abs(Ac - Ar).max() < 1e-14
    if d == 3:
        n = 3 ** (lf - 1)
        c = np.ravel_multi_index((n // 2,) * 3, (n + 1,) * 3)
        assert Ac[c, c] == pytest.approx(3 * 8 / 3 / (3 ** lf), rel=1e-14)


def test_galerkin_of_block_eps_is_rediscretisation_where_blocks_are_coarse():
    eps = inp.eps_blocks(2, 2, 3.0, seed=4)
    H = hierarchy.Hierarchy(2, 4, 1, eps, "boxmg")
    for l in (2, 3):   # coarse cells inside one block: Galerkin = Q1 with that block's eps
        Ar = fem.assemble(fem.cell_eps_from_blocks(eps, l))
        assert abs(H.lev[l].A.mat - Ar).max() < 1e-12 * abs(Ar).max()


# --- smoothed auxiliary restriction (Sec. 3.2) -------------------------------

def _golden_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "smoothed_operator_2d.txt")) if not l.startswith("#")]
    return np.array([[float(x) for x in r] for r in rows if r])


def test_smoothed_operator_matches_printed_table():
    T = hierarchy.smoothed_operator_eps1(2)
    G = _golden_table()
    assert G.shape == (7, 7)
    # printed to 3-4 significant digits; one entry printed as -0.083 for -0.0833
    assert np.abs(T - G).max() < 5e-4
    exact = np.array([[-1, -3, -6, -7, -6, -3, -1], [-3, 0, 0, 6, 0, 0, -3], [-6, 0, 0, 12, 0, 0, -6],
                      [-7, 6, 12, 32, 12, 6, -7], [-6, 0, 0, 12, 0, 0, -6], [-3, 0, 0, 6, 0, 0, -3],
                      [-1, -3, -6, -7, -6, -3, -1]]) / 72.0
    assert np.abs(T - exact).max() < 1e-15


def test_smoothed_operator_3d_symmetry_and_zero_sum():
    # A annihilates constants and P reproduces them, so the full 7^3 stencil sums to zero
    T = hierarchy.smoothed_operator_eps1(3)
    assert abs(T.sum()) < 1e-13
    for perm in itertools.permutations(range(3)):
        assert np.allclose(T, np.transpose(T, perm), atol=1e-15)
    assert np.allclose(T, T[::-1], atol=1e-15)
    # the dropped ring (offset 3 along some axis) holds no positive entry
    ring = np.ones(T.shape, bool)
    ring[1:6, 1:6, 1:6] = False
    assert np.all(T[ring] <= 1e-15)


def test_smoothed_operator_3d_exact_values():
    """The 7^3 stencil of M^-1 A P at eps = 1 in closed form.  The 3D Q1 operator is
    h sum_a K1(a) M1(b) M1(c) with the 1D stiffness K1 = [-1 2 -1] / h and mass
    M1 = h [1 4 1] / 6, the coarse hat is the tensor product of the 1D hat
    p = (1/3, 2/3, 1, 2/3, 1/3), and M = diag(A) = 8h/3.  So the entry at offset o is
    (3/8) sum_a k(o_a) m(o_b) m(o_c) with k = K1 p = {0: 2/3, +-3: -1/3} and
    m = M1 p = {0: 8/9, +-1: 2/3, +-2: 1/3, +-3: 1/18}: inside |o| <= 2 only the planar terms
    survive (16/27 at the centre, 8/27 and 4/27 on the axes, 1/9, 1/18, 1/36 in the
    coordinate planes, 61 nonzeros summing to 169/27)."""
    from fractions import Fraction as Fr
    k = {0: Fr(2, 3), 3: Fr(-1, 3)}
    m = {0: Fr(8, 9), 1: Fr(2, 3), 2: Fr(1, 3), 3: Fr(1, 18)}
    T = hierarchy.smoothed_operator_eps1(3)
    for o in itertools.product(range(-3, 4), repeat=3):
        a = [abs(v) for v in o]
        e = Fr(3, 8) * sum(k.get(a[i], Fr(0)) * m[a[(i + 1) % 3]] * m[a[(i + 2) % 3]] for i in range(3))
        assert abs(T[tuple(v + 3 for v in o)] - float(e)) < 1e-15, o
    core = T[1:6, 1:6, 1:6]
    assert np.count_nonzero(np.abs(core) > 1e-15) == 61
    assert abs(core.sum() - 169.0 / 27.0) < 1e-13
    want = {(0, 0, 0): Fr(16, 27), (1, 0, 0): Fr(8, 27), (2, 0, 0): Fr(4, 27), (1, 1, 0): Fr(1, 9),
            (2, 1, 0): Fr(1, 18), (2, 2, 0): Fr(1, 36), (1, 1, 1): Fr(0), (2, 2, 2): Fr(0)}
    for o, v in want.items():
        for q in itertools.permutations(o):
            assert abs(T[tuple(x + 3 for x in q)] - float(v)) < 1e-15


def test_rtilde_const_is_truncated_omega_scaled_table():
    H = hierarchy.Hierarchy(2, 3, 1, None, "dlinear", "const", omega=0.6)
    Rt = H.lev[3].Rt.mat.toarray()
    nc, nf = 10, 28
    c = np.ravel_multi_index((4, 5), (nc,) * 2)
    row = Rt[c].reshape((nf,) * 2)
    core = 0.6 * np.array([[0, 0, 6, 0, 0], [0, 0, 12, 0, 0], [6, 12, 32, 12, 6],
                           [0, 0, 12, 0, 0], [0, 0, 6, 0, 0]]) / 72.0
    assert np.allclose(row[10:15, 13:18], core, atol=1e-15)
    assert abs(row.sum() - core.sum()) < 1e-14


def test_rtilde_operator_equals_const_for_poisson_interior():
    Hc = hierarchy.Hierarchy(2, 3, 1, None, "dlinear", "const")
    Ho = hierarchy.Hierarchy(2, 3, 1, None, "dlinear", "operator")
    a, b = Hc.lev[3].Rt.mat.toarray(), Ho.lev[3].Rt.mat.toarray()
    c = np.ravel_multi_index((4, 4), (10, 10))
    assert np.allclose(a[c], b[c], atol=1e-14)


# --- the cycle (Sec. 3.1, eq. (adaFACx), Algorithms 1-2) ---------------------

def _dense_ops(H):
    ops = {}
    for l in range(H.lmin, H.L + 1):
        lv = H.lev[l]
        o = {"Dinv": np.diag(lv.Dinv)}
        if l > H.lmin:
            o["P"] = lv.P.mat.toarray()
            o["I"] = lv.I.mat.toarray()
            o["Rt"] = lv.Rt.mat.toarray()
        ops[l] = o
    return ops


def _Ppow(ops, l, L):
    """P^{L-l}: prolongation from level l to level L as one dense matrix."""
    n = ops[l]["Dinv"].shape[0]
    M = np.eye(n)
    for j in range(l + 1, L + 1):
        M = ops[j]["P"] @ M
    return M


def _setup(d, L, seed, kind="dlinear", k=0):
    eps = inp.eps_blocks(d, k, 3.0, seed) if k else None
    H = hierarchy.Hierarchy(d, L, 1, eps, kind)
    rng = np.random.default_rng(seed)
    m = H.lev[L].mask.ravel()
    u = rng.standard_normal(m.size) * m
    b = rng.standard_normal(m.size) * m
    return H, u, b


@pytest.mark.parametrize("form", ["correction", "fas"])
def test_single_level_is_damped_jacobi(form):
    H = hierarchy.Hierarchy(2, 2, 2)
    rng = np.random.default_rng(0)
    m = H.lev[2].mask.ravel()
    u, b = rng.standard_normal(m.size) * m, rng.standard_normal(m.size) * m
    A = H.lev[2].A.mat.toarray()
    D = np.diag(A)
    want = u + 0.6 * np.where(m, 1 / np.where(m, D, 1), 0) * (b - A @ u)
    f = cycle.cycle_fas if form == "fas" else cycle.cycle_correction
    assert np.allclose(f(H, u, b)[0], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("d,L,kind,k", [(2, 3, "dlinear", 0), (2, 3, "boxmg", 2), (3, 2, "boxmg", 1)])
def test_cycle_equals_explicit_adafacx_sum(d, L, kind, k):
    """u + [sum_l P^{L-l} w D_l^-1 R^{L-l} - sum_{l<L} w~ P^{L-l} D_l^-1 R~ R^{L-l-1}] (b - A u)."""
    H, u, b = _setup(d, L, 11, kind, k)
    ops = _dense_ops(H)
    A = H.lev[L].A.mat.toarray()
    r = b - A @ u
    w, wt = 0.6, 0.6
    M = np.zeros_like(A)
    for l in range(H.lmin, L + 1):
        Pp = _Ppow(ops, l, L)
        M += Pp @ (w * ops[l]["Dinv"]) @ Pp.T
    for l in range(H.lmin, L):
        Pp = _Ppow(ops, l, L)
        Rrest = _Ppow(ops, l + 1, L).T
        M -= wt * Pp @ ops[l]["Dinv"] @ ops[l + 1]["Rt"] @ Rrest
    want = u + M @ r
    for f in (cycle.cycle_correction, cycle.cycle_fas):
        got = f(H, u, b)[0]
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_no_damping_is_plain_additive_multigrid():
    H, u, b = _setup(2, 3, 12)
    ops = _dense_ops(H)
    A = H.lev[3].A.mat.toarray()
    M = sum(_Ppow(ops, l, 3) @ (0.6 * ops[l]["Dinv"]) @ _Ppow(ops, l, 3).T for l in range(1, 4))
    want = u + M @ (b - A @ u)
    got = cycle.cycle_correction(H, u, b, damping="none")[0]
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # omega~ = 0 reduces adAFAC-Jac to the same scheme
    assert np.allclose(cycle.cycle_correction(H, u, b, omega_t=0.0)[0], got, atol=1e-14)


def test_pi_damping_is_hierarchical_surplus_of_each_correction():
    """adAFAC-PI: every level but the coarsest contributes (id - P I) of its Jacobi correction."""
    H, u, b = _setup(2, 3, 13)
    ops = _dense_ops(H)
    A = H.lev[3].A.mat.toarray()
    M = _Ppow(ops, 1, 3) @ (0.6 * ops[1]["Dinv"]) @ _Ppow(ops, 1, 3).T
    for l in (2, 3):
        n = ops[l]["Dinv"].shape[0]
        surplus = np.eye(n) - ops[l]["P"] @ ops[l]["I"]
        M += _Ppow(ops, l, 3) @ surplus @ (0.6 * ops[l]["Dinv"]) @ _Ppow(ops, l, 3).T
    want = u + M @ (b - A @ u)
    for f in (cycle.cycle_correction, cycle.cycle_fas):
        assert np.abs(f(H, u, b, damping="pi")[0] - want).max() < 1e-12 * np.abs(want).max()


def test_exponential_damping():
    H, u, b = _setup(2, 3, 14)
    ops = _dense_ops(H)
    A = H.lev[3].A.mat.toarray()
    M = sum(0.7 ** (3 - l) * _Ppow(ops, l, 3) @ (0.6 * ops[l]["Dinv"]) @ _Ppow(ops, l, 3).T
            for l in range(1, 4))
    want = u + M @ (b - A @ u)
    got = cycle.cycle_correction(H, u, b, damping="exp", omega_hat=0.7)[0]
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("d,L,kind,k", [(2, 4, "dlinear", 0), (2, 3, "boxmg", 2), (3, 3, "dlinear", 0)])
def test_fas_form_equals_correction_form(d, L, kind, k):
    eps = inp.eps_blocks(d, k, 3.0, 5) if k else None
    H = hierarchy.Hierarchy(d, L, 1, eps, kind)
    b = H.rhs(inp.rhs(d, L, 6))
    u1, h1 = cycle.solve(H, b, 8, form="correction")
    u2, h2 = cycle.solve(H, b, 8, form="fas")
    assert np.abs(u1 - u2).max() < 1e-12 * np.abs(u1).max()
    for a, c in zip(h1, h2):
        assert abs(a[0] - c[0]) < 1e-12 * h1[0][0]


@pytest.mark.parametrize("damping", ["jac", "pi"])
def test_fixed_point_is_direct_solve(damping):
    # Sec. 5.1: the stable variants are real solvers and converge to the same solution
    H = hierarchy.Hierarchy(2, 3, 1, inp.eps_blocks(2, 2, 2.0, 9), "boxmg")
    b = H.rhs(inp.rhs(2, 3, 9))
    us = dense.direct_solve(H, b)
    u, hist = cycle.solve(H, b, 400, tol=1e-11, damping=damping)
    assert hist[-1][0] / hist[0][0] <= 1e-11
    assert np.abs(u - us).max() < 1e-10 * np.abs(us).max()


def test_asymptotic_rate_matches_iteration_matrix():
    H = hierarchy.Hierarchy(2, 3, 1)
    rho = dense.spectral_radius(dense.iteration_matrix(H))
    b = H.rhs(inp.rhs(2, 3, 2))
    _, hist = cycle.solve(H, b, 120)
    rate = (hist[-1][0] / hist[-21][0]) ** (1 / 20)
    assert 0 < rho < 1
    assert rate == pytest.approx(rho, rel=0.02)


def test_manufactured_solution_second_order():
    # u* = sin(pi x) sin(pi y), f = 2 pi^2 u*: nodal error shrinks by ~9 per level (h/3, O(h^2))
    errs = []
    for L in (2, 3, 4):
        H = hierarchy.Hierarchy(2, L, 1)
        x = np.indices((3 ** L + 1,) * 2) / 3 ** L
        us = np.sin(np.pi * x[0]) * np.sin(np.pi * x[1])
        uh = dense.direct_solve(H, H.rhs(2 * np.pi ** 2 * us))
        errs.append(np.abs(uh - us.ravel()).max())
    assert 7.0 < errs[0] / errs[1] < 11.0 and 7.0 < errs[1] / errs[2] < 11.0


def test_norms_closed_form():
    H = hierarchy.Hierarchy(3, 2, 1)
    r = 2.5 * H.lev[2].mask.ravel()
    l2, linf = cycle.norms(H, r)
    assert l2 == pytest.approx(2.5 * np.sqrt(8 ** 3 / 9 ** 3), rel=1e-15)
    assert linf == 2.5


def test_defect_correction_in_fp64_equals_plain_cycles():
    # the cycle is linear: k inner cycles from e = 0 on A e = r equal k outer cycles
    H = hierarchy.Hierarchy(2, 3, 1)
    b = H.rhs(inp.rhs(2, 3, 4))
    u_dc, hist_dc, inner = cycle.defect_correction(H, b, 4, 0.0, 3, inner_dtype=np.float64)
    u_pl, hist_pl = cycle.solve(H, b, 12)
    assert inner == 12
    assert np.abs(u_dc - u_pl).max() < 1e-13 * np.abs(u_pl).max()


def test_defect_correction_fp32_reaches_fp64_tolerance():
    H = hierarchy.Hierarchy(3, 3, 1)
    b = H.rhs(inp.rhs(3, 3, 4, "normal"))
    u, hist, inner = cycle.defect_correction(H, b, 6, 1e-8, 20)
    assert hist[-1][0] / hist[0][0] <= 1e-8
    us = dense.direct_solve(H, b)
    assert np.abs(u - us).max() < 1e-7 * np.abs(us).max()


def test_plain_additive_degrades_with_depth_while_adafac_does_not():
    # Sec. 5.1 (qualitative): plain additive overshoots more as levels are added; adAFAC stays stable
    rates = {}
    for L in (2, 3):
        H = hierarchy.Hierarchy(2, L, 1)
        rates[("none", L)] = dense.spectral_radius(dense.iteration_matrix(H, damping="none"))
        rates[("jac", L)] = dense.spectral_radius(dense.iteration_matrix(H, damping="jac"))
    assert rates[("none", 3)] > rates[("none", 2)]
    assert rates[("jac", 3)] < 1 and rates[("jac", 2)] < 1


# --- inhomogeneous Dirichlet data (the set-ups of Sec. 5) -------------------------------------

def _lattice(d, L):
    """Coordinates of the (3^L + 1)^d vertices, coordinate a on array axis d - 1 - a."""
    n = 3 ** L
    idx = np.indices((n + 1,) * d).astype(float) / n
    return [idx[d - 1 - a] for a in range(d)]


@pytest.mark.parametrize("d,L", [(2, 3), (3, 2)])
def test_dirichlet_lift_reproduces_harmonic_multilinear_functions(d, L):
    # a harmonic function in the d-linear space (x y + 2 x - y + 0.5; x y z + x - z in 3D) with
    # f = 0 is its own discrete solution: the lift and a direct solve must give it back exactly
    X = _lattice(d, L)
    ue = X[0] * X[1] + 2 * X[0] - X[1] + 0.5 if d == 2 else X[0] * X[1] * X[2] + X[0] - X[2]
    H = hierarchy.Hierarchy(d, L, 1)
    b = H.rhs(np.zeros_like(ue), g=ue)
    u0 = dense.direct_solve(H, b)
    u = fem.with_boundary(u0, ue)
    assert np.abs(u - ue).max() < 1e-13


def test_dirichlet_lift_on_the_split_field_reproduces_a_flux_free_profile():
    # eps depending on x_1 only (the split set-up with a 10^5 jump): u = x_2 carries the flux
    # eps (0, 1), whose divergence vanishes, so u = x_2 is the exact and the discrete solution
    L = 3
    eps = inp.paper_eps_cells(L, "split", 5)
    X = _lattice(2, L)
    ue = X[1]
    H = hierarchy.Hierarchy(2, L, 1, eps)
    u0 = dense.direct_solve(H, H.rhs(np.zeros_like(ue), g=ue))
    assert np.abs(fem.with_boundary(u0, ue) - ue).max() < 1e-12


def test_paper_setup_fixed_point_is_the_lifted_direct_solve():
    # f = 0, u = 1 on x_2 = 0: adAFAC-Jac converges to the direct solve of the lifted system,
    # and the solution lies between the boundary values 0 and 1 (discrete maximum principle of
    # the Q1 Laplacian with nonpositive off-diagonal entries)
    L = 3
    g = inp.paper_boundary(2, L)
    H = hierarchy.Hierarchy(2, L, 1)
    b = H.rhs(np.zeros_like(g), g=g)
    us = dense.direct_solve(H, b)
    u, hist = cycle.solve(H, b, 400, tol=1e-12)
    assert hist[-1][0] / hist[0][0] <= 1e-12
    assert np.abs(u - us).max() < 1e-10
    full = fem.with_boundary(us, g)
    assert full.min() >= -1e-14 and full.max() <= 1 + 1e-14
    # symmetric in x_1 about 1/2
    assert np.abs(full - full[:, ::-1]).max() < 1e-12
