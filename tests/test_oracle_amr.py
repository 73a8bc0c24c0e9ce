"""Pins of the oracle's feature-based refinement (oracle/amr.py): the bottom-boundary growth,
the second-derivative marks and their bin sort, and the move onto the next tree."""
import numpy as np
import pytest

import adafac_inputs as inp
from oracle import adaptive, amr


def g_of(L):
    return inp.paper_boundary(2, L)


def test_boundary_refinement_grows_one_level_per_move_along_the_bottom():
    """With no feature marks, each move deepens the tree by one level, and the new finest level
    holds exactly the children of the bottom row of cells."""
    T = adaptive.AdaptiveTree(2, 2, 1, 2, {}, g=g_of(2))
    U = T.spread({l: np.zeros(T.shape(l)) for l in (1, 2)})
    for depth in (3, 4, 5):
        flags, top = amr.mark(T, U, 0.0, 2, 6)
        assert top == depth
        T, U = amr.grow(T, U, flags, top, 2, g_of=g_of)
        E = T.E[depth]
        # children of the bottom-row cells of the previous level: the three bottom rows
        assert E[:3].all() and not E[3:].any()
    # at l_cap the boundary marks stop
    flags, top = amr.mark(T, U, 0.0, 2, 5)
    assert top == 5


def test_second_derivative_marks_pick_the_peak():
    """A tree without Dirichlet data and a level array with one kink: with a fraction below one
    dof, the 2^d cells around the dof with the largest second difference are marked, and only
    those (besides the tree's own refined cells)."""
    L = 3
    T = adaptive.AdaptiveTree(2, L, 1, L, {})
    U = {l: np.zeros(T.shape(l)) for l in range(1, L + 1)}
    U[L][10, 7] = 1.0            # (x, y) = (7, 10)
    U = T.spread(U)
    flags, top = amr.mark(T, U, 1e-9, L, L + 1)
    assert top == L + 1
    want = np.zeros((27, 27), dtype=bool)
    want[9:11, 6:8] = True
    assert np.array_equal(flags[L], want)


def test_bin_sort_takes_at_least_the_fraction_and_a_top_set():
    rng = np.random.default_rng(5)
    L = 4
    T = adaptive.AdaptiveTree(2, L, 1, L, {})
    U = {l: np.zeros(T.shape(l)) for l in range(1, L + 1)}
    U[L][1:-1, 1:-1] = rng.standard_normal((3 ** L - 1, 3 ** L - 1))
    U = T.spread(U)
    tr = {}
    flags, _ = amr.mark(T, U, 0.1, L, L + 1, trace=tr)
    # the values, recomputed independently: second differences along x and y, max per dof
    u = U[L]
    h2 = 1.0 / 81.0 ** 2
    vx = np.abs(u[1:-1, 2:] - 2 * u[1:-1, 1:-1] + u[1:-1, :-2]) / h2
    vy = np.abs(u[2:, 1:-1] - 2 * u[1:-1, 1:-1] + u[:-2, 1:-1]) / h2
    v = np.maximum(vx, vy).ravel()
    assert np.allclose(tr["values"], v, rtol=1e-13, atol=0)
    sel = tr["selected"]
    assert sel.sum() >= 0.1 * v.size
    assert sel.sum() <= 0.1 * v.size + np.bincount(np.minimum(amr.BINS - 1, (v / v.max() * amr.BINS).astype(int))).max()
    # a top set up to one bin: every unselected value lies below the smallest selected one plus a bin width
    assert (v[~sel] < v[sel].min() + v.max() / amr.BINS).all()
    # the flags are the four cells around each selected dof
    want = np.zeros((81, 81), dtype=bool)
    for (l, (y, x)), s_ in zip(tr["dofs"], sel):
        if s_:
            want[y - 1:y + 1, x - 1:x + 1] = True
    assert np.array_equal(flags[L], want)


def test_grow_keeps_the_composite_function():
    """Every dof of the next tree takes the old composite function at its position (the
    boundary vertices take the data of the finer lattice, which may differ from the old trace
    where the data jump, at the corners of the u = 1 edge)."""
    T = adaptive.AdaptiveTree(2, 3, 1, 2, inp.refine_ball(2, 3, 2, (0.5, 0.3), 0.2), g=g_of(3))
    U, _ = adaptive.solve(T, np.zeros(T.shape(3)), 5)
    flags, top = amr.mark(T, U, 0.1, 2, 5)
    T2, U2 = amr.grow(T, U, flags, top, 2, g_of=g_of)
    F = adaptive.finest_values(T, U)
    # the old composite function at the new lattice: exact d-linear interpolation per old cell
    x = np.linspace(0.0, 1.0, 3 ** top + 1)
    from scipy.interpolate import RegularGridInterpolator
    xs = np.linspace(0.0, 1.0, 28)
    f = RegularGridInterpolator((xs, xs), F, method="linear")
    Y, X = np.meshgrid(x, x, indexing="ij")
    Fn = f(np.stack([Y.ravel(), X.ravel()], axis=1)).reshape(Y.shape)
    for l in range(1, top + 1):
        s = 3 ** (top - l)
        m = T2.dof[l]
        assert np.abs(U2[l][m] - Fn[::s, ::s][m]).max() <= 1e-13, l


def test_run_from_two_levels_reaches_l_cap_and_converges():
    """The Sec. 5 homogeneous set-up from l_max = 2 with moves every other cycle up to l_max = 5:
    the depth grows to 5, and the residual falls once the refinement settles."""
    hist, moves = amr.run(2, 2, 5, 40, g_of)
    depths = [h[1] for h in hist]
    assert depths[0] == 2 and depths[-1] == 5
    assert all(b >= a for a, b in zip(depths, depths[1:]))
    # the tree settles (no new dofs over the last 30 cycles) and the residual then falls steadily
    assert len({h[2] for h in hist[-30:]}) == 1
    r = [h[0][0] for h in hist[-30:]]
    assert all(b < a for a, b in zip(r, r[1:])) and r[-1] < 1e-2 * r[0]
