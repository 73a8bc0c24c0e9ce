"""Feature-based dynamic refinement with the full-multigrid-like start (the runs of Sec. 5) on
the GPU against the oracle (oracle/amr.py).

* adafac_amr_mark, given the same iterate (set through the composite order), marks exactly
  the oracle's cells, on a uniform and on an adaptive tree;
* a run from l_max = 2 with a move every other cycle (marks, a deeper tree, the solution
  interpolated onto it with adafac_set_solution_coarse) matches the oracle's run cycle by
  cycle (residual norms within 1e-12 of the first one) and move by move (identical trees).
"""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import adaptive, amr

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def g_of(L):
    return inp.paper_boundary(2, L)


def gpu_run(l_start, l_cap, cycles, fraction=0.1, every=2):
    from paper_1903_10367_amd import Solver
    lu = l_start
    s = Solver(2, 1, l_start, np.zeros_like(g_of(l_start)), dirichlet=g_of(l_start))
    hist, moves = [], []
    for n in range(cycles):
        s.cycle(1)
        hist.append((s.residuals()[-1], s.lmax, s.composite_dofs()))
        if (n + 1) % every == 0 and n + 1 < cycles:
            flags, top = s.amr_mark(fraction, lu, l_cap)
            moves.append((flags, top))
            u, lold = s.solution(), s.lmax
            refine = {l: flags[l] for l in range(lu, top)}
            s2 = Solver(2, 1, top, np.zeros_like(g_of(top)), refine=refine, dirichlet=g_of(top))
            s2.set_solution_coarse(u, lold)
            s.close()
            s = s2
    s.close()
    return hist, moves


@pytest.mark.parametrize("adaptive_tree", [False, True])
def test_marks_match_the_oracle_on_the_same_iterate(adaptive_tree):
    from paper_1903_10367_amd import Solver
    say("case amr marks, adaptive tree", adaptive_tree)
    if adaptive_tree:
        # the oracle's state after a few moves: a ragged tree of depth 4
        T = adaptive.AdaptiveTree(2, 2, 1, 2, {}, g=g_of(2))
        U = T.spread({l: np.zeros(T.shape(l)) for l in (1, 2)})
        for _ in range(2):
            U, _ = adaptive.cycle(T, U, T.load(np.zeros(T.shape(T.L))))
            flags, top = amr.mark(T, U, 0.1, 2, 6)
            T, U = amr.grow(T, U, flags, top, 2, g_of=g_of)
        for _ in range(3):
            U, _ = adaptive.cycle(T, U, T.load(np.zeros(T.shape(T.L))))
        L = T.L
        s = Solver(2, 1, L, np.zeros_like(g_of(L)), refine={l: T.Rf[l] for l in range(2, L)}, dirichlet=g_of(L))
    else:
        L = 3
        T = adaptive.AdaptiveTree(2, L, 1, L, {}, g=g_of(L))
        U, _ = adaptive.solve(T, np.zeros(T.shape(L)), 4)
        s = Solver(2, 1, L, np.zeros_like(g_of(L)), dirichlet=g_of(L))
    assert s.composite_dofs() == len(T.composite_index())
    s.set_composite(adaptive.to_composite(T, U))
    lu = 2 if adaptive_tree else L
    for frac in (0.1, 0.3):
        fg, tg = s.amr_mark(frac, lu, 6)
        fo, to = amr.mark(T, U, frac, lu, 6)
        say(f"fraction {frac}: depth {tg} / {to}, marked {sum(int(f.sum()) for f in fg.values())}")
        assert tg == to
        for l in fo:
            assert np.array_equal(fg[l], fo[l]), f"level {l}"
    s.close()


def test_growth_run_matches_the_oracle():
    say("case amr growth run l_max 2 -> 5")
    cycles = 16
    hg, mg = gpu_run(2, 5, cycles)
    ho, mo = amr.run(2, 2, 5, cycles, g_of)
    assert len(mg) == len(mo)
    for k, ((fg, tg), (fo, to)) in enumerate(zip(mg, mo)):
        assert tg == to, f"move {k}"
        for l in fo:
            assert np.array_equal(fg[l], fo[l]), f"move {k} level {l}"
    r0 = ho[0][0][0]
    for n, ((a, La, na), (b, Lb, nb)) in enumerate(zip(hg, ho)):
        say(f"cycle {n}: depth {La} dofs {na} ||r||_h {a[0]:.6e} / {b[0]:.6e}")
        assert La == Lb and na == nb
        assert abs(a[0] - b[0]) <= 1e-12 * r0, f"cycle {n}"
