"""GPU checks of the boundary calls beyond the cycle itself: the OPERATOR form of R~ (Sec. 3.2)
against the oracle, normalised residuals (Sec. 5), composite-order read-out and warm start, and
a right-hand side given as a function.  Everything runs through the C ABI."""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import cycle, hierarchy

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("d,L,k,cycles", [(2, 4, 2, 12), (3, 3, 2, 6)])
def test_operator_rtilde_matches_oracle(d, L, k, cycles):
    from paper_1903_10367_amd import Solver
    eps = inp.eps_blocks(d, k, 3.0 if d == 2 else 4.0, seed=30 + d)
    f = inp.rhs(d, L, seed=32 + d)
    say("case operator R~", d, L, k)
    s = Solver(d, 1, L, f, eps_blocks=eps, transfer="boxmg", rtilde="operator")
    s.cycle(cycles)
    hg, ug = s.residuals(), s.solution()
    s.close()
    H = hierarchy.Hierarchy(d, L, 1, eps, "boxmg", rtilde="operator")
    uo, ho = cycle.solve(H, H.rhs(f), cycles)
    r0, m0 = ho[0]
    for n, (a, b) in enumerate(zip(hg, ho)):
        assert abs(a[0] - b[0]) <= 1e-12 * r0 and abs(a[1] - b[1]) <= 1e-12 * m0, n
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    say(f"rel. error {err:.3e}")
    assert err <= 1e-12
    # the two forms of R~ really differ on this coefficient field
    Hc = hierarchy.Hierarchy(d, L, 1, eps, "boxmg")
    uc, _ = cycle.solve(Hc, Hc.rhs(f), cycles)
    assert np.linalg.norm(uc - uo) > 1e-6 * np.linalg.norm(uo)


def test_normalised_residuals():
    from paper_1903_10367_amd import Solver
    f = inp.rhs(2, 4, seed=34)
    s = Solver(2, 1, 4, f)
    s.cycle(6)
    h = s.residuals()
    for i in range(6):
        a, b = s.residual_normalised(i)
        assert a == h[i][0] / h[0][0] and b == h[i][1] / h[0][1]
    s.close()


def _disk_ball(d):
    return ((0.5, 0.5), 0.2, 2) if d == 2 else ((0.45, 0.5, 0.55), 0.15, 2)


@pytest.mark.parametrize("adaptive", [False, True])
def test_composite_order_readout_and_warm_start(adaptive):
    from paper_1903_10367_amd import Solver
    from oracle import adaptive as ad
    d, L = 2, 4
    f = inp.rhs(d, L, seed=35)
    kw = dict(ball=_disk_ball(d)) if adaptive else {}
    say("case composite read-out, adaptive", adaptive)
    s = Solver(d, 1, L, f, **kw)
    s.cycle(5)
    uc = s.composite()
    xyz, lev = s.dof_coords()
    lat = s.solution().reshape((3 ** L + 1,) * d)
    g = np.rint(xyz * 3 ** L).astype(int)
    assert np.array_equal(uc, lat[g[:, 1], g[:, 0]])
    if adaptive:
        centre, radius, lu = _disk_ball(d)
        T = ad.AdaptiveTree(d, L, 1, lu, inp.refine_ball(d, L, lu, centre, radius))
        U, _ = ad.solve(T, f, 5)
        assert np.abs(uc - ad.to_composite(T, U)).max() <= 1e-12 * np.abs(uc).max()
    # warm start from the composite values: the next cycles equal those of the same run
    s.cycle(3)
    h_cont, u_cont = s.residuals()[5:], s.composite()
    s2 = Solver(d, 1, L, f, **kw)
    s2.set_composite(uc)
    s2.cycle(3)
    h_warm, u_warm = s2.residuals(), s2.composite()
    s.close()
    s2.close()
    for a, b in zip(h_cont, h_warm):
        assert abs(a[0] - b[0]) <= 1e-13 * h_cont[0][0]
    assert np.abs(u_cont - u_warm).max() <= 1e-13 * np.abs(u_cont).max()


@pytest.mark.parametrize("adaptive", [False, True])
def test_rhs_function_equals_lattice(adaptive):
    from paper_1903_10367_amd import Solver
    d, L = 2, 4
    n = 3 ** L

    def fx(x):
        return np.sin(3.0 * x[0]) * np.cos(2.0 * x[1]) + x[0] * x[1]

    # the library places vertex g at g * (1 / n)
    t = np.arange(n + 1) * (1.0 / n)
    yy, xx = np.meshgrid(t, t, indexing="ij")
    lat = np.sin(3.0 * xx) * np.cos(2.0 * yy) + xx * yy
    kw = dict(ball=_disk_ball(d)) if adaptive else {}
    a = Solver(d, 1, L, fx, **kw)
    b = Solver(d, 1, L, lat, **kw)
    a.cycle(4)
    b.cycle(4)
    assert a.residuals() == b.residuals()
    assert np.array_equal(a.solution(), b.solution())
    a.close()
    b.close()
