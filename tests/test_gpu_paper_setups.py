"""The paper's own set-ups (Sec. 5) on the GPU against the oracle: f = 0, u = 1 on x_2 = 0 and
u = 0 on the rest of the boundary, with the four coefficient fields (homogeneous, a split that
no 3:1 level resolves, a 0.02-wide needle, a slanted checkerboard; eps = 10^-k in one region,
evaluated at the finest cell centres), regular grids, d-linear and BoxMG transfers, and the
damping variants.  Per cycle the residual norms agree within 1e-12 of the initial norm, the
iterate within 1e-12 relative (or twice the oracle's own rounding spread)."""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import cycle, fem, hierarchy

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_setup(L, field, k, transfer="dlinear", damping="jac", cycles=10, **kw):
    from paper_1903_10367_amd import Solver
    eps = inp.paper_eps_cells(L, field, k)
    g = inp.paper_boundary(2, L)
    s = Solver(2, 1, L, np.zeros_like(g), eps_blocks=eps, transfer=transfer, damping=damping, dirichlet=g, **kw)
    s.cycle(cycles)
    h, u = s.residuals(), s.solution()
    s.close()
    return h, u


def oracle_setup(L, field, k, transfer="dlinear", damping="jac", cycles=10):
    eps = inp.paper_eps_cells(L, field, k)
    g = inp.paper_boundary(2, L)
    H = hierarchy.Hierarchy(2, L, 1, eps, transfer)
    b = H.rhs(np.zeros_like(g), g=g)
    u0, h = cycle.solve(H, b, cycles, damping=damping)
    spread = lambda: _spread(H, b, cycles, damping)
    return h, fem.with_boundary(u0, g).ravel(), spread


def _spread(H, b, cycles, damping):
    u1, _ = cycle.solve(H, b, cycles, form="correction", damping=damping)
    u2, _ = cycle.solve(H, b, cycles, form="fas", damping=damping)
    return np.linalg.norm(u1 - u2) / np.linalg.norm(u1)


def check(hg, ug, ho, uo, spread):
    r0, m0 = ho[0]
    assert len(hg) == len(ho)
    for n, (a, b) in enumerate(zip(hg, ho)):
        assert abs(a[0] - b[0]) <= 1e-12 * r0, f"cycle {n}: {a[0]!r} vs {b[0]!r}"
        assert abs(a[1] - b[1]) <= 1e-12 * m0, f"cycle {n} linf"
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    if err > 1e-12:
        fl = spread()
        say(f"rel. error {err:.3e}, oracle spread {fl:.3e}")
        assert err <= 2 * fl
    # the Dirichlet values stay on the boundary
    g = inp.paper_boundary(2, int(round(np.log(np.sqrt(ug.size) - 1) / np.log(3)))).ravel()
    m = ~fem.interior_mask(2, int(round(np.log(np.sqrt(ug.size) - 1) / np.log(3)))).ravel()
    assert np.array_equal(ug[m], g[m])


@pytest.mark.parametrize("field", inp.PAPER_FIELDS)
@pytest.mark.parametrize("transfer", ["dlinear", "boxmg"])
def test_fields_adafac_jac(field, transfer):
    say("case paper set-up", field, transfer)
    hg, ug = gpu_setup(4, field, 3, transfer)
    ho, uo, sp = oracle_setup(4, field, 3, transfer)
    check(hg, ug, ho, uo, sp)


@pytest.mark.parametrize("damping", ["none", "pi", "exp"])
def test_damping_variants_on_the_checkerboard(damping):
    say("case paper set-up damping", damping)
    hg, ug = gpu_setup(4, "checkerboard", 5, "boxmg", damping)
    ho, uo, sp = oracle_setup(4, "checkerboard", 5, "boxmg", damping)
    check(hg, ug, ho, uo, sp)


@pytest.mark.parametrize("fused", [True, False])
def test_poisson_with_dirichlet_data_fused_and_unfused(fused):
    """The homogeneous set-up, L = 5: the single-pass sweep reads the boundary values."""
    say("case paper set-up Poisson L=5 fused", fused)
    hg, ug = gpu_setup(5, "homogeneous", 1, cycles=12, fused=fused)
    ho, uo, sp = oracle_setup(5, "homogeneous", 1, cycles=12)
    check(hg, ug, ho, uo, sp)


def test_solution_readout_keeps_boundary_values():
    from paper_1903_10367_amd import Solver
    L = 3
    g = inp.paper_boundary(2, L)
    s = Solver(2, 1, L, np.zeros_like(g), dirichlet=g)
    s.cycle(3)
    s.set_solution(np.zeros_like(g))      # boundary entries are replaced by the data
    u = s.solution()
    s.close()
    assert np.array_equal(u.reshape(g.shape), np.where(fem.interior_mask(2, L), 0.0, g))
