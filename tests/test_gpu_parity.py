"""Parity of the gfx950 cycle (through the C ABI) with the FP64 oracle.

Bar (FP64 path): per-cycle residual norms within 1e-12 of the oracle's, relative to the
initial norm, and the iterate within 1e-12 in relative 2-norm.  Inputs are the seeded
synthetic workloads of ``adafac_inputs``.
"""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import cycle, hierarchy

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(d, L, f, eps=None, cycles=10, **kw):
    from paper_1903_10367_amd import Solver
    s = Solver(d, 1, L, f, eps_blocks=eps, **kw)
    s.cycle(cycles)
    hist = s.residuals()
    u = s.solution()
    s.close()
    return hist, u


def oracle_run(d, L, f, eps=None, cycles=10, transfer="dlinear", **kw):
    # BoxMG weights are solved only where coarse cells straddle coefficient blocks (elsewhere
    # they equal the d-linear ones, a pinned identity of the oracle)
    H = hierarchy.Hierarchy(d, L, 1, eps, transfer, boxmg_inside_blocks=False)
    b = H.rhs(f)
    u, hist = cycle.solve(H, b, cycles, **kw)
    return hist, u


def oracle_floor(H, b, cycles, **kw):
    """Relative 2-norm spread between the oracle's correction and FAS forms of the same cycles:
    two exact evaluations of one iteration that differ only in rounding."""
    u1, _ = cycle.solve(H, b, cycles, form="correction", **kw)
    u2, _ = cycle.solve(H, b, cycles, form="fas", **kw)
    return np.linalg.norm(u1 - u2) / np.linalg.norm(u1)


def assert_parity(hg, ug, ho, uo, tol=TOL, floor=None):
    """Norms: |gpu - oracle| <= 1e-12 of the initial norm, every cycle.  Solution: relative
    2-norm error <= max(1e-12, 2 x the oracle's own rounding spread) (the reading of the
    "1e-12 relative" bar near convergence: r = b - A u cancels, and two exact evaluations of
    the same cycles differ by about eps times the condition number)."""
    assert len(hg) == len(ho)
    r0, m0 = ho[0]
    for n, (a, b) in enumerate(zip(hg, ho)):
        assert abs(a[0] - b[0]) <= tol * r0, f"cycle {n}: l2h {a[0]!r} vs {b[0]!r}"
        assert abs(a[1] - b[1]) <= tol * m0, f"cycle {n}: linf {a[1]!r} vs {b[1]!r}"
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    if err > tol and floor is not None:
        fl = floor()
        say(f"solution rel. error {err:.3e} above {tol:g}; oracle spread {fl:.3e}")
        assert err <= 2 * fl, f"solution rel. error {err:.3e} vs oracle spread {fl:.3e}"
        return
    assert err <= tol, f"solution rel. error {err:.3e}"


@pytest.mark.parametrize("fused", [True, False])
def test_2d_poisson_l4_twenty_cycles(fused):
    w = inp.workload_2d_poisson_l4()
    say("case 2d poisson L=4 fused", fused)
    hg, ug = gpu_run(2, 4, w["f"], cycles=20, fused=fused)
    ho, uo = oracle_run(2, 4, w["f"], cycles=20)
    assert_parity(hg, ug, ho, uo)


@pytest.mark.parametrize("fused", [True, False])
def test_3d_poisson_l4(fused):
    f = inp.rhs(3, 4, seed=3, dist="normal")
    say("case 3d poisson L=4 fused", fused)
    hg, ug = gpu_run(3, 4, f, cycles=8, fused=fused)
    ho, uo = oracle_run(3, 4, f, cycles=8)
    assert_parity(hg, ug, ho, uo)


@pytest.mark.parametrize("fused", [True, False])
def test_2d_jump_coefficient_boxmg(fused):
    eps = inp.eps_blocks(2, 2, 3.0, seed=4)
    f = inp.rhs(2, 4, seed=5)
    say("case 2d jump L=4 boxmg fused", fused)
    hg, ug = gpu_run(2, 4, f, eps, cycles=12, transfer="boxmg", fused=fused)
    ho, uo = oracle_run(2, 4, f, eps, cycles=12, transfer="boxmg")
    assert_parity(hg, ug, ho, uo)


def test_3d_jump_coefficient_boxmg():
    eps = inp.eps_blocks(3, 2, 4.0, seed=6)
    f = inp.rhs(3, 4, seed=7)
    say("case 3d jump 9^3 blocks L=4 boxmg")
    hg, ug = gpu_run(3, 4, f, eps, cycles=6, transfer="boxmg")
    ho, uo = oracle_run(3, 4, f, eps, cycles=6, transfer="boxmg")
    assert_parity(hg, ug, ho, uo)


def test_3d_coefficient_per_fine_cell():
    # eps on every finest cell: BoxMG on every transfer, stored Galerkin operators below L
    eps = inp.eps_blocks(3, 2, 2.0, seed=8)
    f = inp.rhs(3, 2, seed=9)
    say("case 3d eps per fine cell L=2")
    hg, ug = gpu_run(3, 2, f, eps, cycles=6, transfer="boxmg")
    ho, uo = oracle_run(3, 2, f, eps, cycles=6, transfer="boxmg")
    assert_parity(hg, ug, ho, uo)


@pytest.mark.parametrize("damping", ["none", "pi", "exp"])
def test_damping_variants(damping):
    w = inp.workload_2d_poisson_l4(seed=2)
    say("case damping", damping)
    hg, ug = gpu_run(2, 4, w["f"], cycles=10, damping=damping, omega_hat=0.7)
    ho, uo = oracle_run(2, 4, w["f"], cycles=10, damping=damping, omega_hat=0.7)
    assert_parity(hg, ug, ho, uo)


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("d,L", [(2, 4), (3, 3), (3, 4), (2, 6)])
def test_pi_single_pass_and_one_kernel_per_step(d, L, fused):
    """adAFAC-PI (c~_l = P I c_l, Sec. 3.2) in the single-pass sweeps (I c written by the sweep,
    subtracted from S_{L-1} by the last prolongation) and in the one-kernel-per-step form."""
    f = inp.rhs(d, L, seed=13 + d + L)
    say("case pi", d, L, fused)
    cycles = 8 if d == 2 else 5
    hg, ug = gpu_run(d, L, f, cycles=cycles, damping="pi", fused=fused)
    ho, uo = oracle_run(d, L, f, cycles=cycles, damping="pi")
    H = hierarchy.Hierarchy(d, L, 1)
    assert_parity(hg, ug, ho, uo, floor=lambda: oracle_floor(H, H.rhs(f), cycles, damping="pi"))


@pytest.mark.parametrize("d,L,fused", [(2, 4, True), (3, 3, True), (3, 3, False), (3, 4, True), (2, 6, True),
                                        (2, 6, False)])
def test_level_arrays_match_fas_oracle(d, L, fused):
    """u_l (injection), b_l (FAS rhs with tau), b~_l, r_l and S_l of the second cycle (3D L=4
    and 2D L=6 prolongate two and three levels in one chained launch)."""
    from paper_1903_10367_amd import Solver
    f = inp.rhs(d, L, seed=10)
    say("case level arrays", d, L, fused)
    s = Solver(d, 1, L, f, fused=fused)
    s.cycle(2)
    got = {(l, w): s.level(l, w) for l in range(1, L) for w in ("u", "b", "btilde", "r", "S")}
    s.close()
    H = hierarchy.Hierarchy(d, L, 1)
    b = H.rhs(f)
    u1, _ = cycle.cycle_fas(H, np.zeros_like(b), b)
    tr = {}
    cycle.cycle_fas(H, u1, b, trace=tr)
    for (l, w), g in got.items():
        ref = tr[w][l]
        scale = np.abs(ref).max()
        assert np.abs(g - ref).max() <= 1e-12 * scale, f"level {l} {w}"


@pytest.mark.parametrize("damping", ["jac", "pi"])
def test_full_size_3d_poisson_l5(damping):
    """The benchmark workload itself (243^3 cells), three cycles, in the benchmark's launch shape
    (with adAFAC-PI also the level-4 FAS sweep writes I c_4)."""
    w = inp.workload_3d_poisson_l5()
    say("case 3d poisson L=5 full size", damping)
    hg, ug = gpu_run(3, 5, w["f"], cycles=3, damping=damping)
    say("oracle 3d L=5")
    ho, uo = oracle_run(3, 5, w["f"], cycles=3, damping=damping)
    assert_parity(hg, ug, ho, uo)


def test_full_size_3d_jump_27_blocks():
    """243^3 cells with 27^3 coefficient blocks 10^U(0,4): the variable-eps single-pass sweep at
    block size 9 (the serving mix's largest request shape), two cycles."""
    eps = inp.eps_blocks(3, 3, 4.0, seed=14)
    f = inp.rhs(3, 5, seed=15)
    say("case 3d jump 27^3 blocks L=5 full size")
    hg, ug = gpu_run(3, 5, f, eps, cycles=2)
    say("oracle 3d L=5 27^3 blocks")
    ho, uo = oracle_run(3, 5, f, eps, cycles=2)
    assert_parity(hg, ug, ho, uo)


def test_repeat_runs_are_bitwise_identical():
    f = inp.rhs(3, 4, seed=11)
    say("case determinism")
    h1, u1 = gpu_run(3, 4, f, cycles=4)
    h2, u2 = gpu_run(3, 4, f, cycles=4)
    assert h1 == h2
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("d,L,lmin", [(2, 2, 2), (2, 3, 2), (3, 2, 1), (2, 6, 1)])
def test_edge_sizes(d, L, lmin):
    """One level (damped Jacobi), two levels, a level too small for the single-pass sweep,
    and a 2D level spanning many tiles."""
    from paper_1903_10367_amd import Solver
    f = inp.rhs(d, L, seed=12)
    say("case edge", d, L, lmin)
    s = Solver(d, lmin, L, f)
    s.cycle(5)
    hg, ug = s.residuals(), s.solution()
    s.close()
    H = hierarchy.Hierarchy(d, L, lmin)
    b = H.rhs(f)
    uo, ho = cycle.solve(H, b, 5)
    assert_parity(hg, ug, ho, uo, floor=lambda: oracle_floor(H, b, 5))


def test_solve_to_tolerance_matches_oracle():
    from paper_1903_10367_amd import Solver
    f = inp.rhs(3, 4, seed=13, dist="normal")
    say("case solve 1e-8")
    s = Solver(3, 1, 4, f)
    n = s.solve(1e-8, 100)
    hg, ug = s.residuals(), s.solution()
    s.close()
    H = hierarchy.Hierarchy(3, 4, 1)
    uo, ho = cycle.solve(H, H.rhs(f), 100, tol=1e-8)
    assert n == len(ho) and hg[-1][0] / hg[0][0] <= 1e-8
    assert_parity(hg, ug, ho, uo)


def test_divergence_is_reported():
    from paper_1903_10367_amd import AdafacError, Solver
    f = inp.rhs(2, 3, seed=14)
    say("case divergence")
    s = Solver(2, 1, 3, f, omega=1.5)
    with pytest.raises(AdafacError) as e:
        s.solve(1e-8, 200)
    assert e.value.code == 5
    s.close()


@pytest.mark.parametrize("d,L,damping,fused,cap", [(3, 4, "jac", True, 100), (2, 5, "jac", True, 13),
                                                   (2, 5, "pi", True, 100), (3, 3, "jac", False, 100),
                                                   (2, 6, "jac", False, 100)])
def test_pipelined_solve_matches_a_check_after_every_cycle(d, L, damping, fused, cap):
    """adafac_solve launches FP64 cycles in batches and stops them on the device: the cycle count,
    every norm and the solution are bitwise those of running one cycle at a time and checking the
    relative residual after each (also when the cap ends a batch early, and for a second solve
    that continues the first)."""
    from paper_1903_10367_amd import Solver
    f = inp.rhs(d, L, seed=40 + d + L)
    say("case pipelined solve", d, L, damping, fused, cap)
    tols = (1e-4, 1e-9, 1e-4)   # the third stops at its first check (a batch of one step run)
    s1 = Solver(d, 1, L, f, damping=damping, fused=fused)
    n1 = [s1.solve(t, cap) for t in tols]
    assert s1.solve(1e-12, 0) == 0
    h1 = s1.residuals()
    u1 = s1.solution()
    s1.close()
    s2 = Solver(d, 1, L, f, damping=damping, fused=fused)
    counts = []
    for tol in tols:
        n = 0
        while n < cap:
            s2.cycle(1)
            n += 1
            k = len(s2.residuals()) - 1
            if s2.residual(k)[0] / s2.residual(0)[0] <= tol:
                break
        counts.append(n)
        s2.solution()   # a solve ends by adding the pending coarse correction; so does this read
    h2 = s2.residuals()
    u2 = s2.solution()
    s2.close()
    say(f"cycles {n1} / {counts}")
    assert n1 == counts
    if counts[0] < cap:         # the first solve met 1e-4, so the third one stops at its first check
        assert counts[2] == 1
    assert h1 == h2
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("k,cap,tols", [(4, 100, (1e-5, 1e-9)), (3, 100, (1e-9,)), (4, 3, (1e-9,))])
def test_pipelined_fp32_refined_solve_matches_the_host_checked_one(k, cap, tols, monkeypatch):
    """The one-pass 3D FP32_REFINED solve in batches (outer step and inner cycles gated, the inner
    solve of the step that met the rule skipped): outer-step counts, norms and the solution bitwise
    those of the solve that checks on the host after every outer step (ADAFAC_SOLVE_HOST_CHECK=1),
    with an odd inner cycle count, a cap inside the first batch and a continued second solve."""
    from paper_1903_10367_amd import Solver
    d, L = 3, 4
    f = inp.rhs(d, L, seed=61)
    say("case pipelined fp32_refined solve, k", k, "cap", cap, "tols", tols)
    out = []
    for host_check in ("0", "1"):
        monkeypatch.setenv("ADAFAC_SOLVE_HOST_CHECK", host_check)
        s = Solver(d, 1, L, f, precision="fp32_refined", inner_k=k)
        n = [s.solve(t, cap) for t in tols]
        out.append((n, s.residuals(), s.solution()))
        s.close()
    say(f"steps {out[0][0]} / {out[1][0]}")
    assert out[0][0] == out[1][0]
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])
