"""FP32 cycles inside FP64 defect correction: the gfx950 path against the oracle.

An outer step computes the FP64 defect r = b - A u of the outer iterate, runs k adAFAC cycles in
FP32 on A e = r from e = 0, and adds e to u in FP64.  The GPU and the oracle round the FP32 cycles
differently. Per outer step, each side's rounding moves the next residual by a vector of the
same size as the FP32 rounding itself.  That size is measured as the spread between the oracle
with FP32 inner cycles and the oracle with FP64 inner cycles (same steps, exact arithmetic
otherwise).  The bar, per outer step n:

    | ||r^n||_gpu - ||r^n||_oracle32 |  <=  4 * ||r^n_oracle32 - r^n_oracle64||_h + 1e-12 ||r^0||_h,

and the same for the final iterate in the 2-norm.  A solve to 1e-8 is also checked against the
FP64 solution: ||u - u*||_2 <= ||A^-1||_2 ||b - A u||_2, with ||A^-1||_2 computed exactly on the
small grid.
"""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import cycle, dense, hierarchy

pytestmark = pytest.mark.gpu

K = 4


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_steps(d, L, f, eps=None, steps=5, **kw):
    from paper_1903_10367_amd import Solver
    s = Solver(d, 1, L, f, eps_blocks=eps, precision="fp32_refined", inner_k=K, **kw)
    s.cycle(steps)
    hist = s.residuals()
    u = s.solution()
    s.close()
    return hist, u


def oracle_steps(H, b, steps, dtype):
    its = []
    u, hist, _ = cycle.defect_correction(H, b, K, 0.0, steps, inner_dtype=dtype, iterates=its)
    return hist, its


def check_outer_steps(H, b, hg, ug, steps):
    h32, it32 = oracle_steps(H, b, steps, np.float32)
    h64, it64 = oracle_steps(H, b, steps, np.float64)
    assert len(hg) == steps and len(h32) >= steps + 1
    A = H.lev[H.L].A
    r0 = h32[0][0]
    for n in range(steps):
        spread = cycle.norms(H, A(it32[n]) - A(it64[n]))[0]
        gate = 4 * spread + 1e-12 * r0
        say(f"outer {n}: gpu {hg[n][0]:.6e} oracle32 {h32[n][0]:.6e} spread {spread:.2e}")
        assert abs(hg[n][0] - h32[n][0]) <= gate, f"outer step {n}"
    # the iterate after the last step
    u32, u64 = it32[steps], it64[steps]
    spread = np.linalg.norm(u32 - u64)
    err = np.linalg.norm(ug - u32)
    say(f"final iterate: |gpu - oracle32| {err:.3e}, |oracle32 - oracle64| {spread:.3e}")
    assert err <= 4 * spread + 1e-12 * np.linalg.norm(u64)


@pytest.mark.parametrize("fused", [True, False])
def test_2d_poisson_l4_outer_steps(fused):
    w = inp.workload_2d_poisson_l4()
    say("case mixed 2d poisson L=4 fused", fused)
    steps = 5
    hg, ug = gpu_steps(2, 4, w["f"], steps=steps, fused=fused)
    H = hierarchy.Hierarchy(2, 4, 1)
    check_outer_steps(H, H.rhs(w["f"]), hg, ug, steps)


@pytest.mark.parametrize("fused", [True, False])
def test_3d_poisson_l4_outer_steps(fused):
    f = inp.rhs(3, 4, seed=21, dist="normal")
    say("case mixed 3d poisson L=4 fused", fused)
    steps = 3
    hg, ug = gpu_steps(3, 4, f, steps=steps, fused=fused)
    H = hierarchy.Hierarchy(3, 4, 1)
    check_outer_steps(H, H.rhs(f), hg, ug, steps)


def test_2d_jump_boxmg_outer_steps():
    eps = inp.eps_blocks(2, 2, 3.0, seed=22)
    f = inp.rhs(2, 4, seed=23)
    say("case mixed 2d jump boxmg")
    steps = 4
    hg, ug = gpu_steps(2, 4, f, eps, steps=steps, transfer="boxmg")
    H = hierarchy.Hierarchy(2, 4, 1, eps, "boxmg", boxmg_inside_blocks=False)
    check_outer_steps(H, H.rhs(f), hg, ug, steps)


def test_3d_jump_boxmg_outer_steps():
    eps = inp.eps_blocks(3, 2, 4.0, seed=24)
    f = inp.rhs(3, 3, seed=25)
    say("case mixed 3d jump boxmg L=3")
    steps = 3
    hg, ug = gpu_steps(3, 3, f, eps, steps=steps, transfer="boxmg")
    H = hierarchy.Hierarchy(3, 3, 1, eps, "boxmg", boxmg_inside_blocks=False)
    check_outer_steps(H, H.rhs(f), hg, ug, steps)


@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
def test_solve_to_1e8_and_error_against_fp64_solution(d, L):
    from paper_1903_10367_amd import Solver
    f = inp.rhs(d, L, seed=26, dist="normal")
    say("case mixed solve", d, L)
    s = Solver(d, 1, L, f, precision="fp32_refined", inner_k=K)
    n = s.solve(1e-8, 40)
    hg, ug = s.residuals(), s.solution()
    s.close()
    H = hierarchy.Hierarchy(d, L, 1)
    b = H.rhs(f)
    # the FP64 defect of the returned iterate, recomputed by the oracle, meets the tolerance
    r = cycle.norms(H, b - H.lev[L].A(ug))
    assert hg[-1][0] / hg[0][0] <= 1e-8 and n == len(hg)
    assert r[0] / hg[0][0] <= 1e-8 * (1 + 1e-6)
    assert abs(r[0] - hg[-1][0]) <= 1e-12 * hg[0][0]
    # error against the FP64 solution within what the residual allows
    ustar = dense.direct_solve(H, b)
    m = H.lev[L].mask.ravel()
    Ad = H.lev[L].A.mat.tocsr()[m][:, m].toarray()
    inv_norm = 1.0 / np.linalg.eigvalsh(Ad)[0]
    res2 = np.linalg.norm((b - H.lev[L].A(ug))[m])
    err = np.linalg.norm(ug - ustar)
    say(f"outer steps {n}, ||u - u*|| / ||u*|| = {err / np.linalg.norm(ustar):.3e}, "
        f"bound {inv_norm * res2 / np.linalg.norm(ustar):.3e}")
    assert err <= inv_norm * res2 * (1 + 1e-6) + 1e-14 * np.linalg.norm(ustar)
    # the same number of outer steps as the oracle's defect correction, give or take one
    _, ho, _ = cycle.defect_correction(H, b, K, 1e-8, 40)
    assert abs(len(ho) - n) <= 1


def test_full_size_3d_poisson_l5_outer_steps():
    """The 243^3 workload: two outer steps (the defect of iterates 0 and 1) of 2 FP32 cycles."""
    from paper_1903_10367_amd import Solver
    w = inp.workload_3d_poisson_l5()
    say("case mixed 3d poisson L=5 full size")
    s = Solver(3, 1, 5, w["f"], precision="fp32_refined", inner_k=2)
    s.cycle(2)
    hg = s.residuals()
    s.close()
    say("oracle 3d L=5 fp32 / fp64 inner")
    H = hierarchy.Hierarchy(3, 5, 1)
    b = H.rhs(w["f"])
    i32, i64 = [], []
    _, h32, _ = cycle.defect_correction(H, b, 2, 0.0, 1, inner_dtype=np.float32, iterates=i32)
    _, h64, _ = cycle.defect_correction(H, b, 2, 0.0, 1, inner_dtype=np.float64, iterates=i64)
    assert abs(hg[0][0] - h32[0][0]) <= 1e-12 * h32[0][0]
    A = H.lev[5].A
    spread = cycle.norms(H, A(i32[1]) - A(i64[1]))[0]
    say(f"outer 1: gpu {hg[1][0]:.6e} oracle32 {h32[1][0]:.6e} spread {spread:.2e}")
    assert abs(hg[1][0] - h32[1][0]) <= 4 * spread + 1e-12 * h32[0][0]
