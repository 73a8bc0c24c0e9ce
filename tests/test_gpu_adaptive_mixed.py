"""FP32 cycles inside FP64 defect correction on adaptive trees: the gfx950 path against the
adaptive oracle.

An outer step computes, in FP64, the composite residual of the outer iterate and its norms; k
adAFAC cycles in FP32 solve the correction equation from zero, with the composite residual at
the composite dofs as their leaf loads; the correction is added to every dof in FP64.  The GPU
and the oracle round the FP32 cycles differently.  Per outer step n the bar is

    | ||r^n||_gpu - ||r^n||_oracle32 |  <=  G * ||r^n_oracle32 - r^n_oracle64||_h + 1e-12 ||r^0||_h

where oracle64 runs the same steps with FP64 inner cycles, so the right-hand side measures the
size of FP32 rounding in this problem (G = 8: the oracle's FP32 cycles round only where they
store arrays, the kernels after every operation).  The function read out after n steps is
checked in FP64 through its composite residual (the oracle's must equal the one the GPU measures
on it in step n + 1) and to FP32 resolution against the oracle's iterate.  A solve to a
tolerance below FP32
resolution is checked in FP64 from the oracle: the composite residual of the returned function
is the one the GPU reported, and the error against the direct composite solve stays within
||A^-1||_2 ||r||_2.
"""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import adaptive

pytestmark = pytest.mark.gpu

K = 4
G = 8.0


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def storage_from_finest(T, F):
    """Per-level storage of a composite function given on the finest lattice."""
    F = F.reshape(T.shape(T.L))
    U = {}
    for l in range(T.lmin, T.L + 1):
        s = 3 ** (T.L - l)
        U[l] = np.where(T.dof[l], F[tuple(slice(None, None, s) for _ in range(T.d))], 0.0)
    return T.spread(U)


def rounding_scale(T, U32, U64):
    zero = {l: np.zeros(T.shape(l)) for l in U32}
    D = {l: U32[l] - U64[l] for l in U32}
    return adaptive.composite_residual(T, D, zero)[1][0]


def check_steps(T, f, hg, steps, U0=(None, None), label="", **kw):
    """Outer-step norms hg against the oracle with FP32 and FP64 inner cycles, started from
    U0[0] and U0[1] respectively; returns both sides' iterates."""
    i32, i64 = [], []
    _, h32 = adaptive.defect_correction(T, f, K, 0.0, steps, np.float32, i32, U0=U0[0], **kw)
    _, h64 = adaptive.defect_correction(T, f, K, 0.0, steps, np.float64, i64, U0=U0[1], **kw)
    r0 = h64[0][0]
    assert len(hg) >= steps
    for n in range(steps):
        spread = rounding_scale(T, i32[n], i64[n])
        gate = G * spread + 1e-12 * r0
        say(f"{label} outer {n}: gpu {hg[n][0]:.9e} oracle32 {h32[n][0]:.9e} oracle64 {h64[n][0]:.9e} "
            f"|gpu-o32| {abs(hg[n][0] - h32[n][0]):.2e} spread {spread:.2e}")
        assert abs(hg[n][0] - h32[n][0]) <= gate, f"{label} outer step {n}"
    return i32, i64


def solver(d, L, lu, f, eps, centre, radius, **kw):
    from paper_1903_10367_amd import Solver
    return Solver(d, 1, L, f, eps_blocks=eps, ball=(centre, radius, lu), precision="fp32_refined", inner_k=K, **kw)


@pytest.mark.parametrize("damping", ["jac", "none"])
def test_2d_disk_outer_steps(damping):
    say("case mixed adaptive 2d disk L=4", damping)
    eps = inp.eps_blocks(2, 2, 2.0, seed=90)
    f = inp.rhs(2, 4, seed=91)
    s = solver(2, 4, 2, f, eps, (0.5, 0.5), 0.2, damping=damping)
    steps = 5
    s.cycle(steps)
    ug = s.solution()          # iterate `steps`: the pending correction is added on read-out
    s.cycle(1)                 # measures that iterate in FP64
    hg = s.residuals()
    s.close()
    T = adaptive.AdaptiveTree(2, 4, 1, 2, inp.refine_ball(2, 4, 2, (0.5, 0.5), 0.2), eps)
    check_steps(T, f, hg, steps + 1, label="2d", damping=damping)
    # the read-out function is the one the next step measured: its FP64 composite residual,
    # from the oracle, is the GPU's (FP64 rounding only)
    U = storage_from_finest(T, ug)
    _, nr = adaptive.composite_residual(T, U, T.load(f))
    say(f"read-out function: oracle residual {nr[0]:.9e}, GPU {hg[steps][0]:.9e}")
    assert abs(nr[0] - hg[steps][0]) <= 1e-12 * hg[0][0]
    # and it is the oracle's iterate to FP32 resolution (100 eps32 of its size)
    i64 = []
    adaptive.defect_correction(T, f, K, 0.0, steps, np.float64, i64, damping=damping)
    F64 = adaptive.finest_values(T, i64[steps])
    err = np.abs(ug.reshape(F64.shape) - F64).max()
    say(f"|gpu - oracle64| {err:.3e} of {np.abs(F64).max():.3e}")
    assert err <= 100 * np.finfo(np.float32).eps * np.abs(F64).max()


def test_3d_ball_outer_steps():
    say("case mixed adaptive 3d ball L=3")
    eps = inp.eps_blocks(3, 1, 2.0, seed=92)
    f = inp.rhs(3, 3, seed=93)
    c = (0.45, 0.5, 0.55)
    s = solver(3, 3, 2, f, eps, c, 0.15)
    s.cycle(4)
    hg = s.residuals()
    s.close()
    T = adaptive.AdaptiveTree(3, 3, 1, 2, inp.refine_ball(3, 3, 2, c, 0.15), eps)
    check_steps(T, f, hg, 4, label="3d")


@pytest.mark.parametrize("transfer", ["dlinear", "boxmg"])
def test_disk_workload_l6_outer_steps(transfer):
    say("case mixed adaptive 2d disk workload L=6", transfer)
    eps = inp.eps_blocks(2, 2, 3.0, seed=94)
    f = inp.rhs(2, 6, seed=95)
    s = solver(2, 6, 2, f, eps, (0.5, 0.5), 0.25, transfer=transfer)
    s.cycle(2)
    hg = s.residuals()
    s.close()
    T = adaptive.AdaptiveTree(2, 6, 1, 2, inp.refine_ball(2, 6, 2, (0.5, 0.5), 0.25), eps, transfer=transfer)
    check_steps(T, f, hg, 2, label="L6")


@pytest.mark.parametrize("d", [2, 3])
def test_solve_below_fp32_resolution(d):
    say("case mixed adaptive solve 1e-11", d)
    L = 4 if d == 2 else 3
    c = (0.5,) * d
    rad = 0.2 if d == 2 else 0.15
    eps = inp.eps_blocks(d, 1, 1.0, seed=96)
    f = inp.rhs(d, L, seed=97)
    s = solver(d, L, 2, f, eps, c, rad)
    n = s.solve(1e-11, 400)
    hg = s.residuals()
    ug = s.solution()
    s.close()
    T = adaptive.AdaptiveTree(d, L, 1, 2, inp.refine_ball(d, L, 2, c, rad), eps)
    _, h64 = adaptive.defect_correction(T, f, K, 1e-11, 400, np.float64)
    say(f"outer steps gpu {n}, oracle64 {len(h64)}; final rel {hg[-1][0] / hg[0][0]:.3e}")
    assert hg[-1][0] / hg[0][0] <= 1e-11
    assert abs(n - len(h64)) <= 1
    # FP64 residual of the returned function, from the oracle
    U = storage_from_finest(T, ug)
    _, nr = adaptive.composite_residual(T, U, T.load(f))
    say(f"oracle residual of the GPU solution {nr[0]:.6e}, GPU's own {hg[-1][0]:.6e}")
    assert abs(nr[0] - hg[-1][0]) <= 1e-12 * hg[0][0]
    if d == 2:
        A, b, pos, lev, Psi, C = adaptive.dense_system(T, f)
        ustar = np.linalg.solve(A, b)
        u = adaptive.to_composite(T, U)
        bound = np.linalg.norm(b - A @ u) / np.linalg.eigvalsh(A)[0]
        say(f"|u - u*| {np.linalg.norm(u - ustar):.3e} bound {bound:.3e}")
        assert np.linalg.norm(u - ustar) <= bound * (1 + 1e-6) + 1e-14 * np.linalg.norm(ustar)


def test_regrid_between_outer_steps():
    """Outer steps on one tree, regrid (the pending correction is added first), outer steps on
    the moved tree with a new right-hand side."""
    say("case mixed adaptive regrid 2d")
    eps = inp.eps_blocks(2, 1, 2.0, seed=98)
    f1, f2 = inp.rhs(2, 4, seed=99), inp.rhs(2, 4, seed=100)
    c1, c2 = (0.45, 0.5), (0.55, 0.52)
    s = solver(2, 4, 2, f1, eps, c1, 0.2)
    s.cycle(3)
    s.regrid(c2, 0.2, 2, f2)
    s.cycle(3)
    hg = s.residuals()
    s.close()
    T1 = adaptive.AdaptiveTree(2, 4, 1, 2, inp.refine_ball(2, 4, 2, c1, 0.2), eps)
    T2 = adaptive.AdaptiveTree(2, 4, 1, 2, inp.refine_ball(2, 4, 2, c2, 0.2), eps)
    check_steps(T1, f1, hg[:3], 3, label="before")
    i32, i64 = [], []
    adaptive.defect_correction(T1, f1, K, 0.0, 3, np.float32, i32)
    adaptive.defect_correction(T1, f1, K, 0.0, 3, np.float64, i64)
    U0 = (adaptive.transfer(T1, i32[3], T2), adaptive.transfer(T1, i64[3], T2))
    check_steps(T2, f2, hg[3:], 3, U0=U0, label="after")


def test_3d_tiled_restriction_outer_steps(monkeypatch):
    """FP32_REFINED with the tiled 3D restriction on every level (the composite-residual-only
    FP64 pass and the FP32 Jacobi cycles)."""
    monkeypatch.setenv("ADAFAC_AD_TILED_MIN_TILES", "0")
    say("case mixed adaptive 3d tiled restriction")
    eps = inp.eps_blocks(3, 1, 2.0, seed=101)
    f = inp.rhs(3, 4, seed=102)
    c = (0.45, 0.5, 0.55)
    s = solver(3, 4, 2, f, eps, c, 0.2)
    s.cycle(3)
    hg = s.residuals()
    s.close()
    T = adaptive.AdaptiveTree(3, 4, 1, 2, inp.refine_ball(3, 4, 2, c, 0.2), eps)
    check_steps(T, f, hg, 3, label="3d tiled")
