"""adafac_bind_static, the binding that allocates nothing: the library's own device array in place
of a caller workspace.  Its cycles must give exactly what adafac_bind gives on the same inputs,
on two binds in a row (the second hierarchy smaller, so stale contents of the first would show),
and a context whose array was taken by a later bind must refuse to cycle.  Runs through the C ABI
(Solver(static_workspace=True) calls adafac_bind_static)."""
import sys

import numpy as np
import pytest

import adafac_inputs as inp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solve(static, d, L, eps, f, cycles, precision, transfer="boxmg"):
    from paper_1903_10367_amd import Solver
    s = Solver(d, 1, L, f, eps_blocks=eps, transfer=transfer, precision=precision, inner_k=4,
               static_workspace=static)
    s.cycle(cycles)
    return s, s.residuals(), s.solution()


def test_static_workspace_gives_the_caller_workspace_results():
    from paper_1903_10367_amd import AdafacError, _abi
    cases = [
        # the larger hierarchy first: 3D L = 4 (82^3 vertices) in FP32 cycles + FP64 refinement
        (3, 4, 2, 4.0, 3, "fp32_refined"),
        # then a smaller one: 2D L = 4 (82^2 vertices) in FP64
        (2, 4, 2, 3.0, 8, "fp64"),
    ]
    prev = None
    for n, (d, L, k, decades, cycles, precision) in enumerate(cases):
        say("case static workspace", d, L, precision)
        eps = inp.eps_blocks(d, k, decades, seed=50 + n)
        f = inp.rhs(d, L, seed=60 + n)
        ref, hr, ur = _solve(False, d, L, eps, f, cycles, precision)
        ref.close()
        st, hs, us = _solve(True, d, L, eps, f, cycles, precision)
        assert len(hs) == len(hr) == cycles
        # same kernels, same launch shapes, same inputs: the same bits
        assert hs == hr
        assert np.array_equal(us, ur), np.max(np.abs(us - ur))
        assert np.isfinite(us).all() and np.linalg.norm(us) > 0
        if prev is not None:
            # the earlier context lost the array to this bind and refuses to cycle
            with pytest.raises(AdafacError) as ei:
                prev.cycle(1)
            assert ei.value.code == _abi.ESTATE
            prev.close()
        prev = st
    prev.close()


def test_static_workspace_rejects_a_hierarchy_beyond_its_size():
    from paper_1903_10367_amd import AdafacError, _abi
    # 2D L = 7 needs about 179 MiB of workspace
    with pytest.raises(AdafacError) as ei:
        _solve(True, 2, 7, None, np.zeros((3 ** 7 + 1) ** 2), 1, "fp64", transfer="dlinear")
    assert ei.value.code == _abi.ENOMEM
    assert "static workspace" in str(ei.value)
