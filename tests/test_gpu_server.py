"""Request server (continuous batching) through the C ABI.

Every request, of any depth and dimension, advances in shared phase-slot launches whose work
items are the phases of all requests' cycles (the largest ones sweep their finest level in a
launch of their own).  Checked here:

- A served request gives the same iterate as the one-kernel-per-step solver.
- Its cycle count and solution match the oracle.
- Each result is bitwise the same served alone and in a mix, including a mix with staggered
  arrivals.
- Admission honours the device-memory budget, and later requests are admitted as memory frees.
- The queue limit and impossible requests are reported.
"""
import sys

import numpy as np
import pytest

import adafac_inputs as inp
from oracle import cycle, hierarchy

pytestmark = pytest.mark.gpu

MB = 1 << 20


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def requests():
    """A mix of dimensions, depths, coefficients and precisions (2D and 3D, batched and not)."""
    return [
        dict(dim=2, lmin=1, lmax=3, f=inp.rhs(2, 3, seed=40), eps_blocks=inp.eps_blocks(2, 2, 3.0, seed=41)),
        dict(dim=3, lmin=1, lmax=3, f=inp.rhs(3, 3, seed=42), precision="fp32_refined", inner_k=4),
        dict(dim=2, lmin=1, lmax=5, f=inp.rhs(2, 5, seed=43), eps_blocks=inp.eps_blocks(2, 2, 3.0, seed=44)),
        dict(dim=3, lmin=1, lmax=4, f=inp.rhs(3, 4, seed=45, dist="normal")),
        dict(dim=2, lmin=1, lmax=6, f=inp.rhs(2, 6, seed=46), precision="fp32_refined", inner_k=8),
        dict(dim=2, lmin=2, lmax=4, f=inp.rhs(2, 4, seed=47), damping="pi"),
    ]


def serve(reqs, budget=2048 * MB, stagger=0, **cfg):
    """Serve reqs; with stagger > 0 the second half arrives after that many rounds."""
    from paper_1903_10367_amd import Server
    srv = Server(budget, **cfg)
    tickets = [None] * len(reqs)
    first = reqs if not stagger else reqs[: len(reqs) // 2]
    for i, r in enumerate(first):
        tickets[i] = srv.submit(**r)
    rounds = 0
    import time
    t0 = time.perf_counter()
    while True:
        a, q = srv.step()
        rounds += 1
        if stagger and rounds == stagger:
            for i in range(len(reqs) // 2, len(reqs)):
                tickets[i] = srv.submit(**reqs[i])
            continue
        if a == 0 and q == 0 and (not stagger or rounds >= stagger):
            break
        assert time.perf_counter() - t0 < 300, "the server did not drain"
    out = []
    for t in tickets:
        res = srv.poll(t)
        out.append((res, srv.fetch(t)))
    srv.close()
    return out


def test_batched_request_equals_one_kernel_per_step_solver():
    from paper_1903_10367_amd import Solver
    f = inp.rhs(2, 4, seed=48)
    say("case server vs solver, 2D L=4")
    [(res, u)] = serve([dict(dim=2, lmin=1, lmax=4, f=f, rel_tol=1e-8)])
    assert res["state"] == "converged" and res["batched"] == 1
    s = Solver(2, 1, 4, f, fused=False)
    n = s.solve(1e-8, 200)
    us = s.solution()
    hs = s.residuals()
    s.close()
    say(f"served cycles {res['cycles']}, solver cycles {n}, identical {np.array_equal(u, us)}")
    assert res["cycles"] == n
    assert np.abs(u - us).max() <= 1e-14 * np.abs(us).max()
    assert abs(res["l2h0"] - hs[0][0]) <= 1e-14 * hs[0][0]


@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_served_results_match_oracle(k):
    r = requests()[k]
    say("case server vs oracle", k, r["dim"], r["lmax"])
    [(res, u)] = serve([dict(r, rel_tol=1e-8, max_cycles=600)])
    assert res["state"] == "converged", res
    H = hierarchy.Hierarchy(r["dim"], r["lmax"], r["lmin"], r.get("eps_blocks"))
    b = H.rhs(r["f"])
    if r.get("precision") == "fp32_refined":
        uo, ho, _ = cycle.defect_correction(H, b, r["inner_k"], 1e-8, 600)
        # the oracle's FP64 defect of the served iterate meets the tolerance, as the oracle's own
        rel = cycle.norms(H, b - H.lev[H.L].A(u))[0] / ho[0][0]
        say(f"outer steps {res['cycles']} (oracle {len(ho)}), final rel. residual {rel:.3e}")
        assert rel <= 1e-8 * (1 + 1e-6) and abs(res["cycles"] - len(ho)) <= 1
        return
    uo, ho = cycle.solve(H, b, 600, tol=1e-8, damping=r.get("damping", "jac"))
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    say(f"cycles {res['cycles']} (oracle {len(ho)}), rel. error {err:.3e}")
    assert res["cycles"] == len(ho)
    assert abs(res["l2h0"] - ho[0][0]) <= 1e-12 * ho[0][0]
    assert err <= 1e-12


def test_alone_and_in_the_mix_are_identical():
    reqs = [dict(r, rel_tol=1e-8, max_cycles=600) for r in requests()]
    say("case alone vs mix")
    alone = [serve([r])[0] for r in reqs]
    mixed = serve(reqs)
    staggered = serve(reqs, stagger=3)
    for i, ((ra, ua), (rm, um), (rs, us)) in enumerate(zip(alone, mixed, staggered)):
        say(f"request {i}: {ra['state']} batched={ra['batched']} cycles {ra['cycles']} / {rm['cycles']} / "
            f"{rs['cycles']}")
        assert ra["state"] == rm["state"] == rs["state"] == "converged"
        assert ra["cycles"] == rm["cycles"] == rs["cycles"]
        assert np.array_equal(ua, um) and np.array_equal(ua, us)
    assert {r["batched"] for r, _ in alone} == {1}


def test_served_large_requests_match_oracle():
    """The largest shapes of the serving mix in the same launch: 3D L = 5 (243^3 cells) with 27^3
    coefficient blocks 10^U(0,4) in FP64, and 2D L = 7 (2187^2 cells) with 9 x 9 blocks, capped at
    3 cycles and checked cycle by cycle against the oracle (norms) and in the iterate."""
    eps3 = inp.eps_blocks(3, 3, 4.0, seed=62)
    f3 = inp.rhs(3, 5, seed=63)
    eps2 = inp.eps_blocks(2, 2, 3.0, seed=64)
    f2 = inp.rhs(2, 7, seed=65)
    say("case served large requests")
    reqs = [dict(dim=3, lmin=1, lmax=5, f=f3, eps_blocks=eps3, rel_tol=1e-12, max_cycles=3),
            dict(dim=2, lmin=1, lmax=7, f=f2, eps_blocks=eps2, rel_tol=1e-12, max_cycles=3),
            dict(dim=2, lmin=1, lmax=3, f=inp.rhs(2, 3, seed=66), rel_tol=1e-8)]
    out = serve(reqs)
    assert all(r["batched"] == 1 for r, _ in out)
    for (res, u), r in zip(out[:2], reqs[:2]):
        assert res["state"] == "capped" and res["cycles"] == 3, res
        say("oracle", r["dim"], r["lmax"])
        H = hierarchy.Hierarchy(r["dim"], r["lmax"], 1, r["eps_blocks"])
        b = H.rhs(r["f"])
        uo, ho = cycle.solve(H, b, 3)
        err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
        say(f"rel. error {err:.3e}, l2h {res['l2h']:.6e} vs {ho[-1][0]:.6e}")
        assert abs(res["l2h0"] - ho[0][0]) <= 1e-12 * ho[0][0]
        assert abs(res["l2h"] - ho[-1][0]) <= 1e-12 * ho[0][0]
        assert err <= 1e-12
    assert out[2][0]["state"] == "converged"


def _check_swept_fp32(res, u, d, L, f, eps, k):
    """A served FP32_REFINED request capped at 3 outer steps against the oracle's iterate after 2
    outer steps (FP32 inner cycles) and against the one-request solver."""
    assert res["state"] == "capped" and res["cycles"] == 3, res
    H = hierarchy.Hierarchy(d, L, 1, eps)
    b = H.rhs(f)
    i32, i64 = [], []
    _, h32, _ = cycle.defect_correction(H, b, k, 0.0, 2, inner_dtype=np.float32, iterates=i32)
    cycle.defect_correction(H, b, k, 0.0, 2, inner_dtype=np.float64, iterates=i64)
    A = H.lev[H.L].A
    spread = cycle.norms(H, A(i32[2]) - A(i64[2]))[0]
    say(f"FP32 {d}D L={L}: l2h {res['l2h']:.6e} vs {h32[2][0]:.6e}, spread {spread:.2e}")
    assert abs(res["l2h0"] - h32[0][0]) <= 1e-12 * h32[0][0]
    assert abs(res["l2h"] - h32[2][0]) <= 4 * spread + 1e-12 * h32[0][0]
    # the iterate, in the norm of the stopping rule: the served and the oracle's FP32 iterates
    # differ by no more than 4x the oracle's own FP32 rounding (the 2-norm of the difference is
    # dominated by smooth components that the two FP32 evaluations round differently; printed)
    dr = cycle.norms(H, A(u) - A(i32[2]))[0]
    err, sp = np.linalg.norm(u - i32[2]), np.linalg.norm(i32[2] - i64[2])
    say(f"  ||A(gpu - oracle32)||_h {dr:.3e}; 2-norm |gpu - oracle32| {err:.3e}, |oracle32 - oracle64| {sp:.3e}")
    assert dr <= 4 * spread + 1e-12 * h32[0][0]
    # the served iterate is the one-request solver's (same one-pass kernels on the finest level;
    # the coarse levels differ at most in rounding order)
    from paper_1903_10367_amd import Solver
    sv = Solver(d, 1, L, f, eps_blocks=eps, precision="fp32_refined", inner_k=k)
    sv.cycle(2)
    us = sv.solution()
    sv.close()
    ds = np.linalg.norm(u - us)
    say(f"  |served - solver| {ds:.3e}")
    assert ds <= 0.1 * sp + 1e-12 * np.linalg.norm(us)


def test_served_swept_requests_match_oracle():
    """Requests large enough to sweep their finest level in one pass (a launch of their own, the
    prolongation into it left pending): 2D L = 6 under adAFAC-PI (the prolongation into level
    L-1 subtracts I c_L) in FP64, capped at 3 cycles, exact against the oracle; 2D L = 6 in FP32
    cycles inside FP64 defect correction (the outer step adds e + P S_{L-1}) and 3D L = 4 in the
    same precision (the outer step in one pass, u + e + P S_{L-1} and the FP64 defect, into the
    other FP64 buffer), each capped at 3 outer steps."""
    f = inp.rhs(2, 6, seed=67)
    eps = inp.eps_blocks(2, 2, 3.0, seed=68)
    f3 = inp.rhs(3, 4, seed=69)
    eps3 = inp.eps_blocks(3, 3, 4.0, seed=70)
    say("case served swept requests")
    reqs = [dict(dim=2, lmin=1, lmax=6, f=f, eps_blocks=eps, damping="pi", rel_tol=1e-12, max_cycles=3),
            dict(dim=2, lmin=1, lmax=6, f=f, eps_blocks=eps, precision="fp32_refined", inner_k=4, rel_tol=1e-12,
                 max_cycles=3),
            dict(dim=3, lmin=1, lmax=4, f=f3, eps_blocks=eps3, precision="fp32_refined", inner_k=4, rel_tol=1e-12,
                 max_cycles=3)]
    out = serve(reqs)
    H = hierarchy.Hierarchy(2, 6, 1, eps)
    b = H.rhs(f)
    (res, u) = out[0]
    assert res["state"] == "capped" and res["cycles"] == 3, res
    uo, ho = cycle.solve(H, b, 3, damping="pi")
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    say(f"PI: rel. error {err:.3e}, l2h {res['l2h']:.6e} vs {ho[-1][0]:.6e}")
    assert abs(res["l2h0"] - ho[0][0]) <= 1e-12 * ho[0][0]
    assert abs(res["l2h"] - ho[-1][0]) <= 1e-12 * ho[0][0]
    assert err <= 1e-12
    _check_swept_fp32(*out[1], 2, 6, f, eps, 4)
    _check_swept_fp32(*out[2], 3, 4, f3, eps3, 4)


def test_admission_waits_for_memory_and_slots():
    # four equal 3D L=4 requests and a pool that holds two of them
    from paper_1903_10367_amd import Server
    reqs = [dict(dim=3, lmin=1, lmax=4, f=inp.rhs(3, 4, seed=50 + i), rel_tol=1e-8) for i in range(4)]
    probe = serve([reqs[0]])[0][0]
    fp = probe["footprint"]
    say("case admission, footprint", fp)
    srv = Server(2 * fp + 8 * MB, max_streams=4)
    tickets = [srv.submit(**r) for r in reqs]
    peak = 0
    while True:
        a, q = srv.step()
        states = [srv.poll(t) for t in tickets]
        running = [s for s in states if s["state"] == "running"]
        assert sum(s["footprint"] for s in running) <= 2 * fp + 8 * MB
        peak = max(peak, len(running))
        if a == 0 and q == 0:
            break
    states = [srv.poll(t) for t in tickets]
    for t in tickets:
        srv.fetch(t)
    srv.close()
    assert peak == 2
    assert all(s["state"] == "converged" for s in states)
    # the last two admitted (a request whose host set-up finished first may pass an earlier one)
    # were admitted only after one of the first two had finished
    by_admit = sorted(states, key=lambda s: s["t_admit"])
    first_done = min(s["t_done"] for s in by_admit[:2])
    assert min(s["t_admit"] for s in by_admit[2:]) >= first_done


def test_queue_limit_and_impossible_request():
    from paper_1903_10367_amd import Server
    say("case queue limit")
    srv = Server(64 * MB, max_queued=2)
    f = inp.rhs(2, 3, seed=60)
    t1 = srv.submit(2, 1, 3, f)
    t2 = srv.submit(3, 1, 5, inp.rhs(3, 5, seed=61))   # far beyond a 64 MB pool
    assert srv.submit(2, 1, 3, f) is None               # queue full
    srv.run_until_idle()
    assert srv.poll(t1)["state"] == "converged"
    r2 = srv.poll(t2)
    assert r2["state"] == "failed" and r2["error"] == 3   # ADAFAC_ENOMEM
    srv.fetch(t1)
    srv.fetch(t2)
    srv.close()
