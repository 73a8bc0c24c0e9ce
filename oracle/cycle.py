"""One additive adAFAC cycle, its variants, residual norms and FP32 defect correction.

The cycle is eq. (adaFACx) / Algorithm 1 of the paper (Sec. 3.1):

    u <- u + sum_{l=lmin}^{L}   P^{L-l} omega D_l^{-1} R^{L-l} r
           - sum_{l=lmin}^{L-1} P^{L-l} omega~ D_l^{-1} R~ R^{L-l-1} r,     r = b - A_L u,

i.e. every level takes one damped Jacobi step from a zero guess on its
restricted residual, and every level below L additionally solves (one Jacobi
step) an auxiliary equation whose right-hand side is the smoothed restriction
R~ of the next finer level's residual; its result damps the finer level's
correction.  The coarsest level gets no damping term (the garbled
"M_{lmax-1}^{-1} = 0" is read as: no level below lmin, Sec. 3.1).

Readings taken where the paper is silent (listed with the rest in the design
notes of the repository): omega = 0.6 (Sec. 5), omega~ = omega, omega_add = 1
with the Jacobi damping inside M^{-1} = omega D^{-1}, u^0 = 0.

``cycle_correction`` evaluates the corrections level by level from restricted
residuals (the AFAC correction form).  ``cycle_fas`` carries the full
approximation storage of Sec. 2.4: coarse levels hold the injected solution,
their right-hand side is the restricted hierarchical residual
R (b - A (u - P I u)) (eq. (fas-with-htmg)), and their residual is
b_l - A_l u_l.  Under Ritz-Galerkin operators both forms give the same
iterates in exact arithmetic.

Variants (Sec. 3.2, Sec. 5.1): damping "jac" (adAFAC-Jac, auxiliary equation
with R~), "pi" (adAFAC-PI, c~_l = P I c_l on the level itself, Algorithm 2),
"none" (plain additive multigrid, eq. (additive-mg)) and "exp" (exponential
damping omega_add(l) = omega_hat^(L-l)).
"""
import numpy as np


def norms(H, r):
    """h-weighted l2 norm sqrt(sum_i h^d r_i^2) and max |r_i| over dofs (Sec. 5, normalised residual)."""
    lv = H.lev[H.L]
    ri = np.asarray(r, dtype=np.float64)[lv.mask.ravel()]
    if ri.size == 0:
        return 0.0, 0.0
    return float(np.sqrt(np.sum(lv.h ** H.d * ri * ri))), float(np.max(np.abs(ri)))


def _damping_terms(H, c, rhs_for_aux, damping, omega_t):
    """c~_l for every level: the subtracted damping correction living on level l."""
    L, lmin, lev = H.L, H.lmin, H.lev
    ct = {}
    for l in range(lmin, L + 1):
        ct[l] = np.zeros_like(c[l])
    if damping == "jac":
        # auxiliary equation one level coarser, zero initial guess, one Jacobi step
        for l in range(lmin, L):
            ct[l] = omega_t * lev[l].Dinv * rhs_for_aux[l]
    elif damping == "pi":
        # c~_l = P I c_l, none on the coarsest level
        for l in range(lmin + 1, L + 1):
            ct[l] = lev[l].P(lev[l].I(c[l]))
    return ct


def _accumulate(H, c, ct, trace=None):
    """u increment sum_l P^{L-l}(c_l - c~_l), accumulated from the coarsest level upwards."""
    S = c[H.lmin] - ct[H.lmin]
    if trace is not None:
        trace.setdefault("S", {})[H.lmin] = S
    for l in range(H.lmin + 1, H.L + 1):
        S = c[l] - ct[l] + H.lev[l].P(S)
        if trace is not None:
            trace["S"][l] = S
    return S


def _check(damping):
    assert damping in ("jac", "pi", "none", "exp")


def cycle_correction(H, u, b, omega=0.6, omega_t=0.6, damping="jac", omega_hat=0.5):
    """One cycle in correction form.  Returns (new iterate, residual of the old one)."""
    _check(damping)
    L, lmin, lev = H.L, H.lmin, H.lev
    r = b - lev[L].A(u)
    bl = {L: r}
    for l in range(L - 1, lmin - 1, -1):
        bl[l] = lev[l + 1].P.T(bl[l + 1])
    c = {l: omega * lev[l].Dinv * bl[l] for l in range(lmin, L + 1)}
    if damping == "exp":
        c = {l: omega_hat ** (L - l) * c[l] for l in c}
    aux = {l: lev[l + 1].Rt(bl[l + 1]) for l in range(lmin, L)} if damping == "jac" else {}
    ct = _damping_terms(H, c, aux, damping, omega_t)
    return u + _accumulate(H, c, ct), r


def cycle_fas(H, u, b, omega=0.6, omega_t=0.6, damping="jac", omega_hat=0.5, trace=None):
    """One cycle in FAS/HTMG form (Sec. 2.4, Algorithm 3's use of r and r^).

    Level l < L: u_l = I u_{l+1}; b_l = R r^_{l+1} with the hierarchical
    residual r^_{l+1} = b_{l+1} - A_{l+1}(u_{l+1} - P I u_{l+1}); the residual
    r_l = b_l - A_l u_l drives the Jacobi correction, and the auxiliary
    right-hand side is b~_l = R~ r_{l+1} (plain residual).  If ``trace`` is a dict it
    receives the per-level arrays u, b, btilde, r and S (for inspection only).
    """
    _check(damping)
    L, lmin, lev = H.L, H.lmin, H.lev
    ul, bF, rl, bt = {L: u}, {L: b}, {}, {}
    for l in range(L, lmin, -1):
        rl[l] = bF[l] - lev[l].A(ul[l])
        ul[l - 1] = lev[l].I(ul[l])
        uhat = ul[l] - lev[l].P(ul[l - 1])
        rhat = bF[l] - lev[l].A(uhat)
        bF[l - 1] = lev[l].P.T(rhat)
        bt[l - 1] = lev[l].Rt(rl[l])
    rl[lmin] = bF[lmin] - lev[lmin].A(ul[lmin])
    c = {l: omega * lev[l].Dinv * rl[l] for l in range(lmin, L + 1)}
    if damping == "exp":
        c = {l: omega_hat ** (L - l) * c[l] for l in c}
    ct = _damping_terms(H, c, bt, damping, omega_t)
    if trace is not None:
        trace.update(u=ul, b=bF, btilde=bt, r=rl)
    return u + _accumulate(H, c, ct, trace), rl[L]


def solve(H, b, max_cycles, tol=None, form="correction", u0=None, **kw):
    """Run cycles from u^0 = 0 (or u0).

    Cycle n forms the residual of iterate n and produces iterate n+1.  Stops
    after the first cycle whose input iterate satisfies ||r||_h / ||r^0||_h <=
    tol, or after ``max_cycles``.  Returns (u, [(l2h, linf) per cycle]).
    """
    cyc = cycle_fas if form == "fas" else cycle_correction
    u = np.zeros_like(b) if u0 is None else u0.copy()
    hist = []
    for _ in range(max_cycles):
        u_new, r = cyc(H, u, b, **kw)
        hist.append(norms(H, r))
        u = u_new
        if tol is not None and hist[0][0] > 0 and hist[-1][0] / hist[0][0] <= tol:
            break
    return u, hist


def defect_correction(H, b, k_inner, tol, max_outer, inner_dtype=np.float32, form="correction",
                      iterates=None, **kw):
    """FP64 defect correction around k inner adAFAC cycles in ``inner_dtype``.

    Outer step: r = b - A u in FP64; stop if ||r||_h/||r^0||_h <= tol;
    otherwise solve A e = r approximately with k cycles from e = 0 computed
    entirely in ``inner_dtype`` (operators, smoothing, transfers, damping),
    then u <- u + e in FP64.  The cycle is linear, so in exact arithmetic k
    inner cycles equal k outer cycles.  Returns (u, outer residual history,
    total inner cycles); ``iterates`` (a list) receives every outer iterate.
    """
    L = H.L
    Hs = H.astype(inner_dtype)
    cyc = cycle_fas if form == "fas" else cycle_correction
    u = np.zeros_like(b)
    hist, inner = [], 0
    for _ in range(max_outer + 1):
        r = b - H.lev[L].A(u)
        hist.append(norms(H, r))
        if iterates is not None:
            iterates.append(u.copy())
        if hist[0][0] == 0 or hist[-1][0] / hist[0][0] <= tol or len(hist) > max_outer:
            break
        rs = r.astype(inner_dtype)
        e = np.zeros_like(rs)
        for _ in range(k_inner):
            e, _ = cyc(Hs, e, rs, **kw)
            inner += 1
        u = u + e.astype(np.float64)
    return u, hist, inner
