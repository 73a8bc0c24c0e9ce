"""Tiny-grid tools: direct solve of the discrete system and the cycle's iteration matrix.

The paper states that all stable variants are real solvers that converge to
the same solution (Sec. 5.1); the direct solve is that solution.  The
iteration matrix E (the cycle applied to unit vectors with b = 0) gives the
asymptotic convergence factor rho(E) of a linear stationary iteration.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import cycle as cyc


def direct_solve(H, b):
    """u with A_L u = b on the dofs (boundary zero), by sparse LU."""
    lv = H.lev[H.L]
    m = lv.mask.ravel()
    A = lv.A.mat.tocsr()[m][:, m]
    u = np.zeros_like(b)
    u[m] = spla.spsolve(A.tocsc(), b[m])
    return u


def iteration_matrix(H, form="correction", **kw):
    """E with e_{n+1} = E e_n: the cycle applied to unit vectors of the dofs with b = 0."""
    lv = H.lev[H.L]
    m = lv.mask.ravel()
    idx = np.flatnonzero(m)
    f = cyc.cycle_fas if form == "fas" else cyc.cycle_correction
    E = np.zeros((idx.size, idx.size))
    zero = np.zeros(m.size)
    for j, i in enumerate(idx):
        e = np.zeros(m.size)
        e[i] = 1.0
        E[:, j] = f(H, e, zero, **kw)[0][idx]
    return E


def spectral_radius(E):
    return float(np.max(np.abs(np.linalg.eigvals(E))))
