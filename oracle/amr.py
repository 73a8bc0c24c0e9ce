"""Feature-based dynamic refinement of the Sec. 5 runs, with the full-multigrid-like start.

TEST INFRASTRUCTURE (part of the oracle package; see its header).

The runs of Sec. 5 (text around the description of the experimental set-up):

* They start from a two-grid tree (l_max = 2) and add levels up to l_max = 8.
* In every other cycle the cells along the bottom boundary (those with a face that carries
  u = 1) are refined, until the grid meets l_max.
* In parallel, the absolute second derivatives of the solution along each coordinate axis are
  measured in every unknown; a bin sort picks the vertices with the (approximately) 10 percent
  largest directional derivatives, and they are refined unless they already sit on l_max.
* Coarse-grid solutions serve as initial guesses on the refined grids; new vertices take the
  d-linear interpolation (as hanging vertices do).

Readings (the text does not fix them): the second derivative at a dof is the second difference
along each axis on the dof's level, and the vertex's value is the largest over the axes;
"refining a vertex" refines the 2^d cells of its level around it; the bin sort uses 1024 equal
bins over [0, max] and takes whole bins from the top until they hold at least the fraction;
the boundary refinement marks the finest level's cells with a face whose corners all carry
nonzero data.  Parity unpinned by the paper beyond these definitions.
"""
import numpy as np

from . import adaptive

BINS = 1024


def mark(T, U, fraction, l_uniform, l_cap, trace=None):
    """Refinement flags {l: bool array over the (3^l)^d cells} of the next tree, l_uniform <= l <
    l_cap, and its depth.  U: the current per-level storage (spread: dofs, hanging values and
    boundary data).  ``trace`` (a dict) receives the dofs' (level, index), values and the
    selected ones."""
    d, L = T.d, T.L
    U = T.spread(U)
    flags = {l: np.zeros((3 ** l,) * d, dtype=bool) for l in range(l_uniform, l_cap)}
    # the cells the current tree refines
    for l in range(l_uniform, min(L, l_cap)):
        flags[l] |= T.Rf[l]
    # the finest level's cells with a face whose corners all carry nonzero Dirichlet data
    if L < l_cap and T.g is not None:
        m = 3 ** L
        nz = T.g[L] != 0.0
        E = T.E[L]
        for a in range(d):                    # array axis a (axis 0 is the last coordinate)
            for f in (0, m):
                # corners of the faces at coordinate f along axis a: the vertex plane there
                plane = np.take(nz, f, axis=a)
                allc = plane.copy()
                # a face of a cell (index c along the other axes) has corners c and c + 1 along
                # each of the other d - 1 axes
                for b in range(d - 1):
                    n = allc.shape[b] - 1
                    allc = np.take(allc, np.arange(n), axis=b) & np.take(allc, np.arange(1, n + 1), axis=b)
                cellidx = 0 if f == 0 else m - 1
                sl = [slice(None)] * d
                sl[a] = cellidx
                sel = np.zeros_like(E)
                sel[tuple(sl)] = allc
                flags[L] |= sel & E
    # the composite dofs with the largest directional second derivatives
    vals, where = [], []
    for l in range(T.lmin, L + 1):
        m = 3 ** l
        h2 = 1.0 / (float(m) * m)
        u = U[l]
        idx = np.argwhere(T.comp[l])
        if not len(idx):
            continue
        v = np.zeros(len(idx))
        for a in range(d):
            e = np.zeros(d, dtype=int)
            e[a] = 1
            up = u[tuple((idx + e).T)]
            um = u[tuple((idx - e).T)]
            u0 = u[tuple(idx.T)]
            v = np.maximum(v, np.abs(up - 2.0 * u0 + um) / h2)
        vals.append(v)
        where += [(l, tuple(i)) for i in idx]
    if trace is not None:
        trace["dofs"] = where
        trace["values"] = np.concatenate(vals) if vals else np.zeros(0)
        trace["selected"] = np.zeros(len(where), dtype=bool)
    if vals and fraction > 0.0:
        v = np.concatenate(vals)
        vmax = float(v.max())
        b = np.minimum(BINS - 1, (v / vmax * BINS).astype(int)) if vmax > 0.0 else np.zeros(len(v), dtype=int)
        cnt = np.bincount(b, minlength=BINS)
        want = fraction * float(len(v))
        cut, have = BINS, 0
        while cut > 0 and float(have) < want:
            cut -= 1
            have += int(cnt[cut])
        if trace is not None:
            trace["selected"] = b >= cut
        for k in np.flatnonzero(b >= cut):
            l, i = where[k]
            if l >= l_cap or l < l_uniform:
                continue
            for corner in np.ndindex(*(2,) * d):
                flags[l][tuple(i[a] - 1 + corner[a] for a in range(d))] = True
    top = L
    for l in range(l_uniform, l_cap):
        if flags[l].any():
            top = max(top, l + 1)
    return flags, top


def upsample_to(F, levels):
    """d-linear interpolation of a finest-lattice function by `levels` levels."""
    for _ in range(levels):
        F = adaptive._upsample(F)
    return F


def grow(T, U, flags, l_new, l_uniform, eps=None, g_of=None):
    """The next tree (depth l_new, flags for l_uniform..l_new-1) with the composite function of
    (T, U) as its iterate; g_of(L) gives the Dirichlet data on the depth-L lattice."""
    d = T.d
    refine = {l: flags[l] for l in range(l_uniform, l_new)}
    T2 = adaptive.AdaptiveTree(d, l_new, T.lmin, l_uniform, refine, eps, omega=T.omega, transfer=T.transfer,
                               g=None if g_of is None else g_of(l_new))
    F = upsample_to(adaptive.finest_values(T, U), l_new - T.L)
    U2 = {}
    for l in range(T2.lmin, l_new + 1):
        s = 3 ** (l_new - l)
        U2[l] = np.where(T2.dof[l], F[tuple(slice(None, None, s) for _ in range(d))], 0.0)
    return T2, T2.spread(U2)


def run(d, l_start, l_cap, cycles, g_of, eps=None, fraction=0.1, every=2, l_uniform=None, **kw):
    """Cycles on the growing tree: a uniform tree of depth l_start, then after every `every`-th
    cycle the marks above and a move onto the next tree.  Returns the per-cycle (norms, depth,
    composite dofs) and the list of (flags, depth) of every move."""
    lu = l_start if l_uniform is None else l_uniform
    T = adaptive.AdaptiveTree(d, l_start, 1, l_start, {}, eps, g=g_of(l_start))
    U = T.spread({l: np.zeros(T.shape(l)) for l in range(1, l_start + 1)})
    hist, moves = [], []
    for n in range(cycles):
        bleaf = T.load(np.zeros(T.shape(T.L)))
        U, nr = adaptive.cycle(T, U, bleaf, **kw)
        hist.append((nr, T.L, len(T.composite_index())))
        if (n + 1) % every == 0 and n + 1 < cycles:
            flags, top = mark(T, U, fraction, lu, l_cap)
            moves.append((flags, top))
            T, U = grow(T, U, flags, top, lu, eps, g_of)
    return hist, moves
