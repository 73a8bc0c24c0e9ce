"""Inter-grid transfers between two uniform levels of the 3:1 spacetree.

* d-linear prolongation (Sec. 2.5 "geometric" choice; Sec. 3.2 switch),
* BoxMG operator-dependent prolongation for 3-partitioning (Sec. 2.5),
* injection of a fine vertex value into the coinciding coarse vertex (Sec. 2.4).

Restriction is the transpose of prolongation, R = P^T (the Ritz-Galerkin
setting of Sec. 2.2; the paper does not state a scaling, this is the unscaled
reading).  All matrices act on full vertex lattices (C order, x last) with
boundary rows and columns removed.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from .fem import interior_mask


def linear_1d(nc):
    """1D linear interpolation from ``nc`` coarse cells to ``3 nc`` fine cells.

    Fine vertex i = 3c + s takes (1 - s/3) of coarse vertex c and s/3 of c+1.
    """
    nf = 3 * nc
    rows, cols, vals = [], [], []
    for i in range(nf + 1):
        c, s = divmod(i, 3)
        rows.append(i); cols.append(c); vals.append((3 - s) / 3.0)
        if s:
            rows.append(i); cols.append(c + 1); vals.append(s / 3.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf + 1, nc + 1))


def _mask_diag(d, level):
    return sp.diags(interior_mask(d, level).ravel().astype(np.float64))


def dlinear_prolongation(d, level_f):
    """d-linear P from level ``level_f - 1`` to ``level_f``: tensor product of 1D linear."""
    P1 = linear_1d(3 ** (level_f - 1))
    P = P1
    for _ in range(d - 1):
        P = sp.kron(P1, P, format="csr")
    return (_mask_diag(d, level_f) @ P @ _mask_diag(d, level_f - 1)).tocsr()


def injection(d, level_f):
    """I: coarse vertex v takes the value of the fine vertex at 3v (Sec. 2.4)."""
    nc = 3 ** (level_f - 1)
    cshape = (nc + 1,) * d
    fshape = (3 * nc + 1,) * d
    idx = np.indices(cshape).reshape(d, -1)
    rows = np.ravel_multi_index(idx, cshape)
    cols = np.ravel_multi_index(3 * idx, fshape)
    I = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(rows.size, int(np.prod(fshape))))
    return (_mask_diag(d, level_f - 1) @ I @ _mask_diag(d, level_f)).tocsr()


def boxmg_prolongation(A_f, d, level_f):
    """BoxMG prolongation for 3-partitioning (Sec. 2.5), built from the fine operator.

    For every coarse cell and every one of its corners e, the column of P for e
    restricted to the closed cell is determined by
      * c-points (fine vertices on coarse vertices): identity, 1 at e, 0 elsewhere;
      * gamma-points (on coarse edges/faces): the fine stencil is lumped
        (summed) along every direction normal to the edge/face, and the
        collapsed homogeneous equations are solved for the points inside that
        edge/face, with the values on its boundary as data.  Edges come
        before faces (collapsing "iteratively", lower dimension first);
      * f-points (strictly inside the coarse cell): A P e = 0 with the full
        stencil, values on the cell boundary as data.
    A gamma-point's equations involve only the corners of its edge/face, so
    cells sharing it compute the same weights.  Edges and faces on the domain
    boundary hold no degrees of freedom and get zero weights; couplings to
    boundary vertices multiply zero values.
    """
    A_f = sp.csr_matrix(A_f)
    nc = 3 ** (level_f - 1)
    nf = 3 * nc
    fshape = (nf + 1,) * d
    cshape = (nc + 1,) * d
    fmask = interior_mask(d, level_f)
    cmask = interior_mask(d, level_f - 1)

    def entry_row(g):
        gi = np.ravel_multi_index(g, fshape)
        lo, hi = A_f.indptr[gi], A_f.indptr[gi + 1]
        return dict(zip(A_f.indices[lo:hi].tolist(), A_f.data[lo:hi].tolist()))

    offs = list(itertools.product((-1, 0, 1), repeat=d))
    rows, cols, vals = [], [], []
    # sub-faces of the reference cell {0..3}^d, by dimension: free axes vary in {1,2}
    subfaces = []
    for m in range(1, d + 1):
        for free in itertools.combinations(range(d), m):
            fixed = [a for a in range(d) if a not in free]
            for fixed_vals in itertools.product((0, 3), repeat=len(fixed)):
                subfaces.append((free, dict(zip(fixed, fixed_vals))))

    for cell in itertools.product(range(nc), repeat=d):
        base = tuple(3 * c for c in cell)
        for corner in itertools.product((0, 1), repeat=d):
            cv = tuple(cell[a] + corner[a] for a in range(d))
            if not cmask[cv]:
                continue
            val = {}
            for loc in itertools.product((0, 3), repeat=d):
                val[loc] = 1.0 if loc == tuple(3 * c for c in corner) else 0.0
            for free, fixed in subfaces:
                pts = []
                for fv in itertools.product((1, 2), repeat=len(free)):
                    loc = [0] * d
                    for a, v in zip(free, fv):
                        loc[a] = v
                    for a, v in fixed.items():
                        loc[a] = v
                    pts.append(tuple(loc))
                on_boundary = any(base[a] + v in (0, nf) for a, v in fixed.items())
                if on_boundary:
                    for p in pts:
                        val[p] = 0.0
                    continue
                index = {p: k for k, p in enumerate(pts)}
                M = np.zeros((len(pts), len(pts)))
                rhs = np.zeros(len(pts))
                for k, p in enumerate(pts):
                    g = tuple(base[a] + p[a] for a in range(d))
                    row = entry_row(g)
                    coll = {}
                    for o in offs:
                        w = tuple(g[a] + o[a] for a in range(d))
                        if any(x < 0 or x > nf for x in w):
                            continue
                        a_gw = row.get(int(np.ravel_multi_index(w, fshape)), 0.0)
                        # lump along the normal (fixed) axes: keep only the free offsets
                        key = tuple(o[a] if a in free else 0 for a in range(d))
                        coll[key] = coll.get(key, 0.0) + a_gw
                    for key, a in coll.items():
                        q = tuple(p[a_] + key[a_] for a_ in range(d))
                        if q in index:
                            M[k, index[q]] += a
                        else:
                            rhs[k] -= a * val[q]
                sol = np.linalg.solve(M, rhs)
                for p, s in zip(pts, sol):
                    val[p] = s
            ci = np.ravel_multi_index(cv, cshape)
            for loc, v in val.items():
                g = tuple(base[a] + loc[a] for a in range(d))
                if v != 0.0 and fmask[g]:
                    rows.append(np.ravel_multi_index(g, fshape)); cols.append(ci); vals.append(v)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(int(np.prod(fshape)), int(np.prod(cshape))))
    # a shared point is visited from several cells with identical values: keep one copy
    P = P.tocsr()
    P.sum_duplicates()
    counts = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=P.shape).tocsr()
    counts.sum_duplicates()
    P.data = P.data / counts.data
    return P
