"""Q1 (d-linear) finite elements on one level of a uniform 3:1 spacetree.

Follows Sec. 2.1 of the paper (spacetree levels, d-linear shape functions,
boundary vertices carry no test function) and the element-wise mat-vec of
Sec. 4.2 (each cell contributes its element matrix to its 2^d vertices).

Level ``l`` of the unit square/cube has ``n = 3**l`` cells per axis and mesh
width ``h = 3**-l``.  Arrays over vertices have shape ``(n+1,)*d`` and arrays
over cells ``(n,)*d``, both C order with x on the last axis.  Local corner
``i`` of a cell sits at offset bit ``k`` of ``i`` along coordinate ``k``
(k = 0 is x).
"""
import itertools

import numpy as np
import scipy.sparse as sp


def ref_stiffness(d):
    """Element stiffness of the d-linear element on the unit cell.

    K[i, j] = integral over [0,1]^d of grad(phi_i) . grad(phi_j), where corner ``i`` has shape
    function prod_k (x_k if bit k of i else 1 - x_k).  The integrand is a sum over the
    derivative axis k of products of one-variable factors, so the integral is
    sum_k d_k(i) d_k(j) prod_{m != k} int_0^1 f_i^m f_j^m dx with d_k = +-1 the derivative of
    the k-th factor and int x x = int (1-x)(1-x) = 1/3, int x (1-x) = 1/6.  It is evaluated in
    exact rational arithmetic and rounded once per entry, so the entries are the correctly
    rounded 2/3, -1/6, -1/3 (2D) and 1/3, 0, -1/12 (3D): the assembled interior rows then sum
    to exactly zero, as the exact operator's do (a quadrature in floating point leaves a row
    sum of a few ulp, an artificial zero-order term that the smoothest modes feel).
    """
    from fractions import Fraction
    nc = 2 ** d
    K = np.zeros((nc, nc))
    for i in range(nc):
        for j in range(nc):
            s = Fraction(0)
            for k in range(d):
                bi, bj = (i >> k) & 1, (j >> k) & 1
                term = Fraction(1 if bi == bj else -1)
                for m in range(d):
                    if m != k:
                        term *= Fraction(1, 3) if ((i >> m) & 1) == ((j >> m) & 1) else Fraction(1, 6)
                s += term
            K[i, j] = float(s)
    return K


def corner_offset(i, d):
    """Offset of local corner ``i`` as a numpy index tuple (axis order z, y, x)."""
    return tuple((i >> k) & 1 for k in reversed(range(d)))


def vertex_shape(d, level):
    return (3 ** level + 1,) * d


def interior_mask(d, level):
    """True at vertices carrying a degree of freedom (not on the boundary)."""
    n = 3 ** level
    m = np.zeros(vertex_shape(d, level), dtype=bool)
    m[(slice(1, n),) * d] = True
    return m


def cell_eps_from_blocks(eps_blocks, level):
    """Coefficient of every level-``level`` cell from a block field.

    ``eps_blocks`` has shape ``(3**k,)*d``: it is constant on the cells of
    spacetree level k.  A level-l cell with l >= k lies inside exactly one
    block; for l < k the field is not constant on a cell and no FEM element
    exists (the coarse operator is then the Galerkin one, Sec. 2.2).
    """
    eps_blocks = np.asarray(eps_blocks, dtype=np.float64)
    d = eps_blocks.ndim
    nb = eps_blocks.shape[0]
    k = int(round(np.log(nb) / np.log(3)))
    assert 3 ** k == nb, "blocks per axis must be a power of three"
    assert level >= k, "cells of this level straddle several coefficient blocks"
    rep = 3 ** (level - k)
    out = eps_blocks
    for a in range(d):
        out = np.repeat(out, rep, axis=a)
    return out


def assemble(eps_cells):
    """Sparse stiffness matrix of one uniform level, boundary rows/columns removed.

    Element matrix of cell c: eps_c * h^(d-2) * K_ref (gradients scale with 1/h,
    the volume with h^d).  Entries are summed over all cells sharing the two
    vertices (element-wise assembly, Sec. 4.2).  Boundary vertices carry no
    test function (Sec. 2.1), so their rows and columns are dropped; their
    value is zero for the homogeneous Dirichlet problems treated here.
    """
    eps_cells = np.asarray(eps_cells, dtype=np.float64)
    d = eps_cells.ndim
    n = eps_cells.shape[0]
    h = 1.0 / n
    K = ref_stiffness(d)
    vshape = (n + 1,) * d
    cell_idx = np.indices((n,) * d)
    rows, cols, vals = [], [], []
    scale = eps_cells * h ** (d - 2)
    for i in range(2 ** d):
        oi = corner_offset(i, d)
        vi = np.ravel_multi_index(tuple(cell_idx[a] + oi[a] for a in range(d)), vshape)
        for j in range(2 ** d):
            if K[i, j] == 0.0:
                continue
            oj = corner_offset(j, d)
            vj = np.ravel_multi_index(tuple(cell_idx[a] + oj[a] for a in range(d)), vshape)
            rows.append(vi.ravel())
            cols.append(vj.ravel())
            vals.append((scale * K[i, j]).ravel())
    N = int(np.prod(vshape))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    z = sp.diags(interior_mask(d, int(round(np.log(n) / np.log(3)))).ravel().astype(np.float64))
    return (z @ A @ z).tocsr()


def apply_matrix_free(u, eps_cells):
    """A u for the operator of :func:`assemble`, without storing the matrix.

    Same element-wise accumulation: for each cell and each pair of its
    corners, eps_c h^(d-2) K_ref[i, j] u_j is added to vertex i.  The result is
    zero on the boundary.  Used where the level is too large to assemble.  The
    arithmetic is that of u's dtype (FP32 inner cycles round every product and
    sum in FP32).
    """
    eps_cells = np.asarray(eps_cells, dtype=np.float64)
    d = eps_cells.ndim
    n = eps_cells.shape[0]
    h = 1.0 / n
    K = ref_stiffness(d)
    u = np.asarray(u)
    out = np.zeros_like(u)
    scale = (eps_cells * h ** (d - 2)).astype(out.dtype)
    for j in range(2 ** d):
        oj = corner_offset(j, d)
        uj = u[tuple(slice(oj[a], oj[a] + n) for a in range(d))]
        su = scale * uj
        for i in range(2 ** d):
            if K[i, j] == 0.0:
                continue
            oi = corner_offset(i, d)
            out[tuple(slice(oi[a], oi[a] + n) for a in range(d))] += out.dtype.type(K[i, j]) * su
    out[~interior_mask(d, int(round(np.log(n) / np.log(3))))] = 0.0
    return out


def lumped_rhs(f, level):
    """Right-hand side b_v = m_v f_v with lumped mass m_v = sum over cells of |cell|/2^d.

    The paper gives f but not its quadrature; this is the lumped-mass reading
    (one quarter / one eighth of every adjacent cell's volume per vertex).  On
    a uniform level every interior vertex gets h^d f_v.  Boundary entries are
    zero.  Parity unpinned beyond that closed form.
    """
    f = np.asarray(f, dtype=np.float64)
    d = f.ndim
    n = 3 ** level
    assert f.shape == (n + 1,) * d
    h = 1.0 / n
    m = np.zeros_like(f)
    for i in range(2 ** d):
        oi = corner_offset(i, d)
        m[tuple(slice(oi[a], oi[a] + n) for a in range(d))] += h ** d / 2 ** d
    b = m * f
    b[~interior_mask(d, level)] = 0.0
    return b


def dirichlet_lift(g, eps_cells):
    """Load of inhomogeneous Dirichlet data (the u = 1 on x_2 = 0 set-ups of Sec. 5).

    With u = u_0 + G, G the data on the boundary vertices and zero inside, the interior
    equations of A u = b become A u_0 = b - A G: every element couples its boundary corners to
    its interior ones.  Returns -A G at the interior vertices (zero on the boundary), from the
    element-wise operator of :func:`apply_matrix_free`."""
    g = np.asarray(g, dtype=np.float64)
    d = g.ndim
    n = g.shape[0] - 1
    level = int(round(np.log(n) / np.log(3)))
    G = np.where(interior_mask(d, level), 0.0, g)
    return -apply_matrix_free(G, eps_cells)


def with_boundary(u0, g):
    """The full vertex lattice of u = u_0 + G: u_0 inside, the Dirichlet data on the boundary."""
    g = np.asarray(g, dtype=np.float64)
    d = g.ndim
    level = int(round(np.log(g.shape[0] - 1) / np.log(3)))
    m = interior_mask(d, level)
    return np.where(m, np.asarray(u0).reshape(g.shape), g)
