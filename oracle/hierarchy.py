"""Multilevel operators of a uniform 3:1 spacetree.

* A_L from the Q1 discretisation of -div(eps grad u) = f (Sec. 2.1, Sec. 4.2);
* P_l from d-linear or BoxMG transfers (Sec. 2.5), R_l = P_l^T;
* Ritz-Galerkin coarse operators A_{l-1} = R A_l P (Sec. 2.2);
* Jacobi diagonals D_l = diag(A_l) (Sec. 2.2: Jacobi on every level);
* the smoothed auxiliary restriction R~ = omega R A M^{-1}, truncated to the
  support of P (Sec. 3.2, first damping choice).

Levels too large to assemble (a fine level beyond ``assemble_limit`` vertices)
are applied matrix-free with the same element-wise definition; for them the
next coarser operator is the Q1 rediscretisation with the coarse cell's
coefficient, which the tests pin equal to R A P whenever every coarse cell
lies inside one coefficient block.
"""
import numpy as np
import scipy.sparse as sp

from . import fem, transfer


class Op:
    """A linear map given either as a sparse matrix or as a pair of functions."""

    def __init__(self, mat=None, fn=None, fnT=None):
        self.mat, self.fn, self.fnT = mat, fn, fnT

    def __call__(self, x):
        return self.mat @ x if self.mat is not None else self.fn(x)

    def T(self, x):
        return self.mat.T @ x if self.mat is not None else self.fnT(x)

    def astype(self, dtype):
        if self.mat is not None:
            return Op(mat=self.mat.astype(dtype))
        return Op(fn=lambda x, f=self.fn: f(x).astype(dtype, copy=False),
                  fnT=None if self.fnT is None else (lambda x, f=self.fnT: f(x).astype(dtype, copy=False)))


def smoothed_operator_eps1(d):
    """The 7^d stencil of M^{-1} A P for eps = 1, d-linear P, Jacobi M = diag(A).

    This is the operator the paper prints for d = 2 (Sec. 3.2): the column of
    M^{-1} A P belonging to one coarse vertex, shown on the fine vertices
    within distance 3 of it.  Computed on a two-level reference grid (levels
    2 and 3) around an interior coarse vertex.  Returns an array of shape
    (7,)*d indexed by offset + 3 (axis order z, y, x).
    """
    lf = 3
    A = fem.assemble(np.ones((3 ** lf,) * d))
    P = transfer.dlinear_prolongation(d, lf)
    D = A.diagonal()
    cshape = (3 ** (lf - 1) + 1,) * d
    fshape = (3 ** lf + 1,) * d
    c = (4,) * d
    e = np.zeros(int(np.prod(cshape)))
    e[np.ravel_multi_index(c, cshape)] = 1.0
    col = (A @ (P @ e))
    with np.errstate(divide="ignore", invalid="ignore"):
        col = np.where(D != 0, col / np.where(D != 0, D, 1.0), 0.0)
    col = col.reshape(fshape)
    sl = tuple(slice(3 * c[a] - 3, 3 * c[a] + 4) for a in range(d))
    return col[sl].copy()


def _offsets(d, radius):
    return np.stack(np.meshgrid(*([np.arange(-radius, radius + 1)] * d), indexing="ij"), -1).reshape(-1, d)


def stencil_restriction(weights, d, level_f):
    """Sparse map level_f -> level_f-1: coarse v gathers sum_o w[o] x[3v + o], |o| <= 2."""
    nc = 3 ** (level_f - 1)
    cshape = (nc + 1,) * d
    fshape = (3 * nc + 1,) * d
    cm = fem.interior_mask(d, level_f - 1)
    fm = fem.interior_mask(d, level_f)
    cidx = np.argwhere(cm)
    rows, cols, vals = [], [], []
    for o in _offsets(d, 2):
        w = weights[tuple(o + 2)]
        if w == 0.0:
            continue
        f = 3 * cidx + o
        ok = np.all((f >= 0) & (f <= 3 * nc), axis=1)
        f, cv = f[ok], cidx[ok]
        ok2 = fm[tuple(f.T)]
        f, cv = f[ok2], cv[ok2]
        rows.append(np.ravel_multi_index(tuple(cv.T), cshape))
        cols.append(np.ravel_multi_index(tuple(f.T), fshape))
        vals.append(np.full(len(f), w))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(int(np.prod(cshape)), int(np.prod(fshape))))


def stencil_restriction_fn(weights, d, level_f):
    """Matrix-free form of :func:`stencil_restriction` (strided gathers)."""
    nc = 3 ** (level_f - 1)
    nf = 3 * nc
    cm = fem.interior_mask(d, level_f - 1)

    def fn(x):
        x = x.reshape((nf + 1,) * d)
        xp = np.pad(x, 2)
        out = np.zeros((nc + 1,) * d, dtype=x.dtype)
        for o in _offsets(d, 2):
            w = weights[tuple(o + 2)]
            if w == 0.0:
                continue
            sl = tuple(slice(2 + o[a], 2 + o[a] + nf + 1, 3) for a in range(d))
            out += x.dtype.type(w) * xp[sl]
        out[~cm] = 0.0
        return out.ravel()
    return fn


def dlinear_fns(d, level_f):
    """Matrix-free d-linear P and P^T: the 1D linear map applied along each axis."""
    nc = 3 ** (level_f - 1)
    P1 = transfer.linear_1d(nc)
    P1T = P1.T.tocsr()
    cm = fem.interior_mask(d, level_f - 1)
    fm = fem.interior_mask(d, level_f)

    def along(x, M):
        for a in range(d):
            x = np.moveaxis(x, a, 0)
            sh = x.shape
            y = M.astype(x.dtype) @ x.reshape(sh[0], -1)
            x = np.moveaxis(y.reshape((M.shape[0],) + sh[1:]), 0, a)
        return x

    def P(x):
        x = np.where(cm, x.reshape(cm.shape), 0.0).astype(x.dtype)
        y = along(x, P1)
        y[~fm] = 0.0
        return y.ravel()

    def PT(x):
        x = np.where(fm, x.reshape(fm.shape), 0.0).astype(x.dtype)
        y = along(x, P1T)
        y[~cm] = 0.0
        return y.ravel()
    return P, PT


class Level:
    pass


class Hierarchy:
    """All operators of an adAFAC solve on a uniform grid, levels lmin..L."""

    def __init__(self, d, L, lmin=1, eps_blocks=None, transfer_kind="dlinear",
                 rtilde="const", omega=0.6, assemble_limit=2_000_000, boxmg_inside_blocks=True):
        """``boxmg_inside_blocks=False`` takes the d-linear transfer for BoxMG wherever every
        coarse cell lies inside one coefficient block, where the two coincide (pinned by
        the tests); it only saves the slow per-cell solves on large levels."""
        assert d in (2, 3) and 1 <= lmin <= L
        assert transfer_kind in ("dlinear", "boxmg") and rtilde in ("const", "operator")
        if eps_blocks is None:
            eps_blocks = np.ones((1,) * d)
        eps_blocks = np.asarray(eps_blocks, dtype=np.float64)
        assert eps_blocks.ndim == d and np.all(eps_blocks > 0) and np.all(np.isfinite(eps_blocks))
        nb = eps_blocks.shape[0]
        k = int(round(np.log(nb) / np.log(3)))
        assert 3 ** k == nb and k <= L
        self.d, self.L, self.lmin, self.k = d, L, lmin, k
        self.eps_blocks, self.transfer_kind, self.rtilde_kind = eps_blocks, transfer_kind, rtilde
        self.omega = omega
        self.lev = {}
        T = smoothed_operator_eps1(d)
        self.smoothed_eps1 = T
        w_const = omega * T[(slice(1, 6),) * d]

        nvert = (3 ** L + 1) ** d
        big = nvert > assemble_limit
        for l in range(L, lmin - 1, -1):
            lv = Level()
            lv.level, lv.n, lv.h = l, 3 ** l, 3.0 ** -l
            lv.shape = (3 ** l + 1,) * d
            lv.mask = fem.interior_mask(d, l)
            self.lev[l] = lv
        # finest operator
        fine = self.lev[L]
        eps_L = fem.cell_eps_from_blocks(eps_blocks, L)
        self.eps_L = eps_L
        if big:
            fine.A = Op(fn=lambda x, e=eps_L: fem.apply_matrix_free(
                x.reshape((e.shape[0] + 1,) * e.ndim), e).ravel())
            fine.D = self._fem_diagonal(eps_L)
        else:
            A = fem.assemble(eps_L)
            fine.A = Op(mat=A)
            fine.D = A.diagonal().copy()
        # coarser operators, transfers and auxiliary restrictions
        for l in range(L, lmin, -1):
            lv, cv = self.lev[l], self.lev[l - 1]
            if lv.A.mat is None:
                assert transfer_kind == "dlinear" or l - 1 >= k, \
                    "matrix-free level needs d-linear transfers"
                assert l - 1 >= k, "matrix-free level needs block-constant eps on coarse cells"
                Pf, PTf = dlinear_fns(d, l)
                lv.P = Op(fn=Pf, fnT=PTf)
                Ac = fem.assemble(fem.cell_eps_from_blocks(eps_blocks, l - 1))
            else:
                if transfer_kind == "dlinear" or (not boxmg_inside_blocks and l - 1 >= k):
                    P = transfer.dlinear_prolongation(d, l)
                else:
                    P = transfer.boxmg_prolongation(lv.A.mat, d, l)
                lv.P = Op(mat=P)
                Ac = (P.T @ lv.A.mat @ P).tocsr()
                Ac.sum_duplicates()
            cv.A = Op(mat=Ac)
            cv.D = Ac.diagonal().copy()
            lv.I = Op(mat=transfer.injection(d, l)) if lv.A.mat is not None else \
                Op(fn=self._inject_fn(l))
            if rtilde == "const":
                if lv.A.mat is None:
                    lv.Rt = Op(fn=stencil_restriction_fn(w_const, d, l))
                else:
                    lv.Rt = Op(mat=stencil_restriction(w_const, d, l))
            else:
                assert lv.A.mat is not None, "operator R~ needs an assembled level"
                lv.Rt = Op(mat=self._operator_rtilde(lv, l))
        for l in range(lmin, L + 1):
            lv = self.lev[l]
            lv.Dinv = np.where(lv.mask.ravel(), 1.0 / np.where(lv.D != 0, lv.D, 1.0), 0.0)

    def _fem_diagonal(self, eps_cells):
        d = self.d
        n = eps_cells.shape[0]
        h = 1.0 / n
        K = fem.ref_stiffness(d)
        out = np.zeros((n + 1,) * d)
        for i in range(2 ** d):
            oi = fem.corner_offset(i, d)
            out[tuple(slice(oi[a], oi[a] + n) for a in range(d))] += eps_cells * h ** (d - 2) * K[i, i]
        out[~fem.interior_mask(d, int(round(np.log(n) / np.log(3))))] = 0.0
        return out.ravel()

    def _inject_fn(self, l):
        d = self.d
        nc = 3 ** (l - 1)
        cm = fem.interior_mask(d, l - 1)

        def fn(x):
            x = x.reshape((3 * nc + 1,) * d)
            y = x[(slice(0, 3 * nc + 1, 3),) * d].copy()
            y[~cm] = 0.0
            return y.ravel()
        return fn

    def _operator_rtilde(self, lv, l):
        """R~ = omega * trunc(P^T A D^{-1}): entries more than 2 fine widths away dropped."""
        d = self.d
        P = lv.P.mat
        Dinv = sp.diags(np.where(lv.mask.ravel(), 1.0 / np.where(lv.D != 0, lv.D, 1.0), 0.0))
        M = (P.T @ lv.A.mat @ Dinv).tocoo()
        cshape = self.lev[l - 1].shape
        cr = np.array(np.unravel_index(M.row, cshape))
        fc = np.array(np.unravel_index(M.col, lv.shape))
        keep = np.all(np.abs(fc - 3 * cr) <= 2, axis=0)
        return sp.csr_matrix((self.omega * M.data[keep], (M.row[keep], M.col[keep])), shape=M.shape)

    def rhs(self, f, g=None):
        """b_L from the vertex samples f of the right-hand side (lumped mass); with Dirichlet
        data g (on the finest vertex lattice, boundary entries used) the load of its lift is
        added, and the iterate is then u_0 = u - G (zero on the boundary)."""
        b = fem.lumped_rhs(f, self.L).ravel()
        if g is not None:
            b = b + fem.dirichlet_lift(g, self.eps_L).ravel()
        return b

    def astype(self, dtype):
        """A copy whose operators compute in ``dtype`` (FP32 inner cycles)."""
        import copy
        H = copy.copy(self)
        H.lev = {}
        for l, lv in self.lev.items():
            nv = Level()
            nv.__dict__.update(lv.__dict__)
            for name in ("A", "P", "I", "Rt"):
                if hasattr(lv, name):
                    setattr(nv, name, getattr(lv, name).astype(dtype))
            nv.D = lv.D.astype(dtype)
            nv.Dinv = lv.Dinv.astype(dtype)
            H.lev[l] = nv
        return H
