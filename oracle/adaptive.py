"""adAFAC-Jac on an adaptive 3:1 spacetree: ragged levels with hanging vertices.

TEST INFRASTRUCTURE (part of the oracle package; see its header).

Definitions follow Sec. 2.1 (spacetree, shape functions, hanging vertices), Sec. 2.3 (the
hierarchical generating system over all levels), Sec. 2.4 (every level holds a nodal value;
coinciding coarse vertices copy the finer one) and eq. (adaFACx) / Algorithm 1 (Sec. 3.1):

* Level l has the cells of the spacetree on that level, E_l.  A refined cell has its 3^d
  children on level l+1; unrefined cells are leaves.
* A level-l vertex is a degree of freedom of level l if it is interior and all 2^d level-l
  cells around it exist.  Other interior vertices of existing cells are hanging: they carry
  the d-linear interpolation of the next coarser level and no test function.
* The composite (adaptive) grid holds every level-l dof that is not a dof of level l+1: the
  finest level on which it is a dof.  Its FE space is continuous Q1 on the leaf cells.
* The composite system is A_h = sum_l C_l^T A^leaf_l C_l and b_h = sum_l C_l^T b^leaf_l.  C_l
  maps composite values to the level-l lattice (dofs: the value at that position; hanging:
  interpolation).  A^leaf_l sums the Q1 elements of the level-l leaf cells, and b^leaf_l is
  the lumped load of those cells, m_v = sum over leaf cells around v of |cell| / 2^d.

One cycle, in correction form over the generating system:

1. Residual of each level's leaf cells.
2. Bottom-up accumulation b_l = r^leaf_l + R b_{l+1}, i.e. the level-l hats tested against
   the composite residual.
3. Jacobi corrections c_l = omega D_l^-1 b_l on every level.
4. The auxiliary correction of the next coarser level, c~_l = omega~ D_l^-1 R~ b_{l+1}.
5. Top-down prolongation of the sums (c_l - c~_l), added to every composite dof on its finest
   level.

The per-level arrays ("FAS storage") hold the composite value at every dof position and the
interpolated value at hanging vertices.

Inhomogeneous Dirichlet data (the set-ups of Sec. 5, u = 1 on x_2 = 0): the boundary vertices of
existing cells carry the data g on every level, and the composite space is the continuous Q1
functions on the leaf cells with those boundary values (hanging vertices still interpolate the
next coarser level, boundary values included).  The residual of the interior dofs then contains
the coupling to the boundary values; corrections stay zero on the boundary.

Pinned by: the uniform tree reduces to cycle.cycle_correction, the cycle equals the dense
generating-system form of eq. (adaFACx) built here independently from hat functions, and
the fixed point is the direct solve of the composite system.  Border semantics beyond these
definitions: parity unpinned by the paper.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from . import fem, hierarchy


def omega_rtilde(d, omega):
    """The 5^d weights of R~: omega times the eps = 1 stencil of M^-1 A P truncated to |o| <= 2."""
    return omega * hierarchy.smoothed_operator_eps1(d)[(slice(1, 6),) * d]


class AdaptiveTree:
    """Ragged levels lmin..L of a 3:1 spacetree.

    ``refine[l]`` (l_uniform <= l < L): boolean array over the (3^l)^d cells of level l, the
    refinement flags; only flags of existing cells matter.  Levels below l_uniform are fully
    refined.  ``eps_blocks`` as in hierarchy.Hierarchy (blocks on a level k <= l_uniform).

    ``transfer`` "boxmg": operator-dependent transfers (Sec. 2.5) into the levels l <= k, which
    are uniform, so the level hats there are phi^l = sum_w P_wv phi^{l+1}_w with BoxMG's P of
    the uniform hierarchy of levels lmin..k.  Above level k every cell lies inside one
    coefficient block, where BoxMG's P is the d-linear one (pinned in the uniform tests), so
    those levels keep d-linear transfers (and hanging vertices always interpolate d-linearly).

    ``g``: Dirichlet data on the finest vertex lattice (only its boundary entries are used);
    None: u = 0 on the boundary.
    """

    def __init__(self, d, L, lmin, l_uniform, refine, eps_blocks=None, omega=0.6, transfer="dlinear", g=None):
        assert 1 <= lmin <= l_uniform <= L
        assert transfer in ("dlinear", "boxmg")
        self.d, self.L, self.lmin, self.lu = d, L, lmin, l_uniform
        self.omega = omega
        self.transfer = transfer
        eps_blocks = np.ones((1,) * d) if eps_blocks is None else np.asarray(eps_blocks, dtype=np.float64)
        self.eps_blocks = eps_blocks
        k = int(round(np.log(eps_blocks.shape[0]) / np.log(3)))
        assert k <= l_uniform, "coefficient blocks must be no finer than the uniform levels"
        self.k = k
        self.E, self.Rf, self.leaf = {}, {}, {}
        E = np.ones((1,) * d, dtype=bool)
        for l in range(0, L + 1):
            if l >= lmin:
                self.E[l] = E
            if l < L:
                R = E.copy() if l < l_uniform else (E & np.asarray(refine[l], dtype=bool))
            else:
                R = np.zeros_like(E)
            if l >= lmin:
                self.Rf[l] = R
                self.leaf[l] = E & ~R
            nxt = R
            for a in range(d):
                nxt = np.repeat(nxt, 3, axis=a)
            E = nxt
        self._classify()
        self._operators()
        self.g = None
        if g is not None:
            g = np.asarray(g, dtype=np.float64).reshape(self.shape(L))
            self.g = {l: g[tuple(slice(None, None, 3 ** (L - l)) for _ in range(d))].copy()
                      for l in range(lmin, L + 1)}

    # --- vertex classes ---------------------------------------------------------
    def _classify(self):
        d = self.d
        self.cnt, self.dof, self.hang, self.comp, self.exists_v, self.bnd = {}, {}, {}, {}, {}, {}
        for l in range(self.lmin, self.L + 1):
            E = self.E[l].astype(np.int32)
            n = 3 ** l
            cnt = np.zeros((n + 1,) * d, dtype=np.int32)
            for corner in itertools.product((0, 1), repeat=d):
                cnt[tuple(slice(c, c + n) for c in corner)] += E
            inter = fem.interior_mask(d, l)
            self.cnt[l] = cnt
            self.exists_v[l] = cnt > 0
            self.dof[l] = inter & (cnt == 2 ** d)
            self.hang[l] = inter & (cnt > 0) & (cnt < 2 ** d)
            self.bnd[l] = ~inter & (cnt > 0)
        for l in range(self.lmin, self.L + 1):
            if l == self.L:
                self.comp[l] = self.dof[l].copy()
            else:
                finer = self.dof[l + 1][tuple(slice(None, None, 3) for _ in range(d))]
                self.comp[l] = self.dof[l] & ~finer

    # --- operators ---------------------------------------------------------------
    def _operators(self):
        d, L = self.d, self.L
        self.h = {l: 3.0 ** -l for l in range(self.lmin, L + 1)}
        self.eps_cells, self.leaf_eps, self.bmass, self.D = {}, {}, {}, {}
        kref = fem.ref_stiffness(d)[0, 0]
        gal = None
        if self.k > self.lmin:
            gal = hierarchy.Hierarchy(d, self.k, self.lmin, self.eps_blocks, self.transfer)
        self.gal = gal
        for l in range(self.lmin, L + 1):
            n = 3 ** l
            if l >= self.k:
                ec = fem.cell_eps_from_blocks(self.eps_blocks, l)
                self.eps_cells[l] = ec
                self.leaf_eps[l] = np.where(self.leaf[l], ec, 0.0)
                # Q1 diagonal: every dof has its 2^d cells
                s = np.zeros((n + 1,) * d)
                for corner in itertools.product((0, 1), repeat=d):
                    s[tuple(slice(c, c + n) for c in corner)] += ec
                self.D[l] = np.where(self.dof[l], kref * self.h[l] ** (d - 2) * s, 0.0)
            else:
                # coarse levels below the coefficient blocks are uniform: Ritz-Galerkin (Sec. 2.2)
                self.leaf_eps[l] = np.zeros((n,) * d)
                self.D[l] = np.where(self.dof[l], gal.lev[l].D.reshape((n + 1,) * d), 0.0)
            m = np.zeros((n + 1,) * d)
            lf = self.leaf[l].astype(np.float64) * self.h[l] ** d / 2 ** d
            for corner in itertools.product((0, 1), repeat=d):
                m[tuple(slice(c, c + n) for c in corner)] += lf
            m[~fem.interior_mask(d, l)] = 0.0
            self.bmass[l] = m
        self.P, self.PT, self.Rt = {}, {}, {}
        # R~ = omega trunc(M^-1 A P) from the eps = 1 stencil (Sec. 3.2), as on uniform grids
        rt = omega_rtilde(d, self.omega)
        for l in range(self.lmin + 1, L + 1):
            if gal is not None and self.transfer == "boxmg" and l <= self.k:
                Pm = gal.lev[l].P.mat
                self.P[l] = lambda x, M=Pm: M @ x
                self.PT[l] = lambda x, M=Pm: M.T @ x
            else:
                self.P[l], self.PT[l] = hierarchy.dlinear_fns(d, l)
            self.Rt[l] = hierarchy.stencil_restriction_fn(rt, d, l)

    def shape(self, l):
        return (3 ** l + 1,) * self.d

    def leaf_apply(self, l, u):
        """sum over the level-l leaf cells of their Q1 element times u (zero on the boundary)."""
        return fem.apply_matrix_free(u.reshape(self.shape(l)), self.leaf_eps[l])

    def load(self, f):
        """b^leaf_l = m * f with f sampled at the level-l vertices from the finest lattice."""
        f = np.asarray(f, dtype=np.float64).reshape(self.shape(self.L))
        out = {}
        for l in range(self.lmin, self.L + 1):
            s = 3 ** (self.L - l)
            out[l] = self.bmass[l] * f[tuple(slice(None, None, s) for _ in range(self.d))]
        return out

    # --- composite vectors <-> per-level storage ------------------------------------
    def composite_index(self):
        """(level, flat index) of every composite dof, coarse levels first."""
        out = []
        for l in range(self.lmin, self.L + 1):
            for i in np.flatnonzero(self.comp[l].ravel()):
                out.append((l, int(i)))
        return out

    def spread(self, U, homogeneous=False):
        """Complete per-level storage from the composite values: coarse copies of finer dofs
        (injection), the Dirichlet data on the boundary vertices of existing cells (zero when
        homogeneous: corrections, or no data), then hanging vertices interpolated top-down."""
        d, L = self.d, self.L
        U = {l: U[l].copy() for l in U}
        for l in range(L, self.lmin, -1):
            fine_at_coarse = U[l][tuple(slice(None, None, 3) for _ in range(d))]
            copy = self.dof[l - 1] & ~self.comp[l - 1]
            U[l - 1][copy] = fine_at_coarse[copy]
        keep = {}
        for l in range(self.lmin, L + 1):
            keep[l] = self.dof[l] | self.hang[l]
            if self.g is not None and not homogeneous:
                U[l][self.bnd[l]] = self.g[l][self.bnd[l]].astype(U[l].dtype)
                keep[l] = keep[l] | self.bnd[l]
            else:
                U[l][self.bnd[l]] = 0.0
        for l in range(self.lmin + 1, L + 1):
            if self.g is not None and not homogeneous:
                # hanging vertices next to the boundary interpolate its values too
                Pu = _upsample(U[l - 1])
            else:
                Pu = self.P[l](U[l - 1].ravel()).reshape(self.shape(l))
            U[l][self.hang[l]] = Pu[self.hang[l]]
        for l in range(self.lmin, L + 1):
            U[l][~keep[l]] = 0.0
        return U


def norms(T, rh):
    """sqrt(sum over composite dofs of h^d r^2) with h of the dof's level, and max |r|."""
    s, m = 0.0, 0.0
    for l, r in rh.items():
        rr = r[T.comp[l]]
        s += T.h[l] ** T.d * float(np.sum(rr * rr))
        if rr.size:
            m = max(m, float(np.max(np.abs(rr))))
    return np.sqrt(s), m


def cycle(T, U, bleaf, omega=0.6, omega_t=0.6, damping="jac", trace=None, dtype=np.float64, homogeneous=False):
    """One adAFAC cycle on the adaptive tree (correction form over the generating system).

    U: per-level storage of the iterate (see AdaptiveTree.spread).  Returns the new storage and
    the norms of the composite residual of the input iterate.  ``dtype`` float32 stores every
    intermediate array in FP32 (the inner cycles of defect correction); the operators are
    applied as FP64 factors and their results rounded, so this gives the size of FP32
    rounding, not any particular rounding order.  ``homogeneous``: zero boundary values (a
    correction equation) whatever the tree's Dirichlet data.
    """
    assert damping in ("jac", "pi", "none")
    d, L, lmin = T.d, T.L, T.lmin
    U = T.spread({l: U[l].astype(dtype) for l in U}, homogeneous)
    bleaf = {l: bleaf[l].astype(dtype) for l in bleaf}
    # leaf residuals, per level, at every vertex of a leaf cell
    rl = {l: bleaf[l] - T.leaf_apply(l, U[l]).reshape(T.shape(l)) for l in range(lmin, L + 1)}
    # the level-l hats tested against the composite residual: b_l = r^leaf_l + R b_{l+1}
    bbar = {L: rl[L]}
    for l in range(L - 1, lmin - 1, -1):
        bbar[l] = rl[l] + T.PT[l + 1](bbar[l + 1].ravel()).reshape(T.shape(l))
    b = {l: np.where(T.dof[l], bbar[l], 0.0) for l in bbar}
    # composite residual: own leaf part plus what hanging copies of the vertex collected
    hh = {L: np.where(T.hang[L], rl[L], 0.0)}
    rh = {L: np.where(T.comp[L], rl[L], 0.0)}
    for l in range(L - 1, lmin - 1, -1):
        acc = rl[l] + T.PT[l + 1](hh[l + 1].ravel()).reshape(T.shape(l))
        hh[l] = np.where(T.hang[l], acc, 0.0)
        rh[l] = np.where(T.comp[l], acc, 0.0)
    nr = norms(T, rh)
    Dinv = {l: np.where(T.dof[l], 1.0 / np.where(T.dof[l], T.D[l], 1.0), 0.0).astype(dtype) for l in T.D}
    c = {l: omega * Dinv[l] * b[l] for l in b}
    ct = {l: np.zeros(T.shape(l), dtype=dtype) for l in b}
    if damping == "jac":
        for l in range(lmin, L):
            ct[l] = omega_t * Dinv[l] * T.Rt[l + 1](b[l + 1].ravel()).reshape(T.shape(l))
    elif damping == "pi":
        # adAFAC-PI (Sec. 3.2): c~_l = P I c_l, the level's correction injected to level l-1 (its
        # values at the coinciding level-(l-1) dofs) and prolongated back, none on l_min
        for l in range(lmin + 1, L + 1):
            Ic = np.where(T.dof[l - 1], c[l][tuple(slice(None, None, 3) for _ in range(d))], 0.0)
            ct[l] = T.P[l](Ic.ravel()).reshape(T.shape(l)).astype(dtype)
    S = {lmin: c[lmin] - ct[lmin]}
    for l in range(lmin + 1, L + 1):
        S[l] = c[l] - ct[l] + T.P[l](S[l - 1].ravel()).reshape(T.shape(l))
    V = {l: np.where(T.comp[l], U[l] + S[l], U[l]) for l in U}
    if trace is not None:
        trace.update(rleaf=rl, b=b, rh=rh, c=c, ct=ct, S=S)
    return T.spread(V, homogeneous), nr


def solve(T, f, max_cycles, tol=None, **kw):
    """Cycles from u = 0; stops after the first cycle whose input iterate meets tol."""
    bleaf = T.load(f)
    U = {l: np.zeros(T.shape(l)) for l in range(T.lmin, T.L + 1)}
    hist = []
    for _ in range(max_cycles):
        U, nr = cycle(T, U, bleaf, **kw)
        hist.append(nr)
        if tol is not None and hist[0][0] > 0 and hist[-1][0] / hist[0][0] <= tol:
            break
    return U, hist


def composite_residual(T, U, bleaf):
    """The composite residual of the iterate U at every composite dof (on the dof's level, zero
    elsewhere) and its norms: the first steps of :func:`cycle`, in FP64."""
    U = T.spread(U)
    rl = {l: bleaf[l] - T.leaf_apply(l, U[l]).reshape(T.shape(l)) for l in range(T.lmin, T.L + 1)}
    hh = np.where(T.hang[T.L], rl[T.L], 0.0)
    rh = {T.L: np.where(T.comp[T.L], rl[T.L], 0.0)}
    for l in range(T.L - 1, T.lmin - 1, -1):
        acc = rl[l] + T.PT[l + 1](hh.ravel()).reshape(T.shape(l))
        hh = np.where(T.hang[l], acc, 0.0)
        rh[l] = np.where(T.comp[l], acc, 0.0)
    return rh, norms(T, rh)


def defect_correction(T, f, k_inner, tol, max_outer, inner_dtype=np.float32, iterates=None, U0=None, **kw):
    """FP64 defect correction around k adAFAC cycles in ``inner_dtype`` on the tree.

    Outer step: the composite residual r of u in FP64 and its norms; stop if
    ||r||_h / ||r^0||_h <= tol; otherwise k cycles on the correction equation from e = 0, then
    u <- u + e at every dof in FP64.  The inner leaf loads are r at the composite dofs and zero
    elsewhere: the same functional as the leaf residuals of u (a composite-space function is
    the sum of its composite-dof values times the composite hats), but without the large
    per-level leaf parts that cancel at refinement boundaries and would be rounded to FP32
    before they cancel.  The cycle is linear, so k inner cycles equal k cycles on u in exact
    arithmetic.  Starts from U0 (per-level storage; default zero).  Returns (U, outer residual
    history); ``iterates`` (a list) receives every outer iterate's per-level storage.
    """
    U = {l: np.zeros(T.shape(l)) for l in range(T.lmin, T.L + 1)} if U0 is None else U0
    bleaf = T.load(f)
    hist = []
    for _ in range(max_outer + 1):
        U = T.spread(U)
        rh, nr = composite_residual(T, U, bleaf)
        hist.append(nr)
        if iterates is not None:
            iterates.append({l: U[l].copy() for l in U})
        if hist[0][0] == 0 or hist[-1][0] / hist[0][0] <= tol or len(hist) > max_outer:
            break
        E = {l: np.zeros(T.shape(l), dtype=inner_dtype) for l in U}
        for _ in range(k_inner):
            E, _ = cycle(T, E, rh, dtype=inner_dtype, homogeneous=True, **kw)
        U = {l: np.where(T.dof[l], U[l] + E[l].astype(np.float64), U[l]) for l in U}
    return T.spread(U), hist


def _upsample(u):
    """d-linear interpolation of a whole vertex lattice (boundary included) onto the lattice of
    the next finer level: fine index 3c + s takes (1 - s/3) u[c] + (s/3) u[c + 1] per axis."""
    for a in range(u.ndim):
        n = u.shape[a] - 1
        lo = np.take(u, np.arange(n), axis=a)
        hi = np.take(u, np.arange(1, n + 1), axis=a)
        parts = [lo, (2.0 * lo + hi) / 3.0, (lo + 2.0 * hi) / 3.0]
        st = np.stack(parts, axis=a + 1)
        shp = list(u.shape)
        shp[a] = 3 * n
        st = st.reshape(shp)
        last = np.take(u, [n], axis=a)
        u = np.concatenate([st, last], axis=a)
    return u


def finest_values(T, U):
    """The composite FE function at every vertex of the finest lattice (d-linear from the
    coarsest level where the point is not covered by finer cells; with Dirichlet data the
    boundary traces of coarse leaf cells are d-linear in their corner values too)."""
    d, L = T.d, T.L
    out = U[T.lmin].copy()
    for l in range(T.lmin + 1, L + 1):
        if T.g is None:
            up = T.P[l](out.ravel()).reshape(T.shape(l))
            have = T.dof[l] | T.hang[l]
        else:
            up = _upsample(out)
            have = T.dof[l] | T.hang[l] | T.bnd[l]
        out = np.where(have, U[l], up)
    return out


# --- dense generating-system form (independent restatement, for small trees) -----------

def hat(d, l, v, x):
    """Level-l d-linear hat of vertex v evaluated at points x (n, d) in the unit cube."""
    h = 3.0 ** -l
    w = np.ones(len(x))
    for a in range(d):
        w *= np.maximum(0.0, 1.0 - np.abs(x[:, a] - v[a] * h) / h)
    return w


def dense_system(T, f):
    """(A_h, b_h, positions, levels, Psi, C) of the composite system, built from unit vectors.

    positions: (n, d) coordinates of the composite dofs (x on the last axis); Psi[l]: composite
    values of the level-l hats of the level-l dofs (columns in flat-index order of dof[l]).
    Homogeneous Dirichlet data only.
    """
    assert T.g is None
    d, L = T.d, T.L
    idx = T.composite_index()
    n = len(idx)
    pos = np.zeros((n, d))
    lev = np.zeros(n, dtype=int)
    for j, (l, i) in enumerate(idx):
        v = np.array(np.unravel_index(i, T.shape(l)))[::-1]     # (x, y[, z])
        pos[j] = v * 3.0 ** -l
        lev[j] = l
    # C_l from unit composite vectors
    C = {l: np.zeros((int(np.prod(T.shape(l))), n)) for l in range(T.lmin, L + 1)}
    for j, (l, i) in enumerate(idx):
        U = {m: np.zeros(T.shape(m)) for m in range(T.lmin, L + 1)}
        U[l].ravel()[i] = 1.0
        U = T.spread(U)
        for m in U:
            C[m][:, j] = U[m].ravel()
    bleaf = T.load(f)
    A = np.zeros((n, n))
    b = np.zeros(n)
    for l in range(T.lmin, L + 1):
        Al = fem.assemble(T.leaf_eps[l]).toarray() if l >= T.k else np.zeros((C[l].shape[0],) * 2)
        A += C[l].T @ Al @ C[l]
        b += C[l].T @ bleaf[l].ravel()
    Psi = {}
    for l in range(T.lmin, L + 1):
        dofs = np.flatnonzero(T.dof[l].ravel())
        cols = []
        for i in dofs:
            v = np.array(np.unravel_index(i, T.shape(l)))[::-1]
            cols.append(hat(d, l, v, pos))
        Psi[l] = np.array(cols).T if cols else np.zeros((n, 0))
    if T.transfer == "boxmg" and T.gal is not None:
        # operator-dependent hats below level k: phi^l_v = sum_w P_wv phi^{l+1}_w (Sec. 2.5)
        for l in range(T.k - 1, T.lmin - 1, -1):
            Pm = T.gal.lev[l + 1].P.mat.toarray()
            dof_f = np.flatnonzero(T.dof[l + 1].ravel())
            dof_c = np.flatnonzero(T.dof[l].ravel())
            Psi[l] = Psi[l + 1] @ Pm[np.ix_(dof_f, dof_c)]
    return A, b, pos, lev, Psi, C


def dense_cycle(T, A, b, lev, Psi, u, omega=0.6, omega_t=0.6, damping="jac"):
    """u + sum_l Psi_l (omega D_l^-1 Psi_l^T r - omega~ D_l^-1 R~ Psi_{l+1}^T r) with
    r = b - A u: eq. (adaFACx) over the generating system, in composite coefficients."""
    d, L = T.d, T.L
    r = b - A @ u
    du = np.zeros_like(u)
    Dl = {}
    for l in range(T.lmin, L + 1):
        # D_l = a(phi^l_v, phi^l_v) of the level hats in the composite space
        Dl[l] = np.einsum("iv,ij,jv->v", Psi[l], A, Psi[l])
        du += Psi[l] @ (omega * (Psi[l].T @ r) / Dl[l])
    if damping == "jac":
        rt = omega_rtilde(d, T.omega)
        for l in range(T.lmin, L):
            Rt = hierarchy.stencil_restriction(rt, d, l + 1)
            dof_c = np.flatnonzero(T.dof[l].ravel())
            dof_f = np.flatnonzero(T.dof[l + 1].ravel())
            bt = Rt[dof_c][:, dof_f] @ (Psi[l + 1].T @ r)
            du -= Psi[l] @ (omega_t * bt / Dl[l])
    elif damping == "pi":
        # minus the level-(l-1) function whose dof coefficients are c_l at the same positions
        for l in range(T.lmin + 1, L + 1):
            cl = np.zeros(int(np.prod(T.shape(l))))
            cl[np.flatnonzero(T.dof[l].ravel())] = omega * (Psi[l].T @ r) / Dl[l]
            at = cl.reshape(T.shape(l))[tuple(slice(None, None, 3) for _ in range(d))].ravel()
            du -= Psi[l - 1] @ at[np.flatnonzero(T.dof[l - 1].ravel())]
    s = float(np.sum((3.0 ** (-lev * d)) * r * r))
    return u + du, (np.sqrt(s), float(np.max(np.abs(r))) if r.size else 0.0)


def to_composite(T, U):
    return np.array([U[l].ravel()[i] for l, i in T.composite_index()])


def transfer(T_old, U_old, T_new):
    """Storage of tree T_new holding the composite function of (T_old, U_old): every dof takes
    its value at the dof's position (kept vertices keep theirs; new ones get the d-linear
    interpolation of the finest old cell around them)."""
    assert T_old.d == T_new.d and T_old.L == T_new.L and T_old.lmin == T_new.lmin
    F = finest_values(T_old, U_old)
    d, L = T_new.d, T_new.L
    U = {}
    for l in range(T_new.lmin, L + 1):
        s = 3 ** (L - l)
        U[l] = np.where(T_new.dof[l], F[tuple(slice(None, None, s) for _ in range(d))], 0.0)
    return T_new.spread(U)
