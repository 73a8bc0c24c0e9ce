"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic.  Every array is produced with numpy's PCG64
generator (``numpy.random.default_rng(seed)``) in C order with x on the last
axis, on the vertex lattice of the finest level ((3^L + 1)^d entries; the
boundary entries are drawn too and ignored) or on a block grid of the
coefficient ((3^k)^d entries).

The workloads mirror the paper's setting: -div(eps grad u) = f on the unit
square/cube, zero Dirichlet boundary, uniform spacetree levels, eps piecewise
constant on aligned blocks with log10(eps) uniform.
"""
import numpy as np


def rhs(d, L, seed=0, dist="uniform"):
    """Vertex samples of f: U(-1, 1) or N(0, 1) on the (3^L+1)^d lattice."""
    rng = np.random.default_rng(seed)
    shape = (3 ** L + 1,) * d
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, shape)
    if dist == "normal":
        return rng.standard_normal(shape)
    raise ValueError(dist)


def eps_blocks(d, k, log10_max, seed=0):
    """Coefficient blocks 10**U(0, log10_max) on the (3^k)^d cells of level k."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(0.0, log10_max, (3 ** k,) * d)


def poisson_blocks(d):
    """eps = 1 everywhere: a single block."""
    return np.ones((1,) * d)


# Named workloads ------------------------------------------------------------

def workload_2d_poisson_l4(seed=0):
    """2D Poisson, 81 x 81 finest cells (L = 4), f ~ U(-1, 1), 20 cycles."""
    return dict(d=2, L=4, lmin=1, eps=poisson_blocks(2), f=rhs(2, 4, seed, "uniform"), cycles=20)


def workload_3d_poisson_l5(seed=0):
    """3D Poisson, 243^3 finest cells (L = 5), f ~ N(0, 1)."""
    return dict(d=3, L=5, lmin=1, eps=poisson_blocks(3), f=rhs(3, 5, seed, "normal"))


def workload_jump(d, L, seed=0):
    """Jump-coefficient solve of the request stream: 9x9 blocks log10 U(0,3) in 2D,
    27^3 blocks log10 U(0,4) in 3D, f ~ U(-1, 1)."""
    k, p = (2, 3.0) if d == 2 else (3, 4.0)
    k = min(k, L)
    return dict(d=d, L=L, lmin=1, eps=eps_blocks(d, k, p, seed), f=rhs(d, L, seed + 1, "uniform"))


def request_stream(n, seed=0):
    """The mixed request stream of the serving workload, in arrival order.

    Half 2D with L ~ U{3..7} (eps on 9x9 blocks, log10 U(0, 3)), half 3D with L ~ U{3..5}
    (eps on 27^3 blocks, log10 U(0, 4)); f ~ U(-1, 1); precision FP64 or FP32 inner cycles
    with FP64 defect correction, half each.  Request i draws its coefficient with seed
    seed + i; its right-hand side is one of two per (d, L) (``f_seed``) so that a long stream
    does not hold thousands of large arrays.  Returns dicts with d, L, eps_seed, f_seed and
    precision.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        d = 2 if rng.random() < 0.5 else 3
        L = int(rng.integers(3, 8)) if d == 2 else int(rng.integers(3, 6))
        prec = "fp64" if rng.random() < 0.5 else "fp32_refined"
        out.append(dict(d=d, L=L, eps_seed=seed + i, f_seed=1000 * L + d * 10 + int(rng.integers(0, 2)),
                        precision=prec))
    return out


def poisson_arrivals(n, rate, seed=0):
    """Arrival times (s) of a Poisson process of the given rate (requests per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def refine_ball(d, L, l_uniform, centre, radius):
    """Refinement flags of a spacetree refined around a ball: a cell of level l (l_uniform <= l
    < L) is refined when its closure meets the closed ball.  Returns {l: bool array over the
    (3^l)^d cells} (C order, x on the last axis); the flags of cells that do not exist are
    ignored by the tree."""
    centre = np.asarray(centre, dtype=np.float64)
    out = {}
    for l in range(l_uniform, L):
        n = 3 ** l
        h = 1.0 / n
        idx = np.indices((n,) * d).astype(np.float64)        # axis 0 is the slowest (z or y)
        dist2 = np.zeros((n,) * d)
        for a in range(d):
            c = centre[d - 1 - a]                              # idx[a] runs along coordinate d-1-a
            lo, hi = idx[a] * h, (idx[a] + 1) * h
            gap = np.maximum(0.0, np.maximum(lo - c, c - hi))
            dist2 += gap * gap
        out[l] = dist2 <= radius * radius
    return out


def gaussian(d, L, centre, sigma, amplitude=1.0):
    """Samples of the source amplitude * exp(-|x - centre|^2 / (2 sigma^2)) on the finest
    vertex lattice (C order, x on the last axis)."""
    n = 3 ** L
    x = np.arange(n + 1) / n
    grids = np.meshgrid(*([x] * d), indexing="ij")            # axis a is coordinate d-1-a
    r2 = sum((grids[a] - centre[d - 1 - a]) ** 2 for a in range(d))
    return amplitude * np.exp(-r2 / (2.0 * sigma * sigma))


def moving_source(seed=0, steps=4, d=3):
    """Centres of the moving Gaussian source: x0 ~ U[0.3, 0.7]^d, then steps of 0.03 along a
    seeded unit vector, reflected at the faces of [0.3, 0.7]^d."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.3, 0.7, d)
    v = rng.standard_normal(d)
    v /= np.linalg.norm(v)
    out = [x.copy()]
    for _ in range(steps):
        x = x + 0.03 * v
        for a in range(d):
            if x[a] > 0.7:
                x[a], v[a] = 1.4 - x[a], -v[a]
            elif x[a] < 0.3:
                x[a], v[a] = 0.6 - x[a], -v[a]
        out.append(x.copy())
    return out


# The paper's own set-ups (Sec. 5): f = 0, u = 1 on the boundary part x_2 = 0 and u = 0 on the
# rest of the boundary, and four coefficient fields on the unit square with eps = 1 in one
# region and eps = 10^-k in the other.  x_1 is the first coordinate (the last array axis),
# x_2 the second.

PAPER_FIELDS = ("homogeneous", "split", "needle", "checkerboard")


def paper_eps_cells(L, kind, k):
    """eps on the (3^L)^2 finest cells, evaluated at the cell centres (array [x_2, x_1]):
    homogeneous: 1; split: 10^-k where x_1 > 1/2 (an axis-aligned split that no 3:1 level
    resolves); needle: 10^-k on the strip |x_1 - 1/2| <= 0.01, x_2 <= 1/2 (width 0.02, from
    the x_1 axis half-way into the domain); checkerboard: the lines x_2 = 5 x_1 - 2.5 and
    x_2 = 0.2 x_1 + 0.5 cut the square into four regions, and eps = 10^-k in the two where
    (x_2 - 5 x_1 + 2.5)(x_2 - 0.2 x_1 - 0.5) < 0."""
    n = 3 ** L
    c = (np.arange(n) + 0.5) / n
    x1, x2 = np.meshgrid(c, c, indexing="xy")       # x1 varies along the last axis
    low = 10.0 ** (-k)
    if kind == "homogeneous":
        inside = np.zeros((n, n), dtype=bool)
    elif kind == "split":
        inside = x1 > 0.5
    elif kind == "needle":
        inside = (np.abs(x1 - 0.5) <= 0.01) & (x2 <= 0.5)
    elif kind == "checkerboard":
        inside = (x2 - 5.0 * x1 + 2.5) * (x2 - 0.2 * x1 - 0.5) < 0.0
    else:
        raise ValueError(kind)
    return np.where(inside, low, 1.0)


def paper_boundary(d, L):
    """Dirichlet data on the (3^L + 1)^d vertex lattice: 1 on x_2 = 0, 0 on the rest of the
    boundary and in the interior (interior entries are ignored)."""
    n = 3 ** L
    g = np.zeros((n + 1,) * d)
    idx = [slice(None)] * d
    idx[d - 2] = 0                                   # the x_2 axis is the second-to-last
    g[tuple(idx)] = 1.0
    return g
