"""MI355X-native additively damped asynchronous FAC (adAFAC) solver.

Python face of the C ABI in ``include/adafac.h``: the arguments are marshalled with
ctypes, device memory for the workspace comes from a torch uint8 tensor and the
stream from torch's current stream.  Every step of the cycle runs in the gfx950
kernels of ``libadafac.so``; there is no CPU path.
"""
import ctypes as C

import numpy as np

from . import _abi
from ._abi import AdafacError, DAMPING, LEVEL_ARRAY, PRECISION, RTILDE, TRANSFER

__all__ = ["Solver", "Server", "AdafacError", "lib", "stream_copy"]

lib = _abi.lib


def _check(L, ctx, rc):
    if rc != _abi.OK:
        msg = L.adafac_last_error(ctx)
        raise AdafacError(rc, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def stream_copy(src, dst, stream=None):
    """Reference streaming copy of device tensor src into dst (same number of bytes, 16-byte
    aligned; roofline context, see adafac_stream_copy).  Runs on `stream` (default: torch's
    current stream of src's device)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise AdafacError(1, "stream_copy: two device tensors of the same size")
    st = stream or torch.cuda.current_stream(src.device)
    L = lib()
    rc = L.adafac_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                              C.c_void_p(st.cuda_stream))
    if rc:
        raise AdafacError(rc, "adafac_stream_copy: null, misaligned or not a multiple of 16 bytes")


class Solver:
    """One adAFAC solve on a uniform 3:1 spacetree of dimension ``dim`` with levels lmin..lmax.

    ``eps_blocks``: coefficient on the (3^k)^dim cells of level k (None: Poisson);
    ``f``: right-hand side samples on the (3^lmax + 1)^dim finest vertices, a callable
    f(x) of the dim coordinates (x first), or {"gaussian": (centre, sigma, amplitude)};
    ``rtilde``: "const" (the eps = 1 smoothed restriction) or "operator" (built per vertex from
    the level's own operator).
    """

    def __init__(self, dim, lmin, lmax, f, eps_blocks=None, transfer="dlinear", damping="jac",
                 precision="fp64", inner_k=4, fused=True, omega=0.6, omega_tilde=0.6, omega_hat=0.5,
                 device=None, stream=None, refine=None, ball=None, rtilde="const", static_workspace=False,
                 dirichlet=None):
        """``refine``: {level: flags over the (3^level)^dim cells} of an adaptive tree;
        ``ball``: (centre, radius, l_from) refinement around a ball (adaptive tree);
        ``static_workspace``: bind to the library's own device array (adafac_bind_static)
        instead of a torch-allocated workspace; ``dirichlet``: values of u on the boundary, given
        on the finest vertex lattice (interior entries ignored)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("adafac needs a ROCm GPU (gfx950); none is visible")
        self.L = _abi.lib()
        self.dim, self.lmin, self.lmax = dim, lmin, lmax
        ctx = C.c_void_p()
        rc = self.L.adafac_create(C.byref(ctx), dim, lmin, lmax)
        if rc:
            raise AdafacError(rc, "adafac_create")
        self.ctx = ctx
        if eps_blocks is not None:
            e = np.ascontiguousarray(eps_blocks, dtype=np.float64)
            _check(self.L, ctx, self.L.adafac_set_coefficient_blocks(ctx, e.shape[0], _dptr(e)))
        if isinstance(f, dict):
            # {"gaussian": (centre, sigma, amplitude)}: a Gaussian source evaluated by the library
            centre, sigma, amp = f["gaussian"]
            cc = np.ascontiguousarray(centre, dtype=np.float64)
            _check(self.L, ctx, self.L.adafac_set_rhs_gaussian(ctx, _dptr(cc), sigma, amp))
        elif callable(f):
            fn = f
            self._rhs_cb = _abi.RHS_FN(lambda x, user: float(fn(tuple(x[a] for a in range(dim)))))
            _check(self.L, ctx, self.L.adafac_set_rhs_fn(ctx, self._rhs_cb, None))
        else:
            fa = np.ascontiguousarray(f, dtype=np.float64).ravel()
            _check(self.L, ctx, self.L.adafac_set_rhs_lattice(ctx, _dptr(fa), fa.size))
        if dirichlet is not None:
            g = np.ascontiguousarray(dirichlet, dtype=np.float64).ravel()
            _check(self.L, ctx, self.L.adafac_set_dirichlet_lattice(ctx, _dptr(g), g.size))
        for level, flags in (refine or {}).items():
            fl = np.ascontiguousarray(flags, dtype=np.uint8).ravel()
            _check(self.L, ctx, self.L.adafac_set_refinement(ctx, level, fl.ctypes.data_as(C.POINTER(C.c_uint8)),
                                                             fl.size))
        if ball is not None:
            centre, radius, l_from = ball
            cc = np.ascontiguousarray(centre, dtype=np.float64)
            _check(self.L, ctx, self.L.adafac_refine_ball(ctx, _dptr(cc), radius, l_from))
        o = _abi.Opts()
        self.L.adafac_default_opts(C.byref(o))
        o.transfer, o.damping, o.precision = TRANSFER[transfer], DAMPING[damping], PRECISION[precision]
        o.rtilde = RTILDE[rtilde]
        o.inner_k, o.fused = inner_k, int(bool(fused))
        o.omega, o.omega_tilde, o.omega_hat = omega, omega_tilde, omega_hat
        _check(self.L, ctx, self.L.adafac_build_operators(ctx, C.byref(o)))
        nbytes = C.c_size_t()
        _check(self.L, ctx, self.L.adafac_workspace_bytes(ctx, C.byref(nbytes)))
        self.device = torch.device(device or "cuda:0")
        self.stream = stream or torch.cuda.current_stream(self.device)
        if static_workspace:
            self.workspace = None
            _check(self.L, ctx, self.L.adafac_bind_static(ctx, C.c_void_p(self.stream.cuda_stream)))
        else:
            self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
            _check(self.L, ctx, self.L.adafac_bind(ctx, C.c_void_p(self.workspace.data_ptr()),
                                                   self.workspace.numel(), C.c_void_p(self.stream.cuda_stream)))
        self.nvert = (3 ** lmax + 1) ** dim

    # --- cycle ----------------------------------------------------------------
    def cycle(self, n=1):
        _check(self.L, self.ctx, self.L.adafac_cycle(self.ctx, n))

    def solve(self, rel_tol, max_cycles):
        done = C.c_int()
        rc = self.L.adafac_solve(self.ctx, rel_tol, max_cycles, C.byref(done))
        _check(self.L, self.ctx, rc)
        return done.value

    def residual(self, i):
        a, b = C.c_double(), C.c_double()
        _check(self.L, self.ctx, self.L.adafac_residual(self.ctx, i, C.byref(a), C.byref(b)))
        return a.value, b.value

    def residuals(self):
        return [self.residual(i) for i in range(self.L.adafac_cycles_run(self.ctx))]

    def residual_normalised(self, i):
        a, b = C.c_double(), C.c_double()
        _check(self.L, self.ctx, self.L.adafac_residual_normalised(self.ctx, i, C.byref(a), C.byref(b)))
        return a.value, b.value

    def dof_coords(self):
        """(positions (n, dim), levels (n,)) of the composite dofs, in composite order."""
        n = self.composite_dofs()
        xyz = np.empty((n, self.dim))
        lev = np.empty(n, dtype=np.int32)
        _check(self.L, self.ctx, self.L.adafac_dof_coords(self.ctx, _dptr(xyz), lev.ctypes.data_as(C.POINTER(C.c_int)),
                                                          n))
        return xyz, lev

    def composite(self):
        u = np.empty(self.composite_dofs())
        _check(self.L, self.ctx, self.L.adafac_get_composite(self.ctx, _dptr(u), u.size))
        return u

    def set_composite(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        _check(self.L, self.ctx, self.L.adafac_set_composite(self.ctx, _dptr(u), u.size))

    def solution(self):
        u = np.empty(self.nvert)
        _check(self.L, self.ctx, self.L.adafac_get_solution(self.ctx, _dptr(u), u.size))
        return u

    def set_solution(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        _check(self.L, self.ctx, self.L.adafac_set_solution(self.ctx, _dptr(u), u.size))

    def set_solution_coarse(self, u, l_src):
        """Start from a shallower tree's finest-lattice solution (interpolated by the library)."""
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        _check(self.L, self.ctx, self.L.adafac_set_solution_coarse(self.ctx, _dptr(u), u.size, int(l_src)))

    def amr_mark(self, fraction, l_uniform, l_cap):
        """Refinement flags of the next tree ({level: bool array}, levels l_uniform..l_cap-1) and
        its depth, from adafac_amr_mark."""
        sizes = [(3 ** l) ** self.dim for l in range(l_uniform, l_cap)]
        flags = np.zeros(sum(sizes), dtype=np.uint8)
        lnew = C.c_int()
        _check(self.L, self.ctx, self.L.adafac_amr_mark(self.ctx, float(fraction), int(l_uniform), int(l_cap),
                                                         flags.ctypes.data_as(C.POINTER(C.c_uint8)), flags.size,
                                                         C.byref(lnew)))
        out, k = {}, 0
        for l, n in zip(range(l_uniform, l_cap), sizes):
            out[l] = flags[k:k + n].reshape((3 ** l,) * self.dim).astype(bool)
            k += n
        return out, int(lnew.value)

    def level(self, level, which):
        out = np.empty((3 ** level + 1) ** self.dim)
        _check(self.L, self.ctx, self.L.adafac_get_level(self.ctx, level, LEVEL_ARRAY[which], _dptr(out), out.size))
        return out

    def dofs_per_cycle(self):
        return int(self.L.adafac_dofs_per_cycle(self.ctx))

    def composite_dofs(self):
        return int(self.L.adafac_composite_dofs(self.ctx))

    def regrid(self, centre, radius, l_from, f=None):
        """Move an adaptive solve onto the tree refined around a new ball, with a new right-hand
        side; the iterate is transferred and the residual history kept."""
        import torch
        cc = np.ascontiguousarray(centre, dtype=np.float64)
        nbytes = C.c_size_t()
        if f is None:   # Gaussian source: it moves with the ball
            rc = self.L.adafac_regrid_prepare(self.ctx, _dptr(cc), radius, l_from, None, 0, C.byref(nbytes))
        else:
            fa = np.ascontiguousarray(f, dtype=np.float64).ravel()
            rc = self.L.adafac_regrid_prepare(self.ctx, _dptr(cc), radius, l_from, _dptr(fa), fa.size, C.byref(nbytes))
        _check(self.L, self.ctx, rc)
        ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        _check(self.L, self.ctx, self.L.adafac_regrid(self.ctx, C.c_void_p(ws.data_ptr()), ws.numel()))
        self.workspace = ws

    def set_kernel_timing(self, on):
        _check(self.L, self.ctx, self.L.adafac_set_kernel_timing(self.ctx, int(on)))

    def kernel_time(self):
        ms, n = C.c_double(), C.c_int()
        _check(self.L, self.ctx, self.L.adafac_kernel_time(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "ctx", None):
            self.L.adafac_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server of the C ABI (continuous batching of independent solves).

    The pool for the request hierarchies is a torch uint8 tensor of ``budget_bytes`` on
    ``device``; all work runs on torch's current stream there (plus the server's own streams
    for requests above ``batch_max_vertices``, when set).
    """

    def __init__(self, budget_bytes, max_active=256, max_queued=4096, cycles_per_round=4, max_streams=4,
                 batch_max_vertices=None, device=None, stream=None):
        """``batch_max_vertices``: finest-level vertex count above which a request runs on a
        stream of its own (None: every request joins the batched launch)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("adafac needs a ROCm GPU (gfx950); none is visible")
        self.L = _abi.lib()
        cfg = _abi.ServerCfg()
        self.L.adafac_server_default_cfg(C.byref(cfg))
        cfg.max_active, cfg.max_queued, cfg.cycles_per_round = max_active, max_queued, cycles_per_round
        cfg.max_streams = max_streams
        if batch_max_vertices is not None:
            cfg.batch_max_vertices = batch_max_vertices
        self.device = torch.device(device or "cuda:0")
        self.workspace = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        srv = C.c_void_p()
        rc = self.L.adafac_server_create(C.byref(cfg), C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(srv))
        if rc:
            raise AdafacError(rc, "adafac_server_create")
        self.srv = srv
        self._sizes = {}

    def _err(self, rc, what):
        if rc != _abi.OK:
            msg = self.L.adafac_server_last_error(self.srv)
            raise AdafacError(rc, f"{what}: {msg.decode() if msg else ''}")

    def submit(self, dim, lmin, lmax, f, eps_blocks=None, rel_tol=1e-8, max_cycles=200, transfer="dlinear",
               damping="jac", precision="fp64", inner_k=4, fused=True, omega=0.6, omega_tilde=0.6,
               omega_hat=0.5):
        """Queue a solve; returns its ticket, or None when the queue is full (submit again later)."""
        q = _abi.Request()
        q.dim, q.l_min, q.l_max = dim, lmin, lmax
        fa = np.ascontiguousarray(f, dtype=np.float64).ravel()
        q.f = _dptr(fa)
        if eps_blocks is not None:
            e = np.ascontiguousarray(eps_blocks, dtype=np.float64)
            q.blocks_per_axis, q.eps = e.shape[0], _dptr(e)
        else:
            q.blocks_per_axis = 0
        self.L.adafac_default_opts(C.byref(q.opts))
        q.opts.transfer, q.opts.damping, q.opts.precision = TRANSFER[transfer], DAMPING[damping], PRECISION[precision]
        q.opts.inner_k, q.opts.fused = inner_k, int(bool(fused))
        q.opts.omega, q.opts.omega_tilde, q.opts.omega_hat = omega, omega_tilde, omega_hat
        q.rel_tol, q.max_cycles = rel_tol, max_cycles
        t = C.c_uint64()
        rc = self.L.adafac_server_submit(self.srv, C.byref(q), C.byref(t))
        if rc == _abi.EAGAIN:
            return None
        self._err(rc, "submit")
        self._sizes[t.value] = fa.size
        return t.value

    def step(self):
        """One scheduling round; returns (active, queued)."""
        a, q = C.c_int(), C.c_int()
        self._err(self.L.adafac_server_step(self.srv, C.byref(a), C.byref(q)), "step")
        return a.value, q.value

    def poll(self, ticket):
        r = _abi.Result()
        self._err(self.L.adafac_server_poll(self.srv, ticket, C.byref(r)), "poll")
        return {name: getattr(r, name) for name, _ in r._fields_} | {"state": _abi.REQ_STATUS[r.status]}

    def fetch(self, ticket):
        n = self._sizes.pop(ticket)
        u = np.empty(n)
        self._err(self.L.adafac_server_fetch(self.srv, ticket, _dptr(u), n), "fetch")
        return u

    def run_until_idle(self, max_rounds=100000):
        for _ in range(max_rounds):
            a, q = self.step()
            if a == 0 and q == 0:
                return
        raise RuntimeError("server did not drain")

    def close(self):
        if getattr(self, "srv", None):
            self.L.adafac_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
