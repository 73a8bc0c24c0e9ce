"""Plain FP64 CPU oracle of the additively damped asynchronous FAC cycle (adAFAC).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_1903_10367_amd``) and imports nothing from it.

It restates, in slow and obvious form, what the method of Murray & Weinzierl,
"Stabilised asynchronous fast adaptive composite multigrid using additive
damping" (Numer. Linear Algebra Appl., arXiv:1903.10367) computes:

* ``fem``        Q1 finite elements on a level of the 3:1 spacetree (Sec. 2.1),
                 element-wise assembly (Sec. 4.2), lumped right-hand side.
* ``transfer``   d-linear and BoxMG prolongation (Sec. 2.5), injection (Sec. 2.4).
* ``hierarchy``  Ritz-Galerkin coarse operators (Sec. 2.2), Jacobi diagonals,
                 the smoothed auxiliary restriction R~ (Sec. 3.2).
* ``cycle``      one adAFAC-Jac cycle (eq. (adaFACx), Algorithm 1) in the
                 correction form and in the FAS/HTMG form (eq. (fas-with-htmg)),
                 plus the adAFAC-PI, plain additive and exponentially damped
                 variants, residual norms (Sec. 5) and FP32 defect correction.
* ``dense``      tiny-grid dense tools: direct solve, iteration matrix.

All vectors live on the full vertex lattice of a level, shape ``(n+1,)*d`` in C
order with x fastest (last axis), boundary entries identically zero; the
operators are ``scipy.sparse`` matrices whose boundary rows and columns are
removed, so boundary vertices carry no equation (Sec. 2.1).

Every function states the passage of the paper it follows.  Functions whose
result the paper does not fix, and that no test pins to an outside value, say
"parity unpinned" in their docstring.
"""
