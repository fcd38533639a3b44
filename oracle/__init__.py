"""Plain FP64 CPU oracle for the photoacoustic k-space solver.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference the GPU
library is checked against: slow, unfused, written from the paper's
equations.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library and
imports nothing from it.

Modules
-------
kspace    forward operator H and its exact transpose (sections II-A, III)
prox      FGP dual solver of the bound-constrained TV prox (section IV)
transfer  restriction / prolongation (section V) and FP64 reductions
solver    ISTA / FISTA and the two-level MG-FISTA (sections IV and V)

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or library routines.  The
heterogeneous lossy terms (tau and eta with per-point c0, alpha0 and rho0)
are pinned by the first-order convergence of the paper's own
adjoint-then-discretize system to the exact transpose.  The PML's profile
and placement are pinned only structurally (transpose, linearity, the
lossless limit and the decay it causes).
"""
from . import kspace, prox, solver, transfer  # noqa: F401
from .kspace import make_plan, forward, adjoint  # noqa: F401
from .prox import tv_prox  # noqa: F401
from .transfer import restrict, prolong, dot  # noqa: F401
