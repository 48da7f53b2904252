"""MI355X library for the semiclassical nonlinear-Poisson Newton-Krylov solve
of gate-defined quantum-dot stacks (Gao et al., QCAD, Sec. II.A).

The compute path is the HIP library ``libqe.so`` (C ABI in include/qe.h);
``qe`` is its ctypes binding and ``autograd`` wraps the adjoint as a
``torch.autograd.Function``.
"""
from . import qe  # noqa: F401
from .qe import (  # noqa: F401
    Physics,
    Problem,
    QeError,
    Workspace,
    load_library,
    qe_adjoint,
    qe_count_electrons,
    qe_default_options,
    qe_density,
    qe_jv,
    qe_jv_f32,
    qe_last_error,
    qe_residual,
    qe_solve,
    qe_solve_batch,
    qe_workspace_bytes,
)
