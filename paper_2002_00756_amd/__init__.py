"""MI355X-native Helmholtz multigrid solver (tensor-product V-cycle + CG).

The computation lives in the HIP library ``libhelmholtz.so`` (C ABI in
``include/helmholtz.h``); this package only marshals arguments:

* :class:`Operator`      operator hierarchy with ``apply``, ``vcycle``,
                         ``vcycle_f32``, ``solve`` and ``face_grad``;
* :func:`helmholtz_solve` / :class:`HelmholtzSolve`  differentiable solve;
* :func:`mesh_tables`    the library's cubed-sphere tables.
"""
from ._lib import HelmholtzError, load  # noqa: F401
from .solver import Operator, SolveResult, mesh_tables  # noqa: F401
from .autograd import HelmholtzNotConverged, HelmholtzSolve, helmholtz_solve  # noqa: F401
