"""CPU float64 oracle for the Helmholtz multigrid hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or run
anything in this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code with the GPU library.

It is a plain, slow, obviously-correct restatement of what the paper's
pressure solver computes (Maynard, Melvin and Mueller, "Multigrid
preconditioners for the mixed finite element dynamical core of the LFRic
atmospheric model"):

* ``mesh``       cubed-sphere columns, horizontal neighbours, the face table and
                 the 2x2 nested hierarchy (Section 3.6 coarsens horizontally
                 only; the mesh topology itself is not in the paper, which
                 reads mesh files).
* ``helmholtz`` the synthetic symmetric face-coupling operator that stands in
                 for H (Eq. helmholtz_operator, Section 3.4), its split into
                 the column part H_z and the rest (Section 3.5), and the coarse
                 operators by re-discretisation (Section 3.6).
* ``smoother``   the column tridiagonal solve (Thomas algorithm) and the
                 block-Jacobi iteration (Section 3.6, Eq. jacobi).
* ``multigrid``  prolongation by natural injection, restriction as its dual,
                 and the recursive V-cycle (Section 3.6, Algorithm 1).
* ``krylov``     preconditioned conjugate gradients (Section 4.1, CG(A, P, eps))
                 and the float32 preconditioner emulation.
* ``adjoint``    gradients of a linear loss of the solution (not in the paper).

Everything is float64 NumPy unless a function says otherwise.

Parity status: every float64 function is pinned by the CPU tests against
closed forms, dense linear algebra, brute force or library routines. The
float32 emulation (``krylov.mg_preconditioner_f32``, ``Hierarchy.astype``) is
pinned by its parts: its coefficients bit for bit against the exact
re-discretised values rounded once, its column solve against a float64 banded
solver within the Thomas algorithm's forward-error bound, and the one-level
V-cycle against its closed form within that bound. A whole float32 V-cycle
has no bit-exact target (float32 results depend on the order of operations).
"""
from . import mesh, helmholtz, smoother, multigrid, krylov, adjoint  # noqa: F401
