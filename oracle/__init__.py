"""Plain FP64 CPU oracle for one explicit ADER-DG step on a periodic Cartesian grid.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, calls or links anything in this package.  Only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it, to check and to time the GPU path.

It is written from the paper (Charrier & Weinzierl, "Stop talking to me -- a
communication-avoiding ADER-DG realisation", arXiv:1801.08682):

* the PDE in first-order conservative form, Eq. (1), without the
  non-conservative, source and point-source terms (neglected in Sec. 3);
* nodal tensor-product Lagrange basis on Gauss-Legendre points (Sec. 3);
* the cell-local space-time predictor, Eq. (3), solved by Picard iteration with
  quadrature-free (collocated) operators (Sec. 3, "ADER-DG step 1");
* extrapolation of the predicted solution and its normal flux onto the cell
  faces (Sec. 3, task ``extrapolate``; Table 1);
* the Rusanov numerical flux, Eq. (4) (Sec. 3, "ADER-DG step 2");
* the corrector, Eq. (2), split into ``integrateVolume``, ``integrateFace`` and
  ``update`` (Sec. 3, "ADER-DG step 3"; Eq. (5)/(6));
* ``calcTimeStep``: the CFL-admissible step (Sec. 3, "Time stepping").

Readings of passages where the paper is silent or garbled are listed in
``DESIGN.md`` (section "Readings of the paper").

Modules
-------
tables       1D Gauss-Legendre nodal operators
pde          fluxes and wave speeds (advection, Euler, acoustics, elasticity)
step         predictor, traces, Rusanov, corrector, time step; sampled step
diagnostics  L2 norms, conserved totals, point evaluation, kinetic energy
adjoint      reverse mode through a rollout (torch autograd), functionals
fused        shifted, fused, optimistic time stepping (Alg. 2)
spacetime    the step with space-time traces and per-time-node Rusanov (Table 1)
mixed        the step with a float32 or bfloat16-input predictor and a float64
             corrector (precision emulation of the mixed GPU path)
fv           finite-volume subcell patches of the limiter: projection, least-
             squares reconstruction and the first-order Rusanov step (App. A)

Every function works on float64 torch CPU tensors so that torch.autograd gives
an adjoint that shares nothing with the hand-written GPU adjoint.
"""

from . import tables, pde, step, diagnostics, fused, spacetime, mixed, fv  # noqa: F401
