"""Plain, slow, FP64 CPU oracle of the split-form DGSEM Navier-Stokes operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with
the HIP path (no kernels, headers, tables or helpers); the two meet only
through the seeded inputs of ``paper_2606_18927_amd.workloads``, which holds
none of the method's arithmetic.

What it computes (paper: Sec. 2.1-2.2 split-form DG on Legendre-Gauss-Lobatto
nodes; Sec. 4 low-storage 4th-order RK, ideal gas, viscous fluxes):

* ``basis``   LGL nodes, weights and the nodal derivative matrix.
* ``mesh``    axis-aligned tensor-product hexahedral meshes (periodic or
              isothermal-wall ends per direction).
* ``physics`` ideal-gas primitive recovery, Euler, Kennedy-Gruber two-point and
              viscous fluxes, local Lax-Friedrichs surface flux, wall state.
* ``dgsem``   BR1 lifting, the strong-form split DG right-hand side, the
              five-stage low-storage RK step, the kinetic-energy functional.
* ``adjoint`` reverse-mode (torch.autograd on the oracle itself) and
              complex-step forward derivatives of the above.

All floating point is float64 (complex128 for the complex step), written in
plain torch CPU tensor operations with no blocking, fusion or reordering beyond
the definitions.  Pins of every function live in ``tests/test_oracle_*.py``.
The readings taken where the paper is silent are listed in the module
docstrings where they are used.
"""

from . import basis, mesh, physics, dgsem, adjoint  # noqa: F401
