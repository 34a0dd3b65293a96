"""CPU FP64 oracle for the space-time multigrid hot path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
reference written from the paper (Benedusi, Minion, Krause: space-time
multigrid vs PFASST for a reaction-diffusion problem).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The GPU library never calls into it and shares no code with it.

Modules
-------
radau     right-Radau nodes, collocation matrix Q, DG matrices (Sec. 2)
space     finite-difference spatial operators (Sec. 3, lumped linear FE)
stepper   sequential Radau IIA time stepping with a direct sparse solve
          per step (the collocation form, Eq. collocation), linear and
          Allen-Cahn (Newton per step)
allatonce dense assembly of the all-at-once DG system (Eq. st_system) and
          its residual; brute-force solve on tiny grids
fourier   closed-form solution of the linear periodic problem mode by mode
adjoint   discrete adjoint of the sequential stepper (gradients of a
          terminal loss w.r.t. u0 and the diffusion coefficient)
mg        the multigrid components (transfers, block-Jacobi smoother,
          level hierarchy, V-cycle) spelled out plainly in NumPy
krylov    restarted flexible GMRES with the V-cycle as right preconditioner
ilu       ILU(0) and the ILU(0)-preconditioned GMRES smoother of the paper
galerkin  assembled transfers and Galerkin coarse operators R A P
paper_hierarchies  runner: the paper's hierarchies on its 1D heat example
          with both smoothers and both coarse-operator choices
"""
