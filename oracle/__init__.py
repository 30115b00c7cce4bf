"""FP64 CPU oracle for the decoupled ensemble Elsasser MHD scheme (test infrastructure).

This package is test infrastructure only.  It is a plain, slow, direct
implementation of Algorithm 1 of the paper (Section 3, equations (weaknew1) and
(weaknew2)) with Taylor-Hood P2-P1 elements (Scott-Vogelius on barycentre-refined
meshes, and tetrahedral Taylor-Hood in 3D, as options): its own mesher, its own
quadrature-based FE assembly, and every member's saddle-point system solved
with its own sparse direct LU.  It shares no code with the GPU library; only
the seeded problem data of ``workloads`` feeds both.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it; the product path never does.

Modules:
  mesh    -- structured triangulations and P2/P1 node numbering
  tet     -- tetrahedral meshes of the unit cube, quadrature and P2/P1 bases (3D)
  fem     -- quadrature, P2/P1 bases, element integrals, global matrices
  scheme  -- Algorithm 1 (ensemble means, eddy viscosity, shared matrix,
             per-member right-hand sides, per-member LU solves)
  plain   -- the plain decoupled Elsasser scheme for one member (J = 1)
  adjoint -- discrete adjoint of Algorithm 1 for an ensemble-mean energy
"""
