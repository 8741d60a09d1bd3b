"""FP64 CPU oracle for the lumped-mass Gaussian-random-field sampler.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library: it assembles the global finite-element matrices and solves them
directly (dense, sparse LU, or through the generalised eigen-decomposition),
while the library uses static condensation, per-edge recurrences and a vertex
Schur-complement PCG.

Modules
-------
mesh        Phase-1 mesh and DOF numbering, mass/stiffness assembly
            (paper: "Phase 1: Initialization", "Phase 2: Global Setup").
quadrature  Balakrishnan sinc-quadrature shift schedule
            (paper: eq. balakrishnan_quadrature, eq. coefficients, limits in
            the "Strong error" subsection).
noise       Counter-based Philox4x64-10 normals and lumped white noise
            (paper: eq. wh_def and the "Mass Lumping" subsection).
solve       Direct solves of the shifted systems and the quadrature sum
            (paper: eq. spde_approx_fem).
spectral    Generalised-eigenvector route and the closed-form Neumann cosine
            expansion on one interval (textbook pins, not from the paper).

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against something other than itself (numpy's own
Philox, closed forms, invariants, brute force, printed paper values); none is
"parity unpinned".
"""
