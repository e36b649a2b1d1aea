"""Plain FP64 CPU oracle for the actuated PD+IPC quasi-static solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library may import, call,
link or execute this package; only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
the two meet only in ``meshgen`` (seeded inputs, no solver arithmetic).

What it computes, following the paper (Li, Yang, Solenthaler 2023):

* ``fem``       per-tet rest data, gradient operators G_i, weights w_i and the
                constant PD matrix H of Eq. (2), assembled explicitly.
* ``local``     the local step of Eq. (1): R_i = argmin over SO(3) of
                ||F_i - R A_i||, via an SVD of F_i A_i.
* ``geometry``  unsigned point-triangle and edge-edge distances between closed
                primitives, with the closest-feature classification.
* ``barrier``   the IPC barrier of Eq. (3), its gradient and Hessian (autograd
                of the explicit per-feature distance formula), and the
                per-pair positive-definite projection of Algorithm 1.
* ``contact``   constraint sets and swept candidate sets by brute force.
* ``ccd``       conservative-advancement step bound (Section 2.2).
* ``solver``    Algorithm 1 with the global step of Eq. (4) solved by a sparse
                LU of the assembled H + B every iteration (no prefactoring,
                no Schur complement, no Woodbury update), plus the adjoint of a
                converged solve.

Readings where the paper is silent are listed in the repository's design
notes and repeated in each function's docstring.
"""
