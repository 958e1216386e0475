"""FP64 CPU oracle for the localized fully implicit Newton solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never calls it, and this package never imports the library: the two share
only the seeded input generator ``fimgen``.

Contents (each function cites the passage of Jiang 2020, "Localized
nonlinear solution strategies for efficient simulation of unconventional
reservoirs", that it follows):

* ``physics``  : properties, accumulation and the TPFA/PPU residual of
                 Appendix A, written complex-safe;
* ``jacobian`` : the Jacobian dF/du by complex-step differentiation of that
                 residual (exact to rounding), columns grouped by a
                 distance-2 colouring;
* ``newton``   : the Newton method of Section 4.1 with a direct sparse LU
                 solve (SuperLU), timestep commit / rollback;
* ``sets``     : the set logic of Algorithms 1 and 2 and of the
                 residual-based estimate with Python sets;
* ``localized``: Algorithm 1 (localized Newton), Algorithm 2 (adaptive
                 nonlinear domain decomposition) and the residual-based
                 localization of Sections 1 and 4.2, built from the pieces
                 above.

Readings where the paper is silent are listed in each module header.
"""
