"""Plain CPU reference ("oracle") for the cascaded lattice Boltzmann (CLB) step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path.

Source of truth: Liu & He, "Numerical modelling of microchannel gas flows in
the transition flow regime using the cascaded lattice Boltzmann method"
(arXiv:1603.01955), Section 2 (Eqs. 1-21) and Section 3.

Modules
-------
lattice   D2Q9 velocities (Eq. 1), K (Eq. 3), T and its exact inverse (Eq. 10),
          the binomial raw->central moment shift, the equilibrium (Eq. 11).
clb_ref   Parameters (Eqs. 14-18, 21, Section 3), streaming with walls and
          inlet/outlet (Eqs. 5, 20, Sections 3.1-3.2), the collision in two
          forms (explicit moment matrices; the closed form of Eqs. 6-9),
          diagnostics (Eqs. 12-13, Sections 3.1-3.2) and time stepping.
exact     Exact rational (fractions.Fraction) evaluation of the closed-form
          collision and of a whole step on tiny grids, node by node.
analytic  Closed-form steady solutions used to pin the above (discrete
          slip-channel profile, continuum second-order slip profile, Knudsen
          minimum, lubrication mass flow).
rng       SplitMix64 counter-based generator for the seeded perturbed start.
clb3d_ref The 3-D extension to rectangular microducts (D3Q27, central
          moments by definition, walls of Eq. 20 carried to 3-D), which the
          paper names as future work; pinned by mathematics and by reduction
          to the 2-D reference (tests/test_oracle_3d.py).
"""
