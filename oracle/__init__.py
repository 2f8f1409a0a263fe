"""Plain FP64 CPU oracle of the rotating IMEX-DG method (test infrastructure).

This package is the reference that the HIP path is checked against. It is
slow on purpose and written for reading against the paper: the nodal DG
space and quadrature of Sec. 3, the weak forms of the momentum and energy
stage equations (matrices A, B, R, C, D, M_g and vectors f, f_g, g, k), the
Schur complement systems of the R1 and R2 fixed-point treatments, GMRES on
the pressure system, the rotational factorisation of Sec. 3.1 and the
IMEX-ARK2 step built from the Butcher tableau of Sec. 3.

Only the test suite, the smoke check and the CPU-baseline leg of the bench
may import it. The product path never calls into it and shares no code,
tables or helpers with it.

Pins (tests/test_oracle_bruteforce.py, tests/test_oracle_pins.py): dense
brute-force assembly of every stage matrix and of the explicit residual on
periodic, walled, terrain-following and hanging-face meshes; quadrature and
tableau order conditions; the closed-form inertial oscillation; reduction to
1D upwind DG for linear advection; free stream, polynomial rest state, mass
conservation, R1 = R2 fixed point, slice invariance; the DoF counts and
Courant numbers printed in Sec. 4.

The Rayleigh sponge term of Sec. 4.3 is pinned by hand values of its profile
and by its closed form on a free stream; its place in the IMEX split (the
non-stiff part) and what it relaxes are readings, not stated in the paper:
by default the momentum towards rho u_target, or, with Phys.sponge_target, the
whole conserved state towards a given state (pinned against the first: with
the state's own density and energy and momentum rho u_target as the target
the two agree, and with the state itself as the target the layers vanish).

Face values are formed from the traces of the nodal (rho, u, p), the
variables in which Sec. 3 writes its averages and jumps and on whose traces
the stage operators B and C act. The energy dissipation is split into
lambda/2 [rho kappa] (non-stiff) and lambda/2 [rho e] (stiff). Its sum is
pinned against a textbook total-energy Rusanov residual of the full Euler
equations (tests/test_oracle_bruteforce.py); the implicit stage operators
(C^k, M_g, Lambda^k, k^k, B, R, f_g) are pinned term by term against the
explicit stiff part T_S, and the whole stage equation of Sec. 3 is pinned at
converged stages of ARK2 steps from random states, row by row to round-off
(tests/test_oracle_stage_pins.py), so the lagged Lambda^k is the stiff
dissipation of the explicit residual. Which part of the split is stiff is the
paper's statement (the energy stage equations of Sec. 3), not a derived
result. The Picard variation measure (the stop criterion of the fixed-point
loop, a reading: the paper names only a prescribed tolerance) is pinned by
closed forms.
"""
