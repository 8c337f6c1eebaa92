"""Plain FP64 CPU oracle of the non-cutoff collision operator.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference against which the GPU library is checked.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the GPU product
path never does, and it shares no code with that path (the only common input is
the seeded data from the `workloads` module).

Contents
  quadrature  Gauss-Legendre in |q|, Lebedev on S^2, Gauss-Jacobi in t (eq. approxG)
  angular     the angular weight F (eq. FF) and its independent pins
  collision   the direct weighted sum (eq. sum with eq. approxG; eq. realQ regrouped)
  physics     moments, entropy dissipation, Heun and RK4 steps of the Galerkin ODE
  fast_fft    the fast algorithm (eq. realQ) with FFTs, for the CPU throughput baseline
  collision2d the two-dimensional operator (circle rule, eq. FF2D1) and the 2-D BKW solution
  bkw         the BKW exact solution and its closed-form Q (Section 5.1)

Every function here is pinned by a CPU test against something other than
itself (closed forms, library routines on special cases, brute force, the BKW
solution, the conservation laws).
"""
from .angular import (AngularKernel, DEBYE_KERNELS, DebyeKernel, PAPER_KERNELS, bkw_lambda, cutoff_kernel,
                      power_kernel, psi, F_weight, F_sphere, psi_cutoff_closed_form, psi_small_argument,
                      F_eps_split)
from .collision import (Discretization, collision_direct, mode_vectors, quadrature_nodes,
                        weight_table)
from .physics import entropy_dissipation, heun_step, moments, rk4_step, to_physical
from .fast_fft import collision_fft
from . import collision2d
from . import bkw, quadrature
