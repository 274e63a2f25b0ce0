"""Plain FP64 CPU oracle for the asymptotic-preserving (AP) step of
Tang, Wang & Zhang, "Accurate front capturing asymptotic preserving scheme
for nonlinear gray radiative transfer equation" (arXiv 1811.05579).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it. The GPU library and
its Python binding never import, call or link anything here, and nothing here
imports the GPU library: the two implementations share no code. The only
module both sides see is the seeded workload generator, which holds none of
the method's arithmetic.

Modules
-------
quadrature   Gauss-Legendre parity pairs (reading of the velocity grid) and
             the equally spaced circle directions of the 2-D workloads.
ap1d         One fully discrete AP step in 1-D, Algorithm 2 (Section 4) and its
             temperature-dependent-opacity variant (Section 5), solved with
             direct sparse linear algebra.
ap2d         The same step on a 2-D rectangle (staggered parity reading:
             E in cells, O on the faces), direct sparse linear algebra.
diffusion1d  The three-stage diffusion scheme (2.7) / its sigma/T^3 form, the
             two-stage counter-example (2.8), and the fully implicit
             reference solvers (6.1) and (6.7).
diffusion2d  The three-stage scheme (2.7)/(2.9) on a 2-D rectangle (the eps -> 0
             reference of ap2d).
energy       Energy bookkeeping used by the conservation pins, (3.12)-(3.13).
alt314       The alternative correction of the remark closing Section 3,
             (3.14): no nonlinear solve, T^{n+1} explicit, not energy
             conservative.
"""
