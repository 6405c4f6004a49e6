"""CPU FP64 oracle for the many-beam RHEED/TRHEPD reflection problem.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
GPU library; both sides consume the seeded inputs of ``synth`` and nothing
else.

Contents (section numbers are the paper's, arXiv 2306.00271):

* ``physics``      -- wavenumber, interaction constant, incident wavevector
                      and the diagonal Gamma (Sec. 2.1, Eq. sch3).
* ``potential``    -- Fourier coefficients of the slab potential on the
                      slice nodes, and their derivatives w.r.t. atom
                      coordinates (Sec. 2.1, Eq. sch2).
* ``tableaux``     -- explicit Runge-Kutta tableaux (classical RK4,
                      Butcher's 7-stage sixth-order method).
* ``rk``           -- the proposed method: matrix ODE in economical form
                      stepped by explicit RK with the right-hand-side
                      transformation (Sec. 3.1-3.4, Algorithm 1).
* ``conventional`` -- the conventional multi-slice method: piecewise
                      constant potential, exact slice exponential by
                      eigendecomposition, recursive reflection (Sec. 2.2).
* ``closed_form``  -- single-beam homogeneous slab (textbook result used
                      as a pin).
* ``tangent``      -- tangent-linear (forward-mode) derivative of the RK
                      method, for checking gradients.
* ``splitting``    -- BAB splitting steppers (Sec. 3.4).
* ``bulk``         -- the bulk layer: reflection matrix of the ideal bulk
                      by iterating one unit layer until it converges, used
                      as the bottom condition of the surface (Sec. 2.2).

Every function here is pinned by ``tests/test_oracle_*.py`` against what
the paper and the mathematics fix rather than against itself: handbook
constants, rooted-tree order conditions, a real-space quadrature of the
potential and of the coupling matrix element (which fixes the orientation
of l(j,k)), closed-form single-beam slabs, the Fresnel limit, agreement of
independent formulations (eigen, Ichimiya recursion, global product, RK),
order under step halving, flux conservation, RHST invariance, symmetries
and central differences.  The pins of each module are listed in its
docstring.
"""
