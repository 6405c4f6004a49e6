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

Parity status of every function is listed in the module docstrings; no
function here is "parity unpinned": each is checked by ``tests/test_oracle_*``
against closed forms, invariants, independent formulations or brute force.
"""
