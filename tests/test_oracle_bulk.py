"""Pins for the oracle's bulk layer (oracle/bulk.py): the bottom state and
its reflection matrix, composition of a slab from its parts, the
single-beam closed form after k unit layers and its Fresnel limit,
decoupled beams, the fixed point and its stability (CPU only)."""
import dataclasses

import numpy as np
import pytest

from oracle import bulk, closed_form, driver, rk, tangent
from oracle.tableaux import RK4, RK6
from synth import bulk_layer, small_2d


def _const(M):
    return lambda i, r: M


def test_bottom_state_and_its_reflection_matrix():
    gam = np.array([0.7, 2.0, -3.0j])
    # the vacuum is Y = i Gamma, whose reflection matrix is 0
    z0 = rk.initial_state(gam)
    assert np.abs(rk.initial_state(gam, y_bottom=1j * np.diag(gam)) - z0).max() == 0.0
    assert np.abs(bulk.reflection_of_state(1j * np.diag(gam), gam)).max() < 1e-15
    # S [I; Y] = [tau; rho] with rho = R tau, R = (Gamma + iY)(Gamma - iY)^{-1}
    rng = np.random.default_rng(3)
    Y = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    tr = rk.boundary_matrix(gam) @ rk.initial_state(gam, y_bottom=Y)
    R = bulk.reflection_of_state(Y, gam)
    assert np.abs(tr[3:] - R @ tr[:3]).max() < 1e-13 * np.abs(tr).max()
    # and the reflection of the final state of a solve is the same formula
    Z = np.vstack([rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)), Y])
    Y2 = rk.normalised_lower(Z)
    assert np.abs(rk.reflection_matrix(Z, gam) - bulk.reflection_of_state(Y2, gam)).max() < 1e-13


@pytest.mark.parametrize("tab", [RK4, RK6])
def test_slab_equals_its_upper_part_on_the_lower_parts_state(tab):
    """Sec. 2.2 and 3.2: rho(0) of a slab from the vacuum equals that of its
    upper part started from the normalised state at the top of its lower
    part."""
    wl = small_2d(n_beams=13, n_slices=40, thickness=6.0, n_layers=2, n_angles=2)
    st = driver.StructureSetup(wl, wl.structures[0], tab)
    L1 = 23
    for th in wl.theta0:
        gam, _ = st.angle(float(th))
        M = st.mfun(gam)
        whole, _ = rk.solve_ode_str(M, gam, st.h, 40, tab)
        Ymid = bulk.layer_map(M, gam, st.h, L1, tab, 1j * np.diag(gam))
        upper, _ = rk.solve_ode_str(lambda i, r: M(i + L1, r), gam, st.h, 40 - L1, tab, y_bottom=Ymid)
        scale = np.abs(whole).max()
        assert np.abs(upper - whole).max() <= 1e-11 * scale
        # a transposed state or the vacuum below breaks it
        for wrong in (Ymid.T, 1j * np.diag(gam)):
            bad, _ = rk.solve_ode_str(lambda i, r: M(i + L1, r), gam, st.h, 40 - L1, tab, y_bottom=wrong)
            assert np.abs(bad - whole).max() > 1e-6 * scale


@pytest.mark.parametrize("U0", [4.0 - 0.3j, -4.0 - 0.3j])
def test_layers_of_a_constant_potential_follow_the_closed_form(U0):
    """k unit layers of a constant coupling are one slab of thickness k d:
    R_k is the closed-form single-beam reflection, and the limit is the
    Fresnel value of the half space."""
    gam = np.array([1.1 + 0j])
    M = np.array([[U0 + gam[0] ** 2]])
    d, L = 3.1, 124
    Y = 1j * np.diag(gam)
    for k in range(1, 7):
        Y = bulk.layer_map(_const(M), gam, d / L, L, RK6, Y)
        R = bulk.reflection_of_state(Y, gam)
        assert R[0, 0] == pytest.approx(closed_form.slab_rt(gam[0], U0, k * d)[0], abs=1e-10)
    _, Rb, n = bulk.bulk_reflection(_const(M), gam, d / L, L, RK6, tol=1e-12, max_layers=400)
    assert n > 0
    assert Rb[0, 0] == pytest.approx(closed_form.fresnel_r(gam[0], U0), abs=1e-9)


def test_decoupled_beams_have_a_diagonal_bulk_matrix():
    gam = np.array([0.9, 2.0, 1.3])
    U0 = 3.0 - 0.4j
    M = np.diag(U0 + gam ** 2)
    d, L = 3.1, 124
    Yb, Rb, n = bulk.bulk_reflection(_const(M), gam, d / L, L, RK6, tol=1e-12, max_layers=400)
    assert n > 0
    assert np.abs(Rb - np.diag(np.diag(Rb))).max() < 1e-14
    assert np.abs(Yb - np.diag(np.diag(Yb))).max() < 1e-13
    for j in range(3):
        assert Rb[j, j] == pytest.approx(closed_form.fresnel_r(gam[j], U0), abs=1e-9)
        # the half space's state: c' = -iK c for the wave decaying downward (Im K < 0)
        K = np.sqrt(gam[j] ** 2 + U0 + 0j)
        K = -K if K.imag > 0 else K
        assert Yb[j, j] == pytest.approx(1j * K, abs=1e-8)


def test_bulk_iteration_stops_at_the_tolerance_and_stays_converged():
    wl = small_2d(n_beams=21, n_slices=40, thickness=6.0, n_layers=2, n_angles=4)
    b = bulk_layer(dataclasses.replace(wl, theta0=wl.theta0[:1]), 31)
    st = driver.StructureSetup(b, b.structures[0], RK6)
    gam, _ = st.angle(float(b.theta0[0]))
    M = st.mfun(gam)
    tol = 1e-6
    Yb, Rb, n = bulk.bulk_reflection(M, gam, st.h, 31, RK6, tol=tol, max_layers=400)
    assert n > 1
    # one layer fewer is not converged; the last step is within tol
    Yp, Rp, m = bulk.bulk_reflection(M, gam, st.h, 31, RK6, tol=tol, max_layers=n - 1)
    assert m == -1
    assert np.abs(bulk.layer_map(M, gam, st.h, 31, RK6, Yp) - Yb).max() == 0.0
    assert np.abs(Rb - Rp).max() <= tol
    # 150 more layers keep contracting: the change per layer keeps falling
    # and R stays a bounded reflection matrix
    Y, R = Yb, Rb
    for _ in range(150):
        Y = bulk.layer_map(M, gam, st.h, 31, RK6, Y)
        Rn = bulk.reflection_of_state(Y, gam)
        last, R = np.abs(Rn - R).max(), Rn
    assert last < 0.1 * tol
    assert np.abs(R).max() < 1.0 + 1e-9


def test_tangent_with_a_fixed_bulk_matches_central_differences():
    wl = small_2d(n_beams=9, n_slices=30, thickness=4.0, n_layers=1, n_angles=1)
    st = driver.StructureSetup(wl, wl.structures[0], RK4)
    th = float(wl.theta0[0])
    gam, _ = st.angle(th)
    rng = np.random.default_rng(8)
    Y = 1j * np.diag(gam) + 0.5 * (rng.normal(size=(9, 9)) + 1j * rng.normal(size=(9, 9)))
    dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)

    def dU(i, r):
        return dt[RK4.node_index(i, r)][st.cidx]
    rho, drho = tangent.solve_ode_str_tangent(st.mfun(gam), dU, gam, st.h, 30, RK4, y_bottom=Y)
    base, _ = rk.solve_ode_str(st.mfun(gam), gam, st.h, 30, RK4, y_bottom=Y)
    assert np.abs(rho - base).max() < 1e-13
    eps = 1e-6
    rp = rk.solve_ode_str(st.mfun(gam, table=st.table + eps * dt), gam, st.h, 30, RK4, y_bottom=Y)[0]
    rm = rk.solve_ode_str(st.mfun(gam, table=st.table - eps * dt), gam, st.h, 30, RK4, y_bottom=Y)[0]
    fd = (rp - rm) / (2 * eps)
    assert np.abs(drho - fd).max() <= 1e-6 * np.abs(fd).max()


def test_unit_layer_table_is_periodic():
    """The bulk's unit layer (one atomic layer at its centre with two periodic
    images on each side) has the same coupling at its bottom and top faces,
    up to the Gaussian tails of the images left out."""
    from oracle import physics, potential
    wl = small_2d(n_beams=21, n_slices=40, thickness=6.0, n_layers=2, n_angles=1)
    b = bulk_layer(wl, 31)
    s = b.structures[0]
    kappa = physics.interaction_constant(b.energy_eV)
    z = np.array([-s.thickness, -0.5 * s.thickness, 0.0])
    t = potential.potential_table(s, z, kappa, b.charge, b.absorption, b.mean_inner_potential)
    assert np.abs(t[0] - t[2]).max() < 1e-12 * np.abs(t).max()
    # the layer at the centre dominates: the faces hold less than the middle
    assert np.abs(t[0]).max() < np.abs(t[1]).max()
    # and the mean inner potential (the g = 0 coefficient's mean over the layer)
    # equals the surface's value: the images' atoms are counted per spacing
    zz = np.linspace(-s.thickness, 0.0, 2001)
    hd, kd = potential.difference_box(s.beams)
    g0 = hd * (2 * kd + 1) + kd
    u0 = potential.potential_table(s, zz, kappa, b.charge, 0.0, b.mean_inner_potential)[:, g0].real
    mean = np.trapezoid(u0, zz) / s.thickness
    assert mean == pytest.approx(kappa * wl.mean_inner_potential, rel=1e-3)
