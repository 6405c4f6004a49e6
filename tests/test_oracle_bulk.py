"""Pins for the oracle's bulk layer (oracle/bulk.py): composition of a slab
from its parts, the single-beam closed form after k unit layers and its
Fresnel limit, decoupled beams, and the fixed point (CPU only)."""
import numpy as np
import pytest

from oracle import bulk, closed_form, driver, rk, tangent
from oracle.tableaux import RK4, RK6
from synth import bulk_layer, small_2d


def _const(M):
    return lambda i, r: M


def test_initial_state_of_a_zero_bulk_is_the_vacuum_state():
    gam = np.array([0.7, 2.0, -3.0j])
    z0 = rk.initial_state(gam)
    assert np.abs(rk.initial_state(gam, r_bottom=np.zeros((3, 3))) - z0).max() < 1e-15
    # the bottom condition holds: S Z0 = [tau; rho] with rho = R tau
    rng = np.random.default_rng(3)
    R = 0.3 * (rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
    tr = rk.boundary_matrix(gam) @ rk.initial_state(gam, r_bottom=R)
    assert np.abs(tr[3:] - R @ tr[:3]).max() < 1e-14
    assert np.abs(tr[:3] - np.diag(2 * gam)).max() < 1e-14


@pytest.mark.parametrize("tab", [RK4, RK6])
def test_slab_equals_its_upper_part_on_the_lower_parts_reflection(tab):
    """Sec. 2.2: rho(0) of a slab from rho(z_e) = 0 equals that of its upper
    part started from the top reflection matrix of its lower part."""
    wl = small_2d(n_beams=13, n_slices=40, thickness=6.0, n_layers=2, n_angles=2)
    st = driver.StructureSetup(wl, wl.structures[0], tab)
    L1 = 23
    for th in wl.theta0:
        gam, _ = st.angle(float(th))
        M = st.mfun(gam)
        whole, _ = rk.solve_ode_str(M, gam, st.h, 40, tab)
        _, info = rk.solve_ode_str(M, gam, st.h, L1, tab)
        Rmid = rk.reflection_matrix(info["Z"], gam)
        upper, _ = rk.solve_ode_str(lambda i, r: M(i + L1, r), gam, st.h, 40 - L1, tab, r_bottom=Rmid)
        scale = np.abs(whole).max()
        assert np.abs(upper - whole).max() <= 1e-11 * scale
        # a transposed or unscaled bottom matrix breaks it
        for wrong in (Rmid.T, Rmid * (gam[None, :] / gam[:, None])):
            bad, _ = rk.solve_ode_str(lambda i, r: M(i + L1, r), gam, st.h, 40 - L1, tab, r_bottom=wrong)
            assert np.abs(bad - whole).max() > 1e-6 * scale


@pytest.mark.parametrize("U0", [4.0 - 0.3j, -4.0 - 0.3j])
def test_layers_of_a_constant_potential_follow_the_closed_form(U0):
    """k unit layers of a constant coupling are one slab of thickness k d:
    R_k is the closed-form single-beam reflection, and the limit is the
    Fresnel value of the half space."""
    gam = np.array([1.1 + 0j])
    M = np.array([[U0 + gam[0] ** 2]])
    d, L = 3.1, 124
    R = np.zeros((1, 1), complex)
    for k in range(1, 7):
        R, _ = bulk.layer_map(_const(M), gam, d / L, L, RK6, R)
        assert R[0, 0] == pytest.approx(closed_form.slab_rt(gam[0], U0, k * d)[0], abs=1e-10)
    Rb, n = bulk.bulk_reflection(_const(M), gam, d / L, L, RK6, tol=1e-12, max_layers=400)
    assert n > 0
    assert Rb[0, 0] == pytest.approx(closed_form.fresnel_r(gam[0], U0), abs=1e-9)


def test_decoupled_beams_have_a_diagonal_bulk_matrix():
    gam = np.array([0.9, 2.0, 1.3])
    U0 = 3.0 - 0.4j
    M = np.diag(U0 + gam ** 2)
    d, L = 3.1, 124
    Rb, n = bulk.bulk_reflection(_const(M), gam, d / L, L, RK6, tol=1e-12, max_layers=400)
    assert n > 0
    assert np.abs(Rb - np.diag(np.diag(Rb))).max() < 1e-14
    for j in range(3):
        assert Rb[j, j] == pytest.approx(closed_form.fresnel_r(gam[j], U0), abs=1e-9)


def test_bulk_matrix_is_a_fixed_point_and_stops_at_the_tolerance():
    wl = small_2d(n_beams=9, n_slices=30, thickness=4.0, n_layers=1, n_angles=1)
    b = bulk_layer(wl, 31)
    st = driver.StructureSetup(b, b.structures[0], RK4)
    gam, _ = st.angle(float(b.theta0[0]))
    M = st.mfun(gam)
    tol = 1e-6
    Rb, n = bulk.bulk_reflection(M, gam, st.h, 31, RK4, tol=tol, max_layers=300)
    assert n > 1
    # the previous layer's matrix was farther than tol, the last step within it
    prev, m = bulk.bulk_reflection(M, gam, st.h, 31, RK4, tol=tol, max_layers=n - 1)
    assert m == -1
    Fb, _ = bulk.layer_map(M, gam, st.h, 31, RK4, prev)
    assert np.abs(Fb - Rb).max() == 0.0
    assert np.abs(Rb - prev).max() <= tol < np.abs(prev - bulk.bulk_reflection(M, gam, st.h, 31, RK4, tol=tol,
                                                                                  max_layers=n - 2)[0]).max()
    # the limit is a fixed point of the layer map (contraction: the next step is smaller)
    F2, _ = bulk.layer_map(M, gam, st.h, 31, RK4, Rb)
    assert np.abs(F2 - Rb).max() < tol


def test_tangent_with_a_fixed_bulk_matches_central_differences():
    wl = small_2d(n_beams=9, n_slices=30, thickness=4.0, n_layers=1, n_angles=1)
    st = driver.StructureSetup(wl, wl.structures[0], RK4)
    th = float(wl.theta0[0])
    gam, _ = st.angle(th)
    rng = np.random.default_rng(8)
    R = 0.4 * (rng.normal(size=(9, 9)) + 1j * rng.normal(size=(9, 9))) / 3
    dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)

    def dU(i, r):
        return dt[RK4.node_index(i, r)][st.cidx]
    rho, drho = tangent.solve_ode_str_tangent(st.mfun(gam), dU, gam, st.h, 30, RK4, r_bottom=R)
    base, _ = rk.solve_ode_str(st.mfun(gam), gam, st.h, 30, RK4, r_bottom=R)
    assert np.abs(rho - base).max() < 1e-13
    eps = 1e-6
    rp = rk.solve_ode_str(st.mfun(gam, table=st.table + eps * dt), gam, st.h, 30, RK4, r_bottom=R)[0]
    rm = rk.solve_ode_str(st.mfun(gam, table=st.table - eps * dt), gam, st.h, 30, RK4, r_bottom=R)[0]
    fd = (rp - rm) / (2 * eps)
    assert np.abs(drho - fd).max() <= 1e-6 * np.abs(fd).max()
