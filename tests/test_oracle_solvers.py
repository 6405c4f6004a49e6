"""Pins for the oracle's solvers: closed form, conventional vs proposed
method, convergence order, flux, absorption, RHST invariance, symmetry,
brute force, tangent-linear gradient (CPU only)."""
import copy
import dataclasses
import math

import numpy as np
import pytest

from oracle import closed_form, conventional, driver, physics, potential, rk, tangent
from oracle.tableaux import RK4, RK6
from synth import small_2d, small_row, config1


def _const_fun(M):
    return lambda *args: M


# ------------------------------------------------------- single-beam slab
def test_closed_form_identities():
    # flux R + T = 1 for a real coupling, limits U0 -> 0 and D -> infinity
    for gam, U0, D in [(0.9, 4.0, 7.3), (2.5, -3.0, 4.1), (0.3, -1.0, 12.0)]:
        r, t = closed_form.slab_rt(gam, U0, D)
        assert abs(r) ** 2 + abs(t) ** 2 == pytest.approx(1.0, abs=1e-13)
        r0, t0 = closed_form.slab_rt(gam, 1e-14, D)
        assert abs(r0) < 1e-13 and t0 == pytest.approx(np.exp(-1j * gam * D), abs=1e-12)
    rr, _ = closed_form.slab_rt(1.2, 3.0 - 0.4j, 400.0)
    assert rr == pytest.approx(closed_form.fresnel_r(1.2, 3.0 - 0.4j), abs=1e-12)
    # positron below the critical angle: total reflection of a thick slab
    r, t = closed_form.slab_rt(0.8, -4.0, 40.0)
    assert abs(r) == pytest.approx(1.0, abs=1e-12) and abs(t) < 1e-20


@pytest.mark.parametrize("U0", [4.0 - 0.3j, -4.0 - 0.3j, 2.0])
def test_solvers_reproduce_single_beam_slab(U0):
    gam = np.array([1.1 + 0j])
    D = 6.0
    M = np.array([[U0 + gam[0] ** 2]])
    r_ref, t_ref = closed_form.slab_rt(gam[0], U0, D)
    # conventional methods are exact for a constant coupling at any L
    for L in (1, 7, 40):
        h = D / L
        assert conventional.eigen_multislice(_const_fun(M), gam, h, L)[0] == pytest.approx(r_ref, abs=1e-12)
        assert conventional.ichimiya_recursion(_const_fun(np.array([[U0]])), gam, h, L)[0] == pytest.approx(r_ref, abs=1e-12)
    # RK converges at its order: error ratio under step halving -> 2^p
    for tab in (RK4, RK6):
        errs, terrs = [], []
        Ls = [8 * 2 ** k for k in range(6)]
        for L in Ls:
            rho, info = rk.solve_ode_str(_const_fun(M), gam, D / L, L, tab, track_transform=True)
            errs.append(abs(rho[0] - r_ref))
            terrs.append(abs(rk.transmission(info["Z"], info["T"], gam)[0] - t_ref))
        for e in (errs, terrs):
            # last halving still well above roundoff
            k = max(i for i in range(len(e) - 1) if e[i + 1] > 2e-13)
            ratio = e[k] / e[k + 1]
            # at least order p (exactly p is pinned by the order conditions)
            assert ratio > 2 ** tab.order * 0.85, (tab.name, e)


# --------------------------------------------------------- multi-beam
def _setup(wl, tab=RK4):
    return driver.StructureSetup(wl, wl.structures[0], tab)


def test_eigen_equals_ichimiya_and_global_product():
    wl = small_2d(n_beams=5, n_slices=12, thickness=2.0, n_layers=1, n_angles=3)
    st = _setup(wl)
    for th in wl.theta0:
        rho_e, gam, _ = st.solve_eigen(float(th))
        rho_i, _, _ = st.solve_ichimiya(float(th))
        assert np.abs(rho_e - rho_i).max() < 1e-12 * max(1.0, np.abs(rho_e).max())
        cs = [float(c) for c in st.tab.cset]
        m = cs.index(0.5)
        rho_g = conventional.global_product(lambda i: st.U_node(i * len(cs) + m), gam, st.h, st.s.n_slices)
        assert np.abs(rho_g - rho_i).max() < 1e-9 * max(1.0, np.abs(rho_i).max())


def test_eigen_is_exact_for_piecewise_constant_coupling():
    wl = small_2d(n_beams=9, n_slices=8, thickness=3.0, n_layers=1)
    st = _setup(wl)
    gam, _ = st.angle(float(wl.theta0[1]))
    U = st.U_node(5)
    M = U + np.diag(gam ** 2)
    # (a single 3 A slice loses digits to exp(3 |Gamma|) of the evanescent beams)
    rhos = [conventional.eigen_multislice(_const_fun(M), gam, 3.0 / L, L) for L in (10, 3, 29)]
    for r in rhos[1:]:
        assert np.abs(r - rhos[0]).max() < 1e-12 * np.abs(rhos[0]).max()
    # RK on the same constant coupling converges to it at order 4
    e = [np.abs(rk.solve_ode_str(_const_fun(M), gam, 3.0 / L, L, RK4)[0] - rhos[0]).max() for L in (60, 120, 240)]
    assert 13 < e[1] / e[2] < 19


@pytest.mark.parametrize("tab", [RK4, RK6], ids=lambda t: t.name)
def test_rk_order_on_z_dependent_potential(tab):
    base = small_row(hmax=2, n_slices=400, thickness=6.0, n_layers=2)
    base.structures[0].scat_b = np.array([0.5, 0.8, 1.1, 1.5])   # smooth enough for the asymptotic regime
    th = float(base.theta0[2])

    def run(L):
        s = dataclasses.replace(base.structures[0], n_slices=L)
        w = dataclasses.replace(base, structures=[s])
        return driver.StructureSetup(w, s, tab).solve(th)[0]
    ref = run(1920 if tab is RK4 else 640)
    e = [np.abs(run(L) - ref).max() for L in (30, 60, 120)]
    r = e[1] / e[2]
    assert 2 ** tab.order * 0.8 < r < 2 ** tab.order * 1.25, e


def test_rk_and_eigen_converge_to_the_same_solution():
    """Two different discretisations (order 6 RK with node sampling, order 2
    midpoint exponential) share their continuum limit; Richardson on the
    order-2 pair removes its leading error."""
    wl = small_row(hmax=2, n_slices=300, thickness=6.0, n_layers=2)
    wl.structures[0].scat_b = np.array([0.5, 0.8, 1.1, 1.5])
    th = float(wl.theta0[1])
    rk6 = driver.StructureSetup(wl, wl.structures[0], RK6).solve(th)[0]
    eig = []
    for L in (300, 600):
        s = dataclasses.replace(wl.structures[0], n_slices=L)
        w = dataclasses.replace(wl, structures=[s])
        eig.append(_setup(w).solve_eigen(th)[0])
    rich = (4 * eig[1] - eig[0]) / 3
    assert np.abs(eig[1] - rk6).max() > 1e-6          # the raw order-2 error is visible
    assert np.abs(rich - rk6).max() < 1e-8


def _flux(st, th, tab_solver="rk"):
    gam, mask = st.angle(th)
    if tab_solver == "rk":
        rho, _, _, info = st.solve(th, track_transform=True)
        tau = rk.transmission(info["Z"], info["T"], gam)
    R = rk.intensity(rho, gam, mask, th)
    T = np.zeros_like(R)
    T[mask] = np.abs(tau[mask]) ** 2 * gam[0].real / gam[mask].real
    return R, T


def test_flux_conservation_without_absorption():
    wl = small_2d(n_beams=9, n_slices=300, thickness=4.0, n_layers=1, absorption=0.0, n_angles=3)
    wl.structures[0].scat_b = np.array([0.5, 0.8, 1.1, 1.5])
    st = driver.StructureSetup(wl, wl.structures[0], RK6)
    for th in wl.theta0:
        R, T = _flux(st, float(th))
        assert R.sum() + T.sum() == pytest.approx(1.0, abs=1e-9)


def test_absorption_removes_flux_and_bounds_intensity():
    wl = small_2d(n_beams=9, n_slices=200, thickness=4.0, n_layers=1, absorption=0.1, n_angles=4)
    st = driver.StructureSetup(wl, wl.structures[0], RK6)
    for th in wl.theta0:
        R, T = _flux(st, float(th))
        assert R.sum() + T.sum() < 1.0 - 1e-6
        assert np.all(R >= 0) and np.all(R <= 1)


def test_rhst_invariance_and_initial_state_reading():
    wl = small_2d(n_beams=13, n_slices=40, thickness=3.0, n_layers=1, n_angles=2)
    st = driver.StructureSetup(wl, wl.structures[0], RK6)
    th = float(wl.theta0[1])
    ref, _, _, info = st.solve(th)
    assert info["n_rhst"] > 0
    for thr in (0.0, 10.0, 1e30):
        rho, _, _, _ = st.solve(th, threshold=thr)
        assert np.abs(rho - ref).max() < 1e-12 * np.abs(ref).max() + 1e-14
    lit, _, _, _ = st.solve(th, literal_z0=True)
    assert np.abs(lit - ref).max() < 1e-12 * np.abs(ref).max() + 1e-14


def test_decoupled_beams_reduce_to_closed_form():
    gam = np.array([0.9, 2.0, -3.0j, 1.3])
    U0 = 3.0 - 0.2j
    M = np.diag(U0 + gam ** 2)
    D, L = 5.0, 50
    rho = conventional.eigen_multislice(_const_fun(M), gam, D / L, L)
    assert rho[0] == pytest.approx(closed_form.slab_rt(gam[0], U0, D)[0], abs=1e-12)
    assert np.abs(rho[1:]).max() < 1e-14
    rho_rk, _ = rk.solve_ode_str(_const_fun(M), gam, D / 400, 400, RK6)
    assert rho_rk[0] == pytest.approx(rho[0], abs=1e-9)
    assert np.abs(rho_rk[1:]).max() < 1e-14


def test_mirror_symmetry_of_the_row_workload():
    wl = config1()
    wl.structures[0].n_slices = 120
    wl.structures[0].thickness = 12.0
    st = driver.StructureSetup(wl, wl.structures[0], RK4)
    b = wl.structures[0].beams
    th = float(wl.theta0[7])
    rho, gam, mask, _ = st.solve(th)
    eta = rk.intensity(rho, gam, mask, th)
    for j in range(1, b.shape[0]):
        jm = [k for k in range(b.shape[0]) if b[k, 0] == -b[j, 0]][0]
        assert eta[j] == pytest.approx(eta[jm], rel=1e-11, abs=1e-16)


# -------------------------------------------------------- gradient
def test_tangent_linear_matches_central_differences():
    wl = small_2d(n_beams=9, n_slices=30, thickness=4.0, n_layers=1, n_angles=2)
    s = wl.structures[0]
    rng = np.random.default_rng(5)
    d = np.zeros_like(s.atoms)
    d[:4] = rng.normal(size=(4, 3))
    target = np.array([0.01, 0.02])
    loss, dl = driver.rfactor_directional(wl, 0, d, target, stepper="rk6")
    eps = 1e-5

    def loss_at(shift):
        w2 = copy.deepcopy(wl)
        w2.structures[0].atoms = s.atoms + shift * d
        eta = driver.rocking_curve(w2, stepper="rk6")[0][:, 0]
        return driver.rfactor(eta, target)[0]
    fd = (loss_at(eps) - loss_at(-eps)) / (2 * eps)
    assert loss == pytest.approx(loss_at(0.0), rel=1e-12)
    assert dl == pytest.approx(fd, rel=2e-6)


def test_tangent_along_a_table_direction_on_a_thick_slab():
    """Tangent vs central differences along a random complex perturbation of
    the potential table, over a slab thick enough for many right-hand-side
    transformations (the tangent must differentiate Q^{-1} too, or it grows
    along the dominant modes and cancels catastrophically)."""
    from oracle.tableaux import TABLEAUX
    wl = small_2d(n_beams=21, n_slices=80, thickness=4.0, n_layers=1, n_angles=3)
    tab = TABLEAUX["rk4"]
    st = driver.StructureSetup(wl, wl.structures[0], tab)
    rng = np.random.default_rng(11)
    dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)
    th = float(wl.theta0[0])
    gam, mask = st.angle(th)

    def dU(i, r):
        return dt[tab.node_index(i, r)][st.cidx]
    rho, drho, = tangent.solve_ode_str_tangent(st.mfun(gam), dU, gam, st.h, st.s.n_slices, tab)
    eps = 1e-6
    rp = rk.solve_ode_str(st.mfun(gam, table=st.table + eps * dt), gam, st.h, st.s.n_slices, tab)[0]
    rm = rk.solve_ode_str(st.mfun(gam, table=st.table - eps * dt), gam, st.h, st.s.n_slices, tab)[0]
    fd = (rp - rm) / (2 * eps)
    assert np.abs(drho - fd).max() <= 1e-6 * np.abs(fd).max()
