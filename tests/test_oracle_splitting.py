"""Pins of the oracle's splitting steppers (Sec. 3.4, BAB and ABA forms) against what
the mathematics fixes: the triple-jump conditions, the observed order under
step halving on a z-dependent potential, and exact flux conservation
without absorption at a step where the RK steppers visibly violate it."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import driver, rk
from oracle.splitting import SP4, SP4_ABA, SP6, SP6_ABA, VERLET
from oracle.tableaux import RK4
from synth import small_2d, small_row


def test_triple_jump_weights():
    g1, g2 = SP4.a[0], SP4.a[1]
    assert SP4.a[2] == g1
    assert 2 * g1 + g2 == pytest.approx(1.0, abs=1e-15)
    assert 2 * g1 ** 3 + g2 ** 3 == pytest.approx(0.0, abs=1e-14)    # cancels the third-order error of Verlet
    assert SP4.b.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(SP4.b, [g1 / 2, (g1 + g2) / 2, (g1 + g2) / 2, g1 / 2], atol=0)
    # kick positions: 0, g1, g1 + g2 inside the slice and 1 (the next slice's 0)
    assert np.allclose(SP4.tau, [0.0, g1, g1 + g2, 1.0], atol=1e-15)
    assert SP4.cset == pytest.approx([0.0, g1, g1 + g2])
    assert SP4.node_index(5, 0) == 15 and SP4.node_index(5, 2) == 17 and SP4.node_index(5, 3) == 18


def test_sixth_order_triple_jump_weights():
    """SP6: the triple jump of SP4 with outer weight w1 and inner w0,
    2 w1 + w0 = 1 and 2 w1^5 + w0^5 = 0 (cancels SP4's fifth-order error);
    its nine drifts are w_i times SP4's, its kicks their half sums."""
    w1 = SP6.a[0] / SP4.a[0]
    w0 = SP6.a[3] / SP4.a[0]
    assert 2 * w1 + w0 == pytest.approx(1.0, abs=1e-15)
    assert 2 * w1 ** 5 + w0 ** 5 == pytest.approx(0.0, abs=1e-14)
    assert np.allclose(SP6.a, np.concatenate([w1 * SP4.a, w0 * SP4.a, w1 * SP4.a]), atol=1e-15)
    assert SP6.b.size == 10 and SP6.b.sum() == pytest.approx(1.0, abs=1e-14)
    assert len(SP6.cset) == 9 and SP6.n_nodes(10) == 91


def test_aba_forms_swap_the_roles():
    """ABA: drifts at both ends of the slice, kick weights the Stormer-Verlet
    step lengths, drift weights their half sums; every kick inside the slice."""
    for aba, bab in ((SP4_ABA, SP4), (SP6_ABA, SP6)):
        assert np.allclose(aba.b, bab.a, atol=0) and np.allclose(aba.a, bab.b, atol=0)
        assert aba.a.size == aba.b.size + 1
        assert np.allclose(aba.tau, np.cumsum(aba.a)[:-1], atol=0)
        assert all(0.0 < t < 1.0 for t in aba.tau)
    assert SP4_ABA.tau[1] == pytest.approx(0.5, abs=1e-15)   # the middle kick of a symmetric method


ORDER_CASES = [(VERLET, (80, 160, 320), 5120), (SP4, (40, 80, 160), 2560), (SP4_ABA, (40, 80, 160), 2560),
               (SP6, (40, 80, 160), 2560), (SP6_ABA, (40, 80, 160), 2560)]


@pytest.mark.parametrize("comp,Ls,Lref", ORDER_CASES, ids=lambda c: getattr(c, "name", ""))
def test_splitting_order_on_z_dependent_potential(comp, Ls, Lref):
    """Error ratio under step halving -> 2^order; a kick evaluated at the
    wrong position (e.g. after its drift) or a wrong weight drops it."""
    base = small_row(hmax=2, n_slices=400, thickness=6.0, n_layers=2)
    base.structures[0].scat_b = np.array([0.5, 0.8, 1.1, 1.5])
    th = float(base.theta0[2])

    def run(L):
        s = dataclasses.replace(base.structures[0], n_slices=L)
        w = dataclasses.replace(base, structures=[s])
        return driver.StructureSetup(w, s, comp).solve(th)[0]
    ref = run(Lref)
    e = [np.abs(run(L) - ref).max() for L in Ls]
    r = e[1] / e[2]
    assert 2 ** comp.order * 0.8 < r < 2 ** comp.order * 1.25, e


def _flux(st, th):
    gam, mask = st.angle(th)
    rho, _, _, info = st.solve(th, track_transform=True)
    tau = rk.transmission(info["Z"], info["T"], gam)
    R = rk.intensity(rho, gam, mask, th)
    T = np.zeros_like(R)
    T[mask] = np.abs(tau[mask]) ** 2 * gam[0].real / gam[mask].real
    return R.sum() + T.sum()


@pytest.mark.parametrize("comp", [SP4, SP4_ABA, SP6, SP6_ABA], ids=lambda c: c.name)
def test_splitting_conserves_flux_exactly_without_absorption(comp):
    """Each kick and drift keeps Im(c^H c') for Hermitian M, so R + T = 1 to
    rounding even at a coarse step, where RK4 is off by far more."""
    wl = small_2d(n_beams=9, n_slices=20, thickness=4.0, n_layers=1, absorption=0.0, n_angles=3)
    s = wl.structures[0]
    st = driver.StructureSetup(wl, s, comp)
    st4 = driver.StructureSetup(wl, s, RK4)
    worst_rk = 0.0
    for th in wl.theta0:
        assert _flux(st, float(th)) == pytest.approx(1.0, abs=1e-12)
        worst_rk = max(worst_rk, abs(_flux(st4, float(th)) - 1.0))
    assert worst_rk > 1e-6


@pytest.mark.parametrize("name", ["sp4", "sp4a", "sp6"])
def test_splitting_tangent_matches_central_differences(name):
    """The splitting methods' tangent (kicks and drifts differentiated,
    through the right-hand-side transformations of a slab thick enough for
    several) against central differences of the oracle's own forward along
    a random complex direction of the potential table."""
    from oracle import driver, rk, tangent
    from oracle.tableaux import TABLEAUX
    from synth import small_2d
    wl = small_2d(n_beams=13, n_slices=40, thickness=4.0, n_layers=1, n_angles=2)
    tab = TABLEAUX[name]
    st = driver.StructureSetup(wl, wl.structures[0], tab)
    rng = np.random.default_rng(19)
    dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)
    th = float(wl.theta0[1])
    gam, _ = st.angle(th)

    def dU(i, r):
        return dt[tab.node_index(i, r)][st.cidx]
    rho, drho = tangent.solve_ode_str_tangent(st.mfun(gam), dU, gam, st.h, st.s.n_slices, tab)
    r0, info = rk.solve_ode_str(st.mfun(gam), gam, st.h, st.s.n_slices, tab)
    assert info["n_rhst"] >= 3
    assert np.allclose(rho, r0, rtol=0, atol=1e-14 * np.abs(r0).max())
    eps = 1e-6
    rp = rk.solve_ode_str(st.mfun(gam, table=st.table + eps * dt), gam, st.h, st.s.n_slices, tab)[0]
    rm = rk.solve_ode_str(st.mfun(gam, table=st.table - eps * dt), gam, st.h, st.s.n_slices, tab)[0]
    fd = (rp - rm) / (2 * eps)
    assert np.abs(drho - fd).max() <= 1e-6 * np.abs(fd).max()


def test_splitting_atom_tangent_matches_central_differences():
    """The R-factor's derivative along atom displacements with the
    fourth-order BAB method against central differences."""
    import copy
    from oracle import driver
    from synth import small_2d
    wl = small_2d(n_beams=9, n_slices=30, thickness=4.0, n_layers=1, n_angles=2)
    s = wl.structures[0]
    d = np.zeros_like(s.atoms)
    d[:4] = np.random.default_rng(5).normal(size=(4, 3))
    target = np.array([0.01, 0.02])
    loss, dl = driver.rfactor_directional(wl, 0, d, target, stepper="sp4")
    eps = 1e-5

    def loss_at(shift):
        w2 = copy.deepcopy(wl)
        w2.structures[0].atoms = s.atoms + shift * d
        eta = driver.rocking_curve(w2, stepper="sp4")[0][:, 0]
        return driver.rfactor(eta, target)[0]
    fd = (loss_at(eps) - loss_at(-eps)) / (2 * eps)
    assert loss == pytest.approx(loss_at(0.0), rel=1e-12)
    assert dl == pytest.approx(fd, rel=2e-6)
