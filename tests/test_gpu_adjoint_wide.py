"""Parity of the HIP adjoint for 64 < N <= 256 (states padded to 128 or 256
beams, kept by the kernels for N > 64, for N > 128 by one workgroup per
pair or by a group of them; the vector adjoint on 16 waves; the gradient
assembly binning C = G^T conj(V) in blocks) with the oracle's
tangent-linear derivatives, with central finite differences of the GPU
forward, and with the N <= 64 path inside one plan."""
import dataclasses

import numpy as np
import pytest

from oracle import driver
from synth import small_2d
from tests.gpu_util import assert_entrywise, oracle_atom_gradient

pytestmark = pytest.mark.gpu


def _target(n, seed=3):
    return np.random.default_rng(seed).uniform(0.0, 0.3, size=n)


def _run(wl, stepper, target, checkpoint_every=1, layout="auto"):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    print(f"[adjoint-wide] {[s.n_beams for s in wl.structures]} beams, {stepper}, K={checkpoint_every}", flush=True)
    plan = api.plan_for(wl, stepper=stepper, checkpoint_every=checkpoint_every, layout=layout)
    atoms = api.atoms_for(wl, dev)
    U = plan.potential(atoms)
    ang = api.angles_for(wl, dev)
    ws = plan.workspace(dev)
    out = plan.forward(U, ang, workspace=ws, want_nrhst=True)
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64)).to(dev)
    loss, dI = api.rfactor(out["intensity"], tgt)
    dU = plan.backward(U, ang, dI, ws)
    dA = plan.potential_backward(atoms, dU)
    torch.cuda.synchronize()
    res = {"loss": float(loss.item()), "dU": dU.cpu().numpy(), "datoms": dA.cpu().numpy(),
           "eta": out["intensity"].cpu().numpy(), "status": out["status"].cpu().numpy(),
           "table_offsets": plan.table_offsets.copy(), "atom_offsets": plan.atom_offsets.copy(),
           "large_pairs": plan.info.large_pairs, "xl_group": plan.info.xl_group,
           "n_rhst": out["n_rhst"].cpu().numpy()}
    del ws, plan
    return res


def _loss_only(wl, stepper, target, atoms_np):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper=stepper)
    U = plan.potential(torch.from_numpy(atoms_np).to(dev))
    out = plan.forward(U, api.angles_for(wl, dev))
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64)).to(dev)
    loss, _ = api.rfactor(out["intensity"], tgt)
    return float(loss.item())


@pytest.mark.parametrize("every", [1, 7])
@pytest.mark.parametrize("stepper,n_beams", [("rk4", 65), ("rk6", 91), ("rk6", 128), ("rk4", 150), ("rk6", 199),
                                             ("rk6", 256)])
def test_wide_table_gradient_matches_oracle_tangent(stepper, n_beams, every):
    """The table gradient along random directions against the oracle's
    tangent-linear derivative, with states kept at every slice and every 7
    (a partial top segment), at N = 65, 91, 128 (states padded to 128) and
    150, 199, 256 (padded to 256)."""
    L = 24 if stepper == "rk6" else 40
    wl = small_2d(n_beams=n_beams, n_slices=L, thickness=0.1 * L, n_layers=1, n_angles=3)
    tgt = _target(3)
    res = _run(wl, stepper, tgt, checkpoint_every=every)
    assert (res["status"] == 0).all()
    st = driver.StructureSetup(wl, wl.structures[0], driver.TABLEAUX[stepper])
    rng = np.random.default_rng(11)
    for _ in range(2):
        dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)
        loss, dl = driver.rfactor_directional_table(wl, 0, dt, tgt, stepper=stepper)
        got = float(np.real(np.sum(np.conj(res["dU"]) * dt.ravel())))
        print(f"[adjoint-wide] N={n_beams} {stepper} K={every} table direction: gpu {got:.12e} oracle {dl:.12e}",
              flush=True)
        assert res["loss"] == pytest.approx(loss, rel=1e-10)
        assert got == pytest.approx(dl, rel=1e-9)


@pytest.mark.parametrize("n_beams,every", [(91, 1), (91, 20), (170, 1), (170, 20)])
def test_wide_atom_gradient_every_coordinate(n_beams, every):
    """Every coordinate of the 9 atoms of an N = 91 or 170 slab (RK6, 40
    slices) against the oracle's tangent-linear derivative along that
    coordinate, entry by entry (1e-8 relative to the entry, or to 1e-6 of
    the largest)."""
    wl = small_2d(n_beams=n_beams, n_slices=40, thickness=4.0, n_layers=1, n_angles=3)
    tgt = _target(3, seed=13)
    res = _run(wl, "rk6", tgt, checkpoint_every=every)
    assert (res["status"] == 0).all()
    n_atoms = wl.structures[0].atoms.shape[0]
    coords = [(ia, c) for ia in range(n_atoms) for c in range(3)]
    ref = oracle_atom_gradient(wl, tgt, coords, stepper="rk6")
    got = np.array([res["datoms"][ia, c] for ia, c in coords])
    assert_entrywise(got, ref, what=f"N={n_beams} slab K={every}, all {len(coords)} coordinates")


def test_wide_atom_gradient_against_central_differences():
    """Two atom coordinates of an N = 121 slab against central differences
    (h = 1e-5 A) of the GPU forward."""
    wl = small_2d(n_beams=121, n_slices=30, thickness=3.0, n_layers=2, n_angles=3)
    tgt = _target(3, seed=5)
    res = _run(wl, "rk6", tgt, checkpoint_every=10)
    assert (res["status"] == 0).all()
    g = res["datoms"]
    s = wl.structures[0]
    for (ia, c) in [(0, 2), (10, 0)]:
        e = np.zeros_like(s.atoms)
        e[ia, c] = 1e-5
        fd = (_loss_only(wl, "rk6", tgt, s.atoms + e) - _loss_only(wl, "rk6", tgt, s.atoms - e)) / 2e-5
        print(f"[adjoint-wide] N=121 fd atom {ia} coord {c}: gpu {g[ia, c]:.10e} fd {fd:.10e}", flush=True)
        assert g[ia, c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max())


@pytest.mark.parametrize("stepper,n_beams", [("rk4", 91), ("rk6", 91), ("rk6", 199)])
def test_wide_checkpoint_segments_match_every_slice_states(stepper, n_beams):
    """States every 20 slices give the every-slice adjoint's table gradient
    to rounding (50 slices: a partial top segment)."""
    wl = small_2d(n_beams=n_beams, n_slices=50, thickness=5.0, n_layers=1, n_angles=3)
    tgt = _target(3, seed=6)
    ref = _run(wl, stepper, tgt, checkpoint_every=1)
    got = _run(wl, stepper, tgt, checkpoint_every=20)
    assert (ref["status"] == 0).all()
    err = np.abs(got["dU"] - ref["dU"]).max() / np.abs(ref["dU"]).max()
    print(f"[adjoint-wide] N={n_beams} {stepper} K=20 vs K=1: {err:.3e}", flush=True)
    np.testing.assert_allclose(got["dU"], ref["dU"], rtol=0.0, atol=1e-13 * np.abs(ref["dU"]).max())


@pytest.mark.parametrize("layout", ["whole", "split"])
def test_mixed_plan_gradient_equals_separate_plans(layout):
    """A plan with N = 29, 91 and 150 structures (three backward launches,
    the three state layouts in one workspace) gives each structure the table
    and atom gradient of a plan holding that structure alone."""
    a = small_2d(n_beams=29, n_slices=30, thickness=3.0, n_layers=1, n_angles=3, seed=41)
    b = small_2d(n_beams=91, n_slices=24, thickness=2.4, n_layers=1, n_angles=3, seed=42)
    c = small_2d(n_beams=150, n_slices=16, thickness=1.6, n_layers=1, n_angles=3, seed=43)
    wl = dataclasses.replace(a, structures=[a.structures[0], b.structures[0], c.structures[0]])
    tgt = _target(9, seed=8)
    both = _run(wl, "rk6", tgt, checkpoint_every=7, layout=layout)
    assert (both["status"] == 0).all()
    for s, part in enumerate((a, b, c)):
        alone = _run(part, "rk6", tgt[3 * s:3 * s + 3], checkpoint_every=7, layout=layout)
        t0, t1 = both["table_offsets"][s], both["table_offsets"][s + 1]
        a0, a1 = both["atom_offsets"][s], both["atom_offsets"][s + 1]
        du = both["dU"][t0:t1]
        print(f"[adjoint-wide] mixed plan structure {s}: max |dU - alone| = "
              f"{np.abs(du - alone['dU']).max():.3e} of {np.abs(alone['dU']).max():.3e}", flush=True)
        np.testing.assert_allclose(du, alone["dU"], rtol=0.0, atol=1e-14 * np.abs(alone["dU"]).max())
        np.testing.assert_allclose(both["datoms"][a0:a1], alone["datoms"], rtol=1e-12,
                                   atol=1e-14 * np.abs(alone["datoms"]).max())


@pytest.mark.parametrize("stepper,n_beams,every", [("rk6", 150, 1), ("rk4", 199, 7), ("rk6", 256, 7)])
def test_group_and_one_workgroup_gradients_agree(stepper, n_beams, every):
    """For N > 128 the forward on a group of workgroups per pair (each
    copying the column blocks it steps into the kept states, and a share of
    the row blocks of T and R) keeps what the one-workgroup launch keeps:
    the same transformation counts and the same table and atom gradients."""
    L = 24 if stepper == "rk6" else 40
    wl = small_2d(n_beams=n_beams, n_slices=L, thickness=0.1 * L, n_layers=2, n_angles=3, seed=17)
    tgt = _target(3, seed=21)
    grp = _run(wl, stepper, tgt, checkpoint_every=every, layout="auto")
    one = _run(wl, stepper, tgt, checkpoint_every=every, layout="whole")
    assert grp["xl_group"] == (n_beams + 15) // 16 and one["xl_group"] == 1
    assert (grp["status"] == 0).all() and (one["status"] == 0).all()
    assert grp["n_rhst"].tolist() == one["n_rhst"].tolist()
    assert grp["loss"] == pytest.approx(one["loss"], rel=1e-13)
    du = np.abs(grp["dU"] - one["dU"]).max() / np.abs(one["dU"]).max()
    da = np.abs(grp["datoms"] - one["datoms"]).max() / np.abs(one["datoms"]).max()
    print(f"[adjoint-wide] N={n_beams} {stepper} K={every} group of {grp['xl_group']} vs one workgroup: "
          f"dU {du:.3e}, datoms {da:.3e}", flush=True)
    assert du <= 1e-12 and da <= 1e-12


def test_wide_gradient_full_size_n121():
    """An N = 121 structure of the uneven-N workload at full size (40 A in
    600 slices, RK6, states every 20 slices) at three angles: every pair
    through the validity gate, and the atom gradient along a random
    direction of all 90 atoms against the oracle's tangent-linear
    derivative."""
    from synth import config3
    from tests.gpu_util import physical
    wl = config3(16)
    s = next(i for i, st in enumerate(wl.structures) if st.n_beams == 121)
    idx = [5, 30, 60]
    sub = dataclasses.replace(wl, structures=[wl.structures[s]], theta0=wl.theta0[idx])
    assert sub.structures[0].n_slices == 600
    tgt = _target(3, seed=19)
    res = _run(sub, "rk6", tgt, checkpoint_every=20)
    assert (res["status"] == 0).all()
    assert physical(res["eta"][:, :121], sub.absorption).all()
    atoms = sub.structures[0].atoms
    d = np.random.default_rng(23).normal(size=atoms.shape)
    loss, dl = driver.rfactor_directional(sub, 0, d, tgt, stepper="rk6")
    got = float(np.sum(res["datoms"] * d))
    print(f"[adjoint-wide] N=121 full size (3 angles) direction: gpu {got:.12e} oracle {dl:.12e}", flush=True)
    assert res["loss"] == pytest.approx(loss, rel=1e-10)
    assert got == pytest.approx(dl, rel=1e-8)


def test_n199_gradient_full_size_one_angle():
    """The N = 199 slab of the large workload at full size (60 A in 1000
    slices, RK6, states every 20 slices) at one angle: the pair through the
    validity gate and the atom gradient along a random direction of all its
    atoms against the oracle's tangent-linear derivative."""
    from synth import config5
    from tests.gpu_util import physical
    wl = config5(1)
    sub = dataclasses.replace(wl, theta0=wl.theta0[[120]])
    tgt = _target(1, seed=29)
    res = _run(sub, "rk6", tgt, checkpoint_every=20)
    assert (res["status"] == 0).all()
    assert physical(res["eta"][:, :199], sub.absorption).all()
    atoms = sub.structures[0].atoms
    d = np.random.default_rng(31).normal(size=atoms.shape)
    loss, dl = driver.rfactor_directional(sub, 0, d, tgt, stepper="rk6")
    got = float(np.sum(res["datoms"] * d))
    print(f"[adjoint-wide] N=199 full size (one angle) direction: gpu {got:.12e} oracle {dl:.12e}", flush=True)
    assert res["loss"] == pytest.approx(loss, rel=1e-10)
    assert got == pytest.approx(dl, rel=1e-8)
