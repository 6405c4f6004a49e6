"""Parity of the HIP adjoint (through the C ABI) with the oracle's
tangent-linear derivatives and with central finite differences."""
import dataclasses

import numpy as np
import pytest

from oracle import driver
from synth import config4, small_2d, small_row

pytestmark = pytest.mark.gpu


def _run(wl, stepper, target, convention="flux", checkpoint_every=1):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    plan = api.plan_for(wl, stepper=stepper, convention=convention, checkpoint_every=checkpoint_every)
    atoms = api.atoms_for(wl, dev)
    U = plan.potential(atoms)
    ang = api.angles_for(wl, dev)
    ws = plan.workspace(dev)
    out = plan.forward(U, ang, workspace=ws)
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64)).to(dev)
    loss, dI = api.rfactor(out["intensity"], tgt)
    dU = plan.backward(U, ang, dI, ws)
    dA = plan.potential_backward(atoms, dU)
    torch.cuda.synchronize()
    return {"loss": float(loss.item()), "dU": dU.cpu().numpy(), "datoms": dA.cpu().numpy(),
            "eta": out["intensity"].cpu().numpy(), "status": out["status"].cpu().numpy(), "plan": plan}


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


def _target(n, seed=3):
    return np.random.default_rng(seed).uniform(0.0, 0.3, size=n)


@pytest.mark.parametrize("every", [1, 20])
@pytest.mark.parametrize("stepper", ["rk4", "rk6"])
def test_table_gradient_matches_oracle_tangent(stepper, every):
    """Table gradient along random directions against the oracle's
    tangent-linear derivative, with a stored state at every slice and every
    20 slices."""
    wl = small_2d(n_beams=21, n_slices=40 if stepper == "rk6" else 80, thickness=4.0, n_layers=1, n_angles=3)
    tgt = _target(3)
    res = _run(wl, stepper, tgt, checkpoint_every=every)
    assert (res["status"] == 0).all()
    ub = res["dU"]
    rng = np.random.default_rng(11)
    st = driver.StructureSetup(wl, wl.structures[0], driver.TABLEAUX[stepper])
    for _ in range(2):
        dt = rng.normal(size=st.table.shape) + 1j * rng.normal(size=st.table.shape)
        loss, dl = driver.rfactor_directional_table(wl, 0, dt, tgt, stepper=stepper)
        got = float(np.real(np.sum(np.conj(ub) * dt.ravel())))
        print(f"[adjoint] {stepper} every {every} table direction: gpu {got:.12e} oracle {dl:.12e}", flush=True)
        assert res["loss"] == pytest.approx(loss, rel=1e-10)
        assert got == pytest.approx(dl, rel=1e-9, abs=1e-14 * abs(dl) + 1e-300)


@pytest.mark.parametrize("case", ["2d-rk6", "row-rk4-paper"])
def test_atom_gradient_matches_oracle_and_fd(case):
    if case == "2d-rk6":
        wl, stepper, conv = small_2d(n_beams=29, n_slices=40, thickness=4.0, n_layers=2, n_angles=3), "rk6", "flux"
    else:
        wl, stepper, conv = small_row(hmax=4, n_slices=80, thickness=8.0, n_layers=2, n_angles=3), "rk4", "paper"
    tgt = _target(len(wl.theta0), seed=5)
    res = _run(wl, stepper, tgt, convention=conv)
    g = res["datoms"]
    s = wl.structures[0]
    rng = np.random.default_rng(7)
    d = np.zeros_like(s.atoms)
    d[s.grad_atoms] = rng.normal(size=(len(s.grad_atoms), 3))
    loss, dl = driver.rfactor_directional(wl, 0, d, tgt, stepper=stepper, convention=conv)
    got = float(np.sum(g * d))
    print(f"[adjoint] {case} atom direction: gpu {got:.12e} oracle {dl:.12e}", flush=True)
    assert got == pytest.approx(dl, rel=1e-8)
    if conv == "flux":
        # central differences of the GPU forward, h = 1e-5 A
        for (ia, c) in [(0, 2), (1, 0)]:
            e = np.zeros_like(s.atoms)
            e[ia, c] = 1e-5
            fd = (_loss_only(wl, stepper, tgt, s.atoms + e) - _loss_only(wl, stepper, tgt, s.atoms - e)) / 2e-5
            print(f"[adjoint] fd atom {ia} coord {c}: gpu grad {g[ia, c]:.10e} fd {fd:.10e}", flush=True)
            assert g[ia, c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max())


def test_rfactor_kernel():
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1)
    I = torch.from_numpy(rng.uniform(size=(37, 5))).to(dev)
    t = torch.from_numpy(rng.uniform(size=37)).to(dev)
    loss, dI = api.rfactor(I, t)
    In, tn = I.cpu().numpy(), t.cpu().numpy()
    assert loss.item() == pytest.approx(np.sum((In[:, 0] - tn) ** 2), rel=1e-14)
    ref = np.zeros_like(In)
    ref[:, 0] = 2 * (In[:, 0] - tn)
    assert np.array_equal(dI.cpu().numpy(), ref)


def test_gradient_workload_full_size():
    """N=61, 400 slices, RK6, 128 angles, states kept every 20 slices as the
    workload states: the gradient w.r.t. atom coordinates against central
    differences of the same GPU forward, and the oracle's tangent-linear
    derivative on three of the angles (same N, L)."""
    wl = config4()
    tgt = _target(len(wl.theta0), seed=9)
    res = _run(wl, "rk6", tgt, checkpoint_every=20)
    assert (res["status"] == 0).all()
    g = res["datoms"]
    s = wl.structures[0]
    for (ia, c) in [(4, 2), (10, 0)]:
        e = np.zeros_like(s.atoms)
        e[ia, c] = 1e-5
        fd = (_loss_only(wl, "rk6", tgt, s.atoms + e) - _loss_only(wl, "rk6", tgt, s.atoms - e)) / 2e-5
        print(f"[adjoint] full size fd atom {ia} coord {c}: gpu {g[ia, c]:.10e} fd {fd:.10e}", flush=True)
        assert g[ia, c] == pytest.approx(fd, rel=1e-5, abs=1e-8 * np.abs(g).max())
    idx = [5, 60, 120]
    sub = dataclasses.replace(wl, theta0=wl.theta0[idx])
    res_sub = _run(sub, "rk6", tgt[idx], checkpoint_every=20)
    rng = np.random.default_rng(2)
    d = np.zeros_like(s.atoms)
    d[:27] = rng.normal(size=(27, 3))
    loss, dl = driver.rfactor_directional(sub, 0, d, tgt[idx], stepper="rk6")
    got = float(np.sum(res_sub["datoms"] * d))
    print(f"[adjoint] full size (3 angles) direction: gpu {got:.12e} oracle {dl:.12e}", flush=True)
    assert got == pytest.approx(dl, rel=1e-8)


def test_autograd_wrapper_matches_explicit_adjoint():
    """api.intensity under torch.autograd gives the same loss and atom
    gradient as the explicit rfactor -> backward -> potential_backward path."""
    import torch
    from paper_2306_00271_amd import api
    wl = small_2d(n_beams=21, n_slices=40, thickness=4.0, n_layers=1, n_angles=3)
    tgt = _target(3)
    res = _run(wl, "rk6", tgt)
    dev = torch.device("cuda:0")
    plan = res["plan"]
    atoms = api.atoms_for(wl, dev).requires_grad_(True)
    inten, status = api.intensity(plan, atoms, api.angles_for(wl, dev))
    t = torch.from_numpy(tgt).to(dev)
    loss = ((inten[:, 0] - t) ** 2).sum()
    loss.backward()
    assert (status.cpu().numpy() == 0).all()
    np.testing.assert_allclose(loss.item(), res["loss"], rtol=1e-13)
    np.testing.assert_allclose(atoms.grad.cpu().numpy(), res["datoms"], rtol=1e-12, atol=1e-15)
    # without a gradient the wrapper keeps no workspace and returns the same intensities
    with torch.no_grad():
        inten2, _ = api.intensity(plan, atoms.detach(), api.angles_for(wl, dev))
    np.testing.assert_array_equal(inten2.cpu().numpy(), res["eta"])


def test_mfma_peak_probe():
    from paper_2306_00271_amd import api
    tf = api.mfma_f64_peak(blocks=256, iters=500)
    assert 5.0 < tf < 200.0


def _table_grad(wl, stepper, target, every):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    print(f"[adjoint] {wl.name} {stepper} checkpoint_every={every}", flush=True)
    plan = api.plan_for(wl, stepper=stepper, checkpoint_every=every)
    atoms = api.atoms_for(wl, dev)
    U = plan.potential(atoms)
    ang = api.angles_for(wl, dev)
    ws = plan.workspace(dev)
    out = plan.forward(U, ang, workspace=ws)
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64)).to(dev)
    _, dI = api.rfactor(out["intensity"], tgt)
    dU = plan.backward(U, ang, dI, ws)
    torch.cuda.synchronize()
    res = dU.cpu().numpy(), out["status"].cpu().numpy(), plan.split
    del ws, plan
    return res


@pytest.mark.parametrize("stepper", ["rk4", "rk6"])
def test_checkpoint_segments_match_every_slice_states(stepper):
    """States kept every 7 or 20 slices (the physical column re-stepped
    through each segment from its stored state) give the table gradient of
    the adjoint that reads a stored state at every slice, to rounding.  50
    slices leave a partial top segment; a second structure of 33 slices ends
    inside a lower one."""
    wl = small_2d(n_beams=21, n_slices=50, thickness=5.0, n_layers=1, n_angles=3)
    s2 = dataclasses.replace(wl.structures[0], n_slices=33, thickness=3.3)
    wl = dataclasses.replace(wl, structures=[wl.structures[0], s2])
    tgt = _target(6)
    ref, st, _ = _table_grad(wl, stepper, tgt, 1)
    assert (st == 0).all()
    for every in (7, 20):
        got, _, _ = _table_grad(wl, stepper, tgt, every)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"[adjoint] small slab {stepper} K={every}: max |dU(K) - dU(K=1)| / max |dU| = {err:.3e}", flush=True)
        np.testing.assert_allclose(got, ref, rtol=0.0, atol=1e-13 * np.abs(ref).max())


def test_checkpoint_every_20_gradient_workload():
    """The gradient workload at its stated checkpoint interval of 20 slices
    matches the every-slice adjoint to rounding, with one structure (split
    forward) and with two (256 pairs, one workgroup per pair)."""
    for ns in (1, 2):
        wl = config4(ns)
        tgt = _target(len(wl.theta0) * ns, seed=9)
        ref, st, _ = _table_grad(wl, "rk6", tgt, 1)
        got, _, _ = _table_grad(wl, "rk6", tgt, 20)
        assert (st == 0).all()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"[adjoint] c4 x{ns}: max |dU(K=20) - dU(K=1)| / max |dU| = {err:.3e}", flush=True)
        np.testing.assert_allclose(got, ref, rtol=0.0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("layout", ["whole", "split"])
def test_graph_capture_of_the_gradient_step(layout):
    """The whole gradient step (tables, forward keeping a state every 20
    slices, R-factor, adjoint, atom gradient) captured once in a HIP graph:
    every replay, with eager steps and synchronisations between replays,
    reproduces the eager step bit for bit."""
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    wl = small_2d(n_beams=21, n_slices=50, thickness=5.0, n_layers=1, n_angles=3)
    plan = api.plan_for(wl, stepper="rk6", layout=layout, checkpoint_every=20)
    atoms = api.atoms_for(wl, dev)
    ang = api.angles_for(wl, dev)
    ws = plan.workspace(dev)
    tgt = torch.from_numpy(_target(3)).to(dev)

    def step():
        U = plan.potential(atoms)
        out = plan.forward(U, ang, workspace=ws)
        loss, dI = api.rfactor(out["intensity"], tgt)
        dU = plan.backward(U, ang, dI, ws)
        return out["intensity"], loss, plan.potential_backward(atoms, dU)

    ref = [t.clone() for t in step()]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        for o, rf in zip(outs, ref):
            assert torch.equal(o, rf), f"replay {r}"
        step()
        torch.cuda.synchronize()


@pytest.mark.parametrize("every", [1, 20])
@pytest.mark.parametrize("stepper", ["rk4", "rk6"])
def test_atom_gradient_every_coordinate(stepper, every):
    """Every coordinate of every atom of a small slab (9 atoms, 27 entries)
    against the oracle's tangent-linear derivative along that coordinate,
    entry by entry (1e-8 relative to the entry, or to 1e-6 of the largest)."""
    from tests.gpu_util import assert_entrywise, oracle_atom_gradient
    wl = small_2d(n_beams=21, n_slices=40 if stepper == "rk6" else 80, thickness=4.0, n_layers=1, n_angles=3)
    tgt = _target(3, seed=13)
    res = _run(wl, stepper, tgt, checkpoint_every=every)
    assert (res["status"] == 0).all()
    n_atoms = wl.structures[0].atoms.shape[0]
    coords = [(ia, c) for ia in range(n_atoms) for c in range(3)]
    ref = oracle_atom_gradient(wl, tgt, coords, stepper=stepper)
    got = np.array([res["datoms"][ia, c] for ia, c in coords])
    assert_entrywise(got, ref, what=f"small slab {stepper} K={every}, all {len(coords)} coordinates")


def test_gradient_workload_every_coordinate_at_one_angle():
    """The gradient workload (N = 61, 400 slices, RK6, states every 20
    slices) at one angle: all 81 differentiated coordinates (27 atoms x 3)
    against the oracle's tangent-linear derivative, entry by entry."""
    from tests.gpu_util import assert_entrywise, oracle_atom_gradient
    wl = config4()
    a = 60
    sub = dataclasses.replace(wl, theta0=wl.theta0[[a]])
    tgt = _target(len(wl.theta0), seed=9)[[a]]
    res = _run(sub, "rk6", tgt, checkpoint_every=20)
    assert (res["status"] == 0).all()
    coords = [(int(ia), c) for ia in wl.structures[0].grad_atoms for c in range(3)]
    assert len(coords) == 81
    ref = oracle_atom_gradient(sub, tgt, coords, stepper="rk6")
    got = np.array([res["datoms"][ia, c] for ia, c in coords])
    assert_entrywise(got, ref, what="gradient workload, one angle, 81 coordinates")


@pytest.mark.parametrize("every", [1, 3])
@pytest.mark.parametrize("stepper", ["rk4", "rk6"])
def test_table_gradient_every_entry(stepper, every):
    """dR/d(Re u) and dR/d(Im u) of every entry of a tiny case's tables
    (N = 5 beams, 4 slices: 9 or 17 nodes x 25 rod differences) against the
    oracle's tangent-linear derivative along that single entry."""
    from tests.gpu_util import assert_entrywise
    wl = small_2d(n_beams=5, n_slices=4, thickness=2.0, n_layers=1, n_angles=2, theta_range=(1.0, 3.0))
    tgt = _target(2, seed=17)
    res = _run(wl, stepper, tgt, checkpoint_every=every)
    assert (res["status"] == 0).all()
    st = driver.StructureSetup(wl, wl.structures[0], driver.TABLEAUX[stepper])
    shape = st.table.shape
    ref = np.zeros(shape, dtype=np.complex128)
    for k in range(st.table.size):
        for part, unit in ((0, 1.0), (1, 1j)):
            dt = np.zeros(shape, dtype=np.complex128)
            dt.flat[k] = unit
            _, dl = driver.rfactor_directional_table(wl, 0, dt, tgt, stepper=stepper)
            if part == 0:
                ref.flat[k] += dl
            else:
                ref.flat[k] += 1j * dl
    got = res["dU"].reshape(shape)
    both_got = np.concatenate([got.real.ravel(), got.imag.ravel()])
    both_ref = np.concatenate([ref.real.ravel(), ref.imag.ravel()])
    assert_entrywise(both_got, both_ref, what=f"tiny tables {stepper} K={every}, {both_ref.size} real entries")
