"""Parity of the forward path for 64 < N <= 128 beams (the kernel that keeps a
pair's state in plan-owned device memory) with the CPU oracle, through the C
ABI."""
import dataclasses

import numpy as np
import pytest

from synth import config3, small_2d
from tests.gpu_util import eacc, gpu_forward, oracle_forward, physical

pytestmark = pytest.mark.gpu

TOL = 1e-10   # relative intensity (eacc form), as for N <= 64


def _report(name, e):
    print(f"[parity] {name}: eacc={e:.3e}", flush=True)


@pytest.mark.parametrize("stepper", ["rk4", "rk6"])
@pytest.mark.parametrize("n_beams", [65, 91, 121, 128])
def test_forward_large_n(stepper, n_beams):
    wl = small_2d(n_beams=n_beams, n_slices=80 if stepper == "rk4" else 40, thickness=4.0, n_layers=2, n_angles=4)
    res = gpu_forward(wl, stepper=stepper, want_rho=True)
    info = res["plan"].info
    assert info.large_pairs == 4 and info.large_slots >= 1
    ref, rho_ref, nr = oracle_forward(wl, stepper=stepper)
    got = res["intensity"][:, :n_beams]
    assert (res["status"] == 0).all()
    e = eacc(got, ref)
    _report(f"large N={n_beams} {stepper} rhst={nr.tolist()} gpu_rhst={res['n_rhst'].tolist()}", e)
    assert e <= TOL
    big = ref > 1e-6
    assert np.all(np.abs(got[big] - ref[big]) <= 1e-9 * ref[big])
    # the reflected amplitudes themselves (unique: rho(0) does not depend on the transformations)
    rho = res["rho"][:, :n_beams]
    assert np.abs(rho - rho_ref).max() <= 1e-9 * np.abs(rho_ref).max()


def test_uneven_batch_small_and_large_in_one_call():
    """Structures of N = 31, 61, 91 and 121 beams with different slice counts in
    one plan: the N <= 64 pairs go to the one-workgroup kernel, the others to
    the large kernel, both from one rheed_forward call; every structure
    against the oracle, and the outputs past each structure's N are zero."""
    parts = [small_2d(n_beams=n, n_slices=L, thickness=0.1 * L, n_layers=2, n_angles=3, seed=20 + i)
             for i, (n, L) in enumerate(((31, 30), (91, 24), (61, 36), (121, 20)))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    res = gpu_forward(wl, stepper="rk6")
    info = res["plan"].info
    assert info.large_pairs == 6 and info.max_beams == 121
    assert (res["status"] == 0).all()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, nr = oracle_forward(wl, s_idx=s, stepper="rk6")
        got = res["intensity"][s * A:(s + 1) * A, :N]
        e = eacc(got, ref)
        _report(f"small+large batch structure {s} N={N} L={p.structures[0].n_slices}", e)
        assert e <= TOL
        assert np.all(res["intensity"][s * A:(s + 1) * A, N:] == 0.0)


def test_more_pairs_than_resident_workgroups():
    """300 angles of an N = 91 slab: more pairs than the large kernel keeps
    resident, so workgroups run several pairs one after another in their
    slots; sampled angles against the oracle."""
    wl = small_2d(n_beams=91, n_slices=6, thickness=0.6, n_layers=2, n_angles=300, theta_range=(0.3, 6.0))
    res = gpu_forward(wl, stepper="rk6")
    info = res["plan"].info
    assert info.large_pairs == 300
    assert (res["status"] == 0).all()
    idx = np.array([0, 1, 97, 150, 255, 256, 257, 299])
    ref, _, _ = oracle_forward(wl, stepper="rk6", angle_idx=idx)
    e = eacc(res["intensity"][idx, :91], ref)
    _report(f"N=91, 300 pairs on {info.large_slots} workgroups, sampled", e)
    assert e <= TOL


def test_uneven_workload_full_size_sample():
    """The uneven-N batched workload at full size (40 A, RK6, slices per N
    from the step rule h max|Gamma_j| <= 1.45: 540 for N = 91, 600 for
    N = 121): the first structures with N = 91 and N = 121 at the lowest,
    a middle and the highest angle, against the oracle at 1e-10.  Both
    curves pass the validity gate (finite, eta >= 0, summed flux <= 1 under
    absorption)."""
    wl = config3(16)
    picks = []
    for n in (91, 121):
        s = next(i for i, st in enumerate(wl.structures) if st.n_beams == n)
        picks.append(s)
    sub = dataclasses.replace(wl, structures=[wl.structures[s] for s in picks],
                              theta0=wl.theta0[[0, 40, 63]])
    res = gpu_forward(sub, stepper="rk6")
    assert (res["status"] == 0).all()
    A = len(sub.theta0)
    for k, s in enumerate(picks):
        N = sub.structures[k].n_beams
        ref, _, nr = oracle_forward(sub, s_idx=k, stepper="rk6")
        got = res["intensity"][k * A:(k + 1) * A, :N]
        assert physical(ref, sub.absorption).all(), f"oracle off the physical solution at N = {N}"
        assert physical(got, sub.absorption).all()
        e = eacc(got, ref)
        _report(f"uneven workload structure {s} N={N} L={sub.structures[k].n_slices} rhst={nr.tolist()} "
                f"gpu={res['n_rhst'][k * A:(k + 1) * A].tolist()} sum eta={ref.sum(axis=1).round(6).tolist()}", e)
        assert e <= TOL


def test_uniform_grid_is_flagged_at_large_n():
    """On the uniform 0.1 A grid (400 slices) the N = 121 structure of the
    uneven-N workload is off the physical solution; the GPU reproduces the
    discretised result and the validity gate flags it (what bench.py counts
    as invalid pairs)."""
    wl = config3(16, slices={31: 400, 61: 400, 91: 400, 121: 400})
    s = next(i for i, st in enumerate(wl.structures) if st.n_beams == 121)
    sub = dataclasses.replace(wl, structures=[wl.structures[s]], theta0=wl.theta0[[40]])
    res = gpu_forward(sub, stepper="rk6")
    got = res["intensity"][:, :121]
    assert not physical(got, sub.absorption).any()


def test_adjoint_workspace_of_large_plans():
    """Plans with N > 64 keep states for the adjoint with the RK steppers
    (their workspace is sized for states padded to 128 beams and refused
    when short); the splitting stepper keeps none above 64 beams."""
    import torch
    from paper_2306_00271_amd import api
    from paper_2306_00271_amd._lib import RheedError
    wl = small_2d(n_beams=91, n_slices=4, thickness=0.4, n_layers=2, n_angles=2)
    plan = api.plan_for(wl, stepper="rk6")
    dev = torch.device("cuda:0")
    # per pair at least the final state and B^{-1} (2 + 1 matrices of 128 x 128 complex)
    assert plan.info.fwd_workspace >= plan.n_pairs * 3 * 128 * 128 * 16
    assert plan.info.bwd_workspace > 0
    U = plan.potential(api.atoms_for(wl, dev))
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    with pytest.raises(RheedError, match="workspace of"):
        plan.forward(U, api.angles_for(wl, dev), workspace=ws)
    dI = torch.zeros((plan.n_pairs, plan.max_beams), dtype=torch.float64, device=dev)
    with pytest.raises(RheedError, match="workspace of"):
        plan.backward(U, api.angles_for(wl, dev), dI, ws)
    sp = api.plan_for(wl, stepper="sp4")
    assert sp.info.fwd_workspace == 0
    with pytest.raises(RheedError, match="N <= 64"):
        sp.forward(sp.potential(api.atoms_for(wl, dev)), api.angles_for(wl, dev), workspace=ws)


def test_graph_capture_of_a_mixed_forward():
    """A forward call over structures with N = 45 and N = 91 (two launches:
    the N <= 64 kernel and the N > 64 kernel) captured once in a HIP graph:
    every replay, with eager calls and synchronisations between replays,
    reproduces the eager outputs bit for bit."""
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    parts = [small_2d(n_beams=n, n_slices=12, thickness=1.2, n_layers=2, n_angles=3, seed=40 + i)
             for i, n in enumerate((45, 91))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    plan = api.plan_for(wl, stepper="rk6")
    assert plan.info.large_pairs == 3
    atoms = api.atoms_for(wl, dev)
    ang = api.angles_for(wl, dev)

    def step():
        U = plan.potential(atoms)
        out = plan.forward(U, ang, want_rho=True, want_nrhst=True)
        return out["intensity"], out["rho"], out["status"], out["n_rhst"]

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
    assert (ref[2] == 0).all()


def test_autotune_picks_the_fastest_candidate_and_keeps_the_results():
    """rheed_autotune on a batch with N = 45 and N = 91 structures times the
    five candidates (one persistent launch over both kinds of pair; two
    launches with the split or whole layout for N <= 64 x cost or pair order
    for N > 64), keeps the fastest, and later forward calls still match the
    oracle."""
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    parts = [small_2d(n_beams=n, n_slices=16, thickness=1.6, n_layers=2, n_angles=3, seed=50 + i)
             for i, n in enumerate((45, 91))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    plan = api.plan_for(wl, stepper="rk6")
    U = plan.potential(api.atoms_for(wl, dev))
    ang = api.angles_for(wl, dev)
    before = plan.forward(U, ang)["intensity"].cpu().numpy()
    assert plan.info.queue == 1
    rep = plan.autotune(U, ang, reps=2)
    cands = rep["candidates"]
    assert len(cands) == 5
    assert cands[0]["queue"] and not any(c["queue"] for c in cands[1:])
    assert {(c["split"], c["large_cost_order"]) for c in cands[1:]} == {(a, b) for a in (True, False)
                                                                        for b in (True, False)}
    assert all(c["ms"] > 0.0 for c in cands)
    best = min(range(5), key=lambda c: cands[c]["ms"])
    assert rep["chosen"] == best
    assert plan.info.queue == int(cands[best]["queue"])
    if not cands[best]["queue"]:
        assert plan.split == cands[best]["split"]
    out = plan.forward(U, ang)
    torch.cuda.synchronize()
    after = out["intensity"].cpu().numpy()
    assert (out["status"].cpu().numpy() == 0).all()
    assert np.abs(after - before).max() <= 1e-12 * np.abs(before).max()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, _ = oracle_forward(wl, s_idx=s, stepper="rk6")
        e = eacc(after[s * A:(s + 1) * A, :N], ref)
        _report(f"after autotune structure {s} N={N}", e)
        assert e <= TOL


@pytest.mark.parametrize("layout", ["whole", "split"])
@pytest.mark.parametrize("bad", [1, 2])
def test_nonfinite_table_marks_only_its_pairs(layout, bad):
    """A NaN in one structure's potential table (the zero rod difference at
    the first node, which every pair of that structure uses) makes exactly
    that structure's pairs RHEED_PAIR_NONFINITE with non-finite amplitudes;
    the call succeeds and every other pair (both kernels, split or whole
    layout for N <= 64) still matches the oracle."""
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    parts = [small_2d(n_beams=n, n_slices=12, thickness=1.2, n_layers=2, n_angles=3, seed=60 + i)
             for i, n in enumerate((21, 45, 91))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    plan = api.plan_for(wl, stepper="rk6", layout=layout)
    assert plan.split == (layout == "split")
    U = plan.potential(api.atoms_for(wl, dev))
    offs = plan.table_offsets
    n_nodes = 12 * plan.info.nodes_per_slice + 1
    box = int(offs[bad + 1] - offs[bad]) // n_nodes
    U[int(offs[bad]) + box // 2] = complex(float("nan"), 0.0)
    out = plan.forward(U, api.angles_for(wl, dev), want_rho=True)
    torch.cuda.synchronize()
    status = out["status"].cpu().numpy()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        rows = slice(s * A, (s + 1) * A)
        if s == bad:
            assert (status[rows] == 2).all(), status
            assert not np.isfinite(out["rho"][rows, :N].cpu().numpy()).all()
        else:
            assert (status[rows] == 0).all(), status
            ref, _, _ = oracle_forward(wl, s_idx=s, stepper="rk6")
            e = eacc(out["intensity"][rows, :N].cpu().numpy(), ref)
            _report(f"NaN in structure {bad} ({layout}): structure {s} N={N}", e)
            assert e <= TOL


@pytest.mark.parametrize("n_slices,threshold", [(1, 1.0), (3, 1e300), (6, 1.0)])
def test_large_edge_cases(n_slices, threshold):
    """One slice (and a transformation right after it), no transformation at
    all on a thin slab, and one after every slice; N = 97."""
    wl = small_2d(n_beams=97, n_slices=n_slices, thickness=0.1 * n_slices, n_layers=1, n_angles=3)
    res = gpu_forward(wl, stepper="rk6", threshold=threshold)
    ref, _, nr = oracle_forward(wl, stepper="rk6", threshold=threshold)
    assert (res["status"] == 0).all()
    assert res["n_rhst"].tolist() == nr.tolist()
    e = eacc(res["intensity"][:, :97], ref)
    _report(f"N=97 L={n_slices} threshold={threshold:g} rhst={nr.tolist()}", e)
    assert e <= TOL


def test_large_paper_convention():
    wl = small_2d(n_beams=81, n_slices=12, thickness=1.2, n_layers=2, n_angles=3)
    res = gpu_forward(wl, stepper="rk6", convention="paper")
    ref, _, _ = oracle_forward(wl, stepper="rk6", convention="paper")
    e = eacc(res["intensity"][:, :81], ref)
    _report("N=81 printed convention", e)
    assert e <= TOL


def test_thick_slab_without_transformations_is_flagged():
    """N > 64: the transformation switched off on a 40 A slab of the
    uneven-N workload (N = 91): the pair comes back flagged
    (RHEED_PAIR_BREAKDOWN, or SINGULAR / NONFINITE) with NaN intensities,
    and the call succeeds."""
    wl = config3(16)
    s = next(i for i, st in enumerate(wl.structures) if st.n_beams == 91)
    sub = dataclasses.replace(wl, structures=[wl.structures[s]], theta0=wl.theta0[[10, 50]])
    res = gpu_forward(sub, stepper="rk6", threshold=float("inf"))
    st = res["status"]
    print(f"[edge] threshold inf, N=91: status {st.tolist()}, n_rhst {res['n_rhst'].tolist()}", flush=True)
    assert (res["n_rhst"] == 0).all()
    assert np.isin(st, [1, 2, 4]).all()
    assert np.all(np.isnan(res["intensity"][:, :91]))


def test_one_launch_queue_matches_two_launches():
    """A batch mixing N = 21, 61, 91 and 121 structures with different slice
    counts: the one persistent launch (workgroups taking pairs of either kind
    from one queue, dearest first) against the same batch in two launches
    (layout SPLIT keeps the N <= 64 pairs on their own launch), and against
    the oracle; then 300 pairs, more than the launch has workgroups."""
    parts = [small_2d(n_beams=n, n_slices=L, thickness=0.1 * L, n_layers=2, n_angles=10, seed=80 + i)
             for i, (n, L) in enumerate(((21, 30), (61, 24), (91, 20), (121, 12)))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    res_q = gpu_forward(wl, stepper="rk6")
    res_2 = gpu_forward(wl, stepper="rk6", layout="split")
    assert res_q["plan"].info.queue == 1 and res_2["plan"].info.queue == 0
    assert (res_q["status"] == 0).all()
    assert np.abs(res_q["intensity"] - res_2["intensity"]).max() <= 1e-12 * np.abs(res_2["intensity"]).max()
    A = len(wl.theta0)
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, nr = oracle_forward(wl, s_idx=s, stepper="rk6")
        e = eacc(res_q["intensity"][s * A:(s + 1) * A, :N], ref)
        _report(f"queue structure {s} N={N} rhst={nr.tolist()} gpu={res_q['n_rhst'][s * A:(s + 1) * A].tolist()}", e)
        assert e <= TOL
        assert res_q["n_rhst"][s * A:(s + 1) * A].tolist() == nr.tolist()
    parts = [small_2d(n_beams=n, n_slices=6, thickness=0.6, n_layers=1, n_angles=150, seed=90 + i,
                      theta_range=(0.3, 6.0)) for i, n in enumerate((31, 69))]
    wl = dataclasses.replace(parts[0], structures=[p.structures[0] for p in parts])
    res_q = gpu_forward(wl, stepper="rk4")
    assert res_q["plan"].info.queue == 1 and (res_q["status"] == 0).all()
    idx = np.array([0, 77, 149])
    for s, p in enumerate(parts):
        N = p.structures[0].n_beams
        ref, _, _ = oracle_forward(wl, s_idx=s, angle_idx=idx, stepper="rk4")
        e = eacc(res_q["intensity"][s * 150 + idx, :N], ref)
        _report(f"queue, 300 pairs, structure {s} N={N} (sampled)", e)
        assert e <= TOL

