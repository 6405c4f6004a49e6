"""Throughput of the many-beam RHEED/TRHEPD path on one MI355X.

One step = one pass of the whole hot path over the gradient workload
(15 keV electrons, N = 61 rods of a 3x3 supercell, 9 atoms x 10 layers,
40 A in 400 slices, 128 glancing angles 0.3..6.0 deg, 6th-order RK):
potential tables from atoms -> forward propagation with RHST and reflection,
keeping the state every 20 slices -> R-factor against a target curve ->
adjoint propagation, segment by segment, each segment's states recomputed
from its checkpoint -> gradient with respect to atom coordinates.  Inputs
are seeded synthetic slabs, resident in HBM before the timed region.  Prints
one JSON line; "variants" adds the same step with every slice state kept and
the plain per-angle form (the same kernels on one pair at a time).

``--mode fwd`` times the forward pass alone (potential + propagation).
``--traffic-probe`` runs one forward launch and a 1 GiB device copy for the
HBM counter runs whose summary is kept under profiles/.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 matrix, published
CHECKPOINT_EVERY = 20           # the gradient workload keeps the state every 20 slices


def kernel_name(split):
    return "forward_split_kernel<1, false>" if split else "forward_kernel<1, false>"


def traffic_summary(split):
    stem = "forward_split_kernel" if split else "forward_kernel"
    return os.path.join(ROOT, "profiles", f"{stem}_rk6_n61_traffic.md")


def _flops_forward(N, L, stages, n_rhst_total, n_pairs):
    """Algorithmic FP64 flops of the propagation kernel for one launch:
    L * s complex N^3 products (8 flops per complex MAC), (8/3 + 8) N^3 per
    right-hand-side transformation (LU + N-row right division), and
    (8/3) N^3 for the final single-column solve per pair."""
    n3 = float(N) ** 3
    return n_pairs * (L * stages * 8.0 * n3 + (8.0 / 3.0) * n3) + n_rhst_total * (8.0 / 3.0 + 8.0) * n3


def invalid_pairs(intensity, status, absorption):
    """Pairs whose rocking curve fails the validity gate (Sec. 2.1: the
    reflected flux cannot exceed the incident one under absorption): a
    numerical failure status, a non-finite or negative intensity, or summed
    intensities above 1 + 1e-9 when absorption > 0."""
    import torch
    eta = intensity.double()
    bad = (status != 0) | ~torch.isfinite(eta).all(dim=1) | (eta < 0).any(dim=1)
    if absorption > 0.0:
        bad |= eta.sum(dim=1) > 1.0 + 1e-9
    return int(bad.sum().item())


# ---------------------------------------------------------------- CPU baseline
def _cpu_worker(args):
    kind, idx, stepper = args[:3]
    # one BLAS thread per process, except for the single-pair case, which the
    # paper also times with threaded BLAS (idx = threads there)
    nthr = str(idx) if kind == "n521" else "1"
    os.environ["OMP_NUM_THREADS"] = nthr
    os.environ["OPENBLAS_NUM_THREADS"] = nthr
    os.environ["MKL_NUM_THREADS"] = nthr
    import numpy as np
    from synth import config3, config4
    from oracle import driver
    if kind == "bulk_layer":
        # one unit layer of the bulk under the gradient workload's slab, from the vacuum
        from oracle import bulk
        from oracle.tableaux import TABLEAUX
        from synth import bulk_layer
        wb = bulk_layer(config4(1), BULK_SLICES)
        st = driver.StructureSetup(wb, wb.structures[0], TABLEAUX[stepper])
        gam, _ = st.angle(float(wb.theta0[idx]))
        Y = 1j * np.diag(gam)
        t0 = time.perf_counter()
        for _ in range(args[3]):
            Y = bulk.layer_map(st.mfun(gam), gam, st.h, BULK_SLICES, TABLEAUX[stepper], Y)
        return (time.perf_counter() - t0) / args[3]
    if kind == "uneven":
        # one pair of the uneven-N workload: structure idx of the first args[3], one angle
        wl3 = config3(args[3])
        t0 = time.perf_counter()
        driver.rocking_curve(wl3, s_idx=idx, angle_idx=[(idx * 37) % len(wl3.theta0)], stepper=stepper)
        return time.perf_counter() - t0
    if kind == "n521":
        # the single-angle n = 521 case over its first args[3] slices (same step)
        import dataclasses
        from synth import single_angle_n521
        w6 = single_angle_n521()
        st6 = w6.structures[0]
        part = dataclasses.replace(st6, n_slices=args[3], thickness=st6.thickness * args[3] / st6.n_slices)
        w6 = dataclasses.replace(w6, structures=[part])
        t0 = time.perf_counter()
        driver.rocking_curve(w6, stepper=stepper)
        return time.perf_counter() - t0
    if kind == "n199":
        # one pair of the N = 199 workload over its first args[3] slices (same step)
        import dataclasses
        from synth import config5
        w5 = config5(1)
        st5 = w5.structures[0]
        part = dataclasses.replace(st5, n_slices=args[3], thickness=st5.thickness * args[3] / st5.n_slices)
        w5 = dataclasses.replace(w5, structures=[part])
        t0 = time.perf_counter()
        driver.rocking_curve(w5, angle_idx=[idx], stepper=stepper)
        return time.perf_counter() - t0
    wl = config4(1)
    t0 = time.perf_counter()
    if kind == "fwd":
        driver.rocking_curve(wl, angle_idx=[idx], stepper=stepper)
    else:
        # one tangent-linear pass: forward plus the derivative along one atom coordinate
        direction = np.zeros((wl.structures[0].atoms.shape[0], 3))
        direction[idx % len(wl.structures[0].grad_atoms), idx % 3] = 1.0
        driver.rfactor_directional(wl, 0, direction, np.zeros(1), angle_idx=[idx], stepper=stepper)
    return time.perf_counter() - t0


def cpu_baseline(stepper, n_angles, n_coords, cores, mode):
    """The oracle (NumPy FP64, one BLAS thread per process) on `cores` host
    processes, each timing two (structure, angle) pairs of the workload, all
    at different angles.  fwd+adj: the oracle's gradient of a point is one
    tangent-linear pass (forward + directional derivative) per atom
    coordinate, so a point costs n_coords passes and the rate is
    cores / (n_coords * mean pass time).  fwd: cores / mean forward time."""
    import multiprocessing as mp
    kind = "fwd" if mode == "fwd" else "tl"
    jobs = [(kind, (c * n_angles) // (2 * cores), stepper) for c in range(2 * cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        times = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    per_pass = float(sum(times) / len(times))
    per_point = per_pass if kind == "fwd" else n_coords * per_pass
    # one core alone: the same pass in a single process with nothing beside it
    with ctx.Pool(1) as pool:
        alone = float(pool.map(_cpu_worker, [(kind, n_angles // 3, stepper)])[0])
    per_point_1 = alone if kind == "fwd" else n_coords * alone
    return cores / per_point, per_pass, wall, 1.0 / per_point_1, alone


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ------------------------------------------------------------- HBM traffic
def kernel_source_hash():
    """sha256 of the sources the forward kernel is built from."""
    h = hashlib.sha256()
    for f in ("rheed_forward.hip", "rheed_forward_all.hip", "rheed_gj.h", "rheed_internal.h"):
        with open(os.path.join(ROOT, "paper_2306_00271_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profile(split):
    """HBM bytes per forward launch from the committed counter summary, or
    None if the summary is missing or was taken on other kernel sources."""
    path = traffic_summary(split)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def traffic_probe(checkpoint_every):
    """One forward launch of the timed workload (with the adjoint's state
    saving) and one device copy of 1 GiB, for FETCH_SIZE / WRITE_SIZE counter
    runs; prints the copy size so the counters can be calibrated."""
    import torch
    from paper_2306_00271_amd import api
    from synth import config4
    dev = torch.device("cuda:0")
    wl = config4(1)
    plan = api.plan_for(wl, stepper="rk6", checkpoint_every=checkpoint_every)
    angles = api.angles_for(wl, dev)
    U = plan.potential(api.atoms_for(wl, dev))
    ws = plan.workspace(dev)
    plan.forward(U, angles, workspace=ws)
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 8, "source_sha256": kernel_source_hash(),
                      "kernel": kernel_name(plan.split), "checkpoint_every": checkpoint_every}))


# ------------------------------------------------------ uneven-N workload
def uneven_forward(n_structures, steps=2, cpu=True):
    """Forward throughput on the first n_structures of the uneven-N batched
    workload (N drawn from {31, 61, 91, 121}, 64 angles each, 440 to 600
    slices by N, RK6): the whole batch through one rheed_forward call (N <= 64 pairs on the
    one-workgroup kernel, the rest on the N > 64 kernel), then the N > 64
    pairs alone for the large kernel's algorithmic rate, and one pair of each
    N alone for the per-angle form."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import config3

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = config3(n_structures)

    tune = {}

    def timed(w, reps, autotune=False):
        def note(msg):
            print(f"[uneven] {len(w.structures)} structures: {msg}", file=sys.stderr, flush=True)
        plan = api.plan_for(w, stepper="rk6")
        U = plan.potential(api.atoms_for(w, dev))
        ang = api.angles_for(w, dev)
        torch.cuda.synchronize()
        note(f"plan and tables ready ({plan.n_pairs} pairs, {U.numel() * 16 / 2**30:.2f} GiB of tables)")
        if autotune:  # launch configuration picked by timing the candidates on this batch
            tune.update(plan.autotune(U, ang, reps=1))
        plan.forward(U, ang)
        torch.cuda.synchronize()
        note("warm-up forward done")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = plan.forward(U, ang, want_nrhst=True)
        e1.record(stream)
        torch.cuda.synchronize()
        return plan, e0.elapsed_time(e1) / reps, out

    # the launch configuration is tuned on batches of up to 64 structures;
    # larger ones (the full 1024-structure workload) run the default, the
    # one persistent launch over every pair
    plan, ms, out = timed(wl, steps, autotune=n_structures <= 64)
    n_pairs = plan.n_pairs
    bad = invalid_pairs(out["intensity"], out["status"], wl.absorption)
    big = [st for st in wl.structures if st.n_beams > 64]
    res = {"structures": n_structures, "pairs": n_pairs, "ms_per_forward": round(ms, 3),
           "value": round(n_pairs / (ms / 1e3), 2), "unit": "points/s", "invalid_pairs": bad,
           "beams": {str(n): sum(1 for st in wl.structures if st.n_beams == n) for n in (31, 61, 91, 121)},
           "slices": {str(st.n_beams): st.n_slices for st in wl.structures},
           "autotune": {"chosen": tune.get("chosen"),
                        "candidates_ms": [round(c["ms"], 2) for c in tune.get("candidates", [])],
                        "candidates": ["one-launch-queue" if c.get("queue") else
                                       ("split" if c["split"] else "whole") + "/" +
                                       ("cost-order" if c["large_cost_order"] else "pair-order")
                                       for c in tune.get("candidates", [])]},
           "one_launch": bool(plan.info.queue)}
    if big and n_structures <= 64:
        wb = dataclasses.replace(wl, structures=big)
        pb, msb, outb = timed(wb, steps)
        nr = outb["n_rhst"].cpu().numpy()
        A = len(wl.theta0)
        fl = 0.0
        for k, st in enumerate(big):
            fl += _flops_forward(st.n_beams, st.n_slices, 7, int(nr[k * A:(k + 1) * A].sum()), A)
        res["large_kernel"] = {"pairs": pb.n_pairs, "ms": round(msb, 3), "slots": int(pb.info.large_slots),
                               "achieved_tflops": round(fl / (msb / 1e3) / 1e12, 3),
                               "frac_of_published": round(fl / (msb / 1e3) / 1e12 / MFMA_FP64_PEAK_TFLOPS, 4),
                               "rhst_per_pair": round(float(nr.mean()), 1)}
        del pb
    # per-angle form: one pair of each N at a time, projected over the batch
    per = {}
    proj = 0.0
    for n in (31, 61, 91, 121):
        sts = [st for st in wl.structures if st.n_beams == n]
        if not sts:
            continue
        one = dataclasses.replace(wl, structures=sts[:1], theta0=wl.theta0[:1])
        _, ms1, _ = timed(one, 1)
        per[str(n)] = round(ms1, 3)
        proj += ms1 * len(sts) * len(wl.theta0)
    res["per_angle"] = {"ms_per_pair": per, "projected_ms_per_forward": round(proj, 1),
                        "speedup_of_batched": round(proj / ms, 1),
                        "note": "one pair of each N timed alone, times the pairs of that N in the batch"}
    if cpu:
        # the oracle on one pair of every structure (each structure has the same
        # number of angles, so the mean over structures is the batch's mean per pair)
        import multiprocessing as mp
        cores = min(16, os.cpu_count() or 1)
        jobs = [("uneven", s, "rk6", n_structures) for s in range(min(n_structures, 16))]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            times = pool.map(_cpu_worker, jobs)
        cwall = time.perf_counter() - t0
        mean = float(sum(times) / len(times))
        res["cpu_baseline"] = {"value": round(cores / mean, 4), "unit": "points/s", "cores": cores, "kind": "oracle",
                               "sample": f"one pair of each of the first {len(jobs)} structures (one angle each), "
                                         f"oracle forward, mean {mean:.2f} s per pair; {cores} processes x 1 BLAS "
                                         f"thread, {cwall:.1f} s wall"}
    return res


# ------------------------------------------------------- FP32 stage products
def fp32_stages(steps=3):
    """Forward of the gradient workload's slab (N = 61, 400 slices, 128
    angles, RK6) with the stage products U X in FP32 (the lower-precision
    evaluation the paper leaves for future work) against the same forward in
    FP64: time per call and eacc between the two curves, beside the grid's
    own discretisation error (RK6 at 400 against 1600 slices)."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import config4

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = config4(1)

    def run(w, precision, reps):
        plan = api.plan_for(w, stepper="rk6", stage_precision=precision)
        U = plan.potential(api.atoms_for(w, dev))
        ang = api.angles_for(w, dev)
        out = plan.forward(U, ang)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = plan.forward(U, ang)
        e1.record(stream)
        torch.cuda.synchronize()
        return out["intensity"].cpu().numpy()[:, :61], e0.elapsed_time(e1) / reps

    eta32, ms32 = run(wl, "fp32", steps)
    eta64, ms64 = run(wl, "fp64", steps)
    fine = dataclasses.replace(wl, structures=[dataclasses.replace(wl.structures[0], n_slices=1600)])
    eta_f, _ = run(fine, "fp64", 1)
    den = float(np.max(np.linalg.norm(eta64, axis=1)))
    e = float(np.max(np.linalg.norm(eta32 - eta64, axis=1))) / den
    disc = float(np.max(np.linalg.norm(eta64 - eta_f, axis=1))) / den
    return {"ms_fp32": round(ms32, 3), "ms_fp64": round(ms64, 3), "speedup": round(ms64 / ms32, 3),
            "value_fp32": round(len(wl.theta0) / (ms32 / 1e3), 2), "unit": "points/s (forward only)",
            "eacc_fp32_vs_fp64": float(f"{e:.3e}"), "eacc_grid_vs_1600_slices": float(f"{disc:.3e}")}


def wide_gradient(steps=2):
    """The gradient step at N = 121: one N = 121 structure of the uneven-N
    workload (40 A in 600 slices, RK6, 64 angles, states every 20 slices),
    potential -> forward keeping states -> R-factor -> adjoint -> atom
    gradient, against the forward alone; time per step and the validity
    gate."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import config3

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    base = config3(16)
    s = next(i for i, st in enumerate(base.structures) if st.n_beams == 121)
    wl = dataclasses.replace(base, structures=[base.structures[s]])
    plan = api.plan_for(wl, stepper="rk6", checkpoint_every=20)
    atoms = api.atoms_for(wl, dev)
    ang = api.angles_for(wl, dev)
    ws = plan.workspace(dev)
    tgt = torch.from_numpy(np.random.default_rng(31).uniform(0.0, 0.3, size=plan.n_pairs)).to(dev)

    def step():
        U = plan.potential(atoms)
        out = plan.forward(U, ang, workspace=ws)
        _, dI = api.rfactor(out["intensity"], tgt)
        dU = plan.backward(U, ang, dI, ws)
        return out, plan.potential_backward(atoms, dU)

    def fwd():
        return plan.forward(plan.potential(atoms), ang)

    res = {}
    for name, fn in (("gradient_step", step), ("forward_only", fwd)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / steps
        if name == "gradient_step":
            out, g = r
            bad = invalid_pairs(out["intensity"], out["status"], wl.absorption)
            finite = bool(torch.isfinite(g).all().item())
    ms = res["gradient_step"]
    return {"structure": s, "n_beams": 121, "slices": wl.structures[0].n_slices, "angles": plan.n_pairs,
            "checkpoint_every": 20, "ms_per_step": round(ms, 3), "value": round(plan.n_pairs / (ms / 1e3), 2),
            "unit": "points/s (gradient step)", "ms_forward_only": round(res["forward_only"], 3),
            "workspace_gb": round((plan.info.fwd_workspace + plan.info.bwd_workspace) / 1e9, 2),
            "invalid_pairs": bad, "gradient_finite": finite}


def n199_forward(steps=1, cpu=True):
    """Forward throughput on one structure of the N = 199 workload (7x7
    supercell, 49 atoms x 12 layers, 60 A in 1000 slices, RK6, all 256
    angles: one pair per CU), the kernel for 128 < N <= 256, with its
    algorithmic FP64 rate; the whole workload (64 structures) is 64 such
    batches."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import config5

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = config5(1)
    plan = api.plan_for(wl, stepper="rk6")
    U = plan.potential(api.atoms_for(wl, dev))
    ang = api.angles_for(wl, dev)
    out = plan.forward(U, ang, want_nrhst=True)
    torch.cuda.synchronize()
    print(f"[n199] warm-up forward done ({plan.n_pairs} pairs)", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = plan.forward(U, ang, want_nrhst=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = wl.structures[0]
    nr = out["n_rhst"].cpu().numpy()
    fl = _flops_forward(st.n_beams, st.n_slices, 7, int(nr.sum()), plan.n_pairs)
    res = {"pairs": plan.n_pairs, "n_beams": st.n_beams, "slices": st.n_slices, "ms_per_forward": round(ms, 2),
           "value": round(plan.n_pairs / (ms / 1e3), 3), "unit": "points/s (forward)",
           "achieved_tflops": round(fl / (ms / 1e3) / 1e12, 3),
           "frac_of_published": round(fl / (ms / 1e3) / 1e12 / MFMA_FP64_PEAK_TFLOPS, 4),
           "rhst_per_pair": round(float(nr.mean()), 1), "xl_slots": int(plan.info.xl_slots),
           "invalid_pairs": invalid_pairs(out["intensity"], out["status"], wl.absorption),
           "projected_s_whole_workload": round(64 * ms / 1e3, 1)}
    # the same batch with the stage products in FP32 (the lower-precision
    # evaluation; everything else FP64)
    p32 = api.plan_for(wl, stepper="rk6", stage_precision="fp32")
    U32 = p32.potential(api.atoms_for(wl, dev))
    p32.forward(U32, ang)
    torch.cuda.synchronize()
    e0.record(stream)
    o32 = p32.forward(U32, ang)
    e1.record(stream)
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1)
    a64 = out["intensity"][:, :st.n_beams].cpu().numpy()
    a32 = o32["intensity"][:, :st.n_beams].cpu().numpy()
    e32 = float(np.max(np.linalg.norm(a32 - a64, axis=1)) / np.max(np.linalg.norm(a64, axis=1)))
    res["fp32_stages"] = {"ms_per_forward": round(ms32, 2), "speedup": round(ms / ms32, 3),
                          "eacc_vs_fp64_stages": float(f"{e32:.3e}"),
                          "invalid_pairs": invalid_pairs(o32["intensity"], o32["status"], wl.absorption)}
    print(f"[n199] FP32 stages: {ms32:.1f} ms, eacc vs FP64 {e32:.2e}", file=sys.stderr, flush=True)
    del plan, U, p32, U32
    # one pair alone (the paper's single-angle case): on one workgroup, and
    # on a group of workgroups that step its column blocks side by side
    single = dataclasses.replace(wl, theta0=wl.theta0[100:101])
    res["single_pair"] = {}
    for layout in ("whole", "auto"):
        p1 = api.plan_for(single, stepper="rk6", layout=layout)
        U1 = p1.potential(api.atoms_for(single, dev))
        a1 = api.angles_for(single, dev)
        p1.forward(U1, a1)
        torch.cuda.synchronize()
        e0.record(stream)
        o1 = p1.forward(U1, a1)
        e1.record(stream)
        torch.cuda.synchronize()
        key = "one_workgroup" if p1.info.xl_group == 1 else f"group_of_{p1.info.xl_group}"
        res["single_pair"][key] = {"ms": round(e0.elapsed_time(e1), 2),
                                   "invalid_pairs": invalid_pairs(o1["intensity"], o1["status"], wl.absorption)}
        print(f"[n199] single pair, {key}: {res['single_pair'][key]['ms']} ms", file=sys.stderr, flush=True)
        del p1, U1
    # the gradient step (potential -> forward keeping states every 20 slices ->
    # R-factor -> adjoint -> atom gradient) on 64 angles per call: the T and R
    # slots of every slice take about 2.3 GB per pair at this size, 145 GB of
    # the 288 GB of HBM for the call (16 pairs per call: 22 points/s; 100: 37)
    ga = 64
    gw = dataclasses.replace(wl, theta0=wl.theta0[::256 // ga][:ga])
    pg = api.plan_for(gw, stepper="rk6", checkpoint_every=20)
    atoms = api.atoms_for(gw, dev)
    ag = api.angles_for(gw, dev)
    torch.cuda.empty_cache()  # the earlier variants' cached blocks, before the large workspace
    ws = pg.workspace(dev)
    tgt = torch.from_numpy(np.random.default_rng(37).uniform(0.0, 0.3, size=pg.n_pairs)).to(dev)

    def gstep():
        Ug = pg.potential(atoms)
        og = pg.forward(Ug, ag, workspace=ws)
        _, dI = api.rfactor(og["intensity"], tgt)
        return og, pg.potential_backward(atoms, pg.backward(Ug, ag, dI, ws))
    gstep()
    torch.cuda.synchronize()
    e0.record(stream)
    og, grad = gstep()
    e1.record(stream)
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1)
    res["gradient"] = {"pairs": pg.n_pairs, "checkpoint_every": 20, "xl_group": pg.info.xl_group,
                       "ms_per_step": round(gms, 1),
                       "value": round(pg.n_pairs / (gms / 1e3), 3), "unit": "points/s (gradient step)",
                       "workspace_gb": round((pg.info.fwd_workspace + pg.info.bwd_workspace) / 1e9, 1),
                       "invalid_pairs": invalid_pairs(og["intensity"], og["status"], wl.absorption),
                       "gradient_finite": bool(torch.isfinite(grad).all().item())}
    print(f"[n199] gradient step, {pg.n_pairs} pairs: {gms:.1f} ms", file=sys.stderr, flush=True)
    del pg, ws
    torch.cuda.empty_cache()
    if cpu:
        import multiprocessing as mp
        cores = min(16, os.cpu_count() or 1)
        part = 100
        jobs = [("n199", (c * 256) // cores, "rk6", part) for c in range(cores)]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            times = pool.map(_cpu_worker, jobs)
        cwall = time.perf_counter() - t0
        per_pair = float(sum(times) / len(times)) * st.n_slices / part
        res["cpu_baseline"] = {"value": round(cores / per_pair, 5), "unit": "points/s", "cores": cores, "kind": "oracle",
                               "sample": f"{cores} pairs (one angle each) over the first {part} of the {st.n_slices} "
                                         f"slices, oracle forward, scaled to the whole slab: {per_pair:.1f} s per "
                                         f"pair; {cores} processes x 1 BLAS thread, {cwall:.1f} s wall"}
    return res


# ------------------------------------------- single angle, n = 521 (Sec. 4)
def n521_single(steps=2, cpu=True):
    """The paper's single-angle case at its size (n = 521 rods, one angle,
    9.91 A in 661 RK4 slices of 0.015 A; synthetic 7x7 cell): one pair on a
    group of ceil(N / 16) workgroups, the kernel for 256 < N <= 576.  The
    paper's own figure for this case (its RK4 at this step, 8 CPU cores with
    threaded BLAS) is 23.97 s, quoted as context: other hardware, other
    input."""
    import torch
    from paper_2306_00271_amd import api
    from synth import single_angle_n521

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = single_angle_n521()
    plan = api.plan_for(wl, stepper="rk4")
    U = plan.potential(api.atoms_for(wl, dev))
    ang = api.angles_for(wl, dev)
    out = plan.forward(U, ang, want_nrhst=True)
    torch.cuda.synchronize()
    print(f"[n521] warm-up forward done (group of {plan.info.xxl_group})", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = plan.forward(U, ang, want_nrhst=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = wl.structures[0]
    nr = out["n_rhst"].cpu().numpy()
    eta = out["intensity"].cpu().numpy()[0, :st.n_beams]
    fl = _flops_forward(st.n_beams, st.n_slices, 4, int(nr.sum()), 1)
    res = {"n_beams": st.n_beams, "slices": st.n_slices, "stepper": "rk4", "group": int(plan.info.xxl_group),
           "ms_per_forward": round(ms, 2), "achieved_tflops": round(fl / (ms / 1e3) / 1e12, 3),
           "n_rhst": int(nr[0]), "specular": float(f"{eta[0]:.6e}"), "sum_eta": float(f"{eta.sum():.6e}"),
           "invalid_pairs": invalid_pairs(out["intensity"], out["status"], wl.absorption),
           "paper_rk4_s_8_cpu_cores": 23.97}
    print(f"[n521] forward {ms:.1f} ms", file=sys.stderr, flush=True)
    del plan, U
    if cpu:
        import multiprocessing as mp
        threads = min(16, os.cpu_count() or 1)
        part = 40
        with mp.get_context("spawn").Pool(1) as pool:
            t = pool.map(_cpu_worker, [("n521", threads, "rk4", part)])[0]
        per_pair = t * st.n_slices / part
        res["cpu_baseline"] = {"value": round(1.0 / per_pair, 5), "unit": "points/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"the pair over the first {part} of the {st.n_slices} slices, oracle forward "
                                         f"with {threads} BLAS threads, scaled to the whole slab: {per_pair:.1f} s"}
    return res


# ------------------------------------------------------------- bulk layer
BULK_SLICES = 62   # per 3.1 A unit layer (h = 0.05 A): at 0.1 A the 61-beam stack drifts to the wrong modes


def bulk_bench(cpu=True, tol=1e-6):
    """The bulk layer under the benchmark's slab (N = 61, 128 angles, RK6):
    rheed_bulk_reflection stacks the ideal bulk's 3.1 A unit layer
    (BULK_SLICES slices) from the vacuum until R changes by at most ``tol``
    per layer, then one forward pass over the surface slab on that bulk
    (rheed_forward_bulk) beside the same pass over the vacuum."""
    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import bulk_layer, config4

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = config4(1)
    wb = bulk_layer(wl, BULK_SLICES)
    pb = api.plan_for(wb, stepper="rk6")
    Ub = pb.potential(api.atoms_for(wb, dev))
    angb = api.angles_for(wb, dev)
    pb.bulk_reflection(Ub, angb, tol=1e300, max_layers=1)  # untimed: one layer
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    res = pb.bulk_reflection(Ub, angb, tol=tol, max_layers=2000)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_bulk = e0.elapsed_time(e1)
    layers = res["layers"].cpu().numpy()
    bad = int((res["status"] != 0).sum().item()) + int((layers < 0).sum())
    n_layers = int(layers.max())

    ps = api.plan_for(wl, stepper="rk6")
    Us = ps.potential(api.atoms_for(wl, dev))
    angs = api.angles_for(wl, dev)

    def fwd_ms(**kw):
        ps.forward(Us, angs, **kw)
        torch.cuda.synchronize()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(3):
            out = ps.forward(Us, angs, **kw)
        f1.record(stream)
        torch.cuda.synchronize()
        return f0.elapsed_time(f1) / 3, out
    ms_on_bulk, out = fwd_ms(y_bottom=res["y"])
    ms_vac, vac = fwd_ms()
    d = (out["intensity"] - vac["intensity"]).abs().max().item()
    # stage products of every layer each pair ran (a lower bound on the work:
    # the transformations are left out), over the whole iteration
    N = wb.structures[0].n_beams
    fl = float(layers.clip(min=0).sum()) * BULK_SLICES * 7 * 8.0 * float(N) ** 3
    rec = {"pairs": pb.n_pairs, "unit_layer_slices": BULK_SLICES, "tol": tol, "layers_max": n_layers,
           "layers_mean": round(float(layers.mean()), 1), "ms_bulk": round(ms_bulk, 2),
           "ms_per_layer": round(ms_bulk / max(n_layers, 1), 3), "bad_pairs": bad,
           "stage_tflops": round(fl / (ms_bulk / 1e3) / 1e12, 2),
           "note": "pairs stop at their own convergence, so the last layers run few pairs on few CUs",
           "forward_on_bulk_ms": round(ms_on_bulk, 3), "forward_vacuum_ms": round(ms_vac, 3),
           "max_intensity_change_from_the_bulk": round(d, 6)}
    if cpu:
        # the oracle's unit layer at 16 angles, one per process; a pair's bulk
        # costs layers_mean of them
        import multiprocessing as mp
        cores = min(16, os.cpu_count() or 1)
        jobs = [("bulk_layer", (c * len(wl.theta0)) // cores, "rk6", 20) for c in range(cores)]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            times = pool.map(_cpu_worker, jobs)
        cwall = time.perf_counter() - t0
        per_layer = float(sum(times) / len(times))
        rec["cpu_baseline"] = {"value": round(cores / (per_layer * float(layers.mean())), 5), "unit": "pairs/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"20 unit layers of the bulk at each of {cores} angles, one angle per "
                                         f"process, mean {per_layer:.3f} s per layer; a pair's bulk takes "
                                         f"layers_mean layers; "
                                         f"{cores} processes x 1 BLAS thread, {cwall:.1f} s wall"}
        rec["value"] = round(pb.n_pairs / (ms_bulk / 1e3), 3)
        rec["unit"] = "pairs/s"
    return rec


# ------------------------------------------------- steppers: accuracy vs time
def stepper_comparison(steps=2):
    """The paper's comparison of steppers (Sec. 5: accuracy against time) on
    the N = 61 slab, 128 angles: each stepper at several slice counts, eacc
    (max over angles of the 2-norm error of the intensities over the largest
    2-norm of the reference) against RK6 at 1600 slices (h = 0.025 A), and
    the mean time of one forward call.  RK steppers run on the N <= 64
    kernels (split layout at 128 pairs), the splitting steppers (BAB and ABA
    forms of the fourth- and sixth-order compositions) on the one-workgroup
    kernel.  The reference is RK6 at 3200 slices; eacc below ~1e-9 is the
    reference's own distance from convergence."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import config2

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    base = config2()

    def run(stepper, L, reps):
        s = dataclasses.replace(base.structures[0], n_slices=L)
        w = dataclasses.replace(base, structures=[s])
        plan = api.plan_for(w, stepper=stepper)
        U = plan.potential(api.atoms_for(w, dev))
        ang = api.angles_for(w, dev)
        out = plan.forward(U, ang)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = plan.forward(U, ang)
        e1.record(stream)
        torch.cuda.synchronize()
        return out["intensity"].cpu().numpy()[:, :61], e0.elapsed_time(e1) / reps, int((out["status"] != 0).sum())

    ref, _, _ = run("rk6", 3200, 1)
    den = float(np.max(np.linalg.norm(ref, axis=1)))
    rows = []
    for stepper, Ls in (("rk4", (800, 1600, 3200)), ("rk6", (400, 800, 1600)),
                        ("sp4", (400, 800, 1600, 3200)), ("sp4a", (400, 800, 1600, 3200)),
                        ("sp6", (400, 800, 1600)), ("sp6a", (400, 800, 1600))):
        for L in Ls:
            eta, ms, bad = run(stepper, L, steps)
            e = float(np.max(np.linalg.norm(eta - ref, axis=1))) / den
            rows.append({"stepper": stepper, "slices": L, "h": round(40.0 / L, 5), "eacc": float(f"{e:.3e}"),
                         "ms": round(ms, 3), "bad_pairs": bad})
    return {"workload": "N=61 slab, 128 angles, forward", "reference": "rk6 at 3200 slices", "points": rows}


def large_source_hash():
    """sha256 of the sources the kernel for N > 64 and the one-launch queue
    kernel are built from."""
    h = hashlib.sha256()
    for f in ("rheed_forward_large.hip", "rheed_forward.hip", "rheed_forward_all.hip", "rheed_large.h", "rheed_gj.h",
              "rheed_internal.h"):
        with open(os.path.join(ROOT, "paper_2306_00271_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_probe_uneven(n_structures):
    """One forward launch of the N > 64 pairs of the uneven-N variant, one
    one-launch forward of the whole batch and one device copy of 1 GiB, for
    FETCH_SIZE / WRITE_SIZE counter runs."""
    import dataclasses
    import torch
    from paper_2306_00271_amd import api
    from synth import config3
    dev = torch.device("cuda:0")
    wl = config3(n_structures)
    w = dataclasses.replace(wl, structures=[st for st in wl.structures if st.n_beams > 64])
    plan = api.plan_for(w, stepper="rk6")
    U = plan.potential(api.atoms_for(w, dev))
    plan.forward(U, api.angles_for(w, dev))
    torch.cuda.synchronize()
    del plan, U
    whole = api.plan_for(wl, stepper="rk6")
    assert whole.info.queue
    Uw = whole.potential(api.atoms_for(wl, dev))
    whole.forward(Uw, api.angles_for(wl, dev))
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 8, "source_sha256": large_source_hash(),
                      "kernels": ["forward_large_kernel<1>", "forward_queue_kernel<1>"],
                      "pairs": [len(w.structures) * len(w.theta0), whole.n_pairs]}))


def xl_source_hash():
    """sha256 of the sources the kernel for 128 < N <= 256 is built from."""
    h = hashlib.sha256()
    for f in ("rheed_forward_xl.hip", "rheed_forward_large.hip", "rheed_forward.hip", "rheed_forward_all.hip",
              "rheed_large.h", "rheed_gj.h", "rheed_internal.h"):
        with open(os.path.join(ROOT, "paper_2306_00271_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_probe_n199():
    """One forward launch of one structure of the N = 199 workload (256
    pairs, one workgroup each) and one device copy of 1 GiB, for FETCH_SIZE /
    WRITE_SIZE counter runs."""
    import torch
    from paper_2306_00271_amd import api
    from synth import config5
    dev = torch.device("cuda:0")
    wl = config5(1)
    plan = api.plan_for(wl, stepper="rk6")
    U = plan.potential(api.atoms_for(wl, dev))
    plan.forward(U, api.angles_for(wl, dev))
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 8, "source_sha256": xl_source_hash(),
                      "kernel": "forward_xl_kernel<1, false>", "pairs": plan.n_pairs}))


# -------------------------------------------------------------------- bench
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["fwd", "fwd+adj", "uneven", "steppers", "bulk", "fp32", "wide-grad", "n199",
                                       "n521"],
                    default="fwd+adj",
                    help="uneven: only the uneven-N batched forward variant; steppers: only the accuracy-vs-time "
                         "comparison of the steppers; bulk: only the bulk-layer variant; fp32, wide-grad, n199, "
                         "n521: only that variant; each as its own JSON line")
    ap.add_argument("--structures", type=int, default=1, help="structures in the batch (128 angles each)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-per-angle", action="store_true",
                    help="skip timing the plain per-angle form (the same step one (structure, angle) pair at a time)")
    ap.add_argument("--checkpoint-every", type=int, default=CHECKPOINT_EVERY,
                    help="slices between states kept for the adjoint (the gradient workload keeps every 20th)")
    ap.add_argument("--uneven-structures", type=int, default=16,
                    help="structures of the uneven-N batched forward variant (64 angles each; 0 skips it)")
    ap.add_argument("--no-bulk", action="store_true", help="skip the bulk-layer variant")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run one forward launch and a 1 GiB copy for HBM counter runs, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every box in this setup has a single MI355X; "
              "pairs are independent and would shard across GPUs, each GPU running its share of the (structure, angle) pairs.", file=sys.stderr)
        sys.exit(2)
    if args.traffic_probe and args.mode == "n199":
        traffic_probe_n199()
        return
    if args.traffic_probe:
        if args.mode == "uneven":
            traffic_probe_uneven(max(1, args.uneven_structures))
        else:
            traffic_probe(args.checkpoint_every)
        return
    if args.mode == "steppers":
        print(json.dumps({"stepper_comparison": stepper_comparison(steps=args.steps)}))
        return
    if args.mode == "bulk":
        print(json.dumps({"bulk_layer": bulk_bench(cpu=not args.no_cpu)}))
        return
    if args.mode == "fp32":
        print(json.dumps({"fp32_stages_forward": fp32_stages(steps=args.steps)}))
        return
    if args.mode == "wide-grad":
        print(json.dumps({"gradient_n121": wide_gradient(steps=args.steps)}))
        return
    if args.mode == "n199":
        print(json.dumps({"n199_forward": n199_forward(steps=args.steps, cpu=not args.no_cpu)}))
        return
    if args.mode == "n521":
        print(json.dumps({"n521_single_angle": n521_single(steps=args.steps, cpu=not args.no_cpu)}))
        return
    if args.mode == "uneven":
        print(json.dumps({"uneven_n_forward": uneven_forward(max(1, args.uneven_structures), steps=args.steps,
                                                             cpu=not args.no_cpu)}))
        return

    import numpy as np
    import torch
    from paper_2306_00271_amd import api
    from synth import config4

    dev = torch.device("cuda:0")
    wl = config4(args.structures)
    stepper = "rk6"
    tplan = api.plan_for(dataclasses_replace(wl, wl.target), stepper=stepper)
    angles = api.angles_for(wl, dev)
    atoms = api.atoms_for(wl, dev)
    tatoms = api.atoms_for(wl, dev, structures=wl.target)
    # target curve (setup, not timed): specular intensities of the perturbed slabs
    tU = tplan.potential(tatoms)
    target = tplan.forward(tU, angles)["intensity"][:, 0].contiguous()
    del tplan, tU
    do_adj = args.mode == "fwd+adj"
    stream = torch.cuda.current_stream()

    def measure(every):
        """(plan, ms per step, forward event pairs, last forward output, wall s)"""
        plan = api.plan_for(wl, stepper=stepper, checkpoint_every=every)
        ws = plan.workspace(dev) if do_adj else None
        fwd_events = []

        def step(record):
            U = plan.potential(atoms)
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            out = plan.forward(U, angles, workspace=ws, want_nrhst=True)
            if record:
                e1.record(stream)
                fwd_events.append((e0, e1))
            if do_adj:
                loss, dI = api.rfactor(out["intensity"], target)
                dU = plan.backward(U, angles, dI, ws)
                plan.potential_backward(atoms, dU)
            return out

        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        wall0 = time.perf_counter()
        for _ in range(args.steps):
            out = step(True)
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        return plan, t0.elapsed_time(t1) / args.steps, fwd_events, out, wall

    every = args.checkpoint_every if do_adj else 1
    plan, ms, fwd_events, out, wall = measure(every)
    n_pairs = plan.n_pairs
    split = plan.split
    value = n_pairs / (ms / 1e3)
    status = out["status"].cpu().numpy()
    nrhst = int(out["n_rhst"].sum().item())
    N = int(wl.structures[0].n_beams)
    L = int(wl.structures[0].n_slices)
    stages = 7 if stepper == "rk6" else 4
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in fwd_events]))
    fl = _flops_forward(N, L, stages, nrhst, n_pairs)
    achieved = fl / (fwd_ms / 1e3) / 1e12
    # counters were taken on the single-structure launch with state saving
    traffic = traffic_from_profile(split) if (do_adj and args.structures == 1 and every == CHECKPOINT_EVERY) else None
    # the published peak is the reference; the probe gives the rate this device
    # actually reaches with register-resident operands
    measured_peak = api.mfma_f64_peak()
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": MFMA_FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / MFMA_FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": kernel_name(split), "kernel_ms": round(fwd_ms, 4), "flops_per_launch": fl,
                "measured_peak": round(measured_peak, 2), "frac_of_measured": round(achieved / measured_peak, 4)}

    cpu = None
    if not args.no_cpu:
        cores = min(16, os.cpu_count() or 1)
        n_coords = 3 * len(wl.structures[0].grad_atoms)
        rate, per_pass, cwall, rate1, alone = cpu_baseline(stepper, len(wl.theta0), n_coords, cores, args.mode)
        if do_adj:
            sample = (f"{2 * cores} (structure, angle) pairs of this workload, two per process at different angles, "
                      f"each one tangent-linear pass of the oracle (forward plus the derivative along one atom "
                      f"coordinate), mean {per_pass:.2f} s per pass; a point's gradient takes {n_coords} passes "
                      f"({n_coords // 3} atoms x 3 coordinates), so value = {cores} / ({n_coords} x "
                      f"{per_pass:.2f} s); {cores} processes x 1 BLAS thread, {cwall:.1f} s wall")
        else:
            sample = (f"{2 * cores} (structure, angle) pairs of this workload, two per process at different angles, "
                      f"oracle forward, mean {per_pass:.2f} s per pair; {cores} processes x 1 BLAS thread, "
                      f"{cwall:.1f} s wall")
        cpu = {"value": round(rate, 5), "unit": "points/s", "cores": cores, "kind": "oracle", "sample": sample,
               "value_1core": round(rate1, 6), "sample_1core": f"one pass alone in one process: {alone:.2f} s",
               "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}

    variants = None
    if do_adj and every != 1:
        del plan
        _, ms1, _, _, _ = measure(1)
        variants = {"checkpoint_every_1": {"value": round(n_pairs / (ms1 / 1e3), 3), "ms_per_step": round(ms1, 4)}}
    if not args.no_per_angle and args.structures == 1:
        # the plain per-angle GPU form: the same kernels on one pair at a time,
        # the table gradient summed over the angles, one atom gradient at the end
        import dataclasses
        one = dataclasses.replace(wl, theta0=wl.theta0[:1])
        p1 = api.plan_for(one, stepper=stepper, checkpoint_every=every if do_adj else 1)
        ws1 = p1.workspace(dev) if do_adj else None
        ang_all = angles

        def per_angle_step():
            U = p1.potential(atoms)
            dU_sum = torch.zeros_like(U) if do_adj else None
            for k in range(ang_all.shape[0]):
                a1 = ang_all[k:k + 1]
                o1 = p1.forward(U, a1, workspace=ws1)
                if do_adj:
                    _, dI1 = api.rfactor(o1["intensity"], target[k:k + 1])
                    dU_sum += p1.backward(U, a1, dI1, ws1)
            if do_adj:
                p1.potential_backward(atoms, dU_sum)

        per_angle_step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        per_angle_step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_pa = e0.elapsed_time(e1)
        variants = variants or {}
        variants["per_angle"] = {"value": round(n_pairs / (ms_pa / 1e3), 3), "ms_per_step": round(ms_pa, 3),
                                 "speedup_of_batched": round(ms_pa / ms, 2)}

    if args.uneven_structures > 0:
        variants = variants or {}
        variants["uneven_n_forward"] = uneven_forward(args.uneven_structures, cpu=not args.no_cpu)
    if not args.no_bulk and args.structures == 1:
        variants = variants or {}
        variants["bulk_layer"] = bulk_bench(cpu=not args.no_cpu)
    if args.structures == 1:
        variants = variants or {}
        variants["fp32_stages_forward"] = fp32_stages()
        variants["gradient_n121"] = wide_gradient()
        variants["n199_forward"] = n199_forward(cpu=not args.no_cpu)
        variants["n521_single_angle"] = n521_single(cpu=not args.no_cpu)

    rec = {
        "metric": "rocking-curve points (structure x angle)/s at N=61 FP64; " +
                  ("fwd+adjoint" if do_adj else "forward only"),
        "value": round(value, 3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name + ("" if do_adj else "-forward"), "structures": len(wl.structures),
                   "angles": len(wl.theta0), "n_beams": N, "slices": L, "stepper": stepper,
                   "pairs": n_pairs, "layout": "split" if split else "whole",
                   "checkpoint_every": every if do_adj else None, "rhst_per_pair": round(nrhst / n_pairs, 2),
                   "invalid_pairs": invalid_pairs(out["intensity"], out["status"], wl.absorption),
                   "wall_s": round(wall, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(rec))


def dataclasses_replace(wl, structures):
    import dataclasses
    return dataclasses.replace(wl, structures=structures, target=None)


if __name__ == "__main__":
    main()
