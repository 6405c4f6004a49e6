"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
binding and the CPU oracle on the same seeded synthetic inputs."""
import numpy as np

from oracle import driver


def gpu_forward(wl, stepper=None, threshold=1000.0, convention="flux", want_rho=False, structures=None,
                layout="auto"):
    import torch
    from paper_2306_00271_amd import api
    dev = torch.device("cuda:0")
    if structures is not None:
        import dataclasses
        wl = dataclasses.replace(wl, structures=structures)
    plan = api.plan_for(wl, stepper=stepper, threshold=threshold, convention=convention, layout=layout)
    atoms = api.atoms_for(wl, dev)
    U = plan.potential(atoms)
    out = plan.forward(U, api.angles_for(wl, dev), want_rho=want_rho, want_nrhst=True)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["plan"] = plan
    res["U"] = U.cpu().numpy()
    return res


def oracle_forward(wl, s_idx=0, angle_idx=None, stepper=None, threshold=1000.0, convention="flux"):
    eta, rho, nr = driver.rocking_curve(wl, s_idx=s_idx, angle_idx=angle_idx, stepper=stepper,
                                        threshold=threshold, convention=convention)
    return eta, rho, nr


def eacc(eta, ref):
    """Paper's eacc form: max over angles of ||eta - ref||_2 / max over angles of ||ref||_2."""
    num = np.max(np.linalg.norm(eta - ref, axis=1))
    den = np.max(np.linalg.norm(ref, axis=1))
    return num / den


def physical(eta, absorption):
    """Per-angle validity of a rocking curve (Sec. 2.1): finite, every
    eta_j >= 0, and with absorption (alpha > 0) sum_j eta_j <= 1 + 1e-9, since
    the reflected flux cannot exceed the incident flux.  A discretisation off
    the physical solution (a step outside the stepper's accurate range on the
    most evanescent rods) fails it.  Returns a boolean per angle."""
    eta = np.atleast_2d(np.asarray(eta, dtype=np.float64))
    ok = np.all(np.isfinite(eta), axis=1) & np.all(eta >= 0.0, axis=1)
    if absorption > 0.0:
        ok &= eta.sum(axis=1) <= 1.0 + 1e-9
    return ok


def _tangent_unit(args):
    """Worker: the oracle's tangent-linear derivative of the R-factor along
    one atom coordinate (structure 0)."""
    from threadpoolctl import threadpool_limits
    wl, ia, c, target, angle_idx, stepper = args
    d = np.zeros_like(np.asarray(wl.structures[0].atoms, dtype=np.float64))
    d[ia, c] = 1.0
    with threadpool_limits(1):   # one BLAS thread per process
        return driver.rfactor_directional(wl, 0, d, target, angle_idx=angle_idx, stepper=stepper)[1]


def oracle_atom_gradient(wl, target, coords, angle_idx=None, stepper=None, processes=8):
    """dR/d(atom coordinate) for every (atom, axis) in ``coords``, one
    tangent-linear pass of the oracle per coordinate, in host processes."""
    import multiprocessing as mp
    jobs = [(wl, ia, c, np.asarray(target), angle_idx, stepper) for ia, c in coords]
    with mp.get_context("spawn").Pool(min(processes, len(jobs))) as pool:
        return np.array(pool.map(_tangent_unit, jobs))


def assert_entrywise(got, ref, rel=1e-8, floor=1e-6, what=""):
    """Every entry within rel of the reference, relative to the entry itself
    where it is above floor * max|ref| and to floor * max|ref| below."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max())
    err = np.abs(got - ref) / scale
    k = int(np.argmax(err))
    print(f"[adjoint] {what}: {ref.size} entries, worst rel err {err.flat[k]:.3e} at {k} "
          f"(got {got.flat[k]:.6e}, ref {ref.flat[k]:.6e})", flush=True)
    assert err.max() <= rel
