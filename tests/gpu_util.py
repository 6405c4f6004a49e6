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
