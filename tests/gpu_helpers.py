"""Shared helpers of the GPU parity tests: run the same seeded case on the
oracle (FP64 CPU) and through the HIP library's C ABI, and compare."""
import sys

import numpy as np

import oracle as O


def oracle_for(case, steps=0, tangent=False, wall_dist="case"):
    p = O.make_params(case.q, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force, wall_model=case.wall_model, kappa=case.kappa, E=case.E,
                      fringe_len=case.fringe_len, u_ref=case.u_ref, z0=case.z0, lid=case.lid,
                      collision=case.collision, fd_weight=case.fd_weight, open_x=case.open_x,
                      rho_out=case.rho_out, slip=getattr(case, "slip", 0))
    wd = case.wall_dist if isinstance(wall_dist, str) else wall_dist
    s = O.Oracle(p, mask=case.mask, wall_dist=wd, porosity=case.porosity, rho0=case.rho0, u0=case.u0,
                 tangent=tangent)
    if steps:
        s.step(steps)
    return s


def rel_maxnorm(a, b, ref=None):
    """max |a - b| / max |ref| (ref defaults to b)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = np.abs(b if ref is None else ref).max()
    return float(np.abs(a - b).max() / max(r, 1e-300))


def moment_errors(gpu_rho, gpu_u, orc_rho, orc_u):
    """Errors of density and velocity, each relative to the max-norm of the
    oracle's field, and of the density deviation rho - 1 relative to its own
    max-norm (a stricter measure: the oracle sums full populations, so its
    rho - 1 carries absolute rounding of order 1e-15 per step)."""
    e_rho = rel_maxnorm(gpu_rho, orc_rho)
    e_u = rel_maxnorm(gpu_u, orc_u)
    e_drho = rel_maxnorm(gpu_rho - 1.0, orc_rho - 1.0)
    return e_rho, e_u, e_drho


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()
