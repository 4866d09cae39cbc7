"""Full-slip box faces (specular reflection, the outer walls of the
street-canyon setup of Sec. 3.2) on the GPU against the FP64 oracle, through
the C ABI: a box with full-slip y and z faces from a random non-equilibrium
state (population by population, both parities), the urban canopy with
full-slip side and top faces over a wall-modeled ground, and the adjoint's
transpose test across full-slip faces."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, moment_errors, oracle_for, rel_maxnorm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("q,collision", [(19, 0), (27, 0), (27, 1)])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_slip_box_random_state(gpu, q, collision, storage, tol):
    shape = (67, 9, 7)   # two tiles and a ragged tail in x
    N = int(np.prod(shape))
    c, w, _ = O.velocity_set(q)
    f0 = I.random_state(w, N, seed_offset=60 + q, amp=0.05)
    case = I.Case(name="slipbox", q=q, shape=shape, periodic=(1, 0, 0), tau0=0.57, cs_smag=0.12,
                  force=(2e-5, 0.0, 0.0), collision=collision, slip=0b111100)
    announce(f"slip box q={q} collision={collision} {storage}")
    lat = gpu.Lattice(case, storage=storage)
    lat.set_populations(torch.as_tensor(f0))
    orc = oracle_for(case)
    orc.set_populations(f0)
    # populations (deviations from the weights) after one and five steps,
    # while the random non-equilibrium is still of its initial size
    for n in (1, 4):
        lat.step(n)
        orc.step(n)
        f = lat.populations().cpu().numpy().astype(np.float64)
        err = rel_maxnorm(f - w[:, None], orc.populations() - w[:, None])
        announce(f"slip box q={q} {storage} after {lat.steps}: {err:.3e}")
        assert err <= tol, (lat.steps, err)
    # after 41 steps the non-equilibrium has relaxed by orders of magnitude:
    # moments against the fields' max-norms (the bars of the other parity
    # tests), populations against the populations' max-norm
    lat.step(36)
    orc.step(36)
    rho, u = (t.cpu().numpy().astype(np.float64) for t in lat.moments())
    orho, ou = orc.moments()
    e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
    e_f = rel_maxnorm(lat.populations().cpu().numpy(), orc.populations())
    announce(f"slip box q={q} {storage} after 41: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e} f {e_f:.3e}")
    assert e_rho <= tol and e_u <= tol, (e_rho, e_u)
    if storage == "f64":
        assert e_drho <= 1e-10 and e_f <= 1e-13, (e_drho, e_f)


@pytest.mark.parametrize("storage,tol,steps", [("f64", 1e-12, 41), ("f32", 1e-5, 100)])
def test_urban_slip_walls(gpu, storage, tol, steps):
    case = I.urban(nx=160, ny=72, nz=48, q=27, tau0=0.5003, fringe_len=24, x_lo=16, x_hi=110, h_mean=14.0,
                   h_max=30, fp_lo=6, fp_hi=20, slip_walls=True)
    case.collision = 1
    announce(f"urban slip walls {storage} {steps} steps")
    for wd in ("case", None):   # generator's wall distance, then the library's own
        lat = gpu.Lattice(case, storage=storage, wall_dist=wd)
        lat.step(steps)
        rho, u = (t.cpu().numpy().astype(np.float64) for t in lat.moments())
        if wd == "case":
            orc = oracle_for(case, steps)
            orho, ou = orc.moments()
            info = orc.wall_info()
        e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
        announce(f"urban slip {storage} wall_dist={wd}: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e}")
        assert e_rho <= tol and e_u <= tol, (e_rho, e_u)
        g = lat.wall_records()
        np.testing.assert_array_equal(g["cells"], info["cells"])
        # no wall cell on the full-slip faces' own rows (only ground and buildings)
        nx, ny, nz = case.shape
        zc = g["cells"] // (nx * ny)
        assert (zc < nz - 1).all()


@pytest.mark.parametrize("parity", [0, 1])
def test_slip_adjoint_transpose(gpu, parity):
    """<L v, w> from the oracle's tangent step equals <v, L^T w> from one GPU
    reverse step on the porous channel with full-slip z faces, FP64."""
    case = I.porous_channel(shape=(20, 12, 8))
    case.slip = 0b110000
    q, N = case.q, case.ncells
    c, w, _ = O.velocity_set(q)
    f_n = I.random_state(w, N, seed_offset=71, amp=0.05)
    rng = np.random.default_rng(72)
    v = rng.standard_normal((q, N))
    dphi = rng.standard_normal(N)
    wv = rng.standard_normal((q, N))
    orc = oracle_for(case, tangent=True)
    orc.set_populations(f_n, v)
    orc.set_phi_tangent(dphi)
    orc.step(1)
    _, Lv = orc.populations(with_tangent=True)
    lhs = float((Lv * wv).sum())
    lat = gpu.Lattice(case, storage="f64")
    if parity:
        lat.step(1)
    lat.set_populations(torch.as_tensor(f_n))
    snap = lat.new_state_buffer()
    lat.save_state(snap)
    lat.step(1)
    lam = lat.new_adjoint()
    gpu.lbm_adjoint_from_natural(lat.ctx, torch.as_tensor(wv, device="cuda"), lam)
    lat.load_state(snap)
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    gpu.lbm_adjoint_step(lat.ctx, lam, grad)
    nat = lat.new_natural()
    gpu.lbm_adjoint_to_natural(lat.ctx, lam, nat)
    lat.sync()
    rhs = float((v * nat.cpu().numpy()).sum() + (dphi * grad.cpu().numpy()).sum())
    announce(f"slip transpose parity {parity}: <Lv,w> {lhs:.15e} <v,L^T w> {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
