"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 storage within 1e-12 of the oracle (density and velocity, each
relative to the max-norm of the oracle's field; the density deviation
rho - 1 within 1e-10 of its own max-norm, the oracle's rounding floor for a
sum of full populations); FP32
deviation storage within 1e-5 (density relative to its max-norm, velocity
relative to its max-norm) after 100 steps; FP16 deviation storage reported
(bounded loosely, its error is a measured quantity, not a target).
Sizes span several tiles and ragged tails in x and y.
"""
import numpy as np
import pytest

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, moment_errors, oracle_for, rel_maxnorm

pytestmark = pytest.mark.gpu


def _run_both(lbm, case, steps, storage, wall_dist="case"):
    announce(f"{case.name} q={case.q} storage={storage} steps={steps}")
    lat = lbm.Lattice(case, storage=storage, wall_dist=wall_dist)
    lat.step(steps)
    rho, u = lat.moments()
    orc = oracle_for(case, steps)
    orho, ou = orc.moments()
    return lat, orc, rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64), orho, ou


@pytest.mark.parametrize("q", [19, 27])
def test_tgv_fp64_parity(gpu, q):
    case = I.taylor_green(32, u0=0.05, q=q, tau0=0.6, cs_smag=0.1)
    lat, orc, rho, u, orho, ou = _run_both(gpu, case, 100, "f64")
    e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
    msg = f"tgv q={q} f64: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e}"
    announce(msg)
    assert e_rho <= 1e-12 and e_u <= 1e-12 and e_drho <= 1e-10, msg
    f = lat.populations().cpu().numpy()
    e_f = rel_maxnorm(f, orc.populations())
    assert e_f <= 1e-13, e_f


@pytest.mark.parametrize("q", [19, 27])
def test_tgv_fp32_fp16(gpu, q):
    case = I.taylor_green(32, u0=0.05, q=q, tau0=0.6, cs_smag=0.1)
    _, orc, rho, u, orho, ou = _run_both(gpu, case, 100, "f32")
    e_rho = rel_maxnorm(rho, orho)
    e_u = rel_maxnorm(u, ou)
    msg = f"tgv q={q} f32: rho {e_rho:.3e} u {e_u:.3e}"
    announce(msg)
    assert e_rho <= 1e-5 and e_u <= 1e-5, msg
    _, _, rho, u, _, _ = _run_both(gpu, case, 100, "f16")
    e_rho16 = rel_maxnorm(rho, orho)
    e_u16 = rel_maxnorm(u, ou)
    msg = f"tgv q={q} f16: rho {e_rho16:.3e} u {e_u16:.3e}"
    announce(msg)
    assert e_rho16 <= 1e-3 and e_u16 <= 5e-2, msg


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_ragged_random_state(gpu, storage, tol):
    """A generic non-equilibrium state on a 263x7x9 periodic box (several
    tiles plus a ragged tail in x and y), odd and even step counts, checked
    population by population."""
    q = 27
    shape = (263, 7, 9)
    N = int(np.prod(shape))
    c, w, _ = O.velocity_set(q)
    f0 = I.random_state(w, N, seed_offset=11, amp=0.05)
    case = I.Case(name="ragged", q=q, shape=shape, periodic=(1, 1, 1), tau0=0.58, cs_smag=0.12,
                  force=(2e-5, -1e-5, 5e-6))
    lat = gpu.Lattice(case, storage=storage)
    import torch
    lat.set_populations(torch.as_tensor(f0))
    p = O.make_params(q, shape, tau0=0.58, cs_smag=0.12, force=(2e-5, -1e-5, 5e-6))
    orc = O.Oracle(p)
    orc.set_populations(f0)
    for n in (1, 4):  # after 1 (odd layout) and 5 (odd) and then 6 (even)
        lat.step(n)
        orc.step(n)
        f = lat.populations().cpu().numpy().astype(np.float64)
        err = rel_maxnorm(f - w[:, None], orc.populations() - w[:, None])
        announce(f"ragged {storage} after {lat.steps}: {err:.3e}")
        assert err <= (1e-12 if storage == "f64" else 1e-5), (storage, lat.steps, err)
    lat.step(1)
    orc.step(1)
    rho, u = lat.moments()
    orho, ou = orc.moments()
    e_u = rel_maxnorm(u.cpu().numpy(), ou)
    assert e_u <= tol, e_u


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("wall_model", [0, 1])
def test_channel_walls_fp64(gpu, q, wall_model):
    """Walls outside z: halfway bounce-back, with and without the Spalding
    wall model; 70x10x9 with a seeded perturbation, 51 steps (odd)."""
    case = I.channel(70, 10, 9, q=q, utau=0.01, nu=1e-3, tau0=0.503, cs_smag=0.1, amp=0.01,
                     wall_model=wall_model)
    lat, orc, rho, u, orho, ou = _run_both(gpu, case, 51, "f64")
    e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
    msg = f"channel q={q} wm={wall_model}: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e}"
    announce(msg)
    assert e_rho <= 1e-12 and e_u <= 1e-12 and e_drho <= 1e-10, msg
    if wall_model:
        g = lat.wall_records()
        o = orc.wall_info()
        np.testing.assert_array_equal(g["cells"], o["cells"])
        np.testing.assert_array_equal(g["refs"], o["refs"])
        np.testing.assert_allclose(g["utau"], o["utau"], rtol=1e-11)
        np.testing.assert_allclose(g["G"], o["G"], rtol=1e-10)


@pytest.mark.parametrize("storage,tol,steps", [("f64", 1e-12, 41), ("f32", 1e-5, 100)])
def test_urban_crop(gpu, storage, tol, steps):
    """Urban canopy crop: random buildings, wall-modeled ground and faces
    (D3Q27 diagonal wall cells), fringe, lid; the GPU side runs once with the
    generator's wall distances and once with the library's own voxel
    distance routine."""
    case = I.urban(nx=160, ny=72, nz=48, q=27, tau0=0.5003, fringe_len=24, x_lo=16, x_hi=110,
                   h_mean=14.0, h_max=36, fp_lo=6, fp_hi=16)
    orc = oracle_for(case, steps)
    orho, ou = orc.moments()
    for wd in ("case", None):
        announce(f"urban {storage} wd={'lib' if wd is None else 'case'}")
        lat = gpu.Lattice(case, storage=storage, wall_dist=wd)
        lat.step(steps)
        rho, u = (t.cpu().numpy().astype(np.float64) for t in lat.moments())
        e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
        msg = (f"urban {storage}: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e} "
               f"walls={len(lat.wall_records()['cells'])}")
        announce(msg)
        assert e_rho <= tol and e_u <= tol, msg
        if storage == "f64":
            assert e_drho <= 1e-10, msg


def test_porosity_fp64(gpu):
    case = I.porous_channel(shape=(40, 24, 12))
    lat, orc, rho, u, orho, ou = _run_both(gpu, case, 30, "f64")
    e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
    msg = f"porous f64: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e}"
    announce(msg)
    assert e_rho <= 1e-12 and e_u <= 1e-12 and e_drho <= 1e-10, msg
    J = lat.objective(case.extra["planes"])
    Jo, _ = orc.objective(case.extra["planes"])
    assert abs(J - Jo) <= 1e-12 * abs(Jo), (J, Jo)


def test_porosity_fp32(gpu):
    case = I.porous_channel(shape=(40, 24, 12))
    lat, orc, rho, u, orho, ou = _run_both(gpu, case, 100, "f32")
    e_rho, e_u = rel_maxnorm(rho, orho), rel_maxnorm(u, ou)
    msg = f"porous f32: rho {e_rho:.3e} u {e_u:.3e}"
    announce(msg)
    assert e_rho <= 1e-5 and e_u <= 1e-5, msg
    J = lat.objective(case.extra["planes"])
    Jo, _ = orc.objective(case.extra["planes"])
    announce(f"porous f32 objective rel err {abs(J - Jo) / abs(Jo):.3e}")
    assert abs(J - Jo) <= 1e-5 * abs(Jo), (J, Jo)


def test_conservation_and_diagnostics(gpu):
    case = I.taylor_green(24, u0=0.05, q=27, cs_smag=0.1)
    lat = gpu.Lattice(case, storage="f64")
    d0 = lat.diagnostics()
    orc = oracle_for(case)
    do = orc.diagnostics()
    # mass to 1e-13 relative; momenta (zero net for this flow) to rounding of the sums
    assert abs(d0[0] - do[0]) <= 1e-13 * do[0], (d0, do)
    assert np.abs(d0[1:] - do[1:]).max() <= 1e-12, (d0, do)
    lat.step(100)
    d1 = lat.diagnostics()
    announce(f"diagnostics start {d0} after 100 steps {d1}")
    assert abs(d1[0] - d0[0]) <= 1e-13 * d0[0], (d0, d1)
    assert np.abs(d1[1:] - d0[1:]).max() <= 1e-13 * d0[0], (d0, d1)
    # deterministic: the same run twice gives identical bits
    lat2 = gpu.Lattice(case, storage="f64")
    lat2.step(100)
    assert np.array_equal(lat2.diagnostics(), d1)
    assert np.array_equal(lat2.populations().cpu().numpy(), lat.populations().cpu().numpy())


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_save_load_resume_bitwise(gpu, storage):
    case = I.channel(64, 8, 12, q=19, utau=0.01, nu=1e-3, tau0=0.503, wall_model=1)
    a = gpu.Lattice(case, storage=storage)
    a.step(7)
    buf = a.new_state_buffer()
    a.save_state(buf)
    a.step(7)
    fa = a.populations().cpu().numpy()
    b = gpu.Lattice(case, storage=storage)
    b.load_state(buf)
    assert b.steps == 7
    b.step(7)
    assert np.array_equal(b.populations().cpu().numpy(), fa)


def test_error_paths(gpu):
    case = I.taylor_green(16, u0=0.35, q=19, tau0=0.5001, cs_smag=0.0)
    lat = gpu.Lattice(case, storage="f32")
    with pytest.raises(gpu.LbmError) as e:
        for _ in range(40):
            lat.step(10)
            lat.sync()
    assert e.value.code == gpu.ENONFINITE
    c2 = I.channel(16, 4, 6, q=19, wall_model=1)
    c2.wall_dist = np.zeros(c2.ncells)
    with pytest.raises(gpu.LbmError) as e:
        gpu.Lattice(c2, storage="f32")
    assert e.value.code == gpu.EINVAL
    # a friction Reynolds number far outside the wall law's range: the
    # laminar start already needs exp(kappa U / u_tau) beyond exp(700), so
    # the Newton solve refuses; the oracle refuses the same step
    c3 = I.channel(16, 4, 6, q=19, utau=0.01, nu=1e-9, tau0=0.5 + 3e-9, cs_smag=0.1, amp=0.0)
    c3.u0[0] = 0.1
    lat = gpu.Lattice(c3, storage="f64")
    lat.step(1)
    with pytest.raises(gpu.LbmError) as e:
        lat.sync()
    assert e.value.code == gpu.ENEWTON
    with pytest.raises(O.OracleError) as e:
        oracle_for(c3, 1)
    assert e.value.code == O.ENEWTON


@pytest.mark.parametrize("q,storage,tol", [(19, "f64", 1e-12), (27, "f64", 1e-12), (19, "f32", 1e-5)])
def test_lid_driven_cavity(gpu, q, storage, tol):
    """Lid-driven cavity (every face a halfway bounce-back wall, the top plane
    held at the lid equilibrium) on a 140x20x18 box: 80 steps from rest."""
    case = I.cavity((140, 20, 18), q=q)
    _, orc, rho, u, orho, ou = _run_both(gpu, case, 80, storage)
    e_rho, e_u, e_drho = moment_errors(rho, u, orho, ou)
    msg = f"cavity q={q} {storage}: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e}"
    announce(msg)
    assert e_rho <= tol and e_u <= tol, msg
    if storage == "f64":
        assert e_drho <= 1e-10, msg
