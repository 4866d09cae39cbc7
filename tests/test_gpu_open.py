"""Parity of the open x faces (regularized velocity inlet, fixed-pressure
outlet; Sec. 2.2.2, Sec. 3.2) of the HIP path with the FP64 oracle, through
the C ABI.  Same bars as the other parity tests: FP64 storage within 1e-12
of the oracle (density and velocity relative to the oracle field's max-norm,
rho - 1 within 1e-10 of its own); FP32 within 1e-5 after 100 steps.  The
cases cover the open-face rebuild in the bulk kernel at both parities, with and without
porosity, with both collision models, next to wall-modeled ground and
buildings (whose reference cells may lie on the inlet plane), the fringe
before the outlet, the lid above both faces, and the vortex method on the
inlet."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, moment_errors, oracle_for

pytestmark = pytest.mark.gpu


def _run_both(lbm, case, steps, storage):
    announce(f"open {case.name} q={case.q} storage={storage} collision={case.collision} steps={steps}")
    lat = lbm.Lattice(case, storage=storage, wall_dist="case" if case.wall_dist is not None else None)
    lat.step(steps)
    rho, u = lat.moments()
    orc = oracle_for(case, steps, wall_dist=case.wall_dist)
    orho, ou = orc.moments()
    return lat, rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64), orho, ou


def _check(msg, errs, tol):
    e_rho, e_u, e_drho = errs
    announce(f"{msg}: rho {e_rho:.3e} u {e_u:.3e} drho {e_drho:.3e}")
    assert e_rho <= tol and e_u <= tol, msg
    if tol <= 1e-12:
        assert e_drho <= 1e-10, msg


def _stream(q, shape, U, collision=0):
    nx, ny, nz = shape
    N = nx * ny * nz
    u0 = np.zeros((3, N))
    u0[0] = U
    return I.Case(name=f"stream{nx}x{ny}x{nz}", q=q, shape=shape, periodic=(0, 1, 1), tau0=0.6, cs_smag=0.1,
                  u_ref=U, z0=1.0, collision=collision, open_x=1, rho_out=1.0, u0=u0)


@pytest.mark.parametrize("q,collision", [(19, 0), (27, 1)])
def test_open_uniform_stream(gpu, q, collision):
    """nz = 1: the inflow profile is the constant u_ref, and the stream between
    the faces stays uniform; the smallest box (nx = 3) has one interior plane."""
    for shape in ((12, 3, 1), (3, 5, 1)):
        case = _stream(q, shape, 0.04, collision)
        lat, rho, u, orho, ou = _run_both(gpu, case, 41, "f64")
        _check(f"stream {shape} q={q} f64", moment_errors(rho, u, orho, ou), 1e-12)
        x = np.arange(case.ncells) % shape[0]
        inner = (x > 0) & (x < shape[0] - 1)
        np.testing.assert_allclose(rho[inner], 1.0, rtol=0, atol=1e-13)
        np.testing.assert_allclose(u[0, inner], 0.04, rtol=0, atol=1e-13)


@pytest.mark.parametrize("storage,tol,steps", [("f64", 1e-12, 301), ("f32", 1e-5, 100)])
def test_open_laminar_channel(gpu, storage, tol, steps):
    """Log-law inlet, pressure outlet, bounce-back walls outside z (no wall
    model): the developing laminar channel of the oracle's Poiseuille pin."""
    nx, ny, nz = 40, 1, 8
    case = I.Case(name="openchannel", q=19, shape=(nx, ny, nz), periodic=(0, 1, 0), tau0=0.8, cs_smag=0.0,
                  u_ref=0.02, z0=1.0, open_x=1, rho_out=1.0)
    _, rho, u, orho, ou = _run_both(gpu, case, steps, storage)
    _check(f"open channel {storage}", moment_errors(rho, u, orho, ou), tol)


def _urban_open(q=27, collision=0):
    case = I.urban(nx=160, ny=72, nz=48, q=q, tau0=0.5003, fringe_len=24, x_lo=16, x_hi=110, h_mean=14.0,
                   h_max=36, fp_lo=6, fp_hi=16, open_x=True)
    return dataclasses.replace(case, collision=collision)


@pytest.mark.parametrize("collision,storage,tol,steps", [(0, "f64", 1e-12, 41), (1, "f64", 1e-12, 40),
                                                         (0, "f32", 1e-5, 100), (1, "f32", 1e-5, 100)])
def test_open_urban_crop(gpu, collision, storage, tol, steps):
    """Buildings on a wall-modeled ground, fringe before the outlet, lid on
    top, inlet and outlet planes; the ground's wall cells next to the inlet
    take reference cells on the inlet plane."""
    case = _urban_open(collision=collision)
    _, rho, u, orho, ou = _run_both(gpu, case, steps, storage)
    _check(f"open urban collision={collision} {storage}", moment_errors(rho, u, orho, ou), tol)


@pytest.mark.parametrize("collision", [0, 1])
def test_open_urban_crop_d3q19(gpu, collision):
    """The same canopy with open faces on D3Q19 (FP64)."""
    case = _urban_open(q=19, collision=collision)
    _, rho, u, orho, ou = _run_both(gpu, case, 41, "f64")
    _check(f"open urban d3q19 collision={collision} f64", moment_errors(rho, u, orho, ou), 1e-12)


def test_open_urban_fp16(gpu):
    """FP16 deviation storage: reported against the oracle with a loose bound."""
    case = _urban_open()
    _, rho, u, orho, ou = _run_both(gpu, case, 100, "f16")
    e_rho, e_u, _ = moment_errors(rho, u, orho, ou)
    announce(f"open urban f16: rho {e_rho:.3e} u {e_u:.3e}")
    assert e_rho < 5e-3 and e_u < 5e-2


@pytest.mark.parametrize("q", [19, 27])
def test_open_ragged_porous(gpu, q):
    """A ragged box (x and y not multiples of the tiles) with a porosity field,
    walls outside z and a uniform start: the porous open-face kernel."""
    case = I.porous_channel(shape=(131, 5, 7), q=q)
    case = dataclasses.replace(case, name="porous_open", periodic=(0, 1, 0), force=(0.0, 0.0, 0.0), open_x=1,
                               rho_out=1.002, u_ref=0.05, z0=1.0)
    _, rho, u, orho, ou = _run_both(gpu, case, 33, "f64")
    _check(f"open porous q={q} f64", moment_errors(rho, u, orho, ou), 1e-12)


def _vortices(case, n, seed):
    nx, ny, nz = case.shape
    rng = np.random.default_rng(seed)
    yz = np.stack([rng.uniform(0, ny, n), rng.uniform(0, nz, n)], 1)
    sign = np.where(rng.uniform(size=n) < 0.5, -1, 1)
    return yz, sign


@pytest.mark.parametrize("collision,storage,tol,steps", [(0, "f64", 1e-12, 41), (1, "f64", 1e-12, 40),
                                                         (0, "f32", 1e-5, 100)])
def test_vortex_inlet_urban_crop(gpu, collision, storage, tol, steps):
    """The vortex method's perturbation on the inlet (40 seed vortices,
    intensity 0.2, size 3 cells), in the urban crop with open faces."""
    case = _urban_open(collision=collision)
    yz, sign = _vortices(case, 40, 11)
    announce(f"vortex urban collision={collision} storage={storage} steps={steps}")
    lat = gpu.Lattice(case, storage=storage, wall_dist="case")
    lat.set_vortices(yz, sign, 0.2, 3.0)
    lat.step(steps)
    rho, u = lat.moments()
    orc = oracle_for(case, 0, wall_dist=case.wall_dist)
    orc.set_vortices(yz, sign, 0.2, 3.0)
    orc.step(steps)
    orho, ou = orc.moments()
    rho, u = rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64)
    _check(f"vortex urban collision={collision} {storage}", moment_errors(rho, u, orho, ou), tol)
    # the perturbation reaches the inlet plane's neighbours
    x = np.arange(case.ncells) % case.shape[0]
    assert np.abs(ou[1:, x == 1]).max() > 1e-4


def test_vortex_inlet_fp16(gpu):
    """FP16 deviation storage with the vortex method: loose bound, as for FP16."""
    case = _urban_open()
    yz, sign = _vortices(case, 40, 12)
    lat = gpu.Lattice(case, storage="f16", wall_dist="case")
    lat.set_vortices(yz, sign, 0.2, 3.0)
    lat.step(100)
    rho, u = lat.moments()
    orc = oracle_for(case, 0, wall_dist=case.wall_dist)
    orc.set_vortices(yz, sign, 0.2, 3.0)
    orc.step(100)
    orho, ou = orc.moments()
    e_rho, e_u, _ = moment_errors(rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64), orho, ou)
    announce(f"vortex urban f16: rho {e_rho:.3e} u {e_u:.3e}")
    assert e_rho < 5e-3 and e_u < 5e-2


def test_vortex_reset_and_clear(gpu):
    """Vortices replaced by a smaller set, then cleared, between steps."""
    case = _urban_open()
    lat = gpu.Lattice(case, storage="f64", wall_dist="case")
    orc = oracle_for(case, 0, wall_dist=case.wall_dist)
    for n, steps in ((40, 10), (5, 11), (0, 10)):
        yz, sign = _vortices(case, n, 100 + n)
        announce(f"vortex reset n={n} steps={steps}")
        lat.set_vortices(yz, sign, 0.25, 2.5)
        orc.set_vortices(yz, sign, 0.25, 2.5)
        lat.step(steps)
        orc.step(steps)
    rho, u = lat.moments()
    orho, ou = orc.moments()
    rho, u = rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64)
    _check("vortex reset f64", moment_errors(rho, u, orho, ou), 1e-12)


def test_vortex_clear_restores_mean_profile_bitwise(gpu):
    """Clearing the vortices (n = 0) before stepping gives the same bits as a
    run that never set any: the inlet field is rebuilt from the mean profile."""
    case = _urban_open()
    a = gpu.Lattice(case, storage="f32", wall_dist="case")
    yz, sign = _vortices(case, 40, 13)
    a.set_vortices(yz, sign, 0.2, 3.0)
    a.set_vortices(np.zeros((0, 2)), np.zeros(0, int), 0.2, 3.0)
    a.step(9)
    b = gpu.Lattice(case, storage="f32", wall_dist="case")
    b.step(9)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_vortex_arguments_checked(gpu):
    case = _stream(19, (12, 3, 4), 0.04)
    lat = gpu.Lattice(case, storage="f64")
    yz, sign = np.array([[1.0, 1.0]]), np.array([1])
    for bad in ((yz, sign, 0.1, 0.0), (yz, sign, -0.1, 1.0), (np.array([[np.nan, 1.0]]), sign, 0.1, 1.0),
                (np.array([[1.0, -0.5]]), sign, 0.1, 1.0), (np.array([[3.5, 1.0]]), sign, 0.1, 1.0),
                (np.zeros((gpu.MAX_VORTICES + 1, 2)), np.ones(gpu.MAX_VORTICES + 1), 0.1, 1.0)):
        with pytest.raises(gpu.LbmError) as e:
            lat.set_vortices(*bad)
        assert e.value.code == gpu.EINVAL
    closed = gpu.Lattice(I.taylor_green(8, q=19), storage="f64")
    with pytest.raises(gpu.LbmError):
        closed.set_vortices(yz, sign, 0.1, 1.0)


def _open_porous(collision=0, fringe=0):
    c = I.porous_channel(shape=(20, 12, 8), q=19 if collision == 0 else 27)
    return dataclasses.replace(c, name="porous_open", periodic=(0, 1, 0), force=(0.0, 0.0, 0.0), open_x=1,
                               rho_out=1.002, u_ref=0.05, z0=1.0, collision=collision, fringe_len=fringe)


@pytest.mark.parametrize("collision,fringe,vort", [(0, 0, False), (1, 4, True)])
def test_open_adjoint_transpose(gpu, collision, fringe, vort):
    """<L v, w> from the oracle's tangent step equals <v, L^T w> from one GPU
    reverse step, with open x faces (the rebuild's transpose at both faces),
    at both parities, FP64; with a fringe before the outlet and vortices on
    the inlet in the second case."""
    case = _open_porous(collision, fringe)
    q, N = case.q, case.ncells
    c, w, _ = O.velocity_set(q)
    f_n = I.random_state(w, N, seed_offset=31, amp=0.05)
    rng = np.random.default_rng(32)
    v, dphi, wv = rng.standard_normal((q, N)), rng.standard_normal(N), rng.standard_normal((q, N))
    yz, sign = _vortices(case, 6, 33)
    for parity in (0, 1):
        orc = oracle_for(case, tangent=True)
        if vort:
            orc.set_vortices(yz, sign, 0.3, 2.0)
        orc.set_populations(f_n, v)
        orc.set_phi_tangent(dphi)
        orc.step(1)
        _, Lv = orc.populations(with_tangent=True)
        lhs = float((Lv * wv).sum())
        lat = gpu.Lattice(case, storage="f64")
        if vort:
            lat.set_vortices(yz, sign, 0.3, 2.0)
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
        announce(f"open transpose collision={collision} parity={parity}: <Lv,w> {lhs:.15e} <v,L^T w> {rhs:.15e}")
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("collision", [0, 1])
def test_open_gradient_matches_tangent(gpu, collision):
    """Checkpointed dJ/dphi with open x faces against the oracle's tangent,
    at cells on the inlet and outlet planes and inside (FP64)."""
    case = _open_porous(collision)
    planes = (2, 17)
    T, nsnap = 15, 3
    N, nx = case.ncells, case.shape[0]
    lat = gpu.Lattice(case, storage="f64")
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    J, _ = gpu.lbm_gradient(lat.ctx, T, planes, lat.new_state_buffer(nsnap), nsnap, lat.new_adjoint(), grad)
    g = grad.cpu().numpy()
    Jo, _ = oracle_for(case, T).objective(planes)
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    for cell in (0 + nx * 5, nx - 1 + nx * 30, 7 + nx * 17):
        t = oracle_for(case, tangent=True)
        e = np.zeros(N)
        e[cell] = 1.0
        t.set_phi_tangent(e)
        t.step(T)
        _, dJ = t.objective(planes)
        announce(f"open gradient cell {cell} (x={cell % nx}): gpu {g[cell]:.12e} tangent {dJ:.12e}")
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())


@pytest.mark.parametrize("collision", [0, 1])
def test_open_gradient_mean_with_lid(gpu, collision):
    """The time-averaged objective's gradient with open x faces and a lid
    (the reverse kernel's seeded open-face and seeded lid branches), against
    the oracle's tangent summed over the steps, FP64."""
    case = dataclasses.replace(_open_porous(collision, 4), lid=1)
    planes = (2, 17)
    T, nsnap = 11, 3
    N, nx = case.ncells, case.shape[0]
    lat = gpu.Lattice(case, storage="f64")
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    J, _ = gpu.lbm_gradient_mean(lat.ctx, T, planes, lat.new_state_buffer(nsnap), nsnap, lat.new_adjoint(), grad)
    g = grad.cpu().numpy()
    nz_ = case.shape[2]
    lid_cell = 9 + nx * (3 + case.shape[1] * (nz_ - 1))
    for cell in (0 + nx * 5, nx - 1 + nx * 30, 7 + nx * 17, lid_cell - nx * case.shape[1]):
        t = oracle_for(case, tangent=True)
        e = np.zeros(N)
        e[cell] = 1.0
        t.set_phi_tangent(e)
        dJ = 0.0
        for _ in range(T):
            t.step(1)
            dJ += t.objective(planes)[1]
        dJ /= T
        announce(f"open mean gradient (lid) cell {cell}: gpu {g[cell]:.12e} tangent {dJ:.12e}")
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())


def test_open_gradient_fp32(gpu):
    """FP32 storage with open x faces (the rebuild's transpose in FP32, its
    common part in FP64): the gradient against the oracle's tangent, per cell
    relative to max(|dJ|, 1e-3 max|g|)."""
    case = _open_porous(1, 4)
    planes = (2, 17)
    T, nsnap = 15, 3
    N, nx = case.ncells, case.shape[0]
    lat = gpu.Lattice(case, storage="f32")
    grad = lat.new_gradient()
    gpu.lbm_gradient(lat.ctx, T, planes, lat.new_state_buffer(nsnap), nsnap, lat.new_adjoint(), grad)
    g = grad.cpu().numpy()
    errs = []
    for cell in (0 + nx * 5, nx - 1 + nx * 30, 7 + nx * 17):
        t = oracle_for(case, tangent=True)
        e = np.zeros(N)
        e[cell] = 1.0
        t.set_phi_tangent(e)
        t.step(T)
        _, dJ = t.objective(planes)
        errs.append(abs(g[cell] - dJ) / max(abs(dJ), 1e-3 * np.abs(g).max()))
    announce(f"open gradient fp32: per-cell errors {['%.2e' % x for x in errs]}")
    assert max(errs) <= 1e-4, errs
