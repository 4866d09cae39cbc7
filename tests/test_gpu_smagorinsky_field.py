"""Per-cell Smagorinsky constant (Sec. 2.3: the dynamics take C_S from the
cell) through the C ABI (lbm_set_smagorinsky, lbm_gradient_cs,
lbm_adjoint_step_cs), against the oracle with the same field:

 - forward: a random field on a wall-modeled porous channel (BGK and
   recursive regularized; the wall records use the wall cell's C_S) and on
   an urban crop, FP64 populations to 1e-12, FP32 moments to 1e-5; a field
   equal to the scalar everywhere reproduces the scalar run to rounding;
 - the entry point's refusals: no room reserved, a negative or NaN entry
   (the field in force is kept);
 - gradients: dJ/dC_S of the terminal and of the time-averaged objective
   against the oracle's tangent along C_S directions (single cells at a wall,
   at a reference cell and in the bulk, and a random direction), FP64 1e-10;
   FP32 storage against the same tangent; dJ/dphi unchanged by the request.
"""
import numpy as np
import pytest
import torch

from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, moment_errors, oracle_for, rel_maxnorm

pytestmark = pytest.mark.gpu


def _wall_porous(shape=(16, 12, 8), collision=0):
    c = I.porous_channel(shape=shape)
    c.wall_model = 1
    c.wall_dist = I.voxel_wall_distance(c.mask, c.shape, c.periodic)
    c.collision = collision
    return c


def _urban_crop():
    c = I.urban(nx=40, ny=24, nz=16, q=19, tau0=0.52, fringe_len=6, x_lo=6, x_hi=30, h_mean=6.0, h_max=10,
                fp_lo=3, fp_hi=7)
    c.collision = 1
    return c


def _field(N, seed):
    return np.random.default_rng(seed).uniform(0.05, 0.25, N)


@pytest.mark.parametrize("name,collision", [("porous", 0), ("porous", 1), ("urban", 1)])
def test_field_forward_fp64(gpu, name, collision):
    case = _wall_porous(collision=collision) if name == "porous" else _urban_crop()
    cs = _field(case.ncells, 301 + collision)
    steps = 30
    announce(f"C_S field forward: {name} collision {collision}, FP64, {steps} steps")
    lat = gpu.Lattice(case, storage="f64", cs_field=True)
    lat.set_smagorinsky(cs)
    lat.step(steps)
    orc = oracle_for(case)
    orc.set_smagorinsky(cs)
    orc.step(steps)
    f = lat.populations().cpu().numpy()
    mask = np.ones(case.ncells) if case.mask is None else np.asarray(case.mask, float)
    e_f = rel_maxnorm(f * mask, orc.populations() * mask)
    # the field must matter: the scalar run differs by far more than the bar
    ref = oracle_for(case, steps).populations() * mask
    d_scalar = rel_maxnorm(ref, orc.populations() * mask)
    announce(f"populations {e_f:.3e} (scalar C_S run differs by {d_scalar:.3e})")
    assert e_f <= 1e-12 and d_scalar > 1e-8


def test_field_forward_fp32(gpu):
    case = _wall_porous(collision=1)
    cs = _field(case.ncells, 305)
    lat = gpu.Lattice(case, storage="f32", cs_field=True)
    lat.set_smagorinsky(torch.as_tensor(cs, device="cuda"))
    lat.step(30)
    rho, u = lat.moments()
    orc = oracle_for(case)
    orc.set_smagorinsky(cs)
    orc.step(30)
    orho, ou = orc.moments()
    e_rho, e_u, _ = moment_errors(rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64), orho, ou)
    announce(f"C_S field FP32: rho {e_rho:.3e} u {e_u:.3e}")
    assert e_rho <= 1e-5 and e_u <= 1e-5


def test_uniform_field_matches_scalar(gpu):
    case = _wall_porous(collision=1)
    a = gpu.Lattice(case, storage="f64")
    a.step(20)
    b = gpu.Lattice(case, storage="f64", cs_field=True)
    b.set_smagorinsky(np.full(case.ncells, case.cs_smag))
    b.step(20)
    e = rel_maxnorm(b.populations().cpu().numpy(), a.populations().cpu().numpy())
    announce(f"uniform field vs scalar: {e:.3e}")
    assert e <= 1e-14
    # back to the scalar: the next steps match the scalar run's
    b.set_smagorinsky(None)
    a.step(5)
    b.step(5)
    assert rel_maxnorm(b.populations().cpu().numpy(), a.populations().cpu().numpy()) <= 1e-14


def test_field_refusals(gpu):
    case = _wall_porous()
    N = case.ncells
    plain = gpu.Lattice(case, storage="f64")
    with pytest.raises(gpu.LbmError) as e:
        plain.set_smagorinsky(np.full(N, 0.1))
    assert e.value.code == gpu.EINVAL
    lat = gpu.Lattice(case, storage="f64", cs_field=True)
    good = _field(N, 307)
    lat.set_smagorinsky(good)
    for bad_value in (-0.01, np.nan, np.inf):
        bad = good.copy()
        bad[N // 2] = bad_value
        with pytest.raises(gpu.LbmError) as e:
            lat.set_smagorinsky(bad)
        assert e.value.code == gpu.EINVAL
    # the good field is still in force
    lat.step(10)
    orc = oracle_for(case)
    orc.set_smagorinsky(good)
    orc.step(10)
    assert rel_maxnorm(lat.populations().cpu().numpy() * case.mask, orc.populations() * case.mask) <= 1e-12


def _cells(case):
    nx, ny, nz = case.shape
    return [3 + nx * (4 + ny * 0), 3 + nx * (4 + ny * 1), 11 + nx * (5 + ny * 4)]


def _tangent(case, cs, direction, T, planes, mean=False):
    t = oracle_for(case, tangent=True)
    t.set_smagorinsky(cs, direction)
    if not mean:
        t.step(T)
        return t.objective(planes)[1]
    dJ = 0.0
    for _ in range(T):
        t.step(1)
        dJ += t.objective(planes)[1]
    return dJ / T


@pytest.mark.parametrize("collision,mean", [(0, False), (1, False), (1, True)])
def test_cs_gradient_matches_oracle_tangent(gpu, collision, mean):
    case = _wall_porous(collision=collision)
    planes = (2, 13)
    T, nsnap = (20, 4) if not mean else (13, 3)
    N = case.ncells
    cs = _field(N, 311 + collision)
    lat = gpu.Lattice(case, storage="f64", cs_field=True)
    lat.set_smagorinsky(cs)
    gphi = lat.new_gradient()
    gcs = lat.new_gradient()
    J, _ = gpu.lbm_gradient_cs(lat.ctx, T, planes, lat.new_state_buffer(nsnap), nsnap, lat.new_adjoint(), gphi,
                               gcs, mean=mean)
    g = gcs.cpu().numpy()
    announce(f"C_S gradient collision {collision} mean {mean}: J {J:.12e}, max |dJ/dC_S| {np.abs(g).max():.3e}")
    assert np.all(g[np.asarray(case.mask) == 0] == 0.0)
    for cell in _cells(case):
        e = np.zeros(N)
        e[cell] = 1.0
        dJ = _tangent(case, cs, e, T, planes, mean)
        announce(f"  cell {cell}: gpu {g[cell]:.12e} tangent {dJ:.12e}")
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())
    d = np.random.default_rng(313).standard_normal(N) * case.mask
    dJ = _tangent(case, cs, d, T, planes, mean)
    gd = float((g * d).sum())
    announce(f"  random direction: gpu {gd:.12e} tangent {dJ:.12e}")
    assert abs(gd - dJ) <= 1e-10 * abs(dJ)
    # the porosity gradient is the one lbm_gradient gives
    ref = gpu.Lattice(case, storage="f64", cs_field=True)
    ref.set_smagorinsky(cs)
    gphi2 = ref.new_gradient()
    sweep = gpu.lbm_gradient_mean if mean else gpu.lbm_gradient
    sweep(ref.ctx, T, planes, ref.new_state_buffer(nsnap), nsnap, ref.new_adjoint(), gphi2)
    assert torch.equal(gphi, gphi2)


def test_cs_gradient_at_scalar(gpu):
    """Without a field the derivative is taken at the scalar C_S, per cell."""
    case = _wall_porous(collision=1)
    planes = (2, 13)
    T = 16
    N = case.ncells
    lat = gpu.Lattice(case, storage="f64")
    gcs = lat.new_gradient()
    gpu.lbm_gradient_cs(lat.ctx, T, planes, lat.new_state_buffer(4), 4, lat.new_adjoint(), lat.new_gradient(), gcs)
    g = gcs.cpu().numpy()
    cs = np.full(N, case.cs_smag)
    for cell in _cells(case)[:2]:
        e = np.zeros(N)
        e[cell] = 1.0
        dJ = _tangent(case, cs, e, T, planes)
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())


def test_cs_gradient_fp32(gpu):
    case = _wall_porous(collision=0)
    planes = (2, 13)
    T = 20
    N = case.ncells
    cs = _field(N, 317)
    lat = gpu.Lattice(case, storage="f32", cs_field=True)
    lat.set_smagorinsky(cs)
    gcs = lat.new_gradient()
    gpu.lbm_gradient_cs(lat.ctx, T, planes, lat.new_state_buffer(4), 4, lat.new_adjoint(), lat.new_gradient(), gcs)
    g = gcs.cpu().numpy()
    errs = []
    for cell in _cells(case):
        e = np.zeros(N)
        e[cell] = 1.0
        dJ = _tangent(case, cs, e, T, planes)
        errs.append(abs(g[cell] - dJ) / max(abs(dJ), 1e-3 * np.abs(g).max()))
    announce(f"C_S gradient FP32: per-cell errors {['%.2e' % x for x in errs]}")
    assert max(errs) <= 1e-4, errs


def test_adjoint_step_cs_transpose(gpu):
    """One reverse step: <L v, w> = <v, L^T w> with a C_S direction among the
    inputs (the tangent of one oracle step along populations v and C_S
    direction dc, against lambda and grad_cs of one lbm_adjoint_step_cs)."""
    from oracle import velocity_set
    case = _wall_porous(collision=1)
    q, N = case.q, case.ncells
    _, w, _ = velocity_set(q)
    cs = _field(N, 319)
    f_n = I.random_state(w, N, seed_offset=321, amp=0.03)
    rng = np.random.default_rng(323)
    v = rng.standard_normal((q, N)) * case.mask
    wv = rng.standard_normal((q, N)) * case.mask
    dc = rng.standard_normal(N) * case.mask
    orc = oracle_for(case, tangent=True)
    orc.set_populations(f_n, v)
    orc.set_smagorinsky(cs, dc)
    orc.step(1)
    _, Lv = orc.populations(with_tangent=True)
    lhs = float((Lv * wv).sum())
    lat = gpu.Lattice(case, storage="f64", cs_field=True)
    lat.set_smagorinsky(cs)
    lat.set_populations(torch.as_tensor(f_n))
    snap = lat.new_state_buffer()
    lat.save_state(snap)
    lat.step(1)
    lam = lat.new_adjoint()
    gpu.lbm_adjoint_from_natural(lat.ctx, torch.as_tensor(wv, device="cuda"), lam)
    lat.load_state(snap)
    gphi = lat.new_gradient()
    gcs = lat.new_gradient()
    gpu.lbm_adjoint_step_cs(lat.ctx, lam, gphi, gcs)
    nat = lat.new_natural()
    gpu.lbm_adjoint_to_natural(lat.ctx, lam, nat)
    lat.sync()
    rhs = float((v * nat.cpu().numpy()).sum()) + float((dc * gcs.cpu().numpy()).sum())
    announce(f"C_S transpose: <Lv,w> {lhs:.15e} <v,L^T w> {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_autograd_with_cs_field(gpu):
    """autograd.objective(phi, ..., cs=...): backward gives lbm_gradient_cs's
    dJ/dphi and dJ/dC_S; the value matches a run without gradients."""
    from paper_2506_21804_amd.autograd import objective
    case = _wall_porous(collision=1)
    planes = (2, 13)
    N = case.ncells
    cs0 = _field(N, 331)
    phi = torch.tensor(case.porosity, dtype=torch.float64, requires_grad=True)
    cs = torch.tensor(cs0, dtype=torch.float64, requires_grad=True)
    J = objective(phi, case, storage="f64", T=10, planes=planes, nsnap=3, cs=cs)
    J.backward()
    J0 = objective(phi.detach(), case, storage="f64", T=10, planes=planes, nsnap=3, cs=cs.detach())
    assert abs(J.item() - J0.item()) <= 1e-13 * abs(J.item())
    lat = gpu.Lattice(case, storage="f64", cs_field=True)
    lat.set_smagorinsky(cs0)
    gphi, gcs = lat.new_gradient(), lat.new_gradient()
    gpu.lbm_gradient_cs(lat.ctx, 10, planes, lat.new_state_buffer(3), 3, lat.new_adjoint(), gphi, gcs)
    np.testing.assert_array_equal(phi.grad.numpy(), gphi.cpu().numpy())
    np.testing.assert_array_equal(cs.grad.numpy(), gcs.cpu().numpy())
