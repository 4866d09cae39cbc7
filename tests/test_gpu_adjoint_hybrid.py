"""Discrete adjoint through the hybrid collision (Eqs. (7), (10)): the
finite-difference strain of a cell reads the velocities of its axis
neighbours, so the reverse step has a second pass that carries each cell's
strain adjoint back to those velocities and from them to the neighbours'
populations; wall cells take the full strain with the law's wall-normal
shear (Sec. 2.2.1).  Checked against the oracle's forward-mode derivatives,
which differentiate the same hybrid:

 - transpose test <L v, w> = <v, L^T w> of one step, both parities, FP64
   (1e-12): a periodic porous box (central differences only), a porous
   channel with walls (one-sided differences at the walls, half-way
   bounce-back, D3Q19 and D3Q27), the same channel wall-modeled (full strain
   in the wall cells), an urban crop (buildings, fringe, lid), the crop with
   full-slip sides and top, and a box with full-slip y and z faces;
 - the checkpointed gradient (terminal and time-averaged objective, and the
   per-cell C_S gradient) against the oracle's tangent, FP64 (1e-10), and
   FP32 and FP16 storage against the FP64 gradient.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, oracle_for

pytestmark = pytest.mark.gpu


def _hyb(case, fdw=0.3):
    c = dataclasses.replace(case, collision=1)
    c.fd_weight = fdw
    return c


def _porous_box():
    c = I.porous_channel(shape=(14, 10, 8))
    c.periodic = (1, 1, 1)
    c.mask = None
    return _hyb(c, 0.4)


def _porous_channel(q=19, wall=False):
    c = I.porous_channel(shape=(18, 12, 8), q=q)
    if wall:
        c.wall_model = 1
        c.wall_dist = I.voxel_wall_distance(c.mask, c.shape, c.periodic)
    return _hyb(c)


def _urban_crop(slip=False):
    c = I.urban(nx=40, ny=24, nz=16, q=19, tau0=0.52, fringe_len=6, x_lo=6, x_hi=30, h_mean=6.0, h_max=10,
                fp_lo=3, fp_hi=7, slip_walls=slip)
    return _hyb(c, 0.5)


def _slip_box():
    # full-slip y and z faces: the strain is one-sided at them
    case = I.Case(name="slipbox", q=27, shape=(37, 9, 7), periodic=(1, 0, 0), tau0=0.57, cs_smag=0.12,
                  force=(2e-5, 0.0, 0.0), collision=1, slip=0b111100)
    return _hyb(case, 0.4)


def _transpose(gpu, case, parity, seed):
    q, N = case.q, case.ncells
    c, w, _ = O.velocity_set(q)
    fluid = np.ones(N) if case.mask is None else np.asarray(case.mask, float)
    f_n = I.random_state(w, N, seed_offset=seed, amp=0.03)
    rng = np.random.default_rng(seed + 1)
    v = rng.standard_normal((q, N)) * fluid
    wv = rng.standard_normal((q, N)) * fluid
    dphi = rng.standard_normal(N) if case.porosity is not None else None
    orc = oracle_for(case, tangent=True)
    orc.set_populations(f_n, v)
    if dphi is not None:
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
    rhs = float((v * nat.cpu().numpy()).sum())
    if dphi is not None:
        rhs += float((dphi * grad.cpu().numpy()).sum())
    return lhs, rhs


CASES = {
    "porous box": lambda: _porous_box(),
    "porous channel q19": lambda: _porous_channel(19),
    "porous channel q27": lambda: _porous_channel(27),
    "wall-modeled channel": lambda: _porous_channel(19, wall=True),
    "urban crop": lambda: _urban_crop(),
    "urban crop, full-slip sides and top": lambda: _urban_crop(slip=True),
    "full-slip box": lambda: _slip_box(),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("parity", [0, 1])
def test_hybrid_adjoint_transpose(gpu, name, parity):
    case = CASES[name]()
    announce(f"hybrid adjoint transpose: {name} fd_weight {case.fd_weight} parity {parity}")
    lhs, rhs = _transpose(gpu, case, parity, 131 + parity)
    announce(f"<Lv,w> {lhs:.15e} <v,L^T w> {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def _cells(case):
    nx, ny, nz = case.shape
    return [3 + nx * (4 + ny * 0), 3 + nx * (4 + ny * 1), 9 + nx * (7 + ny * (nz - 1)), 11 + nx * (5 + ny * 4)]


def _tangent(case, T, planes, cell):
    t = oracle_for(case, tangent=True)
    e = np.zeros(case.ncells)
    e[cell] = 1.0
    t.set_phi_tangent(e)
    t.step(T)
    return t.objective(planes)[1]


@pytest.mark.parametrize("wall", [False, True])
def test_hybrid_gradient_matches_oracle_tangent(gpu, wall):
    case = _porous_channel(19, wall=wall)
    planes = (2, 13)
    T = 16
    N = case.ncells
    lat = gpu.Lattice(case, storage="f64")
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    J, _ = gpu.lbm_gradient(lat.ctx, T, planes, lat.new_state_buffer(4), 4, lat.new_adjoint(), grad)
    g = grad.cpu().numpy()
    Jo, _ = oracle_for(case, T).objective(planes)
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    for cell in _cells(case):
        dJ = _tangent(case, T, planes, cell)
        announce(f"hybrid gradient wall {wall} cell {cell}: gpu {g[cell]:.12e} tangent {dJ:.12e}")
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())


def test_hybrid_gradient_mean_and_cs(gpu):
    """Time-averaged objective; dJ/dphi and dJ/dC_S of a per-cell C_S field."""
    case = _porous_channel(19, wall=True)
    planes = (2, 13)
    T, nsnap = 11, 3
    N = case.ncells
    cs = 0.1 + 0.05 * np.random.default_rng(77).random(N)
    lat = gpu.Lattice(case, storage="f64", cs_field=True)
    lat.set_smagorinsky(cs)
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    gcs = torch.zeros(N, dtype=torch.float64, device="cuda")
    gpu.lbm_gradient_cs(lat.ctx, T, planes, lat.new_state_buffer(nsnap), nsnap, lat.new_adjoint(), grad, gcs,
                        mean=True)
    g, gc = grad.cpu().numpy(), gcs.cpu().numpy()
    for cell in _cells(case)[:3]:
        t = oracle_for(case, tangent=True)
        t.set_smagorinsky(cs)
        e = np.zeros(N)
        e[cell] = 1.0
        t.set_phi_tangent(e)
        dphi = 0.0
        for _ in range(T):
            t.step(1)
            dphi += t.objective(planes)[1]
        dphi /= T
        t = oracle_for(case, tangent=True)
        t.set_smagorinsky(cs, e)
        dcs = 0.0
        for _ in range(T):
            t.step(1)
            dcs += t.objective(planes)[1]
        dcs /= T
        announce(f"hybrid mean gradient cell {cell}: phi gpu {g[cell]:.12e} tangent {dphi:.12e}; "
                 f"C_S gpu {gc[cell]:.12e} tangent {dcs:.12e}")
        assert abs(g[cell] - dphi) <= 1e-10 * max(abs(dphi), 1e-3 * np.abs(g).max())
        assert abs(gc[cell] - dcs) <= 1e-10 * max(abs(dcs), 1e-3 * np.abs(gc).max())


def test_hybrid_gradient_fp32_fp16(gpu):
    """FP32 and FP16 storage against the FP64 gradient, same schedule, as
    max-norm errors: FP32 within 1e-5 (the non-hybrid FP32 bar; measured
    1.7e-7), FP16 within 1e-3 (measured 2.6e-4)."""
    case = _porous_channel(19, wall=True)
    planes = (2, 13)
    T = 16
    N = case.ncells
    out = {}
    for st in ("f64", "f32", "f16"):
        lat = gpu.Lattice(case, storage=st)
        grad = torch.zeros(N, dtype=torch.float64, device="cuda")
        gpu.lbm_gradient(lat.ctx, T, planes, lat.new_state_buffer(4), 4, lat.new_adjoint(), grad)
        out[st] = grad.cpu().numpy()
    ref = np.abs(out["f64"]).max()
    e32 = np.abs(out["f32"] - out["f64"]).max() / ref
    e16 = np.abs(out["f16"] - out["f64"]).max() / ref
    announce(f"hybrid gradient max-norm error: FP32 {e32:.3e}, FP16 {e16:.3e}")
    assert e32 <= 1e-5
    assert e16 <= 1e-3


@pytest.mark.parametrize("storage,db", [("f64", 8), ("f32", 4), ("f16", 4)])
def test_hybrid_adjoint_buffer_holds_strain_adjoints(gpu, storage, db):
    """With the hybrid the adjoint buffer grows by six compute-type values per
    cell (the strain adjoints, from a 256-byte boundary)."""
    case = _porous_channel(19, wall=True)
    plain = dataclasses.replace(case, fd_weight=0.0)
    b_hyb = gpu.lbm_adjoint_bytes(gpu.Lattice(case, storage=storage).ctx)
    b_plain = gpu.lbm_adjoint_bytes(gpu.Lattice(plain, storage=storage).ctx)
    extra = 6 * case.ncells * db
    assert extra <= b_hyb - b_plain <= extra + 255, (b_hyb, b_plain, extra)

