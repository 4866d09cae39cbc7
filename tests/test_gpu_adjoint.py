"""Discrete adjoint of the HIP path checked against the oracle's forward-mode
(dual-number) derivatives and central finite differences.

 - transpose test: <L v, w> from the oracle's tangent step equals <v, L^T w>
   from one GPU reverse step (populations and porosity directions), FP64;
 - the checkpointed GPU gradient dJ/dphi equals the oracle's tangent
   derivative at sampled cells (FP64, 1e-10), for the terminal objective
   and for its time average over the trajectory;
 - the checkpointed gradient is bitwise equal to the full-storage one, and
   the sweep takes the binomial-optimal number of forward steps (plus the
   step to T and the re-advance to T-1);
 - the gradient matches FP64 central differences (h = 1e-3) of the oracle:
   FP64 storage per cell within 1e-4 (|g - g_FD| / max(|g_FD|, 1e-3
   max|g_FD|)), FP32 storage within 1e-4 of the gradient's max-norm.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, oracle_for

pytestmark = pytest.mark.gpu

# bars of the FP16-storage gradient against the FP64 one (measured after 100
# steps: max-norm 2.4e-4 BGK, 3.9e-4 RR3; per cell 6.2e-2, 4.3e-2)
FP16_GRAD_NORM, FP16_GRAD_CELL = 1e-3, 0.2


def _case(shape=(20, 12, 8), collision=0):
    c = I.porous_channel(shape=shape)
    c.collision = collision
    return c


@pytest.mark.parametrize("collision", [0, 1])
def test_transpose_one_step(gpu, collision):
    """collision 0: BGK; 1: recursive regularized (its own vector-Jacobian product)."""
    case = _case(collision=collision)
    q, N = case.q, case.ncells
    c, w, _ = O.velocity_set(q)
    f_n = I.random_state(w, N, seed_offset=21, amp=0.05)
    rng = np.random.default_rng(22)
    v = rng.standard_normal((q, N))
    dphi = rng.standard_normal(N)
    wv = rng.standard_normal((q, N))
    for parity in (0, 1):
        announce(f"transpose test collision {collision} parity {parity}")
        # oracle: tangent of one step from f_n in direction (v, dphi)
        orc = oracle_for(case, tangent=True)
        orc.set_populations(f_n, v)
        orc.set_phi_tangent(dphi)
        orc.step(1)
        _, Lv = orc.populations(with_tangent=True)
        lhs = float((Lv * wv).sum())
        # GPU: state f_n at step count n with the requested parity
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
        announce(f"<Lv,w> {lhs:.15e} <v,L^T w> {rhs:.15e}")
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("collision", [0, 1])
def test_gradient_matches_oracle_tangent(gpu, collision):
    case = _case((16, 12, 8), collision=collision)
    planes = (2, 13)
    T = 20
    lat = gpu.Lattice(case, storage="f64")
    N = case.ncells
    lam = lat.new_adjoint()
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    snaps = lat.new_state_buffer(4)
    J, nfwd = gpu.lbm_gradient(lat.ctx, T, planes, snaps, 4, lam, grad)
    g = grad.cpu().numpy()
    cost = gpu.lbm_revolve_cost(T, 4)
    assert cost + 1 <= nfwd <= cost + T, (nfwd, cost)
    Jo, _ = oracle_for(case, T).objective(planes)
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    for cell in I.sample_cells(N, 6, seed_offset=5):
        orc = oracle_for(case, tangent=True)
        e = np.zeros(N)
        e[cell] = 1.0
        orc.set_phi_tangent(e)
        orc.step(T)
        _, dJ = orc.objective(planes)
        announce(f"cell {cell}: gpu {g[cell]:.12e} tangent {dJ:.12e}")
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())
    assert lat.steps == 0  # the context is back at step 0


@pytest.mark.parametrize("collision", [0, 1])
def test_gradient_mean_matches_oracle_tangent(gpu, collision):
    """Time-averaged objective J = (1/T) sum_{t=1..T} j(f_t): value and
    gradient against the oracle summed step by step (value; dual-number
    derivative along unit porosity directions), FP64, with a schedule that
    recomputes (T = 23 steps on 3 snapshot slots)."""
    case = _case((16, 12, 8), collision=collision)
    planes = (2, 13)
    T, nsnap = 23, 3
    lat = gpu.Lattice(case, storage="f64")
    N = case.ncells
    lam = lat.new_adjoint()
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    snaps = lat.new_state_buffer(nsnap)
    J, nfwd = gpu.lbm_gradient_mean(lat.ctx, T, planes, snaps, nsnap, lam, grad)
    g = grad.cpu().numpy()
    _, nfwd_terminal = gpu.lbm_gradient(lat.ctx, T, planes, snaps, nsnap, lam, torch.zeros_like(grad))
    assert nfwd == nfwd_terminal
    orc = oracle_for(case)
    Jo = 0.0
    for _ in range(T):
        orc.step(1)
        Jo += orc.objective(planes)[0]
    Jo /= T
    announce(f"mean objective collision={collision}: gpu {J:.15e} oracle {Jo:.15e}")
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    for cell in I.sample_cells(N, 5, seed_offset=6):
        t = oracle_for(case, tangent=True)
        e = np.zeros(N)
        e[cell] = 1.0
        t.set_phi_tangent(e)
        dJ = 0.0
        for _ in range(T):
            t.step(1)
            dJ += t.objective(planes)[1]
        dJ /= T
        announce(f"mean objective cell {cell}: gpu {g[cell]:.12e} tangent {dJ:.12e}")
        assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())
    assert lat.steps == 0


def test_checkpointed_equals_full_storage(gpu):
    case = _case((16, 12, 8))
    planes = (2, 13)
    T = 33
    N = case.ncells
    out = []
    for nsnap in (3, T + 1):
        lat = gpu.Lattice(case, storage="f32")
        lam = lat.new_adjoint()
        grad = lat.new_gradient()
        snaps = lat.new_state_buffer(nsnap)
        J, nfwd = gpu.lbm_gradient(lat.ctx, T, planes, snaps, nsnap, lam, grad)
        cost = gpu.lbm_revolve_cost(T, nsnap)
        assert cost + 1 <= nfwd <= cost + T, (nsnap, nfwd, cost)
        if nsnap > T:
            assert nfwd == T  # full storage: every state computed exactly once
        out.append(grad.cpu().numpy())
    assert gpu.lbm_revolve_cost(T, T + 1) == T - 1
    assert np.array_equal(out[0], out[1])


def _fd_gradient(case, planes, T, cells, h=1e-3):
    """Central differences of the oracle's objective in the porosity of each
    cell.  h = 1e-3: at these sizes the rounding noise of J over 2h and the
    O(h^2) truncation both stay near 1e-5 of the derivative (checked against
    the oracle's dual-number tangent)."""
    fd = []
    for cell in cells:
        Js = []
        for sgn in (1, -1):
            c2 = I.porous_channel(shape=case.shape)
            c2.porosity = case.porosity.copy()
            c2.porosity[cell] += sgn * h
            Js.append(oracle_for(c2, T).objective(planes)[0])
        fd.append((Js[0] - Js[1]) / (2 * h))
    return np.array(fd)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_gradient_vs_central_differences(gpu, storage):
    """GPU gradient after 100 steps vs the oracle's exact (dual-number)
    derivative and its FP64 central differences, per sampled cell relative to
    max(|dJ/dphi|, 1e-3 of the largest).  FP64 storage: within 1e-10 of the
    exact derivative and 1e-4 of the central differences.  FP32 storage:
    within 1e-5 of the exact derivatives' max-norm, and per cell within
    2e-4.  The FP32 run's smallest sampled derivative (1.6 % of the largest)
    is off by 1.35e-4 of itself: the exact derivative along the FP32
    trajectory already differs from the FP64 one by about that much there,
    and the FP32 adjoint arithmetic adds a similar amount (measured split);
    at the full porous-channel size every sampled cell meets 1e-4
    (test_gpu_c4_gradient.py)."""
    case = _case((32, 24, 16))
    planes = (4, 28)
    T = 100
    N = case.ncells
    lat = gpu.Lattice(case, storage=storage)
    lam = lat.new_adjoint()
    grad = lat.new_gradient()
    snaps = lat.new_state_buffer(11)
    gpu.lbm_gradient(lat.ctx, T, planes, snaps, 11, lam, grad)
    g = grad.cpu().numpy()
    cells = I.sample_cells(N, 8, seed_offset=5)
    fd = _fd_gradient(case, planes, T, cells)
    scale = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    err_cell = (np.abs(g[cells] - fd) / scale).max()
    err_norm = np.abs(g[cells] - fd).max() / np.abs(fd).max()
    tan = []
    for cell in cells:
        t = oracle_for(case, tangent=True)
        e = np.zeros(N)
        e[cell] = 1.0
        t.set_phi_tangent(e)
        t.step(T)
        tan.append(t.objective(planes)[1])
    tan = np.array(tan)
    err_tan = (np.abs(g[cells] - tan) / np.maximum(np.abs(tan), 1e-3 * np.abs(tan).max())).max()
    fd_tan = (np.abs(fd - tan) / np.maximum(np.abs(tan), 1e-3 * np.abs(tan).max())).max()
    announce(f"{storage} gradient: per-cell vs exact {err_tan:.3e}; vs FD per-cell {err_cell:.3e}, max-norm "
             f"{err_norm:.3e}; FD vs exact per-cell {fd_tan:.3e}")
    if storage == "f64":
        assert err_tan <= 1e-10 and err_cell <= 1e-4, (err_tan, err_cell)
    else:
        err_tan_norm = np.abs(g[cells] - tan).max() / np.abs(tan).max()
        assert err_tan <= 2e-4 and err_tan_norm <= 1e-5 and err_norm <= 1e-4, (err_tan, err_tan_norm, err_norm)


@pytest.mark.parametrize("collision", [0, 1])
def test_fp16_gradient_against_fp64(gpu, collision):
    """FP16 deviation storage (FP32 adjoint arithmetic and deviations): the
    checkpointed gradient after 100 steps against the FP64 one on the same
    schedule, as a max-norm error over all cells and per cell where the
    derivative is at least 1e-3 of the largest."""
    case = _case((32, 24, 16), collision=collision)
    planes = (4, 28)
    T = 100
    N = case.ncells
    out = {}
    for st in ("f64", "f16"):
        lat = gpu.Lattice(case, storage=st)
        grad = lat.new_gradient()
        gpu.lbm_gradient(lat.ctx, T, planes, lat.new_state_buffer(11), 11, lat.new_adjoint(), grad)
        out[st] = grad.cpu().numpy()
    g, ref = out["f16"], out["f64"]
    big = np.abs(ref).max()
    err_norm = np.abs(g - ref).max() / big
    sel = np.abs(ref) >= 1e-3 * big
    err_cell = (np.abs(g - ref)[sel] / np.abs(ref)[sel]).max()
    announce(f"fp16 gradient collision {collision}: max-norm {err_norm:.3e}, per cell {err_cell:.3e}")
    assert np.isfinite(g).all()
    assert err_norm <= FP16_GRAD_NORM and err_cell <= FP16_GRAD_CELL, (err_norm, err_cell)


def test_autograd_function(gpu):
    from paper_2506_21804_amd.autograd import objective
    case = _case((16, 12, 8))
    planes = (2, 13)
    phi = torch.tensor(case.porosity, dtype=torch.float64, requires_grad=True)
    J = objective(phi, case, storage="f64", T=12, planes=planes, nsnap=3)
    J.backward()
    orc = oracle_for(case, 12)
    assert abs(J.item() - orc.objective(planes)[0]) <= 1e-12 * abs(J.item())
    cell = int(I.sample_cells(case.ncells, 1, seed_offset=9)[0])
    t = oracle_for(case, tangent=True)
    e = np.zeros(case.ncells)
    e[cell] = 1.0
    t.set_phi_tangent(e)
    t.step(12)
    _, dJ = t.objective(planes)
    g = phi.grad.numpy()
    assert abs(g[cell] - dJ) <= 1e-10 * max(abs(dJ), 1e-3 * np.abs(g).max())


def test_autograd_function_mean(gpu):
    """objective(..., mean=True): the forward value without a gradient equals
    the one with it, and backward gives lbm_gradient_mean's dJ/dphi."""
    from paper_2506_21804_amd.autograd import objective
    case = _case((16, 12, 8))
    planes = (2, 13)
    phi = torch.tensor(case.porosity, dtype=torch.float64, requires_grad=True)
    J = objective(phi, case, storage="f64", T=9, planes=planes, nsnap=3, mean=True)
    J.backward()
    J_nograd = objective(phi.detach(), case, storage="f64", T=9, planes=planes, nsnap=3, mean=True)
    assert abs(J.item() - J_nograd.item()) <= 1e-13 * abs(J.item())
    lat = gpu.Lattice(case, storage="f64")
    grad = torch.zeros(case.ncells, dtype=torch.float64, device="cuda")
    gpu.lbm_gradient_mean(lat.ctx, 9, planes, lat.new_state_buffer(3), 3, lat.new_adjoint(), grad)
    np.testing.assert_array_equal(phi.grad.numpy(), grad.cpu().numpy())


def test_fp32_gradient_error_split(gpu):
    """Where the FP32 gradient's error comes from, on the case above: the
    oracle's exact derivative taken along the GPU's FP32 trajectory (its
    states exported every step as FP32 full populations and loaded into the
    tangent run, the tangent carried over) against the FP64 derivative (the
    trajectory part, an upper bound: the export rounds full populations), and
    the GPU's FP32 gradient against the derivative along its own trajectory
    (the adjoint arithmetic part).  Both are reported per cell; each stays
    within 5e-4 of the derivative (floor 1e-3 of the largest), and the total
    within 2e-4."""
    case = _case((32, 24, 16))
    planes = (4, 28)
    T = 100
    N = case.ncells
    cells = I.sample_cells(N, 8, seed_offset=5)
    lat = gpu.Lattice(case, storage="f32")
    traj = [lat.populations().double().cpu().numpy()]
    for _ in range(T):
        lat.step(1)
        traj.append(lat.populations().double().cpu().numpy())
    run = gpu.Lattice(case, storage="f32")
    g = run.new_gradient()
    gpu.lbm_gradient(run.ctx, T, planes, run.new_state_buffer(11), 11, run.new_adjoint(), g)
    g = g.cpu().numpy()[cells]
    exact, along = [], []
    for cell in cells:
        e = np.zeros(N)
        e[cell] = 1.0
        t = oracle_for(case, tangent=True)
        t.set_phi_tangent(e)
        t.step(T)
        exact.append(t.objective(planes)[1])
        o = oracle_for(case, tangent=True)
        o.set_phi_tangent(e)
        v = np.zeros_like(traj[0])
        for s in range(T):
            o.set_populations(traj[s], v)
            o.step(1)
            v = o.populations(with_tangent=True)[1]
        o.set_populations(traj[T], v)
        along.append(o.objective(planes)[1])
    exact, along = np.array(exact), np.array(along)
    sc = np.maximum(np.abs(exact), 1e-3 * np.abs(exact).max())
    tot, traj_part, adj_part = np.abs(g - exact) / sc, np.abs(along - exact) / sc, np.abs(g - along) / sc
    for k, c in enumerate(cells):
        announce(f"cell {c}: dJ/dphi {exact[k]: .4e}  total {tot[k]:.2e}  trajectory {traj_part[k]:.2e}  "
                 f"adjoint {adj_part[k]:.2e}")
    assert tot.max() <= 2e-4 and traj_part.max() <= 5e-4 and adj_part.max() <= 5e-4
