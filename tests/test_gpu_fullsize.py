"""Full-size checks in the launch configuration the benchmark times.

The oracle cannot step a 14 M- or 151 M-cell domain in seconds, but one
step's output at a cell depends only on the state within two cells of it
(neighbours' collisions, their wall-model reference cells).  So after the GPU
has run the full domain for a while, sampled cells are checked one by one:
the GPU state around each sampled cell (a radius-5 crop, so that wall
distances and cell classes are exact within radius 3) is handed to the
oracle, which takes one step; the oracle's populations at the sampled cell
must equal the GPU's after its own next step.  Properties that hold at any
size (mass conservation with walls and the wall model) are checked on the
whole domain.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce

pytestmark = pytest.mark.gpu

R = 5  # crop radius


def _axis_index(c, n, periodic):
    idx = np.arange(c - R, c + R + 1)
    if periodic:
        return idx % n, R
    keep = (idx >= 0) & (idx < n)
    return idx[keep], int(np.flatnonzero(idx == c)[0] - np.flatnonzero(keep)[0])


def _crop(shape, periodic, cell):
    nx, ny, nz = shape
    x, y, z = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    ix, cx = _axis_index(x, nx, periodic[0])
    iy, cy = _axis_index(y, ny, periodic[1])
    iz, cz = _axis_index(z, nz, periodic[2])
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    flat = (X + nx * (Y + ny * Z)).reshape(-1)
    return flat, (len(ix), len(iy), len(iz)), cx + len(ix) * (cy + len(iy) * cz)


def _check_samples(lat, case, cells, f_now, f_next, tol_rel, label):
    q = case.q
    _, w, _ = O.velocity_set(q)
    worst = 0.0
    for cell in cells:
        flat, cshape, center = _crop(case.shape, case.periodic, int(cell))
        idx = torch.as_tensor(flat, device="cuda")
        f0 = f_now[:, idx].double().cpu().numpy()
        f1 = f_next[:, int(cell)].double().cpu().numpy()
        mask = None if case.mask is None else case.mask[flat]
        wd = None
        if case.wall_model:
            wd = I.voxel_wall_distance(np.ones(len(flat), np.uint8) if mask is None else mask, cshape, (0, 0, 0))
            if case.name.startswith("channel"):
                nz = case.shape[2]
                z = flat // (case.shape[0] * case.shape[1])
                wd = np.minimum(z + 0.5, nz - 0.5 - z).astype(np.float64)
        p = O.make_params(q, cshape, periodic=(0, 0, 0), tau0=case.tau0, cs_smag=case.cs_smag, force=case.force,
                          wall_model=case.wall_model, kappa=case.kappa, E=case.E, collision=case.collision,
                          fd_weight=case.fd_weight)
        orc = O.Oracle(p, mask=mask, wall_dist=wd)
        orc.set_populations(f0)
        orc.step(1)
        fo = orc.populations()[:, center]
        err = np.abs(fo - f1).max() / np.abs(f0 - w[:, None]).max()
        worst = max(worst, err)
        assert err <= tol_rel, (label, int(cell), err)
    announce(f"{label}: {len(cells)} sampled cells, worst one-step error {worst:.3e} (of max |g|)")


def _run_sampled(lat, case, steps, cells, tol_rel, label):
    lat.step(steps)
    f_now = lat.populations()
    lat.step(1)
    f_next = lat.populations()
    _check_samples(lat, case, cells, f_now, f_next, tol_rel, label)


@pytest.mark.parametrize("storage,tol", [("f32", 2e-5), ("f16", 3e-3)])
def test_channel_fullsize_sampled(gpu, storage, tol):
    """384x192x192 D3Q27 channel with the wall model: the benchmark's
    configuration, 40 steps, then 24 sampled cells (walls, next to walls, bulk)."""
    case = I.channel(384, 192, 192, q=27)
    announce(f"channel full size {storage}")
    lat = gpu.Lattice(case, storage=storage)
    d0 = lat.diagnostics()
    rng = np.random.default_rng(7)
    nx, ny, nz = case.shape
    cells = []
    for zz in (0, nz - 1, 1, nz - 2, 50, 120):
        for _ in range(4):
            cells.append(int(rng.integers(nx)) + nx * (int(rng.integers(ny)) + ny * zz))
    _run_sampled(lat, case, 40, cells, tol, f"channel {storage}")
    d1 = lat.diagnostics()
    drift = abs(d1[0] - d0[0]) / d0[0]
    announce(f"channel {storage}: mass drift over 41 steps {drift:.3e}")
    assert drift <= (1e-6 if storage == "f32" else 1e-4)


def test_channel_hybrid_fullsize_sampled(gpu):
    """The same channel with RR3 and the hybrid at weight 0.3 (the benchmark's
    hybrid configuration), FP32: a cell's next state also depends on its
    neighbours' velocities, within the crop."""
    case = I.channel(384, 192, 192, q=27)
    case.collision = 1
    case.fd_weight = 0.3
    announce("channel full size, hybrid, f32")
    lat = gpu.Lattice(case, storage="f32")
    rng = np.random.default_rng(9)
    nx, ny, nz = case.shape
    cells = [int(rng.integers(nx)) + nx * (int(rng.integers(ny)) + ny * zz) for zz in (0, nz - 1, 1, nz - 2, 60, 130)
             for _ in range(3)]
    _run_sampled(lat, case, 40, cells, 2e-5, "channel hybrid f32")


def test_urban_fullsize_sampled(gpu):
    """768x768x256 urban canopy (151 M cells, FP32): 20 steps, then sampled
    wall-modeled cells on buildings and ground, and bulk cells (away from the
    fringe and the lid, whose inflow profile depends on the full height)."""
    case = I.urban(768, 768, 256, q=27, with_wall_dist=False)
    announce("urban full size f32")
    lat = gpu.Lattice(case, storage="f32", wall_dist=None)
    rec = lat.wall_records()
    nx, ny, nz = case.shape
    rng = np.random.default_rng(8)
    wc = rec["cells"]
    x = wc % nx
    z = wc // (nx * ny)
    ok = (x >= R + 1) & (x < nx - case.fringe_len - R - 2) & (z < nz - R - 2)
    cells = list(rng.choice(wc[ok], 16, replace=False))
    fl = np.flatnonzero(case.mask)
    xf = fl % nx
    zf = fl // (nx * ny)
    okb = (xf >= R + 1) & (xf < nx - case.fringe_len - R - 2) & (zf < nz - R - 2)
    cells += list(rng.choice(fl[okb], 8, replace=False))
    _run_sampled(lat, case, 20, cells, 2e-5, "urban f32")
