"""Edge cases of the HIP path against the oracle: degenerate domains (one
cell, one-cell-thick slabs, an all-solid box), a one-cell gap whose solid
links cancel (such cells fall back to plain bounce-back under the wall
model), zero-step calls, and the maximum size: a 1024^3 D3Q27 FP32 state,
whose 27 direction arrays are each exactly 4 GiB, the largest one
population array may be, checked on sampled cells."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce, moment_errors, oracle_for, rel_maxnorm

pytestmark = pytest.mark.gpu


def _parity(gpu, case, steps, storage="f64", wall_dist="case"):
    lat = gpu.Lattice(case, storage=storage, wall_dist=wall_dist)
    lat.step(steps)
    f = lat.populations().cpu().numpy().astype(np.float64)
    orc = oracle_for(case, steps)
    fo = orc.populations()
    c, w, _ = O.velocity_set(case.q)
    return lat, rel_maxnorm(f - w[:, None], fo - w[:, None])


@pytest.mark.parametrize("shape,periodic", [((1, 1, 1), (1, 1, 1)), ((5, 3, 1), (1, 1, 1)),
                                            ((1, 7, 4), (1, 1, 0)), ((3, 1, 6), (0, 1, 1))])
def test_degenerate_domains(gpu, shape, periodic):
    """One cell (every neighbour is the cell itself) and one-cell-thick slabs,
    periodic and walled, from a generic non-equilibrium state with a force."""
    q = 27
    N = int(np.prod(shape))
    c, w, _ = O.velocity_set(q)
    f0 = I.random_state(w, N, seed_offset=51, amp=0.04)
    force = (1e-5, 2e-5, -1e-5)
    case = I.Case(name="degenerate", q=q, shape=shape, periodic=periodic, tau0=0.6, cs_smag=0.1, force=force)
    lat = gpu.Lattice(case, storage="f64")
    lat.set_populations(torch.as_tensor(f0))
    orc = O.Oracle(O.make_params(q, shape, periodic=periodic, tau0=0.6, cs_smag=0.1, force=force))
    orc.set_populations(f0)
    for n in (1, 6):
        lat.step(n)
        orc.step(n)
        f = lat.populations().cpu().numpy().astype(np.float64)
        err = rel_maxnorm(f - w[:, None], orc.populations() - w[:, None])
        announce(f"degenerate {shape} per={periodic} after {lat.steps}: {err:.3e}")
        assert err <= 1e-12, err


def test_one_cell_gap_wall_model(gpu):
    """Two solid slabs one cell apart in x inside a channel with the wall model:
    the cells of the gap see cancelling solid links and must run the bulk
    collision with bounce-back, as in the oracle; wall distances from the
    library's voxel routine on the GPU side."""
    nx, ny, nz = 12, 6, 9
    mask3 = np.ones((nz, ny, nx), np.uint8)
    mask3[2:7, :, 3] = 0
    mask3[2:7, :, 5] = 0
    mask = I.flat(mask3)
    case = I.channel(nx, ny, nz, q=19, utau=0.01, nu=1e-3, tau0=0.503, cs_smag=0.1, amp=0.01, wall_model=1)
    case.mask = mask
    case.u0 = case.u0 * mask
    case.wall_dist = I.voxel_wall_distance(mask, case.shape, case.periodic)
    lat, err = _parity(gpu, case, 31, wall_dist=None)
    rec = lat.wall_records()
    gap = [int(x + nx * (y + ny * z)) for z in range(3, 6) for y in range(ny) for x in (4,)]
    announce(f"gap: err {err:.3e}, wall cells {len(rec['cells'])}, gap cells modeled "
             f"{np.isin(gap, rec['cells']).sum()}")
    assert err <= 1e-12, err
    assert not np.isin(gap, rec["cells"]).any()


def test_all_solid_and_zero_steps(gpu):
    case = I.Case(name="solid", q=19, shape=(8, 4, 3), periodic=(1, 1, 0), tau0=0.6, cs_smag=0.1,
                  mask=np.zeros(96, np.uint8))
    lat = gpu.Lattice(case, storage="f32")
    lat.step(0)
    lat.step(3)
    d = lat.diagnostics()
    assert lat.steps == 3 and np.all(np.asarray(d) == 0.0), d
    rho, u = lat.moments()
    assert float(rho.abs().max()) == 0.0 and float(u.abs().max()) == 0.0
    case2 = I.taylor_green(8, q=19)
    lat2 = gpu.Lattice(case2, storage="f64")
    f0 = lat2.populations().cpu().numpy()
    lat2.step(0)
    assert lat2.steps == 0 and np.array_equal(lat2.populations().cpu().numpy(), f0)


R = 5  # crop radius: two steps depend on cells within radius 4


def _crop(shape, cell):
    nx, ny, nz = shape
    x, y, z = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    ix = np.arange(x - R, x + R + 1) % nx
    iy = np.arange(y - R, y + R + 1) % ny
    iz = np.arange(z - R, z + R + 1)
    keep = (iz >= 0) & (iz < nz)
    iz = iz[keep]
    cz = int(np.flatnonzero(np.arange(z - R, z + R + 1)[keep] == z)[0])
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    flat = (X + nx * (Y + ny * Z)).reshape(-1)
    return flat, (len(ix), len(iy), len(iz)), R + len(ix) * (R + len(iy) * cz)


def test_max_size_1024_cubed_sampled(gpu):
    """1024^3 D3Q27 FP32 urban-style canopy (116 GB of populations, each of the
    27 direction arrays exactly 4 GiB) in the benchmark's launch
    configuration: after 10 steps, sampled cells across the whole address
    range (wall cells on the ground and on buildings, bulk cells up to the
    last planes) are stepped twice by the oracle from the GPU state around
    them and compared with the GPU's own two steps.  At an even step count
    the in-place layout is the natural one, so the state is read directly
    from the library's buffer (no export of 116 GB)."""
    case = I.urban(1024, 1024, 1024, q=27, with_wall_dist=False, x_lo=64, x_hi=896, host_fields=False)
    case.u0 = I.urban_u0_device(case)
    announce("max size: 1024^3 D3Q27 f32")
    lat = gpu.Lattice(case, storage="f32", wall_dist=None)
    case.u0 = None
    torch.cuda.empty_cache()
    q, N = 27, case.ncells
    assert N * 4 == 1 << 32
    pops = lat.ws[: q * N * 4].view(torch.float32).view(q, N)
    nx, ny, nz = case.shape
    rng = np.random.default_rng(9)
    rec = lat.wall_records()
    wc = rec["cells"]
    xw, zw = wc % nx, wc // (nx * ny)
    okw = (xw < nx - case.fringe_len - R - 2) & (zw < nz - R - 2)
    cells = list(rng.choice(wc[okw], 6, replace=False))
    # bulk cells spread over the address range, including the top of the array
    for frac in (0.1, 0.5, 0.8, 0.99):
        for _ in range(200):
            cell = int(rng.integers(int(frac * N) - 2000000, int(frac * N)))
            x, z = cell % nx, cell // (nx * ny)
            if case.mask[cell] and x < nx - case.fringe_len - R - 2 and z < nz - R - 2:
                cells.append(cell)
                break
    lat.step(10)
    lat.sync()
    crops = [_crop(case.shape, int(cell)) for cell in cells]
    before = [pops[:, torch.as_tensor(fl, device="cuda")].double().cpu().numpy() for fl, _, _ in crops]
    lat.step(2)
    lat.sync()
    after = pops[:, torch.as_tensor(np.array(cells, dtype=np.int64), device="cuda")].double().cpu().numpy()
    _, w, _ = O.velocity_set(q)
    worst = 0.0
    for k, (cell, (flat, cshape, center)) in enumerate(zip(cells, crops)):
        mask = case.mask[flat]
        wd = I.voxel_wall_distance(mask, cshape, (0, 0, 0))
        p = O.make_params(q, cshape, periodic=(0, 0, 0), tau0=case.tau0, cs_smag=case.cs_smag,
                          wall_model=case.wall_model, kappa=case.kappa, E=case.E)
        orc = O.Oracle(p, mask=mask, wall_dist=wd)
        orc.set_populations(before[k] + w[:, None] * mask[None, :])
        orc.step(2)
        fo = orc.populations()[:, center] - w
        err = np.abs(fo - after[:, k]).max() / np.abs(before[k]).max()
        worst = max(worst, err)
        assert err <= 2e-5, (int(cell), err)
    announce(f"max size: {len(cells)} sampled cells (last at {max(cells)} of {N}), worst {worst:.3e}")
