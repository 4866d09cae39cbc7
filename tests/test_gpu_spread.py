"""Workspace and adjoint buffers with their arrays spread in physical memory
(lbm_workspace_alloc, lbm_adjoint_alloc, lbm_spread_free): the layout is the
ordinary one, so every result must be bit-identical to a run on a plain
allocation.  Shapes include arrays whose byte size is not a multiple of the
mapping granularity (arrays straddle the pieces)."""
import numpy as np
import pytest
import torch

from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _wall_porous(shape=(16, 12, 8), collision=0):
    c = I.porous_channel(shape=shape)
    c.wall_model = 1
    c.wall_dist = I.voxel_wall_distance(c.mask, c.shape, c.periodic)
    c.collision = collision
    return c


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("shape", [(37, 23, 19), (64, 48, 40)])
def test_spread_workspace_bitwise(gpu, storage, shape):
    case = I.channel(*shape, q=27)
    announce(f"spread workspace: channel {shape} {storage}")
    a = gpu.Lattice(case, storage=storage)
    b = gpu.Lattice(case, storage=storage, spread=True)
    assert isinstance(b.workspace, gpu.SpreadBuffer) and b.workspace.data_ptr() % 256 == 0
    for n in (1, 8):
        a.step(n)
        b.step(n)
        assert torch.equal(a.populations(), b.populations())
    assert np.array_equal(a.diagnostics(), b.diagnostics())


def test_spread_urban_crop(gpu):
    case = I.urban(nx=40, ny=24, nz=16, q=19, tau0=0.52, fringe_len=6, x_lo=6, x_hi=30, h_mean=6.0, h_max=10,
                   fp_lo=3, fp_hi=7)
    a = gpu.Lattice(case, storage="f32")
    b = gpu.Lattice(case, storage="f32", spread=True)
    a.step(15)
    b.step(15)
    assert torch.equal(a.populations(), b.populations())


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_spread_adjoint_bitwise(gpu, storage):
    case = _wall_porous(collision=1)
    planes = (2, 13)
    out = []
    for spread in (False, True):
        lat = gpu.Lattice(case, storage=storage, spread=spread)
        lam = lat.new_adjoint(spread=spread)
        if spread:
            assert isinstance(lam, gpu.SpreadBuffer)
        grad = lat.new_gradient()
        J, _ = gpu.lbm_gradient(lat.ctx, 12, planes, lat.new_state_buffer(3), 3, lam, grad)
        nat = lat.new_natural()
        gpu.lbm_adjoint_to_natural(lat.ctx, lam, nat)
        lat.sync()
        out.append((J, grad.cpu(), nat.cpu()))
        if spread:
            lam.free()
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1]) and torch.equal(out[0][2], out[1][2])


def test_spread_free_and_errors(gpu):
    case = I.channel(24, 16, 12, q=19)
    lat = gpu.Lattice(case, storage="f32", spread=True)
    lam = lat.new_adjoint(spread=True)
    lam.free()
    lam.free()  # a second free is a no-op
    with pytest.raises(ValueError):
        lam.data_ptr()
    # a pointer the allocator did not make is refused
    t = torch.empty(1024, dtype=torch.uint8, device="cuda")
    rc = gpu.load().lbm_spread_free(gpu.C.c_void_p(t.data_ptr()))
    assert rc == gpu.EINVAL
    lat.step(3)
    assert np.isfinite(lat.diagnostics()[0])
