"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, validates arguments, and its checkpoint
schedule is the binomial optimum."""
import math
import os
import re

import numpy as np
import pytest

import paper_2506_21804_amd as lbm
from paper_2506_21804_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_library_loads_and_exports_header_symbols():
    L = lbm.load()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbm.exported_symbols()) == names


def test_workspace_bytes_and_validation():
    p = lbm.make_params(19, (32, 32, 32), storage=lbm.F32DEV, tau0=0.6)
    n = lbm.lbm_workspace_bytes(p)
    assert n >= 19 * 32 ** 3 * 4 + 32 ** 3
    p64 = lbm.make_params(19, (32, 32, 32), storage=lbm.F64, tau0=0.6)
    assert lbm.lbm_workspace_bytes(p64) > n
    p16 = lbm.make_params(27, (32, 32, 32), storage=lbm.F16DEV, tau0=0.6)
    assert lbm.lbm_workspace_bytes(p16) >= 27 * 32 ** 3 * 2
    for bad in (dict(tau0=0.5), dict(tau0=float("nan")), dict(cs_smag=-1.0), dict(storage=7),
                dict(fringe_len=99), dict(collision=2), dict(collision=-1), dict(fd_weight=0.5),
                dict(collision=1, fd_weight=1.5), dict(collision=1, fd_weight=-0.1)):
        kw = dict(tau0=0.6)
        kw.update(bad)
        with pytest.raises(lbm.LbmError):
            lbm.lbm_workspace_bytes(lbm.make_params(19, (32, 32, 32), **kw))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(23, (32, 32, 32), tau0=0.6))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(19, (2048, 1024, 1024), tau0=0.6))
    # one population array at most 4 GiB: 1024^3 FP32 fits exactly, FP64 does not
    assert lbm.lbm_workspace_bytes(lbm.make_params(27, (1024, 1024, 1024), storage=lbm.F32DEV, tau0=0.6)) > 0
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(27, (1024, 1024, 1024), storage=lbm.F64, tau0=0.6))
    assert lbm.lbm_workspace_bytes(lbm.make_params(19, (16, 16, 16), tau0=0.6, collision="rr3")) > 0


def test_wall_cells_counted_in_workspace():
    c = I.channel(16, 8, 10, q=27)
    p = lbm.make_params(27, c.shape, periodic=c.periodic, storage=lbm.F32DEV, tau0=c.tau0, wall_model=1)
    p0 = lbm.make_params(27, c.shape, periodic=c.periodic, storage=lbm.F32DEV, tau0=c.tau0, wall_model=0)
    diff = lbm.lbm_workspace_bytes(p, c.mask) - lbm.lbm_workspace_bytes(p0, c.mask)
    nwall = 2 * 16 * 8
    assert diff >= nwall * (2 * 4 + 12 * 8)


def test_open_x_validation_and_wall_cells():
    """Open x faces: the same constraints as the oracle's, and the cells of
    the two planes are never wall-modeled (the wall list shrinks by exactly
    the ground cells on those planes, counted through the workspace size)."""
    ok = dict(periodic=(0, 1, 0), tau0=0.6, u_ref=0.05, z0=1.0, open_x=1, rho_out=1.0)
    assert lbm.lbm_workspace_bytes(lbm.make_params(19, (16, 8, 10), **ok)) > 0
    for bad in (dict(periodic=(1, 1, 0)), dict(force=(1e-6, 0.0, 0.0)), dict(collision=1, fd_weight=0.3),
                dict(fringe_len=15), dict(rho_out=0.0), dict(rho_out=float("inf")), dict(open_x=2),
                dict(z0=0.0)):
        kw = dict(ok)
        kw.update(bad)
        with pytest.raises(lbm.LbmError):
            lbm.lbm_workspace_bytes(lbm.make_params(19, (16, 8, 10), **kw))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(19, (2, 8, 10), **ok))
    # walls outside z and (closed) outside x: with the wall model every boundary
    # cell of the closed box is a wall cell, N - 14*8*8 = 384 of them; with open
    # x faces only the z walls between the faces remain, 2*14*8 = 224
    shape = (16, 8, 10)
    common = dict(periodic=(0, 1, 0), storage=lbm.F32DEV, tau0=0.6, u_ref=0.05, z0=1.0, wall_model=1)
    n_open = lbm.lbm_workspace_bytes(lbm.make_params(27, shape, open_x=1, **common))
    n_closed = lbm.lbm_workspace_bytes(lbm.make_params(27, shape, open_x=0, **common))
    per_wall = 2 * 4 + 12 * 8  # cell and reference indices, FP64 record
    # open faces add the inlet velocity field (3 ny nz FP32) and the vortex list
    align = lambda b: (b + 255) // 256 * 256
    extra = align(3 * 8 * 10 * 4) + align(lbm.MAX_VORTICES * 3 * 8)
    assert 160 * per_wall <= n_closed - n_open + extra <= 160 * (per_wall + 8) + 4096


def _beta(s, t):
    return math.comb(s + t, s)


@pytest.mark.parametrize("T", [1, 2, 3, 7, 20, 55, 100, 400])
@pytest.mark.parametrize("nsnap", [1, 2, 3, 5, 20])
def test_revolve_cost_is_binomial_optimum(T, nsnap):
    """Forward steps of the reverse sweep equal the Griewank-Walther optimum
    t*l - beta(s+1, t-1), t the least repetition number with l <= beta(s, t)."""
    t = 0
    while _beta(nsnap, t) < T:
        t += 1
    expect = t * T - _beta(nsnap + 1, t - 1) if t > 0 else 0
    assert lbm.lbm_revolve_cost(T, nsnap) == expect


def test_revolve_brute_force_small():
    """Brute-force minimum over all split points for tiny cases."""
    from functools import lru_cache

    @lru_cache(None)
    def best(l, s):
        if l == 1:
            return 0
        if s == 0:
            return l * (l - 1) // 2
        return min(m + best(l - m, s - 1) + best(m, s) for m in range(1, l))

    for l in range(1, 30):
        for snaps in range(1, 6):
            assert lbm.lbm_revolve_cost(l, snaps) == best(l, snaps - 1)


def test_binding_refuses_host_buffers():
    """Device pointers come only from GPU tensors: a host array or CPU tensor
    is refused before any library call."""
    import torch
    with pytest.raises(ValueError):
        lbm._dptr(torch.zeros(4))
    with pytest.raises(ValueError):
        lbm._dptr(np.zeros(4))
