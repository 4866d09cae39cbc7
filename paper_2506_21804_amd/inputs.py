"""Seeded synthetic inputs for the LBM-LES workloads.

This module only builds input arrays: voxel masks, wall-distance fields,
porosity fields and initial density/velocity fields, all from numpy's
``Generator(PCG64(seed))`` with seed base 2506.  It contains none of the
lattice Boltzmann arithmetic, so the HIP path and the CPU oracle can both be
fed from it without sharing any of the method.

Array conventions: a scalar field has N = nx*ny*nz entries indexed
``x + nx*(y + ny*z)``; a vector field is [3][N].  ``mask`` is uint8, 1 for
fluid and 0 for solid.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2506


def _rng(offset: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + offset))


def flat(a3: np.ndarray) -> np.ndarray:
    """[nz][ny][nx] array -> flat cell order x + nx*(y + ny*z)."""
    return np.ascontiguousarray(a3).reshape(-1)


@dataclass
class Case:
    """A complete input set for one run (physical parameters plus arrays)."""
    name: str
    q: int
    shape: tuple  # (nx, ny, nz)
    periodic: tuple
    tau0: float
    cs_smag: float
    force: tuple = (0.0, 0.0, 0.0)
    wall_model: int = 0
    kappa: float = 0.41
    E: float = 9.0
    fringe_len: int = 0
    u_ref: float = 0.0
    z0: float = 1.0
    lid: int = 0
    collision: int = 0  # 0 BGK, 1 recursive regularized (third order)
    fd_weight: float = 0.0  # 1 - sigma: weight of the finite-difference strain (collision 1 only)
    open_x: int = 0  # 1: velocity inlet at x = 0, pressure outlet at x = nx - 1 (x not periodic)
    rho_out: float = 1.0  # outlet density (open_x only)
    slip: int = 0  # full-slip box faces: bit 2a the low face of axis a, bit 2a+1 the high face
    mask: np.ndarray | None = None
    wall_dist: np.ndarray | None = None
    porosity: np.ndarray | None = None
    rho0: np.ndarray | None = None
    u0: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def nfluid(self) -> int:
        return self.ncells if self.mask is None else int(np.count_nonzero(self.mask))


# ---------------------------------------------------------------------------
# Geometry helpers
# ---------------------------------------------------------------------------

def voxel_wall_distance(mask: np.ndarray, shape, periodic, radius: int = 2, slip: int = 0) -> np.ndarray:
    """Distance from each cell centre to the nearest solid voxel (a unit cube)
    within ``radius`` cells in every axis; cells outside a non-periodic axis
    count as solid, except beyond a full-slip face (``slip`` bit 2a: the low
    face of axis a, 2a+1 the high face), where the geometry continues as its
    mirror image.  Cells with no solid voxel in that neighbourhood get +inf.

    A cell next to a flat wall gets 0.5, next to a convex edge sqrt(0.5), next
    to a corner sqrt(0.75).  Radius 2 covers every wall cell and every cell
    one lattice step away from one.
    """
    nx, ny, nz = shape
    solid = (np.asarray(mask).reshape(nz, ny, nx) == 0)
    R = radius
    # pad with wrap on periodic axes, with solid on the others, mirrored
    # beyond full-slip faces (array axis 0 is z, 2 is x)
    padded = solid
    for ax, a in zip((0, 1, 2), (2, 1, 0)):
        if periodic[a]:
            widths = [(0, 0)] * 3
            widths[ax] = (R, R)
            padded = np.pad(padded, widths, mode="wrap")
            continue
        for side in (0, 1):
            widths = [(0, 0)] * 3
            widths[ax] = (R, 0) if side == 0 else (0, R)
            if (slip >> (2 * a + side)) & 1:
                padded = np.pad(padded, widths, mode="symmetric")
            else:
                padded = np.pad(padded, widths, mode="constant", constant_values=True)
    offs = []
    for dz in range(-R, R + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                if dx == dy == dz == 0:
                    continue
                g = [max(abs(d) - 0.5, 0.0) for d in (dx, dy, dz)]
                offs.append((float(np.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])), dx, dy, dz))
    offs.sort()
    dist = np.full((nz, ny, nx), np.inf)
    for d, dx, dy, dz in offs:
        sh = padded[R + dz:R + dz + nz, R + dy:R + dy + ny, R + dx:R + dx + nx]
        sel = sh & np.isinf(dist)
        dist[sel] = d
    return flat(dist)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def taylor_green(n: int = 32, u0: float = 0.05, q: int = 19, tau0: float = 0.6, cs_smag: float = 0.1,
                 two_d: bool = False) -> Case:
    """Fully periodic Taylor-Green vortex on an n^3 box (k = 2 pi / n).

    3D form: u = u0 sin kx cos ky cos kz, v = -u0 cos kx sin ky cos kz, w = 0,
    rho = 1 + 3 (u0^2/16)(cos 2kx + cos 2ky)(cos 2kz + 2).
    2D form (used for the analytic decay check): u = -u0 cos kx sin ky,
    v = u0 sin kx cos ky, w = 0, rho = 1 - 3 (u0^2/4)(cos 2kx + cos 2ky).
    """
    k = 2.0 * np.pi / n
    c = np.arange(n) + 0.0
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    if two_d:
        ux = -u0 * np.cos(k * X) * np.sin(k * Y)
        uy = u0 * np.sin(k * X) * np.cos(k * Y)
        rho = 1.0 - 3.0 * (u0 * u0 / 4.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    else:
        ux = u0 * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z)
        uy = -u0 * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z)
        rho = 1.0 + 3.0 * (u0 * u0 / 16.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * (np.cos(2 * k * Z) + 2.0)
    uz = np.zeros_like(ux)
    u = np.stack([flat(ux), flat(uy), flat(uz)])
    return Case(name=f"tgv{n}", q=q, shape=(n, n, n), periodic=(1, 1, 1), tau0=tau0, cs_smag=cs_smag,
                rho0=flat(rho), u0=u, extra=dict(u0=u0, k=k))


def channel(nx: int = 384, ny: int = 192, nz: int = 192, q: int = 27, seed_offset: int = 2,
            utau: float = 0.0045, nu: float = 4.32e-4, tau0: float = 0.501296, cs_smag: float = 0.1,
            amp: float = 0.01, wall_model: int = 1, kappa: float = 0.41, E: float = 9.0) -> Case:
    """Body-force-driven plane channel, x streamwise, walls outside z.

    Half height h = nz/2, Re_tau = utau h / nu (1000 at the defaults;
    tau0 = 3 nu + 1/2 written out), force F_x = utau^2 / h.  The initial
    streamwise velocity is a two-layer mean profile (u+ = y+ up to y+ = 11,
    ln(E y+)/kappa above) plus seeded uniform noise of amplitude ``amp`` on
    every component.
    """
    N = nx * ny * nz
    h = nz / 2.0
    z = np.arange(nz) + 0.0
    y = np.minimum(z + 0.5, nz - 0.5 - z)
    yp = y * utau / nu
    up = np.where(yp < 11.0, yp, np.log(E * np.maximum(yp, 1e-30)) / kappa)
    prof = utau * up
    rng = _rng(seed_offset)
    u = np.empty((3, N))
    noise = rng.uniform(0.0, 1.0, size=(3, N))
    u[0] = np.repeat(prof, nx * ny) + amp * (2.0 * noise[0] - 1.0)
    u[1] = amp * (2.0 * noise[1] - 1.0)
    u[2] = amp * (2.0 * noise[2] - 1.0)
    wd = np.repeat(y, nx * ny)
    return Case(name=f"channel{nx}x{ny}x{nz}", q=q, shape=(nx, ny, nz), periodic=(1, 1, 0), tau0=tau0,
                cs_smag=cs_smag, force=(utau * utau / h, 0.0, 0.0), wall_model=wall_model, kappa=kappa,
                E=E, mask=np.ones(N, np.uint8), wall_dist=wd, rho0=np.ones(N), u0=u,
                extra=dict(utau=utau, nu=nu, h=h))


def building_mask(nx: int, ny: int, nz: int, seed_offset: int = 3, x_lo: int = 64, x_hi: int | None = None,
                  fp_lo: int = 8, fp_hi: int = 40, h_mean: float = 40.0, h_sigma: float = 0.5,
                  h_max: int = 192, plan_frac: float = 0.30) -> np.ndarray:
    """Random rectangular buildings on a flat ground, as [nz][ny][nx] uint8 (1 = fluid).

    Footprints uniform integer fp_lo..fp_hi per side, heights
    round(lognormal(ln h_mean - sigma^2/2, sigma)) clipped to [4, h_max],
    uniform positions with x in [x_lo, x_hi) and y anywhere (no wrap), added
    until the plan-area fraction of that region reaches ``plan_frac``.
    """
    if x_hi is None:
        x_hi = nx - 128
    rng = _rng(seed_offset)
    foot = np.zeros((ny, nx), bool)
    height = np.zeros((ny, nx), np.int32)
    area = (x_hi - x_lo) * ny
    mu = np.log(h_mean) - 0.5 * h_sigma * h_sigma
    h_cap = min(h_max, nz - 8)
    while foot[:, x_lo:x_hi].sum() < plan_frac * area:
        wx = int(rng.integers(fp_lo, fp_hi + 1))
        wy = int(rng.integers(fp_lo, fp_hi + 1))
        hh = int(np.clip(np.round(rng.lognormal(mu, h_sigma)), 4, h_cap))
        x0 = int(rng.integers(x_lo, max(x_lo + 1, x_hi - wx + 1)))
        y0 = int(rng.integers(0, max(1, ny - wy + 1)))
        foot[y0:y0 + wy, x0:x0 + wx] = True
        height[y0:y0 + wy, x0:x0 + wx] = np.maximum(height[y0:y0 + wy, x0:x0 + wx], hh)
    z = np.arange(nz)[:, None, None]
    solid = z < height[None, :, :]
    return (~solid).astype(np.uint8)


def urban(nx: int = 768, ny: int = 768, nz: int = 256, q: int = 27, seed_offset: int = 3,
          u_ref: float = 0.08, tau0: float = 0.5003, cs_smag: float = 0.2, fringe_len: int = 64,
          with_wall_dist: bool = True, x_lo: int = 64, x_hi: int | None = None,
          h_mean: float = 40.0, h_max: int = 192, fp_lo: int = 8, fp_hi: int = 40,
          host_fields: bool = True, open_x: bool = False, slip_walls: bool = False) -> Case:
    """Synthetic urban canopy: random buildings on a wall-modeled ground,
    periodic x with a fringe over the last ``fringe_len`` planes, periodic y,
    lid layer on top (with ``open_x``: a velocity inlet at x = 0 and a
    pressure outlet at x = nx - 1 instead of the periodic x axis, the fringe
    kept before the outlet; the wall distance still treats x as unbounded);
    initial velocity u_ref ln(1 + z_c/z0)/ln(1 + z_top/z0)
    in x (z_c = z + 1/2, z_top = nz - 1/2, z0 = 1) in fluid cells.  With
    ``slip_walls`` the outer walls are full-slip faces, as in the street-canyon
    setup: the two y faces and the top face (no lid, y not periodic).

    C_S defaults to 0.2: with the BGK collision, nu = 1e-4 and wall-modeled
    building faces, C_S = 0.1 lets the flow between buildings accelerate past
    Mach 0.6 within ~80 steps; 0.2 keeps max|u| near 0.25 over 600 steps."""
    if x_hi is None:
        x_hi = nx - fringe_len - 64
    m3 = building_mask(nx, ny, nz, seed_offset, x_lo=x_lo, x_hi=x_hi, h_mean=h_mean, h_max=h_max,
                       fp_lo=fp_lo, fp_hi=fp_hi)
    mask = flat(m3)
    del m3
    N = nx * ny * nz
    z0 = 1.0
    u = None
    if host_fields:
        u = np.zeros((3, N))
        u[0] = np.repeat(log_profile(nz, u_ref, z0), nx * ny) * mask
    periodic = (0 if open_x else 1, 0 if slip_walls else 1, 0)
    slip = 0b101100 if slip_walls else 0
    wd = voxel_wall_distance(mask, (nx, ny, nz), (1, periodic[1], 0), slip=slip) if with_wall_dist else None
    return Case(name=f"urban{nx}x{ny}x{nz}" + ("_open" if open_x else "") + ("_slip" if slip_walls else ""), q=q,
                shape=(nx, ny, nz), periodic=periodic, tau0=tau0, cs_smag=cs_smag, wall_model=1,
                fringe_len=fringe_len, u_ref=u_ref, z0=z0, lid=0 if slip_walls else 1, open_x=int(open_x),
                slip=slip, mask=mask, wall_dist=wd, rho0=None, u0=u)


def log_profile(nz: int, u_ref: float, z0: float = 1.0) -> np.ndarray:
    """u_ref ln(1 + z_c/z0) / ln(1 + z_top/z0) at cell centres z_c = z + 1/2, z_top = nz - 1/2."""
    zc = np.arange(nz) + 0.5
    return u_ref * np.log(1.0 + zc / z0) / np.log(1.0 + (nz - 0.5) / z0)


def urban_u0_device(case: Case):
    """The urban initial velocity [3][N] (float64) built directly in GPU
    memory from the inflow profile and the mask, for domains whose host copy
    would not fit (a 1024^3 field is 25.8 GB)."""
    import torch
    nx, ny, nz = case.shape
    prof = torch.as_tensor(log_profile(nz, case.u_ref, case.z0), device="cuda")
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float64, device="cuda")
    u[0] = prof[:, None, None]
    u[0] *= torch.as_tensor(case.mask.reshape(nz, ny, nx), device="cuda").to(torch.float64)
    return u.reshape(3, -1)


def cavity(n=575, q: int = 19, u_lid: float = 0.05, tau0: float = 0.51, cs_smag: float = 0.1) -> Case:
    """Lid-driven cavity: a box of fluid (n^3, or n = (nx, ny, nz)) with every
    axis non-periodic, so all six faces are halfway bounce-back walls, and the
    top plane held at the lid equilibrium of velocity u_lid along x.  Starts at
    rest; no wall model, no force.  575^3 is the smallest of the paper's
    scaling problems and one GPU's share of 1449^3 on 16 GPUs."""
    shape = (n, n, n) if isinstance(n, int) else tuple(n)
    name = f"cavity{shape[0]}" if len(set(shape)) == 1 else "cavity{}x{}x{}".format(*shape)
    return Case(name=name, q=q, shape=shape, periodic=(0, 0, 0), tau0=tau0, cs_smag=cs_smag, u_ref=u_lid, lid=1)


def porosity_field(shape, seed_offset: int = 4, passes: int = 3, width: int = 9) -> np.ndarray:
    """Smoothed noise in [0, 1]: U(0,1) noise, ``passes`` periodic box filters
    of ``width`` cells along each axis, then min-max normalisation."""
    nx, ny, nz = shape
    a = _rng(seed_offset).uniform(0.0, 1.0, size=(nz, ny, nx))
    half = width // 2
    for _ in range(passes):
        for ax in range(3):
            acc = np.zeros_like(a)
            for s in range(-half, half + 1):
                acc += np.roll(a, s, axis=ax)
            a = acc / width
    a = (a - a.min()) / (a.max() - a.min())
    return flat(a)


def porous_channel(n: int = 128, q: int = 19, tau0: float = 0.6, cs_smag: float = 0.1, fx: float = 1e-5,
                   u0x: float = 0.05, seed_offset: int = 4, shape=None) -> Case:
    """Porosity-gradient workload: x/y periodic, bounce-back walls outside z,
    body force F_x, uniform initial velocity u0x, porosity from
    ``porosity_field``; objective planes at x = n/8 and x = 7n/8."""
    if shape is None:
        shape = (n, n, n)
    nx, ny, nz = shape
    N = nx * ny * nz
    u = np.zeros((3, N))
    u[0] = u0x
    return Case(name=f"porous{nx}x{ny}x{nz}", q=q, shape=shape, periodic=(1, 1, 0), tau0=tau0,
                cs_smag=cs_smag, force=(fx, 0.0, 0.0), mask=np.ones(N, np.uint8),
                porosity=porosity_field(shape, seed_offset), rho0=np.ones(N), u0=u,
                extra=dict(planes=(nx // 8, 7 * nx // 8)))


def sample_cells(ncells: int, count: int, seed_offset: int = 5, mask=None) -> np.ndarray:
    """``count`` distinct cell indices, uniform over (fluid) cells."""
    rng = _rng(seed_offset)
    pool = np.arange(ncells) if mask is None else np.flatnonzero(np.asarray(mask))
    return np.sort(rng.choice(pool, size=count, replace=False))


def random_state(base, ncells: int, seed_offset: int, amp: float = 0.01) -> np.ndarray:
    """Random positive populations base[i] * (1 + amp * U(-1, 1)), [q][N]
    (for checks that need a generic non-equilibrium state)."""
    base = np.asarray(base, dtype=np.float64)
    rng = _rng(seed_offset)
    return base[:, None] * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(base.size, ncells)))
