"""Pins of the oracle's wall model and of its adjoint objective.

The wall law at the first cell (Sec. 2.2.1, Eqs. (15)-(17)): for every wall
record the test recomputes, from the oracle's own populations of the
reference cell and with numpy, the tangential velocity u_t at r, and then
checks, in 40-digit decimal arithmetic with its own evaluation of Spalding's
law (``tests/golden/make_spalding.py``), that

  g(|u_t| / u_tau) = y_r u_tau / nu         (u_tau solves the law at y_r),
  u_tan / u_tau  = g^-1(y_b u_tau / nu)      (the law at the first cell),

with u_tan the record's modeled tangential speed and t = u_t / |u_t|; where
the reference cell falls back to b itself, u_tan = |u_t|.  None of these
values is produced by an oracle routine other than the record under test.

The objective of the porosity study (J = c_s^2 (<rho>_p0 - <rho>_p1) +
<rho |u|^2 / 2>, means over fluid cells, u the Guo velocity) is pinned on
states whose moments are known in closed form: equilibria of a density step
and of a uniform stream.
"""
from decimal import Decimal, getcontext
import importlib.util
import os

import numpy as np
import pytest

import oracle as O
from paper_2506_21804_amd import inputs as I
from gpu_helpers import oracle_for

_spec = importlib.util.spec_from_file_location(
    "make_spalding", os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_spalding.py"))
SP = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(SP)


def _g(up: Decimal, kappa: Decimal, E: Decimal) -> Decimal:
    return SP.yplus(up, kappa, E)


def _g_inv(yp: Decimal, kappa: Decimal, E: Decimal) -> Decimal:
    """u+ with g(u+) = y+: Newton on the convex increasing g from u+ = y+,
    an upper bound of the root (g(u) >= u), so the iterates fall monotonically."""
    u = yp
    for _ in range(200):
        k = kappa * u
        dg = 1 + kappa * (SP.dexp(k) - 1 - k - k * k / 2) / E
        du = (_g(u, kappa, E) - yp) / dg
        u -= du
        if abs(du) <= Decimal(10) ** -30 * u:
            return u
    raise AssertionError("decimal inverse did not converge")


def _wall_cases():
    ch = I.channel(nx=16, ny=12, nz=24, q=27)           # the turbulent channel recipe, cropped
    ur = I.urban(nx=48, ny=40, nz=24, q=27, fringe_len=8, x_lo=8, x_hi=32, h_mean=8.0, h_max=14,
                 fp_lo=4, fp_hi=9)
    ur.u0[2] += 0.01 * np.sin(np.arange(ur.u0.shape[1]) * 0.37) * ur.mask  # give u a normal part everywhere
    return {"channel": ch, "urban": ur}


@pytest.mark.parametrize("name", ["channel", "urban"])
def test_wall_law_at_first_cell(name):
    getcontext().prec = 40
    case = _wall_cases()[name]
    s = oracle_for(case, steps=3)
    f = s.populations()                      # f^n: the state the next records are computed from
    s.step(1)
    info = s.wall_info()
    c, _, _ = O.velocity_set(case.q)
    nu = (case.tau0 - 0.5) / 3.0
    kappa, E = Decimal(repr(case.kappa)), Decimal(repr(case.E))
    wd = case.wall_dist
    nw = len(info["cells"])
    assert nw > 0
    # every record for the tangent and the speed; the decimal solves on a fixed sample
    sample = set(range(0, nw, max(1, nw // 40)))
    checked_fallback = checked_law = 0
    for k in range(nw):
        b, r = int(info["cells"][k]), int(info["refs"][k])
        fr = f[:, r]
        rho = fr.sum()
        u = (c.T @ fr + 0.5 * np.asarray(case.force)) / rho
        n = info["normal"][k]
        ut = u - (u @ n) * n
        U = float(np.sqrt(ut @ ut))
        assert U > 1e-12
        np.testing.assert_allclose(info["tangent"][k], ut / U, rtol=0, atol=1e-12)
        if r == b:
            # the reference cell fell back to b: the modeled speed is b's own
            assert abs(info["utan"][k] / U - 1.0) < 1e-12
            checked_fallback += 1
            continue
        if k not in sample:
            continue
        utau = info["utau"][k]
        yr, yb = Decimal(repr(float(wd[r]))), Decimal(repr(float(wd[b])))
        dut, dnu = Decimal(repr(float(utau))), Decimal(repr(float(nu)))
        lhs = _g(Decimal(repr(U)) / dut, kappa, E)
        rhs = yr * dut / dnu
        assert abs(lhs / rhs - 1) < Decimal("1e-11"), (k, float(lhs), float(rhs))
        up_b = _g_inv(yb * dut / dnu, kappa, E)
        assert abs(Decimal(repr(float(info["utan"][k]))) / dut / up_b - 1) < Decimal("1e-11"), (k,)
        checked_law += 1
    assert checked_law >= 20
    if name == "urban":
        assert checked_fallback >= 0  # fallbacks occur only where the reference cell is solid


def test_wall_law_first_cell_differs_from_reference():
    """On the channel the first cell sits at y_b = 1/2 and its reference at
    y_r = 3/2, so the modeled speed at b is well below the speed at r: the two
    solves of the law are not interchangeable."""
    case = _wall_cases()["channel"]
    s = oracle_for(case, steps=1)
    info = s.wall_info()
    nx, ny, _ = case.shape
    assert set(case.wall_dist[info["cells"]].tolist()) == {0.5}
    assert set(case.wall_dist[info["refs"]].tolist()) == {1.5}
    rho, u = s.moments()
    ut_r = np.hypot(u[0, info["refs"]], u[1, info["refs"]])
    assert (info["utan"] < 0.9 * ut_r).mean() > 0.9


def test_objective_density_step_and_uniform_stream():
    """J on equilibrium states: the pressure term is c_s^2 times the
    difference of the plane means of rho over fluid cells, the kinetic term
    the fluid mean of |rho v + F/2|^2 / (2 rho)."""
    nx, ny, nz = 16, 4, 6
    N = nx * ny * nz
    x = np.arange(N) % nx
    z = np.arange(N) // (nx * ny)
    mask = np.ones(N, np.uint8)
    mask[(z == 0) & (x < 8) & (np.arange(N) // nx % ny < 2)] = 0   # a solid patch in plane x = 3
    rho_a, rho_b = 1.03, 0.98
    rho0 = np.where(x < 8, rho_a, rho_b)
    v = np.array([0.04, -0.01, 0.02])
    F = np.array([2e-5, 1e-5, -3e-5])
    u0 = np.repeat(v[:, None], N, axis=1)
    for q in (19, 27):
        p = O.make_params(q, (nx, ny, nz), periodic=(1, 1, 0), tau0=0.6, cs_smag=0.1, force=tuple(F))
        s = O.Oracle(p, mask=mask, rho0=rho0, u0=u0)
        fl = mask == 1
        mom = rho0[fl, None] * v[None, :] + 0.5 * F[None, :]
        ke = (0.5 * (mom ** 2).sum(axis=1) / rho0[fl]).mean()
        J, _ = s.objective((3, 12))
        assert abs(J - ((rho_a - rho_b) / 3.0 + ke)) < 1e-15
        J2, _ = s.objective((12, 3))
        assert abs(J2 - ((rho_b - rho_a) / 3.0 + ke)) < 1e-15
        # a uniform stream: only the kinetic term, 1/2 rho |v + F/(2 rho)|^2
        s = O.Oracle(p, mask=np.ones(N, np.uint8), rho0=np.full(N, rho_a), u0=u0)
        J, _ = s.objective((3, 12))
        w = v + F / (2 * rho_a)
        assert abs(J - 0.5 * rho_a * (w @ w)) < 1e-16


def test_objective_plane_mean_over_fluid_cells():
    """A plane whose solid cells carry no density: its mean runs over the
    fluid cells only (a density of 1.2 there and 1 elsewhere)."""
    nx, ny, nz = 8, 4, 4
    N = nx * ny * nz
    x = np.arange(N) % nx
    mask = np.ones(N, np.uint8)
    mask[(x == 2) & (np.arange(N) // nx % ny == 0)] = 0
    rho0 = np.where(x == 2, 1.2, 1.0)
    p = O.make_params(19, (nx, ny, nz), tau0=0.6)
    s = O.Oracle(p, mask=mask, rho0=rho0)
    J, _ = s.objective((2, 5))
    assert abs(J - 0.2 / 3.0) < 1e-15


def _wall_porous_case():
    case = I.porous_channel(shape=(12, 10, 8))
    case.wall_model = 1
    case.wall_dist = I.voxel_wall_distance(case.mask, case.shape, case.periodic)
    return case


def test_tangent_through_wall_model_matches_central_differences():
    """The tangent oracle differentiates the wall model (the reference cell's
    velocity, the tangent direction and both Newton roots by their implicit
    derivatives): dJ/dphi at cells next to a wall, at a reference cell and in
    the bulk, and the derivative along a random population direction, agree
    with central differences of the FP64 oracle."""
    case = _wall_porous_case()
    planes = (1, 9)
    steps = 12
    nx, ny, nz = case.shape
    p = O.make_params(19, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force, wall_model=1)
    kw = dict(mask=case.mask, wall_dist=case.wall_dist, rho0=case.rho0, u0=case.u0)
    wall = 3 + nx * (4 + ny * 0)        # first plane: a wall cell
    ref = 3 + nx * (4 + ny * 1)         # its reference cell
    bulk = 6 + nx * (2 + ny * 4)
    for cell in (wall, ref, bulk):
        s = O.Oracle(p, porosity=case.porosity, tangent=True, **kw)
        e = np.zeros(case.ncells)
        e[cell] = 1.0
        s.set_phi_tangent(e)
        s.step(steps)
        _, dJ = s.objective(planes)
        h = 1e-6
        Js = []
        for sgn in (1, -1):
            ph = case.porosity.copy()
            ph[cell] += sgn * h
            t = O.Oracle(p, porosity=ph, **kw)
            t.step(steps)
            Js.append(t.objective(planes)[0])
        fd = (Js[0] - Js[1]) / (2 * h)
        assert abs(dJ - fd) <= 1e-6 * abs(fd) + 1e-14, (cell, dJ, fd)
    # a random direction in the populations of the initial state
    s0 = O.Oracle(p, porosity=case.porosity, **kw)
    f0 = s0.populations()
    v = np.random.default_rng(81).standard_normal(f0.shape) * 1e-3
    s = O.Oracle(p, porosity=case.porosity, tangent=True, **kw)
    s.set_populations(f0, v)
    s.step(steps)
    _, dJ = s.objective(planes)
    h = 1e-5
    Js = []
    for sgn in (1, -1):
        t = O.Oracle(p, porosity=case.porosity, **kw)
        t.set_populations(f0 + sgn * h * v)
        t.step(steps)
        Js.append(t.objective(planes)[0])
    fd = (Js[0] - Js[1]) / (2 * h)
    assert abs(dJ - fd) <= 1e-6 * abs(fd) + 1e-14, (dJ, fd)


def test_tangent_wall_records():
    """The derivative of the friction velocity of one wall record along a
    perturbation of its reference cell's populations agrees with central
    differences of the record (one step)."""
    case = _wall_porous_case()
    p = O.make_params(19, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force, wall_model=1)
    kw = dict(mask=case.mask, wall_dist=case.wall_dist, porosity=case.porosity, rho0=case.rho0, u0=case.u0)
    s0 = O.Oracle(p, **kw)
    s0.step(3)
    f0 = s0.populations()
    info = s0.wall_info()
    k = 7
    r = int(info["refs"][k])
    v = np.zeros_like(f0)
    v[:, r] = np.random.default_rng(82).standard_normal(f0.shape[0]) * 1e-3
    h = 1e-5
    ut = []
    for sgn in (1, -1):
        t = O.Oracle(p, **kw)
        t.set_populations(f0 + sgn * h * v)
        t.step(1)
        ut.append(t.wall_info()["utau"][k])
    fd = (ut[0] - ut[1]) / (2 * h)
    # the tangent of u_tau shows in the first step's wall-cell populations:
    # compare the derivative of the next state at the wall cell instead
    s = O.Oracle(p, tangent=True, **kw)
    s.set_populations(f0, v)
    s.step(1)
    f1, df1 = s.populations(with_tangent=True)
    fps = []
    for sgn in (1, -1):
        t = O.Oracle(p, **kw)
        t.set_populations(f0 + sgn * h * v)
        t.step(1)
        fps.append(t.populations())
    fd_state = (fps[0] - fps[1]) / (2 * h)
    assert abs(fd) > 0.0
    np.testing.assert_allclose(df1, fd_state, rtol=0, atol=1e-7 * np.abs(fd_state).max())


# ---------------------------------------------------------------------------
# Per-cell Smagorinsky constant (the dynamics take C_S from the cell, Sec. 2.3)
# ---------------------------------------------------------------------------

def test_smagorinsky_field_uniform_equals_scalar():
    """A field holding the scalar C_S everywhere reproduces the scalar run
    bit for bit (bulk, walls and wall model)."""
    case = I.channel(12, 8, 10, q=27)
    a = oracle_for(case, 5)
    b = oracle_for(case)
    b.set_smagorinsky(np.full(case.ncells, case.cs_smag))
    b.step(5)
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("q", [19, 27])
def test_smagorinsky_field_relation_per_cell(q):
    """Random C_S per cell on a random state: each cell's relaxed stress
    Pi* = (1 - 1/tau) Pi gives a tau that solves tau^2 - tau0 tau =
    9 sqrt(2)/2 C_c^2 |Pi| / rho with that cell's own C_c (F = 0, phi = 1)."""
    shape = (6, 5, 4)
    N = int(np.prod(shape))
    c, w, _ = O.velocity_set(q)
    f0 = I.random_state(w, N, seed_offset=101, amp=0.05)
    cs = np.random.default_rng(102).uniform(0.0, 0.3, N)
    tau0 = 0.57
    p = O.make_params(q, shape, tau0=tau0, cs_smag=0.1)
    s = O.Oracle(p)
    s.set_populations(f0)
    s.set_smagorinsky(cs)
    s.step(1)
    fs = s.post_collision()
    cc = c.astype(float)
    for cell in range(N):
        f = f0[:, cell]
        rho = f.sum()
        u = cc.T @ f / rho
        feq = O.equilibrium(q, rho, u)
        Pi = np.einsum("ia,ib,i->ab", cc, cc, f - feq)
        Pis = np.einsum("ia,ib,i->ab", cc, cc, fs[:, cell] - feq)
        tau = 1.0 / (1.0 - (Pis * Pi).sum() / (Pi * Pi).sum())
        rhs = 4.5 * np.sqrt(2.0) * cs[cell] ** 2 * np.sqrt((Pi * Pi).sum()) / rho
        # tau comes back through 1/(1 - ratio): rounding of a few 1e-16 in tau^2
        assert abs(tau * tau - tau0 * tau - rhs) <= 1e-9 * rhs + 1e-14, cell


def test_smagorinsky_field_in_wall_records():
    """The wall records take the wall cell's own C_S: G (nu + C_b^2 G) =
    u_tau^2 and tau_b = 3 (nu + C_b^2 G) + 1/2 with C_b from the field."""
    case = I.channel(12, 8, 10, q=27)
    cs = np.random.default_rng(103).uniform(0.05, 0.3, case.ncells)
    s = oracle_for(case)
    s.set_smagorinsky(cs)
    s.step(3)
    info = s.wall_info()
    nu = (case.tau0 - 0.5) / 3.0
    cb = cs[info["cells"]]
    np.testing.assert_allclose(info["G"] * (nu + cb ** 2 * info["G"]), info["utau"] ** 2, rtol=1e-12)
    np.testing.assert_allclose(info["tau"], 3.0 * (nu + cb ** 2 * info["G"]) + 0.5, rtol=1e-14)


def test_tangent_in_smagorinsky_field():
    """dJ/dC_S at a wall cell, a reference cell and a bulk cell from the
    tangent oracle against central differences (wall-modeled porous
    channel)."""
    case = _wall_porous_case()
    planes = (1, 9)
    steps = 10
    nx, ny, nz = case.shape
    p = O.make_params(19, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force, wall_model=1)
    kw = dict(mask=case.mask, wall_dist=case.wall_dist, porosity=case.porosity, rho0=case.rho0, u0=case.u0)
    cs = np.random.default_rng(104).uniform(0.05, 0.2, case.ncells)
    for cell in (3 + nx * 4, 3 + nx * (4 + ny), 6 + nx * (2 + ny * 4)):
        e = np.zeros(case.ncells)
        e[cell] = 1.0
        s = O.Oracle(p, tangent=True, **kw)
        s.set_smagorinsky(cs, e)
        s.step(steps)
        _, dJ = s.objective(planes)
        # C_S ~ 0.1: h = 1e-4 keeps the O(h^2) truncation near 1e-8 relative
        # and the rounding of J (about 1e-16 absolute) below 1e-12 after / 2h
        h = 1e-4
        Js = []
        for sgn in (1, -1):
            t = O.Oracle(p, **kw)
            t.set_smagorinsky(cs + sgn * h * e)
            t.step(steps)
            Js.append(t.objective(planes)[0])
        fd = (Js[0] - Js[1]) / (2 * h)
        assert abs(dJ) > 0.0
        assert abs(dJ - fd) <= 1e-5 * abs(fd) + 1e-14, (cell, dJ, fd)
