"""Pins of the oracle's hybrid collision (Sec. 2.2, Eqs. (7), (10), and the
wall region of Sec. 2.2.1) against closed forms.  The states are exact
third-order equilibria of prescribed velocity fields, optionally plus a
perturbation without mass or momentum, so that the finite-difference strain
of the field is known exactly (central differences are exact for quadratic
profiles, one-sided ones next to a wall are written out here), and every
post-collision second moment follows from the collision's definition:

  sum_i c_a c_b f*_i - rho c_s^2 d_ab - rho u_a u_b
      = (1 - 1/tau) [sigma Pi^neq - (1 - sigma) 2 rho c_s^2 tau S^FD]_ab

in the bulk (no force).  The third moments keep the factor
sigma on the recursive part.  In a wall cell the wall law replaces the
wall-normal shear of S^FD (in every tangential direction) by its own,
(G/2)(t n^T + n t^T), and the rest of S^FD is kept."""
import numpy as np
import pytest

import oracle as O
import test_oracle_pins_rr as prr

CS2 = 1.0 / 3.0


def _eq_state(q, shape, u):
    """f = f^eq3(1, u(x)) at every cell; u is [3][N]."""
    N = int(np.prod(shape))
    f = np.empty((q, N))
    for c in range(N):
        f[:, c] = O.equilibrium3(q, 1.0, u[:, c])
    return f


def _second(c, f):
    return np.einsum("ia,ib,in->nab", c, c, f)


@pytest.mark.parametrize("q", [19, 27])
def test_hybrid_fd_stress_quadratic_shear(q):
    """sigma = 0 on u_x = g y_c + k y_c^2 between walls in y (y_c = y + 1/2):
    central differences inside, one-sided at the first and last row."""
    nx, ny, nz = 4, 10, 3
    shape = (nx, ny, nz)
    N = nx * ny * nz
    gam, kap = 1e-3, 2e-4
    yc = (np.arange(N) // nx) % ny + 0.5
    u = np.zeros((3, N))
    u[0] = gam * yc + kap * yc ** 2
    c, w, _ = O.velocity_set(q)
    f = _eq_state(q, shape, u)
    tau0 = 0.7
    p = O.make_params(q, shape, periodic=(1, 0, 1), tau0=tau0, cs_smag=0.0, collision=1, fd_weight=1.0)
    s = O.Oracle(p)
    s.set_populations(f)
    s.step(1)
    fs = s.post_collision()
    M2 = _second(c, fs)
    y = (np.arange(N) // nx) % ny
    dudy = np.where(y == 0, (gam * 1.5 + kap * 1.5 ** 2) - (gam * 0.5 + kap * 0.25),
                    np.where(y == ny - 1, (gam * (ny - 0.5) + kap * (ny - 0.5) ** 2) -
                             (gam * (ny - 1.5) + kap * (ny - 1.5) ** 2), gam + 2 * kap * yc))
    Sxy = 0.5 * dudy
    expect_xy = (1 - 1 / tau0) * (-2.0 * CS2 * tau0 * Sxy) + u[0] * u[1]
    assert np.abs(M2[:, 0, 1] - expect_xy).max() <= 1e-16
    # diagonal: rho c_s^2 + rho u_a^2 (S has no diagonal part)
    assert np.abs(M2[:, 0, 0] - (CS2 + u[0] ** 2)).max() <= 1e-15
    assert np.abs(M2[:, 2, 2] - CS2).max() <= 1e-15


@pytest.mark.parametrize("q", [19, 27])
def test_hybrid_blend_and_third_moments(q):
    """sigma = 0.7 on a periodic box with u_y = a sin(2 pi x / nx) plus a
    perturbation without mass or momentum: the second moments blend Pi^neq
    and the FD stress, the third keep sigma on the recursive part.  In a wall cell the wall law replaces the
wall-normal shear of S^FD (in every tangential direction) by its own,
(G/2)(t n^T + n t^T), and the rest of S^FD is kept."""
    nx, ny, nz = 8, 3, 3
    shape = (nx, ny, nz)
    N = nx * ny * nz
    x = np.arange(N) % nx
    a = 0.01
    u = np.zeros((3, N))
    u[1] = a * np.sin(2 * np.pi * x / nx)
    c, w, _ = O.velocity_set(q)
    f = _eq_state(q, shape, u)
    rng = np.random.default_rng(3)
    C = np.vstack([np.ones(q), c.T.astype(float)])
    r = 1e-4 * rng.standard_normal((q, N)) * w[:, None] / w.max()
    g = r - C.T @ np.linalg.solve(C @ C.T, C @ r)  # no mass, no momentum
    assert np.abs(C @ g).max() < 1e-18
    f = f + g
    tau0, cs, fdw = 0.6, 0.12, 0.3
    p = O.make_params(q, shape, periodic=(1, 1, 1), tau0=tau0, cs_smag=cs, collision=1, fd_weight=fdw)
    s = O.Oracle(p)
    s.set_populations(f)
    s.step(1)
    fs = s.post_collision()
    M2 = _second(c, fs)
    du = a * (np.sin(2 * np.pi * (x + 1) / nx) - np.sin(2 * np.pi * (x - 1) / nx)) / 2
    for cell in range(0, N, 7):
        rho = f[:, cell].sum()
        uc = (c.T @ f[:, cell]) / rho
        Pi = np.einsum("ia,ib,i->ab", c, c, f[:, cell]) - rho * CS2 * np.eye(3) - rho * np.outer(uc, uc)
        tau = O.tau_eff(tau0, cs, float(np.sqrt((Pi ** 2).sum())), rho)
        S = np.zeros((3, 3))
        S[0, 1] = S[1, 0] = 0.5 * du[cell]
        Ph = (1 - fdw) * Pi - fdw * 2.0 * CS2 * rho * tau * S
        exp2 = rho * CS2 * np.eye(3) + rho * np.outer(uc, uc) + (1 - 1 / tau) * Ph
        assert np.abs(M2[cell] - exp2).max() <= 1e-15, cell
        A0 = rho * np.einsum("a,b,g->abg", uc, uc, uc)
        A1 = np.einsum("a,bg->abg", uc, Pi) + np.einsum("b,ag->abg", uc, Pi) + np.einsum("g,ab->abg", uc, Pi)
        for terms in prr._admissible(q):
            m = float(prr._poly(c, terms) @ fs[:, cell])
            e = prr._contract(terms, A0) + (1 - 1 / tau) * (1 - fdw) * prr._contract(terms, A1)
            assert abs(m - e) <= 1e-15, (cell, terms, m, e)


def _wall_run(fdw, u, shape, tau0=0.55):
    q = 19
    c, w, _ = O.velocity_set(q)
    f = _eq_state(q, shape, u)
    nx, ny, nz = shape
    zc = np.arange(nx * ny * nz) // (nx * ny) + 0.5
    zdist = np.minimum(zc, nz - zc)
    p = O.make_params(q, shape, periodic=(1, 1, 0), tau0=tau0, cs_smag=0.1, wall_model=1, collision=1,
                      fd_weight=fdw)
    s = O.Oracle(p, wall_dist=zdist)
    s.set_populations(f)
    s.step(1)
    info = s.wall_info()
    ground = np.flatnonzero(info["cells"] < nx * ny)
    assert len(ground) == nx * ny
    return _second(c, s.post_collision()), info, ground


@pytest.mark.parametrize("fdw", [0.0, 1.0])
def test_hybrid_wall_shear_replaced(fdw):
    """Ground cells of a channel carrying u_x = a + b z_c, u_y = d z_c
    (z_c = z + 1/2): the finite-difference strain has only the wall-normal
    shear S_xz = b/2, S_yz = d/2, which the wall law replaces by
    (G/2)(t n^T + n t^T), with or without the hybrid collision."""
    nx, ny, nz = 4, 4, 6
    N = nx * ny * nz
    zc = np.arange(N) // (nx * ny) + 0.5
    a, b, d = 0.02, 0.004, 0.002
    u = np.zeros((3, N))
    u[0] = a + b * zc
    u[1] = d * zc
    M2, info, ground = _wall_run(fdw, u, (nx, ny, nz))
    ur = np.array([a + 1.5 * b, 1.5 * d, 0.0])  # reference cell of a ground cell: one step up
    t = ur / np.linalg.norm(ur)
    for k in ground:
        G, tau = info["G"][k], info["tau"][k]
        cell = info["cells"][k]
        # the modeled velocity has no z component, so these moments are the stress alone
        for (i, j), tn in (((0, 2), t[0]), ((1, 2), t[1])):
            expect = (1 - 1 / tau) * (-2.0 * CS2 * tau * 0.5 * G * tn)
            assert abs(M2[cell, i, j] - expect) <= 1e-18 + 1e-12 * abs(expect), (k, fdw, i, j)


def test_hybrid_wall_keeps_normal_strain():
    """With the hybrid collision the wall cell keeps the rest of the
    finite-difference strain: u_z = h z_c gives the one-sided S_zz = h at the
    ground, and the zz moment is rho (c_s^2 + u_z^2) + (1 - 1/tau)(-2 rho c_s^2 tau h)
    (the modeled velocity keeps the local normal component u_z = h/2)."""
    nx, ny, nz = 4, 4, 6
    N = nx * ny * nz
    zc = np.arange(N) // (nx * ny) + 0.5
    h = 3e-4
    u = np.zeros((3, N))
    u[0] = 0.02 + 0.004 * zc
    u[2] = h * zc
    M2, info, ground = _wall_run(1.0, u, (nx, ny, nz))
    for k in ground:
        tau = info["tau"][k]
        cell = info["cells"][k]
        expect = CS2 + (0.5 * h) ** 2 + (1 - 1 / tau) * (-2.0 * CS2 * tau * h)
        assert abs(M2[cell, 2, 2] - expect) <= 1e-15, (k, M2[cell, 2, 2], expect)


def test_fd_weight_checked():
    with pytest.raises(O.OracleError):
        O.Oracle(O.make_params(19, (4, 4, 4), tau0=0.6, collision=0, fd_weight=0.5))
    with pytest.raises(O.OracleError):
        O.Oracle(O.make_params(19, (4, 4, 4), tau0=0.6, collision=1, fd_weight=1.5))


def test_tangent_through_the_hybrid_matches_central_differences():
    """The tangent oracle differentiates the hybrid collision (the
    finite-difference strain of the neighbours' velocities, the blend, and at
    wall cells the full strain with the law's wall-normal shear): dJ/dphi at
    a wall cell, a reference cell and a bulk cell, and along a random
    population direction, against central differences of the FP64 oracle.
    (The wall cell's own porosity does not enter its reconstruction: there
    both are exactly 0.)"""
    from paper_2506_21804_amd import inputs as I
    case = I.porous_channel(shape=(12, 10, 8))
    case.wall_model = 1
    case.wall_dist = I.voxel_wall_distance(case.mask, case.shape, case.periodic)
    planes = (1, 9)
    steps = 10
    nx, ny, nz = case.shape
    p = O.make_params(19, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force, wall_model=1, collision=1, fd_weight=0.3)
    kw = dict(mask=case.mask, wall_dist=case.wall_dist, rho0=case.rho0, u0=case.u0)
    for cell in (3 + nx * 4, 3 + nx * (4 + ny), 6 + nx * (2 + ny * 4)):
        s = O.Oracle(p, porosity=case.porosity, tangent=True, **kw)
        e = np.zeros(case.ncells)
        e[cell] = 1.0
        s.set_phi_tangent(e)
        s.step(steps)
        _, dJ = s.objective(planes)
        h = 1e-5
        Js = []
        for sgn in (1, -1):
            ph = case.porosity.copy()
            ph[cell] += sgn * h
            t = O.Oracle(p, porosity=ph, **kw)
            t.step(steps)
            Js.append(t.objective(planes)[0])
        fd = (Js[0] - Js[1]) / (2 * h)
        assert cell == 3 + nx * 4 or abs(dJ) > 0.0
        assert abs(dJ - fd) <= 2e-5 * abs(fd) + 1e-13, (cell, dJ, fd)
    # a random direction in the populations
    c, w, _ = O.velocity_set(19)
    f0 = I.random_state(w, case.ncells, seed_offset=61, amp=0.02) * case.mask
    v = np.random.default_rng(62).standard_normal(f0.shape) * case.mask
    s = O.Oracle(p, porosity=case.porosity, tangent=True, **kw)
    s.set_populations(f0, v)
    s.step(steps)
    _, dJ = s.objective(planes)
    h = 1e-6
    Js = []
    for sgn in (1, -1):
        t = O.Oracle(p, porosity=case.porosity, **kw)
        t.set_populations(f0 + sgn * h * v)
        t.step(steps)
        Js.append(t.objective(planes)[0])
    fd = (Js[0] - Js[1]) / (2 * h)
    assert abs(dJ - fd) <= 1e-5 * abs(fd) + 1e-13, (dJ, fd)
