"""Pins of the oracle's open x faces: the regularized local velocity inlet
(Sec. 2.2.2, last sentence) and the fixed local pressure outlet (Sec. 3.2).

- Exactness: on a state that is exactly regularized, f = f^eq(rho, u) +
  w H^(2) : Pi / (2 c_s^4), the inlet (velocity prescribed) recovers the
  whole state from its known populations, whatever the unknown ones hold,
  and must collide exactly like an interior cell that holds the complete
  state. The outlet (density prescribed) recovers the normal velocity exactly
  and holds f^eq(rho_out, u).
- Stability: a slightly perturbed uniform stream at tau0 - 1/2 = 3e-4
  (nearly inviscid, no Smagorinsky) keeps its perturbation at its size. A
  regularized outlet fails this: it grows the perturbation by orders of
  magnitude and diverges within 400 steps.
- Invariance: a uniform stream f^eq(1, U x) between an inlet imposing U and
  an outlet imposing rho = 1 stays exactly uniform.
- Vortex method: with seed points on the inflow plane the inlet imposes the
  mean profile plus the sum of Lamb-Oseen vortices about +x (exactness as
  above, with that velocity).
- The outlet plane is left out of the fringe; the planes before it are
  blended as usual.
- Poiseuille: between two bounce-back walls, the developed laminar flow is
  a parabola that carries the inlet's mass flux. Its pressure gradient
  balances the viscous stress: c_s^2 d rho / dx = rho nu d^2u/dz^2."""
import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def _u_in(z, nz, u_ref, z0=1.0):
    """Inflow profile u_ref ln(1 + z_c/z0) / ln(1 + z_top/z0), z_c = z + 1/2, z_top = nz - 1/2."""
    return u_ref * np.log(1.0 + (z + 0.5) / z0) / np.log(1.0 + (nz - 0.5) / z0)


def _eq2(c, w, rho, u):
    cu = c @ u
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (u @ u))


def _reg_neq(c, w, Pi):
    """w_i H^(2)_i : Pi / (2 c_s^4) = 9/2 w_i (c.Pi.c - c_s^2 tr Pi)."""
    cPc = np.einsum("ia,ab,ib->i", c, Pi, c)
    return 4.5 * w * (cPc - CS2 * np.trace(Pi))


def _rand_sym(rng, scale):
    A = rng.uniform(-scale, scale, (3, 3))
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("collision", [0, 1])
def test_open_faces_exact_on_regularized_states(q, collision):
    nx, ny, nz = 5, 3, 4
    N = nx * ny * nz
    u_ref, rho_out, tau0, cs = 0.05, 1.013, 0.62, 0.12
    c, w, opp = O.velocity_set(q)
    rng = np.random.default_rng(2506 + q + collision)
    f = np.empty((q, N))
    u_out = np.empty((ny, nz))
    eq = (lambda rho, u: _eq2(c, w, rho, u)) if collision == 0 else (lambda rho, u: O.equilibrium3(q, rho, u))
    for z in range(nz):
        for y in range(ny):
            base = nx * (y + ny * z)
            # inlet column x = 0 and its copy at x = 1
            u = np.array([_u_in(z, nz, u_ref), 0.0, 0.0])
            st = eq(rng.uniform(0.98, 1.02), u) + _reg_neq(c, w, _rand_sym(rng, 2e-3))
            f[:, base + 0] = st
            f[:, base + 1] = st
            # outlet column x = nx - 1 (its velocity kept for the check)
            u = np.array([rng.uniform(-0.03, 0.06), 0.0, 0.0])
            u_out[y, z] = u[0]
            f[:, base + nx - 1] = eq(rho_out, u) + _reg_neq(c, w, _rand_sym(rng, 2e-3))
            f[:, base + nx - 2] = eq(1.0, np.array([0.01, 0.0, 0.02])) + _reg_neq(c, w, _rand_sym(rng, 2e-3))
            # the middle column: any state
            f[:, base + 2] = eq(1.0, np.array([0.02, 0.01, -0.01])) + _reg_neq(c, w, _rand_sym(rng, 2e-3))
            # the populations entering through each face are overwritten with noise
            for i in range(q):
                if c[i, 0] > 0:
                    f[i, base + 0] = rng.uniform(0.0, 0.2)
                if c[i, 0] < 0:
                    f[i, base + nx - 1] = rng.uniform(0.0, 0.2)
    p = O.make_params(q, (nx, ny, nz), periodic=(0, 1, 1), tau0=tau0, cs_smag=cs, u_ref=u_ref, z0=1.0,
                      collision=collision, open_x=1, rho_out=rho_out)
    s = O.Oracle(p)
    s.set_populations(f)
    s.step(1)
    fs = s.post_collision()
    for z in range(nz):
        for y in range(ny):
            base = nx * (y + ny * z)
            np.testing.assert_allclose(fs[:, base + 0], fs[:, base + 1], rtol=0, atol=2e-15)
            # the outlet's equilibrium has no third-order part for a velocity along x
            expect = _eq2(c, w, rho_out, np.array([u_out[y, z], 0.0, 0.0]))
            np.testing.assert_allclose(fs[:, base + nx - 1], expect, rtol=0, atol=2e-15)


def _vortex_velocity(yc, zc, vort, sign, intensity, sigma, nz, ny, u_ref):
    """In-plane velocity of the vortex method at the point (yc, zc) from the
    Lamb-Oseen form of each vortex: speed Gamma/(2 pi r) (1 - exp(-r^2/(2
    sigma^2))) about its centre, turning right-handed about the inflow
    direction +x for Gamma > 0 (direction x-hat cross r-hat); Gamma_i from
    k_i = 3/2 (|u_mean(p_i)| I)^2 as the paper defines it."""
    n = len(sign)
    u = np.zeros(3)
    for (py, pz), s in zip(vort, sign):
        um = abs(u_ref * np.log(1.0 + pz) / np.log(1.0 + (nz - 0.5)))
        k = 1.5 * (um * intensity) ** 2
        gam = 4.0 * s * np.sqrt(np.pi / (6 * np.log(3) - 9 * np.log(2)) * k * ny * nz / n)
        ry, rz = yc - py, zc - pz
        r = np.hypot(ry, rz)
        speed = gam / (2 * np.pi * r) * (1.0 - np.exp(-r * r / (2 * sigma * sigma)))
        u += speed * np.array([0.0, -rz / r, ry / r])
    return u


@pytest.mark.parametrize("q,collision", [(19, 0), (27, 1)])
def test_vortex_inlet_exact(q, collision):
    """The inlet with vortex-method seed points imposes u_mean(z) x + the
    Lamb-Oseen sum: on a regularized state with exactly that velocity the
    inlet cell collides like an interior copy of the complete state."""
    nx, ny, nz = 4, 6, 5
    N = nx * ny * nz
    u_ref, tau0, cs, intensity, sigma = 0.05, 0.62, 0.12, 0.3, 1.3
    vort = [(2.3, 1.7), (4.1, 3.2), (0.9, 4.4)]
    sign = [1, -1, 1]
    c, w, _ = O.velocity_set(q)
    rng = np.random.default_rng(99 + q)
    eq = (lambda rho, u: _eq2(c, w, rho, u)) if collision == 0 else (lambda rho, u: O.equilibrium3(q, rho, u))
    f = np.empty((q, N))
    for z in range(nz):
        for y in range(ny):
            base = nx * (y + ny * z)
            u = _vortex_velocity(y + 0.5, z + 0.5, vort, sign, intensity, sigma, nz, ny, u_ref)
            u[0] += _u_in(z, nz, u_ref)
            st = eq(rng.uniform(0.98, 1.02), u) + _reg_neq(c, w, _rand_sym(rng, 2e-3))
            f[:, base + 0] = st
            f[:, base + 1] = st
            for xx in range(2, nx):
                f[:, base + xx] = eq(1.0, np.array([0.03, 0.0, 0.0]))
            for i in range(q):
                if c[i, 0] > 0:
                    f[i, base] = rng.uniform(0.0, 0.2)
    p = O.make_params(q, (nx, ny, nz), periodic=(0, 1, 1), tau0=tau0, cs_smag=cs, u_ref=u_ref, z0=1.0,
                      collision=collision, open_x=1, rho_out=1.0)
    s = O.Oracle(p)
    s.set_vortices(vort, sign, intensity, sigma)
    s.set_populations(f)
    s.step(1)
    fs = s.post_collision()
    assert np.abs(f[:, 1::nx] - f[:, 0::nx]).max() > 1e-3  # the unknown populations really were replaced
    for z in range(nz):
        for y in range(ny):
            base = nx * (y + ny * z)
            np.testing.assert_allclose(fs[:, base], fs[:, base + 1], rtol=0, atol=2e-15)


def test_vortices_validated():
    p = O.make_params(19, (6, 4, 4), periodic=(0, 1, 1), tau0=0.6, u_ref=0.05, z0=1.0, open_x=1)
    s = O.Oracle(p)
    for args in (([(1.0, 1.0)], [1], 0.1, 0.0), ([(1.0, 1.0)], [1], -0.1, 1.0), ([(1.0, -0.5)], [1], 0.1, 1.0),
                 ([(4.5, 1.0)], [1], 0.1, 1.0)):
        with pytest.raises(O.OracleError):
            s.set_vortices(*args)
    closed = O.Oracle(O.make_params(19, (6, 4, 4), tau0=0.6))
    with pytest.raises(O.OracleError):
        closed.set_vortices([(1.0, 1.0)], [1], 0.1, 1.0)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("collision", [0, 1])
def test_open_uniform_stream_is_invariant(q, collision):
    """nz = 1 makes the inflow profile the constant u_ref (z_c = z_top)."""
    nx, ny, nz = 12, 3, 1
    N = nx * ny * nz
    U = 0.04
    u0 = np.zeros((3, N))
    u0[0] = U
    p = O.make_params(q, (nx, ny, nz), periodic=(0, 1, 1), tau0=0.6, cs_smag=0.1, u_ref=U, z0=1.0,
                      collision=collision, open_x=1, rho_out=1.0)
    s = O.Oracle(p, u0=u0)
    f0 = s.populations()
    s.step(40)
    fs = s.post_collision()
    np.testing.assert_allclose(fs, f0, rtol=0, atol=5e-15)  # rounding over 40 steps
    rho, u = s.moments()
    x = np.arange(N) % nx
    inner = (x > 0) & (x < nx - 1)
    np.testing.assert_allclose(rho[inner], 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(u[0, inner], U, rtol=0, atol=1e-14)
    np.testing.assert_allclose(u[1:, inner], 0.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("q", [19, 27])
def test_open_low_viscosity_stream_stable(q):
    nx, ny, nz, U = 16, 8, 1, 0.05
    N = nx * ny * nz
    u0 = np.zeros((3, N))
    u0[0] = U
    u0 += 1e-6 * np.random.default_rng(7).standard_normal((3, N))
    p = O.make_params(q, (nx, ny, nz), periodic=(0, 1, 1), tau0=0.5003, cs_smag=0.0, u_ref=U, z0=1.0,
                      open_x=1, rho_out=1.0)
    s = O.Oracle(p, u0=u0)
    x = np.arange(N) % nx
    inner = (x > 0) & (x < nx - 1)
    for _ in range(8):
        s.step(50)
        rho, u = s.moments()
        dev = max(np.abs(u[0, inner] - U).max(), np.abs(u[1:, inner]).max(), np.abs(rho[inner] - 1.0).max())
        assert dev < 2e-5, dev


def test_open_poiseuille():
    """Laminar flow between bounce-back walls at z_c = 0 and z_c = 8 (halfway),
    fed by the log-law inlet and closed by the pressure outlet."""
    q, nx, ny, nz = 19, 40, 1, 8
    N = nx * ny * nz
    tau0, u_ref = 0.8, 0.02
    nu = (tau0 - 0.5) / 3.0
    p = O.make_params(q, (nx, ny, nz), periodic=(0, 1, 0), tau0=tau0, cs_smag=0.0, u_ref=u_ref, z0=1.0,
                      open_x=1, rho_out=1.0)
    x = np.arange(N) % nx
    z = np.arange(N) // (nx * ny)
    uinit = np.zeros((3, N))
    uinit[0] = _u_in(z, nz, u_ref)
    s = O.Oracle(p, u0=uinit)
    s.step(20000)
    rho0, u0 = s.moments()
    s.step(100)
    rho, u = s.moments()
    # steady up to the slowly damped acoustic mode of the pipe between the two
    # faces (quarter wave, period ~ 280 steps), far below the tolerances below
    assert np.abs(u - u0).max() < 1e-8 and np.abs(rho - rho0).max() < 1e-8
    # steady mass flux: the same through every interior plane, and the
    # inlet's velocity flux times the density there (the inlet imposes u, not
    # rho; the viscous pressure drop raises rho at the inlet by about 3 %)
    flux_in = sum(_u_in(k, nz, u_ref) for k in range(nz))
    fluxes = [np.sum((rho * u[0])[x == i]) for i in range(1, nx - 1)]
    np.testing.assert_allclose(fluxes, fluxes[0], rtol=1e-4)
    assert abs(fluxes[0] / (flux_in * rho[x == 1].mean()) - 1.0) < 1e-2
    # developed profile at x = 30: a parabola symmetric about the channel centre
    ux = u[0][x == 30][np.argsort(z[x == 30])]
    zc = np.arange(nz) + 0.5
    A = np.stack([np.ones(nz), zc, zc * zc], 1)
    coef, *_ = np.linalg.lstsq(A, ux, rcond=None)
    assert np.abs(A @ coef - ux).max() < 1e-4 * ux.max()
    np.testing.assert_allclose(ux, ux[::-1], rtol=1e-6)
    assert abs(-coef[1] / (2 * coef[2]) - nz / 2) < 1e-3
    # pressure gradient balances the viscous stress of the parabola
    rho_mid = np.array([rho[(x == i) & (z == 4)][0] for i in range(20, 36)])
    drho = np.polyfit(np.arange(20, 36), rho_mid, 1)[0]
    assert abs(CS2 * drho / (nu * 2.0 * coef[2] * rho_mid.mean()) - 1.0) < 0.01
    # the density extrapolates to the imposed outlet value at the face, within
    # half a cell's pressure drop (the equilibrium outlet drops the shear
    # stress of the last plane, a first-order error there)
    rho_face = np.polyval(np.polyfit(np.arange(20, 36), rho_mid, 1), nx - 1)
    assert abs(rho_face - 1.0) < 0.5 * abs(drho)


def test_open_outlet_outside_the_fringe():
    """A uniform stream at U with the fringe and inlet set to U2: after one
    step the outlet cells hold f^eq(1, U) (rho_out = 1 and the normal velocity
    of their known populations), untouched by the fringe; the last interior
    plane is blended with lambda = s^2 (3 - 2 s), s = (x - x_f + 1)/L_f."""
    q, nx, ny, nz, Lf = 19, 12, 3, 1, 3
    N = nx * ny * nz
    U, U2 = 0.04, 0.07
    c, w, _ = O.velocity_set(q)
    u0 = np.zeros((3, N))
    u0[0] = U
    p = O.make_params(q, (nx, ny, nz), periodic=(0, 1, 1), tau0=0.6, cs_smag=0.1, u_ref=U2, z0=1.0,
                      fringe_len=Lf, open_x=1, rho_out=1.0)
    s = O.Oracle(p, u0=u0)
    s.step(1)
    fs = s.post_collision()
    x = np.arange(N) % nx
    eqU = _eq2(c, w, 1.0, np.array([U, 0.0, 0.0]))
    eqU2 = _eq2(c, w, 1.0, np.array([U2, 0.0, 0.0]))
    for cell in np.nonzero(x == nx - 1)[0]:
        np.testing.assert_allclose(fs[:, cell], eqU, rtol=0, atol=1e-15)
    sv = (nx - 2 - (nx - Lf) + 1) / Lf
    lam = sv * sv * (3.0 - 2.0 * sv)
    for cell in np.nonzero(x == nx - 2)[0]:
        np.testing.assert_allclose(fs[:, cell], (1 - lam) * eqU + lam * eqU2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kw", [dict(periodic=(1, 1, 1)), dict(force=(1e-6, 0.0, 0.0)),
                                dict(collision=1, fd_weight=0.5), dict(fringe_len=5),
                                dict(rho_out=0.0), dict(open_x=2)])
def test_open_faces_validated(kw):
    args = dict(periodic=(0, 1, 1), tau0=0.6, u_ref=0.05, z0=1.0, open_x=1, rho_out=1.0)
    args.update(kw)
    with pytest.raises(O.OracleError):
        O.Oracle(O.make_params(19, (6, 3, 3), **args))
