"""Pins of the oracle's recursive regularized collision (Sec. 2.2, Eqs. (6),
(8), (9), (11) with sigma = 1) against closed forms and invariants that the
paper's definitions fix, independent of the oracle's own code:

 - the third-order equilibrium has the moments rho, rho u, rho (c_s^2 I + u u)
   and, for every third-order Hermite polynomial the lattice carries, the
   moment rho u_a u_b u_c of the continuous equilibrium (the Hermite
   polynomials are written out here from their definition);
 - the regularized collision keeps mass, momentum and second moments of the
   BGK collision (which other pins fix), and its admissible third moments
   are rho <u u u> plus (1 - 1/tau) times the recursive coefficient
   u_a Pi_bc + u_b Pi_ac + u_c Pi_ab;
 - a perturbation with no mass, momentum or stress (a ghost mode) passes
   through BGK scaled by (1 - 1/tau) and is removed by the regularization;
 - Taylor-Green decay at the analytic rate, and exact conservation in a
   periodic box, with the regularized collision.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2506_21804_amd import inputs as I

CS2 = 1.0 / 3.0


def _h3(c, a, b, g):
    """Third-order Hermite polynomial xi_a xi_b xi_g - c_s^2 (xi_a d_bg + xi_b d_ag + xi_g d_ab)."""
    x = c.astype(np.float64)
    return x[:, a] * x[:, b] * x[:, g] - CS2 * (x[:, a] * (b == g) + x[:, b] * (a == g) + x[:, g] * (a == b))


X, Y, Z = 0, 1, 2


def _admissible(q):
    """(polynomial, list of (sign, component)) pairs whose moments the lattice
    reproduces: single components on D3Q27, sums and differences of the
    aliased pairs on D3Q19."""
    if q == 27:
        comps = [(X, X, Y), (X, X, Z), (X, Y, Y), (Y, Y, Z), (X, Z, Z), (Y, Z, Z), (X, Y, Z)]
        return [[(1.0, t)] for t in comps]
    pairs = [((X, X, Y), (Y, Z, Z)), ((X, Z, Z), (X, Y, Y)), ((Y, Y, Z), (X, X, Z))]
    out = []
    for a, b in pairs:
        out.append([(1.0, a), (1.0, b)])
        out.append([(1.0, a), (-1.0, b)])
    return out


def _poly(c, terms):
    return sum(s * _h3(c, *t) for s, t in terms)


def _contract(terms, A):
    return sum(s * A[t] for s, t in terms)


def _state(q, seed, amp=0.02):
    c, w, _ = O.velocity_set(q)
    rng = np.random.default_rng(seed)
    return c, w, w * (1.0 + amp * rng.standard_normal(q)) + 0.003 * w * rng.standard_normal(q)


@pytest.mark.parametrize("q", [19, 27])
def test_equilibrium3_moments(q):
    c, w, _ = O.velocity_set(q)
    rng = np.random.default_rng(31)
    for _ in range(5):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.08 * rng.standard_normal(3)
        f = O.equilibrium3(q, rho, u)
        assert abs(f.sum() - rho) <= 1e-15
        assert np.abs(c.T @ f - rho * u).max() <= 1e-15
        M2 = np.einsum("ia,ib,i->ab", c, c, f)
        assert np.abs(M2 - rho * (CS2 * np.eye(3) + np.outer(u, u))).max() <= 1e-15
        A = np.einsum("a,b,g->abg", u, u, u) * rho
        for terms in _admissible(q):
            m = float(_poly(c, terms) @ f)
            assert abs(m - _contract(terms, A)) <= 1e-15, (q, terms, m, _contract(terms, A))
        # its second-order part is the BGK equilibrium
        f2 = O.equilibrium(q, rho, u)
        assert abs((f - f2).sum()) <= 1e-15 and np.abs(c.T @ (f - f2)).max() <= 1e-15


def _moments_and_pi(c, f, force):
    rho = f.sum()
    u = (c.T @ f + 0.5 * force) / rho
    Pi = np.einsum("ia,ib,i->ab", c, c, f) - rho * CS2 * np.eye(3) - rho * np.outer(u, u)
    return rho, u, Pi


@pytest.mark.parametrize("q", [19, 27])
def test_rr_keeps_bgk_low_moments_and_sets_third(q):
    tau0, cs, phi = 0.56, 0.12, 0.7
    force = np.array([2e-4, -1e-4, 5e-5])
    for seed in (1, 2, 3):
        c, w, f = _state(q, seed)
        rr = O.collide_bulk_rr(q, tau0, cs, force, phi, f)
        bgk = O.collide_bulk(q, tau0, cs, force, phi, f)
        assert abs(rr.sum() - bgk.sum()) <= 1e-15
        assert np.abs(c.T @ (rr - bgk)).max() <= 1e-15
        M2 = np.einsum("ia,ib,i->ab", c, c, rr - bgk)
        assert np.abs(M2).max() <= 1e-15
        rho, u, Pi = _moments_and_pi(c, f, force)
        tau = O.tau_eff(tau0, cs, float(np.sqrt((Pi ** 2).sum())), rho)
        uh = phi * u
        A0 = rho * np.einsum("a,b,g->abg", uh, uh, uh)
        A1 = np.einsum("a,bg->abg", u, Pi) + np.einsum("b,ag->abg", u, Pi) + np.einsum("g,ab->abg", u, Pi)
        for terms in _admissible(q):
            m = float(_poly(c, terms) @ rr)
            expect = _contract(terms, A0) + (1.0 - 1.0 / tau) * _contract(terms, A1)
            assert abs(m - expect) <= 1e-15, (q, terms, m, expect)


@pytest.mark.parametrize("q", [19, 27])
def test_rr_removes_ghost_modes(q):
    tau0, cs, phi = 0.6, 0.1, 1.0
    force = np.zeros(3)
    c, w, f = _state(q, 7)
    # constraints: no mass, momentum or second moment
    C = np.vstack([np.ones(q), c.T.astype(float)] + [c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)])
    _, s, vt = np.linalg.svd(C)
    null = vt[np.sum(s > 1e-12):]
    g = null.T @ np.random.default_rng(8).standard_normal(null.shape[0])
    g *= 1e-3 / np.abs(g).max()
    assert np.abs(C @ g).max() < 1e-15
    rr0 = O.collide_bulk_rr(q, tau0, cs, force, phi, f)
    rr1 = O.collide_bulk_rr(q, tau0, cs, force, phi, f + g)
    assert np.abs(rr1 - rr0).max() <= 1e-16
    bgk0 = O.collide_bulk(q, tau0, cs, force, phi, f)
    bgk1 = O.collide_bulk(q, tau0, cs, force, phi, f + g)
    rho, u, Pi = _moments_and_pi(c, f, force)
    tau = O.tau_eff(tau0, cs, float(np.sqrt((Pi ** 2).sum())), rho)
    assert np.abs((bgk1 - bgk0) - (1.0 - 1.0 / tau) * g).max() <= 1e-16


def _tgv_amplitude(u, n, k):
    X_ = np.arange(n ** 3) % n
    Y_ = (np.arange(n ** 3) // n) % n
    prof = -np.cos(k * X_) * np.sin(k * Y_)
    return float((u[0] * prof).sum() / (prof * prof).sum())


@pytest.mark.parametrize("q", [19, 27])
def test_rr_taylor_green_decay(q):
    """2D Taylor-Green in a periodic 32^3 box, C_S = 0, tau = 0.6: the amplitude
    decays as exp(-2 nu k^2 t) with the regularized collision too."""
    n, u0 = 32, 0.05
    case = I.taylor_green(n, u0=u0, q=q, cs_smag=0.0, two_d=True)
    p = O.make_params(q, case.shape, tau0=0.6, cs_smag=0.0, collision=1)
    s = O.Oracle(p, rho0=case.rho0, u0=case.u0)
    s.step(100)
    _, u = s.moments()
    ratio = _tgv_amplitude(u, n, case.extra["k"]) / u0
    expect = math.exp(-2.0 * (0.1 / 3.0) * case.extra["k"] ** 2 * 100)
    assert abs(ratio / expect - 1.0) < 0.01, (ratio, expect)


@pytest.mark.parametrize("q", [19, 27])
def test_rr_conservation_periodic(q):
    shape = (12, 10, 8)
    N = int(np.prod(shape))
    c, w, _ = O.velocity_set(q)
    f0 = I.random_state(w, N, seed_offset=41, amp=0.03)
    p = O.make_params(q, shape, tau0=0.55, cs_smag=0.15, collision=1)
    s = O.Oracle(p)
    s.set_populations(f0)
    d0 = s.diagnostics()
    s.step(20)
    d1 = s.diagnostics()
    assert abs(d1[0] - d0[0]) <= 1e-12 * d0[0]
    assert np.abs(np.array(d1[1:]) - np.array(d0[1:])).max() <= 1e-13 * d0[0]


def test_collision_parameter_checked():
    p = O.make_params(19, (4, 4, 4), tau0=0.6, collision=2)
    with pytest.raises(O.OracleError):
        O.Oracle(p)
