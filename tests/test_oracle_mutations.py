"""Mutation check of the oracle's pins: each case plants one plausible
mistake in a copy of the oracle's source (a dropped or changed term, a wrong
sign, a swapped index or direction), builds that copy on the CPU, and runs
the pin tests against it.  Every mutant must fail at least one pin; a mutant
that passes them all would mean the pins leave that part of the oracle
unchecked."""
import os
import subprocess
import tempfile

import pytest

import oracle as O
import test_oracle_pins as pins
import test_oracle_pins_rr as pins_rr
import test_oracle_pins_hybrid as pins_hy
import test_oracle_pins_open as pins_open
import test_oracle_pins_wall as pins_wall
import test_oracle_pins_slip as pins_slip

SRC = os.path.join(os.path.dirname(O.__file__), "lbm_oracle.cpp")

# (name, exact text in the oracle, replacement)
MUTATIONS = [
    ("half-force velocity shift dropped", "u[a] = (j[a] + 0.5 * p.force[a]) / rho;\n    T feq[27];",
     "u[a] = (j[a] + 0.0 * p.force[a]) / rho;\n    T feq[27];"),
    ("Guo source prefactor sign", "                (1.0 - 0.5 / tau) * guo_term(vs, i, u, p.force)",
     "                (1.0 + 0.5 / tau) * guo_term(vs, i, u, p.force)"),
    ("equilibrium second-order coefficient", "4.5 * cv * cv", "3.0 * cv * cv"),
    ("Smagorinsky coefficient", "18.0 * std::sqrt(2.0)", "9.0 * std::sqrt(2.0)"),
    ("stress tensor index", "double(vs.c[i][a] * vs.c[i][b]) * fneq;", "double(vs.c[i][a] * vs.c[i][a]) * fneq;"),
    ("streaming direction in x", "neighbor_xyz(x, y, z, -vs.c[i][0], -vs.c[i][1], -vs.c[i][2])",
     "neighbor_xyz(x, y, z, vs.c[i][0], -vs.c[i][1], -vs.c[i][2])"),
    ("bounce-back into the same direction", "fs[(size_t)vs.opp[i] * N + c]", "fs[(size_t)i * N + c]"),
    ("porosity ignored", "uh[a] = phi[c] * u[a];", "uh[a] = u[a];"),
    ("Spalding cubic term", "0.5 * k * k - k * k * k / 6.0", "0.5 * k * k - k * k * k / 3.0"),
    ("wall non-equilibrium sign", "T ffd = -3.0 * vs.w[i]", "T ffd = 3.0 * vs.w[i]"),
    ("stress-consistent strain", "4.0 * cs2 * utau * utau", "2.0 * cs2 * utau * utau"),
    ("fringe ramp", "s * s * (3.0 - 2.0 * s)", "s * (3.0 - 2.0 * s)"),
    ("D3Q27 corner weight", "1.0 / 216.0", "1.0 / 108.0"),
    ("wall normal velocity kept", "uw[a] = wutan[k] * t[a] + un * n[a];", "uw[a] = wutan[k] * t[a];"),
    ("D3Q19 third-order pair sign", "add({X, X, Y}, {Y, Z, Z}, -1.0);", "add({X, X, Y}, {Y, Z, Z}, 1.0);"),
    ("continuous instead of lattice norm", "B.norm[k] += vs.w[i] * v * v;", "B.norm[k] += vs.w[i] * v * v * 1.5;"),
    ("recursion not symmetrised",
     "A[a][b][g] = u[a] * Pi[b][g] + u[b] * Pi[a][g] + u[g] * Pi[a][b];", "A[a][b][g] = 3.0 * u[a] * Pi[b][g];"),
    ("regularization skipped", "fo[i] = feqh[i] + (1.0 - 1.0 / tau) * f1 +",
     "fo[i] = feqh[i] + (1.0 - 1.0 / tau) * (fi[i] - feq[i]) +"),
    ("third-order equilibrium term dropped", "for (int i = 0; i < vs.q; ++i) feq[i] += t[i];",
     "for (int i = 0; i < vs.q; ++i) feq[i] += 0.0 * t[i];"),
    ("finite-difference stress sign", "Ph[a][b] = sig * Pi[a][b] - p.fd_weight * (2.0 / 3.0)",
     "Ph[a][b] = sig * Pi[a][b] + p.fd_weight * (2.0 / 3.0)"),
    ("one-sided difference reversed", "else if (fp) D[a][b] = uf[(size_t)b * N + xp] - uc;",
     "else if (fp) D[a][b] = uc - uf[(size_t)b * N + xp];"),
    ("wall-normal shear of the FD strain kept",
     "S[a][b] = S[a][b] - (sv[a] * n[b] + n[a] * sv[b]) + 0.5 * G * (t[a] * n[b] + n[a] * t[b]);",
     "S[a][b] = S[a][b] + 0.5 * G * (t[a] * n[b] + n[a] * t[b]);"),
    ("wall-law shear in the hybrid wall strain", "+ 0.5 * G * (t[a] * n[b] + n[a] * t[b]);\n    } else {",
     "+ 0.25 * G * (t[a] * n[b] + n[a] * t[b]);\n    } else {"),
    ("hybrid third-order factor dropped", "for (int i = 0; i < vs.q; ++i) t3[i] = sig * t3[i];",
     "for (int i = 0; i < vs.q; ++i) t3[i] = t3[i];"),
    ("inlet density with the wrong sign of u.n", "rho = (s_par + 2.0 * s_out) / (1.0 + un);",
     "rho = (s_par + 2.0 * s_out) / (1.0 - un);"),
    ("outlet leaving populations counted once", "const T un = (s_par + 2.0 * s_out) / rho - 1.0;",
     "const T un = (s_par + s_out) / rho - 1.0;"),
    ("unknown non-equilibrium taken from the unknown population",
     "fneq[i] = unknown ? fi[vs.opp[i]] - feq[vs.opp[i]] : fi[i] - feq[i];", "fneq[i] = fi[i] - feq[i];"),
    ("unknown populations on the wrong side", "const bool unknown = vs.c[i][0] * nx_out < 0;",
     "const bool unknown = vs.c[i][0] * nx_out > 0;"),
    ("regularized trace term dropped", "fr[i] = feq[i] + 4.5 * vs.w[i] * (cPc - trPi / 3.0);",
     "fr[i] = feq[i] + 4.5 * vs.w[i] * cPc;"),
    ("inflow profile at the cell floor", "u[0] = T(u_in(z + 0.5));", "u[0] = T(u_in(z));"),
    ("inlet plane left as bulk cells", "if (p.open_x && kind[c] == K_BULK && x == 0) kind[c] = K_INLET;", ""),
    ("fringe over the outlet plane", "x >= fstart && kind[c] != K_OUTLET)", "x >= fstart)"),
    ("vortex core growing instead of decaying", "(1.0 - std::exp(-r2 / (2.0 * vsig * vsig)))",
     "(1.0 - std::exp(r2 / (2.0 * vsig * vsig)))"),
    ("vortex turning the wrong way", "u[1] += f * dz;", "u[1] -= f * dz;"),
    ("vortex circulation constant", "(6.0 * std::log(3.0) - 9.0 * std::log(2.0))",
     "(6.0 * std::log(3.0) + 9.0 * std::log(2.0))"),
    ("regularized outlet", "if (!inlet) {\n      /* the outlet holds", "if (false) {\n      /* the outlet holds"),
    ("u_tau solved at the first cell's distance", "solve_utau(Uv, wyr[k], nu, p.kappa, p.E, &utv, nullptr);",
     "solve_utau(Uv, wyb[k], nu, p.kappa, p.E, &utv, nullptr);"),
    ("second solve of the law dropped", "if (r == wcell[k]) {", "if (true) {"),
    ("speed of u instead of its tangential part",
     "T U = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);",
     "T U = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);"),
    ("first-cell y+ from the reference distance", "double yplus_b = wyb[k] * utv / nu;",
     "double yplus_b = wyr[k] * utv / nu;"),
    ("objective pressure weight", "T Jv = (1.0 / 3.0) * (s0 / double(n0) - s1 / double(n1))",
     "T Jv = 0.5 * (s0 / double(n0) - s1 / double(n1))"),
    ("objective planes swapped", "(s0 / double(n0) - s1 / double(n1)) + ke", "(s1 / double(n1) - s0 / double(n0)) + ke"),
    ("objective kinetic energy without the half", "ke += 0.5 * (m[0] * m[0]", "ke += (m[0] * m[0]"),
    ("objective momentum without the half force", "for (int a = 0; a < 3; ++a) m[a] = j[a] + 0.5 * p.force[a];",
     "for (int a = 0; a < 3; ++a) m[a] = j[a];"),
    ("full-slip faces bounce back", "            if (m) {\n              int d[3], cj[3];",
     "            if (false) {\n              int d[3], cj[3];"),
    ("reflected population not flipped", "cj[a] = crossed ? -vs.c[i][a] : vs.c[i][a];", "cj[a] = vs.c[i][a];"),
    ("reflected source without the tangential shift", "d[a] = crossed ? 0 : -vs.c[i][a];", "d[a] = 0;"),
    ("reflection flips every component", "cj[a] = crossed ? -vs.c[i][a] : vs.c[i][a];", "cj[a] = -vs.c[i][a];"),
    ("implicit derivative of u_tau with the wrong sign", "T utau = root_of(utv, U, gpr / utv,",
     "T utau = root_of(utv, U, -gpr / utv,"),
    ("implicit derivative of u+ ignoring u_tau", "uplus_b = root_of(upv, utau, -wyb[k] / nu,",
     "uplus_b = root_of(upv, utau, 0.0 * wyb[k] / nu,"),
    ("slip links counted as wall links",
     "if (!is_fluid(nb) && !slip_cross(bx, by, bz, vs.c[i][0], vs.c[i][1], vs.c[i][2])) {",
     "if (!is_fluid(nb)) {"),
    ("per-cell C_S ignored in the bulk", "T tau = tau_effective(p.tau0, cs_at(c), sqrt(pi2), rho);",
     "T tau = tau_effective(p.tau0, T(p.cs_smag), sqrt(pi2), rho);"),
    ("per-cell C_S ignored in the wall records", "const T csb = cs_at(wcell[k]);", "const T csb = T(p.cs_smag);"),
]

PIN_TESTS = [
    (pins.test_velocity_set_isotropy_exact, [(27, {0: pins.Fraction(8, 27), 1: pins.Fraction(2, 27),
                                                  2: pins.Fraction(1, 54), 3: pins.Fraction(1, 216)})]),
    (pins.test_equilibrium_moments, [(19,), (27,)]),
    (pins.test_smagorinsky_relation, [(19,)]),
    (pins.test_porosity_and_force_momentum, [(19,)]),
    (pins.test_conservation_periodic, [(19,)]),
    (pins.test_taylor_green_decay, [()]),
    (pins.test_advected_shear_wave, [()]),
    (pins.test_poiseuille_magic_tau, [()]),
    (pins.test_spalding_closed_form_values, [()]),
    (pins.test_wall_reconstruction_stress, [()]),
    (pins.test_wall_model_channel_records, [(27,)]),
    (pins.test_fringe_and_lid, [()]),
    (pins_rr.test_equilibrium3_moments, [(19,), (27,)]),
    (pins_rr.test_rr_keeps_bgk_low_moments_and_sets_third, [(19,), (27,)]),
    (pins_rr.test_rr_removes_ghost_modes, [(19,)]),
    (pins_hy.test_hybrid_fd_stress_quadratic_shear, [(19,)]),
    (pins_hy.test_hybrid_blend_and_third_moments, [(27,)]),
    (pins_hy.test_hybrid_wall_shear_replaced, [(1.0,)]),
    (pins_hy.test_hybrid_wall_keeps_normal_strain, [()]),
    (pins_open.test_open_faces_exact_on_regularized_states, [(19, 0), (27, 1)]),
    (pins_open.test_open_uniform_stream_is_invariant, [(19, 0)]),
    (pins_open.test_open_outlet_outside_the_fringe, [()]),
    (pins_open.test_open_low_viscosity_stream_stable, [(19,)]),
    (pins_open.test_vortex_inlet_exact, [(19, 0)]),
    (pins_open.test_open_poiseuille, [()]),
    (pins_wall.test_wall_law_at_first_cell, [("channel",), ("urban",)]),
    (pins_wall.test_objective_density_step_and_uniform_stream, [()]),
    (pins_slip.test_slip_faces_mirror_periodic_double, [(19, 0)]),
    (pins_slip.test_slip_top_over_bounce_back_ground_with_buildings, [()]),
    (pins_slip.test_slip_faces_are_not_wall_modeled, [()]),
    (pins_wall.test_tangent_through_wall_model_matches_central_differences, [()]),
    (pins_wall.test_smagorinsky_field_relation_per_cell, [(19,)]),
    (pins_wall.test_smagorinsky_field_in_wall_records, [()]),
    (pins_wall.test_tangent_in_smagorinsky_field, [()]),
]


def _caught(lib_path):
    """Name of the first pin that fails against the library, or None."""
    O.use_library(lib_path)
    try:
        for fn, arglists in PIN_TESTS:
            for args in arglists:
                try:
                    fn(*args)
                except (AssertionError, O.OracleError):
                    return fn.__name__
    finally:
        O.use_library(None)
    return None


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    mut = tmp_path / "mutant.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    cmd = [c if c != O._SRC else str(mut) for c in O.BUILD_CMD]
    cmd[cmd.index(O._LIB)] = str(lib)
    subprocess.run(cmd, check=True)
    failed = _caught(str(lib))
    assert failed, f"mutant '{name}' passed every pin"
