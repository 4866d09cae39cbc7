"""FP64 CPU oracle of the wall-modeled LBM-LES step (arXiv 2506.21804).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports,
links or executes anything here, and nothing here imports the product.

The arithmetic lives in ``lbm_oracle.cpp`` (plain C++17, double precision,
two-lattice pull scheme, built with ``-O3 -ffp-contract=off``, no fast-math).  This module
only builds it, loads it with ctypes and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

BUILD_CMD = ["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             _SRC, "-o", _LIB]

OK, EINVAL, ENONFINITE, ENEWTON = 0, -1, -3, -4


def build() -> str:
    """Compile the oracle library (always recompiles)."""
    subprocess.run(BUILD_CMD, check=True)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("q", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("periodic", C.c_int * 3),
        ("tau0", C.c_double), ("cs_smag", C.c_double),
        ("force", C.c_double * 3),
        ("wall_model", C.c_int),
        ("kappa", C.c_double), ("E", C.c_double),
        ("fringe_len", C.c_int),
        ("u_ref", C.c_double), ("z0", C.c_double),
        ("lid", C.c_int),
        ("collision", C.c_int),
        ("fd_weight", C.c_double),
        ("open_x", C.c_int),
        ("rho_out", C.c_double),
        ("slip", C.c_int),
    ]


_lib = None
_lib_override = None  # path of an alternative build (mutation tests)


def use_library(path):
    """Points the loader at another build of the oracle (None = the normal
    one); used by the mutation tests to load deliberately broken copies."""
    global _lib, _lib_override
    _lib = None
    _lib_override = path


def lib():
    global _lib
    if _lib is None:
        if _lib_override is None and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_lib_override or _LIB)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(Params), vp, vp, vp, vp, vp, C.c_int]
        L.orc_create_error.restype = C.c_char_p
        L.orc_last_error.restype = C.c_char_p
        L.orc_last_error.argtypes = [vp]
        L.orc_free.argtypes = [vp]
        L.orc_step.argtypes = [vp, C.c_int]
        for name in ("orc_moments", "orc_get_populations", "orc_set_populations"):
            getattr(L, name).argtypes = [vp, vp, vp]
        L.orc_diagnostics.argtypes = [vp, vp]
        L.orc_get_post_collision.argtypes = [vp, vp]
        L.orc_collide_wall.argtypes = [C.c_int, C.c_double, C.c_double, vp, vp, vp, vp, C.c_double,
                                       C.c_double, C.c_double, vp]
        L.orc_set_phi_tangent.argtypes = [vp, vp]
        L.orc_set_smagorinsky.argtypes = [vp, vp, vp]
        L.orc_objective.argtypes = [vp, vp, vp, vp]
        L.orc_num_wall.restype = C.c_long
        L.orc_num_wall.argtypes = [vp]
        L.orc_wall_info.argtypes = [vp] + [vp] * 6
        L.orc_wall_velocity.argtypes = [vp, vp, vp]
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_set_vortices.argtypes = [vp, C.c_int, vp, vp, C.c_double, C.c_double]
        L.orc_velocity_set.argtypes = [C.c_int, vp, vp, vp]
        L.orc_equilibrium.argtypes = [C.c_int, C.c_double, vp, vp]
        L.orc_tau_eff.restype = C.c_double
        L.orc_tau_eff.argtypes = [C.c_double] * 4
        L.orc_collide_bulk.argtypes = [C.c_int, C.c_double, C.c_double, vp, C.c_double, vp, vp]
        L.orc_collide_bulk2.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, vp, C.c_double, vp, vp]
        L.orc_equilibrium3.argtypes = [C.c_int, C.c_double, vp, vp]
        L.orc_spalding_yplus.restype = C.c_double
        L.orc_spalding_yplus.argtypes = [C.c_double] * 3
        L.orc_spalding_uplus.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_solve_utau.argtypes = [C.c_double] * 5 + [dp, ip]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(q, shape, periodic=(1, 1, 1), tau0=0.6, cs_smag=0.0, force=(0.0, 0.0, 0.0),
                wall_model=0, kappa=0.41, E=9.0, fringe_len=0, u_ref=0.0, z0=1.0, lid=0,
                collision=0, fd_weight=0.0, open_x=0, rho_out=1.0, slip=0) -> Params:
    p = Params()
    p.q = q
    p.nx, p.ny, p.nz = shape
    p.periodic = (C.c_int * 3)(*periodic)
    p.tau0, p.cs_smag = tau0, cs_smag
    p.force = (C.c_double * 3)(*force)
    p.wall_model, p.kappa, p.E = wall_model, kappa, E
    p.fringe_len, p.u_ref, p.z0, p.lid = fringe_len, u_ref, z0, lid
    p.collision = collision
    p.fd_weight = fd_weight
    p.open_x, p.rho_out = open_x, rho_out
    p.slip = slip
    return p


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """One oracle simulation.  Arrays are numpy, cell index x + nx*(y + ny*z);
    populations and velocities are [q][N] / [3][N]."""

    def __init__(self, params: Params, mask=None, wall_dist=None, porosity=None, rho0=None,
                 u0=None, tangent=False):
        L = lib()
        self.p = params
        self.q = params.q
        self.N = params.nx * params.ny * params.nz
        keep = []

        def arr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a, dtype=dt).reshape(-1))
            keep.append(a)
            return a

        m, wd, ph = arr(mask, np.uint8), arr(wall_dist, np.float64), arr(porosity, np.float64)
        r0, v0 = arr(rho0, np.float64), arr(u0, np.float64)
        self.h = L.orc_create(C.byref(params), _ptr(m), _ptr(wd), _ptr(ph), _ptr(r0), _ptr(v0),
                              1 if tangent else 0)
        if not self.h:
            raise OracleError(EINVAL, L.orc_create_error().decode())
        # held here: at interpreter exit the module's globals may already be gone
        self._free = L.orc_free

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._free(h)
            self.h = None

    def _check(self, rc):
        if rc != OK:
            raise OracleError(rc, lib().orc_last_error(self.h).decode())

    def step(self, n=1):
        self._check(lib().orc_step(self.h, n))

    def step_rc(self, n=1) -> int:
        return lib().orc_step(self.h, n)

    def moments(self):
        rho = np.empty(self.N)
        u = np.empty((3, self.N))
        self._check(lib().orc_moments(self.h, _ptr(rho), _ptr(u)))
        return rho, u

    def diagnostics(self):
        out = np.empty(4)
        self._check(lib().orc_diagnostics(self.h, _ptr(out)))
        return out

    def populations(self, with_tangent=False):
        f = np.empty((self.q, self.N))
        df = np.empty((self.q, self.N)) if with_tangent else None
        self._check(lib().orc_get_populations(self.h, _ptr(f), _ptr(df)))
        return (f, df) if with_tangent else f

    def post_collision(self):
        f = np.empty((self.q, self.N))
        self._check(lib().orc_get_post_collision(self.h, _ptr(f)))
        return f

    def set_populations(self, f, df=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        df = None if df is None else np.ascontiguousarray(df, dtype=np.float64)
        self._check(lib().orc_set_populations(self.h, _ptr(f), _ptr(df)))

    def set_vortices(self, yz, sign, intensity, sigma):
        """Vortex-method seed points (y, z) on the inflow plane, cell-centre
        coordinates (cell j spans [j, j + 1)), signs +-1, intensity I, size sigma."""
        yz = np.ascontiguousarray(np.asarray(yz, dtype=np.float64).reshape(-1, 2))
        sign = np.ascontiguousarray(np.asarray(sign, dtype=np.int32).reshape(-1))
        self._check(lib().orc_set_vortices(self.h, len(sign), _ptr(yz), _ptr(sign), intensity, sigma))

    def set_smagorinsky(self, cs, dcs=None):
        """Per-cell Smagorinsky constants [N] (None: the scalar of the
        parameters everywhere); dcs: their tangent direction (tangent mode)."""
        a = None if cs is None else np.ascontiguousarray(cs, dtype=np.float64)
        d = None if dcs is None else np.ascontiguousarray(dcs, dtype=np.float64)
        self._keep_cs = (a, d)
        self._check(lib().orc_set_smagorinsky(self.h, _ptr(a), _ptr(d)))

    def set_phi_tangent(self, dphi):
        dphi = np.ascontiguousarray(dphi, dtype=np.float64).reshape(-1)
        self._check(lib().orc_set_phi_tangent(self.h, _ptr(dphi)))

    def objective(self, planes):
        pl = np.asarray(planes, dtype=np.int32)
        J = C.c_double()
        dJ = C.c_double()
        self._check(lib().orc_objective(self.h, _ptr(pl), C.byref(J), C.byref(dJ)))
        return J.value, dJ.value

    def wall_info(self):
        nw = lib().orc_num_wall(self.h)
        cells = np.empty(nw, np.int64)
        refs = np.empty(nw, np.int64)
        normal = np.empty((nw, 3))
        utau, G, tau = np.empty(nw), np.empty(nw), np.empty(nw)
        self._check(lib().orc_wall_info(self.h, _ptr(cells), _ptr(refs), _ptr(normal), _ptr(utau),
                                        _ptr(G), _ptr(tau)))
        tangent, utan = np.empty((nw, 3)), np.empty(nw)
        self._check(lib().orc_wall_velocity(self.h, _ptr(tangent), _ptr(utan)))
        return dict(cells=cells, refs=refs, normal=normal, utau=utau, G=G, tau=tau, tangent=tangent, utan=utan)


# ---- pure helpers -----------------------------------------------------------

def velocity_set(q):
    c = np.empty((q, 3), np.int32)
    w = np.empty(q)
    opp = np.empty(q, np.int32)
    rc = lib().orc_velocity_set(q, _ptr(c), _ptr(w), _ptr(opp))
    if rc != OK:
        raise OracleError(rc, "bad q")
    return c, w, opp


def equilibrium(q, rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(q)
    lib().orc_equilibrium(q, float(rho), _ptr(u), _ptr(out))
    return out


def equilibrium3(q, rho, u):
    """Third-order equilibrium of the recursive regularized collision."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(q)
    lib().orc_equilibrium3(q, float(rho), _ptr(u), _ptr(out))
    return out


def tau_eff(tau0, cs, pinorm, rho):
    return lib().orc_tau_eff(tau0, cs, pinorm, rho)


def collide_bulk(q, tau0, cs, force, phi, fin):
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    force = np.ascontiguousarray(force, dtype=np.float64)
    out = np.empty(q)
    lib().orc_collide_bulk(q, tau0, cs, _ptr(force), float(phi), _ptr(fin), _ptr(out))
    return out


def collide_bulk_rr(q, tau0, cs, force, phi, fin):
    """Bulk collision of the recursive regularized model (third order)."""
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    force = np.ascontiguousarray(force, dtype=np.float64)
    out = np.empty(q)
    lib().orc_collide_bulk2(q, 1, tau0, cs, _ptr(force), float(phi), _ptr(fin), _ptr(out))
    return out


def collide_wall(q, tau0, cs, force, fin, normal, tangent, utan, G, tau):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (force, fin, normal, tangent)]
    out = np.empty(q)
    lib().orc_collide_wall(q, tau0, cs, _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(a[3]), float(utan),
                           float(G), float(tau), _ptr(out))
    return out


def spalding_yplus(uplus, kappa=0.41, E=9.0):
    return lib().orc_spalding_yplus(uplus, kappa, E)


def spalding_uplus(yplus, kappa=0.41, E=9.0):
    out = C.c_double()
    rc = lib().orc_spalding_uplus(yplus, kappa, E, C.byref(out))
    if rc != OK:
        raise OracleError(rc, "u+ Newton failed")
    return out.value


def solve_utau(U, y, nu, kappa=0.41, E=9.0):
    out = C.c_double()
    it = C.c_int()
    rc = lib().orc_solve_utau(U, y, nu, kappa, E, C.byref(out), C.byref(it))
    if rc != OK:
        raise OracleError(rc, "u_tau Newton failed")
    return out.value, it.value


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of later oracle steps (the host's default: all cores)."""
    lib().orc_set_num_threads(int(n))
