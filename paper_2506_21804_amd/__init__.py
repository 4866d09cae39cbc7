"""Python binding of the MI355X wall-modeled LBM-LES library (``liblbm_hip.so``).

The functions here carry the C-ABI names of ``include/lbm.h`` and only
marshal arguments: torch tensors supply device memory and the HIP stream,
numpy arrays the host inputs.  Every step of the computation runs in the HIP
kernels of the library.  The library must have been built
(``python -m paper_2506_21804_amd.build``); loading fails loudly otherwise.
There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "load", "LbmError", "Params", "lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_moments",
    "lbm_diagnostics", "lbm_diagnostics_noalloc", "lbm_sync", "lbm_steps_done", "lbm_shape", "lbm_get_populations", "lbm_set_populations",
    "lbm_state_bytes", "lbm_save_state", "lbm_load_state", "lbm_objective", "lbm_adjoint_bytes",
    "lbm_adjoint_seed", "lbm_adjoint_step", "lbm_adjoint_to_natural", "lbm_adjoint_from_natural",
    "lbm_gradient", "lbm_revolve_cost", "lbm_wall_count", "lbm_wall_records", "lbm_profile", "lbm_profile_read",
    "lbm_set_inflow_vortices", "lbm_gradient_mean", "lbm_stream_probe", "lbm_slot_map", "lbm_last_error",
    "lbm_set_smagorinsky", "lbm_adjoint_step_cs", "lbm_gradient_cs",
    "lbm_workspace_alloc", "lbm_adjoint_alloc", "lbm_spread_free", "SpreadBuffer",
    "lbm_free", "params_for", "Lattice", "D3Q19", "D3Q27", "F64", "F32DEV", "F16DEV",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm_hip.so")

OK, EINVAL, EHIP, ENONFINITE, ENEWTON, ESIZE = 0, -1, -2, -3, -4, -5
D3Q19, D3Q27 = 19, 27
F64, F32DEV, F16DEV = 0, 1, 2
STORAGE_NAMES = {"f64": F64, "f32": F32DEV, "f16": F16DEV}
BGK, RR3 = 0, 1
COLLISION_NAMES = {"bgk": BGK, "rr3": RR3}


class Params(C.Structure):
    """Mirror of ``lbm_params``."""
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("periodic", C.c_int * 3),
        ("storage", C.c_int),
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
        ("cs_field", C.c_int),
        ("stream", C.c_void_p),
    ]


MAX_VORTICES = 4096  # LBM_MAX_VORTICES


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Loads the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_21804_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, sz, i, d, ll = C.c_void_p, C.c_size_t, C.c_int, C.c_double, C.c_longlong
    sig = {
        "lbm_workspace_bytes": (sz, [C.POINTER(Params), vp, i]),
        "lbm_init": (i, [C.POINTER(vp), C.POINTER(Params), vp, vp, vp, vp, vp, vp, sz]),
        "lbm_step": (i, [vp, i]),
        "lbm_moments": (i, [vp, vp, vp]),
        "lbm_diagnostics": (i, [vp, vp]),
        "lbm_diagnostics_noalloc": (i, [vp, vp]),
        "lbm_sync": (i, [vp]),
        "lbm_steps_done": (ll, [vp]),
        "lbm_shape": (i, [vp, vp]),
        "lbm_get_populations": (i, [vp, vp]),
        "lbm_set_populations": (i, [vp, vp]),
        "lbm_state_bytes": (sz, [vp]),
        "lbm_save_state": (i, [vp, vp]),
        "lbm_load_state": (i, [vp, vp]),
        "lbm_objective": (i, [vp, vp, C.POINTER(d)]),
        "lbm_adjoint_bytes": (sz, [vp]),
        "lbm_adjoint_seed": (i, [vp, vp, vp]),
        "lbm_adjoint_step": (i, [vp, vp, vp]),
        "lbm_adjoint_to_natural": (i, [vp, vp, vp]),
        "lbm_adjoint_from_natural": (i, [vp, vp, vp]),
        "lbm_gradient": (i, [vp, i, vp, vp, i, vp, vp, C.POINTER(d), C.POINTER(ll)]),
        "lbm_revolve_cost": (ll, [i, i]),
        "lbm_wall_count": (i, [vp]),
        "lbm_wall_records": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "lbm_profile": (i, [vp, i]),
        "lbm_profile_read": (i, [vp, vp, vp]),
        "lbm_set_inflow_vortices": (i, [vp, i, vp, vp, d, d]),
        "lbm_gradient_mean": (i, [vp, i, vp, vp, i, vp, vp, C.POINTER(d), C.POINTER(ll)]),
        "lbm_stream_probe": (i, [vp, i, C.POINTER(d)]),
        "lbm_slot_map": (i, [C.POINTER(Params), vp, i, vp, vp]),
        "lbm_set_smagorinsky": (i, [vp, vp]),
        "lbm_adjoint_step_cs": (i, [vp, vp, vp, vp]),
        "lbm_gradient_cs": (i, [vp, i, vp, vp, i, vp, vp, vp, i, C.POINTER(d), C.POINTER(ll)]),
        "lbm_workspace_alloc": (i, [C.POINTER(Params), vp, i, C.POINTER(vp), C.POINTER(sz)]),
        "lbm_adjoint_alloc": (i, [vp, C.POINTER(vp), C.POINTER(sz)]),
        "lbm_spread_free": (i, [vp]),
        "lbm_last_error": (C.c_char_p, [vp]),
        "lbm_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return ["lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_moments", "lbm_diagnostics",
            "lbm_diagnostics_noalloc", "lbm_sync",
            "lbm_steps_done", "lbm_shape", "lbm_get_populations", "lbm_set_populations", "lbm_state_bytes",
            "lbm_save_state", "lbm_load_state", "lbm_objective", "lbm_adjoint_bytes", "lbm_adjoint_seed",
            "lbm_adjoint_step", "lbm_adjoint_to_natural", "lbm_adjoint_from_natural", "lbm_gradient",
            "lbm_revolve_cost", "lbm_wall_count", "lbm_wall_records", "lbm_profile", "lbm_profile_read",
            "lbm_set_inflow_vortices", "lbm_gradient_mean", "lbm_stream_probe", "lbm_slot_map",
            "lbm_set_smagorinsky", "lbm_adjoint_step_cs", "lbm_gradient_cs", "lbm_workspace_alloc",
            "lbm_adjoint_alloc", "lbm_spread_free", "lbm_last_error", "lbm_free"]


def _dptr(t):
    """Device pointer of a torch tensor (or None); refuses anything that is
    not a contiguous tensor in GPU memory."""
    if t is None:
        return None
    if not hasattr(t, "data_ptr") or not getattr(t, "is_cuda", False):
        raise ValueError("device buffer expected: pass a torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("device buffer must be contiguous")
    return C.c_void_p(t.data_ptr())


def _dbuf(t, nbytes, what, dtype=None):
    """Checks a device buffer's placement, size (bytes) and dtype."""
    p = _dptr(t)
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what}: buffer of {t.numel() * t.element_size()} bytes, need {nbytes}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, need {dtype}")
    return p


def lbm_shape(ctx):
    out = (C.c_int * 5)()
    _check(ctx, load().lbm_shape(ctx, out))
    return tuple(out[:])


def _sizes(ctx):
    """(q, N, compute dtype, compute bytes) of a context."""
    import torch
    q, nx, ny, nz, storage = lbm_shape(ctx)
    f64 = storage == F64
    return q, nx * ny * nz, (torch.float64 if f64 else torch.float32), (8 if f64 else 4)


def _hptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(ctx, rc):
    if rc != OK:
        raise LbmError(rc, load().lbm_last_error(ctx).decode())


def make_params(q, shape, periodic=(1, 1, 1), storage=F64, tau0=0.6, cs_smag=0.0, force=(0.0, 0.0, 0.0),
                wall_model=0, kappa=0.41, E=9.0, fringe_len=0, u_ref=0.0, z0=1.0, lid=0, collision=0,
                fd_weight=0.0, open_x=0, rho_out=1.0, slip=0, cs_field=0, stream=None) -> Params:
    p = Params()
    p.lattice = q
    p.nx, p.ny, p.nz = shape
    p.periodic = (C.c_int * 3)(*[int(v) for v in periodic])
    p.storage = STORAGE_NAMES.get(storage, storage) if isinstance(storage, str) else storage
    p.tau0, p.cs_smag = tau0, cs_smag
    p.force = (C.c_double * 3)(*force)
    p.wall_model, p.kappa, p.E = wall_model, kappa, E
    p.fringe_len, p.u_ref, p.z0, p.lid = fringe_len, u_ref, z0, lid
    p.collision = COLLISION_NAMES.get(collision, collision) if isinstance(collision, str) else collision
    p.fd_weight = fd_weight
    p.open_x, p.rho_out = int(open_x), rho_out
    p.slip = int(slip)
    p.cs_field = int(cs_field)
    p.stream = stream
    return p


# ---- C-ABI wrappers (same names) --------------------------------------------

def lbm_workspace_bytes(p: Params, mask=None, porous=False) -> int:
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    n = load().lbm_workspace_bytes(C.byref(p), _hptr(m), 1 if porous else 0)
    if n == 0:
        raise LbmError(EINVAL, load().lbm_last_error(None).decode())
    return n


def lbm_init(p: Params, mask, wall_dist, porosity, rho0_dev, u0_dev, workspace):
    import torch
    N = p.nx * p.ny * p.nz
    for a, name in ((mask, "mask"), (wall_dist, "wall_dist"), (porosity, "porosity")):
        if a is not None and np.asarray(a).size != N:
            raise ValueError(f"{name} must have nx*ny*nz = {N} entries")
    if rho0_dev is not None:
        _dbuf(rho0_dev, 8 * N, "rho0", torch.float64)
    if u0_dev is not None:
        _dbuf(u0_dev, 24 * N, "u0", torch.float64)
    _dbuf(workspace, 1, "workspace")
    keep = [None if a is None else np.ascontiguousarray(a, dtype=dt)
            for a, dt in ((mask, np.uint8), (wall_dist, np.float64), (porosity, np.float64))]
    ctx = C.c_void_p()
    rc = load().lbm_init(C.byref(ctx), C.byref(p), _hptr(keep[0]), _hptr(keep[1]), _hptr(keep[2]),
                         _dptr(rho0_dev), _dptr(u0_dev), _dptr(workspace), workspace.numel())
    if rc != OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return ctx


def lbm_step(ctx, n=1):
    _check(ctx, load().lbm_step(ctx, int(n)))


def lbm_moments(ctx, rho, u):
    q, N, dt, cb = _sizes(ctx)
    r = None if rho is None else _dbuf(rho, N * cb, "rho", dt)
    v = None if u is None else _dbuf(u, 3 * N * cb, "u", dt)
    _check(ctx, load().lbm_moments(ctx, r, v))


def lbm_diagnostics(ctx):
    out = (C.c_double * 4)()
    _check(ctx, load().lbm_diagnostics(ctx, out))
    return np.array(out[:])


def lbm_diagnostics_noalloc(ctx):
    out = (C.c_double * 4)()
    _check(ctx, load().lbm_diagnostics_noalloc(ctx, out))
    return np.array(out[:])


def lbm_sync(ctx):
    _check(ctx, load().lbm_sync(ctx))


def lbm_steps_done(ctx) -> int:
    return load().lbm_steps_done(ctx)


def lbm_get_populations(ctx, f):
    q, N, dt, cb = _sizes(ctx)
    _check(ctx, load().lbm_get_populations(ctx, _dbuf(f, q * N * cb, "populations", dt)))


def lbm_set_populations(ctx, f):
    q, N, dt, cb = _sizes(ctx)
    _check(ctx, load().lbm_set_populations(ctx, _dbuf(f, q * N * cb, "populations", dt)))


def lbm_state_bytes(ctx) -> int:
    return load().lbm_state_bytes(ctx)


def lbm_save_state(ctx, dst):
    _check(ctx, load().lbm_save_state(ctx, _dbuf(dst, lbm_state_bytes(ctx), "state")))


def lbm_load_state(ctx, src):
    _check(ctx, load().lbm_load_state(ctx, _dbuf(src, lbm_state_bytes(ctx), "state")))


def lbm_objective(ctx, planes) -> float:
    pl = (C.c_int * 2)(*planes)
    J = C.c_double()
    _check(ctx, load().lbm_objective(ctx, pl, C.byref(J)))
    return J.value


def lbm_adjoint_bytes(ctx) -> int:
    return load().lbm_adjoint_bytes(ctx)


def _lam(ctx, t):
    return _dbuf(t, lbm_adjoint_bytes(ctx), "adjoint")


def _nat(ctx, t):
    import torch
    q, N, dt, cb = _sizes(ctx)
    return _dbuf(t, q * N * 8, "natural", torch.float64)


def _grad(ctx, t):
    import torch
    q, N, dt, cb = _sizes(ctx)
    return _dbuf(t, N * 8, "grad_phi", torch.float64)


def lbm_adjoint_seed(ctx, planes, lam):
    pl = (C.c_int * 2)(*planes)
    _check(ctx, load().lbm_adjoint_seed(ctx, pl, _lam(ctx, lam)))


def lbm_adjoint_step(ctx, lam, grad):
    _check(ctx, load().lbm_adjoint_step(ctx, _lam(ctx, lam), _grad(ctx, grad)))


def lbm_adjoint_step_cs(ctx, lam, grad, grad_cs):
    _check(ctx, load().lbm_adjoint_step_cs(ctx, _lam(ctx, lam), _grad(ctx, grad), _grad(ctx, grad_cs)))


def lbm_set_smagorinsky(ctx, cs):
    """cs: float64 device tensor of N values, or None (back to the scalar)."""
    import torch
    q, N, dt, cb = _sizes(ctx)
    _check(ctx, load().lbm_set_smagorinsky(ctx, None if cs is None else _dbuf(cs, N * 8, "C_S field", torch.float64)))


def lbm_adjoint_to_natural(ctx, lam, nat):
    _check(ctx, load().lbm_adjoint_to_natural(ctx, _lam(ctx, lam), _nat(ctx, nat)))


def lbm_adjoint_from_natural(ctx, nat, lam):
    _check(ctx, load().lbm_adjoint_from_natural(ctx, _nat(ctx, nat), _lam(ctx, lam)))


def lbm_gradient(ctx, T, planes, snapshots, nsnap, lam, grad):
    pl = (C.c_int * 2)(*planes)
    J = C.c_double()
    nf = C.c_longlong()
    snaps = _dbuf(snapshots, int(nsnap) * lbm_state_bytes(ctx), "snapshots")
    _check(ctx, load().lbm_gradient(ctx, int(T), pl, snaps, int(nsnap), _lam(ctx, lam), _grad(ctx, grad),
                                    C.byref(J), C.byref(nf)))
    return J.value, nf.value


def lbm_gradient_mean(ctx, T, planes, snapshots, nsnap, lam, grad):
    """As lbm_gradient, for the time average (1/T) sum_{t=1..T} j(f_t)."""
    pl = (C.c_int * 2)(*planes)
    J = C.c_double()
    nf = C.c_longlong()
    snaps = _dbuf(snapshots, int(nsnap) * lbm_state_bytes(ctx), "snapshots")
    _check(ctx, load().lbm_gradient_mean(ctx, int(T), pl, snaps, int(nsnap), _lam(ctx, lam), _grad(ctx, grad),
                                         C.byref(J), C.byref(nf)))
    return J.value, nf.value


def lbm_gradient_cs(ctx, T, planes, snapshots, nsnap, lam, grad, grad_cs, mean=False):
    """lbm_gradient (or, with mean, lbm_gradient_mean) that also writes dJ/dC_S."""
    pl = (C.c_int * 2)(*planes)
    J = C.c_double()
    nf = C.c_longlong()
    snaps = _dbuf(snapshots, int(nsnap) * lbm_state_bytes(ctx), "snapshots")
    _check(ctx, load().lbm_gradient_cs(ctx, int(T), pl, snaps, int(nsnap), _lam(ctx, lam), _grad(ctx, grad),
                                       _grad(ctx, grad_cs), int(bool(mean)), C.byref(J), C.byref(nf)))
    return J.value, nf.value


def lbm_revolve_cost(T, nsnap) -> int:
    return load().lbm_revolve_cost(int(T), int(nsnap))


def lbm_set_inflow_vortices(ctx, yz, sign, intensity, sigma):
    """Vortex-method seed points (y, z) on the inflow plane (host arrays [n][2]
    and [n]), turbulence intensity and vortex size; n = 0 clears them."""
    yz = np.ascontiguousarray(np.asarray(yz, dtype=np.float64).reshape(-1, 2))
    sign = np.ascontiguousarray(np.asarray(sign, dtype=np.int32).reshape(-1))
    if len(sign) != len(yz):
        raise ValueError("one sign per vortex expected")
    ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a.size else None
    _check(ctx, load().lbm_set_inflow_vortices(ctx, len(sign), ptr(yz), ptr(sign), float(intensity), float(sigma)))


def lbm_wall_count(ctx) -> int:
    return load().lbm_wall_count(ctx)


def lbm_wall_records(ctx):
    nw = lbm_wall_count(ctx)
    cell = np.empty(nw, np.int32)
    ref = np.empty(nw, np.int32)
    normal = np.empty((nw, 3))
    utau, G, tau = np.empty(nw), np.empty(nw), np.empty(nw)
    _check(ctx, load().lbm_wall_records(ctx, _hptr(cell), _hptr(ref), _hptr(normal), _hptr(utau), _hptr(G),
                                        _hptr(tau)))
    return dict(cells=cell, refs=ref, normal=normal, utau=utau, G=G, tau=tau)


def lbm_profile(ctx, enable):
    _check(ctx, load().lbm_profile(ctx, 1 if enable else 0))


def lbm_profile_read(ctx):
    ms = (C.c_double * 3)()
    cnt = (C.c_longlong * 3)()
    _check(ctx, load().lbm_profile_read(ctx, ms, cnt))
    return np.array(ms[:]), np.array(cnt[:])


def lbm_stream_probe(ctx, n=20) -> float:
    """Mean milliseconds per launch of the bulk kernel's access pattern
    without the collision (n launches, alternating parity)."""
    ms = C.c_double()
    _check(ctx, load().lbm_stream_probe(ctx, int(n), C.byref(ms)))
    return ms.value


def lbm_slot_map(p: Params, mask, parity):
    """(read, write) int64 [q][N] slot indices of the in-place streaming map
    at the given parity, evaluated on the host (no GPU needed)."""
    q, N = p.lattice, p.nx * p.ny * p.nz
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rd = np.empty((q, N), np.int64)
    wr = np.empty((q, N), np.int64)
    rc = load().lbm_slot_map(C.byref(p), _hptr(m), int(parity), _hptr(rd), _hptr(wr))
    if rc != OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return rd, wr


def params_for(case, storage="f64", stream=None, cs_field=False) -> Params:
    """lbm_params of an ``inputs.Case``."""
    return make_params(case.q, case.shape, periodic=case.periodic, storage=storage, tau0=case.tau0,
                       cs_smag=case.cs_smag, force=case.force, wall_model=case.wall_model, kappa=case.kappa,
                       E=case.E, fringe_len=case.fringe_len, u_ref=case.u_ref, z0=case.z0, lid=case.lid,
                       collision=getattr(case, "collision", 0), fd_weight=getattr(case, "fd_weight", 0.0),
                       open_x=getattr(case, "open_x", 0), rho_out=getattr(case, "rho_out", 1.0),
                       slip=getattr(case, "slip", 0), cs_field=int(bool(cs_field)), stream=stream)


class SpreadBuffer:
    """Device buffer of lbm_workspace_alloc / lbm_adjoint_alloc: its arrays
    lie far apart in physical memory.  Offers the parts of a torch tensor the
    wrappers here use (data_ptr, numel, ...); released by free() or when
    collected."""
    is_cuda = True

    def __init__(self, ptr: int, nbytes: int):
        import torch
        self._ptr, self._n, self.dtype = int(ptr), int(nbytes), torch.uint8

    def data_ptr(self):
        if not self._ptr:
            raise ValueError("buffer already freed")
        return self._ptr

    def is_contiguous(self):
        return True

    def numel(self):
        return self._n

    def element_size(self):
        return 1

    def free(self):
        if self._ptr:
            ptr, self._ptr = self._ptr, 0
            rc = load().lbm_spread_free(C.c_void_p(ptr))
            if rc != OK:
                raise LbmError(rc, load().lbm_last_error(None).decode())

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lbm_workspace_alloc(p: Params, mask=None, porous=False) -> SpreadBuffer:
    keep = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    ptr, nb = C.c_void_p(), C.c_size_t()
    rc = load().lbm_workspace_alloc(C.byref(p), _hptr(keep), int(bool(porous)), C.byref(ptr), C.byref(nb))
    if rc != OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return SpreadBuffer(ptr.value, nb.value)


def lbm_adjoint_alloc(ctx) -> SpreadBuffer:
    ptr, nb = C.c_void_p(), C.c_size_t()
    rc = load().lbm_adjoint_alloc(ctx, C.byref(ptr), C.byref(nb))
    if rc != OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return SpreadBuffer(ptr.value, nb.value)


def lbm_spread_free(buf: SpreadBuffer):
    buf.free()


def lbm_last_error(ctx) -> str:
    return load().lbm_last_error(ctx).decode()


def lbm_free(ctx):
    load().lbm_free(ctx)


# ---- convenience object ------------------------------------------------------

class Lattice:
    """Owns a context and its torch-allocated workspace on the current device.

    ``case`` is an ``inputs.Case`` (or anything with the same attributes);
    ``storage`` one of "f64", "f32", "f16".  rho0/u0 of the case are uploaded
    to the device as float64 for initialisation and then released."""

    def __init__(self, case, storage="f64", stream=None, wall_dist="case", cs_field=False, spread=False):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.q = case.q
        self.shape = tuple(case.shape)
        self.N = int(np.prod(self.shape))
        self.storage = STORAGE_NAMES[storage] if isinstance(storage, str) else storage
        self.rdtype = torch.float64 if self.storage == F64 else torch.float32
        self.p = params_for(case, storage=self.storage, stream=stream.cuda_stream, cs_field=cs_field)
        porous = case.porosity is not None
        self.spread = bool(spread)
        if self.spread:
            # population arrays spread in physical memory (lbm_workspace_alloc)
            self.workspace = lbm_workspace_alloc(self.p, case.mask, porous)
            self.ws = self.workspace
        else:
            nbytes = lbm_workspace_bytes(self.p, case.mask, porous)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            off = (-self.workspace.data_ptr()) % 256
            self.ws = self.workspace[off:off + nbytes]
        dev = torch.device("cuda")

        def to_dev(a):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=torch.float64).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)

        rho0, u0 = to_dev(case.rho0), to_dev(case.u0)
        wd = case.wall_dist if isinstance(wall_dist, str) else wall_dist
        with torch.cuda.stream(stream):
            self.ctx = lbm_init(self.p, case.mask, wd, case.porosity, rho0, u0, self.ws)
        del rho0, u0

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            # at interpreter shutdown the module's globals may already be gone;
            # the process then releases everything itself
            try:
                lbm_sync(ctx)
            except Exception:
                pass
            try:
                lbm_free(ctx)
            except Exception:
                pass
            self.ctx = None

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def sync(self):
        lbm_sync(self.ctx)

    @property
    def steps(self) -> int:
        return lbm_steps_done(self.ctx)

    def moments(self):
        torch = self.torch
        rho = torch.empty(self.N, dtype=self.rdtype, device="cuda")
        u = torch.empty((3, self.N), dtype=self.rdtype, device="cuda")
        lbm_moments(self.ctx, rho, u)
        lbm_sync(self.ctx)
        return rho, u

    def diagnostics(self):
        return lbm_diagnostics(self.ctx)

    def set_smagorinsky(self, cs):
        """Per-cell C_S (array or tensor of N values; None = the scalar);
        the lattice must have been made with cs_field=True."""
        if cs is not None:
            cs = self.torch.as_tensor(np.asarray(cs, dtype=np.float64) if not isinstance(cs, self.torch.Tensor)
                                      else cs, dtype=self.torch.float64, device="cuda").contiguous()
        lbm_set_smagorinsky(self.ctx, cs)

    def populations(self):
        f = self.torch.empty((self.q, self.N), dtype=self.rdtype, device="cuda")
        lbm_get_populations(self.ctx, f)
        lbm_sync(self.ctx)
        return f

    def set_populations(self, f):
        f = f.to(device="cuda", dtype=self.rdtype).contiguous()
        lbm_set_populations(self.ctx, f)
        lbm_sync(self.ctx)

    def new_state_buffer(self, count=1):
        return self.torch.empty(count * lbm_state_bytes(self.ctx), dtype=self.torch.uint8, device="cuda")

    def save_state(self, buf):
        lbm_save_state(self.ctx, buf)

    def load_state(self, buf):
        lbm_load_state(self.ctx, buf)

    def objective(self, planes):
        return lbm_objective(self.ctx, planes)

    def new_adjoint(self, spread=False):
        """Buffer for an adjoint field in the library's in-memory form
        (read it in natural order with lbm_adjoint_to_natural); spread=True
        places its arrays apart in physical memory (lbm_adjoint_alloc)."""
        if spread:
            return lbm_adjoint_alloc(self.ctx)
        return self.torch.zeros(lbm_adjoint_bytes(self.ctx), dtype=self.torch.uint8, device="cuda")

    def new_natural(self):
        """Natural-order [q][N] FP64 buffer for adjoint values."""
        return self.torch.zeros((self.q, self.N), dtype=self.torch.float64, device="cuda")

    def new_gradient(self):
        return self.torch.zeros(self.N, dtype=self.torch.float64, device="cuda")

    def set_vortices(self, yz, sign, intensity, sigma):
        """Vortex-method perturbation of the inlet (open x faces)."""
        lbm_set_inflow_vortices(self.ctx, yz, sign, intensity, sigma)

    def wall_records(self):
        return lbm_wall_records(self.ctx)
