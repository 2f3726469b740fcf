"""ctypes front end of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.  The shared library is compiled
from oracle.c with gcc on first use when it is missing (or by ``build()``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

XI, ETA, ZETA, INV, VIS, ALL = 1, 2, 4, 8, 16, 31
AFWENO_MODIFIED, AFWENO_ORIGINAL = 0, 1
VISC_REFLECT, VISC_ONE_SIDED = 0, 1
BC_PERIODIC, BC_INTERFACE, BC_WALL, BC_FARFIELD, BC_FARFIELD_CHAR = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-std=c99", "-shared", "-fPIC", "-o", _SO + ".tmp",
               os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Cfg(C.Structure):
    _fields_ = [
        ("ni", C.c_int), ("nj", C.c_int), ("nk", C.c_int),
        ("gamma", C.c_double), ("mach", C.c_double), ("reynolds", C.c_double),
        ("prandtl", C.c_double), ("suth", C.c_double), ("eps", C.c_double),
        ("viscous", C.c_int), ("linear_weights", C.c_int), ("scheme", C.c_int), ("bc", C.c_int * 6),
        ("t_wall", C.c_double), ("qinf", C.c_double * 5), ("visc_closure", C.c_int),
    ]


class Iface(C.Structure):
    _fields_ = [("block_a", C.c_int), ("face_a", C.c_int), ("block_b", C.c_int), ("face_b", C.c_int),
                ("orient", C.c_int)]


class Patch(C.Structure):
    """A rectangle of face_a of block_a joined node to node to a rectangle of face_b of
    block_b (see oracle_patch in oracle.h)."""
    _fields_ = [("block_a", C.c_int), ("face_a", C.c_int), ("a_lo", C.c_int * 2), ("n", C.c_int * 2),
                ("block_b", C.c_int), ("face_b", C.c_int), ("b_lo", C.c_int * 2), ("orient", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        P = C.POINTER(C.c_double)
        cp = C.POINTER(Cfg)
        L.oracle_metrics.argtypes = [cp, P, P]
        L.oracle_rhs.argtypes = [cp, P, P, P, C.c_uint, C.c_int, C.c_int]
        L.oracle_rk_stage.argtypes = [cp, P, C.c_int, C.c_double, P, P, P]
        L.oracle_rk_step.argtypes = [cp, P, C.c_double, P]
        L.oracle_periodic_wrap.argtypes = [cp, P, C.c_int]
        L.oracle_periodic_wrap.restype = None
        L.oracle_bc_fill.argtypes = [cp, P]
        L.oracle_bc_fill.restype = None
        L.oracle_bc_fill_met.argtypes = [cp, P, P]
        L.oracle_bc_fill_met.restype = None
        L.oracle_char_farfield.argtypes = [P, P, P, C.c_double, P]
        L.oracle_char_farfield.restype = None
        L.oracle_dt_cfl.argtypes = [cp, P, P, C.c_double]
        L.oracle_dt_cfl.restype = C.c_double
        L.oracle_dt_local.argtypes = [cp, P, P, C.c_double, P]
        L.oracle_dt_local.restype = None
        L.oracle_rk_step_local.argtypes = [cp, P, P, P]
        L.oracle_weno5.argtypes = [P, C.c_double, C.c_int, P, P]
        L.oracle_weno5.restype = None
        L.oracle_eigvec.argtypes = [P, P, C.c_double, P, P]
        L.oracle_split_flux.argtypes = [P, P, C.c_double, P, P]
        L.oracle_split_flux.restype = None
        L.oracle_phys_flux.argtypes = [P, P, C.c_double, P]
        L.oracle_phys_flux.restype = None
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        L.oracle_wall_reset.argtypes = [cp, P]
        L.oracle_wall_reset.restype = None
        L.oracle_viscosity.argtypes = [C.c_double, C.c_double]
        L.oracle_viscosity.restype = C.c_double
        PP = C.POINTER(P)
        L.oracle_exchange.argtypes = [cp, C.c_int, PP, C.c_int, C.POINTER(Iface), C.c_int]
        L.oracle_rhs_multi.argtypes = [cp, C.c_int, PP, PP, PP, C.c_uint, C.POINTER(Iface), C.c_int]
        L.oracle_rk_step_multi.argtypes = [cp, C.c_int, PP, C.c_double, PP, C.POINTER(Iface), C.c_int]
        L.oracle_halo_patched.argtypes = [cp, C.c_int, PP, PP, C.POINTER(Patch), C.c_int]
        L.oracle_rhs_patched.argtypes = [cp, C.c_int, PP, PP, PP, C.c_uint, C.POINTER(Patch), C.c_int]
        L.oracle_rk_step_patched.argtypes = [cp, C.c_int, PP, C.c_double, PP, C.POINTER(Patch), C.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_cfg(ni, nj, nk, gamma=1.4, mach=0.5, reynolds=1000.0, prandtl=0.71,
             suth=110.4 / 288.15, eps=1e-6, viscous=True, linear_weights=False, scheme=0,
             bc=(0, 0, 0, 0, 0, 0), t_wall=1.0, qinf=(1.0, 0.0, 0.0, 0.0, 1.0 / (1.4 * 0.4)),
             visc_closure=VISC_REFLECT) -> Cfg:
    c = Cfg()
    c.ni, c.nj, c.nk = ni, nj, nk
    c.gamma, c.mach, c.reynolds, c.prandtl, c.suth, c.eps = gamma, mach, reynolds, prandtl, suth, eps
    c.viscous = int(bool(viscous))
    c.linear_weights = int(bool(linear_weights))
    c.scheme = int(scheme)
    for n in range(6):
        c.bc[n] = int(bc[n])
    c.t_wall = t_wall
    for n in range(5):
        c.qinf[n] = float(qinf[n])
    c.visc_closure = int(visc_closure)
    return c


def cfg_from_workload(wl, block=0, **over) -> Cfg:
    b = wl.blocks[block]
    kw = dict(gamma=wl.gamma, mach=wl.mach, reynolds=wl.reynolds, prandtl=wl.prandtl, suth=wl.suth,
              eps=wl.eps, viscous=wl.viscous, bc=b.bc, t_wall=wl.t_wall, qinf=wl.qinf,
              visc_closure=getattr(wl, "visc_closure", VISC_REFLECT))
    kw.update(over)
    return make_cfg(b.ni, b.nj, b.nk, **kw)


def state_shape(c: Cfg, nvar=5):
    return (nvar, c.nk + 6, c.nj + 6, c.ni + 6)


def metrics(c: Cfg, xyz: np.ndarray) -> np.ndarray:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    assert xyz.shape == (3, c.nk + 12, c.nj + 12, c.ni + 12)
    met = np.zeros(state_shape(c, 10))
    rc = lib().oracle_metrics(C.byref(c), _p(xyz), _p(met))
    if rc != 0:
        raise ValueError(f"oracle_metrics failed ({rc}): non-positive Jacobian")
    return met


def rhs(c: Cfg, met: np.ndarray, q: np.ndarray, mask: int = ALL, k0: int = 0, k1: int = None) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    r = np.zeros(state_shape(c))
    rc = lib().oracle_rhs(C.byref(c), _p(met), _p(q), _p(r), mask, k0, c.nk if k1 is None else k1)
    if rc != 0:
        raise ValueError(f"oracle_rhs failed ({rc})")
    return r


def rk_stage(c: Cfg, met, stage, dt, qn, qcur) -> np.ndarray:
    out = np.array(qcur, dtype=np.float64, copy=True)
    rc = lib().oracle_rk_stage(C.byref(c), _p(met), stage, dt, _p(np.ascontiguousarray(qn)),
                               _p(np.ascontiguousarray(qcur)), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_rk_stage failed ({rc})")
    return out


def rk_step(c: Cfg, met, dt, q) -> np.ndarray:
    out = np.array(q, dtype=np.float64, copy=True)
    rc = lib().oracle_rk_step(C.byref(c), _p(met), dt, _p(out))
    if rc != 0:
        raise ValueError(f"oracle_rk_step failed ({rc})")
    return out


def periodic_wrap(c: Cfg, a: np.ndarray) -> np.ndarray:
    out = np.array(a, dtype=np.float64, copy=True)
    lib().oracle_periodic_wrap(C.byref(c), _p(out), out.shape[0])
    return out


def bc_fill(c: Cfg, q: np.ndarray, met: np.ndarray = None) -> np.ndarray:
    out = np.array(q, dtype=np.float64, copy=True)
    if met is None:
        lib().oracle_bc_fill(C.byref(c), _p(out))
    else:
        lib().oracle_bc_fill_met(C.byref(c), _p(np.ascontiguousarray(met)), _p(out))
    return out


def char_farfield(qb, n, qf, gamma=1.4) -> np.ndarray:
    a, nn, f = (np.ascontiguousarray(x, dtype=np.float64) for x in (qb, n, qf))
    out = np.zeros(5)
    lib().oracle_char_farfield(_p(a), _p(nn), _p(f), gamma, _p(out))
    return out


def wall_reset(c: Cfg, q: np.ndarray) -> np.ndarray:
    out = np.array(q, dtype=np.float64, copy=True)
    lib().oracle_wall_reset(C.byref(c), _p(out))
    return out


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> int:
    """Use n OpenMP threads from now on; returns the previous count."""
    return int(lib().oracle_set_threads(int(n)))


def dt_cfl(c: Cfg, met, q, cfl) -> float:
    return float(lib().oracle_dt_cfl(C.byref(c), _p(met), _p(np.ascontiguousarray(q)), cfl))


def residual(a_arrays, b_arrays=None, scale: float = 1.0):
    """Residual norms of the iteration loop (Fig 2's residual evaluation; Sec. 4.5.3 forms
    them by reductions over the grid).  Reading: per conserved quantity, the root mean
    square and the maximum of |d| with d = scale * (A - B) over the interior points of all
    blocks (B absent: d = scale * A).  Plain numpy in FP64: returns (rms[5], max[5])."""
    sq = np.zeros(5)
    mx = np.zeros(5)
    n = 0
    for bi, a in enumerate(a_arrays):
        d = np.asarray(a, dtype=np.float64)[:, 3:-3, 3:-3, 3:-3]
        if b_arrays is not None and b_arrays[bi] is not None:
            d = d - np.asarray(b_arrays[bi], dtype=np.float64)[:, 3:-3, 3:-3, 3:-3]
        d = scale * d
        sq += np.sum(d * d, axis=(1, 2, 3))
        mx = np.maximum(mx, np.max(np.abs(d), axis=(1, 2, 3)))
        n += d[0].size
    return list(np.sqrt(sq / n)), list(mx)


def dt_local(c: Cfg, met, q, cfl) -> np.ndarray:
    """Per-point CFL steps (one plane in the state layout; halo entries zero)."""
    out = np.zeros(state_shape(c, 1))
    lib().oracle_dt_local(C.byref(c), _p(met), _p(np.ascontiguousarray(q)), cfl, _p(out))
    return out


def rk_step_local(c: Cfg, met, dt_field, q) -> np.ndarray:
    out = np.array(q, dtype=np.float64, copy=True)
    rc = lib().oracle_rk_step_local(C.byref(c), _p(met), _p(np.ascontiguousarray(dt_field, dtype=np.float64)), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_rk_step_local failed ({rc})")
    return out


def weno5(v: Sequence[float], eps: float = 1e-6, linear: bool = False):
    vv = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(2)
    beta = np.zeros(3)
    lib().oracle_weno5(_p(vv), eps, int(linear), _p(out), _p(beta))
    return out, beta


def eigvec(q, k, gamma=1.4):
    L = np.zeros(25)
    R = np.zeros(25)
    rc = lib().oracle_eigvec(_p(np.ascontiguousarray(q, dtype=np.float64)),
                             _p(np.ascontiguousarray(k, dtype=np.float64)), gamma, _p(L), _p(R))
    if rc != 0:
        raise ValueError("singular eigenvector matrix")
    return L.reshape(5, 5), R.reshape(5, 5)


def split_flux(q, m, gamma=1.4):
    fp = np.zeros(5)
    fm = np.zeros(5)
    lib().oracle_split_flux(_p(np.ascontiguousarray(q, dtype=np.float64)),
                            _p(np.ascontiguousarray(m, dtype=np.float64)), gamma, _p(fp), _p(fm))
    return fp, fm


def phys_flux(q, m, gamma=1.4):
    f = np.zeros(5)
    lib().oracle_phys_flux(_p(np.ascontiguousarray(q, dtype=np.float64)),
                           _p(np.ascontiguousarray(m, dtype=np.float64)), gamma, _p(f))
    return f


def viscosity(T: float, suth: float = 110.4 / 288.15) -> float:
    return float(lib().oracle_viscosity(T, suth))


def _ptr_array(arrs):
    P = C.POINTER(C.c_double)
    return (P * len(arrs))(*[_p(a) for a in arrs])


def _ifaces(ifc):
    arr = (Iface * max(1, len(ifc)))()
    for n, f in enumerate(ifc):
        arr[n].block_a, arr[n].face_a, arr[n].block_b, arr[n].face_b = f.block_a, f.face_a, f.block_b, f.face_b
        arr[n].orient = getattr(f, "orient", 0)
    return arr


def exchange(cfgs, arrays, ifc):
    cs = (Cfg * len(cfgs))(*cfgs)
    rc = lib().oracle_exchange(cs, len(cfgs), _ptr_array(arrays), arrays[0].shape[0], _ifaces(ifc), len(ifc))
    if rc != 0:
        raise ValueError("oracle_exchange failed")


def rhs_multi(cfgs, mets, qs, ifc, mask=ALL):
    cs = (Cfg * len(cfgs))(*cfgs)
    rs = [np.zeros(state_shape(c)) for c in cfgs]
    rc = lib().oracle_rhs_multi(cs, len(cfgs), _ptr_array(mets), _ptr_array(qs), _ptr_array(rs), mask,
                                _ifaces(ifc), len(ifc))
    if rc != 0:
        raise ValueError("oracle_rhs_multi failed")
    return rs


def rk_step_multi(cfgs, mets, dt, qs, ifc):
    cs = (Cfg * len(cfgs))(*cfgs)
    out = [np.array(q, copy=True) for q in qs]
    rc = lib().oracle_rk_step_multi(cs, len(cfgs), _ptr_array(mets), dt, _ptr_array(out), _ifaces(ifc), len(ifc))
    if rc != 0:
        raise ValueError("oracle_rk_step_multi failed")
    return out


def _patches(patches):
    arr = (Patch * max(1, len(patches)))()
    for k, p in enumerate(patches):
        arr[k].block_a, arr[k].face_a = p.block_a, p.face_a
        arr[k].a_lo[0], arr[k].a_lo[1] = p.a_lo
        arr[k].n[0], arr[k].n[1] = p.n
        arr[k].block_b, arr[k].face_b = p.block_b, p.face_b
        arr[k].b_lo[0], arr[k].b_lo[1] = p.b_lo
        arr[k].orient = p.orient
    return arr


def halo_patched(cfgs, mets, qs, patches):
    """Halos of all blocks as after a stage (wall reset, periodic wraps, patch copies,
    ghost fills), on copies of qs."""
    cs = (Cfg * len(cfgs))(*cfgs)
    out = [np.array(q, dtype=np.float64, copy=True) for q in qs]
    mp = _ptr_array(mets) if mets is not None else None
    rc = lib().oracle_halo_patched(cs, len(cfgs), mp, _ptr_array(out), _patches(patches), len(patches))
    if rc != 0:
        raise ValueError("oracle_halo_patched: the patches break a rule")
    return out


def rhs_patched(cfgs, mets, qs, patches, mask=ALL):
    cs = (Cfg * len(cfgs))(*cfgs)
    rs = [np.zeros(state_shape(c)) for c in cfgs]
    rc = lib().oracle_rhs_patched(cs, len(cfgs), _ptr_array(mets), _ptr_array(qs), _ptr_array(rs), mask,
                                  _patches(patches), len(patches))
    if rc != 0:
        raise ValueError("oracle_rhs_patched failed")
    return rs


def rk_step_patched(cfgs, mets, dt, qs, patches):
    cs = (Cfg * len(cfgs))(*cfgs)
    out = [np.array(q, copy=True) for q in qs]
    rc = lib().oracle_rk_step_patched(cs, len(cfgs), _ptr_array(mets), dt, _ptr_array(out), _patches(patches),
                                      len(patches))
    if rc != 0:
        raise ValueError("oracle_rk_step_patched failed")
    return out
