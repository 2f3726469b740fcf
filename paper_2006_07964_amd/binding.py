"""ctypes binding of libcfd (include/cfd.h): argument marshalling only.

Every function named ``cfd_*`` here calls the C function of the same name and raises
``CfdError`` on a non-zero status.  Device memory comes from torch tensors (their
``data_ptr()``); streams are torch streams (``cuda_stream`` handles).  Loading fails
loudly when the HIP library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfd.so")

CFD_OK = 0
CFD_ERR_ARG, CFD_ERR_ALLOC, CFD_ERR_HIP, CFD_ERR_STATE = -1, -2, -3, -4
CFD_ERR_JACOBIAN, CFD_ERR_NONFINITE, CFD_ERR_UNSUPPORTED = -5, -6, -7
CFD_FP64, CFD_MIXED = 0, 1
CFD_WENO_JS, CFD_WENO_LINEAR = 0, 1
CFD_AFWENO_MODIFIED, CFD_AFWENO_ORIGINAL = 0, 1
CFD_VISC_REFLECT, CFD_VISC_ONE_SIDED = 0, 1
CFD_BC_PERIODIC, CFD_BC_INTERFACE, CFD_BC_WALL, CFD_BC_FARFIELD, CFD_BC_FARFIELD_CHAR = 0, 1, 2, 3, 4
CFD_FIELDS_Q, CFD_FIELDS_VISC = 0, 1
CFD_DIR_XI, CFD_DIR_ETA, CFD_DIR_ZETA, CFD_TERM_INV, CFD_TERM_VIS, CFD_ALL = 1, 2, 4, 8, 16, 31


class CfdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libcfd error {code}: {msg}")
        self.code = code


class cfd_params(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("mach", C.c_double), ("reynolds", C.c_double), ("prandtl", C.c_double),
        ("suth", C.c_double), ("weno_eps", C.c_double), ("viscous", C.c_int32), ("weights", C.c_int32),
        ("scheme", C.c_int32), ("visc_closure", C.c_int32), ("t_wall", C.c_double), ("qinf", C.c_double * 5),
    ]


class cfd_block_desc(C.Structure):
    _fields_ = [
        ("ni", C.c_int32), ("nj", C.c_int32), ("nk", C.c_int32),
        ("ld_i", C.c_int64), ("ld_j", C.c_int64),
        ("precision", C.c_int32), ("bc", C.c_int32 * 6), ("params", cfd_params),
    ]


class cfd_interface(C.Structure):
    _fields_ = [("block_a", C.c_int32), ("face_a", C.c_int32), ("block_b", C.c_int32), ("face_b", C.c_int32),
                ("orient", C.c_int32)]


class cfd_patch(C.Structure):
    _fields_ = [("block_a", C.c_int32), ("face_a", C.c_int32), ("a_lo", C.c_int32 * 2), ("n", C.c_int32 * 2),
                ("block_b", C.c_int32), ("face_b", C.c_int32), ("b_lo", C.c_int32 * 2), ("orient", C.c_int32)]


_lib = None
_VP = C.c_void_p
_DP = C.POINTER(C.c_double)


def lib():
    """Load libcfd.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2006_07964_amd.build` "
                           "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    sig = {
        "cfd_last_error": ([], C.c_char_p),
        "cfd_block_create": ([C.POINTER(cfd_block_desc), _VP, C.POINTER(_VP)], C.c_int),
        "cfd_block_destroy": ([_VP], C.c_int),
        "cfd_block_set_stream": ([_VP, _VP], C.c_int),
        "cfd_block_bytes": ([_VP, C.POINTER(C.c_int64)], C.c_int),
        "cfd_metrics": ([_VP, _VP, C.c_int64, C.c_int64], C.c_int),
        "cfd_metrics_ptr": ([_VP, C.POINTER(_VP)], C.c_int),
        "cfd_rhs": ([_VP, _VP, _VP, C.c_uint], C.c_int),
        "cfd_rk_stage": ([_VP, C.c_int, C.c_double, _VP, _VP, _VP], C.c_int),
        "cfd_rk_stage_dev": ([_VP, C.c_int, _VP, _VP, _VP, _VP], C.c_int),
        "cfd_viscous_fluxes": ([_VP, _VP], C.c_int),
        "cfd_rhs_sweeps": ([_VP, _VP, _VP, C.c_uint], C.c_int),
        "cfd_rk_sweeps": ([_VP, C.c_int, C.c_double, _VP, _VP, _VP], C.c_int),
        "cfd_exchange_create": ([C.POINTER(_VP), C.c_int, C.POINTER(cfd_interface), C.c_int, C.POINTER(_VP)], C.c_int),
        "cfd_exchange_create_patched": ([C.POINTER(_VP), C.c_int, C.POINTER(cfd_patch), C.c_int, C.POINTER(_VP)],
                                        C.c_int),
        "cfd_exchange_destroy": ([_VP], C.c_int),
        "cfd_halo_exchange": ([_VP, C.c_int, C.POINTER(_VP), _VP], C.c_int),
        "cfd_dt_cfl": ([C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.c_double, _DP], C.c_int),
        "cfd_dt_cfl_dev": ([C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.c_double, _VP], C.c_int),
        "cfd_dt_local": ([C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.c_double, C.POINTER(_VP)], C.c_int),
        "cfd_block_set_local_dt": ([_VP, _VP], C.c_int),
        "cfd_residual": ([C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.POINTER(_VP), C.c_double, _DP], C.c_int),
        "cfd_residual_noalloc": ([C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.POINTER(_VP), C.c_double, _DP],
                                 C.c_int),
        "cfd_check_finite": ([_VP, _VP, C.POINTER(C.c_int)], C.c_int),
        "cfd_sync": ([_VP], C.c_int),
        "cfd_batch_create": ([C.POINTER(_VP), C.c_int, _VP, _VP, C.POINTER(_VP)], C.c_int),
        "cfd_batch_destroy": ([_VP], C.c_int),
        "cfd_batch_step": ([_VP, _VP, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP)], C.c_int),
        "cfd_batch_tuning": ([_VP, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "cfd_batch_set_tuning": ([_VP, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "cfd_batch_tuning_times": ([_VP, C.POINTER(C.c_float), C.c_int], C.c_int),
        "cfd_tile_config_count": ([], C.c_int),
        "cfd_sweep_order": ([C.POINTER(C.c_int)], C.c_int),
        "cfd_tile_config": ([C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "cfd_block_set_tiles": ([_VP, C.POINTER(C.c_int)], C.c_int),
        "cfd_block_tiles": ([_VP, C.POINTER(C.c_int)], C.c_int),
        "cfd_profile_enable": ([_VP, C.c_int], C.c_int),
        "cfd_profile_read": ([_VP, C.POINTER(C.c_char_p), C.POINTER(C.c_int64), _DP, C.c_int, C.POINTER(C.c_int)], C.c_int),
        "cfd_profile_reset": ([_VP], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc != CFD_OK:
        raise CfdError(rc, lib().cfd_last_error().decode(errors="replace"))
    return rc


def _ptr(x) -> Optional[int]:
    """Device address of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _vp_array(items):
    return (_VP * len(items))(*[_ptr(t) for t in items])


# ---- C entry points ----------------------------------------------------------------------
def cfd_last_error() -> str:
    return lib().cfd_last_error().decode(errors="replace")


def cfd_block_create(desc: cfd_block_desc, stream=None) -> int:
    h = _VP()
    _check(lib().cfd_block_create(C.byref(desc), _stream(stream), C.byref(h)))
    return h.value


def cfd_block_destroy(b: int) -> None:
    _check(lib().cfd_block_destroy(b))


def cfd_block_set_stream(b: int, stream) -> None:
    _check(lib().cfd_block_set_stream(b, _stream(stream)))


def cfd_block_bytes(b: int) -> int:
    v = C.c_int64()
    _check(lib().cfd_block_bytes(b, C.byref(v)))
    return v.value


def cfd_metrics(b: int, xyz, cld_i: int, cld_j: int) -> None:
    _check(lib().cfd_metrics(b, _ptr(xyz), cld_i, cld_j))


def cfd_metrics_ptr(b: int) -> int:
    p = _VP()
    _check(lib().cfd_metrics_ptr(b, C.byref(p)))
    return p.value


def cfd_rhs(b: int, q, r, mask: int = CFD_ALL) -> None:
    _check(lib().cfd_rhs(b, _ptr(q), _ptr(r), mask))


def cfd_rk_stage(b: int, stage: int, dt: float, qn, qcur, qout) -> None:
    _check(lib().cfd_rk_stage(b, stage, dt, _ptr(qn), _ptr(qcur), _ptr(qout)))


def cfd_rk_stage_dev(b: int, stage: int, dt_dev, qn, qcur, qout) -> None:
    _check(lib().cfd_rk_stage_dev(b, stage, _ptr(dt_dev), _ptr(qn), _ptr(qcur), _ptr(qout)))


def cfd_viscous_fluxes(b: int, q) -> None:
    _check(lib().cfd_viscous_fluxes(b, _ptr(q)))


def cfd_rhs_sweeps(b: int, q, r, mask: int = CFD_ALL) -> None:
    _check(lib().cfd_rhs_sweeps(b, _ptr(q), _ptr(r), mask))


def cfd_rk_sweeps(b: int, stage: int, dt: float, qn, qcur, qout) -> None:
    _check(lib().cfd_rk_sweeps(b, stage, dt, _ptr(qn), _ptr(qcur), _ptr(qout)))


def cfd_exchange_create(blocks: Sequence[int], interfaces: Sequence) -> int:
    arr = (_VP * len(blocks))(*blocks)
    n = len(interfaces)
    ifc = (cfd_interface * max(1, n))()
    for k, f in enumerate(interfaces):
        ifc[k].block_a, ifc[k].face_a, ifc[k].block_b, ifc[k].face_b = f.block_a, f.face_a, f.block_b, f.face_b
        ifc[k].orient = getattr(f, "orient", 0)
    h = _VP()
    _check(lib().cfd_exchange_create(arr, len(blocks), ifc, n, C.byref(h)))
    return h.value


def cfd_exchange_create_patched(blocks: Sequence[int], patches: Sequence) -> int:
    """patches: objects with block_a, face_a, a_lo, n, block_b, face_b, b_lo, orient."""
    arr = (_VP * len(blocks))(*blocks)
    n = len(patches)
    ps = (cfd_patch * max(1, n))()
    for k, p in enumerate(patches):
        ps[k].block_a, ps[k].face_a = p.block_a, p.face_a
        ps[k].a_lo[0], ps[k].a_lo[1] = p.a_lo
        ps[k].n[0], ps[k].n[1] = p.n
        ps[k].block_b, ps[k].face_b = p.block_b, p.face_b
        ps[k].b_lo[0], ps[k].b_lo[1] = p.b_lo
        ps[k].orient = getattr(p, "orient", 0)
    h = _VP()
    _check(lib().cfd_exchange_create_patched(arr, len(blocks), ps, n, C.byref(h)))
    return h.value


def cfd_exchange_destroy(x: int) -> None:
    _check(lib().cfd_exchange_destroy(x))


def cfd_halo_exchange(x: int, field_set: int, bufs=None, stream=None) -> None:
    arr = None if bufs is None else _vp_array(bufs)
    _check(lib().cfd_halo_exchange(x, field_set, arr, _stream(stream)))


def cfd_dt_cfl(blocks: Sequence[int], qs: Sequence, cfl: float) -> float:
    arr = (_VP * len(blocks))(*blocks)
    out = C.c_double()
    _check(lib().cfd_dt_cfl(arr, len(blocks), _vp_array(qs), cfl, C.byref(out)))
    return out.value


def cfd_dt_cfl_dev(blocks: Sequence[int], qs: Sequence, cfl: float, dt_dev) -> None:
    arr = (_VP * len(blocks))(*blocks)
    _check(lib().cfd_dt_cfl_dev(arr, len(blocks), _vp_array(qs), cfl, _ptr(dt_dev)))


def cfd_dt_local(blocks: Sequence[int], qs: Sequence, cfl: float, dt_fields: Sequence) -> None:
    arr = (_VP * len(blocks))(*blocks)
    _check(lib().cfd_dt_local(arr, len(blocks), _vp_array(qs), cfl, _vp_array(dt_fields)))


def cfd_block_set_local_dt(b: int, dt_field) -> None:
    _check(lib().cfd_block_set_local_dt(b, _ptr(dt_field)))


def cfd_residual(blocks: Sequence[int], a: Sequence, b: Optional[Sequence] = None, scale: float = 1.0):
    """(rms[5], max[5]) of scale * (a - b) over the interior points of all blocks."""
    arr = (_VP * len(blocks))(*blocks)
    out = (C.c_double * 10)()
    _check(lib().cfd_residual(arr, len(blocks), _vp_array(a), None if b is None else _vp_array(b), scale, out))
    return list(out[:5]), list(out[5:])


def cfd_residual_noalloc(blocks: Sequence[int], a: Sequence, b: Optional[Sequence] = None, scale: float = 1.0):
    """cfd_residual through the library's fixed scratch (no device allocation)."""
    arr = (_VP * len(blocks))(*blocks)
    out = (C.c_double * 10)()
    _check(lib().cfd_residual_noalloc(arr, len(blocks), _vp_array(a), None if b is None else _vp_array(b), scale,
                                      out))
    return list(out[:5]), list(out[5:])


def cfd_check_finite(b: int, q) -> bool:
    ok = C.c_int()
    rc = lib().cfd_check_finite(b, _ptr(q), C.byref(ok))
    if rc not in (CFD_OK, CFD_ERR_NONFINITE):
        _check(rc)
    return bool(ok.value)


def cfd_sync(b: int) -> None:
    _check(lib().cfd_sync(b))


def cfd_batch_create(blocks: Sequence[int], x: int, stream=None) -> int:
    arr = (_VP * len(blocks))(*blocks)
    h = _VP()
    _check(lib().cfd_batch_create(arr, len(blocks), x, _stream(stream), C.byref(h)))
    return h.value


def cfd_batch_destroy(bt: int) -> None:
    _check(lib().cfd_batch_destroy(bt))


def cfd_batch_step(bt: int, dt_dev, qn: Sequence, qa: Sequence, qb: Sequence) -> None:
    _check(lib().cfd_batch_step(bt, _ptr(dt_dev), _vp_array(qn), _vp_array(qa), _vp_array(qb)))


def cfd_batch_tuning(bt: int):
    cfg = (C.c_int * 3)()
    per = (C.c_int * 3)()
    _check(lib().cfd_batch_tuning(bt, cfg, per))
    return list(cfg), list(per)


def cfd_batch_set_tuning(bt: int, cfg, persist) -> None:
    c = (C.c_int * 3)(*cfg)
    p = (C.c_int * 3)(*persist)
    _check(lib().cfd_batch_set_tuning(bt, c, p))


def cfd_batch_tuning_times(bt: int):
    """Autotuner timings as {(direction, cfg, persistent): ms per launch}, measured ones only."""
    n = cfd_tile_config_count()
    ms = (C.c_float * (6 * n))()
    _check(lib().cfd_batch_tuning_times(bt, ms, 6 * n))
    return {(d, c, p): ms[(d * n + c) * 2 + p] for d in range(3) for c in range(n) for p in range(2)
            if ms[(d * n + c) * 2 + p] >= 0}


def cfd_sweep_order():
    """Directions (0 = xi, 1 = eta, 2 = zeta) in the order the sweeps run; the last one
    writes R or the RK stage."""
    d = (C.c_int * 3)()
    _check(lib().cfd_sweep_order(d))
    return list(d)


def cfd_tile_config_count() -> int:
    return lib().cfd_tile_config_count()


def cfd_tile_config(cfg: int):
    """(lines across, nodes along the sweep, threads) of tile shape cfg."""
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(lib().cfd_tile_config(cfg, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def cfd_block_set_tiles(b: int, cfg) -> None:
    _check(lib().cfd_block_set_tiles(b, (C.c_int * 3)(*cfg)))


def cfd_block_tiles(b: int):
    cfg = (C.c_int * 3)()
    _check(lib().cfd_block_tiles(b, cfg))
    return list(cfg)


def cfd_profile_enable(b: int, on: bool = True) -> None:
    _check(lib().cfd_profile_enable(b, int(on)))


def cfd_profile_read(b: int, cap: int = 64):
    names = (C.c_char_p * cap)()
    launches = (C.c_int64 * cap)()
    ms = (C.c_double * cap)()
    n = C.c_int()
    _check(lib().cfd_profile_read(b, names, launches, ms, cap, C.byref(n)))
    return {names[k].decode(): (launches[k], ms[k]) for k in range(min(n.value, cap))}


def cfd_profile_reset(b: int) -> None:
    _check(lib().cfd_profile_reset(b))


# ---- layout helpers ------------------------------------------------------------------------
def aligned_pitch(n: int) -> int:
    """Row pitch (elements) with halo 3 rounded up to 16 doubles (one 128-byte line)."""
    return ((n + 6 + 15) // 16) * 16


def state_tensor(desc: "cfd_block_desc", nvar: int = 5, device="cuda"):
    """Zeroed FP64 device tensor (nvar, nk+6, ld_j, ld_i) in the block's pitched layout, offset
    so that the first interior point of every row starts a 128-byte line when ld_i is a
    multiple of 16 (the same alignment libcfd gives its own planes)."""
    import torch
    plane = desc.ld_i * desc.ld_j * (desc.nk + 6)
    flat = torch.zeros(nvar * plane + 64, dtype=torch.float64, device=device)
    off = (-(flat.data_ptr() // 8 + 3)) % 16  # element offset putting (i=0) on a 128-byte line
    return flat[off:off + nvar * plane].view(nvar, desc.nk + 6, desc.ld_j, desc.ld_i)


def upload_state(desc: "cfd_block_desc", arr, device="cuda"):
    """Copy a tight host array (nvar, nk+6, nj+6, ni+6) into a new pitched device tensor."""
    import torch
    t = state_tensor(desc, arr.shape[0], device)
    t[:, :, :arr.shape[2], :arr.shape[3]].copy_(torch.from_numpy(arr))
    return t


def download_state(desc: "cfd_block_desc", t):
    """Tight host copy (nvar, nk+6, nj+6, ni+6) of a pitched device tensor."""
    return t[:, :, :desc.nj + 6, :desc.ni + 6].cpu().numpy()


# ---- descriptor helpers (plain data) -------------------------------------------------------
def make_desc(ni, nj, nk, precision=CFD_FP64, bc=(0, 0, 0, 0, 0, 0), ld_i=None, ld_j=None, gamma=1.4,
              mach=0.5, reynolds=1000.0, prandtl=0.71, suth=110.4 / 288.15, weno_eps=1e-6, viscous=True,
              weights=CFD_WENO_JS, scheme=None, t_wall=1.0,
              qinf=(1.0, 0.0, 0.0, 0.0, 1.0 / (1.4 * 0.4)), visc_closure=CFD_VISC_REFLECT) -> cfd_block_desc:
    d = cfd_block_desc()
    d.ni, d.nj, d.nk = ni, nj, nk
    d.ld_i = ni + 6 if ld_i is None else ld_i
    d.ld_j = nj + 6 if ld_j is None else ld_j
    d.precision = precision
    for f in range(6):
        d.bc[f] = int(bc[f])
    p = d.params
    p.gamma, p.mach, p.reynolds, p.prandtl, p.suth, p.weno_eps = gamma, mach, reynolds, prandtl, suth, weno_eps
    p.viscous = int(bool(viscous))
    p.weights = int(weights)
    p.scheme = CFD_AFWENO_MODIFIED if scheme is None else int(scheme)
    p.visc_closure = int(visc_closure)
    p.t_wall = t_wall
    for n in range(5):
        p.qinf[n] = float(qinf[n])
    return d


def desc_from_workload(wl, block: int = 0, precision=CFD_FP64, **over) -> cfd_block_desc:
    b = wl.blocks[block]
    kw = dict(precision=precision, bc=b.bc, gamma=wl.gamma, mach=wl.mach, reynolds=wl.reynolds,
              prandtl=wl.prandtl, suth=wl.suth, weno_eps=wl.eps, viscous=wl.viscous, t_wall=wl.t_wall,
              qinf=wl.qinf, visc_closure=getattr(wl, "visc_closure", CFD_VISC_REFLECT))
    kw.update(over)
    return make_desc(b.ni, b.nj, b.nk, **kw)
