"""Helpers of the GPU tests: device copies of seeded workloads and the libcfd call sequence."""
import ctypes as C

import numpy as np

from paper_2006_07964_amd import binding as B

_hip = None


def hip():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipDeviceSynchronize.restype = C.c_int
    return _hip


def dev_to_host(ptr: int, shape, dtype=np.float64) -> np.ndarray:
    """Copy raw device memory (library-owned) to a new host array (synchronous)."""
    out = np.empty(shape, dtype=dtype)
    rc = hip().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # device to host
    assert rc == 0, f"hipMemcpy failed {rc}"
    return out


def torch_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


class DevBlock:
    """One block on the GPU: coordinates, metrics and three state buffers."""

    def __init__(self, wl, bi=0, precision=B.CFD_FP64, q=None, **over):
        import torch
        b = wl.blocks[bi]
        self.wl, self.blk = wl, b
        self.desc = B.desc_from_workload(wl, bi, precision, **over)
        self.h = B.cfd_block_create(self.desc, torch.cuda.current_stream())
        self.xyz = torch_dev(b.xyz)
        B.cfd_metrics(self.h, self.xyz, b.ni + 12, b.nj + 12)
        self.q = torch_dev(b.q if q is None else q)
        self.qa = self.q.clone()
        self.qb = self.q.clone()
        self.r = torch.zeros_like(self.q)
        self.x = None

    @property
    def shape(self):
        return self.q.shape

    def metrics_host(self):
        import torch
        torch.cuda.synchronize()
        return dev_to_host(B.cfd_metrics_ptr(self.h), (10,) + tuple(self.q.shape[1:]))

    def exchange(self):
        if self.x is None:
            self.x = B.cfd_exchange_create([self.h], [])
        return self.x

    def halo(self, buf):
        B.cfd_halo_exchange(self.exchange(), B.CFD_FIELDS_Q, [buf])

    def rhs(self, mask=B.CFD_ALL, q=None):
        B.cfd_rhs(self.h, self.q if q is None else q, self.r, mask)
        return self.r.cpu().numpy()

    def step(self, dt):
        B.cfd_rk_stage(self.h, 0, dt, self.q, self.q, self.qa)
        self.halo(self.qa)
        B.cfd_rk_stage(self.h, 1, dt, self.q, self.qa, self.qb)
        self.halo(self.qb)
        B.cfd_rk_stage(self.h, 2, dt, self.q, self.qb, self.q)
        self.halo(self.q)

    def close(self):
        if self.x is not None:
            B.cfd_exchange_destroy(self.x)
            self.x = None
        if self.h:
            B.cfd_block_destroy(self.h)
            self.h = None


def normwise(a, b):
    """Normwise relative error of a state on the interior, per conserved quantity:
    [rho, momentum, e], the momentum taken as one vector (its three components share
    the norm max_c ||b_c||_inf, so a component that is nearly zero everywhere is not
    measured against its own tiny scale)."""
    ai = a[:, 3:-3, 3:-3, 3:-3]
    bi = b[:, 3:-3, 3:-3, 3:-3]

    def rel(sl):
        den = np.max(np.abs(bi[sl]))
        return np.max(np.abs(ai[sl] - bi[sl])) / den

    return np.array([rel(slice(0, 1)), rel(slice(1, 4)), rel(slice(4, 5))])


def per_component(a, b):
    """||a_f - b_f||_inf / ||b_f||_inf for each of the five planes (reported, not gated)."""
    ai = a[:, 3:-3, 3:-3, 3:-3]
    bi = b[:, 3:-3, 3:-3, 3:-3]
    return np.array([np.max(np.abs(ai[f] - bi[f])) / max(np.max(np.abs(bi[f])), 1e-300) for f in range(5)])


def vector_norm_err(a, b):
    """||a - b||_inf / ||b||_inf over all fields of the interior."""
    ai = a[:, 3:-3, 3:-3, 3:-3]
    bi = b[:, 3:-3, 3:-3, 3:-3]
    return float(np.max(np.abs(ai - bi)) / np.max(np.abs(bi)))
