"""GPU (libcfd through its C ABI) against the CPU oracle on identical seeded inputs.

Bar: states after every RK step within a normwise relative 1e-12 per conserved quantity
(density, momentum vector, energy; see tests/_gpu.normwise); the metrics
within 1e-13.  Right-hand sides are compared per conserved quantity (normwise): within
1e-12 with the ideal (linear) weights (rounding of O(1) fluxes whose differences are
O(1e-2), measured ~1e-13), and within 5e-11 with the WENO-JS weights of Eq 15.  The
oracle evaluates the smoothness indicators in the expanded quadratic form printed as
Eq 17, whose rounding is absolute, about 30 * 1.1e-16 * |V|^2 (the GPU forms the same
beta from squared differences, with a relative rounding).  Where beta << eps = 1e-6 the
weights are set by eps + beta, so that difference moves a weight by ~2 * 3.3e-15 |V|^2 /
eps ~ 7e-9 |V|^2 relative, and the interpolated value by that times the spread of the
sub-stencil values, which is below ~1e-3 |V| wherever beta < eps: ~1e-11 of the flux scale
for |V| ~ 1 to 2 (measured 2e-11 on the vortex case).  One RK stage multiplies an RHS
error by dt*|R|/|Q| ~ 1e-2, well inside the 1e-12 state bar.
"""
import numpy as np
import pytest

import oracle as O
from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevBlock, normwise, per_component, vector_norm_err

pytestmark = pytest.mark.gpu

TOL = 1e-12        # states after an RK step, per field
TOL_RHS_JS = 5e-11  # right-hand side with WENO-JS weights, per conserved quantity
TOL_RHS_LIN = 1e-12  # right-hand side with ideal weights, per conserved quantity


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def _pair(wl, pitched=False, **over):
    dev = DevBlock(wl, pitched=pitched, **over)
    c = O.cfg_from_workload(wl, linear_weights=over.get("weights", B.CFD_WENO_JS) == B.CFD_WENO_LINEAR,
                            viscous=over.get("viscous", wl.viscous))
    met = O.metrics(c, wl.blocks[0].xyz)
    return dev, c, met


SIZES = [(32, 32, 32), (23, 17, 11), (7, 9, 8), (40, 7, 19)]


def _vortex(ni, nj, nk, seed=1):
    wl = W.vortex_wavy(ni, nj=nj, nk=nk, seed=seed)
    return wl


@pytest.mark.parametrize("size", SIZES)
def test_metrics(size):
    wl = _vortex(*size)
    dev, c, met = _pair(wl)
    try:
        got = dev.metrics_host()
        for p in range(10):
            err = np.max(np.abs(got[p] - met[p])) / np.max(np.abs(met[p]))
            assert err < 1e-13, (p, err)
    finally:
        dev.close()


@pytest.mark.parametrize("size", SIZES)
@pytest.mark.parametrize("mask", [B.CFD_DIR_XI | B.CFD_TERM_INV, B.CFD_DIR_ETA | B.CFD_TERM_INV,
                                  B.CFD_DIR_ZETA | B.CFD_TERM_INV, 7 | B.CFD_TERM_VIS, B.CFD_ALL])
def test_rhs(size, mask):
    wl = _vortex(*size)
    dev, c, met = _pair(wl)
    try:
        got = dev.rhs(mask)
        ref = O.rhs(c, met, wl.blocks[0].q, mask)
        err = normwise(got, ref)
        print(size, mask, "whole vector", vector_norm_err(got, ref), "per quantity", err)
        assert np.all(err < TOL_RHS_JS), err
    finally:
        dev.close()


@pytest.mark.parametrize("weights", [B.CFD_WENO_LINEAR, B.CFD_WENO_JS])
def test_rhs_weights_and_euler(weights):
    wl = _vortex(24, 20, 16)
    dev, c, met = _pair(wl, weights=weights, viscous=False)
    try:
        got = dev.rhs()
        ref = O.rhs(c, met, wl.blocks[0].q)
        err = normwise(got, ref)
        print(weights, "whole vector", vector_norm_err(got, ref), "per quantity", err)
        assert np.all(err < (TOL_RHS_LIN if weights == B.CFD_WENO_LINEAR else TOL_RHS_JS)), err
    finally:
        dev.close()


def test_free_stream_preservation():
    wl = _vortex(32, 32, 32)
    q = W.uniform_state(wl.blocks[0].q.shape[1:], u=0.5, v=-0.2, w=0.1)
    dev = DevBlock(wl, q=q)
    try:
        r = dev.rhs()
        assert np.max(np.abs(r[:, 3:-3, 3:-3, 3:-3])) < 1e-12
    finally:
        dev.close()


def test_dt_cfl():
    wl = _vortex(32, 32, 32)
    dev, c, met = _pair(wl)
    try:
        dt = B.cfd_dt_cfl([dev.h], [dev.q], 0.5)
        assert dt == pytest.approx(O.dt_cfl(c, met, wl.blocks[0].q, 0.5), rel=1e-14)
    finally:
        dev.close()


@pytest.mark.parametrize("size", [(32, 32, 32), (23, 17, 11)])
def test_periodic_halo_exchange(size):
    import torch
    wl = _vortex(*size)
    dev, c, met = _pair(wl)
    try:
        q = wl.blocks[0].q.copy()
        q[:, :3] = np.nan
        q[:, -3:] = np.nan
        q[:, :, :3] = np.nan
        q[:, :, -3:] = np.nan
        q[:, :, :, :3] = np.nan
        q[:, :, :, -3:] = np.nan
        buf = B.upload_state(dev.desc, q)
        dev.halo(buf)
        got = dev.host(buf)
        ref = O.periodic_wrap(c, q)
        s = slice(3, -3)
        for face in [(slice(None), s, s, slice(0, 3)), (slice(None), s, s, slice(-3, None)),
                     (slice(None), s, slice(0, 3), s), (slice(None), s, slice(-3, None), s),
                     (slice(None), slice(0, 3), s, s), (slice(None), slice(-3, None), s, s)]:
            np.testing.assert_array_equal(got[face], ref[face])
    finally:
        dev.close()


def test_rk_ten_steps_c1():
    """The 32^3 vortex on the wavy grid: 10 RK3 steps, parity after every step."""
    wl = W.vortex_wavy(32, seed=1)
    dev, c, met = _pair(wl)
    try:
        q = wl.blocks[0].q
        dt = O.dt_cfl(c, met, q, wl.cfl)
        qo = q.copy()
        for step in range(10):
            dev.step(dt)
            qo = O.rk_step(c, met, dt, qo)
            got = dev.host(dev.q)
            err = normwise(got, qo)
            print(step, err, per_component(got, qo))
            assert np.all(err < TOL), (step, err)
    finally:
        dev.close()


@pytest.mark.parametrize("size,pitched", [((23, 17, 11), False), ((7, 7, 7), False), ((23, 17, 11), True),
                                          ((40, 33, 9), True)])
def test_rk_ragged(size, pitched):
    wl = _vortex(*size)
    dev, c, met = _pair(wl, pitched=pitched)
    try:
        q = wl.blocks[0].q
        dt = O.dt_cfl(c, met, q, 0.5)
        qo = q.copy()
        for step in range(3):
            dev.step(dt)
            qo = O.rk_step(c, met, dt, qo)
        assert np.all(normwise(dev.host(dev.q), qo) < TOL)
    finally:
        dev.close()


def test_rk_stage_dev_dt_matches_host_dt():
    import torch
    wl = _vortex(24, 20, 16)
    dev, c, met = _pair(wl)
    try:
        dt = 1.3e-3
        B.cfd_rk_stage(dev.h, 0, dt, dev.q, dev.q, dev.qa)
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        B.cfd_rk_stage_dev(dev.h, 0, dt_dev, dev.q, dev.q, dev.qb)
        assert torch.equal(dev.qa, dev.qb)
    finally:
        dev.close()


def test_deterministic():
    wl = _vortex(24, 20, 16)
    dev = DevBlock(wl)
    try:
        a = dev.rhs().copy()
        b = dev.rhs()
        np.testing.assert_array_equal(a, b)
    finally:
        dev.close()


def test_every_tile_shape_agrees():
    """A ragged block (tiles cut unevenly along every direction): RHS and one RK step with
    each sweep tile shape against the default shape.  The arithmetic per node does not
    depend on the tile, but each shape is a separately compiled kernel whose multiply-add
    contraction may differ, so the comparison allows round-off (normwise 1e-13)."""
    wl = _vortex(37, 29, 23)
    dev = DevBlock(wl, pitched=True)
    try:
        ref = dev.rhs().copy()
        dt = 1e-3
        q0 = dev.q.clone()
        dev.step(dt)
        ref_q = dev.host(dev.q).copy()
        for cfg in range(B.cfd_tile_config_count()):
            B.cfd_block_set_tiles(dev.h, [cfg, cfg, cfg])
            assert B.cfd_block_tiles(dev.h) == [cfg, cfg, cfg]
            dev.q.copy_(q0)
            got = dev.rhs()
            diff = got != ref
            print(f"tile shape {cfg} {B.cfd_tile_config(cfg)}: {int(diff.sum())} RHS values differ, "
                  f"vector error {vector_norm_err(got, ref):.2e}")
            if diff.any():
                idx = np.argwhere(diff)
                for ax, name in ((3, "i"), (2, "j"), (1, "k")):
                    vals, cnt = np.unique(idx[:, ax] - 3, return_counts=True)
                    print(f"   along {name}: {dict(zip(vals.tolist(), cnt.tolist()))}")
            assert vector_norm_err(got, ref) < 1e-13
            dev.step(dt)
            err = normwise(dev.host(dev.q), ref_q)
            print(f"   one RK step: normwise {err}")
            assert np.all(err < 1e-13)
    finally:
        dev.close()


def test_shock_tube_rk_steps():
    """Two mirror-image shock tubes (discontinuous data: WENO-JS weights far from the ideal
    ones, Steger-Warming split near sonic points), Euler, 30 RK3 steps against the oracle,
    normwise after every step."""
    wl = W.double_shock_tube(64)
    c = O.cfg_from_workload(wl)
    met = O.metrics(c, wl.blocks[0].xyz)
    dev = DevBlock(wl, pitched=True)
    try:
        dt = 0.3 / 64
        q = wl.blocks[0].q.copy()
        for s in range(30):
            dev.step(dt)
            q = O.rk_step(c, met, dt, q)
            err = normwise(dev.host(dev.q), q)
            print(s, err)
            assert np.all(err < TOL), (s, err)
    finally:
        dev.close()


def test_argument_and_state_errors():
    import torch
    wl = _vortex(16, 16, 16)
    dev = DevBlock(wl)
    try:
        with pytest.raises(B.CfdError) as e:
            B.cfd_rk_stage(dev.h, 1, 1e-3, dev.q, dev.qa, dev.qa)
        assert e.value.code == B.CFD_ERR_ARG
        with pytest.raises(B.CfdError) as e:
            B.cfd_rk_stage(dev.h, 0, 1e-3, dev.q, dev.qa, dev.qb)
        assert e.value.code == B.CFD_ERR_ARG
        with pytest.raises(B.CfdError) as e:
            B.cfd_rk_stage(dev.h, 1, 1e-3, dev.qa, dev.qb, dev.qa)
        assert e.value.code == B.CFD_ERR_ARG
        bad = dev.q.clone()
        bad[0, 10, 10, 10] = float("nan")
        assert not B.cfd_check_finite(dev.h, bad)
        assert B.cfd_check_finite(dev.h, dev.q)
        fresh = B.cfd_block_create(B.desc_from_workload(wl), torch.cuda.current_stream())
        try:
            with pytest.raises(B.CfdError) as e:
                B.cfd_rhs(fresh, dev.q, dev.r)
            assert e.value.code == B.CFD_ERR_STATE
            folded = wl.blocks[0].xyz.copy()
            folded[0] = -folded[0]  # left-handed mapping: 1/J < 0
            with pytest.raises(B.CfdError) as e:
                B.cfd_metrics(fresh, torch.from_numpy(folded).cuda(), 16 + 12, 16 + 12)
            assert e.value.code == B.CFD_ERR_JACOBIAN
        finally:
            B.cfd_block_destroy(fresh)
    finally:
        dev.close()


def test_full_size_taylor_green_first_stage():
    """256^3 Taylor-Green case at its real size, in the benchmark's pitched layout: the
    first RK stage, every point."""
    wl = W.taylor_green_wavy(256)
    dev, c, met = _pair(wl, pitched=True)
    try:
        q = wl.blocks[0].q
        dt = O.dt_cfl(c, met, q, wl.cfl)
        B.cfd_rk_stage(dev.h, 0, dt, dev.q, dev.q, dev.qa)
        got = dev.host(dev.qa)
        r = O.rhs(c, met, q)
        ref = q + dt * r
        err = normwise(got, ref)
        print("256^3 stage-0 normwise error", err)
        assert np.all(err < TOL)
    finally:
        dev.close()
