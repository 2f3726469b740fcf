"""The original AFWENO scheme (characteristic space at the half points, two WENO
interpolations per half point, Sec. 4.5.1, Fig 9) on the GPU against the oracle's
original-scheme operator, with the same bars as the modified scheme: states after every
RK step within normwise 1e-12, right-hand sides within 1e-10 (WENO-JS weights) or 1e-12
(ideal weights) over the whole vector."""
import numpy as np
import pytest

import oracle as O
from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevBlock, DevMulti, normwise, vector_norm_err

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_RHS_JS = 1e-10
TOL_RHS_LIN = 1e-12
ORIG = dict(scheme=B.CFD_AFWENO_ORIGINAL)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def _pair(wl, pitched=False, linear=False, viscous=None, precision=B.CFD_FP64):
    viscous = wl.viscous if viscous is None else viscous
    weights = B.CFD_WENO_LINEAR if linear else B.CFD_WENO_JS
    dev = DevBlock(wl, precision=precision, pitched=pitched, weights=weights, viscous=viscous, **ORIG)
    c = O.cfg_from_workload(wl, linear_weights=linear, viscous=viscous, scheme=O.AFWENO_ORIGINAL)
    met = O.metrics(c, wl.blocks[0].xyz)
    return dev, c, met


@pytest.mark.parametrize("size", [(32, 32, 32), (23, 17, 11), (7, 9, 8), (40, 7, 19)])
@pytest.mark.parametrize("mask", [B.CFD_DIR_XI | B.CFD_TERM_INV, B.CFD_DIR_ETA | B.CFD_TERM_INV,
                                  B.CFD_DIR_ZETA | B.CFD_TERM_INV, B.CFD_ALL])
def test_original_rhs(size, mask):
    wl = W.vortex_wavy(size[0], nj=size[1], nk=size[2], seed=1)
    dev, c, met = _pair(wl)
    try:
        got = dev.rhs(mask)
        ref = O.rhs(c, met, wl.blocks[0].q, mask)
        err = vector_norm_err(got, ref)
        print(size, mask, err, normwise(got, ref))
        assert err < TOL_RHS_JS
    finally:
        dev.close()


def test_original_rhs_ideal_weights_equals_modified():
    """With ideal weights the two schemes are the same operator (the projection cancels):
    the GPU's original scheme matches the oracle and the GPU's modified scheme."""
    wl = W.vortex_wavy(24, nj=20, nk=16, seed=3)
    dev, c, met = _pair(wl, linear=True, viscous=False)
    mod = DevBlock(wl, weights=B.CFD_WENO_LINEAR, viscous=False)
    try:
        got = dev.rhs()
        ref = O.rhs(c, met, wl.blocks[0].q)
        other = mod.rhs()
        e1, e2 = vector_norm_err(got, ref), vector_norm_err(got, other)
        print("ideal weights: original vs oracle", e1, "vs modified", e2)
        assert e1 < TOL_RHS_LIN and e2 < TOL_RHS_LIN
    finally:
        dev.close()
        mod.close()


def test_original_rk_ten_steps_c1():
    wl = W.vortex_wavy(32, seed=1)
    dev, c, met = _pair(wl)
    try:
        q = wl.blocks[0].q
        dt = O.dt_cfl(c, met, q, wl.cfl)
        qo = q.copy()
        for step in range(10):
            dev.step(dt)
            qo = O.rk_step(c, met, dt, qo)
            err = normwise(dev.host(dev.q), qo)
            print(step, err)
            assert np.all(err < TOL), (step, err)
    finally:
        dev.close()


def test_original_shock_tube_rk_steps():
    wl = W.double_shock_tube(64)
    dev, c, met = _pair(wl, pitched=True)
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


def test_original_every_tile_shape_agrees():
    """Ragged block, every sweep tile shape against the oracle (one RK step)."""
    wl = W.vortex_wavy(37, nj=29, nk=23, seed=1)
    dev, c, met = _pair(wl, pitched=True)
    try:
        q0 = dev.q.clone()
        dt = 1e-3
        ref = O.rk_step(c, met, dt, wl.blocks[0].q)
        for cfg in range(B.cfd_tile_config_count()):
            B.cfd_block_set_tiles(dev.h, [cfg, cfg, cfg])
            dev.q.copy_(q0)
            dev.step(dt)
            err = normwise(dev.host(dev.q), ref)
            print(cfg, B.cfd_tile_config(cfg), err)
            assert np.all(err < TOL), (cfg, err)
    finally:
        dev.close()


def test_original_mixed_close_to_oracle():
    wl = W.vortex_wavy(32)
    dev, c, met = _pair(wl, precision=B.CFD_MIXED)
    try:
        got = dev.rhs()
        ref = O.rhs(c, met, wl.blocks[0].q)
        err = vector_norm_err(got, ref)
        print("mixed original RHS vector error", err)
        assert err < 1e-4
    finally:
        dev.close()


def _periodic_split():
    wl = W.vortex_wavy(24, nj=20, nk=16, amp=0.06)
    return wl, W.split_block(wl, [[10, 14], [9, 11], [7, 9]])


def test_original_decomposition_invariance_rhs():
    """Eight uneven blocks of a periodic box with the original scheme: per-block RHS
    (after the viscous-flux exchange) equals the single-block oracle."""
    single, wl = _periodic_split()
    c = O.cfg_from_workload(single, scheme=O.AFWENO_ORIGINAL)
    ref = O.rhs(c, O.metrics(c, single.blocks[0].xyz), single.blocks[0].q)
    dev = DevMulti(wl, **ORIG)
    try:
        for h, q in zip(dev.h, dev.q):
            B.cfd_viscous_fluxes(h, q)
        B.cfd_halo_exchange(dev.x, B.CFD_FIELDS_VISC, None)
        offs = [np.concatenate([[0], np.cumsum(s)]) for s in ([10, 14], [9, 11], [7, 9])]
        n = 0
        for kk in range(2):
            for jj in range(2):
                for ii in range(2):
                    r = B.state_tensor(dev.descs[n])
                    B.cfd_rhs_sweeps(dev.h[n], dev.q[n], r)
                    got = B.download_state(dev.descs[n], r)
                    b = wl.blocks[n]
                    i0, j0, k0 = offs[0][ii], offs[1][jj], offs[2][kk]
                    refb = ref[:, k0:k0 + b.nk + 6, j0:j0 + b.nj + 6, i0:i0 + b.ni + 6]
                    err = vector_norm_err(got, refb)
                    print(n, err)
                    assert err < TOL_RHS_JS
                    n += 1
    finally:
        dev.close()


@pytest.mark.parametrize("precision", [B.CFD_FP64, B.CFD_MIXED])
def test_batched_original_scheme_matches_oracle(precision):
    """The batched graph with the original scheme on eight uneven blocks: three RK steps
    against the oracle (FP64 to 1e-12; mixed within single-precision error), and the
    persistent schedule, which it does not have, is refused."""
    import torch
    single, wl = _periodic_split()
    dev = DevMulti(wl, precision=precision, **ORIG)
    try:
        cfgs, mets, qs = oracle_multi_orig(wl)
        dt = min(O.dt_cfl(c, m, q, 0.5) for c, m, q in zip(cfgs, mets, qs))
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        tol = TOL if precision == B.CFD_FP64 else 1e-6
        for step in range(3):
            dev.batch_step(dt_dev)
            qs = O.rk_step_multi(cfgs, mets, dt, qs, wl.interfaces)
            err = max(np.max(normwise(dev.host(b), qs[b])) for b in range(len(qs)))
            print(step, err)
            assert err < tol, (step, err)
        cfg, persist = B.cfd_batch_tuning(dev.bt)
        assert not any(persist)
        with pytest.raises(B.CfdError) as e:
            B.cfd_batch_set_tuning(dev.bt, cfg, [1, 0, 0])
        assert e.value.code == B.CFD_ERR_UNSUPPORTED
    finally:
        dev.close()


def oracle_multi_orig(wl):
    from tests._gpu import oracle_multi
    cfgs, mets, qs = oracle_multi(wl)
    for c in cfgs:
        c.scheme = O.AFWENO_ORIGINAL
    return cfgs, mets, qs


def test_original_and_modified_vortex_accuracy():
    """The noise-free vortex (Euler) advected one period on the 32^3 and 64^3 wavy grids
    with each scheme: both converge (L2 of rho against the exact solution falls by at least
    4x per refinement) and the original's errors are within a factor 2 of the modified's,
    so the cheaper modified scheme costs no accuracy here."""
    res = {}
    for n in (32, 64):
        wl = W.vortex_wavy(n, seed=None, viscous=False)
        q0 = wl.blocks[0].q
        for scheme in (B.CFD_AFWENO_MODIFIED, B.CFD_AFWENO_ORIGINAL):
            dev = DevBlock(wl, viscous=False, scheme=scheme)
            try:
                dt0 = B.cfd_dt_cfl([dev.h], [dev.q], 0.5)
                steps = int(np.ceil(2.0 / dt0))
                for _ in range(steps):
                    dev.step(2.0 / steps)
                e = (dev.host(dev.q) - q0)[0, 3:-3, 3:-3, 3:-3]
                res[(n, scheme)] = float(np.sqrt(np.mean(e * e)))
            finally:
                dev.close()
        print(n, "L2 rho modified", res[(n, 0)], "original", res[(n, 1)], flush=True)
    for s in (0, 1):
        assert res[(32, s)] > 4 * res[(64, s)]
    for n in (32, 64):
        assert 0.5 < res[(n, 1)] / res[(n, 0)] < 2.0
