"""Multi-block parity on the GPU: interface exchanges, walls, far field, the batched form
(work-list launches + captured HIP graph + autotuned tiles) against the CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevMulti, normwise, oracle_multi, vector_norm_err

pytestmark = pytest.mark.gpu

TOL = 1e-12
SMALL_OGRID = [[24, 16, 32, 16], [16, 24, 16], [16, 8]]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def _periodic_split():
    wl = W.vortex_wavy(24, nj=20, nk=16, amp=0.06)
    return wl, W.split_block(wl, [[10, 14], [9, 11], [7, 9]])


def test_decomposition_invariance_rhs():
    """Eight uneven blocks of a periodic box: per-block RHS equals the single-block oracle."""
    import torch
    single, wl = _periodic_split()
    c = O.cfg_from_workload(single)
    ref = O.rhs(c, O.metrics(c, single.blocks[0].xyz), single.blocks[0].q)
    dev = DevMulti(wl)
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
                    assert err < 1e-10
                    n += 1
    finally:
        dev.close()


def _run_compare(wl, steps, batch=False, precision=B.CFD_FP64, tol=TOL):
    import torch
    cfgs, mets, qs = oracle_multi(wl)
    dt = min(O.dt_cfl(c, m, q, wl.cfl) for c, m, q in zip(cfgs, mets, qs))
    dev = DevMulti(wl, precision=precision)
    errs = []
    try:
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        for s in range(steps):
            if batch:
                dev.batch_step(dt_dev)
            else:
                dev.step(dt)
            qs = O.rk_step_multi(cfgs, mets, dt, qs, wl.interfaces)
            err = max(np.max(normwise(dev.host(bi), qs[bi])) for bi in range(len(qs)))
            errs.append(err)
            print(s, err)
            assert err < tol, (s, err)
        return dev, errs
    except Exception:
        dev.close()
        raise


def test_periodic_split_rk_steps():
    _, wl = _periodic_split()
    dev, _ = _run_compare(wl, 3)
    dev.close()


def test_o_grid_rk_steps_per_block():
    """24 uneven O-grid blocks with a wall, far field and periodic seams: 3 RK3 steps."""
    wl = W.o_grid_vortices(sizes=SMALL_OGRID)
    dev, _ = _run_compare(wl, 3)
    dev.close()


def test_o_grid_batched_graph_matches_oracle_and_per_block():
    """The batched form (one launch per phase over all blocks, HIP graph of the RK step,
    autotuned tiles) against the oracle for 3 steps, and bitwise against per-block launches;
    the graph is replayed several times with eager work in between."""
    import torch
    wl = W.o_grid_vortices(sizes=SMALL_OGRID)
    dev, _ = _run_compare(wl, 3, batch=True)
    ref = DevMulti(wl)
    # the per-block launches use the tile shapes the autotuner chose (the same shape gives
    # the same bits; different shapes agree to round-off)
    cfg, _ = B.cfd_batch_tuning(dev.bt)
    for h in ref.h:
        B.cfd_block_set_tiles(h, cfg)
    try:
        cfgs, mets, qs = oracle_multi(wl)
        dt = min(O.dt_cfl(c, m, q, wl.cfl) for c, m, q in zip(cfgs, mets, qs))
        for _ in range(3):
            ref.step(dt)
        for bi in range(len(wl.blocks)):
            np.testing.assert_array_equal(ref.host(bi), dev.host(bi))
        cfg, per = B.cfd_batch_tuning(dev.bt)
        print("tuned tiles", cfg, per, B.cfd_batch_tuning_times(dev.bt))
        # more replays, each checked against the eager per-block path
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        for _ in range(3):
            dev.batch_step(dt_dev)
            torch.cuda.synchronize()
            ref.step(dt)
            torch.cuda.synchronize()
            for bi in range(len(wl.blocks)):
                np.testing.assert_array_equal(ref.host(bi), dev.host(bi))
    finally:
        ref.close()
        dev.close()


@pytest.mark.parametrize("cfg,persist,precision", [((1, 2, 3), (0, 1, 0), B.CFD_FP64),
                                                   ((3, 0, 1), (1, 0, 1), B.CFD_FP64),
                                                   ((4, 5, 4), (0, 1, 1), B.CFD_FP64),
                                                   ((5, 4, 5), (1, 0, 0), B.CFD_FP64),
                                                   ((5, 2, 2), (0, 0, 0), B.CFD_MIXED),
                                                   ((2, 4, 0), (1, 1, 0), B.CFD_MIXED)])
def test_batched_tilings_agree(cfg, persist, precision):
    """The batched launches with a given tile shape per direction, under both schedules,
    give the same bits as the per-block launches with those shapes (FP64 and mixed)."""
    import torch
    wl = W.o_grid_vortices(sizes=SMALL_OGRID)
    a, b = DevMulti(wl, precision=precision), DevMulti(wl, precision=precision)
    for h in a.h:
        B.cfd_block_set_tiles(h, cfg)
    try:
        cfgs, mets, qs = oracle_multi(wl)
        dt = min(O.dt_cfl(c, m, q, wl.cfl) for c, m, q in zip(cfgs, mets, qs))
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        b.bt = B.cfd_batch_create(b.h, b.x, torch.cuda.current_stream())
        B.cfd_batch_set_tuning(b.bt, cfg, persist)
        for _ in range(2):
            a.step(dt)
            b.batch_step(dt_dev)
        for bi in range(len(wl.blocks)):
            np.testing.assert_array_equal(a.host(bi), b.host(bi))
    finally:
        a.close()
        b.close()


def test_channel_walls_rk_steps():
    """Channel block with isothermal no-slip walls and periodic x, z: 3 RK3 steps."""
    import torch
    from tests._gpu import DevBlock
    wl = W.channel(40, 24, 16)
    c = O.cfg_from_workload(wl)
    met = O.metrics(c, wl.blocks[0].xyz)
    q0 = O.bc_fill(c, O.periodic_wrap(c, O.wall_reset(c, wl.blocks[0].q)))
    dev = DevBlock(wl, q=wl.blocks[0].q, pitched=True)
    try:
        dev.halo(dev.q)
        np.testing.assert_allclose(dev.host(dev.q)[:, 3:-3, :, 3:-3], q0[:, 3:-3, :, 3:-3], rtol=0, atol=1e-15)
        dt = O.dt_cfl(c, met, q0, wl.cfl)
        qo = q0
        for s in range(3):
            dev.step(dt)
            qo = O.rk_step(c, met, dt, qo)
            err = normwise(dev.host(dev.q), qo)
            print(s, err)
            assert np.all(err < TOL)
    finally:
        dev.close()


def _char_far_field(wl):
    """The same workload with its far-field faces switched to the characteristic condition."""
    import dataclasses
    blocks = [dataclasses.replace(b, bc=tuple(W.BC_FARFIELD_CHAR if k == W.BC_FARFIELD else k for k in b.bc))
              for b in wl.blocks]
    return dataclasses.replace(wl, blocks=blocks)


@pytest.mark.parametrize("batch", [False, True])
def test_o_grid_characteristic_far_field(batch):
    """24 uneven O-grid blocks whose outer faces take the characteristic far field (subsonic
    inflow upstream, outflow downstream): 3 RK3 steps against the oracle."""
    wl = _char_far_field(W.o_grid_vortices(sizes=SMALL_OGRID))
    assert any(W.BC_FARFIELD_CHAR in b.bc for b in wl.blocks)
    dev, _ = _run_compare(wl, 3, batch=batch)
    dev.close()
