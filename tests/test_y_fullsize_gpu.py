"""Parity at the benchmark workloads' real sizes, every interior point of the first RK
stage, in the pitched layout and launch configuration the benchmark uses."""
import numpy as np
import pytest

import oracle as O
from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevBlock, DevMulti, normwise, oracle_multi

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def test_o_grid_24_blocks_first_stage():
    """The 24-block O-grid workload (about 40M points, seeded uneven block sizes)."""
    wl = W.o_grid_vortices()
    print(wl.description, flush=True)
    cfgs, mets, qs = oracle_multi(wl)
    dt = min(O.dt_cfl(c, m, q, wl.cfl) for c, m, q in zip(cfgs, mets, qs))
    rs = O.rhs_multi(cfgs, mets, qs, wl.interfaces)
    del mets
    dev = DevMulti(wl)
    try:
        for h, q in zip(dev.h, dev.q):
            B.cfd_viscous_fluxes(h, q)
        B.cfd_halo_exchange(dev.x, B.CFD_FIELDS_VISC, None)
        for h, q, qa in zip(dev.h, dev.q, dev.qa):
            B.cfd_rk_sweeps(h, 0, dt, q, q, qa)
        worst = 0.0
        for bi in range(len(wl.blocks)):
            got = dev.host(bi, dev.qa[bi])
            ref = qs[bi] + dt * rs[bi]
            worst = max(worst, float(np.max(normwise(got, ref))))
        print("24-block first stage, worst normwise error", worst)
        assert worst < TOL
    finally:
        dev.close()


def test_channel_512x512x384_first_stage():
    """The 512 x 512 x 384 channel with walls (about 100M points)."""
    wl = W.channel()
    c = O.cfg_from_workload(wl)
    q0 = O.bc_fill(c, O.periodic_wrap(c, O.wall_reset(c, wl.blocks[0].q)))
    met = O.metrics(c, wl.blocks[0].xyz)
    dt = O.dt_cfl(c, met, q0, wl.cfl)
    r = O.rhs(c, met, q0)
    del met
    dev = DevBlock(wl, q=q0, pitched=True)
    try:
        B.cfd_rk_stage(dev.h, 0, dt, dev.q, dev.q, dev.qa)
        got = dev.host(dev.qa)
        err = normwise(got, q0 + dt * r)
        print("channel first stage normwise error", err)
        assert np.all(err < TOL)
    finally:
        dev.close()
