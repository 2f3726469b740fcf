"""Blocks joined through oriented interfaces (tangential indices swapped or reversed,
faces on different axes) on the GPU against the oracle: the exchange plan's copies map
the state and the face-normal viscous fluxes (with their sign) like the oracle does."""
import numpy as np
import pytest

import oracle as O
from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevMulti, normwise, oracle_multi

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def _rotated(about):
    single = W.vortex_wavy(20, nj=14, nk=12, amp=0.06)
    return single, W.rotated_split(single, 9, about)


@pytest.mark.parametrize("about", ["i", "k"])
@pytest.mark.parametrize("batched", [False, True])
def test_rotated_blocks_rk_steps(about, batched):
    import torch
    _, wl = _rotated(about)
    dev = DevMulti(wl)
    try:
        cfgs, mets, qs = oracle_multi(wl)
        dt = 0.4 * min(O.dt_cfl(c, m, q, 1.0) for c, m, q in zip(cfgs, mets, qs))
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        for step in range(3):
            if batched:
                dev.batch_step(dt_dev)
            else:
                dev.step(dt)
            qs = O.rk_step_multi(cfgs, mets, dt, qs, wl.interfaces)
            for b in range(2):
                err = normwise(dev.host(b), qs[b])
                print(about, batched, step, b, err)
                assert np.all(err < TOL), (step, b, err)
    finally:
        dev.close()


def test_rotated_blocks_mixed_precision():
    _, wl = _rotated("k")
    dev = DevMulti(wl, precision=B.CFD_MIXED)
    try:
        cfgs, mets, qs = oracle_multi(wl)
        dt = 0.4 * min(O.dt_cfl(c, m, q, 1.0) for c, m, q in zip(cfgs, mets, qs))
        dev.step(dt)
        qs = O.rk_step_multi(cfgs, mets, dt, qs, wl.interfaces)
        for b in range(2):
            err = normwise(dev.host(b), qs[b])
            print(b, err)
            assert np.all(err < 1e-6)
    finally:
        dev.close()


def test_oriented_interface_errors():
    _, wl = _rotated("k")
    dev = DevMulti(wl)
    try:
        bad_orient = [W.Interface(0, 1, 1, 3, 8), W.Interface(0, 0, 1, 2, 0)]
        # reversing one tangential index of this pair would turn one block inside out
        mirrored = [W.Interface(0, 1, 1, 3, 2), W.Interface(0, 0, 1, 2, 2)]
        for ifc in (bad_orient, mirrored):
            with pytest.raises(B.CfdError) as e:
                B.cfd_exchange_create(dev.h, ifc)
            assert e.value.code == B.CFD_ERR_ARG
            print(B.cfd_last_error())
    finally:
        dev.close()
