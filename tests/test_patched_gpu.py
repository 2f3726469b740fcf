"""Patched block connections on the GPU (cfd_exchange_create_patched): blocks whose faces
meet several blocks, and faces that are part wall and part connection (Sec. 3), against
the oracle's patched multi-block RK steps."""
import dataclasses

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


def _run(wl, steps, batch=False, precision=B.CFD_FP64, tol=TOL):
    import torch
    cfgs, mets, qs = oracle_multi(wl)
    dt = min(O.dt_cfl(c, m, q, wl.cfl) for c, m, q in zip(cfgs, mets, qs))
    dev = DevMulti(wl, precision=precision)
    try:
        # the ghost fill's divisions may round differently (a few ulp of the state's scale)
        init = max(np.max(np.abs(dev.host(bi) - qs[bi])) / np.max(np.abs(qs[bi])) for bi in range(len(qs)))
        print("initial halo fill, largest difference relative to the state", init)
        assert init <= 8 * np.finfo(np.float64).eps
        dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
        for s in range(steps):
            if batch:
                dev.batch_step(dt_dev)
            else:
                dev.step(dt)
            qs = O.rk_step_patched(cfgs, mets, dt, qs, wl.patches)
            err = max(np.max(normwise(dev.host(bi), qs[bi])) for bi in range(len(qs)))
            print(s, err)
            assert err < tol, (s, err)
        return [dev.host(bi) for bi in range(len(qs))]
    finally:
        dev.close()


def test_patched_box_per_block():
    """Four blocks of the periodic vortex box whose faces meet up to three others:
    3 RK3 steps with per-block launches."""
    _run(W.patched_vortex(32), 3)


def test_patched_box_batched():
    """The batched form (one launch per phase over all blocks, the RK step in a HIP graph,
    autotuned tiles) on the same blocks: 3 RK3 steps against the oracle."""
    _run(W.patched_vortex(32), 3, batch=True)


def test_periodic_step_per_block_and_batched():
    """The periodic backward-facing step (a wall face that is part step face, part
    connection; the step's top and back): 3 RK3 steps per block and batched."""
    wl = W.periodic_step()
    _run(wl, 3)
    _run(wl, 3, batch=True)


def test_wall_face_with_a_connected_slot():
    """A 12-node tall slot [0, 20) x [10, 22) in front of the block [20, 48) x all of the
    48 x 32 x 16 channel: that block's i faces are wall below and above the slot and
    connected in between (their uncovered parts are two rectangles each), the slot's
    j faces are walls.  3 RK3 steps per block and batched."""
    wl = W.split_boxes(W.channel(48, 32, 16, mach=0.3, reynolds=1000.0), [(0, 20, 10, 22, 0, 16), (20, 48, 0, 32, 0, 16)],
                       "channel_slot_48x32x16")
    assert wl.blocks[1].bc[:2] == (B.CFD_BC_WALL, B.CFD_BC_WALL) and wl.blocks[0].bc[2:4] == (B.CFD_BC_WALL,) * 2
    _run(wl, 3)
    _run(wl, 3, batch=True)


def test_periodic_step_mixed_batched():
    """Mixed precision, batched: normwise within 1e-5 of the FP64 oracle after 3 steps."""
    _run(W.periodic_step(), 3, batch=True, precision=B.CFD_MIXED, tol=1e-5)


def test_patched_exchange_errors():
    import torch
    wl = W.patched_vortex(32)
    dev = DevMulti(wl)
    try:
        p0 = wl.patches[0]
        cases = [(wl.patches + [p0], B.CFD_ERR_ARG),                                    # covered twice
                 (wl.patches[1:], B.CFD_ERR_ARG),                                       # interface face open
                 ([dataclasses.replace(p0, a_lo=(0, 1))] + wl.patches[1:], B.CFD_ERR_ARG),  # outside the face
                 ([W.Patch(1, 3, (0, 0), (13, 32), 0, 2, (0, 0))] + wl.patches, B.CFD_ERR_ARG),  # periodic face
                 ([dataclasses.replace(p0, orient=8)] + wl.patches[1:], B.CFD_ERR_ARG),
                 ([dataclasses.replace(p0, orient=2)] + wl.patches[1:], B.CFD_ERR_ARG),     # handedness
                 ([dataclasses.replace(p0, block_b=7)] + wl.patches[1:], B.CFD_ERR_ARG)]
        for ps, code in cases:
            with pytest.raises(B.CfdError) as e:
                B.cfd_exchange_create_patched(dev.h, ps)
            assert e.value.code == code
    finally:
        dev.close()
    # a partly connected wall face needs the split form; the one-sided closure refuses it
    step = W.periodic_step()
    dev = DevMulti(step)
    try:
        q = dev.q[1]
        with pytest.raises(B.CfdError) as e:
            B.cfd_rk_stage(dev.h[1], 0, 1e-4, q, q, dev.qa[1])
        assert e.value.code == B.CFD_ERR_STATE
    finally:
        dev.close()
    os_step = dataclasses.replace(step, visc_closure=B.CFD_VISC_ONE_SIDED)
    with pytest.raises(B.CfdError) as e:
        DevMulti(os_step)
    assert e.value.code == B.CFD_ERR_UNSUPPORTED
