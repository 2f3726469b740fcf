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


@pytest.mark.parametrize("orient", range(8))
def test_oriented_patches_match_the_oracle(orient):
    """Block A's i+ face (9 x 11 nodes along j, k) against block B's k- face under each
    tangential orientation, the faces joined by four patches of a 2 x 2 cut: the GPU's halo
    refill (copies and far-field ghosts) equals the oracle's on random states.  The partner
    rectangles follow from the orientation's definition; orientations that reverse the
    handedness are refused."""
    import torch
    from tests.test_patched_oracle import _two_blocks
    rng = np.random.default_rng(orient)
    ca, cb, qa, qb, (n1, n2) = _two_blocks(orient, rng)
    cuts1, cuts2 = (0, 4, n1), (0, 6, n2)
    patches = []
    for x in range(2):
        for y in range(2):
            lo = (cuts1[x], cuts2[y])
            n = (cuts1[x + 1] - cuts1[x], cuts2[y + 1] - cuts2[y])
            N = (n1, n2)
            rng_b = [(N[q] - lo[q] - n[q]) if (orient >> (1 + q)) & 1 else lo[q] for q in range(2)]
            b_lo = (rng_b[1], rng_b[0]) if orient & 1 else (rng_b[0], rng_b[1])
            patches.append(W.Patch(0, 1, lo, n, 1, 4, b_lo, orient))
    s = torch.cuda.current_stream()
    descs = [B.make_desc(c.ni, c.nj, c.nk, bc=tuple(c.bc), viscous=False) for c in (ca, cb)]
    hs = [B.cfd_block_create(d, s) for d in descs]
    try:
        try:
            x = B.cfd_exchange_create_patched(hs, patches)
        except B.CfdError as e:
            # a map that reverses handedness: the oracle (which does not check it) is not consulted
            assert e.code == B.CFD_ERR_ARG and "handedness" in str(e)
            return
        try:
            bufs = [B.upload_state(d, q) for d, q in zip(descs, (qa, qb))]
            B.cfd_halo_exchange(x, B.CFD_FIELDS_Q, bufs)
            got = [B.download_state(d, t) for d, t in zip(descs, bufs)]
        finally:
            B.cfd_exchange_destroy(x)
        ref = O.halo_patched([ca, cb], None, [qa, qb], patches)
        for g_, r_ in zip(got, ref):
            np.testing.assert_array_equal(g_[:, 3:-3, 3:-3, 3:-3], r_[:, 3:-3, 3:-3, 3:-3])
        np.testing.assert_array_equal(got[0][:, 3:-3, 3:-3, -3:], ref[0][:, 3:-3, 3:-3, -3:])
        np.testing.assert_array_equal(got[1][:, :3, 3:-3, 3:-3], ref[1][:, :3, 3:-3, 3:-3])
        # the far-field faces' ghosts
        np.testing.assert_array_equal(got[0][:, 3:-3, 3:-3, :3], ref[0][:, 3:-3, 3:-3, :3])
        np.testing.assert_array_equal(got[1][:, -3:, 3:-3, 3:-3], ref[1][:, -3:, 3:-3, 3:-3])
    finally:
        for h in hs:
            B.cfd_block_destroy(h)
