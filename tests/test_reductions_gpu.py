"""Device reductions of the iteration loop (Fig 2; Sec. 4.5.3): residual norms and the CFL
time step written to device memory, against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevBlock, DevMulti, normwise, oracle_multi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def test_residual_of_the_rhs():
    """RHS residual: the reduction of the GPU's own R against the oracle's norms of the
    same (downloaded) array, and against the oracle's norms of the oracle's R."""
    wl = W.vortex_wavy(32, seed=1)
    dev = DevBlock(wl)
    try:
        r_host = dev.rhs()
        rms, mx = B.cfd_residual([dev.h], [dev.r])
        rms_o, mx_o = O.residual([r_host])
        print("rms", rms, "max", mx)
        assert _rel(rms, rms_o) < 1e-13 and _rel(mx, mx_o) == 0.0
        c = O.cfg_from_workload(wl)
        r_ref = O.rhs(c, O.metrics(c, wl.blocks[0].xyz), wl.blocks[0].q)
        rms_r, mx_r = O.residual([r_ref])
        assert _rel(rms, rms_r) < 1e-10 and _rel(mx, mx_r) < 1e-10
        # bitwise reproducible
        again = B.cfd_residual([dev.h], [dev.r])
        assert again == (rms, mx)
    finally:
        dev.close()


def test_residual_ignores_halos_and_ragged_blocks():
    """Ragged, pitched block with NaN in every halo and padding value."""
    import torch
    wl = W.vortex_wavy(23, nj=17, nk=11, seed=2)
    dev = DevBlock(wl, pitched=True)
    try:
        t = torch.full_like(dev.q, float("nan"))
        d = dev.desc
        t[:, 3:-3, 3:3 + d.nj, 3:3 + d.ni] = dev.q[:, 3:-3, 3:3 + d.nj, 3:3 + d.ni]
        rms, mx = B.cfd_residual([dev.h], [t], None, 2.0)
        rms_o, mx_o = O.residual([wl.blocks[0].q], None, 2.0)
        assert _rel(rms, rms_o) < 1e-13 and _rel(mx, mx_o) == 0.0
    finally:
        dev.close()


def test_step_residual_over_blocks():
    """(Q^{n+1} - Q^n)/dt over eight uneven blocks, against the oracle's norms of the same
    arrays and of the oracle's own step."""
    import torch
    single = W.vortex_wavy(24, nj=20, nk=16, amp=0.06)
    wl = W.split_block(single, [[10, 14], [9, 11], [7, 9]])
    dev = DevMulti(wl)
    try:
        q0 = [q.clone() for q in dev.q]
        dt = 1e-3
        dev.step(dt)
        torch.cuda.synchronize()
        rms, mx = B.cfd_residual(dev.h, dev.q, q0, 1.0 / dt)
        h1 = [dev.host(b) for b in range(len(wl.blocks))]
        h0 = [B.download_state(dev.descs[b], q0[b]) for b in range(len(wl.blocks))]
        rms_o, mx_o = O.residual(h1, h0, 1.0 / dt)
        print("step residual rms", rms, "max", mx)
        assert _rel(rms, rms_o) < 1e-12 and _rel(mx, mx_o) < 1e-12
        cfgs, mets, qs = oracle_multi(wl)
        qo = O.rk_step_multi(cfgs, mets, dt, qs, wl.interfaces)
        rms_r, mx_r = O.residual(qo, qs, 1.0 / dt)
        assert _rel(rms, rms_r) < 1e-9 and _rel(mx, mx_r) < 1e-9
    finally:
        dev.close()


def test_dt_on_device_matches_host_dt():
    import torch
    single = W.vortex_wavy(24, nj=20, nk=16, amp=0.06)
    wl = W.split_block(single, [[10, 14], [9, 11], [7, 9]])
    dev = DevMulti(wl)
    try:
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        B.cfd_dt_cfl_dev(dev.h, dev.q, 0.5, dt_dev)
        dt_host = B.cfd_dt_cfl(dev.h, dev.q, 0.5)
        assert float(dt_dev.item()) == dt_host
        c = O.cfg_from_workload(single)
        dt_o = O.dt_cfl(c, O.metrics(c, single.blocks[0].xyz), single.blocks[0].q, 0.5)
        assert abs(dt_host - dt_o) <= 1e-14 * dt_o
        with pytest.raises(B.CfdError):
            B.cfd_dt_cfl_dev(dev.h, dev.q, 0.0, dt_dev)
    finally:
        dev.close()


def test_time_loop_with_device_dt_and_batched_steps():
    """Three iterations of: dt from the current state on the device, one batched RK step
    with that dt, the step residual; against the oracle doing the same on the host."""
    import torch
    single = W.vortex_wavy(24, nj=20, nk=16, amp=0.06)
    wl = W.split_block(single, [[10, 14], [9, 11], [7, 9]])
    dev = DevMulti(wl)
    try:
        cfgs, mets, qs = oracle_multi(wl)
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        for it in range(3):
            B.cfd_dt_cfl_dev(dev.h, dev.q, 0.5, dt_dev)
            dev.batch_step(dt_dev)
            torch.cuda.synchronize()
            dt_o = min(O.dt_cfl(c, m, q, 0.5) for c, m, q in zip(cfgs, mets, qs))
            assert abs(float(dt_dev.item()) - dt_o) <= 1e-13 * dt_o
            q_prev = qs
            qs = O.rk_step_multi(cfgs, mets, dt_o, qs, wl.interfaces)
            for b in range(len(wl.blocks)):
                err = normwise(dev.host(b), qs[b])
                assert np.all(err < 1e-12), (it, b, err)
            print(it, float(dt_dev.item()), O.residual(qs, q_prev, 1.0 / dt_o)[0])
    finally:
        dev.close()


def test_residual_argument_errors():
    wl = W.vortex_wavy(16, seed=1)
    dev = DevBlock(wl)
    try:
        with pytest.raises(B.CfdError):
            B.cfd_residual([dev.h], [dev.q], None, float("inf"))
    finally:
        dev.close()


def _dt_plane(desc):
    return B.state_tensor(desc, 1)


def test_local_time_steps_match_the_oracle():
    """Per-point CFL steps and three RK steps with them (a steady-state iteration), against
    the oracle's local steps and its RK step with a step per point."""
    wl = W.vortex_wavy(24, nj=20, nk=16, seed=1)
    dev = DevBlock(wl, pitched=True)
    try:
        c = O.cfg_from_workload(wl)
        met = O.metrics(c, wl.blocks[0].xyz)
        dtf = _dt_plane(dev.desc)
        B.cfd_dt_local([dev.h], [dev.q], 0.5, [dtf])
        got = B.download_state(dev.desc, dtf)[0, 3:-3, 3:-3, 3:-3]
        ref_f = O.dt_local(c, met, wl.blocks[0].q, 0.5)
        assert _rel(got, ref_f[0, 3:-3, 3:-3, 3:-3]) < 1e-14
        B.cfd_block_set_local_dt(dev.h, dtf)
        q = wl.blocks[0].q
        for step in range(3):
            dev.step(123.0)  # the scalar step is ignored while a step field is set
            q = O.rk_step_local(c, met, ref_f, q)
            err = normwise(dev.host(dev.q), q)
            print(step, err)
            assert np.all(err < 1e-12), (step, err)
    finally:
        dev.close()


def test_constant_step_field_equals_the_scalar_step():
    import torch
    wl = W.vortex_wavy(20, nj=16, nk=12, seed=2)
    a = DevBlock(wl)
    b = DevBlock(wl)
    try:
        dt = 2e-3
        dtf = _dt_plane(b.desc)
        dtf.fill_(dt)
        B.cfd_block_set_local_dt(b.h, dtf)
        a.step(dt)
        b.step(0.0)
        assert torch.equal(a.q, b.q)
        B.cfd_block_set_local_dt(b.h, None)  # back to the scalar step
        a.step(dt)
        b.step(dt)
        assert torch.equal(a.q, b.q)
    finally:
        a.close()
        b.close()


def test_batched_steps_with_local_time_steps():
    """Eight uneven blocks, steps per point set on every block: the batched graph follows
    the per-block launches (which follow the oracle above)."""
    import torch
    single = W.vortex_wavy(24, nj=20, nk=16, amp=0.06)
    wl = W.split_block(single, [[10, 14], [9, 11], [7, 9]])
    per = DevMulti(wl)
    bat = DevMulti(wl)
    try:
        fields = []
        for dev in (per, bat):
            f = [_dt_plane(d) for d in dev.descs]
            B.cfd_dt_local(dev.h, dev.q, 0.5, f)
            for h, t in zip(dev.h, f):
                B.cfd_block_set_local_dt(h, t)
            fields.append(f)
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")  # ignored
        for step in range(2):
            per.step(0.0)
            bat.batch_step(dt_dev)
            torch.cuda.synchronize()
            for b in range(len(wl.blocks)):
                err = normwise(bat.host(b), per.host(b))
                assert np.all(err < 1e-13), (step, b, err)
    finally:
        per.close()
        bat.close()
