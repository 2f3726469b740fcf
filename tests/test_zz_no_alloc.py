"""cfd_residual_noalloc (the residual norms through the library's fixed device scratch,
for callers that cannot allocate) against cfd_residual, the allocating entry point with
the same kernels: bitwise equal results on two calls in a row, the second one on a smaller
input, and the block-count limit of the fixed scratch."""
import numpy as np
import pytest

from paper_2006_07964_amd import binding as B
from paper_2006_07964_amd import workloads as W
from tests._gpu import DevBlock

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def test_residual_noalloc_matches_the_allocating_entry_point():
    import torch
    big = [DevBlock(W.vortex_wavy(40, nj=36, nk=30, seed=s)) for s in (1, 2)]
    small = DevBlock(W.vortex_wavy(12, nj=9, nk=8, seed=3))
    try:
        # first call: two blocks, the step residual form (A - B) / dt
        for d in big:
            d.qa.copy_(d.q * 1.001 + 0.25)
        torch.cuda.synchronize()
        hs = [d.h for d in big]
        a = [d.qa for d in big]
        b = [d.q for d in big]
        ref = B.cfd_residual(hs, a, b, 1.0 / 3e-3)
        got = B.cfd_residual_noalloc(hs, a, b, 1.0 / 3e-3)
        print("two blocks:", got)
        assert got == ref  # same kernels, same fixed summation order: bitwise
        assert all(np.isfinite(got[0])) and max(got[1]) > 0
        # second call: one smaller block, the plain norm of one array (B absent), so the
        # scratch still holds the first call's larger partial rows
        small.qa.copy_(small.q * -2.0)
        torch.cuda.synchronize()
        ref2 = B.cfd_residual([small.h], [small.qa])
        got2 = B.cfd_residual_noalloc([small.h], [small.qa])
        print("one small block:", got2)
        assert got2 == ref2
        assert got2 != got
        # the fixed scratch holds the rows of at most 64 blocks
        with pytest.raises(B.CfdError) as e:
            B.cfd_residual_noalloc([small.h] * 65, [small.qa] * 65)
        assert e.value.code == B.CFD_ERR_ARG
    finally:
        for d in big + [small]:
            d.close()
