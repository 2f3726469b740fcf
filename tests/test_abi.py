"""CPU-side checks of the C ABI: the library loads, exports every declared entry point,
the Python structures match the C layout, and argument errors are reported without a GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2006_07964_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libcfd.so is not built (run python -m paper_2006_07964_amd.build)")
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_function():
    names = declared_functions()
    missing = [n for n in names if not hasattr(B, n)]
    assert not missing, missing


def test_struct_layout_matches_header():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "cfd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(cfd_params), sizeof(cfd_block_desc), sizeof(cfd_interface),
         offsetof(cfd_block_desc, ld_i), offsetof(cfd_block_desc, precision), offsetof(cfd_block_desc, params),
         offsetof(cfd_params, qinf));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    py = [C.sizeof(B.cfd_params), C.sizeof(B.cfd_block_desc), C.sizeof(B.cfd_interface),
          B.cfd_block_desc.ld_i.offset, B.cfd_block_desc.precision.offset, B.cfd_block_desc.params.offset,
          B.cfd_params.qinf.offset]
    assert vals == py


def test_argument_errors_without_gpu(lib):
    # WENO epsilon floors of Eq 15's common-denominator form: below 1e-8 in mixed
    # precision (eps^4 leaves the normal FP32 range), below 1e-30 in FP64 (eps^8 leaves it)
    for bad in (dict(ni=5), dict(ld_i=10), dict(precision=7), dict(weights=3), dict(gamma=1.0),
                dict(bc=(0, 2, 0, 0, 0, 0)), dict(scheme=2), dict(visc_closure=2), dict(visc_closure=-1),
                dict(weno_eps=1e-12, precision=B.CFD_MIXED), dict(weno_eps=9.9e-9, precision=B.CFD_MIXED),
                dict(weno_eps=1e-40), dict(weno_eps=9.9e-31)):
        kw = dict(ni=16, nj=16, nk=16)
        kw.update(bad)
        ni = kw.pop("ni")
        nj = kw.pop("nj")
        nk = kw.pop("nk")
        desc = B.make_desc(ni, nj, nk, **kw)
        with pytest.raises(B.CfdError) as e:
            B.cfd_block_create(desc)
        assert e.value.code == B.CFD_ERR_ARG
        assert B.cfd_last_error()
    # one plane of a block (pitched rows x columns x (nk + 6)) must stay below 2^29 points:
    # pitches 1024 x 1024 with nk = 506 give exactly 2^29 and are refused before any allocation
    desc = B.make_desc(1018, 1018, 506, ld_i=1024, ld_j=1024)
    with pytest.raises(B.CfdError) as e:
        B.cfd_block_create(desc)
    assert e.value.code == B.CFD_ERR_UNSUPPORTED
    for call in (lambda: B.cfd_residual([], []), lambda: B.cfd_dt_cfl_dev([], [], 0.5, None)):
        with pytest.raises(B.CfdError) as e:
            call()
        assert e.value.code == B.CFD_ERR_ARG
    with pytest.raises(B.CfdError) as e:
        B.cfd_exchange_create([], [])
    assert e.value.code == B.CFD_ERR_ARG
    with pytest.raises(B.CfdError):
        B.cfd_dt_cfl([], [], 0.5)


def test_oracle_exports():
    import oracle as O
    L = O.lib()
    for n in ("oracle_metrics", "oracle_rhs", "oracle_rk_stage", "oracle_rk_step", "oracle_dt_cfl",
              "oracle_exchange", "oracle_rhs_multi", "oracle_rk_step_multi", "oracle_wall_reset", "oracle_bc_fill"):
        assert hasattr(L, n), n


def test_tile_configurations(lib):
    n = B.cfd_tile_config_count()
    assert n >= 4
    for cfg in range(n):
        lines, nodes, threads = B.cfd_tile_config(cfg)
        assert lines >= 1 and nodes >= 6 and threads % 64 == 0
        # the items of one tile fill the workgroup at most a few times over
        assert lines * (nodes + 6) <= 4 * threads
    for bad in (-1, n):
        with pytest.raises(B.CfdError):
            B.cfd_tile_config(bad)


def test_sweep_order_and_null_handles(lib):
    order = B.cfd_sweep_order()
    assert sorted(order) == [0, 1, 2]
    assert lib.cfd_sweep_order(None) == B.CFD_ERR_ARG
    cfg = (C.c_int * 3)(0, 0, 0)
    assert lib.cfd_block_set_tiles(None, cfg) == B.CFD_ERR_ARG
    assert lib.cfd_block_tiles(None, cfg) == B.CFD_ERR_ARG
    ms = (C.c_float * 64)()
    assert lib.cfd_batch_tuning_times(None, ms, 64) == B.CFD_ERR_ARG
