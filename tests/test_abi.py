"""The C-ABI library loads on a host without a GPU and exports every entry
point declared in include/nvdb.h; argument checks that precede any device
work return their documented status codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "nvdb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nvdb_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def nvdb():
    lib = os.path.join(ROOT, "paper_2208_04448_amd", "libnvdb.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2208_04448_amd import nvdb as m
    return m


def test_exports_every_declared_symbol(nvdb):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(nvdb._lib, n), n
    assert set(names) == set(nvdb.EXPORTED)


def test_version_and_error_string(nvdb):
    assert nvdb._lib.nvdb_abi_version() == 2
    d = nvdb.ModelDesc()
    d.precision = 9
    h = C.c_void_p()
    assert nvdb._lib.nvdb_model_create(C.byref(d), C.byref(h)) == nvdb.E_INVALID
    assert b"precision" in nvdb._lib.nvdb_last_error()


@pytest.mark.parametrize("field,value,code", [
    ("domain_size", 0, -1), ("value_scale", 0.0, -1), ("width", 96, -6), ("n_freq", 65, -6), ("hidden", 7, -6)])
def test_model_desc_validation(nvdb, field, value, code):
    d = nvdb.ModelDesc()
    d.precision = nvdb.BF16
    d.has_net[0] = 1
    d.net[0] = nvdb.NetDesc(128, 4, 64, 1)
    d.domain_size, d.value_scale = 64, 3.0
    if field in ("domain_size", "value_scale"):
        setattr(d, field, value)
    else:
        setattr(d.net[0], field, value)
    h = C.c_void_p()
    assert nvdb._lib.nvdb_model_create(C.byref(d), C.byref(h)) == code
    assert h.value is None


def test_null_arguments(nvdb):
    assert nvdb._lib.nvdb_tree_build_dense(None, None, None, None, None, None) == nvdb.E_INVALID
    assert nvdb._lib.nvdb_tree_get_info(None, None) == nvdb.E_INVALID
    assert nvdb._lib.nvdb_fit(None, None, None, None, None) == nvdb.E_INVALID
    assert nvdb._lib.nvdb_sample_indices_dev(0, 0, 0, 0, 1, None, None) == nvdb.E_INVALID
    rule = nvdb.ActiveRule(5, 1.0)
    dims = (C.c_int32 * 3)(4, 4, 4)
    org = (C.c_int32 * 3)(0, 0, 0)
    h = C.c_void_p()
    assert nvdb._lib.nvdb_tree_build_dense(C.c_void_p(16), dims, org, C.byref(rule), None, C.byref(h)) == nvdb.E_INVALID
    dims = (C.c_int32 * 3)(0, 4, 4)
    rule = nvdb.ActiveRule(0, 1.0)
    assert nvdb._lib.nvdb_tree_build_dense(C.c_void_p(16), dims, org, C.byref(rule), None, C.byref(h)) == nvdb.E_INVALID


def test_subdomain_box_host_call(nvdb):
    """The expert's normalisation box comes from the library (host arithmetic, no GPU):
    the widened box of the oracle's decomposition, edge size + 2 halo."""
    from oracle import moe
    for origin, size, halo, cell in (((0, 0, 0), 256, 8, (1, 0, 1)), ((-40, 7, 1000), 64, 8, (-3, 2, 0)),
                                     ((5, -9, 3), 2048, 16, (0, -1, 4))):
        lo, d = nvdb.subdomain_box(origin, size, halo, cell)
        olo, od = moe.widened_box(np.asarray(cell), np.asarray(origin), size, halo)
        assert list(lo) == [int(a) for a in olo] and d == od == size + 2 * halo
    with pytest.raises(nvdb.NvdbError):
        nvdb.subdomain_box((0, 0, 0), 8, 8, (0, 0, 0))  # size < 2 halo
    with pytest.raises(nvdb.NvdbError):
        nvdb.subdomain_box((0, 0, 0), 1 << 20, 8, (1 << 12, 0, 0))  # corner beyond 2^30
