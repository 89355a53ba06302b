"""The C-ABI library loads and exports every symbol include/subkm.h
declares; host-only entry points and argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "subkm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(subkm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1412_1947_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1412_1947_amd import build
        build.build(verbose=False)
    return pkg.lib()


def test_header_lists_the_calls():
    names = declared_functions()
    for f in ("subkm_scale", "subkm_subcluster", "subkm_lloyd_batched", "subkm_cluster"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    import paper_1412_1947_amd as pkg
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(pkg.EXPORTS)


def test_cluster_sizes(lib):
    import paper_1412_1947_amd as pkg
    assert pkg.cluster_sizes(4096, 512, 32) == (8, 256)
    assert pkg.cluster_sizes(1 << 20, 8192, 256) == (128, 32768)
    assert pkg.cluster_sizes(1000, 300, 32) == (4, 3 * 32 + 11)  # ceil(100*32/300) = 11
    assert pkg.cluster_sizes(5, 100, 3) == (1, 1)  # ceil(5*3/100)
    with pytest.raises(pkg.SubkmError):
        pkg.cluster_sizes(10, 5, 6)  # k_local > N


def test_footprint_monotone(lib):
    import paper_1412_1947_amd as pkg
    a = pkg.cluster_footprint(10000, 8, 8192, 256, 16)
    b = pkg.cluster_footprint(20000, 8, 8192, 256, 16)
    c = pkg.cluster_footprint(20000, 16, 8192, 256, 16)
    assert 0 < a < b < c
    assert a >= 2 * 10000 * 8 * 4
    assert pkg.cluster_footprint(10, 8, 5, 6, 1) == 0  # invalid sizes


def test_null_context_is_einval(lib):
    P = ctypes.c_void_p
    assert lib.subkm_scale(None, None, 1, 1, None, None, None) == 1
    assert lib.subkm_subcluster(None, None, 1, 1, 1, 0, 0, None, None, None, None) == 1
    assert lib.subkm_subcluster_unequal(None, None, 1, 1, 1, 0, None, None, None, None) == 1
    assert lib.subkm_cluster(None, None, 1, 1, 1, 1, 1, 1, 0.0, None, None, None, None, None) == 1
    assert lib.subkm_synchronize(None) == 1
    assert lib.subkm_tune_enable(None, 1) == 1
    assert lib.subkm_tune_count(None, None) == 1
    assert lib.subkm_tune_save(None, b"x") == 1
    assert lib.subkm_tune_load(None, b"x") == 1
    lib.subkm_destroy(None)  # no-op


def test_create_without_gpu_reports(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = lib.subkm_create(0, None, ctypes.byref(h))
    assert st == 3  # SUBKM_EDEVICE
    assert b"device" in lib.subkm_last_error(None)


def test_engine_without_gpu_reports(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert lib.subkm_engine_create(0, 1 << 30, 2, ctypes.byref(h)) == 3  # SUBKM_EDEVICE


def test_engine_argument_checks(lib):
    h = ctypes.c_void_p()
    assert lib.subkm_engine_create(0, 0, 2, ctypes.byref(h)) == 1      # no budget
    assert lib.subkm_engine_create(0, 1 << 30, 0, ctypes.byref(h)) == 1  # no slot
    assert lib.subkm_engine_submit(None, None, None) == 1
    assert lib.subkm_engine_wait(None, 1, None) == 1
    lib.subkm_engine_destroy(None)  # no-op


def test_job_footprint_covers_cluster_scratch(lib):
    import paper_1412_1947_amd as pkg
    for (n, d, N, kl, kf) in [(10000, 4, 8192, 256, 8), (2_000_000, 64, 8192, 256, 256),
                              (1 << 22, 128, 32768, 1024, 256), (777, 3, 100, 7, 5)]:
        fp = pkg.cluster_footprint(n, d, N, kl, kf)
        jf = pkg.job_footprint(n, d, N, kl, kf)
        assert fp > 0 and jf >= fp + n * d * 4 + n * 4 + kf * d * 4
    assert pkg.job_footprint(10, 8, 5, 6, 1) == 0
