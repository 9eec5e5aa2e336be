"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and argument errors come back as status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gapbfs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gap_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1508_03619_amd import gapbfs
    if not os.path.exists(gapbfs.library_path()):
        from paper_1508_03619_amd import build
        build.build(verbose=False)
    return gapbfs.load()


def test_header_declares_the_four_calls():
    fns = declared_functions()
    for f in ("gap_build_csr", "gap_bfs", "gap_bfs_batch", "gap_free"):
        assert f in fns


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1508_03619_amd import gapbfs
    assert sorted(gapbfs.EXPORTED) == declared_functions()


def test_argument_errors_without_device(lib):
    from paper_1508_03619_amd import gapbfs
    out = ctypes.c_void_p()
    # NULL out pointer
    assert lib.gap_build_csr(4, 0, None, None, 0, None, None) == gapbfs.GAP_EINVAL
    # n out of range
    assert lib.gap_build_csr(0, 0, None, None, 0, None, ctypes.byref(out)) == gapbfs.GAP_EINVAL
    assert lib.gap_build_csr(2 ** 31, 0, None, None, 0, None, ctypes.byref(out)) == gapbfs.GAP_EINVAL
    # edges without arrays
    assert lib.gap_build_csr(4, 3, None, None, 0, None, ctypes.byref(out)) == gapbfs.GAP_EINVAL
    # unknown flag bits (only GAP_BUILD_DIRECTED is defined)
    s = (ctypes.c_int32 * 1)(0)
    assert lib.gap_build_csr(4, 1, s, s, 2, None, ctypes.byref(out)) == gapbfs.GAP_EINVAL
    assert b"flag" in lib.gap_last_error()
    assert lib.gap_graph_directed(None) == gapbfs.GAP_EINVAL
    assert lib.gap_graph_export_in(None, None, None) == gapbfs.GAP_EINVAL
    # NULL graph / parent
    assert lib.gap_bfs(None, 0, None, None, None) == gapbfs.GAP_EINVAL
    assert b"NULL" in lib.gap_last_error()
    assert lib.gap_bfs_batch(None, 1, None, None, 1, None, None, None) == gapbfs.GAP_EINVAL
    assert lib.gap_bc(None, None, 4, None, 0, None) == gapbfs.GAP_EINVAL
    assert lib.gap_sssp(None, 0, None, 0, None) == gapbfs.GAP_EINVAL
    assert lib.gap_cc(None, None, None) == gapbfs.GAP_EINVAL
    assert lib.gap_graph_export_weights(None, None) == gapbfs.GAP_EINVAL
    s1 = (ctypes.c_int32 * 1)(0)
    assert lib.gap_build_csr_weighted(4, 1, s1, s1, None, 0, None, ctypes.byref(out)) == gapbfs.GAP_EINVAL
    assert b"NULL" in lib.gap_last_error()
    lib.gap_free(None)  # NULL-safe


def test_params_validation(lib):
    from paper_1508_03619_amd import gapbfs
    p = gapbfs.get_params()
    assert p["block"] in (256, 512, 1024)
    with pytest.raises(gapbfs.GapError):
        gapbfs.set_params(block=100)
    with pytest.raises(gapbfs.GapError):
        gapbfs.set_params(chunk_edges=100)
    with pytest.raises(gapbfs.GapError):
        gapbfs.set_params(alpha=0)
    with pytest.raises(gapbfs.GapError):
        gapbfs.set_params(wait_limit_us=-1)
    assert gapbfs.get_params() == p
    assert p["wait_limit_us"] == 0  # built-in device-side wait bounds


def test_status_and_shutdown_without_work(lib):
    """A stream with no queued search has nothing to report; shutdown with
    nothing allocated is a no-op."""
    from paper_1508_03619_amd import gapbfs
    assert lib.gap_stream_status(None) == gapbfs.GAP_OK
    lib.gap_shutdown()
    assert lib.gap_stream_status(None) == gapbfs.GAP_OK


def test_no_device_reports_edevice(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    import numpy as np
    from paper_1508_03619_amd import gapbfs
    s = np.array([0, 1], np.int32)
    d = np.array([1, 2], np.int32)
    out = ctypes.c_void_p()
    st = lib.gap_build_csr(3, 2, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0, None, ctypes.byref(out))
    assert st == gapbfs.GAP_EDEVICE


def test_package_reexports_what_the_gpu_tests_call():
    """The GPU tests call the binding through the package object that the
    ``gpu`` fixture returns: every public call must be reachable there."""
    import ast
    import paper_1508_03619_amd as pkg
    used = set()
    for fn in os.listdir(os.path.join(ROOT, "tests")):
        if fn.endswith(".py"):
            tree = ast.parse(open(os.path.join(ROOT, "tests", fn)).read())
            for node in ast.walk(tree):
                if (isinstance(node, ast.Attribute) and isinstance(node.value, ast.Name)
                        and node.value.id in ("gpu", "gb") and not node.attr.startswith("_")):
                    used.add(node.attr)
    missing = sorted(a for a in used if not hasattr(pkg, a))
    assert not missing, missing
