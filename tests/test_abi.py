"""The C ABI on the CPU: the library loads, exports what include/dm.h declares,
and rejects bad arguments with the documented status before any device call."""
import ctypes

import pytest

dm = pytest.importorskip("paper_2210_15114_amd")


@pytest.fixture(scope="module")
def L():
    try:
        return dm.lib()
    except ImportError as e:
        pytest.fail("libdm.so must be built before the tests: %s" % e)


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_exports_every_declared_symbol(L):
    names = dm.header_functions()
    assert "dm_prepare" in names and "dm_matvec" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    for code in (dm.OK, dm.ERR_ARG, dm.ERR_NONFINITE, dm.ERR_OVERFLOW, dm.ERR_NOMEM, dm.ERR_DEVICE,
                 dm.ERR_DTYPE, dm.ERR_STATE):
        s = dm.status_string(code)
        assert s and s != "unknown status"
    assert dm.status_string(12345) == "unknown status"


def test_workspace_size_validation(L):
    out = ctypes.c_size_t(0)
    f = L.dm_workspace_size
    assert f(0, 4, dm.L1, dm.F32, ctypes.byref(out)) == dm.ERR_ARG
    assert f(10, 0, dm.L1, dm.F32, ctypes.byref(out)) == dm.ERR_ARG
    assert f(10, 4, 99, dm.F32, ctypes.byref(out)) == dm.ERR_ARG
    assert f(10, 4, 0, dm.F32, ctypes.byref(out)) == dm.ERR_ARG
    assert f(10, 4, dm.L1, 9, ctypes.byref(out)) == dm.ERR_ARG
    assert f(10, 4, dm.L1, dm.F32, None) == dm.ERR_ARG
    assert f(1 << 31, 4, dm.L1, dm.F32, ctypes.byref(out)) == dm.ERR_ARG       # 32-bit positions
    assert f(10, 4096, dm.L2SQ, dm.F32, ctypes.byref(out)) == dm.ERR_ARG        # l2 staging bound
    assert f(1000, 16, dm.L1, dm.F32, ctypes.byref(out)) == dm.OK
    small = out.value
    assert f(4000, 16, dm.L1, dm.F32, ctypes.byref(out)) == dm.OK
    assert out.value > small > 3 * 16 * 1000 * 4
    assert dm.workspace_size(1000, 16, dm.L2SQ, dm.F32) >= 1000 * 16 * 4


def test_prepare_argument_errors_before_device(L):
    h = ctypes.c_void_p(None)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first
    P = L.dm_prepare
    assert P(None, 10, 4, dm.L1, dm.F32, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 0, 4, dm.L1, dm.F32, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 10, -1, dm.L1, dm.F32, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 10, 4, 99, dm.F32, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 10, 4, dm.TV, dm.I32, None, 0, None, ctypes.byref(h)) == dm.ERR_DTYPE
    assert P(fake, 10, 4, dm.L1, 0, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 10, 4, dm.L1, dm.F32, fake, 16, None, ctypes.byref(h)) == dm.ERR_ARG   # short workspace
    assert P(fake, 10, 4, dm.L1, dm.F32, None, 0, None, None) == dm.ERR_ARG
    for metric in (dm.KL, dm.CE):                      # logarithms: float data only
        assert P(fake, 10, 4, metric, dm.I32, None, 0, None, ctypes.byref(h)) == dm.ERR_DTYPE
    for metric in dm.MATRIX_METRICS:                   # the matrix comes through dm_prepare_matrix
        assert P(fake, 10, 4, metric, dm.F32, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert h.value is None


def test_prepare_matrix_argument_errors_before_device(L):
    import numpy as np
    h = ctypes.c_void_p(None)
    fake = ctypes.c_void_p(0x1000)
    M = np.eye(4)
    Mp = M.ctypes.data_as(ctypes.c_void_p)
    P = L.dm_prepare_matrix
    assert P(fake, 10, 4, dm.L1, dm.F32, Mp, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG      # no matrix metric
    assert P(fake, 10, 4, dm.MAHA2, dm.F32, None, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG  # M missing
    assert P(None, 10, 4, dm.MAHA2, dm.F32, Mp, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 10, 4, dm.MAHA2, dm.I32, Mp, None, 0, None, ctypes.byref(h)) == dm.ERR_DTYPE
    assert P(fake, 10, 4, dm.BILINEAR, dm.I64, Mp, None, 0, None, ctypes.byref(h)) == dm.ERR_DTYPE
    assert P(fake, 0, 4, dm.BILINEAR, dm.F32, Mp, None, 0, None, ctypes.byref(h)) == dm.ERR_ARG
    assert P(fake, 10, 4, dm.BILINEAR, dm.F32, Mp, None, 0, None, None) == dm.ERR_ARG
    assert h.value is None
    if not _has_gpu():
        assert P(fake, 10, 4, dm.MAHA2, dm.F32, Mp, None, 0, None, ctypes.byref(h)) == dm.ERR_DEVICE


def test_workspace_of_the_sort_free_metrics(L):
    n, d = 1000, 16
    # the workspace holds the point copy (and, for the divergences, the FP64
    # logarithms; for the quadratic forms M and W) besides the query scratch
    # of b <= 64, which depends on the metric's number of moments
    assert dm.workspace_size(n, d, dm.L4, dm.F32) >= n * d * 4
    assert dm.workspace_size(n, d, dm.L6, dm.I32) >= dm.workspace_size(n, d, dm.L4, dm.F32)
    assert dm.workspace_size(n, d, dm.CE, dm.F32) >= n * d * (4 + 8)
    assert dm.workspace_size(n, d, dm.KL, dm.F32) == dm.workspace_size(n, d, dm.CE, dm.F32)
    assert dm.workspace_size(n, d, dm.MAHA2, dm.F32) >= n * d * 4 + 2 * d * d * 8
    big = 1 << 20   # no sort arrays: far smaller than l1's at a size where arrays dominate
    assert dm.workspace_size(big, d, dm.L4, dm.F32) < dm.workspace_size(big, d, dm.L1, dm.F32) / 2


def test_workspace_holds_the_query_memory(L):
    """Everything a query of any b <= 64 needs lives in the workspace: it
    grows linearly in n with no per-b part left to allocate later."""
    for metric, dtype in ((dm.L1, dm.F32), (dm.L1, dm.I32), (dm.L3, dm.F32), (dm.L2SQ, dm.F32)):
        a = dm.workspace_size(100000, 8, metric, dtype)
        b = dm.workspace_size(200000, 8, metric, dtype)
        assert b > a


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_prepare_without_device(L):
    h = ctypes.c_void_p(None)
    st = L.dm_prepare(ctypes.c_void_p(0x1000), 10, 4, dm.L1, dm.F32, None, 0, None, ctypes.byref(h))
    assert st == dm.ERR_DEVICE
    assert h.value is None


def test_null_handle_calls(L):
    assert L.dm_matvec(None, ctypes.c_void_p(0x1000), dm.F32, 1, ctypes.c_void_p(0x2000), None) == dm.ERR_ARG
    assert L.dm_sync(None) == dm.ERR_ARG
    assert L.dm_reserve(None, 4) == dm.ERR_ARG
    assert L.dm_info(None, None, None, None, None) == dm.ERR_ARG
    assert L.dm_copy_sorted(None, None, None, None, None) == dm.ERR_ARG
    assert L.dm_tune(None, 8, dm.F32, 4, None, None, None) == dm.ERR_ARG
    assert L.dm_set_variant(None, 8, dm.F32, 0) == dm.ERR_ARG
    assert L.dm_get_variant(None, 8, dm.F32, None) == dm.ERR_ARG
    assert L.dm_lowrank(None, 32, 40, 8, None, None, None, None, None) == dm.ERR_ARG
    assert L.dm_embed_l2(None, 10, 2, dm.F32, None, 4, None, None) == dm.ERR_ARG


def test_embed_argument_errors_before_device(L):
    X, G, O = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x40000)
    assert L.dm_embed_l2(X, 0, 2, dm.F32, G, 4, O, None) == dm.ERR_ARG        # n
    assert L.dm_embed_l2(X, 10, 2, dm.F32, G, 0, O, None) == dm.ERR_ARG       # k
    assert L.dm_embed_l2(X, 10, 2, dm.F32, G, 70000, O, None) == dm.ERR_ARG   # k too large
    assert L.dm_embed_l2(X, 10, 2, 99, G, 4, O, None) == dm.ERR_ARG           # dtype
    assert L.dm_embed_l2(X, 10, 2, dm.F32, G, 4, X, None) == dm.ERR_ARG       # overlap
    if not _has_gpu():
        assert L.dm_embed_l2(X, 10, 2, dm.F32, G, 4, O, None) == dm.ERR_DEVICE
    L.dm_free(None)


def test_copy_probe_argument_errors_before_device(L):
    A, B = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x90000)
    assert L.dm_copy_probe(A, B, 0, None) == dm.ERR_ARG            # empty
    assert L.dm_copy_probe(A, B, 24, None) == dm.ERR_ARG           # not a multiple of 16
    assert L.dm_copy_probe(ctypes.c_void_p(0x10008), B, 32, None) == dm.ERR_ARG   # misaligned
    assert L.dm_copy_probe(A, ctypes.c_void_p(0x10010), 32, None) == dm.ERR_ARG   # overlap
    assert L.dm_copy_probe(None, B, 32, None) == dm.ERR_ARG


def test_gather_probe_argument_errors_before_device(L):
    P, Z, O = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x100000), ctypes.c_void_p(0x900000)
    assert L.dm_gather_probe(P, Z, O, 0, 64, None) == dm.ERR_ARG                       # n
    assert L.dm_gather_probe(P, Z, O, 100, 48, None) == dm.ERR_ARG                     # b not a power of two
    assert L.dm_gather_probe(P, Z, O, 100, 2, None) == dm.ERR_ARG                      # b < 4
    assert L.dm_gather_probe(P, Z, O, 100, 128, None) == dm.ERR_ARG                    # b > 64
    assert L.dm_gather_probe(P, ctypes.c_void_p(0x100008), O, 100, 64, None) == dm.ERR_ARG   # misaligned
    assert L.dm_gather_probe(P, Z, ctypes.c_void_p(0x100100), 100, 64, None) == dm.ERR_ARG   # overlap
    assert L.dm_gather_probe(None, Z, O, 100, 64, None) == dm.ERR_ARG


def test_variant_count(L):
    assert L.dm_variant_count() == 4


def test_int_bound_guard(L):
    assert dm.int_bound_ok(1000.0, 1000.0)
    assert dm.int_bound_ok(2.0 ** 31, 2.0 ** 30)
    assert not dm.int_bound_ok(2.0 ** 31, 2.0 ** 31)          # 2^62 is not below 2^62
    assert not dm.int_bound_ok(float("nan"), 1.0)
    assert not dm.int_bound_ok(-1.0, 1.0)


def test_code_hash_ignores_comments_only(tmp_path):
    # the stored counter and error figures name the kernel code by this hash
    from paper_2210_15114_amd.build import code_hash
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {\n    return x + 1;   // one more\n}\n")
    h0 = code_hash([str(a)])
    a.write_text("/* header */\nint f(int x)\n{\n  return x + 1;\n}\n// trailing\n")
    assert code_hash([str(a)]) == h0
    a.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert code_hash([str(a)]) != h0
