"""Host-side validation of the C ABI without a GPU: every entry point
refuses null handles and null required pointers with TRX_E_INVALID_ARG
(1) instead of touching them, and a context cannot be made for a device
that does not exist.  No device work is enqueued by any of these calls."""

import ctypes

import pytest

INVALID_ARG = 1
P = ctypes.c_void_p
I32 = ctypes.c_int32


@pytest.fixture(scope="module")
def lib():
    from paper_1912_07759_amd import trx
    L = ctypes.CDLL(trx.LIB_PATH)
    for name in trx.EXPORTS:
        getattr(L, name).restype = ctypes.c_int
    L.trx_last_error.restype = ctypes.c_char_p
    L.trx_plan_describe.restype = ctypes.c_char_p
    return L


def test_context_for_a_missing_device(lib):
    h = P(12345)
    assert lib.trx_create(-1, ctypes.byref(h)) == INVALID_ARG
    assert h.value is None            # the output is cleared
    assert lib.trx_create(1 << 20, ctypes.byref(h)) == INVALID_ARG
    assert lib.trx_create(0, None) == INVALID_ARG


def test_null_handles(lib):
    n = None
    assert lib.trx_destroy(n) == INVALID_ARG
    assert lib.trx_last_error(n) == b""
    assert lib.trx_set_stream(n, n) == INVALID_ARG
    assert lib.trx_synchronize(n) == INVALID_ARG
    assert lib.trx_tables_create(n, n, n) == INVALID_ARG
    assert lib.trx_tables_destroy(n) == INVALID_ARG
    assert lib.trx_bins_create(n, n, I32(3), n, n, n) == INVALID_ARG
    assert lib.trx_bins_destroy(n) == INVALID_ARG
    assert lib.trx_forward(n, n, n, n, I32(1), n, n, n, n) == INVALID_ARG
    assert lib.trx_emission(n, n, n, n, I32(1), I32(4), n, n, n, n) == INVALID_ARG
    assert lib.trx_forward_noalloc(n, n, n, n, I32(1), n, n, n) == INVALID_ARG
    assert lib.trx_chi2_grad(n, n, n, n, I32(1), n, n, I32(1), n, n, n, n, n, n) == INVALID_ARG
    assert lib.trx_plan_create(n, n, n, I32(4), I32(100), I32(1), I32(0), n) == INVALID_ARG
    assert lib.trx_plan_destroy(n) == INVALID_ARG
    assert lib.trx_plan_set_star(n, n, I32(4)) == INVALID_ARG
    assert lib.trx_plan_batch(n, n) == INVALID_ARG
    assert lib.trx_plan_launch(n, n, n, n, n, n, n, n, n, n, n) == INVALID_ARG
    assert lib.trx_profile(n, I32(1)) == INVALID_ARG
    assert lib.trx_profile_read(n, I32(0), n, n) == INVALID_ARG
    assert lib.trx_autotune(n, n, n) == INVALID_ARG
    assert lib.trx_plan_set_variant(n, n) == INVALID_ARG
    assert lib.trx_plan_describe(n) == b""


def test_every_entry_point_is_covered(lib):
    """The two tests above call every exported entry point."""
    import inspect
    from paper_1912_07759_amd import trx
    src = inspect.getsource(test_null_handles) + inspect.getsource(test_context_for_a_missing_device)
    missing = [n for n in trx.EXPORTS if f"lib.{n}(" not in src]
    assert not missing, missing
