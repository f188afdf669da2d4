"""CPU checks of the C-ABI library: it loads, exports every function the
public header declares, and rejects bad arguments before touching a GPU."""
import ctypes

import pytest

from paper_1707_05354_amd import lsm as L


@pytest.fixture(scope="module")
def lib():
    return L.load_library()


def test_header_declares_the_dictionary_calls():
    names = L.header_symbols()
    for n in ("lsm_create", "lsm_insert_batch", "lsm_delete_batch", "lsm_lookup",
              "lsm_count", "lsm_range", "lsm_destroy"):
        assert n in names


def test_every_header_symbol_is_exported(lib):
    names = L.header_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), "missing export " + n
        assert n in L._SIGNATURES, "binding lacks " + n


def test_strerror(lib):
    assert lib.lsm_strerror(0) == b"ok"
    assert lib.lsm_strerror(3) == b"batch larger than b"
    assert lib.lsm_strerror(99) == b"unknown status"


def test_create_rejects_bad_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.lsm_create(None, 16, 0, None) == L.LSM_EINVAL
    assert lib.lsm_create(ctypes.byref(h), 0, 0, None) == L.LSM_EINVAL
    assert h.value is None
    assert lib.lsm_create(ctypes.byref(h), (1 << 28) + 1, 0, None) == L.LSM_EINVAL
    assert lib.lsm_create(ctypes.byref(h), 16, 0x4, None) == L.LSM_EINVAL
    assert lib.lsm_create(ctypes.byref(h), 16, L.LSM_KEY_BITS(32), None) == L.LSM_EINVAL


def test_null_handle_calls(lib):
    assert lib.lsm_insert_batch(None, None, None, 4) == L.LSM_EINVAL
    assert lib.lsm_delete_batch(None, None, 4) == L.LSM_EINVAL
    assert lib.lsm_update_batch(None, None, None, None, 4) == L.LSM_EINVAL
    assert lib.lsm_lookup(None, None, 4, None, None) == L.LSM_EINVAL
    assert lib.lsm_count(None, None, None, 4, None) == L.LSM_EINVAL
    t = ctypes.c_uint64()
    assert lib.lsm_range(None, None, None, 4, None, None, None, 0, ctypes.byref(t)) == L.LSM_EINVAL
    assert lib.lsm_destroy(None) == L.LSM_EINVAL
    assert lib.lsm_num_batches(None) == 0
    assert lib.lsm_batch_size(None) == 0
    assert lib.lsm_set_stream(None, None) == L.LSM_EINVAL
    st = L.Stats()
    assert lib.lsm_get_stats(None, ctypes.byref(st)) == L.LSM_EINVAL


def test_struct_layouts_match_the_binding(lib):
    ss, ps = ctypes.c_size_t(), ctypes.c_size_t()
    lib.lsm_struct_sizes(ctypes.byref(ss), ctypes.byref(ps))
    assert ss.value == ctypes.sizeof(L.Stats)
    assert ps.value == ctypes.sizeof(L.Profile)
