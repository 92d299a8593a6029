"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/hgref.h declares, and its pure host logic (sizes,
argument checks) behaves as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgref.h")
LIB = os.path.join(ROOT, "paper_2010_10272_amd", "libhgref.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(hg_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    import torch  # noqa: F401  (same HIP runtime the product binds to)
    return ctypes.CDLL(LIB)


def test_header_declares_the_core_calls():
    names = _declared()
    for n in ["hg_load_csr", "hg_compute_pincounts", "hg_km1", "hg_gains", "hg_lp_round",
              "hg_refine", "hg_free", "hg_workspace_size", "hg_last_error"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_net_words_and_workspace_size(lib):
    lib.hg_net_words.restype = ctypes.c_int32
    assert [lib.hg_net_words(k) for k in (1, 2, 32, 33, 64, 65, 128, 129, 256, 257)] == \
        [0, 4, 4, 8, 8, 16, 16, 32, 32, 0]
    f = lib.hg_workspace_size
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    f.restype = ctypes.c_size_t
    assert f(10, 10, 40, 2) > 0
    assert f(10, 10, 40, 300) == 0          # k_max above 256
    assert f(10, 10, 5, 2) == 0             # fewer pins than nets
    assert f(0, 10, 40, 2) == 0
    assert f(1000, 1000, 4000, 64) > f(1000, 1000, 4000, 2)


def test_load_rejects_bad_arguments_before_touching_the_device(lib):
    vp = ctypes.c_void_p
    lib.hg_load_csr.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp,
                                vp, vp, vp, ctypes.c_size_t, ctypes.c_int32, vp,
                                ctypes.POINTER(vp)]
    lib.hg_load_csr.restype = ctypes.c_int32
    lib.hg_last_error.restype = ctypes.c_char_p
    out = vp()
    fake = vp(0x1000)
    # null pointers
    assert lib.hg_load_csr(4, 2, 4, None, None, None, None, None, None, None, 0, 2, None,
                           ctypes.byref(out)) == -1
    assert b"non-NULL" in lib.hg_last_error()
    # k_max out of range
    assert lib.hg_load_csr(4, 2, 4, fake, fake, None, None, fake, fake, fake, 1 << 20, 1, None,
                           ctypes.byref(out)) == -2
    # workspace too small
    assert lib.hg_load_csr(4, 2, 4, fake, fake, None, None, fake, fake, fake, 16, 2, None,
                           ctypes.byref(out)) == -4
    # no out pointer
    assert lib.hg_load_csr(4, 2, 4, fake, fake, None, None, fake, fake, fake, 1 << 20, 2, None,
                           None) == -1
    assert out.value is None


def test_calls_on_null_handle_fail_cleanly(lib):
    vp = ctypes.c_void_p
    lib.hg_km1.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    lib.hg_km1.restype = ctypes.c_int32
    assert lib.hg_km1(None, 2, None, None, None) == -1
    lib.hg_max_block_weight.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    lib.hg_max_block_weight.restype = ctypes.c_int64
    assert lib.hg_max_block_weight(None, 2, 0.03) == -1
    lib.hg_free.argtypes = [vp]
    lib.hg_free(None)


def test_next_row_sizes_and_null_handles(lib):
    vp = ctypes.c_void_p
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.hg_gain_cache_bytes.argtypes = [i32, i32]
    lib.hg_gain_cache_bytes.restype = i64
    # b and w(I) (2n int32, rounded up to whole quads) plus rows of k rounded up to 4
    assert lib.hg_gain_cache_bytes(10, 8) == 4 * (20 + 10 * 8)
    assert lib.hg_gain_cache_bytes(11, 7) == 4 * (24 + 11 * 8)
    assert lib.hg_gain_cache_bytes(0, 8) == -1 and lib.hg_gain_cache_bytes(10, 1) == -1
    lib.hg_moves_workspace_size.argtypes = [i32, i32, i32]
    lib.hg_moves_workspace_size.restype = sz
    assert lib.hg_moves_workspace_size(100, 100, 8) >= 16 * 100 * 8
    assert lib.hg_moves_workspace_size(100, 100, 1) == 0
    lib.hg_rebalance_workspace_size.argtypes = [i32, i32]
    lib.hg_rebalance_workspace_size.restype = sz
    assert lib.hg_rebalance_workspace_size(100, 8) >= lib.hg_gain_cache_bytes(100, 8)
    assert lib.hg_rebalance_workspace_size(0, 8) == 0
    assert lib.hg_rebalance_workspace_size(100, 300) == 0
    lib.hg_contract_workspace_size.argtypes = [i32, i32, i64]
    lib.hg_contract_workspace_size.restype = sz
    assert lib.hg_contract_workspace_size(100, 50, 400) >= 4 * 400
    assert lib.hg_contract_workspace_size(100, 50, 1 << 31) == 0
    assert lib.hg_contract_workspace_size(0, 50, 400) == 0
    # calls on a null graph handle fail before touching the device
    lib.hg_gain_cache_init.argtypes = [vp] * 6
    lib.hg_gain_cache_init.argtypes[1] = i32
    lib.hg_gain_cache_init.restype = i32
    assert lib.hg_gain_cache_init(None, 8, None, None, None, None) == -1
    lib.hg_rebalance.argtypes = [vp, i32, i64, i32] + [vp] * 9 + [sz, vp]
    lib.hg_rebalance.restype = i32
    assert lib.hg_rebalance(None, 8, 10, 1, *([None] * 9), 0, None) == -1
    lib.hg_contract.argtypes = [vp] * 9 + [sz, vp]
    lib.hg_contract.restype = i32
    assert lib.hg_contract(*([None] * 9), 0, None) == -1
    lib.hg_move_gains.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.hg_move_gains.restype = i32
    assert lib.hg_move_gains(None, 8, None, None, 1, None, None, None, None, 0, None) == -1
