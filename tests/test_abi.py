"""The C-ABI library loads without a GPU, exports every symbol the header
declares, and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kbatch.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(ln for ln in text.splitlines() if not ln.lstrip().startswith("typedef"))
    names = re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)
    return [n for n in names if not n.startswith("_")]


@pytest.fixture(scope="module")
def lib():
    from paper_1902_05320_amd import kbatch
    if not os.path.exists(kbatch.LIB_PATH):
        pytest.skip("libkbatch.so not built")
    return kbatch.load_library()


def test_header_declares_the_binding_exports():
    from paper_1902_05320_amd import kbatch
    assert sorted(_declared_functions()) == sorted(kbatch.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_sizes(lib):
    assert [lib.keccak_digest_bytes(v) for v in range(4)] == [28, 32, 48, 64]
    assert [lib.keccak_rate_bytes(v) for v in range(4)] == [144, 136, 104, 72]
    assert lib.keccak_digest_bytes(4) == -1 and lib.keccak_rate_bytes(-1) == -1
    assert lib.keccak_version().startswith(b"kbatch")


def test_argument_errors_need_no_device(lib):
    from paper_1902_05320_amd import kbatch as kb
    p = ctypes.c_void_p(0x1000)
    # unknown variant
    assert lib.keccak_batch(7, p, p, p, 4, p, None) == kb.KB_EINVAL
    assert b"variant" in lib.keccak_last_error()
    assert lib.keccak_batch_noalloc(4, p, p, p, 4, p, None) == kb.KB_EINVAL
    assert lib.keccak_batch_noalloc(1, p, p, p, kb.NOALLOC_MAX_MSGS + 1, p, None) == kb.KB_EINVAL
    assert b"static workspace" in lib.keccak_last_error()
    assert lib.keccak_batch_noalloc(1, None, None, None, 0, None, None) == kb.KB_OK
    # n == 0 is a no-op, NULLs allowed
    assert lib.keccak_batch(1, None, None, None, 0, None, None) == kb.KB_OK
    assert lib.keccak_last_error() == b""
    # NULL with n > 0
    assert lib.keccak_batch(1, p, None, p, 4, p, None) == kb.KB_EINVAL
    assert lib.keccak_batch_mixed(None, p, p, p, 4, p, None) == kb.KB_EINVAL
    # misaligned metadata / output
    assert lib.keccak_batch(1, p, ctypes.c_void_p(0x1004), p, 4, p, None) == kb.KB_EINVAL
    assert lib.keccak_batch(1, p, p, p, 4, ctypes.c_void_p(0x1002), None) == kb.KB_EINVAL
    # unknown mode, bad mixed flag
    assert lib.keccak_batch_ex(1, None, p, p, p, 4, p, 9, None, None) == kb.KB_EINVAL
    assert lib.keccak_batch_ex(-2, None, p, p, p, 4, p, 0, None, None) == kb.KB_EINVAL
    # a tile asking for another workgroup size
    t = kb.Tile()
    t.block_threads = 64
    assert lib.keccak_batch_ex(1, None, p, p, p, 4, p, 0, ctypes.byref(t), None) == kb.KB_EINVAL
    assert b"block_threads" in lib.keccak_last_error()
    # threads per state: 1 or the wide split tail, nothing else
    t = kb.Tile()
    t.class_threads[3] = 5
    assert lib.keccak_batch_ex(1, None, p, p, p, 4, p, 0, ctypes.byref(t), None) == kb.KB_EINVAL
    assert b"class_threads[3]" in lib.keccak_last_error()
    # the wide and pair modes are known modes (only the mode check is
    # exercised here, through n == 0)
    assert lib.keccak_batch_ex(1, None, None, None, None, 0, None, 4, None, None) == kb.KB_OK
    assert lib.keccak_batch_ex(1, None, None, None, None, 0, None, 5, None, None) == kb.KB_OK
    assert lib.keccak_batch_ex(1, None, None, None, None, 0, None, 6, None, None) == kb.KB_EINVAL
    # tree mode
    assert lib.merkle_root(1, p, 100, 0, p, None) == kb.KB_EINVAL
    assert lib.merkle_root(5, p, 100, 10, p, None) == kb.KB_EINVAL
    assert lib.merkle_root(1, p, 100, 10, None, None) == kb.KB_EINVAL


def test_keccak_p_argument_errors_need_no_device(lib):
    from paper_1902_05320_amd import kbatch as kb
    p = ctypes.c_void_p(0x1000)
    assert lib.keccak_p_batch(24, 1, p, 1, None) == kb.KB_EINVAL  # not a Table 1 width
    assert b"b must be" in lib.keccak_last_error()
    assert lib.keccak_p_batch(1600, 0, p, 1, None) == kb.KB_EINVAL
    assert lib.keccak_p_batch(1600, 4097, p, 1, None) == kb.KB_EINVAL
    assert lib.keccak_p_batch(200, 18, None, 3, None) == kb.KB_EINVAL
    assert lib.keccak_p_batch(25, 12, None, 0, None) == kb.KB_OK  # n == 0: nothing to do
    assert lib.keccak_last_error() == b""


def test_probe_argument_errors_need_no_device(lib):
    from paper_1902_05320_amd import kbatch as kb
    g, w = ctypes.c_double(0.0), ctypes.c_int(0)
    assert lib.keccak_probe_perm(0, 0, ctypes.byref(g), ctypes.byref(w), None) == kb.KB_EINVAL
    assert lib.keccak_probe_perm(10, -1, ctypes.byref(g), ctypes.byref(w), None) == kb.KB_EINVAL
    assert lib.keccak_probe_perm(10, 0, None, ctypes.byref(w), None) == kb.KB_EINVAL
    assert lib.keccak_probe_perm(10, 0, ctypes.byref(g), None, None) == kb.KB_EINVAL


def test_timing_kinds_need_no_device(lib):
    from paper_1902_05320_amd import kbatch as kb
    ms, cnt = ctypes.c_double(1.0), ctypes.c_uint64(1)
    assert lib.keccak_timing_enable_kinds(1 << (max(kb.KERNELS.values()) + 1)) == kb.KB_EINVAL
    assert b"kind" in lib.keccak_last_error()
    assert lib.keccak_timing_enable_kinds(1 << kb.KERNELS["first_pass"]) == kb.KB_OK
    assert lib.keccak_timing_read(ctypes.byref(ms), ctypes.byref(cnt)) == kb.KB_OK
    assert (ms.value, cnt.value) == (0.0, 0)
    assert lib.keccak_timing_enable(1) == kb.KB_OK and lib.keccak_timing_enable(0) == kb.KB_OK
    assert lib.keccak_timing_enable_kinds(0) == kb.KB_OK


def test_xof_ex_argument_errors_need_no_device(lib):
    from paper_1902_05320_amd import kbatch as kb
    p = ctypes.c_void_p(0x1000)
    assert lib.keccak_batch_xof_ex(192, p, p, p, 1, 32, p, 0, None) == kb.KB_EINVAL
    assert lib.keccak_batch_xof_ex(128, p, p, p, 1, 0, p, 0, None) == kb.KB_EINVAL
    assert lib.keccak_batch_xof_ex(128, p, p, p, 1, 32, p, 7, None) == kb.KB_EINVAL
    assert b"mode" in lib.keccak_last_error()
    assert lib.keccak_batch_xof_ex(256, None, None, None, 0, 32, None, 3, None) == kb.KB_OK


def _tree_bytes_by_level_walk(leaves, D):
    # every level above the leaves but the root is stored, each level
    # starting 16-byte aligned; plus one digest
    m, off = max(leaves, 1), 0
    while m > 1:
        off = (off + m * D + 15) // 16 * 16
        m = (m + 1) // 2
    return off + D


def test_tree_workspace_covers_every_level(lib):
    # the size a captured tree's private node buffer gets; SHA3-512 needs
    # more than two digests per leaf when the leaf count is 2^k + 1
    import numpy as np
    for v, D in enumerate((28, 32, 48, 64)):
        for leaves in range(1, 100_001):
            assert lib.keccak_tree_workspace_bytes(v, leaves) == _tree_bytes_by_level_walk(leaves, D), (v, leaves)
    for leaves in (2**18 + 1, 2**20 + 1, 3 * 10**6):
        assert lib.keccak_tree_workspace_bytes(3, leaves) == _tree_bytes_by_level_walk(leaves, 64)
    # 17 SHA3-512 leaves: levels of 17, 9, 5, 3, 2 nodes (1088, 576, 320, 192,
    # 128 bytes) and one digest; two digests per leaf plus one (2240) is short
    assert lib.keccak_tree_workspace_bytes(3, 17) == 2368
    assert lib.keccak_tree_workspace_bytes(4, 10) == 0
