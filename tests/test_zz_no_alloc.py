"""GPU: the allocation-free entry point (a static per-device workspace)
gives the same digests as keccak_batch, call after call, called through the
C ABI.  Two calls in a row, the second smaller, for a batch the first pass
hashes whole and for one whose messages go through the bucketed pass."""

import ctypes

import numpy as np
import pytest

from paper_1902_05320_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_05320_amd import kbatch
    kbatch.load_library()
    return kbatch


def _dev(b):
    import torch
    return (torch.from_numpy(b.data).cuda(), torch.from_numpy(b.offsets).cuda(),
            torch.from_numpy(b.lengths).cuda())


def _noalloc_c_abi(kb, v, data, offs, lens, out):
    import torch
    lib = kb.load_library()
    rc = lib.keccak_batch_noalloc(v, ctypes.c_void_p(data.data_ptr()),
                                  ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(lens.data_ptr()),
                                  offs.numel(), ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == kb.KB_OK, lib.keccak_last_error()


@pytest.mark.parametrize("v", [1, 3])
def test_noalloc_equals_keccak_batch_on_two_calls(kb, v):
    import torch
    D = kb.DIGEST_BYTES[v]
    cases = [
        # uneven lengths: deferred chunks, bucketed order, the second pass
        (wl.uneven(kb.NOALLOC_MAX_MSGS, 3000, seed=90, variant=v), wl.uneven(7001, 9000, seed=91, variant=v)),
        # one-block messages: the first pass hashes every chunk
        (wl.uniform(300_001, 40, seed=92, variant=v), wl.uniform(4097, 7, seed=93, variant=v)),
    ]
    for big, small in cases:
        for b in (big, small):
            print("[case] noalloc", v, b.name, flush=True)
            data, offs, lens = _dev(b)
            want = kb.keccak_batch(v, data, offs, lens)
            got = torch.full((b.n, D), 0xA5, dtype=torch.uint8, device="cuda")
            _noalloc_c_abi(kb, v, data, offs, lens, got)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (b.name, int((got != want).any(dim=1).sum()))
            if b is small:  # the binding's wrapper too
                got2 = kb.keccak_batch_noalloc(v, data, offs, lens, torch.empty_like(got))
                torch.cuda.synchronize()
                assert torch.equal(got2, want)


def test_noalloc_rejects_more_than_its_workspace_holds(kb):
    import torch
    lib = kb.load_library()
    n = kb.NOALLOC_MAX_MSGS + 1
    offs = torch.zeros(n, dtype=torch.int64, device="cuda")
    data = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    rc = lib.keccak_batch_noalloc(1, ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(offs.data_ptr()),
                                  ctypes.c_void_p(offs.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == kb.KB_EINVAL and b"static workspace" in lib.keccak_last_error()
    assert not out.any()
