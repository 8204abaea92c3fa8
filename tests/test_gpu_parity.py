"""GPU parity: every digest from the HIP library equals the CPU oracle's,
byte for byte, on seeded inputs.  Needs an MI355X; run with -m gpu."""

import numpy as np
import pytest

from paper_1902_05320_amd import workloads as wl

pytestmark = pytest.mark.gpu

RATES = (144, 136, 104, 72)
DIGEST = (28, 32, 48, 64)
MODES = ("persistent", "plain", "per_bucket", "split", "wide", "pair")


@pytest.fixture(scope="module")
def kb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_05320_amd import kbatch
    kbatch.load_library()
    return kbatch


def _say(*a):
    print("[case]", *a, flush=True)


def _to_dev(batch):
    import torch
    data = torch.from_numpy(batch.data).cuda() if batch.data.size else torch.zeros(1, dtype=torch.uint8, device="cuda")
    offs = torch.from_numpy(batch.offsets.astype(np.int64)).cuda()
    lens = torch.from_numpy(batch.lengths.astype(np.int64)).cuda()
    var = torch.from_numpy(batch.variants.astype(np.uint8)).cuda()
    return data, offs, lens, var


def _gpu_batch(kb, v, batch, mode="persistent"):
    import torch
    data, offs, lens, _ = _to_dev(batch)
    out = kb.keccak_batch(v, data, offs, lens, mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _gpu_mixed(kb, batch, mode="persistent"):
    import torch
    data, offs, lens, var = _to_dev(batch)
    out = kb.keccak_batch_mixed(var, data, offs, lens, mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _mismatches(got, want):
    bad = np.nonzero((got != want).any(axis=1))[0]
    return bad[:10].tolist(), bad.size


@pytest.mark.parametrize("mode", MODES)
def test_uniform_4096x64_sha3_256(kb, o2, mode):
    b = wl.uniform(4096, 64, seed=1)
    _say("uniform 4096x64B sha3_256", mode)
    got = _gpu_batch(kb, 1, b, mode)
    want = o2.sha3_batch(256, b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)


@pytest.mark.parametrize("v", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", MODES)
def test_every_length_to_3R_unaligned(kb, o2, v, mode):
    # every length 0 .. 3R+1, packed with a 3-byte gap so offsets hit every
    # residue mod 16; the first message starts at byte 5
    R = RATES[v]
    b = wl.explicit(np.arange(0, 3 * R + 2), seed=10 + v, variant=v, gap=3, lead=5)
    _say("every length sha3 variant", v, mode)
    got = _gpu_batch(kb, v, b, mode)
    want = o2.sha3_batch(8 * DIGEST[v], b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)


@pytest.mark.parametrize("mode", MODES)
def test_uneven_mixed_small(kb, o2, mode):
    # log-uniform lengths in [0, 16 KiB], variant per message; spans many
    # workgroups and a ragged tail (n not a multiple of 64)
    b = wl.uneven(20000 + 37, 16384, seed=3)
    _say("uneven mixed n=20037", mode)
    got = _gpu_mixed(kb, b, mode)
    want = o2.sha3_batch_mixed(b.variants, b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)


@pytest.mark.parametrize("v", [1, 3])
def test_uneven_single_variant(kb, o2, v):
    b = wl.uneven(5000, 70000, seed=20 + v, variant=v)
    _say("uneven single variant", v)
    got = _gpu_batch(kb, v, b)
    want = o2.sha3_batch(8 * DIGEST[v], b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)


def test_count_pass_boundaries(kb, o2):
    # the count kernel takes whole passes of 8 x 128 messages per wave, then
    # 64-message chunks with bounds checks: sizes around both boundaries, with
    # uneven lengths (bucketed order) and with equal lengths (arrival order)
    rng = np.random.Generator(np.random.PCG64(80))
    for n in (1, 63, 64, 65, 127, 128, 1023, 1024, 1025, 8191, 8192, 8193, 131072 + 64 + 3):
        for equal in (False, True):
            lens = np.full(n, 100) if equal else wl.log_uniform_lengths(rng, n, 3000)
            var = rng.integers(0, 4, n).astype(np.uint8)
            b = wl.explicit(lens, seed=81, variant=var, gap=2, lead=1)
            _say("count boundaries", n, "equal" if equal else "uneven")
            got = _gpu_mixed(kb, b)
            want = o2.sha3_batch_mixed(b.variants, b.data, b.offsets, b.lengths)
            assert _mismatches(got, want)[1] == 0, (n, equal, _mismatches(got, want))
            got1 = _gpu_batch(kb, 1, b)
            assert (got1 == o2.sha3_batch(256, b.data, b.offsets, b.lengths)).all(), (n, equal)


@pytest.mark.parametrize("case", ["few_long", "many_long", "all_long", "few_items"])
def test_persistent_split_tail(kb, o2, case):
    # the longest messages of a bucketed batch go to the wide split tail (at
    # most two per SIMD, and only messages of at least max(32, 2 x blocks
    # per resident lane) blocks); few: 40 messages of ~0.2-1 MB among 60000
    # short ones; many: 12000 messages of ~20 KB among 200000 short ones,
    # more than the split cap, so the rest of their buckets runs one message
    # per thread; all: 3000 messages of ~16 KB and nothing shorter, between
    # one and two caps, so all go to the tail in two rounds; few items:
    # 5000 messages of 1-3 KB (under 32 blocks), fewer queue items than
    # SIMDs and no tail, so only each SIMD's front wave takes items
    rng = np.random.Generator(np.random.PCG64(70))
    if case == "few_long":
        lens = np.concatenate([rng.integers(0, 300, 60000), rng.integers(200_000, 1_000_000, 40)])
    elif case == "many_long":
        lens = np.concatenate([rng.integers(0, 300, 200000), rng.integers(19_000, 21_000, 12000)])
    elif case == "all_long":
        lens = rng.integers(15_000, 17_000, 3000)
    else:
        lens = rng.integers(1_000, 3_000, 5000)
    rng.shuffle(lens)
    var = rng.integers(0, 4, lens.size).astype(np.uint8)
    b = wl.explicit(lens, seed=71, variant=var, gap=1, lead=3)
    _say("persistent split tail", case, b.n)
    got = _gpu_mixed(kb, b)
    want = o2.sha3_batch_mixed(b.variants, b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)
    v1 = wl.explicit(lens, seed=72, variant=1, gap=0, lead=1)
    got1 = _gpu_batch(kb, 1, v1)
    assert (got1 == o2.sha3_batch(256, v1.data, v1.offsets, v1.lengths)).all()


@pytest.mark.parametrize("mode", ["persistent", "split", "wide", "pair"])
def test_mixed_invalid_variant_slot_is_zero(kb, o2, mode):
    b = wl.explicit([10, 200, 0, 77], seed=5, variant=np.array([1, 9, 3, 255], dtype=np.uint8))
    _say("mixed invalid variant", mode)
    got = _gpu_mixed(kb, b, mode)
    assert not got[1].any() and not got[3].any()
    want = o2.sha3_batch_mixed(np.array([1, 1, 3, 3], np.uint8), b.data, b.offsets, b.lengths)
    assert (got[0] == want[0]).all() and (got[2] == want[2]).all()


@pytest.mark.parametrize("mode", ["persistent", "split", "wide", "pair"])
def test_edge_cases(kb, o2, mode):
    import torch
    _say("edge: empty batch", mode)
    data = torch.zeros(16, dtype=torch.uint8, device="cuda")
    empty = torch.zeros(0, dtype=torch.int64, device="cuda")
    out = kb.keccak_batch(1, data, empty, empty, mode=mode)
    assert out.shape == (0, 32)
    _say("edge: all-empty messages")
    b = wl.explicit([0] * 300, seed=6)
    got = _gpu_batch(kb, 1, b, mode)
    want = o2.sha3_batch(256, b.data, b.offsets, b.lengths)
    assert (got == want).all()
    _say("edge: one long message")
    b = wl.explicit([1_000_003], seed=7, lead=9)
    for v in range(4):
        got = _gpu_batch(kb, v, b, mode)
        want = o2.sha3_batch(8 * DIGEST[v], b.data, b.offsets, b.lengths)
        assert (got == want).all(), v
    _say("edge: overlapping slices ending at the buffer end")
    rng = np.random.Generator(np.random.PCG64(8))
    n = 3000
    buf = rng.integers(0, 256, 5000, dtype=np.uint8)
    lens = rng.integers(0, 400, n)
    offs = buf.size - lens - rng.integers(0, 3, n)  # most slices end within 2 bytes of the end
    offs = np.maximum(offs, 0)
    bt = wl.Batch(buf, offs.astype(np.int64), lens.astype(np.int64), np.ones(n, np.uint8), 8, "ov")
    got = _gpu_batch(kb, 1, bt, mode)
    want = o2.sha3_batch(256, bt.data, bt.offsets, bt.lengths)
    assert (got == want).all()


def test_bounds_checked_in_binding(kb):
    import torch
    data = torch.zeros(100, dtype=torch.uint8, device="cuda")
    offs = torch.tensor([90], dtype=torch.int64, device="cuda")
    lens = torch.tensor([11], dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        kb.keccak_batch(1, data, offs, lens)
    with pytest.raises(ValueError):
        kb.merkle_root(1, data, 0)


def test_order_and_repeat_invariance(kb):
    import torch
    b = wl.uneven(30000, 4000, seed=9)
    data, offs, lens, var = _to_dev(b)
    _say("repeat + permutation invariance")
    a = kb.keccak_batch_mixed(var, data, offs, lens)
    c = kb.keccak_batch_mixed(var, data, offs, lens)
    perm = torch.randperm(b.n, generator=torch.Generator().manual_seed(1)).cuda()
    p = kb.keccak_batch_mixed(var[perm].contiguous(), data, offs[perm].contiguous(),
                              lens[perm].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    assert torch.equal(p, a[perm])


def test_timing_brackets_only_the_selected_kinds(kb, o2):
    import torch
    b = wl.uneven(3000, 3000, seed=13)
    data, offs, lens, _ = _to_dev(b)
    _say("timing kinds: first pass only, then every kind")
    kb.timing_enable(True, kinds=["first_pass"])
    for _ in range(3):
        out = kb.keccak_batch(1, data, offs, lens)
    torch.cuda.synchronize()
    ms, n = kb.timing_read()
    assert n == 3 and ms > 0.0
    assert kb.timing_read("first_pass")[1] == 3
    assert kb.timing_read("schedule") == (0.0, 0) and kb.timing_read("second_pass") == (0.0, 0)
    kb.timing_enable(True)
    out = kb.keccak_batch(1, data, offs, lens)
    torch.cuda.synchronize()
    assert kb.timing_read("first_pass")[1] == 1 and kb.timing_read("second_pass")[1] == 1
    assert kb.timing_read("schedule")[1] == 2
    kb.timing_enable(False)
    want = o2.sha3_batch(256, b.data, b.offsets, b.lengths)
    assert _mismatches(out.cpu().numpy(), want)[1] == 0


@pytest.mark.parametrize("v", [0, 1, 2, 3])
def test_merkle_small_trees(kb, o2, v):
    import torch
    rng = np.random.Generator(np.random.PCG64(40 + v))
    # (leaf size, bytes cut from the end when there are several leaves): the
    # last three keep the leaves and the total whole 8-byte words, the form
    # whose blocks load straight into registers
    for n_leaves in list(range(1, 18)) + [64, 65, 1000]:
        for leaf, cut in ((1, 0), (13, 4), (4096, 1365), (8, 0), (136, 8), (4096, 1360)):
            total = n_leaves * leaf - (cut if n_leaves > 1 else 0)
            data = rng.integers(0, 256, max(total, 0), dtype=np.uint8)
            _say("merkle", v, n_leaves, leaf, total)
            d = torch.from_numpy(data).cuda() if total else torch.zeros(0, dtype=torch.uint8, device="cuda")
            got = kb.merkle_root(v, d, leaf)
            torch.cuda.synchronize()
            assert got.cpu().numpy().tobytes() == o2.merkle_root(8 * DIGEST[v], data, leaf)
    _say("merkle whole words at an odd address")
    data = rng.integers(0, 256, 64 * 136 + 1, dtype=np.uint8)
    d = torch.from_numpy(data).cuda()[1:]  # 8-byte multiples, data pointer not 8-byte aligned
    got = kb.merkle_root(v, d, 136)
    torch.cuda.synchronize()
    assert got.cpu().numpy().tobytes() == o2.merkle_root(8 * DIGEST[v], data[1:], 136)
    _say("merkle empty input")
    d = torch.zeros(0, dtype=torch.uint8, device="cuda")
    got = kb.merkle_root(v, d, 64)
    torch.cuda.synchronize()
    assert got.cpu().numpy().tobytes() == o2.merkle_root(8 * DIGEST[v], np.zeros(0, np.uint8), 64)


@pytest.mark.parametrize("v", [0, 3])
def test_merkle_top_workgroup_boundaries(kb, o2, v):
    # the leaf launch reduces one level, then the last workgroup takes at most
    # 1024 nodes: 2047 and 2048 leaves give it 1024 (the first level one pair
    # per thread), 2049 gives 1025 and a middle launch first, 4096 gives 2048;
    # leaf sizes 1 (staged loads) and 8 (whole words, LDS-direct loads)
    import torch
    rng = np.random.Generator(np.random.PCG64(70 + v))
    for n_leaves in (2047, 2048, 2049, 4096):
        for leaf in (1, 8):
            data = rng.integers(0, 256, n_leaves * leaf, dtype=np.uint8)
            _say("merkle top", v, n_leaves, leaf)
            got = kb.merkle_root(v, torch.from_numpy(data).cuda(), leaf)
            torch.cuda.synchronize()
            assert got.cpu().numpy().tobytes() == o2.merkle_root(8 * DIGEST[v], data, leaf)


@pytest.mark.parametrize("v", [1, 3])
def test_merkle_deep_trees(kb, o2, v):
    # more than 2^11 leaves: more than 1024 nodes remain after the leaf
    # launch's one level, so middle launches (up to 8 levels each, the
    # narrowest in the five-lane and wide forms) run before the last
    # workgroup; odd counts at most levels carry unpaired nodes up
    import torch
    rng = np.random.Generator(np.random.PCG64(60 + v))
    for n_leaves, leaf in ((300_001, 1), (2**19 + 3, 5)):
        data = rng.integers(0, 256, n_leaves * leaf - 2 if leaf > 2 else n_leaves * leaf,
                            dtype=np.uint8)
        _say("merkle deep", v, n_leaves, leaf, data.size)
        got = kb.merkle_root(v, torch.from_numpy(data).cuda(), leaf)
        torch.cuda.synchronize()
        assert got.cpu().numpy().tobytes() == o2.merkle_root(8 * DIGEST[v], data, leaf)


@pytest.mark.parametrize("b", [25, 50, 100, 200, 400, 800, 1600])
def test_keccak_p_every_width(kb, o2, b):
    # Keccak-p[b, n_r] in place on packed b-bit states against the bit-level
    # oracle, for one round, the full 12+2l, a reduced count and more rounds
    # than 12+2l (negative round indices)
    import torch
    from oracle import keccak_ref as ref
    w, l = ref.width_params(b)
    nbytes = (b + 7) // 8
    rng = np.random.Generator(np.random.PCG64(100 + b))
    n = 257 if b < 1600 else 33
    states = rng.integers(0, 256, (n, nbytes), dtype=np.uint8)
    if b % 8:
        states[:, -1] &= (1 << (b % 8)) - 1
    for nr in sorted({1, 12 + 2 * l, max(1, 12 + 2 * l - 3), 12 + 2 * l + 7}):
        _say("keccak_p", b, nr)
        d = torch.from_numpy(states.copy()).cuda()
        kb.keccak_p_batch(b, nr, d)
        got = d.cpu().numpy()
        for s in range(n):
            bits = np.unpackbits(states[s], bitorder="little")[:b]
            want = np.packbits(np.concatenate([ref.keccak_p(bits, b, nr),
                                               np.zeros(8 * nbytes - b, np.uint8)]),
                               bitorder="little")
            assert np.array_equal(got[s], want), (b, nr, s)
    if b == 1600:
        _say("keccak_p 1600 x 24 against the lane-level oracle")
        many = rng.integers(0, 256, (3000, 200), dtype=np.uint8)
        d = torch.from_numpy(many.copy()).cuda()
        kb.keccak_p_batch(1600, 24, d)
        got = d.cpu().numpy()
        for s in range(0, 3000, 7):
            assert got[s].tobytes() == o2.keccak_f1600(many[s].tobytes()), s


# --------------------------------------------------------------------------
# Full-size workloads, in the launch configuration the benchmark times
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["persistent", "plain"])
def test_full_uniform_2p24x64(kb, o2, mode):
    # the benchmarked batch, every one of its 2^24 digests against the oracle
    import torch
    b = wl.uniform(1 << 24, 64, seed=2)
    _say("full 2^24 x 64B sha3_256", mode)
    data, offs, lens, _ = _to_dev(b)
    kb.reserve(b.n)
    out = kb.keccak_batch(1, data, offs, lens, mode=mode)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    del data, offs, lens, out
    want = o2.sha3_batch(256, b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)


def test_full_uneven_2p20_mixed(kb, o2):
    import torch
    b = wl.uneven(1 << 20, 16384, seed=3)
    _say("full uneven 2^20 mixed persistent + plain")
    data, offs, lens, var = _to_dev(b)
    got = kb.keccak_batch_mixed(var, data, offs, lens)
    plain = kb.keccak_batch_mixed(var, data, offs, lens, mode="plain")
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert (plain.cpu().numpy() == got).all()
    want = o2.sha3_batch_mixed(b.variants, b.data, b.offsets, b.lengths)
    assert _mismatches(got, want)[1] == 0, _mismatches(got, want)


def test_full_merkle_1gib(kb, o2):
    import torch
    data = wl.merkle(1 << 30, seed=5)
    _say("full merkle 1 GiB / 4 KiB leaves")
    d = torch.from_numpy(data).cuda()
    got = kb.merkle_root(1, d, 4096)
    torch.cuda.synchronize()
    assert got.cpu().numpy().tobytes() == o2.merkle_root(256, data, 4096)


@pytest.mark.parametrize("security", [128, 256])
@pytest.mark.parametrize("mode", ["persistent", "plain", "split", "wide", "pair"])
def test_shake_xof(kb, o2, security, mode):
    import torch
    R = 168 if security == 128 else 136
    b = wl.explicit(list(range(0, 2 * R + 3)) + [5000, 0, 1], seed=60 + security, gap=1, lead=3)
    data, offs, lens, _ = _to_dev(b)
    # lengths below, at and above one rate, and several squeezes; odd lengths
    # take the byte-wise stores
    for out_len in (1, 3, 32, R - 1, R, R + 1, 3 * R + 5, 3 * R + 8):
        _say("shake", security, mode, "out_len", out_len)
        got = kb.keccak_batch_xof(security, data, offs, lens, out_len, mode=mode)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        for i in range(b.n):
            m = b.data[b.offsets[i]:b.offsets[i] + b.lengths[i]].tobytes()
            assert got[i].tobytes() == o2.shake(security, m, out_len), (out_len, i)
