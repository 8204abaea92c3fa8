"""GPU: the serving engine (every request's digests equal the same request
hashed alone, and the oracle), the autotuner's parity gate, graph replays
(each replay equals the eager result, with eager work in between), and the
measurement probes the benchmark reports."""

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


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("graphs", [True, False])
def test_server_results_equal_alone_and_oracle(kb, o2, graphs):
    import torch
    pool_np = wl.random_bytes(wl.rng_for(50), 1 << 24)
    pool = torch.from_numpy(pool_np).cuda()
    _say("server: 400 requests, steps of 4096 messages, 2 in flight, graphs", graphs)
    srv = kb.Server(pool, max_step_msgs=4096, steps_in_flight=2, graphs=graphs)
    rng = np.random.Generator(np.random.PCG64(51))
    reqs = {}
    for _ in range(400):
        k = int(rng.integers(1, 300))
        lens = wl.log_uniform_lengths(rng, k, 8192)
        offs = rng.integers(0, pool_np.size - 8192, k)
        var = int(rng.choice([1, 3]))
        reqs[srv.submit(var, offs, lens)] = (var, offs, lens)
    got = {}
    while len(got) < len(reqs):
        for rid in srv.poll(wait_ms=200):
            got[rid] = srv.result(rid, reqs[rid][1].size)
    st = srv.stats()
    srv.close()
    assert st["completed"] == 400 and st["steps"] >= 2 and st["max_step_msgs_seen"] <= 4096
    _say("server: compare with each request alone")
    for i, (rid, (var, offs, lens)) in enumerate(reqs.items()):
        o = torch.from_numpy(offs.astype(np.int64)).cuda()
        ln = torch.from_numpy(lens.astype(np.int64)).cuda()
        alone = kb.keccak_batch_mixed(torch.full((offs.size,), var, dtype=torch.uint8, device="cuda"),
                                      pool, o, ln).cpu().numpy()
        assert np.array_equal(got[rid][0], alone), rid
        if i % 20 == 0:
            want = o2.sha3_batch_mixed(np.full(offs.size, var, np.uint8), pool_np, offs, lens)
            assert np.array_equal(alone, want), rid


def test_server_stream_at_full_request_size_matches_oracle(kb, o2):
    # requests the size of the serving stream's (1..4096 messages, lengths
    # log-uniform in [0, 64 KiB], SHA3-256 or SHA3-512), steps of up to 65536
    # messages, two in flight, submitted in bursts while steps run; every
    # digest of every request against the oracle
    import time
    import torch
    pool_np, reqs = wl.serving_stream(0.16, 2000.0, 1 << 28, seed=56)
    assert len(reqs) >= 300
    pool = torch.from_numpy(pool_np).cuda()
    _say("server: full-size stream,", len(reqs), "requests,",
         sum(r.lengths.size for r in reqs), "messages")
    srv = kb.Server(pool, max_step_msgs=1 << 16, steps_in_flight=2)
    ids = {}
    for i, r in enumerate(reqs):
        ids[srv.submit(r.variant, r.offsets, r.lengths)] = i
        if i % 40 == 39:
            time.sleep(0.002)  # the next burst arrives while steps run
    got = {}
    while len(got) < len(ids):
        for rid in srv.poll(wait_ms=200):
            got[ids[rid]] = srv.result(rid, reqs[ids[rid]].lengths.size)[0]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["rejected"] == 0 and st["steps"] >= 2
    _say("server: oracle over every request")
    var = np.concatenate([np.full(r.lengths.size, r.variant, np.uint8) for r in reqs])
    offs = np.concatenate([r.offsets for r in reqs])
    lens = np.concatenate([r.lengths for r in reqs])
    want = o2.sha3_batch_mixed(var, pool_np, offs, lens)
    at = 0
    for i, r in enumerate(reqs):
        k = r.lengths.size
        assert np.array_equal(got[i], want[at:at + k]), (i, r.variant, k)
        at += k


def test_autotune_candidates_pass_parity(kb, o2):
    import torch
    b = wl.uneven(30000, 6000, seed=52)
    data = torch.from_numpy(b.data).cuda()
    offs = torch.from_numpy(b.offsets).cuda()
    lens = torch.from_numpy(b.lengths).cuda()
    var = torch.from_numpy(b.variants).cuda()
    _say("autotune mixed")
    tile, ms, rejected = kb.autotune(-1, data, offs, lens, variants=var, reps=2)
    assert rejected == 0 and ms > 0 and tile.steps_per_item >= 0
    got = kb.keccak_batch_mixed(var, data, offs, lens, tile=tile).cpu().numpy()
    assert np.array_equal(got, o2.sha3_batch_mixed(b.variants, b.data, b.offsets, b.lengths))
    _say("autotune sha3_256")
    tile, ms, rejected = kb.autotune(1, data, offs, lens, reps=2)
    assert rejected == 0
    got = kb.keccak_batch(1, data, offs, lens, tile=tile).cpu().numpy()
    assert np.array_equal(got, o2.sha3_batch(256, b.data, b.offsets, b.lengths))


def test_cached_tile_is_chosen_and_matches_oracle(kb, o2, tmp_path, monkeypatch):
    """A tile stored in the tune cache is the one a batch call runs once
    KBATCH_TUNE names the file, and its digests equal the oracle's."""
    import torch
    b = wl.uneven(20000, 9000, seed=53)
    data = torch.from_numpy(b.data).cuda()
    offs = torch.from_numpy(b.offsets).cuda()
    lens = torch.from_numpy(b.lengths).cuda()
    var = torch.from_numpy(b.variants).cuda()
    path = str(tmp_path / "tune.json")
    _say("autotune mixed into a cache file")
    tuned, _, rejected = kb.autotune(-1, data, offs, lens, variants=var, reps=1, cache=path)
    assert rejected == 0
    assert kb.tune_lookup(-1, b.n, path=path).as_dict() == tuned.as_dict()
    # a distinctive tile for SHA3-512 over the same batch: direct staging, two
    # waves per SIMD, every class of 16 or more blocks in the wide split tail
    t = kb.Tile()
    t.waves_per_simd, t.steps_per_item, t.staging = 2, 2, kb.STAGING_DIRECT
    for c in range(kb.NB_CLASSES):
        t.class_threads[c] = kb.THREADS_WIDE if c >= 4 else 1
        t.class_steps[c] = 1 + c
    kb.tune_store(path, 3, b.n, t, 1.0)
    monkeypatch.setenv("KBATCH_TUNE", path)
    for v, want in ((3, o2.sha3_batch(512, b.data, b.offsets, b.lengths)),
                    (-1, o2.sha3_batch_mixed(b.variants, b.data, b.offsets, b.lengths))):
        _say("cached tile, variant", v)
        if v == -1:
            got = kb.keccak_batch_mixed(var, data, offs, lens)
        else:
            got = kb.keccak_batch(v, data, offs, lens)
        used, cached = kb.last_tile()
        assert cached and used.as_dict() == (t if v == 3 else tuned).as_dict()
        assert np.array_equal(got.cpu().numpy(), want)
    monkeypatch.delenv("KBATCH_TUNE")
    kb.keccak_batch(3, data, offs, lens)
    used, cached = kb.last_tile()
    assert not cached and used.waves_per_simd == 0


@pytest.mark.parametrize("mode", ["persistent", "plain", "split", "wide", "pair"])
def test_graph_replays_equal_eager(kb, mode):
    import torch
    b = wl.uneven(20000, 5000, seed=53)
    data = torch.from_numpy(b.data).cuda()
    offs = torch.from_numpy(b.offsets).cuda()
    lens = torch.from_numpy(b.lengths).cuda()
    var = torch.from_numpy(b.variants).cuda()
    eager = kb.keccak_batch_mixed(var, data, offs, lens, mode=mode)
    out = torch.zeros((b.n, 64), dtype=torch.uint8, device="cuda")
    _say("graph capture", mode)
    g = kb.graph_batch(-1, data, offs, lens, out, variants=var, mode=mode)
    for rep in range(4):
        out.zero_()
        # eager work between replays
        other = kb.keccak_batch(1, data, offs[:1000].contiguous(), lens[:1000].contiguous())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        del other
    g.close()


def test_counted_graph_replays_each_count(kb):
    # one capture over a fixed capacity; each replay reads the message count
    # from device memory; every replay's digests (up to that count) equal the
    # eager ones, and the slots past the count are left alone
    import torch
    b = wl.uneven(30000, 6000, seed=57)
    data = torch.from_numpy(b.data).cuda()
    offs = torch.from_numpy(b.offsets).cuda()
    lens = torch.from_numpy(b.lengths).cuda()
    var = torch.from_numpy(b.variants).cuda()
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.zeros((b.n, 64), dtype=torch.uint8, device="cuda")
    eager = kb.keccak_batch_mixed(var, data, offs, lens)
    _say("counted graph")
    g = kb.graph_counted(-1, data, offs, lens, count, out, variants=var)
    for n in (b.n, 1, 0, 12345, 64, b.n + 100, 29999):
        out.fill_(0xA5)
        count.fill_(n)
        other = kb.keccak_batch(1, data, offs[:500].contiguous(), lens[:500].contiguous())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        k = min(n, b.n)
        assert torch.equal(out[:k], eager[:k]), n
        assert bool((out[k:] == 0xA5).all()), n
        del other
    g.close()


def test_merkle_graph_replays(kb, o2):
    import torch
    data_np = wl.merkle(3_000_001, seed=54)
    data = torch.from_numpy(data_np).cuda()
    want = o2.merkle_root(256, data_np, 4096)
    root = torch.zeros(32, dtype=torch.uint8, device="cuda")
    _say("merkle graph")
    g = kb.graph_merkle(1, data, 4096, root)
    for rep in range(3):
        root.zero_()
        kb.merkle_root(3, data, 1000)  # eager work on the same stream
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert root.cpu().numpy().tobytes() == want, rep
    g.close()


@pytest.mark.parametrize("n_leaves,leaf", [(17, 64), (3000, 100), (2**18 + 1, 8)])
def test_merkle_graph_sha3_512_odd_leaf_counts(kb, o2, n_leaves, leaf):
    # a captured tree owns a node buffer sized by the level walk; SHA3-512
    # at 2^k + 1 and other odd leaf counts needs more than two digests per leaf
    import torch
    data_np = wl.merkle(n_leaves * leaf - 3, seed=55)
    data = torch.from_numpy(data_np).cuda()
    want = o2.merkle_root(512, data_np, leaf)
    root = torch.zeros(64, dtype=torch.uint8, device="cuda")
    _say("merkle graph sha3_512", n_leaves, leaf)
    g = kb.graph_merkle(3, data, leaf, root)
    for rep in range(2):
        root.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert root.cpu().numpy().tobytes() == want, rep
    g.close()
    assert kb.merkle_root(3, data, leaf).cpu().numpy().tobytes() == want


def test_probes_report_rates(kb):
    _say("probe_perm, probe_valu")
    g, w = kb.probe_perm(iters=50)
    assert w >= 1 and 0.1 < g < 1000, (g, w)
    g1, w1 = kb.probe_perm(iters=50, waves_per_simd=1)
    assert w1 == 1 and 0.0 < g1 <= 1.5 * g, (g1, g)
    tops, mhz = kb.probe_valu(iters=2000)
    assert 1.0 < tops < 200.0 and 100.0 < mhz < 5000.0, (tops, mhz)
