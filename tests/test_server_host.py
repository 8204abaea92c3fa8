"""The serving engine's admission, step formation and completion logic, run
on the CPU: the step executor is a callback backed by the CPU oracle, so no
GPU is touched.  (The GPU path of the same engine is in test_gpu_serving.py.)"""

import os
import threading

import numpy as np
import pytest

from paper_1902_05320_amd import workloads as wl


@pytest.fixture(scope="module")
def kb():
    from paper_1902_05320_amd import kbatch
    if not os.path.exists(kbatch.LIB_PATH):
        pytest.skip("libkbatch.so not built")
    kbatch.load_library()
    return kbatch


def _oracle_executor(o2, pool, calls):
    def run(var, offs, lens):
        calls.append(int(var.size))
        return o2.sha3_batch_mixed(var, pool, offs, lens, threads=2)
    return run


def test_server_batches_fifo_and_matches_alone(kb, o2):
    pool = wl.random_bytes(wl.rng_for(44), 1 << 16)
    calls = []
    srv = kb.Server(None, max_step_msgs=100, steps_in_flight=2,
                    executor=_oracle_executor(o2, pool, calls), pool_bytes=pool.size)
    rng = np.random.Generator(np.random.PCG64(45))
    reqs = {}
    for _ in range(120):
        k = int(rng.integers(1, 61))
        lens = rng.integers(0, 700, k)
        offs = rng.integers(0, pool.size - 700, k)
        var = int(rng.choice([1, 3]))
        rid = srv.submit(var, offs, lens)
        reqs[rid] = (var, offs, lens)
    # larger than a step: rejected at submit
    with pytest.raises(kb.KbError) as ei:
        srv.submit(1, np.zeros(101, np.uint64), np.zeros(101, np.uint64))
    assert ei.value.code == kb.KB_ENOMEM
    got = {}
    while len(got) < len(reqs):
        for rid in srv.poll(wait_ms=100):
            var, offs, lens = reqs[rid]
            got[rid] = srv.result(rid, offs.size)
    st = srv.stats()
    srv.close()
    assert st["completed"] == 120 and st["rejected"] == 1 and st["pending"] == 0
    assert 1 < st["steps"] <= 120 and st["max_step_msgs_seen"] <= 100
    assert max(calls) <= 100 and sum(calls) == sum(o.size for _, o, _ in reqs.values())
    for rid, (var, offs, lens) in reqs.items():
        digests, lat = got[rid]
        alone = o2.sha3_batch_mixed(np.full(offs.size, var, np.uint8), pool, offs, lens)
        assert np.array_equal(digests, alone), rid
        assert lat >= 0.0


def test_server_accepts_concurrent_submitters(kb, o2):
    pool = wl.random_bytes(wl.rng_for(46), 1 << 14)
    srv = kb.Server(None, max_step_msgs=64, steps_in_flight=3,
                    executor=_oracle_executor(o2, pool, []), pool_bytes=pool.size)
    ids = []
    lock = threading.Lock()

    def submitter(seed):
        rng = np.random.Generator(np.random.PCG64(seed))
        for _ in range(25):
            k = int(rng.integers(1, 20))
            rid = srv.submit(1, rng.integers(0, pool.size - 100, k), rng.integers(0, 100, k))
            with lock:
                ids.append((rid, k))

    ts = [threading.Thread(target=submitter, args=(s,)) for s in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    done = set()
    while len(done) < len(ids):
        done.update(srv.poll(wait_ms=100))
    assert len({rid for rid, _ in ids}) == 100
    for rid, k in ids:
        d, _ = srv.result(rid, k)
        assert d.shape == (k, 64) and d[:, 32:].sum() == 0  # SHA3-256: zero past 32 bytes
    srv.close()


def test_server_rejects_bad_requests(kb):
    srv = kb.Server(None, max_step_msgs=8, steps_in_flight=1,
                    executor=lambda v, o, l: np.zeros((v.size, 64), np.uint8), pool_bytes=100)
    with pytest.raises(kb.KbError):
        srv.submit(1, [90], [20])  # outside the pool
    with pytest.raises(ValueError):
        srv.submit(7, [0], [1])  # not a SHA-3 variant
    rid = srv.submit(1, [0], [100])
    while rid not in srv.poll(wait_ms=100):
        pass
    d, _ = srv.result(rid, 1)
    assert not d.any()
    srv.close()


def test_failed_step_is_reported(kb):
    def boom(v, o, l):
        raise RuntimeError("executor failure")
    srv = kb.Server(None, max_step_msgs=8, steps_in_flight=1, executor=boom, pool_bytes=100)
    rid = srv.submit(1, [0], [10])
    with pytest.raises(kb.KbError):
        for _ in range(50):
            if rid in srv.poll(wait_ms=100):
                srv.result(rid, 1)
    srv.close()


def test_server_admits_by_byte_budget(kb, o2):
    # a step takes requests while both its message slots and its byte budget
    # last; a request with more bytes than a step holds is rejected at submit
    pool = wl.random_bytes(wl.rng_for(46), 1 << 16)
    calls = []

    def run(var, offs, lens):
        calls.append(int(lens.sum()))
        return o2.sha3_batch_mixed(var, pool, offs, lens, threads=2)

    srv = kb.Server(None, max_step_msgs=1000, steps_in_flight=1, executor=run,
                    pool_bytes=pool.size, max_step_bytes=5000)
    rng = np.random.Generator(np.random.PCG64(47))
    reqs = {}
    for _ in range(60):
        k = int(rng.integers(1, 20))
        lens = rng.integers(0, 250, k)
        offs = rng.integers(0, pool.size - 250, k)
        reqs[srv.submit(1, offs, lens)] = (offs, lens)
    with pytest.raises(kb.KbError) as ei:
        srv.submit(1, np.zeros(30, np.uint64), np.full(30, 200, np.uint64))
    assert ei.value.code == kb.KB_ENOMEM
    got = {}
    while len(got) < len(reqs):
        for rid in srv.poll(wait_ms=100):
            got[rid] = srv.result(rid, reqs[rid][0].size)[0]
    st = srv.stats()
    srv.close()
    assert st["rejected"] == 1 and max(calls) <= 5000 and st["steps"] > 1
    assert sum(calls) == sum(int(l.sum()) for _, l in reqs.values())
    for rid, (offs, lens) in reqs.items():
        assert np.array_equal(got[rid], o2.sha3_batch_mixed(np.ones(offs.size, np.uint8), pool, offs, lens))
