"""Seeded input generators: deterministic, in range, packed as documented."""

import numpy as np

from paper_1902_05320_amd import workloads as wl


def test_uniform_is_deterministic_and_packed():
    a = wl.uniform(100, 64, seed=1)
    b = wl.uniform(100, 64, seed=1)
    assert np.array_equal(a.data, b.data)
    assert a.data.size == 6400
    assert np.array_equal(a.offsets, np.arange(100) * 64)
    assert (a.lengths == 64).all()
    c = wl.uniform(100, 64, seed=2)
    assert not np.array_equal(a.data, c.data)


def test_uneven_lengths_log_uniform_in_range():
    b = wl.uneven(20000, 16384, seed=3)
    assert b.lengths.min() >= 0 and b.lengths.max() <= 16384
    assert (b.lengths == 0).any()
    assert np.array_equal(b.offsets[1:], np.cumsum(b.lengths)[:-1])
    assert b.data.size == int(b.lengths.sum())
    assert set(np.unique(b.variants)) == {0, 1, 2, 3}
    # log-uniform: the median is near sqrt(16386) - 1
    assert 80 < np.median(b.lengths) < 180


def test_serving_stream_is_poisson_like():
    pool, reqs = wl.serving_stream(2.0, 500.0, 1 << 20, seed=4, max_len=4096)
    assert 800 < len(reqs) < 1200
    arr = np.array([r.arrival_s for r in reqs])
    assert (np.diff(arr) > 0).all()
    for r in reqs[:50]:
        assert 1 <= r.lengths.size <= 4096
        assert (r.offsets + r.lengths <= pool.size).all()
        assert r.variant in (1, 3)
