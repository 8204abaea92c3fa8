"""Seeded synthetic inputs for batch hashing.

This module only draws random bytes, lengths, variants and arrival times; it
holds none of the hashing arithmetic, so the HIP path and the CPU oracle can
both be fed from it.  Everything is drawn from ``numpy.random.Generator(
PCG64(seed))``; messages are packed back to back in index order, so offsets
are the exclusive prefix sum of the lengths (and unaligned whenever lengths
vary).

Workloads (the paper hashes large batches of short, equal-length messages,
Section 4.3; the others stretch that regime):

* ``uniform``   -- n messages of exactly L bytes (4096 x 64 B and 2^24 x 64 B).
* ``uneven``    -- n messages with lengths log-uniform in [0, max_len] bytes
  (L = floor((max_len + 2)^U) - 1, U ~ U[0, 1)), variant uniform over the
  four SHA-3 digest sizes.
* ``merkle``    -- one seeded byte buffer cut into fixed-size leaves.
* ``serving``   -- a Poisson request stream; each request holds 1..4096
  messages with log-uniform lengths in [0, 64 KiB] sliced from a shared pool.
"""

from __future__ import annotations

import dataclasses

import numpy as np

VARIANT_NAMES = ("sha3_224", "sha3_256", "sha3_384", "sha3_512")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_bytes(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform random bytes.  Large buffers are drawn in 64 MiB pieces to
    bound the temporary memory numpy needs."""
    out = np.empty(n, dtype=np.uint8)
    step = 1 << 26
    for s in range(0, n, step):
        e = min(n, s + step)
        out[s:e] = rng.integers(0, 256, size=e - s, dtype=np.uint8)
    return out


@dataclasses.dataclass
class Batch:
    data: np.ndarray       # uint8, messages packed back to back
    offsets: np.ndarray    # int64 byte offsets into data
    lengths: np.ndarray    # int64 byte lengths
    variants: np.ndarray   # uint8 in 0..3 (SHA3-224/256/384/512)
    seed: int
    name: str

    @property
    def n(self) -> int:
        return int(self.offsets.size)

    @property
    def total_bytes(self) -> int:
        return int(self.lengths.sum()) if self.n else 0


def packed_offsets(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(lengths.size, dtype=np.int64)
    if lengths.size > 1:
        np.cumsum(lengths[:-1], out=off[1:])
    return off


def uniform(n: int, length: int, seed: int, variant: int = 1) -> Batch:
    """n messages of exactly `length` bytes, uniform random bytes."""
    rng = rng_for(seed)
    data = random_bytes(rng, n * length)
    lengths = np.full(n, length, dtype=np.int64)
    return Batch(data, np.arange(n, dtype=np.int64) * length, lengths,
                 np.full(n, variant, dtype=np.uint8), seed, f"uniform_{n}x{length}B")


def log_uniform_lengths(rng: np.random.Generator, n: int, max_len: int) -> np.ndarray:
    """L = floor((max_len + 2)^U) - 1 with U ~ U[0, 1): log-uniform in
    [0, max_len], zero-length messages included."""
    u = rng.random(n)
    lengths = np.floor(np.power(float(max_len + 2), u)).astype(np.int64) - 1
    return np.clip(lengths, 0, max_len)


def uneven(n: int, max_len: int, seed: int, variant: int | None = None) -> Batch:
    """Log-uniform lengths in [0, max_len]; variant uniform over the four
    digest sizes unless fixed."""
    rng = rng_for(seed)
    lengths = log_uniform_lengths(rng, n, max_len)
    if variant is None:
        variants = rng.integers(0, 4, size=n, dtype=np.uint8)
    else:
        variants = np.full(n, variant, dtype=np.uint8)
    data = random_bytes(rng, int(lengths.sum()))
    return Batch(data, packed_offsets(lengths), lengths, variants, seed,
                 f"uneven_{n}x[0,{max_len}]B")


def explicit(lengths, seed: int, variant: int | np.ndarray = 1, gap: int = 0,
             lead: int = 0) -> Batch:
    """Messages with the given lengths, packed with `gap` spare bytes between
    them and `lead` bytes before the first (to force unaligned offsets)."""
    rng = rng_for(seed)
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.size
    offs = np.zeros(n, dtype=np.int64)
    pos = lead
    for i in range(n):
        offs[i] = pos
        pos += int(lengths[i]) + gap
    data = random_bytes(rng, max(pos, 1))
    if np.isscalar(variant):
        variants = np.full(n, int(variant), dtype=np.uint8)
    else:
        variants = np.asarray(variant, dtype=np.uint8)
    return Batch(data, offs, lengths, variants, seed, f"explicit_{n}")


def merkle(total_len: int, seed: int) -> np.ndarray:
    """One seeded buffer for tree hashing."""
    return random_bytes(rng_for(seed), total_len)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    variant: int
    offsets: np.ndarray   # into the shared pool
    lengths: np.ndarray


def serving_stream(duration_s: float, rate_hz: float, pool_bytes: int, seed: int,
                   max_msgs: int = 4096, max_len: int = 65536,
                   variants=(1, 3)) -> tuple[np.ndarray, list[Request]]:
    """A Poisson request stream over a shared random byte pool.

    Arrival gaps are exponential with mean 1/rate_hz.  Each request has
    k ~ U{1..max_msgs} messages whose lengths are log-uniform in
    [0, max_len], each sliced at a uniform random offset of the pool, and a
    variant drawn uniformly from `variants`.
    """
    rng = rng_for(seed)
    pool = random_bytes(rng, pool_bytes)
    reqs: list[Request] = []
    t = 0.0
    rid = 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        k = int(rng.integers(1, max_msgs + 1))
        lengths = log_uniform_lengths(rng, k, max_len)
        offs = rng.integers(0, pool_bytes - max_len, size=k, dtype=np.int64)
        var = int(variants[int(rng.integers(0, len(variants)))])
        reqs.append(Request(rid, t, var, offs, lengths))
        rid += 1
    return pool, reqs
