"""Pins for the CPU oracles: each test checks the oracle against something
other than itself -- the paper's Table 1, Python's hashlib (an independent
SHA-3 implementation that every SHA-3 digest reduces to), closed forms,
invariants of the definitions, inverses of the step mappings and brute force
on tiny inputs.  CPU only."""

import hashlib
import os

import numpy as np
import pytest

from oracle import keccak_ref as ref

HERE = os.path.dirname(os.path.abspath(__file__))
HASHLIB = {224: hashlib.sha3_224, 256: hashlib.sha3_256, 384: hashlib.sha3_384,
           512: hashlib.sha3_512}
RATES = {224: 144, 256: 136, 384: 104, 512: 72}


def _rand_bytes(seed, n):
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 256, n, dtype=np.uint8).tobytes()


# --------------------------------------------------------------------------
# Table 1
# --------------------------------------------------------------------------

def test_table1_widths_match_golden():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_widths.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    assert [r[0] for r in rows] == list(ref.WIDTHS)
    for b, w, l in rows:
        assert ref.width_params(b) == (w, l)


def test_rate_is_1600_minus_twice_digest():
    # Section 3.3: c = 2d, r = 1600 - c
    for d, r in RATES.items():
        assert ref.rate_bytes(d) == r


# --------------------------------------------------------------------------
# Whole SHA-3 against hashlib (pins rho, iota/rc, padding, byte order)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [224, 256, 384, 512])
def test_o1_sha3_boundary_lengths_vs_hashlib(d):
    R = RATES[d]
    for L in (0, 1, 2, 7, 8, 9, R - 2, R - 1, R, R + 1, 2 * R - 1, 2 * R, 2 * R + 1):
        m = _rand_bytes(1000 + L, L)
        assert ref.sha3(d, m) == HASHLIB[d](m).digest(), (d, L)


def test_o1_single_byte_messages_vs_hashlib():
    for v in (0x00, 0x01, 0x06, 0x80, 0x86, 0xFF):
        m = bytes([v])
        for d in (224, 256, 384, 512):
            assert ref.sha3(d, m) == HASHLIB[d](m).digest()


def test_o1_shake_vs_hashlib():
    for L in (0, 1, 167, 168, 169):
        m = _rand_bytes(77 + L, L)
        assert ref.shake(128, m, 200) == hashlib.shake_128(m).digest(200)
    for L in (0, 135, 136, 137):
        m = _rand_bytes(88 + L, L)
        assert ref.shake(256, m, 300) == hashlib.shake_256(m).digest(300)


@pytest.mark.parametrize("d", [224, 256, 384, 512])
def test_o2_every_length_up_to_3R_vs_hashlib(o2, d):
    R = RATES[d]
    for L in range(0, 3 * R + 2):
        m = _rand_bytes(5000 + L, L)
        assert o2.sha3(d, m) == HASHLIB[d](m).digest(), (d, L)


def test_o2_all_one_byte_messages_vs_hashlib(o2):
    data = np.arange(256, dtype=np.uint8)
    offs = np.arange(256)
    lens = np.ones(256, dtype=np.int64)
    for d in (224, 256, 384, 512):
        out = o2.sha3_batch(d, data, offs, lens)
        for v in range(256):
            assert out[v].tobytes() == HASHLIB[d](bytes([v])).digest()


def test_o2_all_two_byte_messages_vs_hashlib(o2):
    vals = np.arange(65536, dtype=np.uint32)
    data = np.empty(2 * 65536, dtype=np.uint8)
    data[0::2] = vals & 0xFF
    data[1::2] = vals >> 8
    offs = np.arange(65536) * 2
    lens = np.full(65536, 2)
    out = o2.sha3_batch(256, data, offs, lens)
    for v in range(65536):
        assert out[v].tobytes() == hashlib.sha3_256(bytes([v & 0xFF, v >> 8])).digest()


def test_o2_random_long_messages_vs_hashlib(o2):
    rng = np.random.Generator(np.random.PCG64(9))
    lengths = rng.integers(0, 65537, size=48)
    data = rng.integers(0, 256, size=int(lengths.sum()), dtype=np.uint8)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    for d in (224, 256, 384, 512):
        out = o2.sha3_batch(d, data, offs, lengths)
        for i in range(lengths.size):
            m = data[offs[i]:offs[i] + lengths[i]].tobytes()
            assert out[i].tobytes() == HASHLIB[d](m).digest()


def test_o2_shake_vs_hashlib(o2):
    for L in (0, 1, 167, 168, 169, 1000):
        m = _rand_bytes(300 + L, L)
        assert o2.shake(128, m, 500) == hashlib.shake_128(m).digest(500)
        assert o2.shake(256, m, 500) == hashlib.shake_256(m).digest(500)


def test_o2_matches_o1(o2):
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(6):
        L = int(rng.integers(0, 400))
        m = rng.integers(0, 256, L, dtype=np.uint8).tobytes()
        d = int(rng.choice([224, 256, 384, 512]))
        assert o2.sha3(d, m) == ref.sha3(d, m)
    s = _rand_bytes(12, 200)
    assert o2.keccak_f1600(s) == ref.keccak_f1600_bytes(s)


# --------------------------------------------------------------------------
# Keccak-f[1600] on its own, through SHAKE128's squeeze phase
# --------------------------------------------------------------------------

def _shake128_padded_block(m: bytes) -> bytes:
    # M || 1111 || pad10*1 for a single 168-byte block, capacity zero
    assert len(m) < 168
    blk = bytearray(200)
    blk[:len(m)] = m
    blk[len(m)] ^= 0x1F
    blk[167] ^= 0x80
    return bytes(blk)


@pytest.mark.parametrize("impl", ["o1", "o2"])
def test_keccak_f_pinned_by_shake128_squeeze(o2, impl):
    f = ref.keccak_f1600_bytes if impl == "o1" else o2.keccak_f1600
    for L in (0, 5, 100, 167):
        m = _rand_bytes(40 + L, L)
        want = hashlib.shake_128(m).digest(168 * 3)
        s = _shake128_padded_block(m)
        for k in range(3):
            s = f(s)
            assert s[:168] == want[168 * k:168 * (k + 1)], (impl, L, k)


# --------------------------------------------------------------------------
# rho: offsets from the (x, y) recurrence
# --------------------------------------------------------------------------

def test_rho_walk_invariants():
    off = ref.rho_offsets(64)
    assert len(off) == 25
    assert off[(0, 0)] == 0
    walked = [k for k in off if k != (0, 0)]
    assert len(set(walked)) == 24
    vals = [off[k] for k in walked]
    assert len(set(vals)) == 24
    assert all(v not in (0, 32) for v in vals)
    # the offsets are the triangular numbers T(t+1) = (t+1)(t+2)/2 mod 64 in
    # walk order; their sum before the mod is sum of T(1..24) = 2600
    tri = sorted(((t + 1) * (t + 2) // 2) % 64 for t in range(24))
    assert sorted(vals) == tri


def test_rho_moves_each_lane_left_by_its_offset():
    rng = np.random.Generator(np.random.PCG64(3))
    A = rng.integers(0, 2, size=(5, 5, 64), dtype=np.uint8)
    out = ref.rho(A)
    off = ref.rho_offsets(64)
    for (x, y), s in off.items():
        # as 64-bit integers (bit z = A[x, y, z]), a left rotation by s
        v = int("".join(str(b) for b in A[x, y][::-1]), 2)
        wv = int("".join(str(b) for b in out[x, y][::-1]), 2)
        assert wv == ((v << s) | (v >> (64 - s))) & (2 ** 64 - 1) if s else wv == v


# --------------------------------------------------------------------------
# rc / RC from the LFSR
# --------------------------------------------------------------------------

def test_rc_sequence_has_minimal_period_255():
    seq = [ref.rc(t) for t in range(2 * 255)]
    assert seq[:255] == seq[255:]
    for p in (1, 3, 5, 15, 17, 51, 85):  # proper divisors of 255
        assert seq[:255] != (seq[p:255] + seq[:p])


def test_rc_lfsr_visits_every_nonzero_state():
    # x^8 + x^6 + x^5 + x^4 + 1 is primitive: the 8-bit register runs through
    # all 255 nonzero states.  Reconstruct states as windows of the output.
    seq = [ref.rc(t) for t in range(255 + 8)]
    windows = {tuple(seq[t:t + 8]) for t in range(255)}
    assert len(windows) == 255
    assert (0,) * 8 not in windows


def test_round_constants_only_use_bits_2j_minus_1():
    allowed = {2 ** j - 1 for j in range(7)}
    for ir in range(24):
        RC = ref.round_constant(ir, 64)
        assert set(np.nonzero(RC)[0]) <= allowed
    # round 0: rc(0..6) = 1, 0, 0, 0, 0, 0, 0 -> only bit 0 set
    assert list(np.nonzero(ref.round_constant(0, 64))[0]) == [0]


# --------------------------------------------------------------------------
# pad10*1 closed forms
# --------------------------------------------------------------------------

def test_pad_makes_a_block_multiple():
    for x in (1, 2, 3, 7, 8, 64, 576, 1088, 1152):
        for m in range(0, 3 * x + 3):
            P = ref.pad10star1(x, m)
            assert (m + P.size) % x == 0
            assert 2 <= P.size <= x + 1
            assert P[0] == 1 and P[-1] == 1 and not P[1:-1].any()


def test_block_count_closed_form():
    # SHA-3 byte messages: suffix (2 bits) + pad fit in the last byte, so the
    # padded message has floor(L / R) + 1 blocks.
    for d, R in RATES.items():
        for L in (0, R - 1, R, R + 1, 2 * R):
            m = 8 * L + 2
            assert (m + ref.pad10star1(8 * R, m).size) // (8 * R) == L // R + 1
        assert [L // R + 1 for L in (0, R - 1, R, R + 1, 2 * R)] == [1, 1, 2, 2, 3]


# --------------------------------------------------------------------------
# Step mappings are bijections: invert each on random states.  The inverses
# are written here from the definitions, independently of the oracle.
# --------------------------------------------------------------------------

def _theta_inverse(Ap):
    w = Ap.shape[2]
    # theta adds D(C) to every lane of a column; the column parities of the
    # output are C' = C + D(C) (five copies of D, five is odd).  Solve the
    # linear system (I + M) C = C' over GF(2), then A = A' + D(C).
    def D_of(C):
        return np.stack([C[(x - 1) % 5] ^ np.roll(C[(x + 1) % 5], 1) for x in range(5)])
    n = 5 * w
    Mcols = []
    for k in range(n):
        e = np.zeros(n, dtype=np.uint8)
        e[k] = 1
        C = e.reshape(5, w)
        Mcols.append((C ^ D_of(C)).reshape(n))
    M = np.array(Mcols, dtype=np.uint8).T  # column k = image of basis k
    Cp = np.bitwise_xor.reduce(Ap, axis=1).reshape(n)
    aug = np.concatenate([M, Cp[:, None]], axis=1)
    row = 0
    piv_cols = []
    for col in range(n):
        piv = next((r for r in range(row, n) if aug[r, col]), None)
        if piv is None:
            continue
        aug[[row, piv]] = aug[[piv, row]]
        for r in range(n):
            if r != row and aug[r, col]:
                aug[r] ^= aug[row]
        piv_cols.append(col)
        row += 1
    assert row == n, "theta is not invertible"
    C = aug[:, n].reshape(5, w)
    return Ap ^ D_of(C)[:, None, :]


def _rho_inverse(Ap):
    w = Ap.shape[2]
    out = Ap.copy()
    for (x, y), s in ref.rho_offsets(w).items():
        out[x, y] = np.roll(Ap[x, y], -s)
    return out


def _pi_inverse(Ap):
    out = np.zeros_like(Ap)
    for x in range(5):
        for y in range(5):
            out[(x + 3 * y) % 5, x] = Ap[x, y]
    return out


def _chi_inverse(Ap):
    # chi acts on each 5-bit row independently: invert by table lookup
    table = {}
    for v in range(32):
        a = [(v >> i) & 1 for i in range(5)]
        b = [a[i] ^ ((a[(i + 1) % 5] ^ 1) & a[(i + 2) % 5]) for i in range(5)]
        table[tuple(b)] = a
    assert len(table) == 32
    out = np.zeros_like(Ap)
    for y in range(5):
        for z in range(Ap.shape[2]):
            out[:, y, z] = table[tuple(int(t) for t in Ap[:, y, z])]
    return out


@pytest.mark.parametrize("b", [200, 1600])
def test_each_step_inverts_on_random_states(b):
    w, _ = ref.width_params(b)
    rng = np.random.Generator(np.random.PCG64(b))
    for _ in range(3):
        A = rng.integers(0, 2, size=(5, 5, w), dtype=np.uint8)
        assert np.array_equal(_theta_inverse(ref.theta(A)), A)
        assert np.array_equal(_rho_inverse(ref.rho(A)), A)
        assert np.array_equal(_pi_inverse(ref.pi(A)), A)
        assert np.array_equal(_chi_inverse(ref.chi(A)), A)
        for ir in (0, 5, 23):
            assert np.array_equal(ref.iota(ref.iota(A, ir), ir), A)


def test_full_round_inverts_round_by_round():
    rng = np.random.Generator(np.random.PCG64(21))
    A = rng.integers(0, 2, size=(5, 5, 64), dtype=np.uint8)
    B = A
    for ir in range(24):
        B = ref.rnd(B, ir)
    for ir in reversed(range(24)):
        B = _theta_inverse(_rho_inverse(_pi_inverse(_chi_inverse(ref.iota(B, ir)))))
    assert np.array_equal(B, A)


def test_state_string_mapping_eq1():
    S = np.arange(1600) % 2
    S = np.random.Generator(np.random.PCG64(2)).integers(0, 2, 1600, dtype=np.uint8)
    A = ref.string_to_state(S, 64)
    for (x, y, z) in ((0, 0, 0), (1, 0, 3), (0, 1, 0), (4, 4, 63), (2, 3, 17)):
        assert A[x, y, z] == S[64 * (5 * y + x) + z]
    assert np.array_equal(ref.state_to_string(A), S)


# --------------------------------------------------------------------------
# Batch semantics and tree mode
# --------------------------------------------------------------------------

def test_batch_is_order_independent(o2):
    rng = np.random.Generator(np.random.PCG64(31))
    n = 300
    lengths = rng.integers(0, 700, n)
    data = rng.integers(0, 256, int(lengths.sum()) + 64, dtype=np.uint8)
    offs = rng.integers(0, data.size - 700, n)  # overlapping slices allowed
    out = o2.sha3_batch(384, data, offs, lengths)
    perm = rng.permutation(n)
    out_p = o2.sha3_batch(384, data, offs[perm], lengths[perm])
    assert np.array_equal(out_p, out[perm])
    ref_list = ref.sha3_batch(384, data.tobytes(), offs[:3], lengths[:3])
    assert [out[i].tobytes() for i in range(3)] == ref_list


def test_mixed_batch_vs_hashlib(o2):
    rng = np.random.Generator(np.random.PCG64(41))
    n = 200
    lengths = rng.integers(0, 500, n)
    variants = rng.integers(0, 4, n).astype(np.uint8)
    data = rng.integers(0, 256, int(lengths.sum()), dtype=np.uint8)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    out = o2.sha3_batch_mixed(variants, data, offs, lengths)
    for i in range(n):
        d = (224, 256, 384, 512)[variants[i]]
        m = data[offs[i]:offs[i] + lengths[i]].tobytes()
        assert out[i, :d // 8].tobytes() == HASHLIB[d](m).digest()
        assert not out[i, d // 8:].any()


def _mth(leaf_hashes, H):
    """Merkle tree hash written as a recursion: split at the largest power of
    two below n (the left subtree is complete)."""
    n = len(leaf_hashes)
    if n == 1:
        return leaf_hashes[0]
    k = 1
    while 2 * k < n:
        k *= 2
    return H(_mth(leaf_hashes[:k], H) + _mth(leaf_hashes[k:], H))


@pytest.mark.parametrize("d", [256, 512])
def test_merkle_root_bruteforce(o2, d):
    H = lambda b: HASHLIB[d](b).digest()
    leaf = 7
    for n in range(1, 18):
        for tail in (0, 3):  # full last leaf, short last leaf
            total = n * leaf - (tail if n > 0 else 0)
            data = np.frombuffer(_rand_bytes(n * 100 + tail, total), dtype=np.uint8)
            leaves = [H(data[i * leaf:(i + 1) * leaf].tobytes()) for i in range(n)]
            want = _mth(leaves, H)
            assert o2.merkle_root(d, data, leaf) == want, (n, tail)
            assert ref.merkle_root(H, data.tobytes(), leaf) == want
    # degenerate cases: one leaf, empty input
    assert o2.merkle_root(d, np.zeros(0, np.uint8), 4) == H(b"")
    a, b = _rand_bytes(1, 4), _rand_bytes(2, 4)
    assert o2.merkle_root(d, np.frombuffer(a + b, np.uint8), 4) == H(H(a) + H(b))


@pytest.mark.parametrize("nr", [1, 5, 12, 23])
def test_reduced_rounds_compose_to_keccak_f(o2, nr):
    # Keccak-p[1600, n_r] runs rounds 24-n_r .. 23 (reading of the round
    # indices): after rounds 0 .. 23-n_r it must give Keccak-f[1600], which
    # hashlib pins through the lane-level oracle.  Indexing the rounds
    # 0 .. n_r-1 instead fails this for every n_r < 24.
    rng = np.random.Generator(np.random.PCG64(90 + nr))
    state = rng.integers(0, 256, 200, dtype=np.uint8).tobytes()
    A = ref.string_to_state(ref.bytes_to_bits(state), 64)
    for ir in range(24 - nr):
        A = ref.rnd(A, ir)
    got = ref.bits_to_bytes(ref.keccak_p(ref.state_to_string(A), 1600, nr))
    assert got == o2.keccak_f1600(state)


# --------------------------------------------------------------------------
# Keccak-p below 1600 bits (Table 1).  The paper prints no value for these
# widths and no independent implementation of them is at hand, so each
# width-dependent part is tied to the 1600-bit permutation, which hashlib
# pins: the round without iota by periodic embedding, iota by truncation of
# the 64-bit round constants, and the round-index reading by composition.
# --------------------------------------------------------------------------

SMALL_WIDTHS = [25, 50, 100, 200, 400, 800]


def _round_without_iota(A):
    return ref.chi(ref.pi(ref.rho(ref.theta(A))))


@pytest.mark.parametrize("b", SMALL_WIDTHS)
def test_round_without_iota_embeds_in_the_1600_bit_round(b):
    # A state whose 64-bit lanes each repeat a w-bit pattern 64/w times stays
    # so under theta, rho, pi and chi (rho's offsets act mod w, theta's
    # z - 1 wraps mod w), and the pattern then follows the width-w round.
    w, _ = ref.width_params(b)
    rng = np.random.Generator(np.random.PCG64(200 + b))
    for _ in range(4):
        a = rng.integers(0, 2, size=(5, 5, w), dtype=np.uint8)
        A = np.tile(a, (1, 1, 64 // w))
        assert np.array_equal(_round_without_iota(A), np.tile(_round_without_iota(a), (1, 1, 64 // w)))


@pytest.mark.parametrize("w", [1, 2, 4, 8, 16, 32])
def test_round_constants_are_the_64_bit_ones_truncated(w):
    # eq. 8 sets bits 2^j - 1 for j = 0..l; with l = log2 w those are exactly
    # the positions below w of the seven 64-bit ones, so RC_w = RC_64 mod 2^w
    # (a "j < l" reading drops bit 2^l - 1 and fails)
    for ir in range(0, 300):
        assert np.array_equal(ref.round_constant(ir, w), ref.round_constant(ir, 64)[:w]), (w, ir)


@pytest.mark.parametrize("b", SMALL_WIDTHS)
def test_theta_of_one_bit_hits_two_columns(b):
    # closed form: a single bit at (x, y, z) sets column parity C[x, z], so
    # theta adds D to columns (x+1, z) and (x-1, z+1): eleven bits in all
    w, _ = ref.width_params(b)
    rng = np.random.Generator(np.random.PCG64(300 + b))
    for _ in range(6):
        x, y, z = (int(v) for v in (rng.integers(0, 5), rng.integers(0, 5), rng.integers(0, w)))
        A = np.zeros((5, 5, w), dtype=np.uint8)
        A[x, y, z] = 1
        want = A.copy()
        want[(x + 1) % 5, :, z] ^= 1
        want[(x - 1) % 5, :, (z + 1) % w] ^= 1
        assert np.array_equal(ref.theta(A), want), (b, x, y, z)
        assert int(ref.theta(A).sum()) == 11


@pytest.mark.parametrize("b", SMALL_WIDTHS + [1600])
def test_reduced_rounds_compose_at_every_width(b):
    # Keccak-p[b, n] after rounds 0 .. 12+2l-n-1 equals Keccak-p[b, 12+2l]:
    # the round indices of n reduced rounds end at 12+2l-1 for every width
    # (indexing them 24-n .. 23 at every width fails this below b = 1600)
    w, l = ref.width_params(b)
    full = 12 + 2 * l
    rng = np.random.Generator(np.random.PCG64(400 + b))
    S = rng.integers(0, 2, size=b, dtype=np.uint8)
    want = ref.keccak_p(S, b, full)
    for n in sorted({1, 2, full // 2, full - 1}):
        A = ref.string_to_state(S, w)
        for ir in range(full - n):
            A = ref.rnd(A, ir)
        assert np.array_equal(ref.keccak_p(ref.state_to_string(A), b, n), want), (b, n)
