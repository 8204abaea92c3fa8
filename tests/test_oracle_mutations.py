"""The pins must be able to fail: plant plausible slips in the bit-level
oracle (on the CPU, by monkeypatching one step) and check that the hashlib
comparison or the inverse tests catch every one."""

import hashlib

import numpy as np
import pytest

from oracle import keccak_ref as ref


def _theta_wrong_rotation(A):
    w = A.shape[2]
    C = np.bitwise_xor.reduce(A, axis=1)
    D = np.stack([C[(x - 1) % 5] ^ np.roll(C[(x + 1) % 5], -1) for x in range(5)])
    return A ^ D[:, None, :]


def _theta_swapped_neighbours(A):
    C = np.bitwise_xor.reduce(A, axis=1)
    D = np.stack([C[(x + 1) % 5] ^ np.roll(C[(x - 1) % 5], 1) for x in range(5)])
    return A ^ D[:, None, :]


def _rho_rotate_right(A):
    out = A.copy()
    for (x, y), s in ref.rho_offsets(A.shape[2]).items():
        out[x, y] = np.roll(A[x, y], -s)
    return out


def _rho_as_printed(A):
    # eq. 5 taken literally: the rotated lane lands on the next walk position
    w = A.shape[2]
    out = A.copy()
    x, y = 1, 0
    for t in range(24):
        s = (t + 1) * (t + 2) // 2
        nx, ny = y, (2 * x + 3 * y) % 5
        out[nx, ny] = np.roll(A[x, y], -s)
        x, y = nx, ny
    return out


def _pi_transposed(A):
    out = np.zeros_like(A)
    for x in range(5):
        for y in range(5):
            out[x, y] = A[x, (x + 3 * y) % 5]
    return out


def _chi_swapped(A):
    out = np.zeros_like(A)
    for x in range(5):
        for y in range(5):
            out[x, y] = A[x, y] ^ ((A[(x + 2) % 5, y] ^ 1) & A[(x + 1) % 5, y])
    return out


def _round_constant_j_below_l(ir, w):
    # the printed range 0 <= j < l drops bit 63
    l = w.bit_length() - 1
    RC = np.zeros(w, dtype=np.uint8)
    for j in range(l):
        RC[2 ** j - 1] = ref.rc(j + 7 * ir)
    return RC


def _pad_as_printed(x, m):
    j = (-m - 1) % x
    P = np.zeros(j + 2, dtype=np.uint8)
    P[0] = P[-1] = 1
    return P


MUTANTS = {
    "theta_wrong_rotation": ("theta", _theta_wrong_rotation),
    "theta_swapped_neighbours": ("theta", _theta_swapped_neighbours),
    "rho_rotate_right": ("rho", _rho_rotate_right),
    "rho_as_printed": ("rho", _rho_as_printed),
    "pi_transposed": ("pi", _pi_transposed),
    "chi_swapped": ("chi", _chi_swapped),
    "rc_j_below_l": ("round_constant", _round_constant_j_below_l),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_hashlib_pin_catches_step_mutant(monkeypatch, name):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(ref, attr, fn)
    m = b"abc"
    assert ref.sha3(256, m) != hashlib.sha3_256(m).digest()


def test_printed_padding_breaks_block_multiple():
    bad = [(x, m) for x in (8, 1088) for m in range(0, 2 * x)
           if (m + _pad_as_printed(x, m).size) % x != 0]
    assert bad, "the printed pad exponent would have been consistent"


def test_sponge_rejects_printed_padding(monkeypatch):
    monkeypatch.setattr(ref, "pad10star1", _pad_as_printed)
    with pytest.raises(AssertionError):
        ref.keccak_c(512, np.zeros(10, dtype=np.uint8), 256)


# Keccak-p below 1600 bits: the pins tie each width to the 1600-bit case.

def _keccak_p_indexed_from_24(S, b, nr):
    # the 1600-bit round indices 24 - n_r .. 23 used at every width
    w, _ = ref.width_params(b)
    A = ref.string_to_state(S, w)
    for ir in range(24 - nr, 24):
        A = ref.rnd(A, ir)
    return ref.state_to_string(A)


def _rho_offsets_unreduced_left_shift(A):
    # a slip in the lane rotation: the lane is shifted inside a wider
    # register and cut back to w bits, so bits that should wrap are lost
    w = A.shape[2]
    out = A.copy()
    for (x, y), s in ref.rho_offsets(64).items():
        lane = np.concatenate([A[x, y], np.zeros(64, np.uint8)])
        out[x, y] = np.roll(lane, s)[:w]
    return out


def test_composition_pin_catches_1600_bit_round_indices(monkeypatch):
    from tests import test_oracle_pins as pins
    monkeypatch.setattr(ref, "keccak_p", _keccak_p_indexed_from_24)
    with pytest.raises(AssertionError):
        pins.test_reduced_rounds_compose_at_every_width(200)
    pins.test_reduced_rounds_compose_at_every_width(1600)  # identical there


def test_truncation_pin_catches_j_below_l(monkeypatch):
    from tests import test_oracle_pins as pins
    monkeypatch.setattr(ref, "round_constant", _round_constant_j_below_l)
    with pytest.raises(AssertionError):
        pins.test_round_constants_are_the_64_bit_ones_truncated(8)


def test_embedding_pin_catches_a_rho_slip_below_64_bits(monkeypatch):
    from tests import test_oracle_pins as pins
    monkeypatch.setattr(ref, "rho", _rho_offsets_unreduced_left_shift)
    with pytest.raises(AssertionError):
        pins.test_round_without_iota_embeds_in_the_1600_bit_round(200)
