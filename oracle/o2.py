"""ctypes binding and build step for the lane-level C oracle (keccak_o2.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "keccak_o2.c")
LIB_PATH = os.path.join(_HERE, "libkeccak_o2.so")

VARIANT_BITS = (224, 256, 384, 512)

_lib = None


def build(force: bool = True) -> str:
    """Compile keccak_o2.c with gcc into libkeccak_o2.so next to it."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-Wall", "-Wextra",
             "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp],
            check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        u8p = ctypes.c_void_p
        lib.o2_keccak_f1600.argtypes = [u8p]
        lib.o2_keccak_f1600.restype = None
        lib.o2_sha3.argtypes = [ctypes.c_int, u8p, ctypes.c_uint64, u8p]
        lib.o2_shake.argtypes = [ctypes.c_int, u8p, ctypes.c_uint64, u8p, ctypes.c_uint64]
        lib.o2_sha3_batch.argtypes = [ctypes.c_int, u8p, u8p, u8p, ctypes.c_uint64, u8p,
                                      ctypes.c_int]
        lib.o2_sha3_batch_mixed.argtypes = [u8p, u8p, u8p, u8p, ctypes.c_uint64, u8p,
                                            ctypes.c_int]
        lib.o2_merkle_root.argtypes = [ctypes.c_int, u8p, ctypes.c_uint64, ctypes.c_uint64,
                                       u8p, ctypes.c_int]
        for f in (lib.o2_sha3, lib.o2_shake, lib.o2_sha3_batch, lib.o2_sha3_batch_mixed,
                  lib.o2_merkle_root):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def keccak_f1600(state: bytes) -> bytes:
    a = np.frombuffer(bytes(state), dtype=np.uint8).copy()
    if a.size != 200:
        raise ValueError("state must be 200 bytes")
    _load().o2_keccak_f1600(_ptr(a))
    return a.tobytes()


def sha3(d_bits: int, msg: bytes) -> bytes:
    m = np.frombuffer(bytes(msg), dtype=np.uint8).copy()
    out = np.zeros(d_bits // 8, dtype=np.uint8)
    if _load().o2_sha3(d_bits, _ptr(m), m.size, _ptr(out)) != 0:
        raise ValueError("bad digest size")
    return out.tobytes()


def shake(security: int, msg: bytes, out_len: int) -> bytes:
    m = np.frombuffer(bytes(msg), dtype=np.uint8).copy()
    out = np.zeros(out_len, dtype=np.uint8)
    if _load().o2_shake(security, _ptr(m), m.size, _ptr(out), out_len) != 0:
        raise ValueError("bad security level")
    return out.tobytes()


def _as_u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a).astype(np.uint64, copy=False))


def sha3_batch(d_bits: int, data: np.ndarray, offsets, lengths, threads: int | None = None):
    """Digests of every slice, as a uint8 array of shape (n, d_bits/8)."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offs, lens = _as_u64(offsets), _as_u64(lengths)
    n = offs.size
    if lens.size != n:
        raise ValueError("offsets and lengths differ in size")
    if n and int((offs + lens).max()) > data.size:
        raise ValueError("a message runs past the end of the data")
    out = np.zeros((n, d_bits // 8), dtype=np.uint8)
    rc = _load().o2_sha3_batch(d_bits, _ptr(data), _ptr(offs), _ptr(lens), n, _ptr(out),
                               threads or default_threads())
    if rc:
        raise ValueError("bad digest size")
    return out


def sha3_batch_mixed(variants, data: np.ndarray, offsets, lengths, threads: int | None = None):
    """Mixed-variant digests, shape (n, 64), zero past each digest."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    var = np.ascontiguousarray(np.asarray(variants, dtype=np.uint8))
    offs, lens = _as_u64(offsets), _as_u64(lengths)
    n = offs.size
    if lens.size != n or var.size != n:
        raise ValueError("variants, offsets and lengths differ in size")
    if n and int((offs + lens).max()) > data.size:
        raise ValueError("a message runs past the end of the data")
    out = np.zeros((n, 64), dtype=np.uint8)
    rc = _load().o2_sha3_batch_mixed(_ptr(var), _ptr(data), _ptr(offs), _ptr(lens), n,
                                     _ptr(out), threads or default_threads())
    if rc:
        raise ValueError("variant out of range")
    return out


def merkle_root(d_bits: int, data: np.ndarray, leaf_size: int, threads: int | None = None):
    data = np.ascontiguousarray(data, dtype=np.uint8)
    out = np.zeros(d_bits // 8, dtype=np.uint8)
    rc = _load().o2_merkle_root(d_bits, _ptr(data), data.size, leaf_size, _ptr(out),
                                threads or default_threads())
    if rc:
        raise ValueError("bad merkle arguments")
    return out.tobytes()
