"""ctypes binding of libkbatch.so (argument marshalling only).

Every step of the hashing path runs in the HIP library; this module checks
arguments, takes device pointers from torch tensors and the HIP stream from
torch, and calls the C ABI declared in include/kbatch.h.  There is no CPU
fallback: if the library is not built or no GPU is present the calls raise.
"""

from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to the HIP runtime torch uses

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkbatch.so")

SHA3_224, SHA3_256, SHA3_384, SHA3_512 = 0, 1, 2, 3
VARIANTS = {"sha3_224": 0, "sha3_256": 1, "sha3_384": 2, "sha3_512": 3}
DIGEST_BYTES = (28, 32, 48, 64)
RATE_BYTES = (144, 136, 104, 72)

MODE_PERSISTENT, MODE_PLAIN, MODE_PER_BUCKET, MODE_SPLIT = 0, 1, 2, 3
MODES = {"persistent": 0, "plain": 1, "per_bucket": 2, "split": 3, "wide": 4, "pair": 5}

KB_OK, KB_EINVAL, KB_ENOMEM, KB_EHIP = 0, -1, -2, -3
NOALLOC_MAX_MSGS = 1 << 20

# the C ABI entry points, in include/kbatch.h order
EXPORTS = (
    "keccak_batch", "keccak_batch_noalloc", "keccak_batch_mixed", "keccak_batch_xof",
    "keccak_batch_xof_ex", "keccak_batch_ex", "merkle_root", "keccak_autotune",
    "keccak_tune_store", "keccak_tune_lookup", "keccak_last_tile", "keccak_graph_create", "keccak_graph_create_counted", "keccak_graph_create_merkle", "keccak_graph_launch",
    "keccak_graph_destroy", "keccak_server_create", "keccak_server_submit", "keccak_server_poll",
    "keccak_server_result", "keccak_server_stats", "keccak_server_destroy",
    "keccak_server_last_error", "keccak_tree_workspace_bytes", "keccak_digest_bytes",
    "keccak_rate_bytes", "keccak_reserve", "keccak_release", "keccak_timing_enable",
    "keccak_timing_enable_kinds", "keccak_timing_read", "keccak_timing_read_kernel",
    "keccak_probe_valu", "keccak_probe_perm",
    "keccak_probe_copy", "keccak_last_error", "keccak_version", "keccak_p_batch",
)


class KbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kbatch error {code}: {msg}")
        self.code = code


NB_CLASSES = 8
STAGING_DEFAULT, STAGING_DIRECT, STAGING_PREFETCH = 0, 1, 2
THREADS_WIDE = 32  # class_threads value of the wide split tail (32 lanes per state)


class Tile(ctypes.Structure):
    """kb_tile: knobs of the persistent form (zero = library default).  The
    class arrays are indexed by block-count class floor(log2(blocks))."""
    _fields_ = [("block_threads", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("steps_per_item", ctypes.c_int32), ("staging", ctypes.c_int32),
                ("class_steps", ctypes.c_int32 * NB_CLASSES),
                ("class_threads", ctypes.c_int32 * NB_CLASSES)]

    def as_dict(self) -> dict:
        return {"waves_per_simd": self.waves_per_simd, "steps_per_item": self.steps_per_item,
                "staging": self.staging, "class_steps": list(self.class_steps),
                "class_threads": list(self.class_threads)}


EXECUTOR = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8),
                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                            ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint8))


SERVER_EAGER = 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("d_pool", ctypes.c_void_p), ("pool_bytes", ctypes.c_uint64),
                ("max_step_msgs", ctypes.c_uint64), ("steps_in_flight", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("executor", EXECUTOR),
                ("executor_user", ctypes.c_void_p), ("max_step_bytes", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("messages", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("max_step_msgs_seen", ctypes.c_uint64), ("step_busy_s", ctypes.c_double),
                ("span_s", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkbatch.so (no GPU needed) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1902_05320_amd.build` "
                           "or __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.keccak_batch.argtypes = [i32, vp, vp, vp, u64, vp, vp]
    lib.keccak_batch_noalloc.argtypes = [i32, vp, vp, vp, u64, vp, vp]
    lib.keccak_batch_mixed.argtypes = [vp, vp, vp, vp, u64, vp, vp]
    lib.keccak_batch_ex.argtypes = [i32, vp, vp, vp, vp, u64, vp, i32, ctypes.POINTER(Tile), vp]
    lib.keccak_batch_xof.argtypes = [i32, vp, vp, vp, u64, u64, vp, vp]
    lib.keccak_batch_xof_ex.argtypes = [i32, vp, vp, vp, u64, u64, vp, i32, vp]
    lib.keccak_p_batch.argtypes = [i32, i32, vp, u64, vp]
    lib.merkle_root.argtypes = [i32, vp, u64, u64, vp, vp]
    lib.keccak_tree_workspace_bytes.argtypes = [i32, u64]
    lib.keccak_tree_workspace_bytes.restype = u64
    lib.keccak_digest_bytes.argtypes = [i32]
    lib.keccak_rate_bytes.argtypes = [i32]
    lib.keccak_reserve.argtypes = [u64, u64, vp]
    lib.keccak_release.argtypes = []
    lib.keccak_timing_enable.argtypes = [i32]
    lib.keccak_timing_enable_kinds.argtypes = [ctypes.c_uint32]
    lib.keccak_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_uint64)]
    lib.keccak_timing_read_kernel.argtypes = [i32, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_uint64)]
    lib.keccak_probe_valu.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), vp]
    lib.keccak_probe_perm.argtypes = [ctypes.c_uint32, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int), vp]
    lib.keccak_probe_copy.argtypes = [vp, vp, u64, ctypes.POINTER(ctypes.c_double), vp]
    lib.keccak_autotune.argtypes = [i32, vp, vp, vp, vp, u64, i32, ctypes.POINTER(Tile),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                    vp]
    cp = ctypes.c_char_p
    lib.keccak_tune_store.argtypes = [cp, cp, cp, i32, u64, ctypes.POINTER(Tile), ctypes.c_double]
    lib.keccak_tune_lookup.argtypes = [cp, cp, cp, i32, u64, ctypes.POINTER(Tile)]
    lib.keccak_last_tile.argtypes = [ctypes.POINTER(Tile)]
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.keccak_graph_create.argtypes = [i32, vp, vp, vp, vp, u64, vp, i32, ctypes.POINTER(Tile),
                                        vp, pp]
    lib.keccak_graph_create_counted.argtypes = [i32, vp, vp, vp, vp, vp, u64, vp, vp, pp]
    lib.keccak_graph_create_merkle.argtypes = [i32, vp, u64, u64, vp, vp, pp]
    lib.keccak_graph_launch.argtypes = [vp, vp]
    lib.keccak_graph_destroy.argtypes = [vp]
    lib.keccak_server_create.argtypes = [ctypes.POINTER(ServerConfig), pp]
    lib.keccak_server_submit.argtypes = [vp, i32, vp, vp, u64, ctypes.POINTER(ctypes.c_uint64)]
    lib.keccak_server_poll.argtypes = [vp, vp, u64, ctypes.POINTER(ctypes.c_uint64), i32]
    lib.keccak_server_result.argtypes = [vp, u64, vp, u64, ctypes.POINTER(ctypes.c_double)]
    lib.keccak_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.keccak_server_destroy.argtypes = [vp]
    lib.keccak_server_last_error.argtypes = []
    lib.keccak_server_last_error.restype = ctypes.c_char_p
    lib.keccak_last_error.argtypes = []
    lib.keccak_last_error.restype = ctypes.c_char_p
    lib.keccak_version.argtypes = []
    lib.keccak_version.restype = ctypes.c_char_p
    for f in ("keccak_batch", "keccak_batch_noalloc", "keccak_batch_mixed", "keccak_batch_xof", "keccak_batch_xof_ex",
              "keccak_batch_ex",
              "merkle_root",
              "keccak_digest_bytes", "keccak_rate_bytes", "keccak_reserve", "keccak_release",
              "keccak_timing_enable", "keccak_timing_enable_kinds", "keccak_timing_read",
              "keccak_timing_read_kernel",
              "keccak_probe_valu",
              "keccak_probe_perm", "keccak_probe_copy", "keccak_autotune",
              "keccak_tune_store", "keccak_tune_lookup", "keccak_last_tile", "keccak_graph_create",
              "keccak_graph_create_counted", "keccak_graph_create_merkle", "keccak_graph_launch",
              "keccak_graph_destroy",
              "keccak_server_create", "keccak_server_submit", "keccak_server_poll",
              "keccak_server_result", "keccak_server_stats", "keccak_server_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("kbatch needs a ROCm GPU; none is visible")


def _check(rc: int):
    if rc != KB_OK:
        msg = load_library().keccak_last_error().decode(errors="replace")
        raise KbError(rc, msg)


def _stream_handle(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def _as_u64_view(t: torch.Tensor, name: str, n: int | None = None) -> torch.Tensor:
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"{name} must be int64/uint64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    t = t.contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t


def variant_id(variant) -> int:
    if isinstance(variant, str):
        return VARIANTS[variant]
    v = int(variant)
    if v not in (0, 1, 2, 3):
        raise ValueError(f"variant {variant!r} is not a SHA-3 variant")
    return v


def _check_bounds(data: torch.Tensor, offsets: torch.Tensor, lengths: torch.Tensor):
    """Every slice must lie inside `data` (the C ABI cannot check this)."""
    if offsets.numel() == 0:
        return
    if bool((offsets < 0).any()) or bool((lengths < 0).any()):
        raise ValueError("offsets and lengths must be non-negative")
    end = int((offsets + lengths).max())
    if end > data.numel():
        raise ValueError(f"a message ends at byte {end}, past the data ({data.numel()} bytes)")


def keccak_batch(variant, data: torch.Tensor, offsets: torch.Tensor, lengths: torch.Tensor,
                 out: torch.Tensor | None = None, stream=None, mode="persistent",
                 tile: Tile | None = None, check_bounds: bool = True) -> torch.Tensor:
    """SHA-3 digests of every (offset, length) slice of `data`; returns
    uint8[n, D] on the device.  `mode` is persistent, plain, per_bucket, split or wide."""
    _require_gpu()
    lib = load_library()
    v = variant_id(variant)
    n = offsets.numel()
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 device tensor")
    data = data.contiguous()
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    if check_bounds:
        _check_bounds(data, offsets, lengths)
    D = DIGEST_BYTES[v]
    if out is None:
        out = torch.empty((n, D), dtype=torch.uint8, device=data.device)
    elif out.dtype != torch.uint8 or out.numel() != n * D or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous uint8 tensor of {n * D} bytes")
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    if n == 0:
        return out
    dptr = _ptr(data) if data.numel() else ctypes.c_void_p(out.data_ptr())
    if m == MODE_PERSISTENT and tile is None:
        rc = lib.keccak_batch(v, dptr, _ptr(offsets), _ptr(lengths), n, _ptr(out),
                              _stream_handle(stream))
    else:
        rc = lib.keccak_batch_ex(v, None, dptr, _ptr(offsets), _ptr(lengths), n, _ptr(out), m,
                                 ctypes.byref(tile) if tile is not None else None,
                                 _stream_handle(stream))
    _check(rc)
    return out


def keccak_batch_noalloc(variant, data: torch.Tensor, offsets: torch.Tensor,
                         lengths: torch.Tensor, out: torch.Tensor, stream=None,
                         check_bounds: bool = True) -> torch.Tensor:
    """keccak_batch through the entry point that allocates nothing (a static
    per-device workspace for up to NOALLOC_MAX_MSGS messages, shared by every
    call on the device: calls must not overlap).  `out` (uint8[n, D]) is
    required, since allocating it would defeat the purpose."""
    _require_gpu()
    lib = load_library()
    v = variant_id(variant)
    n = offsets.numel()
    if data.dtype != torch.uint8 or not data.is_cuda or not data.is_contiguous():
        raise TypeError("data must be a contiguous uint8 device tensor")
    if not offsets.is_contiguous() or not lengths.is_contiguous():
        raise ValueError("offsets and lengths must be contiguous")
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    if check_bounds:
        _check_bounds(data, offsets, lengths)
    D = DIGEST_BYTES[v]
    if out.dtype != torch.uint8 or out.numel() != n * D or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous uint8 tensor of {n * D} bytes")
    dptr = _ptr(data) if data.numel() else ctypes.c_void_p(out.data_ptr())
    _check(lib.keccak_batch_noalloc(v, dptr, _ptr(offsets), _ptr(lengths), n, _ptr(out),
                                    _stream_handle(stream)))
    return out


def keccak_batch_mixed(variants: torch.Tensor, data: torch.Tensor, offsets: torch.Tensor,
                       lengths: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                       mode="persistent", tile: Tile | None = None,
                       check_bounds: bool = True) -> torch.Tensor:
    """Per-message variant (uint8 0..3); returns uint8[n, 64], zero past each digest."""
    _require_gpu()
    lib = load_library()
    n = offsets.numel()
    if variants.dtype != torch.uint8 or variants.numel() != n or not variants.is_cuda:
        raise TypeError("variants must be a uint8 device tensor with one entry per message")
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 device tensor")
    data = data.contiguous()
    variants = variants.contiguous()
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    if check_bounds:
        _check_bounds(data, offsets, lengths)
    if out is None:
        out = torch.empty((n, 64), dtype=torch.uint8, device=data.device)
    elif out.dtype != torch.uint8 or out.numel() != n * 64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous uint8 tensor of {n * 64} bytes")
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    if n == 0:
        return out
    dptr = _ptr(data) if data.numel() else ctypes.c_void_p(out.data_ptr())
    if m == MODE_PERSISTENT and tile is None:
        rc = lib.keccak_batch_mixed(_ptr(variants), dptr, _ptr(offsets), _ptr(lengths), n,
                                    _ptr(out), _stream_handle(stream))
    else:
        rc = lib.keccak_batch_ex(-1, _ptr(variants), dptr, _ptr(offsets), _ptr(lengths), n,
                                 _ptr(out), m, ctypes.byref(tile) if tile is not None else None,
                                 _stream_handle(stream))
    _check(rc)
    return out


def keccak_batch_xof(security: int, data: torch.Tensor, offsets: torch.Tensor,
                     lengths: torch.Tensor, out_len: int, out: torch.Tensor | None = None,
                     stream=None, check_bounds: bool = True,
                     mode: str = "persistent") -> torch.Tensor:
    """SHAKE128/256 of every slice, out_len bytes each; returns uint8[n, out_len].

    mode: "persistent" (default), "plain", "per_bucket", "split" or "wide"."""
    _require_gpu()
    lib = load_library()
    if security not in (128, 256):
        raise ValueError("security must be 128 or 256")
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    n = offsets.numel()
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 device tensor")
    data = data.contiguous()
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    if check_bounds:
        _check_bounds(data, offsets, lengths)
    if out_len <= 0:
        raise ValueError("out_len must be positive")
    if out is None:
        out = torch.empty((n, out_len), dtype=torch.uint8, device=data.device)
    elif out.dtype != torch.uint8 or out.numel() != n * out_len or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous uint8 tensor of {n * out_len} bytes")
    if n == 0:
        return out
    dptr = _ptr(data) if data.numel() else ctypes.c_void_p(out.data_ptr())
    _check(lib.keccak_batch_xof_ex(security, dptr, _ptr(offsets), _ptr(lengths), n, int(out_len),
                                   _ptr(out), MODES[mode], _stream_handle(stream)))
    return out


KECCAK_P_WIDTHS = (25, 50, 100, 200, 400, 800, 1600)


def keccak_p_batch(b: int, n_rounds: int, states: torch.Tensor, stream=None) -> torch.Tensor:
    """Keccak-p[b, n_rounds] applied in place to every row of `states`
    (uint8[n, ceil(b/8)] on the device: the packed b-bit strings); returns
    `states`."""
    _require_gpu()
    lib = load_library()
    if b not in KECCAK_P_WIDTHS:
        raise ValueError(f"b must be one of {KECCAK_P_WIDTHS}")
    nbytes = (b + 7) // 8
    if states.dtype != torch.uint8 or not states.is_cuda or not states.is_contiguous():
        raise TypeError("states must be a contiguous uint8 device tensor")
    if states.dim() != 2 or states.shape[1] != nbytes:
        raise ValueError(f"states must have shape (n, {nbytes})")
    _check(lib.keccak_p_batch(int(b), int(n_rounds), _ptr(states), states.shape[0],
                              _stream_handle(stream)))
    return states


def merkle_root(variant, data: torch.Tensor, leaf_size: int, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Root of the binary hash tree over leaf_size-byte leaves (uint8[D])."""
    _require_gpu()
    lib = load_library()
    v = variant_id(variant)
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 device tensor")
    if leaf_size <= 0:
        raise ValueError("leaf_size must be positive")
    data = data.contiguous()
    D = DIGEST_BYTES[v]
    if out is None:
        out = torch.empty(D, dtype=torch.uint8, device=data.device)
    rc = lib.merkle_root(v, _ptr(data), data.numel(), int(leaf_size), _ptr(out),
                         _stream_handle(stream))
    _check(rc)
    return out


def autotune(variant, data: torch.Tensor, offsets: torch.Tensor, lengths: torch.Tensor,
             variants: torch.Tensor | None = None, reps: int = 3, stream=None,
             cache: str | None = None):
    """Pick the persistent-form tile for this batch (every candidate checked
    bit for bit against the plain form first).  variant=-1 with `variants`
    tunes the mixed form.  With `cache`, the result is merged into that JSON
    tune cache under this device's key.  Returns (Tile, ms, rejected)."""
    _require_gpu()
    lib = load_library()
    v = -1 if variant == -1 else variant_id(variant)
    n = offsets.numel()
    data = data.contiguous()
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    _check_bounds(data, offsets, lengths)
    best, ms, rej = Tile(), ctypes.c_double(0.0), ctypes.c_int(0)
    _check(lib.keccak_autotune(v, _ptr(variants), _ptr(data), _ptr(offsets), _ptr(lengths), n,
                               int(reps), ctypes.byref(best), ctypes.byref(ms), ctypes.byref(rej),
                               _stream_handle(stream)))
    if cache is not None:
        tune_store(cache, v, n, best, ms.value)
    return best, ms.value, rej.value


def tune_store(path: str, variant: int, n: int, tile: Tile, ms: float = -1.0,
               arch: str | None = None, rocm: str | None = None):
    """Merge `tile` into the JSON tune cache at `path` (key: arch, ROCm,
    variant (-1 = mixed), block-count classes, batch class of n; arch and
    rocm default to the current device's)."""
    lib = load_library()
    _check(lib.keccak_tune_store(path.encode(), arch.encode() if arch else None,
                                 rocm.encode() if rocm else None, int(variant), int(n),
                                 ctypes.byref(tile), float(ms)))


def tune_lookup(variant: int, n: int, path: str | None = None, arch: str | None = None,
                rocm: str | None = None) -> Tile | None:
    """The cached tile for a batch of n messages of `variant` (-1 = mixed),
    from `path` or $KBATCH_TUNE; None if no entry matches."""
    lib = load_library()
    out = Tile()
    rc = lib.keccak_tune_lookup(path.encode() if path else None, arch.encode() if arch else None,
                                rocm.encode() if rocm else None, int(variant), int(n),
                                ctypes.byref(out))
    if rc < 0:
        _check(rc)
    return out if rc == 1 else None


def last_tile() -> tuple[Tile, bool]:
    """The tile this thread's last batch call ran, and whether it came from
    the tune cache."""
    lib = load_library()
    out = Tile()
    cached = lib.keccak_last_tile(ctypes.byref(out))
    return out, bool(cached)


class Graph:
    """A captured batch or tree; replay() enqueues it with one launch.  The
    tensors it was created from must stay alive and in place."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def replay(self, stream=None):
        _check(load_library().keccak_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if self._h:
            load_library().keccak_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_batch(variant, data, offsets, lengths, out, variants=None, mode="persistent",
                tile: Tile | None = None, stream=None) -> Graph:
    _require_gpu()
    lib = load_library()
    v = -1 if variant == -1 else variant_id(variant)
    n = offsets.numel()
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    _check_bounds(data, offsets, lengths)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    h = ctypes.c_void_p(0)
    _check(lib.keccak_graph_create(v, _ptr(variants), _ptr(data), _ptr(offsets), _ptr(lengths),
                                   n, _ptr(out), m,
                                   ctypes.byref(tile) if tile is not None else None,
                                   _stream_handle(stream), ctypes.byref(h)))
    return Graph(h, (data, offsets, lengths, out, variants))


def graph_counted(variant, data, offsets, lengths, count, out, variants=None,
                  stream=None) -> Graph:
    """Capture the persistent form over up to offsets.numel() messages whose
    count is read, each replay, from `count` (a one-element uint32/int32
    device tensor)."""
    _require_gpu()
    lib = load_library()
    v = -1 if variant == -1 else variant_id(variant)
    n = offsets.numel()
    offsets = _as_u64_view(offsets, "offsets")
    lengths = _as_u64_view(lengths, "lengths", n)
    _check_bounds(data, offsets, lengths)
    if count.numel() != 1 or count.element_size() != 4 or not count.is_cuda:
        raise TypeError("count must be a one-element 32-bit device tensor")
    h = ctypes.c_void_p(0)
    _check(lib.keccak_graph_create_counted(v, _ptr(variants), _ptr(data), _ptr(offsets),
                                           _ptr(lengths), _ptr(count), n, _ptr(out),
                                           _stream_handle(stream), ctypes.byref(h)))
    return Graph(h, (data, offsets, lengths, count, out, variants))


def graph_merkle(variant, data, leaf_size: int, out, stream=None) -> Graph:
    _require_gpu()
    lib = load_library()
    h = ctypes.c_void_p(0)
    _check(lib.keccak_graph_create_merkle(variant_id(variant), _ptr(data), data.numel(),
                                          int(leaf_size), _ptr(out), _stream_handle(stream),
                                          ctypes.byref(h)))
    return Graph(h, (data, out))


class Server:
    """Continuous-batching hash server over a device byte pool (see
    include/kbatch.h).  With `executor` (a Python callable taking numpy
    arrays variants, offsets, lengths and returning uint8[n, 64]) the server
    runs without a GPU."""

    def __init__(self, pool: torch.Tensor | None, max_step_msgs: int = 1 << 16,
                 steps_in_flight: int = 2, executor=None, pool_bytes: int | None = None,
                 max_step_bytes: int = 0, graphs: bool = True):
        import numpy as np
        lib = load_library()
        self._np = np
        self._cb = None
        cfg = ServerConfig()
        if executor is None:
            _require_gpu()
            if pool is None or pool.dtype != torch.uint8 or not pool.is_cuda:
                raise TypeError("pool must be a uint8 device tensor")
            self._pool = pool.contiguous()
            cfg.d_pool = _ptr(self._pool)
            cfg.pool_bytes = self._pool.numel()
        else:
            self._pool = None
            cfg.d_pool = None
            cfg.pool_bytes = int(pool_bytes if pool_bytes is not None else 1 << 62)

            def _run(user, var_p, off_p, len_p, n, out_p):
                try:
                    var = np.ctypeslib.as_array(var_p, shape=(n,)).copy()
                    off = np.ctypeslib.as_array(off_p, shape=(n,)).copy()
                    ln = np.ctypeslib.as_array(len_p, shape=(n,)).copy()
                    res = np.ascontiguousarray(executor(var, off, ln), dtype=np.uint8)
                    ctypes.memmove(out_p, res.ctypes.data, n * 64)
                    return KB_OK
                except Exception:  # reported to the server as a failed step
                    return KB_EHIP

            self._cb = EXECUTOR(_run)
            cfg.executor = self._cb
        cfg.max_step_msgs = int(max_step_msgs)
        cfg.steps_in_flight = int(steps_in_flight)
        cfg.max_step_bytes = int(max_step_bytes)
        cfg.flags = 0 if graphs else SERVER_EAGER
        h = ctypes.c_void_p(0)
        rc = lib.keccak_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != KB_OK:
            raise KbError(rc, lib.keccak_server_last_error().decode())
        self._h = h

    def _srv_check(self, rc):
        if rc != KB_OK:
            raise KbError(rc, load_library().keccak_server_last_error().decode())

    def submit(self, variant, offsets, lengths) -> int:
        np = self._np
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        lens = np.ascontiguousarray(lengths, dtype=np.uint64)
        rid = ctypes.c_uint64(0)
        self._srv_check(load_library().keccak_server_submit(
            self._h, variant_id(variant), ctypes.c_void_p(offs.ctypes.data),
            ctypes.c_void_p(lens.ctypes.data), offs.size, ctypes.byref(rid)))
        return rid.value

    def poll(self, max_ids: int = 4096, wait_ms: int = 0) -> list[int]:
        np = self._np
        ids = np.zeros(max_ids, dtype=np.uint64)
        cnt = ctypes.c_uint64(0)
        self._srv_check(load_library().keccak_server_poll(
            self._h, ctypes.c_void_p(ids.ctypes.data), max_ids, ctypes.byref(cnt), int(wait_ms)))
        return [int(x) for x in ids[:cnt.value]]

    def result(self, rid: int, n: int):
        """(uint8[n, 64] digests, latency ms) of a finished request."""
        np = self._np
        out = np.zeros((n, 64), dtype=np.uint8)
        lat = ctypes.c_double(0.0)
        self._srv_check(load_library().keccak_server_result(
            self._h, rid, ctypes.c_void_p(out.ctypes.data), out.nbytes, ctypes.byref(lat)))
        return out, lat.value

    def stats(self) -> dict:
        st = ServerStats()
        self._srv_check(load_library().keccak_server_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            load_library().keccak_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tree_workspace_bytes(variant, n_leaves: int) -> int:
    """Device node-buffer bytes merkle_root uses for a tree of n_leaves leaves."""
    return int(load_library().keccak_tree_workspace_bytes(variant_id(variant), int(n_leaves)))


def reserve(max_msgs: int, max_leaves: int = 0, stream=None):
    _check(load_library().keccak_reserve(int(max_msgs), int(max_leaves), _stream_handle(stream)))


def release():
    _check(load_library().keccak_release())


KERNELS = {"first_pass": 0, "second_pass": 1, "plain": 2, "split": 3, "tree": 4, "wide": 5,
           "schedule": 6, "pair": 7}


def timing_enable(on: bool = True, kinds=None):
    """Bracket hashing-kernel launches with HIP events on their stream: every
    kind, or only the kinds named in `kinds` (keys of KERNELS)."""
    lib = load_library()
    if kinds is None:
        _check(lib.keccak_timing_enable(1 if on else 0))
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << KERNELS[k]
        _check(lib.keccak_timing_enable_kinds(mask if on else 0))


def timing_read(kernel: str | None = None) -> tuple[float, int]:
    """(total kernel milliseconds, launches) since timing_enable(), over every
    bracketed kernel or over one kind (a key of KERNELS)."""
    ms, cnt = ctypes.c_double(0.0), ctypes.c_uint64(0)
    lib = load_library()
    if kernel is None:
        _check(lib.keccak_timing_read(ctypes.byref(ms), ctypes.byref(cnt)))
    else:
        _check(lib.keccak_timing_read_kernel(KERNELS[kernel], ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def probe_valu(iters: int = 20000, stream=None) -> tuple[float, float]:
    """(sustained int32 VALU tera-ops/s, shader clock MHz) of the current GPU."""
    _require_gpu()
    tops, mhz = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(load_library().keccak_probe_valu(int(iters), ctypes.byref(tops), ctypes.byref(mhz),
                                            _stream_handle(stream)))
    return tops.value, mhz.value


def probe_perm(iters: int = 400, waves_per_simd: int = 0, stream=None) -> tuple[float, int]:
    """(G permutations/s of the register-held Keccak-f[1600], waves per SIMD used)."""
    _require_gpu()
    g, w = ctypes.c_double(0.0), ctypes.c_int(0)
    _check(load_library().keccak_probe_perm(int(iters), int(waves_per_simd), ctypes.byref(g),
                                            ctypes.byref(w), _stream_handle(stream)))
    return g.value, w.value


def probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> float:
    """Device copy bandwidth (GB/s, read + write) of src -> dst."""
    _require_gpu()
    gbps = ctypes.c_double(0.0)
    _check(load_library().keccak_probe_copy(_ptr(src), _ptr(dst), src.numel(), ctypes.byref(gbps),
                                            _stream_handle(stream)))
    return gbps.value


def version() -> str:
    return load_library().keccak_version().decode()
