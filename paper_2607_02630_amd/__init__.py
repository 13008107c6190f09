"""MI355X-native AES counter mode (and batched SHA-256) behind a C ABI (libaesctr.so).

Thin Python binding with the library's own names.  Buffers are torch CUDA
tensors (any dtype, contiguous) or raw device addresses; streams are
``torch.cuda.Stream`` objects or raw ``hipStream_t`` integers (default: torch's
current stream).  Torch only supplies memory and streams; the cipher runs in
the library's HIP kernels.  There is no CPU path: if the library is missing,
importing this package raises.
"""
from __future__ import annotations

import ctypes

from . import _native as N
from ._native import (AES_VARIANT_AUTO, AES_VARIANT_BITSLICE, AES_VARIANT_TTABLE, AES_VARIANT_VPERM,  # noqa: F401
                      aes_batch_cfg_t, aes_ctr_desc_t, aes_engine_cfg_t, aes_launch_cfg_t,
                      aes_sched_t, aes_stats_t)

lib = N.lib


class AesError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = lib.aes_strerror(status).decode()
        if status == N.AES_EDEVICE:
            msg += f" ({lib.aes_last_device_error().decode()})"
        super().__init__(f"{where}: {msg}" if where else msg)


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise AesError(rc, where)
    return rc


def aes_strerror(status: int) -> str:
    return lib.aes_strerror(status).decode()


def aes_expand_key(key: bytes) -> aes_sched_t:
    """FIPS-197 KeyExpansion of a 16- or 32-byte key (host only)."""
    s = aes_sched_t()
    _check(lib.aes_expand_key(bytes(key), 8 * len(key), ctypes.byref(s)), "aes_expand_key")
    return s


def _is_tensor(x) -> bool:
    return hasattr(x, "data_ptr") and hasattr(x, "element_size")


def _addr(x) -> int | None:
    if x is None:
        return None
    if _is_tensor(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    return int(x)


def _nbytes(x) -> int:
    return x.numel() * x.element_size()


def _check_room(x, n: int, what: str) -> None:
    """A tensor argument must hold at least n bytes: the kernels read and
    write exactly n bytes from its start, so a smaller tensor would be read or
    written past its end."""
    if _is_tensor(x) and _nbytes(x) < n:
        raise ValueError(f"{what} holds {_nbytes(x)} bytes, fewer than the {n} bytes requested")


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _nonce(nonce: bytes) -> bytes:
    nonce = bytes(nonce)
    if len(nonce) != 12:
        raise ValueError("nonce must be 12 bytes")
    return nonce


def launch_cfg(variant: int = 0, blocks_per_lane: int = 0, wg_size: int = 0, grid: int = 0,
               lds_copies: int = 0, lds_tables: int = 0, wave_groups: int = 0) -> aes_launch_cfg_t:
    """Launch shape for aes_ctr_crypt (aes_launch_cfg_t); zero fields keep the
    default.  variant: AES_VARIANT_TTABLE (1), AES_VARIANT_BITSLICE (2) or
    AES_VARIANT_VPERM (3);
    lds_copies / lds_tables: the T-table layout in LDS, 32 or 64 copies of 4
    or 2 tables (64 copies only with 2 tables); wave_groups: the T-table
    kernel's first-chunk mode (0 rule, 1 per-wave group constants, 2 rounds
    1-2 in full, 3 wave 0 for the workgroup)."""
    c = aes_launch_cfg_t()
    c.variant, c.blocks_per_lane, c.wg_size, c.grid, c.lds_copies, c.lds_tables = (
        variant, blocks_per_lane, wg_size, grid, lds_copies, lds_tables)
    c.wave_groups = wave_groups
    return c


def aes_ctr_crypt(sched: aes_sched_t, nonce: bytes, ctr0: int, x, out=None, length: int | None = None,
                  stream=None, cfg: aes_launch_cfg_t | None = None):
    """out = x XOR AES-CTR keystream; returns ``out`` (a new tensor if None).

    ``x``/``out`` are device tensors or raw device addresses (then give
    ``length``).  Asynchronous on ``stream``."""
    if out is None:
        if not _is_tensor(x):
            raise ValueError("out is required when x is a raw address")
        import torch
        out = torch.empty_like(x)
    n = length if length is not None else _nbytes(x)
    if n < 0:
        raise ValueError("length must be >= 0")
    _check_room(x, n, "x")
    _check_room(out, n, "out")
    st = _stream(stream)
    if cfg is None:
        rc = lib.aes_ctr_crypt(ctypes.byref(sched), _nonce(nonce), ctr0 & 0xFFFFFFFF,
                               _addr(x), _addr(out), n, st)
    else:
        rc = lib.aes_ctr_crypt_cfg(ctypes.byref(sched), _nonce(nonce), ctr0 & 0xFFFFFFFF,
                                   _addr(x), _addr(out), n, ctypes.byref(cfg), st)
    _check(rc, "aes_ctr_crypt")
    return out


class Request:
    """One batch/engine request: key schedule, nonce, start counter, buffers."""

    def __init__(self, sched: aes_sched_t, nonce: bytes, ctr0: int, x, out, length: int | None = None):
        self.sched, self.nonce, self.ctr0 = sched, _nonce(nonce), ctr0 & 0xFFFFFFFF
        self.x, self.out = x, out
        self.length = length if length is not None else _nbytes(x)
        if self.length < 0:
            raise ValueError("length must be >= 0")
        _check_room(x, self.length, "x")
        _check_room(out, self.length, "out")

    def desc(self) -> aes_ctr_desc_t:
        d = aes_ctr_desc_t()
        d.in_ = _addr(self.x)
        d.out = _addr(self.out)
        d.len = self.length
        d.sched = ctypes.pointer(self.sched)
        d.nonce[:] = list(self.nonce)
        d.ctr0 = self.ctr0
        return d


class HashRequest:
    """One engine request that hashes ``x`` (``length`` bytes) with SHA-256
    into the 32-byte ``digest`` buffer (flags = AES_FLAG_SHA256)."""

    def __init__(self, x, digest, length: int | None = None):
        self.x, self.digest = x, digest
        self.length = length if length is not None else _nbytes(x)
        if self.length < 0:
            raise ValueError("length must be >= 0")
        _check_room(x, self.length, "x")
        _check_room(digest, 32, "digest")

    def desc(self) -> aes_ctr_desc_t:
        d = aes_ctr_desc_t()
        d.in_ = _addr(self.x) if self.length else None
        d.out = _addr(self.digest)
        d.len = self.length
        d.flags = N.AES_FLAG_SHA256
        return d


def make_desc_array(reqs) -> ctypes.Array:
    arr = (aes_ctr_desc_t * max(len(reqs), 1))()
    for i, r in enumerate(reqs):
        arr[i] = r.desc()
    return arr


def launch_shape(key_bits: int, length: int, cfg: aes_launch_cfg_t | None = None) -> dict:
    """The launch shape aes_ctr_crypt would use (aes_ctr_launch_shape)."""
    out = aes_launch_cfg_t()
    _check(lib.aes_ctr_launch_shape(key_bits, length, ctypes.byref(cfg) if cfg is not None else None,
                                    ctypes.byref(out)), "aes_ctr_launch_shape")
    return {"variant": out.variant, "blocks_per_lane": out.blocks_per_lane, "wg_size": out.wg_size,
            "grid": out.grid, "lds_copies": out.lds_copies, "lds_tables": out.lds_tables,
            "wave_groups": out.wave_groups}


def make_sha_desc_array(items) -> ctypes.Array:
    """Descriptor array for sha256_batch from (input, length, digest) triples;
    input and digest are device tensors or raw device addresses."""
    items = list(items)
    arr = (N.sha256_desc_t * max(len(items), 1))()
    for i, (x, length, digest) in enumerate(items):
        _check_room(x, int(length), f"message {i}")
        _check_room(digest, 32, f"digest {i}")
        arr[i].in_ = _addr(x)
        arr[i].len = int(length)
        arr[i].digest = _addr(digest)
        arr[i].reserved = 0
    return arr


def sha256_batch(items=None, stream=None, descs=None, n: int | None = None) -> None:
    """SHA-256 of many messages in one launch (asynchronous on ``stream``).

    ``items``: (input, length, digest) triples (see make_sha_desc_array), or a
    prebuilt ``descs`` array with its count ``n``."""
    if descs is None:
        items = list(items)
        descs, n = make_sha_desc_array(items), len(items)
    elif n is None:
        raise ValueError("n is required with descs")
    _check(lib.sha256_batch(descs, n, _stream(stream)), "sha256_batch")


def aes_ctr_crypt_batch(reqs, stream=None, cfg: aes_batch_cfg_t | None = None, descs=None) -> None:
    """Encrypt every request with one persistent launch (asynchronous).

    ``descs`` may carry a prebuilt descriptor array (from make_desc_array) to
    keep Python marshalling out of a timed loop."""
    arr = descs if descs is not None else make_desc_array(reqs)
    n = len(reqs)
    st = _stream(stream)
    if cfg is None:
        rc = lib.aes_ctr_crypt_batch(arr, n, st)
    else:
        rc = lib.aes_ctr_crypt_batch_cfg(arr, n, ctypes.byref(cfg), st)
    _check(rc, "aes_ctr_crypt_batch")


def aes_ctr_crypt_batch_noalloc(reqs, stream=None, descs=None) -> None:
    """aes_ctr_crypt_batch without any allocation (at most 4096 requests per
    call; calls that overlap on one GPU race: see include/aesctr.h)."""
    arr = descs if descs is not None else make_desc_array(reqs)
    _check(lib.aes_ctr_crypt_batch_noalloc(arr, len(reqs), _stream(stream)), "aes_ctr_crypt_batch_noalloc")


def batch_cfg(tile_bytes: int = 0, wg_size: int = 0, grid: int = 0, blocks_per_lane: int = 0,
              use_graph: int = 1) -> aes_batch_cfg_t:
    """Launch shape for aes_ctr_crypt_batch (aes_batch_cfg_t); zero fields keep
    the default (tiles sized to the batch, one 1024-thread workgroup per CU,
    two blocks per lane, the captured graph)."""
    c = aes_batch_cfg_t()
    c.tile_bytes, c.wg_size, c.grid, c.blocks_per_lane, c.use_graph = (
        tile_bytes, wg_size, grid, blocks_per_lane, use_graph)
    return c


class Engine:
    """submit -> poll/wait executor (aes_engine_*).

    Its launches run on streams of its own: work that torch queued on its
    stream for a request's buffers must have finished (torch.cuda.synchronize
    or an event) before the request is submitted."""

    def __init__(self, budget_bytes: int = 0, n_streams: int = 0, max_batch_reqs: int = 0,
                 max_batch_bytes: int = 0, key_slots: int = 0, host_buffers: bool = False,
                 device: int = -1):
        c = aes_engine_cfg_t()
        c.budget_bytes, c.n_streams, c.max_batch_reqs = budget_bytes, n_streams, max_batch_reqs
        c.max_batch_bytes, c.key_slots, c.host_buffers, c.device = (
            max_batch_bytes, key_slots, int(host_buffers), device)
        h = ctypes.c_void_p()
        _check(lib.aes_engine_create(ctypes.byref(c), ctypes.byref(h)), "aes_engine_create")
        self._h = h

    def submit(self, req: Request) -> int:
        d = req.desc()
        t = ctypes.c_uint64()
        _check(lib.aes_submit(self._h, ctypes.byref(d), ctypes.byref(t)), "aes_submit")
        return t.value

    def submit_desc(self, d: aes_ctr_desc_t) -> int:
        t = ctypes.c_uint64()
        _check(lib.aes_submit(self._h, ctypes.byref(d), ctypes.byref(t)), "aes_submit")
        return t.value

    def poll(self, ticket: int) -> bool:
        return _check(lib.aes_poll(self._h, ticket), "aes_poll") == 1

    def wait(self, ticket: int, timeout_us: int = -1) -> None:
        _check(lib.aes_wait(self._h, ticket, timeout_us), "aes_wait")

    def stats(self) -> dict:
        s = aes_stats_t()
        _check(lib.aes_engine_stats(self._h, ctypes.byref(s)), "aes_engine_stats")
        return {name: getattr(s, name) for name, _ in aes_stats_t._fields_}

    def reset_stats(self) -> None:
        _check(lib.aes_engine_reset_stats(self._h), "aes_engine_reset_stats")

    def completion_fd(self) -> int:
        return _check(lib.aes_engine_completion_fd(self._h), "aes_engine_completion_fd")

    def close(self) -> None:
        if self._h:
            _check(lib.aes_engine_destroy(self._h), "aes_engine_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
