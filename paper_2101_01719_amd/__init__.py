"""Split block Bloom filters on MI355X (gfx950): Python binding of libsbbf.so.

The functions below carry the names of the C ABI in ``include/sbbf.h`` and
only marshal arguments: torch tensors supply device memory (their data
pointers) and torch supplies the stream (``torch.cuda.current_stream()`` by
default). Every step of insert and lookup runs in the library's HIP kernels;
there is no Python or CPU fallback: when the library has not been built the
first call raises ImportError.

Tensors: hashes are 1-D contiguous int64 or uint64 CUDA tensors (the int64
view carries the same 64 bits); lookup results are uint8 tensors; packed
results are int32 tensors of ceil(n / 32) words; filter words are int32
tensors of 8 * num_blocks elements.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import sbbf_device_info, sbbf_grouped_config, sbbf_launch, sbbf_server_config, sbbf_serving_stats

SBBF_OK = 0
SBBF_EINVAL = 1
SBBF_ENOMEM = 2
SBBF_EDEVICE = 3
SBBF_EBUDGET = 4
SBBF_EUNSUPPORTED = 5
SBBF_EAGAIN = 6

SBBF_INSERT_AUTO = 0
SBBF_INSERT_ATOMIC32 = 1
SBBF_INSERT_ATOMIC64 = 2
SBBF_INSERT_LDS = 3
SBBF_INSERT_PARTITIONED = 4

SBBF_LOOKUP_AUTO = 0
SBBF_LOOKUP_GATHER = 1
SBBF_LOOKUP_PARTITIONED = 2



def _L():
    """The loaded library; raises ImportError when it has not been built."""
    return _lib.load()



class SbbfError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        name = _L().sbbf_status_string(status).decode()
        super().__init__(f"sbbf status {status} ({name}): {detail}")


def _check(status: int) -> None:
    if status != SBBF_OK:
        raise SbbfError(status, _L().sbbf_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _hashes(t: torch.Tensor):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("hashes must be a CUDA (HIP) tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError("hashes must be int64 or uint64")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError("hashes must be a 1-D contiguous tensor")
    if t.device.index != torch.cuda.current_device():
        # the library launches on the current device
        raise ValueError(f"hashes are on {t.device}, the current device is cuda:{torch.cuda.current_device()}")
    return ctypes.c_void_p(t.data_ptr()), t.numel()


def _launch(launch):
    if launch is None:
        return None
    if isinstance(launch, sbbf_launch):
        return ctypes.byref(launch)
    if isinstance(launch, dict):
        names = {name for name, _ in sbbf_launch._fields_}
        unknown = sorted(set(launch) - names)
        if unknown:
            raise ValueError(f"unknown launch settings {unknown}; known: {sorted(names)}")
        return ctypes.byref(sbbf_launch(**launch))
    raise TypeError("launch must be an sbbf_launch or a dict of its fields")


# ---- library ------------------------------------------------------------------

def sbbf_status_string(status: int) -> str:
    return _L().sbbf_status_string(status).decode()


def sbbf_last_error() -> str:
    return _L().sbbf_last_error().decode()


def sbbf_device_query() -> dict:
    info = sbbf_device_info()
    _check(_L().sbbf_device_query(ctypes.byref(info)))
    out = {name: getattr(info, name) for name, _ in sbbf_device_info._fields_}
    out["arch"] = info.arch.decode()
    return out


def sbbf_blocks_for(n: int, bits_per_key: float) -> int:
    return int(_L().sbbf_blocks_for(n, bits_per_key))


def sbbf_fpr_model(keys_per_block: float) -> float:
    return float(_L().sbbf_fpr_model(keys_per_block))


def sbbf_blocks_for_fpr(n: int, fpr: float) -> int:
    b = int(_L().sbbf_blocks_for_fpr(n, fpr))
    if b == 0:
        raise SbbfError(SBBF_EINVAL, _L().sbbf_last_error().decode())
    return b


def sbbf_fpr_model_variant(keys_per_block: float, lanes: int) -> float:
    v = float(_L().sbbf_fpr_model_variant(keys_per_block, lanes))
    if v < 0:
        raise SbbfError(SBBF_EINVAL, _L().sbbf_last_error().decode())
    return v


def sbbf_blocks_for_fpr_variant(n: int, fpr: float, lanes: int) -> int:
    b = int(_L().sbbf_blocks_for_fpr_variant(n, fpr, lanes))
    if b == 0:
        raise SbbfError(SBBF_EINVAL, _L().sbbf_last_error().decode())
    return b


# ---- single filter ------------------------------------------------------------------

def sbbf_create(num_blocks: int) -> int:
    h = ctypes.c_void_p()
    _check(_L().sbbf_create(num_blocks, ctypes.byref(h)))
    return h.value


def sbbf_create_wrapped(words: torch.Tensor, num_blocks: int | None = None) -> int:
    if not words.is_cuda or not words.is_contiguous() or words.element_size() * words.numel() % 32:
        raise ValueError("filter words must be a contiguous CUDA tensor of whole 32-byte blocks")
    nb = words.element_size() * words.numel() // 32 if num_blocks is None else num_blocks
    h = ctypes.c_void_p()
    _check(_L().sbbf_create_wrapped(ctypes.c_void_p(words.data_ptr()), nb, ctypes.byref(h)))
    return h.value


def sbbf_create_variant(num_blocks: int, lanes: int) -> int:
    h = ctypes.c_void_p()
    _check(_L().sbbf_create_variant(num_blocks, lanes, ctypes.byref(h)))
    return h.value


def sbbf_create_wrapped_variant(words: torch.Tensor, num_blocks: int, lanes: int) -> int:
    """Wrap a contiguous CUDA tensor holding num_blocks blocks of `lanes`
    32-bit words (the library checks the lane count and alignment)."""
    if not words.is_cuda or not words.is_contiguous():
        raise ValueError("filter words must be a contiguous CUDA tensor")
    if words.element_size() * words.numel() != 4 * lanes * num_blocks:
        raise ValueError("tensor size does not match num_blocks * lanes words")
    h = ctypes.c_void_p()
    _check(_L().sbbf_create_wrapped_variant(ctypes.c_void_p(words.data_ptr()), num_blocks, lanes, ctypes.byref(h)))
    return h.value


def sbbf_lanes(f: int) -> int:
    return int(_L().sbbf_lanes(f))


def sbbf_destroy(f: int) -> None:
    _check(_L().sbbf_destroy(f))


def sbbf_clear(f: int, stream=None) -> None:
    _check(_L().sbbf_clear(f, _stream(stream)))


def sbbf_num_blocks(f: int) -> int:
    return int(_L().sbbf_num_blocks(f))


def sbbf_device_words(f: int) -> int:
    return _L().sbbf_device_words(f)


def sbbf_copy_words_to_host(f: int, host: torch.Tensor, stream=None) -> torch.Tensor:
    if host.is_cuda or not host.is_contiguous() or host.numel() * host.element_size() != 32 * sbbf_num_blocks(f):
        raise ValueError("host buffer must be a contiguous CPU tensor of 32 * num_blocks bytes")
    _check(_L().sbbf_copy_words_to_host(f, ctypes.c_void_p(host.data_ptr()), _stream(stream)))
    return host


def sbbf_copy_words_from_host(f: int, host: torch.Tensor, stream=None) -> None:
    if host.is_cuda or not host.is_contiguous() or host.numel() * host.element_size() != 32 * sbbf_num_blocks(f):
        raise ValueError("host buffer must be a contiguous CPU tensor of 32 * num_blocks bytes")
    _check(_L().sbbf_copy_words_from_host(f, ctypes.c_void_p(host.data_ptr()), _stream(stream)))


def sbbf_union(dst: int, src: int, stream=None) -> None:
    _check(_L().sbbf_union(dst, src, _stream(stream)))


def sbbf_serialized_bytes(num_blocks: int) -> int:
    return int(_L().sbbf_serialized_bytes(num_blocks))


def sbbf_serialized_bytes_variant(num_blocks: int, lanes: int) -> int:
    return int(_L().sbbf_serialized_bytes_variant(num_blocks, lanes))


def sbbf_serialize(f: int, stream=None) -> bytes:
    """The serialized form of the filter (header + byte image) as bytes."""
    size = sbbf_serialized_bytes_variant(sbbf_num_blocks(f), sbbf_lanes(f))
    buf = ctypes.create_string_buffer(size)
    _check(_L().sbbf_serialize(f, ctypes.cast(buf, ctypes.c_void_p), size, _stream(stream)))
    return buf.raw


def sbbf_deserialize(data: bytes) -> int:
    """A new library-owned filter handle from a serialized form."""
    h = ctypes.c_void_p()
    _check(_L().sbbf_deserialize(ctypes.c_char_p(data), len(data), ctypes.byref(h)))
    return h.value


def sbbf_auto_insert_strategy(f: int, n: int) -> int:
    return int(_L().sbbf_auto_insert_strategy(f, n))


def sbbf_auto_lookup_strategy(f: int, n: int) -> int:
    return int(_L().sbbf_auto_lookup_strategy(f, n))


def sbbf_insert_batch(f: int, hashes: torch.Tensor, stream=None) -> None:
    p, n = _hashes(hashes)
    _check(_L().sbbf_insert_batch(f, p, n, _stream(stream)))


def sbbf_insert_batch_ex(f: int, hashes: torch.Tensor, launch=None, stream=None) -> None:
    p, n = _hashes(hashes)
    _check(_L().sbbf_insert_batch_ex(f, p, n, _launch(launch), _stream(stream)))


def _out_bytes(out, n, device):
    if out is None:
        return torch.empty(n, dtype=torch.uint8, device=device)
    if out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
        raise ValueError("out must be a contiguous uint8 CUDA tensor of at least n elements")
    if out.device != torch.device(device):
        raise ValueError(f"out is on {out.device}, the hashes on {device}")
    return out


def _out_bits(bits, n, device):
    words = (n + 31) // 32
    if bits is None:
        return torch.empty(words, dtype=torch.int32, device=device)
    if bits.dtype not in (torch.int32, torch.uint32) or not bits.is_cuda or not bits.is_contiguous() \
            or bits.numel() < words:
        raise ValueError("bits must be a contiguous int32 CUDA tensor of at least ceil(n/32) words")
    if bits.device != torch.device(device):
        raise ValueError(f"bits are on {bits.device}, the hashes on {device}")
    return bits


def sbbf_lookup_batch(f: int, hashes: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    p, n = _hashes(hashes)
    out = _out_bytes(out, n, hashes.device)
    _check(_L().sbbf_lookup_batch(f, p, n, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def sbbf_lookup_batch_bits(f: int, hashes: torch.Tensor, bits: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
    p, n = _hashes(hashes)
    bits = _out_bits(bits, n, hashes.device)
    _check(_L().sbbf_lookup_batch_bits(f, p, n, ctypes.c_void_p(bits.data_ptr()), _stream(stream)))
    return bits


def sbbf_lookup_batch_ex(f: int, hashes: torch.Tensor, out: torch.Tensor | None = None,
                         bits: torch.Tensor | None = None, launch=None, stream=None) -> torch.Tensor:
    p, n = _hashes(hashes)
    if bits is not None and out is not None:
        raise ValueError("give out or bits, not both")
    if bits is None:
        out = _out_bytes(out, n, hashes.device)
        _check(_L().sbbf_lookup_batch_ex(f, p, n, ctypes.c_void_p(out.data_ptr()), None, _launch(launch),
                                        _stream(stream)))
        return out
    bits = _out_bits(bits, n, hashes.device)
    _check(_L().sbbf_lookup_batch_ex(f, p, n, None, ctypes.c_void_p(bits.data_ptr()), _launch(launch),
                                    _stream(stream)))
    return bits


def sbbf_key_hash(key: int) -> int:
    return int(_L().sbbf_key_hash(key & 0xFFFFFFFFFFFFFFFF))


def sbbf_insert_keys(f: int, keys: torch.Tensor, launch=None, stream=None) -> None:
    p, n = _hashes(keys)
    _check(_L().sbbf_insert_keys(f, p, n, _launch(launch), _stream(stream)))


def sbbf_lookup_keys(f: int, keys: torch.Tensor, out: torch.Tensor | None = None, launch=None,
                     stream=None) -> torch.Tensor:
    p, n = _hashes(keys)
    out = _out_bytes(out, n, keys.device)
    _check(_L().sbbf_lookup_keys(f, p, n, ctypes.c_void_p(out.data_ptr()), _launch(launch), _stream(stream)))
    return out


def sbbf_lookup_select(f: int, hashes: torch.Tensor, indices: torch.Tensor | None = None,
                       count: torch.Tensor | None = None, launch=None, stream=None):
    """Indices (int32 tensor of room n; entries [0, count) valid, ascending)
    of the hashes the filter reports present, and count (one int64 on the
    device). Nothing is synchronised."""
    p, n = _hashes(hashes)
    if indices is None:
        indices = torch.empty(max(n, 1), dtype=torch.int32, device=hashes.device)
    elif indices.dtype not in (torch.int32, torch.uint32) or not indices.is_cuda or not indices.is_contiguous() \
            or indices.numel() < n:
        raise ValueError("indices must be a contiguous int32 CUDA tensor of at least n entries")
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=hashes.device)
    elif count.dtype != torch.int64 or not count.is_cuda or count.numel() < 1:
        raise ValueError("count must be an int64 CUDA tensor")
    _check(_L().sbbf_lookup_select(f, p, n, ctypes.c_void_p(indices.data_ptr()), ctypes.c_void_p(count.data_ptr()),
                                   _launch(launch), _stream(stream)))
    return indices, count


def sbbf_lookup_select_noalloc(f: int, hashes: torch.Tensor, indices: torch.Tensor, count: torch.Tensor,
                               launch=None, stream=None):
    """As sbbf_lookup_select with the library's static workspace: the call
    allocates no device memory, so the caller provides indices (int32, room
    for n) and count (one int64). Gather lookups only; at most 2^28 keys."""
    p, n = _hashes(hashes)
    if indices.dtype not in (torch.int32, torch.uint32) or not indices.is_cuda or not indices.is_contiguous() \
            or indices.numel() < n:
        raise ValueError("indices must be a contiguous int32 CUDA tensor of at least n entries")
    if count.dtype != torch.int64 or not count.is_cuda or count.numel() < 1:
        raise ValueError("count must be an int64 CUDA tensor")
    _check(_L().sbbf_lookup_select_noalloc(f, p, n, ctypes.c_void_p(indices.data_ptr()),
                                           ctypes.c_void_p(count.data_ptr()), _launch(launch), _stream(stream)))
    return indices, count


# ---- measurement kernels ----------------------------------------------------------------

def sbbf_bench_gather(buf: torch.Tensor, num_blocks: int, hashes: torch.Tensor, out: torch.Tensor,
                      launch=None, stream=None) -> None:
    p, n = _hashes(hashes)
    _check(_L().sbbf_bench_gather(ctypes.c_void_p(buf.data_ptr()), num_blocks, p, n, ctypes.c_void_p(out.data_ptr()),
                                 _launch(launch), _stream(stream)))


def sbbf_bench_atomic(buf: torch.Tensor, num_blocks: int, hashes: torch.Tensor, launch=None, stream=None) -> None:
    p, n = _hashes(hashes)
    _check(_L().sbbf_bench_atomic(ctypes.c_void_p(buf.data_ptr()), num_blocks, p, n, _launch(launch),
                                 _stream(stream)))


def sbbf_bench_stream(hashes: torch.Tensor, out: torch.Tensor, launch=None, stream=None) -> None:
    p, n = _hashes(hashes)
    _check(_L().sbbf_bench_stream(p, n, ctypes.c_void_p(out.data_ptr()), _launch(launch), _stream(stream)))


# ---- grouped ---------------------------------------------------------------------------------

def _cfg_struct(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, sbbf_grouped_config):
        return ctypes.byref(cfg)
    base = sbbf_grouped_default_config()
    names = {name for name, _ in sbbf_grouped_config._fields_}
    for k, v in dict(cfg).items():
        if k not in names:
            raise ValueError(f"unknown grouped setting {k!r}; known: {sorted(names)}")
        setattr(base, k, v)
    return ctypes.byref(base)


def _cfg_dict(c: sbbf_grouped_config) -> dict:
    return {name: getattr(c, name) for name, _ in sbbf_grouped_config._fields_}


def _offsets(off):
    import numpy as np

    a = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def sbbf_grouped_default_config() -> sbbf_grouped_config:
    c = sbbf_grouped_config()
    _check(_L().sbbf_grouped_default_config(ctypes.byref(c)))
    return c


def sbbf_grouped_create(filter_handles) -> int:
    arr = (ctypes.c_void_p * len(filter_handles))(*filter_handles)
    g = ctypes.c_void_p()
    _check(_L().sbbf_grouped_create(arr, len(filter_handles), ctypes.byref(g)))
    return g.value


def sbbf_grouped_destroy(g: int) -> None:
    _check(_L().sbbf_grouped_destroy(g))


def sbbf_grouped_plan(g: int, ins_offsets, look_offsets, cfg=None) -> None:
    io, iop = _offsets(ins_offsets)
    lo, lop = _offsets(look_offsets)
    _check(_L().sbbf_grouped_plan(g, iop, lop, _cfg_struct(cfg)))


def sbbf_grouped_plan_capacity(g: int, ins_capacity, look_capacity, cfg=None) -> None:
    """Plan for at most ins_capacity[f] inserts and look_capacity[f] lookups
    of filter f per run (host arrays of num_filters entries)."""
    ic, icp = _offsets(ins_capacity)
    lc, lcp = _offsets(look_capacity)
    _check(_L().sbbf_grouped_plan_capacity(g, icp, lcp, _cfg_struct(cfg)))


def _offsets_tensor(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype not in (torch.int64, torch.uint64) \
            or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int64 CUDA tensor of num_filters + 1 offsets")
    return ctypes.c_void_p(t.data_ptr())


def sbbf_grouped_run_offsets(g: int, d_ins, d_ins_offsets, d_look, d_look_offsets, d_out, stream=None) -> None:
    """One run under a capacity plan; the offsets are int64 CUDA tensors read
    by the kernels when the run executes (nothing is synchronised)."""
    _check(_L().sbbf_grouped_run_offsets(g, _dptr(d_ins), _offsets_tensor(d_ins_offsets, "d_ins_offsets"),
                                         _dptr(d_look), _offsets_tensor(d_look_offsets, "d_look_offsets"),
                                         _dptr(d_out), _stream(stream)))


def sbbf_grouped_check(g: int, stream=None):
    """None when every run since the last check kept within the plan's
    capacities, else the lowest offending filter (the record is cleared)."""
    bad = ctypes.c_uint32(0xFFFFFFFF)
    st = _L().sbbf_grouped_check(g, _stream(stream), ctypes.byref(bad))
    if st == SBBF_OK:
        return None
    if st == SBBF_EINVAL and bad.value != 0xFFFFFFFF:
        return int(bad.value)
    _check(st)


def sbbf_grouped_counters(g: int) -> dict:
    v = [ctypes.c_uint64() for _ in range(3)]
    _check(_L().sbbf_grouped_counters(g, *[ctypes.byref(x) for x in v]))
    return dict(plans=v[0].value, graph_builds=v[1].value, graph_updates=v[2].value)


def sbbf_grouped_get_config(g: int) -> dict:
    c = sbbf_grouped_config()
    _check(_L().sbbf_grouped_get_config(g, ctypes.byref(c)))
    return _cfg_dict(c)


def sbbf_grouped_run(g: int, d_ins, d_look, d_out, stream=None) -> None:
    _check(_L().sbbf_grouped_run(g, _dptr(d_ins), _dptr(d_look), _dptr(d_out), _stream(stream)))


def sbbf_grouped_insert(g: int, d_ins, stream=None) -> None:
    _check(_L().sbbf_grouped_insert(g, _dptr(d_ins), _stream(stream)))


def sbbf_grouped_lookup(g: int, d_look, d_out, stream=None) -> None:
    _check(_L().sbbf_grouped_lookup(g, _dptr(d_look), _dptr(d_out), _stream(stream)))


def sbbf_grouped_run_per_filter(g: int, d_ins, d_look, d_out, stream=None) -> None:
    _check(_L().sbbf_grouped_run_per_filter(g, _dptr(d_ins), _dptr(d_look), _dptr(d_out), _stream(stream)))


def sbbf_grouped_digest(g: int, d_out=None, stream=None) -> int:
    v = ctypes.c_uint64()
    _check(_L().sbbf_grouped_digest(g, _dptr(d_out), _stream(stream), ctypes.byref(v)))
    return v.value


def sbbf_grouped_autotune(g: int, d_ins, d_look, d_out, reps: int = 5, cache_path=None, force: bool = False) -> dict:
    c = sbbf_grouped_config()
    path = cache_path.encode() if cache_path else None
    _check(_L().sbbf_grouped_autotune(g, _dptr(d_ins), _dptr(d_look), _dptr(d_out), reps, path, int(force),
                                      ctypes.byref(c)))
    return _cfg_dict(c)


# ---- serving --------------------------------------------------------------------------------

def sbbf_server_default_config() -> sbbf_server_config:
    c = sbbf_server_config()
    _check(_L().sbbf_server_default_config(ctypes.byref(c)))
    return c


def sbbf_server_create(cfg=None) -> int:
    c = sbbf_server_default_config()
    names = {name for name, _ in sbbf_server_config._fields_}
    for k, v in dict(cfg or {}).items():
        if k not in names:
            raise ValueError(f"unknown server setting {k!r}; known: {sorted(names)}")
        setattr(c, k, v)
    h = ctypes.c_void_p()
    _check(_L().sbbf_server_create(ctypes.byref(c), ctypes.byref(h)))
    return h.value


def sbbf_server_destroy(s: int) -> None:
    _check(_L().sbbf_server_destroy(s))


def sbbf_server_add_filter(s: int, num_blocks: int) -> int:
    fid = ctypes.c_uint32()
    _check(_L().sbbf_server_add_filter(s, num_blocks, ctypes.byref(fid)))
    return fid.value


def sbbf_server_remove_filter(s: int, filter_id: int) -> None:
    _check(_L().sbbf_server_remove_filter(s, filter_id))


def sbbf_server_arena_usage(s: int):
    used, reserved = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_L().sbbf_server_arena_usage(s, ctypes.byref(used), ctypes.byref(reserved)))
    return used.value, reserved.value


def sbbf_server_submit(s: int, filter_id: int, op: int, d_hashes, d_out=None) -> int:
    p, n = _hashes(d_hashes)
    rid = ctypes.c_uint64()
    _check(_L().sbbf_server_submit(s, filter_id, op, p, n, _dptr(d_out), ctypes.byref(rid)))
    return rid.value


def sbbf_server_pump(s: int, wait: bool = False) -> None:
    _check(_L().sbbf_server_pump(s, int(wait)))


def sbbf_server_drain(s: int) -> None:
    _check(_L().sbbf_server_drain(s))


def sbbf_server_poll(s: int, cap: int = 4096) -> list:
    buf = (ctypes.c_uint64 * cap)()
    n = ctypes.c_uint32()
    st = _L().sbbf_server_poll(s, buf, cap, ctypes.byref(n))
    if st not in (SBBF_OK, SBBF_EAGAIN):
        _check(st)
    return list(buf[: n.value])


def sbbf_server_request_times(s: int, req_id: int):
    a, d = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_L().sbbf_server_request_times(s, req_id, ctypes.byref(a), ctypes.byref(d)))
    return a.value, d.value


# numpy layout of sbbf_request (40 bytes)
REQUEST_DTYPE = [("arrival_ns", "<u8"), ("filter_id", "<u4"), ("op", "<u4"), ("d_hashes", "<u8"),
                 ("d_out", "<u8"), ("n", "<u8")]


def sbbf_server_replay(s: int, requests, realtime: bool = True) -> int:
    """requests: a numpy structured array of REQUEST_DTYPE. Returns the id of the first request."""
    import numpy as np

    req = np.ascontiguousarray(requests)
    if req.dtype != np.dtype(REQUEST_DTYPE):
        raise TypeError("requests must use REQUEST_DTYPE")
    first = ctypes.c_uint64()
    _check(_L().sbbf_server_replay(s, ctypes.c_void_p(req.ctypes.data), req.size, int(realtime), ctypes.byref(first)))
    return first.value


def sbbf_server_replay_per_request(s: int, requests) -> float:
    """The same log as one plain call per request, in order, with no batching
    (the baseline); returns its wall time in seconds."""
    import numpy as np

    req = np.ascontiguousarray(requests)
    if req.dtype != np.dtype(REQUEST_DTYPE):
        raise TypeError("requests must use REQUEST_DTYPE")
    sec = ctypes.c_double()
    _check(_L().sbbf_server_replay_per_request(s, ctypes.c_void_p(req.ctypes.data), req.size, ctypes.byref(sec)))
    return sec.value


def sbbf_server_stats(s: int) -> dict:
    st = sbbf_serving_stats()
    _check(_L().sbbf_server_stats(s, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in sbbf_serving_stats._fields_}


def sbbf_server_snapshot(s: int, filter_id: int, host: torch.Tensor) -> torch.Tensor:
    _check(_L().sbbf_server_snapshot(s, filter_id, ctypes.c_void_p(host.data_ptr())))
    return host


def sbbf_server_restore(s: int, filter_id: int, host: torch.Tensor) -> None:
    _check(_L().sbbf_server_restore(s, filter_id, ctypes.c_void_p(host.data_ptr())))


# ---- convenience --------------------------------------------------------------------------

class Filter:
    """A filter whose words live in a torch tensor (so they can be read back
    with ``words.cpu()``), driven through the C ABI."""

    def __init__(self, num_blocks: int, device="cuda", lanes: int = 8):
        """num_blocks blocks of `lanes` 32-bit words: 8 is the method; 4 and
        16 are the block variants (see sbbf_create_variant)."""
        if not 1 <= num_blocks <= 0xFFFFFFFF:
            raise ValueError("num_blocks must be in [1, 2**32 - 1]")
        if lanes not in (4, 8, 16):
            raise ValueError("lanes must be 4, 8 or 16")
        self.num_blocks = int(num_blocks)
        self.lanes = int(lanes)
        self.words = torch.zeros(self.lanes * self.num_blocks, dtype=torch.int32, device=device)
        if self.lanes == 8:
            self.handle = sbbf_create_wrapped(self.words, self.num_blocks)
        else:
            self.handle = sbbf_create_wrapped_variant(self.words, self.num_blocks, self.lanes)

    def insert(self, hashes, launch=None, stream=None):
        sbbf_insert_batch_ex(self.handle, hashes, launch, stream)
        return self

    def lookup(self, hashes, out=None, launch=None, stream=None):
        return sbbf_lookup_batch_ex(self.handle, hashes, out=out, launch=launch, stream=stream)

    def lookup_bits(self, hashes, bits=None, launch=None, stream=None):
        return sbbf_lookup_batch_ex(self.handle, hashes, bits=bits if bits is not None else _out_bits(
            None, hashes.numel(), hashes.device), launch=launch, stream=stream)

    def insert_keys(self, keys, launch=None, stream=None):
        sbbf_insert_keys(self.handle, keys, launch, stream)
        return self

    def lookup_keys(self, keys, out=None, launch=None, stream=None):
        return sbbf_lookup_keys(self.handle, keys, out, launch, stream)

    def union(self, other, stream=None):
        """self |= other (same number of blocks)."""
        sbbf_union(self.handle, other.handle, stream)
        return self

    def serialize(self, stream=None) -> bytes:
        return sbbf_serialize(self.handle, stream)

    def select(self, hashes, launch=None, stream=None):
        """Ascending indices of the hashes reported present (synchronises to
        read the count)."""
        idx, cnt = sbbf_lookup_select(self.handle, hashes, launch=launch, stream=stream)
        return idx[: int(cnt.item())]

    def clear(self, stream=None):
        sbbf_clear(self.handle, stream)
        return self

    def close(self):
        if self.handle:
            sbbf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Group:
    """Many filters driven as one group (see sbbf_grouped_*). The filters are
    Filter objects (torch-backed words); offsets are host CSR arrays."""

    def __init__(self, filters, ins_offsets, look_offsets, cfg=None):
        self.filters = list(filters)
        self.handle = sbbf_grouped_create([f.handle for f in self.filters])
        self.ins_offsets = ins_offsets
        self.look_offsets = look_offsets
        self.capacity = None
        if ins_offsets is not None:
            sbbf_grouped_plan(self.handle, ins_offsets, look_offsets, cfg)

    @classmethod
    def with_capacity(cls, filters, ins_capacity, look_capacity, cfg=None):
        """A group planned for per-filter key capacities; its runs take device
        offsets (run_offsets)."""
        g = cls(filters, None, None)
        g.capacity = (ins_capacity, look_capacity)
        sbbf_grouped_plan_capacity(g.handle, ins_capacity, look_capacity, cfg)
        return g

    def replan(self, cfg=None):
        if self.capacity is not None:
            sbbf_grouped_plan_capacity(self.handle, self.capacity[0], self.capacity[1], cfg)
        else:
            sbbf_grouped_plan(self.handle, self.ins_offsets, self.look_offsets, cfg)

    def run_offsets(self, d_ins, d_ins_offsets, d_look, d_look_offsets, d_out, stream=None):
        sbbf_grouped_run_offsets(self.handle, d_ins, d_ins_offsets, d_look, d_look_offsets, d_out, stream)

    def check(self, stream=None):
        return sbbf_grouped_check(self.handle, stream)

    def counters(self) -> dict:
        return sbbf_grouped_counters(self.handle)

    def config(self) -> dict:
        return sbbf_grouped_get_config(self.handle)

    def run(self, d_ins, d_look, d_out, stream=None):
        sbbf_grouped_run(self.handle, d_ins, d_look, d_out, stream)

    def run_per_filter(self, d_ins, d_look, d_out, stream=None):
        sbbf_grouped_run_per_filter(self.handle, d_ins, d_look, d_out, stream)

    def digest(self, d_out=None, stream=None) -> int:
        return sbbf_grouped_digest(self.handle, d_out, stream)

    def autotune(self, d_ins, d_look, d_out, reps=5, cache_path=None, force=False) -> dict:
        return sbbf_grouped_autotune(self.handle, d_ins, d_look, d_out, reps, cache_path, force)

    def clear(self, stream=None):
        for f in self.filters:
            f.clear(stream)

    def close(self):
        if self.handle:
            sbbf_grouped_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serving_requests(log, d_payload, d_out):
    """The sbbf_request array for a synth ServingLog whose payload is staged in
    d_payload (int64 view, device; or the integer address of the payload in
    memory the device can read, such as mapped pinned host memory) and whose
    lookup outputs go to d_out (uint8)."""
    import numpy as np

    base = int(d_payload) if isinstance(d_payload, int) else d_payload.data_ptr()
    req = np.zeros(log.num_requests, dtype=REQUEST_DTYPE)
    req["arrival_ns"] = log.arrival_ns
    req["filter_id"] = log.filter
    req["op"] = log.op
    req["n"] = log.n
    req["d_hashes"] = np.uint64(base) + log.key_off[:-1].astype(np.uint64) * np.uint64(8)
    look = log.op == 1
    req["d_out"] = np.where(look, np.uint64(d_out.data_ptr()) + log.out_off[:-1].astype(np.uint64), np.uint64(0))
    return req
