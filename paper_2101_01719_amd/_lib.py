"""ctypes declarations of the C ABI in include/sbbf.h.

The library is loaded from this package directory. torch is imported first so
that the HIP runtime bundled with torch is the one the library binds to (both
carry the soname libamdhip64.so.7; whichever is loaded first serves both), and
torch's streams are then valid handles for the library.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading the library; see above)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsbbf.so")

c_u32 = ctypes.c_uint32
c_u64 = ctypes.c_uint64
c_size = ctypes.c_size_t
c_vp = ctypes.c_void_p
c_int = ctypes.c_int


class sbbf_launch(ctypes.Structure):
    _fields_ = [("block_threads", c_u32), ("grid_blocks", c_u32), ("unroll", c_u32), ("strategy", c_u32),
                ("flags", c_u32)]


class sbbf_device_info(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("compute_units", ctypes.c_int32),
        ("max_threads_per_block", ctypes.c_int32),
        ("warp_size", ctypes.c_int32),
        ("lds_per_block", c_u64),
        ("lds_per_cu", c_u64),
        ("l2_bytes", c_u64),
        ("global_mem_bytes", c_u64),
        ("clock_khz", ctypes.c_int32),
        ("memory_clock_khz", ctypes.c_int32),
        ("memory_bus_bits", ctypes.c_int32),
        ("arch", ctypes.c_char * 64),
    ]


class sbbf_grouped_config(ctypes.Structure):
    _fields_ = [
        ("lookup_tile_keys", c_u32),
        ("lookup_threads", c_u32),
        ("lookup_unroll", c_u32),
        ("lookup_blocks_per_cu", c_u32),
        ("insert_slice_shift", c_u32),
        ("xcd_queues", c_u32),
        ("insert_lds_bytes", c_u64),
        ("lookup_lds_slices", c_u32),
        ("lookup_lds_threads", c_u32),
    ]


_CFGP = ctypes.POINTER(sbbf_grouped_config)


class sbbf_server_config(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", c_u64),
        ("max_inflight_steps", c_u32),
        ("max_step_requests", c_u32),
        ("max_step_keys", c_u64),
        ("tile_keys", c_u32),
        ("reserved", c_u32),
    ]


class sbbf_serving_stats(ctypes.Structure):
    _fields_ = [
        ("requests_done", c_u64),
        ("keys_done", c_u64),
        ("steps", c_u64),
        ("p50_us", ctypes.c_double),
        ("p99_us", ctypes.c_double),
        ("max_us", ctypes.c_double),
        ("span_s", ctypes.c_double),
        ("gkeys_per_s", ctypes.c_double),
        ("arena_used_bytes", c_u64),
        ("arena_reserved_bytes", c_u64),
    ]


_SCFGP = ctypes.POINTER(sbbf_server_config)

# name -> (restype, argtypes); every symbol declared in include/sbbf.h.
SIGNATURES = {
    "sbbf_status_string": (ctypes.c_char_p, [c_int]),
    "sbbf_last_error": (ctypes.c_char_p, []),
    "sbbf_device_query": (c_int, [ctypes.POINTER(sbbf_device_info)]),
    "sbbf_blocks_for": (c_u64, [c_u64, ctypes.c_double]),
    "sbbf_fpr_model": (ctypes.c_double, [ctypes.c_double]),
    "sbbf_blocks_for_fpr": (c_u64, [c_u64, ctypes.c_double]),
    "sbbf_fpr_model_variant": (ctypes.c_double, [ctypes.c_double, c_u32]),
    "sbbf_blocks_for_fpr_variant": (c_u64, [c_u64, ctypes.c_double, c_u32]),
    "sbbf_union": (c_int, [c_vp, c_vp, c_vp]),
    "sbbf_serialized_bytes": (c_u64, [c_u32]),
    "sbbf_serialized_bytes_variant": (c_u64, [c_u32, c_u32]),
    "sbbf_serialize": (c_int, [c_vp, c_vp, c_size, c_vp]),
    "sbbf_deserialize": (c_int, [c_vp, c_size, ctypes.POINTER(c_vp)]),
    "sbbf_create": (c_int, [c_u32, ctypes.POINTER(c_vp)]),
    "sbbf_create_wrapped": (c_int, [c_vp, c_u32, ctypes.POINTER(c_vp)]),
    "sbbf_create_variant": (c_int, [c_u32, c_u32, ctypes.POINTER(c_vp)]),
    "sbbf_create_wrapped_variant": (c_int, [c_vp, c_u32, c_u32, ctypes.POINTER(c_vp)]),
    "sbbf_lanes": (c_u32, [c_vp]),
    "sbbf_destroy": (c_int, [c_vp]),
    "sbbf_clear": (c_int, [c_vp, c_vp]),
    "sbbf_num_blocks": (c_u32, [c_vp]),
    "sbbf_device_words": (c_vp, [c_vp]),
    "sbbf_copy_words_to_host": (c_int, [c_vp, c_vp, c_vp]),
    "sbbf_copy_words_from_host": (c_int, [c_vp, c_vp, c_vp]),
    "sbbf_auto_insert_strategy": (c_u32, [c_vp, c_size]),
    "sbbf_auto_lookup_strategy": (c_u32, [c_vp, c_size]),
    "sbbf_insert_batch": (c_int, [c_vp, c_vp, c_size, c_vp]),
    "sbbf_insert_batch_ex": (c_int, [c_vp, c_vp, c_size, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_lookup_batch": (c_int, [c_vp, c_vp, c_size, c_vp, c_vp]),
    "sbbf_lookup_batch_bits": (c_int, [c_vp, c_vp, c_size, c_vp, c_vp]),
    "sbbf_lookup_batch_ex": (c_int, [c_vp, c_vp, c_size, c_vp, c_vp, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_lookup_select": (c_int, [c_vp, c_vp, c_size, c_vp, c_vp, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_lookup_select_noalloc": (c_int, [c_vp, c_vp, c_size, c_vp, c_vp, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_key_hash": (c_u64, [c_u64]),
    "sbbf_insert_keys": (c_int, [c_vp, c_vp, c_size, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_lookup_keys": (c_int, [c_vp, c_vp, c_size, c_vp, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_bench_gather": (c_int, [c_vp, c_u32, c_vp, c_size, c_vp, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_bench_atomic": (c_int, [c_vp, c_u32, c_vp, c_size, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_bench_stream": (c_int, [c_vp, c_size, c_vp, ctypes.POINTER(sbbf_launch), c_vp]),
    "sbbf_grouped_default_config": (c_int, [_CFGP]),
    "sbbf_grouped_create": (c_int, [ctypes.POINTER(c_vp), c_u32, ctypes.POINTER(c_vp)]),
    "sbbf_grouped_destroy": (c_int, [c_vp]),
    "sbbf_grouped_plan": (c_int, [c_vp, ctypes.POINTER(c_u64), ctypes.POINTER(c_u64), _CFGP]),
    "sbbf_grouped_plan_capacity": (c_int, [c_vp, ctypes.POINTER(c_u64), ctypes.POINTER(c_u64), _CFGP]),
    "sbbf_grouped_get_config": (c_int, [c_vp, _CFGP]),
    "sbbf_grouped_run_offsets": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "sbbf_grouped_check": (c_int, [c_vp, c_vp, ctypes.POINTER(c_u32)]),
    "sbbf_grouped_counters": (c_int, [c_vp, ctypes.POINTER(c_u64), ctypes.POINTER(c_u64), ctypes.POINTER(c_u64)]),
    "sbbf_grouped_run": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "sbbf_grouped_insert": (c_int, [c_vp, c_vp, c_vp]),
    "sbbf_grouped_lookup": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "sbbf_grouped_run_per_filter": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "sbbf_grouped_digest": (c_int, [c_vp, c_vp, c_vp, ctypes.POINTER(c_u64)]),
    "sbbf_grouped_autotune": (c_int, [c_vp, c_vp, c_vp, c_vp, c_u32, ctypes.c_char_p, c_int, _CFGP]),
    "sbbf_server_default_config": (c_int, [_SCFGP]),
    "sbbf_server_create": (c_int, [_SCFGP, ctypes.POINTER(c_vp)]),
    "sbbf_server_destroy": (c_int, [c_vp]),
    "sbbf_server_add_filter": (c_int, [c_vp, c_u32, ctypes.POINTER(c_u32)]),
    "sbbf_server_remove_filter": (c_int, [c_vp, c_u32]),
    "sbbf_server_arena_usage": (c_int, [c_vp, ctypes.POINTER(c_u64), ctypes.POINTER(c_u64)]),
    "sbbf_server_submit": (c_int, [c_vp, c_u32, c_int, c_vp, c_u64, c_vp, ctypes.POINTER(c_u64)]),
    "sbbf_server_pump": (c_int, [c_vp, c_int]),
    "sbbf_server_drain": (c_int, [c_vp]),
    "sbbf_server_poll": (c_int, [c_vp, ctypes.POINTER(c_u64), c_u32, ctypes.POINTER(c_u32)]),
    "sbbf_server_request_times": (c_int, [c_vp, c_u64, ctypes.POINTER(c_u64), ctypes.POINTER(c_u64)]),
    "sbbf_server_replay": (c_int, [c_vp, c_vp, c_u64, c_int, ctypes.POINTER(c_u64)]),
    "sbbf_server_replay_per_request": (c_int, [c_vp, c_vp, c_u64, ctypes.POINTER(ctypes.c_double)]),
    "sbbf_server_stats": (c_int, [c_vp, ctypes.POINTER(sbbf_serving_stats)]),
    "sbbf_server_snapshot": (c_int, [c_vp, c_u32, c_vp]),
    "sbbf_server_restore": (c_int, [c_vp, c_u32, c_vp]),
}

_lib = None


def load():
    """Load libsbbf.so, failing loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_01719_amd.build` "
                          "(the library has no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
