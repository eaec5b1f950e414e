"""ctypes binding of librmdec.so: the C ABI of include/rmdec.h, same names.

Argument marshalling only.  The library must have been built in-tree
(``python -m paper_2108_12550_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmdec.so")

RM_OK = 0
RM_E_INVAL = -1
RM_E_NOMEM = -2
RM_E_HIP = -3
RM_E_UNSUPPORTED = -4
RM_E_PTR = -5
RM_E_AGAIN = -6

RM_PERM_NONE = 0
RM_PERM_PFHT = 1
RM_PERM_FRESH = 2

EXPORTED = ("rm_decoder_create", "rm_decoder_create_ex", "rm_decode_batch", "rm_decoder_destroy",
            "rm_decoder_set_stream", "rm_decoder_info", "rm_perm_tables", "rm_perm_tables_frame", "rm_supported", "rm_codeword_to_info",
            "rm_last_error",
            "rm_mixed_create", "rm_mixed_supported", "rm_mixed_set_stream", "rm_mixed_set_grid", "rm_mixed_decode",
            "rm_mixed_capture", "rm_mixed_replay", "rm_mixed_autotune", "rm_mixed_destroy", "rm_mixed_decode_static",
            "rm_server_create", "rm_server_supported", "rm_server_now_us", "rm_server_register_pool",
            "rm_server_submit", "rm_server_poll", "rm_server_pending", "rm_server_run_trace", "rm_server_destroy")

RM_MIXED_MAX_SEGMENTS = 8
RM_MIXED_STATIC_MAX_TILES = 1 << 19


class rm_config(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("r", ctypes.c_int), ("P", ctypes.c_int), ("L", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("perm_mode", ctypes.c_int), ("waves_per_block", ctypes.c_int)]


class rm_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("r", ctypes.c_int), ("P", ctypes.c_int), ("L", ctypes.c_int),
                ("N", ctypes.c_int), ("K", ctypes.c_int), ("perm_mode", ctypes.c_int),
                ("n_perm_nodes", ctypes.c_int), ("maps_per_decoder", ctypes.c_int),
                ("waves_per_block", ctypes.c_int), ("lds_bytes_per_wave", ctypes.c_size_t),
                ("table_bytes", ctypes.c_size_t)]


class rm_segment(ctypes.Structure):
    _fields_ = [("dec", ctypes.c_void_p), ("llr", ctypes.c_void_p), ("n_frames", ctypes.c_int64),
                ("out_bits", ctypes.c_void_p), ("out_metric", ctypes.c_void_p), ("tile_frames", ctypes.c_int)]


class rm_mixed_tuning(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int), ("waves_per_block", ctypes.c_int),
                ("tile_frames", ctypes.c_int * RM_MIXED_MAX_SEGMENTS), ("ms", ctypes.c_float),
                ("trials", ctypes.c_int)]


class rm_server_config(ctypes.Structure):
    _fields_ = [("batch_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int), ("depth", ctypes.c_int),
                ("tile_frames", ctypes.c_int), ("split", ctypes.c_int)]


class rm_request(ctypes.Structure):
    _fields_ = [("dec", ctypes.c_void_p), ("llr", ctypes.c_void_p), ("llr_on_device", ctypes.c_int),
                ("tag", ctypes.c_uint64), ("t_arrival_us", ctypes.c_double), ("out_bits", ctypes.c_void_p),
                ("out_metric", ctypes.c_void_p)]


class rm_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int),
                ("n_bytes", ctypes.c_int), ("metric", ctypes.c_float), ("bits", ctypes.c_uint8 * 128),
                ("t_arrival_us", ctypes.c_double), ("t_launch_us", ctypes.c_double), ("t_done_us", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Load librmdec.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2108_12550_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.rm_decoder_create.restype = vp
    L.rm_decoder_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
    L.rm_decoder_create_ex.restype = vp
    L.rm_decoder_create_ex.argtypes = [P(rm_config)]
    L.rm_decode_batch.restype = ctypes.c_int
    L.rm_decode_batch.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.rm_decoder_destroy.restype = None
    L.rm_decoder_destroy.argtypes = [vp]
    L.rm_decoder_set_stream.restype = ctypes.c_int
    L.rm_decoder_set_stream.argtypes = [vp, vp]
    L.rm_decoder_info.restype = ctypes.c_int
    L.rm_decoder_info.argtypes = [vp, P(rm_info)]
    L.rm_perm_tables.restype = ctypes.c_int
    L.rm_perm_tables.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_int, P(ctypes.c_uint16), P(ctypes.c_uint16), P(ctypes.c_int),
                                 ctypes.c_int]
    L.rm_perm_tables_frame.restype = ctypes.c_int
    L.rm_perm_tables_frame.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_int, ctypes.c_int64, P(ctypes.c_uint16), P(ctypes.c_uint16),
                                       P(ctypes.c_int), ctypes.c_int]
    L.rm_supported.restype = ctypes.c_int
    L.rm_supported.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.rm_codeword_to_info.restype = ctypes.c_int
    L.rm_codeword_to_info.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, vp, P(ctypes.c_int64)]
    L.rm_last_error.restype = ctypes.c_char_p
    L.rm_last_error.argtypes = []
    L.rm_mixed_create.restype = vp
    L.rm_mixed_create.argtypes = [ctypes.c_int64]
    L.rm_mixed_supported.restype = ctypes.c_int
    L.rm_mixed_supported.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.rm_mixed_set_stream.restype = ctypes.c_int
    L.rm_mixed_set_stream.argtypes = [vp, vp]
    L.rm_mixed_set_grid.restype = ctypes.c_int
    L.rm_mixed_set_grid.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    for f in ("rm_mixed_decode", "rm_mixed_capture"):
        getattr(L, f).restype = ctypes.c_int
        getattr(L, f).argtypes = [vp, P(rm_segment), ctypes.c_int]
    L.rm_mixed_decode_static.restype = ctypes.c_int
    L.rm_mixed_decode_static.argtypes = [P(rm_segment), ctypes.c_int, ctypes.c_int, vp]
    L.rm_mixed_replay.restype = ctypes.c_int
    L.rm_mixed_replay.argtypes = [vp]
    L.rm_mixed_autotune.restype = ctypes.c_int
    L.rm_mixed_autotune.argtypes = [vp, P(rm_segment), ctypes.c_int, ctypes.c_int, P(rm_mixed_tuning)]
    L.rm_server_create.restype = vp
    L.rm_server_create.argtypes = [P(rm_server_config)]
    L.rm_server_supported.restype = ctypes.c_int
    L.rm_server_supported.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.rm_server_now_us.restype = ctypes.c_double
    L.rm_server_now_us.argtypes = []
    L.rm_server_register_pool.restype = ctypes.c_int
    L.rm_server_register_pool.argtypes = [vp, vp, ctypes.c_int64]
    L.rm_server_submit.restype = ctypes.c_int
    L.rm_server_submit.argtypes = [vp, P(rm_request), P(ctypes.c_uint64)]
    L.rm_server_poll.restype = ctypes.c_int
    L.rm_server_poll.argtypes = [vp, P(rm_completion), ctypes.c_int]
    L.rm_server_pending.restype = ctypes.c_int64
    L.rm_server_pending.argtypes = [vp]
    L.rm_server_run_trace.restype = ctypes.c_int
    L.rm_server_run_trace.argtypes = [vp, P(rm_request), P(ctypes.c_double), ctypes.c_int64, P(ctypes.c_double),
                                      P(ctypes.c_double)]
    L.rm_server_destroy.restype = None
    L.rm_server_destroy.argtypes = [vp]
    L.rm_mixed_destroy.restype = None
    L.rm_mixed_destroy.argtypes = [vp]
    _lib = L
    return L


def rm_last_error() -> str:
    return load().rm_last_error().decode()


def rm_decoder_create(m: int, r: int, P: int, L: int, seed: int) -> int:
    return load().rm_decoder_create(m, r, P, L, ctypes.c_uint64(seed)) or 0


def rm_decoder_create_ex(cfg: rm_config) -> int:
    return load().rm_decoder_create_ex(ctypes.byref(cfg)) or 0


def rm_decode_batch(dec: int, llr_ptr: int, n_frames: int, out_bits_ptr: int, out_metric_ptr: int | None) -> int:
    return load().rm_decode_batch(dec, llr_ptr, n_frames, out_bits_ptr, out_metric_ptr or None)


def rm_decoder_destroy(dec: int) -> None:
    load().rm_decoder_destroy(dec)


def rm_decoder_set_stream(dec: int, stream_handle: int) -> int:
    return load().rm_decoder_set_stream(dec, stream_handle or None)


def rm_decoder_info(dec: int) -> rm_info:
    out = rm_info()
    rc = load().rm_decoder_info(dec, ctypes.byref(out))
    if rc != RM_OK:
        raise RuntimeError(rm_last_error())
    return out


def rm_perm_tables(m: int, r: int, P: int, L: int, seed: int, perm_mode: int, cap: int):
    rows = (ctypes.c_uint16 * (16 * cap))()
    b = (ctypes.c_uint16 * cap)()
    md = (ctypes.c_int * cap)()
    n = load().rm_perm_tables(m, r, P, L, ctypes.c_uint64(seed), perm_mode, rows, b, md, cap)
    return n, rows, b, md


def rm_perm_tables_frame(m: int, r: int, P: int, L: int, seed: int, perm_mode: int, frame: int, cap: int):
    rows = (ctypes.c_uint16 * (16 * cap))()
    b = (ctypes.c_uint16 * cap)()
    md = (ctypes.c_int * cap)()
    n = load().rm_perm_tables_frame(m, r, P, L, ctypes.c_uint64(seed), perm_mode, frame, rows, b, md, cap)
    return n, rows, b, md


def rm_supported(m: int, r: int, L: int, perm_mode: int) -> bool:
    return bool(load().rm_supported(m, r, L, perm_mode))


def rm_codeword_to_info(m: int, r: int, codewords_ptr: int, n_frames: int, info_ptr: int):
    """Host arrays by address; returns (rc, number of frames that are not codewords)."""
    bad = ctypes.c_int64(0)
    rc = load().rm_codeword_to_info(m, r, codewords_ptr, n_frames, info_ptr, ctypes.byref(bad))
    return rc, bad.value


def rm_mixed_create(max_tiles: int) -> int:
    return load().rm_mixed_create(max_tiles) or 0


def rm_mixed_supported(m: int, r: int, L: int) -> bool:
    return bool(load().rm_mixed_supported(m, r, L))


def rm_mixed_set_stream(mx: int, stream_handle: int) -> int:
    return load().rm_mixed_set_stream(mx, stream_handle or None)


def rm_mixed_set_grid(mx: int, blocks: int, waves_per_block: int) -> int:
    return load().rm_mixed_set_grid(mx, blocks, waves_per_block)


def _segments(segs):
    arr = (rm_segment * max(1, len(segs)))()
    for i, s in enumerate(segs):
        arr[i] = s
    return arr


def rm_mixed_decode(mx: int, segs) -> int:
    return load().rm_mixed_decode(mx, _segments(segs), len(segs))


def rm_mixed_decode_static(segs, waves_per_block: int, stream_handle: int) -> int:
    return load().rm_mixed_decode_static(_segments(segs), len(segs), waves_per_block, stream_handle or None)


def rm_mixed_capture(mx: int, segs) -> int:
    return load().rm_mixed_capture(mx, _segments(segs), len(segs))


def rm_mixed_replay(mx: int) -> int:
    return load().rm_mixed_replay(mx)


def rm_mixed_autotune(mx: int, segs, reps: int):
    out = rm_mixed_tuning()
    rc = load().rm_mixed_autotune(mx, _segments(segs), len(segs), reps, ctypes.byref(out))
    return rc, out


def rm_mixed_destroy(mx: int) -> None:
    load().rm_mixed_destroy(mx)


def rm_server_create(cfg: rm_server_config) -> int:
    return load().rm_server_create(ctypes.byref(cfg)) or 0


def rm_server_supported(m: int, r: int, L: int) -> bool:
    return bool(load().rm_server_supported(m, r, L))


def rm_server_now_us() -> float:
    return load().rm_server_now_us()


def rm_server_register_pool(srv: int, base: int, nbytes: int) -> int:
    return load().rm_server_register_pool(srv, base, nbytes)


def rm_server_submit(srv: int, req: rm_request):
    t = ctypes.c_uint64(0)
    rc = load().rm_server_submit(srv, ctypes.byref(req), ctypes.byref(t))
    return rc, t.value


def rm_server_poll(srv: int, out, max_n: int) -> int:
    return load().rm_server_poll(srv, out, max_n)


def rm_server_pending(srv: int) -> int:
    return load().rm_server_pending(srv)


def rm_server_run_trace(srv: int, reqs, arrival_us, n: int, latency_us, stats) -> int:
    return load().rm_server_run_trace(srv, reqs, arrival_us, n, latency_us, stats)


def rm_server_destroy(srv: int) -> None:
    load().rm_server_destroy(srv)
