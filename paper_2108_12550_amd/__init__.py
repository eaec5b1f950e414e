"""MI355X (gfx950) batched decoder for Reed-Muller codes.

Permuted fast successive-cancellation list decoding with the fast Hadamard
transform, P parallel decoders per frame (p-FHT-FSCL-L-M; Doan, Hashemi and
Gross, arXiv 2108.12550, Alg. 2-5).  All decoding runs in the HIP kernels of
librmdec.so behind the C ABI of include/rmdec.h; PyTorch provides device
memory and streams only.
"""
from __future__ import annotations

import ctypes
from math import comb

from . import _lib
from ._lib import (RM_E_AGAIN, RM_E_HIP, RM_E_INVAL, RM_E_NOMEM, RM_E_PTR, RM_E_UNSUPPORTED, RM_MIXED_MAX_SEGMENTS,
                   RM_OK, RM_PERM_FRESH, RM_PERM_NONE, RM_PERM_PFHT, rm_completion, rm_config, rm_decode_batch, rm_decoder_create,
                   rm_decoder_create_ex, rm_decoder_destroy, rm_decoder_info, rm_decoder_set_stream, rm_last_error,
                   rm_mixed_autotune, rm_mixed_capture, rm_mixed_create, rm_mixed_decode, rm_mixed_decode_static,
                   rm_mixed_destroy, RM_MIXED_STATIC_MAX_TILES,
                   rm_mixed_replay, rm_mixed_set_grid, rm_mixed_set_stream, rm_mixed_supported, rm_mixed_tuning,
                   rm_codeword_to_info, rm_perm_tables, rm_perm_tables_frame, rm_request, rm_segment, rm_server_config, rm_server_create, rm_server_destroy,
                   rm_server_now_us, rm_server_pending, rm_server_poll, rm_server_register_pool, rm_server_run_trace,
                   rm_server_submit, rm_server_supported, rm_supported)

__all__ = ["Decoder", "MixedLauncher", "perm_tables", "code_dimension", "RM_PERM_NONE", "RM_PERM_PFHT",
           "RM_PERM_FRESH", "rm_perm_tables_frame", "rm_codeword_to_info", "codeword_to_info",
           "RM_MIXED_MAX_SEGMENTS", "rm_config", "rm_segment", "rm_decode_batch", "rm_decoder_create",
           "rm_decoder_create_ex", "rm_decoder_destroy", "rm_decoder_info", "rm_decoder_set_stream",
           "rm_last_error", "rm_perm_tables", "rm_supported", "rm_mixed_create", "rm_mixed_supported",
           "rm_mixed_set_stream", "rm_mixed_set_grid", "rm_mixed_decode", "rm_mixed_capture",
           "rm_mixed_replay", "rm_mixed_autotune", "rm_mixed_tuning", "rm_mixed_destroy", "Server",
           "rm_mixed_decode_static", "mixed_decode_static", "RM_MIXED_STATIC_MAX_TILES",
           "RM_E_AGAIN", "rm_server_config", "rm_request", "rm_completion", "rm_server_create",
           "rm_server_supported", "rm_server_now_us", "rm_server_register_pool", "rm_server_submit",
           "rm_server_poll", "rm_server_pending", "rm_server_run_trace", "rm_server_destroy"]


def code_dimension(m: int, r: int) -> int:
    return sum(comb(m, i) for i in range(r + 1))


def codeword_to_info(m: int, r: int, codewords):
    """Information bits u_I of packed codewords ((n, N/8) uint8 host array):
    returns ((n, K) uint8, number of frames that are not codewords)."""
    import numpy as np
    cw = np.ascontiguousarray(codewords, dtype=np.uint8).reshape(-1, (1 << m) // 8)
    out = np.zeros((cw.shape[0], code_dimension(m, r)), dtype=np.uint8)
    rc, bad = rm_codeword_to_info(m, r, cw.ctypes.data, cw.shape[0], out.ctypes.data)
    if rc != RM_OK:
        raise RMError(rc, rm_last_error())
    return out, bad


class RMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librmdec error {code}: {msg}")
        self.code = code


class Decoder:
    """p-FHT-FSCL-L-M decoder of RM(r, m) with P parallel decoders of list size L."""

    def __init__(self, m: int, r: int, P: int, L: int, seed: int = 0, perm_mode: int = RM_PERM_PFHT,
                 waves_per_block: int = 0):
        cfg = rm_config(m, r, P, L, seed, perm_mode, waves_per_block)
        self._h = rm_decoder_create_ex(cfg)
        if not self._h:
            raise RMError(-1, rm_last_error())
        self.m, self.r, self.P, self.L, self.seed, self.perm_mode = m, r, P, L, seed, perm_mode
        self.N = 1 << m
        self.K = code_dimension(m, r)

    def close(self, _destroy=rm_decoder_destroy):
        if getattr(self, "_h", 0):
            _destroy(self._h)
            self._h = 0

    def __del__(self):
        self.close()

    def info(self) -> dict:
        i = rm_decoder_info(self._h)
        return {f: getattr(i, f) for f, _ in i._fields_}

    def decode(self, llr, out_bits=None, out_metric=None, stream=None):
        """Decode a (n_frames, N) float32 CUDA tensor of LLRs.

        Returns (bits, metric): (n_frames, N/8) uint8 packed codewords (bit i
        at byte i>>3, bit i&7) and (n_frames,) float32 final metrics.  The work
        is queued on ``stream`` (default: torch's current stream).
        """
        import torch
        if not (llr.is_cuda and llr.dtype == torch.float32 and llr.is_contiguous()):
            raise ValueError("llr must be a contiguous float32 CUDA tensor")
        llr = llr.view(-1, self.N)
        n = llr.shape[0]
        if out_bits is None:
            out_bits = torch.empty((n, self.N // 8), dtype=torch.uint8, device=llr.device)
        if out_metric is None:
            out_metric = torch.empty((n,), dtype=torch.float32, device=llr.device)
        s = stream if stream is not None else torch.cuda.current_stream(llr.device)
        rc = rm_decoder_set_stream(self._h, s.cuda_stream)
        if rc == RM_OK:
            rc = rm_decode_batch(self._h, llr.data_ptr(), n, out_bits.data_ptr(),
                                 out_metric.data_ptr() if out_metric is not False else None)
        if rc != RM_OK:
            raise RMError(rc, rm_last_error())
        return out_bits, out_metric


class MixedLauncher:
    """One persistent launch over frames of several codes (rm_mixed_* of the C ABI).

    A segment is ``(decoder, llr, out_bits, out_metric, tile_frames)``: a
    ``Decoder`` of a code compiled into the fused kernel, its (n, N) float32
    LLRs, (n, N/8) uint8 and (n,) float32 outputs (CUDA tensors; out_metric
    may be None) and the frames per queue entry (0 = library default).
    """

    def __init__(self, max_tiles: int = 1 << 20, blocks: int = 0, waves_per_block: int = 0):
        self._h = rm_mixed_create(max_tiles)
        if not self._h:
            raise RMError(-1, rm_last_error())
        self._check(rm_mixed_set_grid(self._h, blocks, waves_per_block))
        self._held = None  # tensors a captured graph refers to

    @staticmethod
    def supported(m: int, r: int, L: int) -> bool:
        return rm_mixed_supported(m, r, L)

    def _check(self, rc):
        if rc != RM_OK:
            raise RMError(rc, rm_last_error())

    def set_grid(self, blocks: int, waves_per_block: int):
        self._check(rm_mixed_set_grid(self._h, blocks, waves_per_block))

    @staticmethod
    def _segs(segments):
        import torch
        out = []
        for dec, llr, bits, metric, tf in segments:
            if not (llr.is_cuda and llr.dtype == torch.float32 and llr.is_contiguous()):
                raise ValueError("llr must be a contiguous float32 CUDA tensor")
            n = llr.numel() // dec.N
            if bits.numel() < n * dec.N // 8 or (metric is not None and metric.numel() < n):
                raise ValueError("output tensors too small")
            out.append(rm_segment(dec._h, llr.data_ptr(), n, bits.data_ptr(),
                                  metric.data_ptr() if metric is not None else None, tf))
        return out

    def _bind(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self._check(rm_mixed_set_stream(self._h, s.cuda_stream))

    def decode(self, segments, stream=None):
        """Queue one fused launch over the segments on ``stream``."""
        self._bind(stream)
        self._check(rm_mixed_decode(self._h, self._segs(segments)))

    def capture(self, segments, stream):
        """Record the fused launch for these segments as a graph (replay())."""
        self._bind(stream)
        self._check(rm_mixed_capture(self._h, self._segs(segments)))
        self._held = list(segments)

    def replay(self):
        self._check(rm_mixed_replay(self._h))

    def autotune(self, segments, stream=None, reps: int = 2) -> dict:
        """Time launch choices on these segments (outputs overwritten) and keep
        the best; returns {"waves_per_block", "tile_frames", "ms", "trials"}.
        The segments' own tile_frames entries are ignored."""
        self._bind(stream)
        rc, t = rm_mixed_autotune(self._h, self._segs(segments), reps)
        self._check(rc)
        return {"waves_per_block": t.waves_per_block, "blocks": t.blocks,
                "tile_frames": [t.tile_frames[i] for i in range(len(segments))], "ms": t.ms, "trials": t.trials}

    def close(self, _destroy=rm_mixed_destroy):
        if getattr(self, "_h", 0):
            _destroy(self._h)
            self._h = 0
        self._held = None

    def __del__(self):
        self.close()


def mixed_decode_static(segments, waves_per_block: int = 0, stream=None):
    """The fused launch of ``MixedLauncher.decode`` without a launcher: no
    device allocation (rm_mixed_decode_static).  Segments as for
    ``MixedLauncher``; calls on one device share the library's static queue,
    so calls that may overlap must be ordered by the caller."""
    import torch
    segs = MixedLauncher._segs(segments)
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = rm_mixed_decode_static(segs, waves_per_block, s.cuda_stream)
    if rc != RM_OK:
        raise RMError(rc, rm_last_error())


class Server:
    """Request server (rm_server_* of the C ABI): continuous batching of
    single-frame requests of any served code, P and L."""

    def __init__(self, batch_bytes: int = 64 << 20, max_batch: int = 16384, depth: int = 2, tile_frames: int = 0,
                 split: int = 0):
        self._h = rm_server_create(rm_server_config(batch_bytes, max_batch, depth, tile_frames, split))
        if not self._h:
            raise RMError(-1, rm_last_error())
        self._keep = []  # device pools and decoders the requests refer to
        self._cbuf = (rm_completion * 4096)()

    @staticmethod
    def supported(m: int, r: int, L: int) -> bool:
        return rm_server_supported(m, r, L)

    @staticmethod
    def now_us() -> float:
        return rm_server_now_us()

    def register_pool(self, tensor):
        """Allow device-resident requests to point into this CUDA tensor."""
        rc = rm_server_register_pool(self._h, tensor.data_ptr(), tensor.numel() * tensor.element_size())
        if rc != RM_OK:
            raise RMError(rc, rm_last_error())
        self._keep.append(tensor)

    def submit(self, dec: "Decoder", llr_ptr: int, on_device: bool, tag: int = 0, t_arrival_us: float = 0.0):
        """Returns the ticket, or None if not admitted now (RM_E_AGAIN)."""
        rc, t = rm_server_submit(self._h, rm_request(dec._h, llr_ptr, int(on_device), tag, t_arrival_us, None, None))
        if rc == RM_E_AGAIN:
            return None
        if rc != RM_OK:
            raise RMError(rc, rm_last_error())
        return t

    def poll(self, max_n: int = 4096):
        """Completions now available: list of (ticket, tag, bits bytes, metric, t_arrival, t_launch, t_done)."""
        k = rm_server_poll(self._h, self._cbuf, min(max_n, len(self._cbuf)))
        if k < 0:
            raise RMError(k, rm_last_error())
        return [(c.ticket, c.tag, bytes(c.bits[:c.n_bytes]), c.metric, c.t_arrival_us, c.t_launch_us, c.t_done_us)
                for c in self._cbuf[:k]]

    def pending(self) -> int:
        return rm_server_pending(self._h)

    def run_trace(self, requests, arrival_us, out_bits=None, out_metric=None):
        """Open-loop replay; requests = list of (decoder, llr_ptr, on_device).
        Optional numpy outputs: out_bits (n, 128) uint8, out_metric (n,)
        float32.  Returns (latency_us ndarray, stats dict)."""
        import numpy as np
        handles = np.array([d._h for d, _, _ in requests], dtype=np.uint64)
        ptrs = np.array([p for _, p, _ in requests], dtype=np.uint64)
        dev = np.array([int(v) for _, _, v in requests], dtype=np.int32)
        return self.run_trace_arrays(handles, ptrs, dev, arrival_us, out_bits, out_metric)

    def run_trace_arrays(self, dec_handles, llr_ptrs, on_device, arrival_us, out_bits=None, out_metric=None):
        """run_trace with the requests given as arrays: decoder handles
        (Decoder._h), LLR addresses and on-device flags."""
        import numpy as np
        n = len(arrival_us)
        f = {name: getattr(rm_request, name).offset for name, _ in rm_request._fields_}
        dt = np.dtype({"names": list(f), "offsets": list(f.values()), "itemsize": ctypes.sizeof(rm_request),
                       "formats": ["u8", "u8", "i4", "u8", "f8", "u8", "u8"]})
        reqs = np.zeros(max(1, n), dtype=dt)
        reqs["dec"][:n] = dec_handles
        reqs["llr"][:n] = llr_ptrs
        reqs["llr_on_device"][:n] = on_device
        reqs["tag"][:n] = np.arange(n, dtype=np.uint64)
        if out_bits is not None:
            assert out_bits.dtype == np.uint8 and out_bits.shape == (n, 128) and out_bits.flags.c_contiguous
            reqs["out_bits"][:n] = out_bits.ctypes.data + 128 * np.arange(n, dtype=np.uint64)
        if out_metric is not None:
            assert out_metric.dtype == np.float32 and out_metric.shape == (n,) and out_metric.flags.c_contiguous
            reqs["out_metric"][:n] = out_metric.ctypes.data + 4 * np.arange(n, dtype=np.uint64)
        arr = np.ascontiguousarray(arrival_us, dtype=np.float64)
        lat = np.zeros(n, dtype=np.float64)
        st = np.zeros(4, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = rm_server_run_trace(self._h, reqs.ctypes.data_as(ctypes.POINTER(rm_request)), arr.ctypes.data_as(dp), n,
                                 lat.ctypes.data_as(dp), st.ctypes.data_as(dp))
        if rc != RM_OK:
            raise RMError(rc, rm_last_error())
        return lat, {"elapsed_us": st[0], "batches": int(st[1]), "refused": int(st[2]), "largest_batch": int(st[3])}

    def close(self, _destroy=rm_server_destroy):
        if getattr(self, "_h", 0):
            _destroy(self._h)
            self._h = 0

    def __del__(self):
        self.close()


def perm_tables(m: int, r: int, P: int, L: int, seed: int, perm_mode: int = RM_PERM_PFHT, frame: int = 0):
    """Every affine map the decoder draws (for frame `frame` of a call in the
    fresh mode), in draw order: list of (rows, b)."""
    cap = P * (L + 2 * L * m)
    n, rows, b, md = rm_perm_tables_frame(m, r, P, L, seed, perm_mode, frame, cap)
    if n < 0:
        raise RMError(n, rm_last_error())
    return [(list(rows[16 * k:16 * k + md[k]]), int(b[k])) for k in range(n)]
