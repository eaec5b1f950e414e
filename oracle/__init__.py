"""TEST INFRASTRUCTURE: ctypes binding of the plain CPU oracle (rm_oracle.c).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this package.  It is independent of the HIP decoder: it shares no
code, header, table or generator with ``paper_2108_12550_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rm_oracle.c")
_LIB = os.path.join(_HERE, "librmoracle.so")

PERM_NONE = 0
PERM_PFHT = 1
PERM_FRESH = 2

NODE_INTERNAL, NODE_PERM, NODE_FHTL, NODE_SPCL = 0, 1, 2, 3
NODE_NAMES = {NODE_INTERNAL: "internal", NODE_PERM: "perm", NODE_FHTL: "fhtl", NODE_SPCL: "spcl"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: scalar binary32, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-pthread", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        L.rmo_create.restype = ctypes.c_void_p
        L.rmo_create.argtypes = [ctypes.c_int] * 5 + [ctypes.c_uint64]
        L.rmo_destroy.argtypes = [ctypes.c_void_p]
        L.rmo_decode.argtypes = [ctypes.c_void_p, P(ctypes.c_float), P(ctypes.c_uint8), P(ctypes.c_float)]
        L.rmo_decode_frame.argtypes = [ctypes.c_void_p, P(ctypes.c_float), ctypes.c_int64, P(ctypes.c_uint8),
                                       P(ctypes.c_float)]
        L.rmo_decode_batch.argtypes = [ctypes.c_void_p, P(ctypes.c_float), ctypes.c_int64, P(ctypes.c_uint8),
                                       P(ctypes.c_float), ctypes.c_int]
        L.rmo_decode_batch_at.argtypes = [ctypes.c_void_p, P(ctypes.c_float), ctypes.c_int64, ctypes.c_int64,
                                          P(ctypes.c_uint8), P(ctypes.c_float), ctypes.c_int]
        L.rmo_info_set.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_uint8)]
        L.rmo_encode.argtypes = [ctypes.c_int, P(ctypes.c_uint8), P(ctypes.c_uint8)]
        L.rmo_fht.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_float), ctypes.c_float, P(ctypes.c_uint8),
                              P(ctypes.c_float), P(ctypes.c_int)]
        L.rmo_spcl.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_uint8),
                               P(ctypes.c_float), P(ctypes.c_int)]
        L.rmo_fhtl.argtypes = L.rmo_spcl.argtypes
        L.rmo_schedule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_int), ctypes.c_int]
        L.rmo_perm_count.argtypes = [ctypes.c_void_p]
        L.rmo_perm_export.argtypes = [ctypes.c_void_p, P(ctypes.c_uint16), P(ctypes.c_uint16), P(ctypes.c_int),
                                      ctypes.c_int]
        L.rmo_perm_export_frame.argtypes = [ctypes.c_void_p, ctypes.c_int64, P(ctypes.c_uint16), P(ctypes.c_uint16),
                                            P(ctypes.c_int), ctypes.c_int]
        L.rmo_splitmix64_next.restype = ctypes.c_uint64
        L.rmo_splitmix64_next.argtypes = [P(ctypes.c_uint64)]
        L.rmo_lm.restype = ctypes.c_float
        L.rmo_lm.argtypes = [ctypes.c_int, P(ctypes.c_float), ctypes.c_uint32]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleDecoder:
    """p-FHT-FSCL-L-M (Alg. 5 over Alg. 2-4 and the SPC rules), scalar binary32."""

    def __init__(self, m: int, r: int, P: int, L: int, seed: int = 0, perm_mode: int = PERM_PFHT):
        self.m, self.r, self.P, self.L, self.seed, self.perm_mode = m, r, P, L, seed, perm_mode
        self.N = 1 << m
        self._h = lib().rmo_create(m, r, P, L, perm_mode, ctypes.c_uint64(seed))
        if not self._h:
            raise ValueError(f"oracle rejects RM(r={r}, m={m}) P={P} L={L} mode={perm_mode}")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().rmo_destroy(h)
            self._h = None

    def decode(self, y: np.ndarray, frame: int = 0):
        """Decode one frame; `frame` is its index (it keys the maps of the fresh mode)."""
        y = np.ascontiguousarray(y, dtype=np.float32)
        x = np.zeros(self.N, dtype=np.uint8)
        pm = np.zeros(1, dtype=np.float32)
        lib().rmo_decode_frame(self._h, _p(y, ctypes.c_float), int(frame), _p(x, ctypes.c_uint8),
                               _p(pm, ctypes.c_float))
        return x, float(pm[0])

    def decode_batch(self, llr: np.ndarray, n_threads: int = 1, frame0: int = 0):
        """llr: (n_frames, N) float32, frames numbered frame0, frame0+1, ...
        Returns packed bits (n, N/8) uint8 and metrics (n,)."""
        llr = np.ascontiguousarray(llr, dtype=np.float32).reshape(-1, self.N)
        n = llr.shape[0]
        bits = np.zeros((n, self.N // 8), dtype=np.uint8)
        pm = np.zeros(n, dtype=np.float32)
        rc = lib().rmo_decode_batch_at(self._h, _p(llr, ctypes.c_float), n, int(frame0),
                                       _p(bits, ctypes.c_uint8), _p(pm, ctypes.c_float), int(n_threads))
        if rc != 0:
            raise RuntimeError("oracle batch decode failed")
        return bits, pm

    def perms(self, frame: int = 0):
        """All drawn affine maps in draw order: list of (rows[m], b) (in the
        fresh mode, those of frame `frame`)."""
        L = lib()
        k = L.rmo_perm_count(self._h)
        rows = np.zeros(k * 16, dtype=np.uint16)
        b = np.zeros(k, dtype=np.uint16)
        md = np.zeros(k, dtype=np.int32)
        got = L.rmo_perm_export_frame(self._h, int(frame), _p(rows, ctypes.c_uint16), _p(b, ctypes.c_uint16),
                                      _p(md, ctypes.c_int), k)
        assert got == k
        return [(rows[i * 16:i * 16 + md[i]].copy(), int(b[i])) for i in range(k)]


def lm(v: np.ndarray, d: int) -> float:
    """Alg. 2's LM of the pairs {u, u ^ d} of v (2^m float32 LLRs, d != 0),
    summed in the oracle's order (rmo_lm)."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    m = int(v.size).bit_length() - 1
    assert v.size == 1 << m and 0 < d < v.size
    return float(lib().rmo_lm(m, _p(v, ctypes.c_float), ctypes.c_uint32(d)))


def info_set(m: int, r: int) -> np.ndarray:
    out = np.zeros(1 << m, dtype=np.uint8)
    assert lib().rmo_info_set(m, r, _p(out, ctypes.c_uint8)) == 0
    return out


def encode(m: int, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.uint8)
    x = np.zeros(1 << m, dtype=np.uint8)
    assert lib().rmo_encode(m, _p(u, ctypes.c_uint8), _p(x, ctypes.c_uint8)) == 0
    return x


def fht(s: int, L: int, alpha: np.ndarray, pm_in: float = 0.0):
    """Alg. 4 on one path: (codewords (k, n), metrics (k,), transform indices (k,))."""
    n = 1 << s
    k = min(L, n)
    alpha = np.ascontiguousarray(alpha, dtype=np.float32)
    cw = np.zeros((k, n), dtype=np.uint8)
    pm = np.zeros(k, dtype=np.float32)
    idx = np.zeros(max(k, 1), dtype=np.int32)
    got = lib().rmo_fht(s, L, _p(alpha, ctypes.c_float), ctypes.c_float(pm_in), _p(cw, ctypes.c_uint8),
                        _p(pm, ctypes.c_float), _p(idx, ctypes.c_int))
    assert got == k
    return cw, pm, idx[:k]


def _list_node(fn, s, L, alpha, pm_in):
    n = 1 << s
    alpha = np.ascontiguousarray(alpha, dtype=np.float32).reshape(L, n)
    pm_in = np.ascontiguousarray(pm_in, dtype=np.float32).reshape(L)
    x = np.zeros((L, n), dtype=np.uint8)
    pm = np.zeros(L, dtype=np.float32)
    anc = np.zeros(L, dtype=np.int32)
    assert fn(s, L, _p(alpha, ctypes.c_float), _p(pm_in, ctypes.c_float), _p(x, ctypes.c_uint8),
              _p(pm, ctypes.c_float), _p(anc, ctypes.c_int)) == 0
    return x, pm, anc


def spcl(s: int, L: int, alpha: np.ndarray, pm_in: np.ndarray):
    """SPC list node RM(s-1, s) on L input paths: (x (L, n), pm (L,), anc (L,))."""
    return _list_node(lib().rmo_spcl, s, L, alpha, pm_in)


def fhtl(s: int, L: int, alpha: np.ndarray, pm_in: np.ndarray):
    """Alg. 3 on L input paths of RM(1, s): (x (L, n), pm (L,), anc (L,))."""
    return _list_node(lib().rmo_fhtl, s, L, alpha, pm_in)


def schedule(m: int, r: int, perm_mode: int = PERM_PFHT):
    """Preorder node list [(kind_name, r, m), ...]."""
    cap = 3 * (1 << (m + 1))
    out = np.zeros(cap, dtype=np.int32)
    k = lib().rmo_schedule(m, r, perm_mode, _p(out, ctypes.c_int), cap)
    assert k >= 0
    return [(NODE_NAMES[int(out[3 * i])], int(out[3 * i + 1]), int(out[3 * i + 2])) for i in range(k)]


def splitmix64(seed: int, count: int):
    st = ctypes.c_uint64(seed)
    return [int(lib().rmo_splitmix64_next(ctypes.byref(st))) for _ in range(count)]
