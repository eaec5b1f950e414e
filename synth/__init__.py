"""Seeded synthetic channel inputs shared by the tests, the benchmark and smoke().

This module holds none of the decoder's arithmetic.  It transmits uniformly
random codewords of RM(r, m) over BPSK/AWGN and returns float32 channel LLRs:

* a codeword is the evaluation, at every point z of F2^m (z_k = bit k of the
  position index), of a polynomial of degree <= r with uniform random
  coefficients -- Reed and Muller's own description of the code (Section II-A
  defines the same code through u G^{(x)m});
* y = (1 - 2x) + z with z ~ N(0, sigma^2) and LLR = 2y / sigma^2 (Section II-A);
* sigma^2 = N / (2 K 10^{Eb/N0 / 10}), the rate-adjusted Eb/N0 convention.

Frames are generated in fixed chunks of ``CHUNK`` frames, chunk c seeded by
(seed, c), so a shorter request is always a prefix of a longer one.
"""
from __future__ import annotations

import itertools
import os
from concurrent.futures import ThreadPoolExecutor
from math import comb

import numpy as np

CHUNK = 4096


def code_dimension(m: int, r: int) -> int:
    """K = sum_{i<=r} C(m, i)."""
    return sum(comb(m, i) for i in range(r + 1))


def sigma2(ebn0_db, m: int, r: int):
    n = 1 << m
    k = code_dimension(m, r)
    return n / (2.0 * k * 10.0 ** (np.asarray(ebn0_db, dtype=np.float64) / 10.0))


def monomial_table(m: int, r: int) -> np.ndarray:
    """(K, N) 0/1 table: row S evaluates prod_{k in S} z_k at every point z."""
    n = 1 << m
    z = np.arange(n)
    rows = []
    for deg in range(r + 1):
        for S in itertools.combinations(range(m), deg):
            mask = sum(1 << k for k in S)
            rows.append(((z & mask) == mask).astype(np.uint8))
    return np.stack(rows)


def _chunk(m, r, seed, c, ebn0_db_chunk, mon):
    n = 1 << m
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(c)])))
    coef = rng.integers(0, 2, size=(CHUNK, mon.shape[0]), dtype=np.uint8)
    # integer sums of at most K ones are exact in binary32
    x = ((coef.astype(np.float32) @ mon.astype(np.float32)).astype(np.int32) & 1).astype(np.uint8)
    noise = rng.standard_normal((CHUNK, n))
    s2 = np.broadcast_to(sigma2(ebn0_db_chunk, m, r), (CHUNK,)).reshape(CHUNK, 1)
    y = (1.0 - 2.0 * x) + np.sqrt(s2) * noise
    llr = (2.0 * y / s2).astype(np.float32)
    return x, llr


def frames(m: int, r: int, n_frames: int, ebn0_db, seed: int = 0):
    """Return (codewords (n, N) uint8, llr (n, N) float32).

    ``ebn0_db`` is a scalar or a length-``n_frames`` array (per-frame Eb/N0).
    """
    n = 1 << m
    mon = monomial_table(m, r)
    per_frame = np.ndim(ebn0_db) > 0
    if per_frame:
        ebn0_db = np.asarray(ebn0_db, dtype=np.float64)
        assert ebn0_db.shape == (n_frames,)
    xs = np.empty((n_frames, n), dtype=np.uint8)
    ls = np.empty((n_frames, n), dtype=np.float32)

    def one(c):
        f0 = c * CHUNK
        f1 = min(n_frames, f0 + CHUNK)
        if per_frame:
            e = np.zeros(CHUNK)
            e[: f1 - f0] = ebn0_db[f0:f1]
            e[f1 - f0:] = ebn0_db[f1 - 1]
        else:
            e = float(ebn0_db)
        x, llr = _chunk(m, r, seed, c, e, mon)
        xs[f0:f1] = x[: f1 - f0]
        ls[f0:f1] = llr[: f1 - f0]

    n_chunks = (n_frames + CHUNK - 1) // CHUNK
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1, max(1, n_chunks))) as ex:
        list(ex.map(one, range(n_chunks)))
    return xs, ls


def uniform_ebn0(n_frames: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Per-frame Eb/N0 drawn uniformly from [lo, hi] (seeded)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x5EB0])))
    return rng.uniform(lo, hi, size=n_frames)


def pack_bits(x: np.ndarray) -> np.ndarray:
    """(n, N) 0/1 -> (n, N/8) bytes, bit i at byte i>>3, bit i&7."""
    return np.packbits(np.asarray(x, dtype=np.uint8), axis=-1, bitorder="little")


def unpack_bits(b: np.ndarray, n: int) -> np.ndarray:
    return np.unpackbits(np.asarray(b, dtype=np.uint8), axis=-1, bitorder="little", count=n)
