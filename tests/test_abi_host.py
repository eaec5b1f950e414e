"""Host-side checks of librmdec.so that need no GPU.

* the library loads and exports every function include/rmdec.h declares;
* the permutation draw of the library equals the oracle's own, independent
  implementation of the same published sampler (SplitMix64 + rejection);
* argument validation and the list of built kernels;
* two facts the kernels rely on: no kernel declares static LDS, and the
  large-list selection keys order as doubles the way they order as bits.
"""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2108_12550_amd as rmd
from paper_2108_12550_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rmdec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)


@pytest.mark.parametrize("m,r,P,L,seed", [(9, 2, 20, 4, 0), (8, 3, 8, 8, 3), (7, 2, 3, 1, 9), (6, 3, 2, 2, 1),
                                          (5, 1, 2, 4, 5), (4, 3, 3, 4, 6)])
def test_perm_draw_matches_oracle(m, r, P, L, seed):
    mine = rmd.perm_tables(m, r, P, L, seed)
    ref = oracle.OracleDecoder(m, r, P, L, seed=seed).perms()
    assert len(mine) == len(ref)
    for (rows, b), (rrows, rb) in zip(mine, ref):
        assert list(rows) == [int(x) for x in rrows]
        assert b == rb


@pytest.mark.parametrize("m,r,P,L,seed", [(9, 2, 4, 4, 0), (8, 3, 2, 8, 3), (7, 2, 3, 1, 9), (10, 2, 2, 1, 7),
                                          (5, 1, 2, 4, 5)])
def test_fresh_draw_matches_oracle_per_frame(m, r, P, L, seed):
    dec = oracle.OracleDecoder(m, r, P, L, seed=seed, perm_mode=oracle.PERM_FRESH)
    seen = set()
    for frame in (0, 1, 2, 777, (1 << 43) - 1):
        mine = rmd.perm_tables(m, r, P, L, seed, rmd.RM_PERM_FRESH, frame=frame)
        ref = dec.perms(frame)
        assert len(mine) == len(ref)
        for (rows, b), (rrows, rb) in zip(mine, ref):
            assert list(rows) == [int(x) for x in rrows]
            assert b == rb
        seen.add(tuple((tuple(rw), b) for rw, b in mine))
    assert len(seen) == 5  # every frame draws its own maps


def test_fresh_draw_frame_range_checked():
    for frame in (-1, 1 << 43):
        n, *_ = _lib.rm_perm_tables_frame(7, 2, 1, 1, 0, rmd.RM_PERM_FRESH, frame, 64)
        assert n == _lib.RM_E_INVAL


def test_fixed_modes_ignore_frame():
    assert rmd.perm_tables(8, 2, 3, 2, 5, frame=9) == rmd.perm_tables(8, 2, 3, 2, 5, frame=0)


def test_perm_draw_none_mode_is_identity():
    maps = rmd.perm_tables(7, 2, 1, 1, 0, rmd.RM_PERM_NONE)
    assert maps == [([1 << k for k in range(7)], 0)]


@pytest.mark.parametrize("args", [(2, 1, 1, 1), (11, 2, 1, 1), (7, 0, 1, 1), (7, 7, 1, 1), (7, 2, 0, 1),
                                  (7, 2, 1025, 1), (7, 2, 1, 3), (7, 2, 1, 12), (7, 2, 1, 128)])
def test_invalid_parameters_rejected(args):
    m, r, P, L = args
    n, *_ = _lib.rm_perm_tables(m, r, P, L, 0, rmd.RM_PERM_PFHT, 64)
    assert n == _lib.RM_E_INVAL
    assert rmd.rm_last_error()


def test_none_mode_with_list_draws_identities():
    maps = rmd.perm_tables(7, 2, 1, 4, 0, rmd.RM_PERM_NONE)
    assert maps == [([1 << k for k in range(7)], 0)] * 4


def test_small_cap_rejected():
    n, *_ = _lib.rm_perm_tables(9, 2, 20, 4, 0, rmd.RM_PERM_PFHT, 10)
    assert n == _lib.RM_E_INVAL


@pytest.mark.parametrize("m,r,L", [(7, 2, 1), (9, 2, 4), (9, 2, 1), (8, 3, 8), (8, 2, 4), (10, 2, 4), (5, 2, 2),
                                   (6, 3, 8), (5, 1, 4), (4, 3, 1), (9, 3, 4), (9, 4, 8), (8, 4, 2),
                                   (9, 4, 32), (8, 3, 64), (8, 2, 16), (9, 2, 32), (6, 2, 16), (9, 2, 64)])
def test_kernels_built_for_configs(m, r, L):
    assert rmd.rm_supported(m, r, L, rmd.RM_PERM_PFHT)


def test_kernels_cover_the_domain():
    """Every RM(r, m) with 3 <= m <= 10, 1 <= r <= m-1 is built at L = 1, 2,
    4, 8, 16 and 32 (lists of 16 and more, and the two N = 1024 leaf roots at
    L = 8, run one workgroup of 512 threads per frame)."""
    missing = [(m, r, L) for m in range(3, 11) for r in range(1, m) for L in (1, 2, 4, 8, 16, 32)
               if not rmd.rm_supported(m, r, L, rmd.RM_PERM_PFHT)]
    assert missing == []


def test_unbuilt_kernel_reported():
    # lists of 64 paths: RM(2..4, 8) and RM(2..4, 9) only
    assert not rmd.rm_supported(10, 2, 64, rmd.RM_PERM_PFHT)
    assert not rmd.rm_supported(7, 2, 64, rmd.RM_PERM_PFHT)
    assert not rmd.rm_supported(8, 1, 64, rmd.RM_PERM_PFHT)


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = rmd.rm_decoder_create(9, 2, 20, 4, 0)
    assert h == 0
    assert "HIP" in rmd.rm_last_error() or "hip" in rmd.rm_last_error()
    rmd.rm_decoder_destroy(0)  # NULL-safe


def test_null_decoder_calls():
    assert _lib.load().rm_decode_batch(None, None, 1, None, None) == _lib.RM_E_INVAL
    assert _lib.load().rm_decoder_set_stream(None, None) == _lib.RM_E_INVAL


def test_mixed_codes_compiled_into_fused_kernel():
    for m in (7, 8, 9, 10):
        assert rmd.rm_mixed_supported(m, 2, 4)
    assert not rmd.rm_mixed_supported(9, 2, 1)
    assert not rmd.rm_mixed_supported(8, 3, 8)


def test_mixed_null_and_invalid_calls():
    lib = _lib.load()
    segs = (_lib.rm_segment * 1)()
    assert lib.rm_mixed_decode(None, segs, 1) == _lib.RM_E_INVAL
    assert lib.rm_mixed_capture(None, segs, 1) == _lib.RM_E_INVAL
    assert lib.rm_mixed_replay(None) == _lib.RM_E_INVAL
    assert lib.rm_mixed_set_stream(None, None) == _lib.RM_E_INVAL
    assert lib.rm_mixed_set_grid(None, 0, 0) == _lib.RM_E_INVAL
    lib.rm_mixed_destroy(None)  # NULL-safe
    assert rmd.rm_mixed_create(0) == 0
    assert "max_tiles" in rmd.rm_last_error()


def test_mixed_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert rmd.rm_mixed_create(1024) == 0
    assert "HIP" in rmd.rm_last_error()


def test_server_codes_and_lists():
    for m, r in ((7, 2), (8, 2), (9, 2), (10, 2), (8, 3)):
        for L in (1, 4, 8):
            assert rmd.rm_server_supported(m, r, L)
    assert not rmd.rm_server_supported(9, 2, 2)
    assert not rmd.rm_server_supported(6, 3, 4)


def test_server_null_and_invalid_calls():
    lib = _lib.load()
    assert lib.rm_server_submit(None, None, None) == _lib.RM_E_INVAL
    assert lib.rm_server_poll(None, None, 0) == _lib.RM_E_INVAL
    assert lib.rm_server_register_pool(None, None, 0) == _lib.RM_E_INVAL
    assert lib.rm_server_pending(None) == 0
    lib.rm_server_destroy(None)  # NULL-safe
    for cfg in ((1024, 16, 2, 0, 0), (1 << 20, 0, 2, 0, 0), (1 << 20, 16, 5, 0, 0), (1 << 20, 16, 2, 65, 0),
                (1 << 20, 16, 2, 0, 3)):
        assert rmd.rm_server_create(rmd.rm_server_config(*cfg)) == 0
        assert "config" in rmd.rm_last_error()
    a, b = rmd.rm_server_now_us(), rmd.rm_server_now_us()
    assert 0 < a <= b


def test_server_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert rmd.rm_server_create(rmd.rm_server_config(1 << 20, 64, 2, 0, 0)) == 0
    assert "HIP" in rmd.rm_last_error()


def test_no_kernel_declares_static_lds():
    # The gathers address LDS by absolute address and form element addresses
    # by XOR, which needs the dynamic segment to start at address 0: no
    # kernel may declare a static __shared__ variable.
    csrc = os.path.join(ROOT, "paper_2108_12550_amd", "csrc")
    found = []
    for name in sorted(os.listdir(csrc)):
        if not name.endswith((".hip", ".hpp")):
            continue
        src = re.sub(r"//[^\n]*", "", open(os.path.join(csrc, name)).read())
        for line in src.splitlines():
            if "__shared__" in line and "extern __shared__" not in line:
                found.append(f"{name}: {line.strip()}")
    assert not found, found


def test_selection_keys_order_as_doubles():
    # The large-list kernels compare 64-bit keys (high word: the bits of a
    # non-negative float, finite or +inf; low word: any index code) with
    # v_min_f64 / v_max_f64.  For such patterns the order of the doubles is
    # the unsigned order of the bits, and the double +inf (the padding key)
    # lies above every key.
    rng = np.random.default_rng(7)
    n = 200_000
    hi = rng.integers(0, 0x7F800001, size=n, dtype=np.uint64)
    hi[: n // 10] = rng.integers(0, 4, size=n // 10, dtype=np.uint64)  # near-equal high words
    hi[n // 10 : n // 5] = 0x7F800000  # +inf metrics
    lo = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
    keys = (hi << np.uint64(32)) | lo
    a, b = keys, rng.permutation(keys)
    da, db = a.view(np.float64), b.view(np.float64)
    assert np.all(np.isfinite(da)) and np.all(da >= 0)
    assert np.array_equal(a < b, da < db)
    assert np.array_equal(a == b, da == db)
    pad = np.array([0x7FF0000000000000], dtype=np.uint64).view(np.float64)[0]
    assert np.all(da < pad) and np.all(keys < np.uint64(0x7FF0000000000000))


@pytest.mark.parametrize("m,r", [(7, 2), (9, 2), (8, 3), (5, 1), (4, 3), (10, 2)])
def test_codeword_to_info_inverts_the_oracle_encoder(m, r):
    """rm_codeword_to_info against the oracle's own x = u G^{(x)m} encoder:
    random u on the information set, frozen positions zero."""
    rng = np.random.default_rng(m * 10 + r)
    iset = oracle.info_set(m, r).astype(bool)
    n = 20
    u = np.zeros((n, 1 << m), np.uint8)
    u[:, iset] = rng.integers(0, 2, size=(n, int(iset.sum())))
    x = np.stack([oracle.encode(m, row) for row in u])
    info, bad = rmd.codeword_to_info(m, r, np.packbits(x, axis=-1, bitorder="little"))
    assert bad == 0
    assert info.shape == (n, rmd.code_dimension(m, r))
    assert np.array_equal(info, u[:, iset])


def test_codeword_to_info_flags_non_codewords():
    import synth
    x, _ = synth.frames(9, 2, 16, 3.0, seed=4)  # codewords (polynomial evaluations)
    cw = np.packbits(x, axis=-1, bitorder="little")
    _, bad = rmd.codeword_to_info(9, 2, cw)
    assert bad == 0
    cw[3, 5] ^= 0x10  # one flipped bit: weight-1 error, not a codeword
    cw[7, 0] ^= 0x01
    _, bad = rmd.codeword_to_info(9, 2, cw)
    assert bad == 2
    rc, _ = _lib.rm_codeword_to_info(9, 9, cw.ctypes.data, 1, cw.ctypes.data)
    assert rc == rmd.RM_E_INVAL
