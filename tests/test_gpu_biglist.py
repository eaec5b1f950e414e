"""Parity of the large-list kernels (L = 16, 32, 64: one workgroup per
frame, the list in LDS) with the oracle, through the C ABI.

Codewords must agree bit for bit and final metrics within 1e-5 relative,
in the permuted, plain and fresh-permutation modes, on integer-valued LLRs
(every tie-break rule) and on a larger sampled launch.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2108_12550_amd as rmd
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

NONE, PFHT, FRESH = rmd.RM_PERM_NONE, rmd.RM_PERM_PFHT, rmd.RM_PERM_FRESH
THREADS = min(16, os.cpu_count() or 1)
PM_RTOL = 1e-5
# every internal code (1 < r < m-1) with 4 <= m <= 10 at L = 16 and 32, and
# L = 64 for RM(2..4, 8) and RM(2..4, 9)
BUILT = ([(m, r, L) for m in range(4, 11) for r in range(2, m - 1) for L in (16, 32)]
         + [(m, r, 64) for m in (8, 9) for r in (2, 3, 4)])
# leaf roots RM(1, m) and RM(m-1, m) at L = 16 and 32, and at L = 8 for N = 1024
LEAF = ([(m, r, L) for m in range(3, 11) for r in (1, m - 1) for L in (16, 32)]
        + [(10, 1, 8), (10, 9, 8)])


def gpu_decode(m, r, P, L, seed, mode, llr):
    dec = rmd.Decoder(m, r, P, L, seed=seed, perm_mode=mode)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    bits, pm = dec.decode(t)
    torch.cuda.synchronize()
    out = bits.cpu().numpy(), pm.cpu().numpy()
    dec.close()
    return out


def assert_parity(got, ref, label):
    gb, gp = got
    rb, rp = ref
    bad = np.nonzero(np.any(gb != rb, axis=1))[0]
    assert bad.size == 0, f"{label}: {bad.size} frames differ in bits, first {bad[:8]}"
    rel = np.abs(gp.astype(np.float64) - rp) / np.maximum(1.0, np.abs(rp))
    assert rel.max() <= PM_RTOL, f"{label}: metric rel diff {rel.max()}"


def check(m, r, P, L, mode, llr, seed):
    label = f"RM({r},{m}) P={P} L={L} mode={mode} seed={seed} n={llr.shape[0]}"
    print("case", label, flush=True)
    od = oracle.OracleDecoder(m, r, P, L, seed=seed, perm_mode=mode)
    assert_parity(gpu_decode(m, r, P, L, seed, mode, llr), od.decode_batch(llr, n_threads=THREADS), label)


@pytest.mark.parametrize("m,r,L", BUILT + LEAF)
def test_permuted_large_lists(m, r, L):
    _, llr = synth.frames(m, r, 24, 2.0, seed=700 + m * 10 + r + L)
    check(m, r, 2, L, PFHT, llr, seed=L + r)


@pytest.mark.parametrize("m,r,L", [(9, 4, 32), (8, 3, 64), (9, 2, 16), (8, 2, 32), (8, 4, 64), (7, 3, 16),
                                   (4, 2, 32), (8, 1, 16), (10, 9, 32), (3, 2, 32), (10, 1, 8)])
def test_plain_large_lists(m, r, L):
    """FHT-FSCL-L: one active path at the start, no permutations."""
    _, llr = synth.frames(m, r, 30, 2.5, seed=800 + m * 10 + r + L)
    check(m, r, 1, L, NONE, llr, seed=0)


@pytest.mark.parametrize("m,r,P,L", [(9, 4, 2, 32), (8, 3, 1, 64), (9, 2, 3, 16), (9, 6, 2, 32), (5, 3, 2, 16),
                                     (10, 1, 2, 32), (6, 5, 3, 16), (10, 9, 1, 8)])
def test_fresh_large_lists(m, r, P, L):
    _, llr = synth.frames(m, r, 20, 2.0, seed=900 + m * 10 + r + L)
    check(m, r, P, L, FRESH, llr, seed=5)


@pytest.mark.parametrize("m,r,L", [(8, 3, 32), (9, 2, 16), (8, 4, 64), (6, 2, 16), (4, 2, 32), (9, 7, 32),
                                   (7, 1, 32), (9, 8, 16), (3, 1, 32), (10, 9, 8)])
def test_integer_llr_ties_large_lists(m, r, L):
    rng = np.random.default_rng(m * 1000 + L)
    llr = rng.integers(-2, 3, size=(20, 1 << m)).astype(np.float32)
    check(m, r, 2, L, PFHT, llr, seed=1)
    check(m, r, 1, L, NONE, llr, seed=0)


def test_all_zero_llr_large_list():
    check(8, 3, 2, 32, PFHT, np.zeros((4, 256), np.float32), seed=2)


@pytest.mark.parametrize("m,r,L", [(8, 1, 32), (8, 7, 16), (4, 3, 32), (10, 9, 8)])
def test_all_zero_llr_leaf_roots(m, r, L):
    """Every candidate ties: the leaf-root kernel's order of paths and
    candidates decides the output alone."""
    llr = np.zeros((4, 1 << m), np.float32)
    check(m, r, 2, L, PFHT, llr, seed=2)
    check(m, r, 1, L, NONE, llr, seed=0)


def test_noiseless_large_list():
    x, _ = synth.frames(9, 4, 16, 3.0, seed=9)
    llr = (8.0 * (1.0 - 2.0 * x)).astype(np.float32)
    bits, pm = gpu_decode(9, 4, 1, 32, 0, PFHT, llr)
    assert np.array_equal(synth.unpack_bits(bits, 512), x)
    assert np.all(pm == 0.0)


def test_unbuilt_large_list_reported():
    assert rmd.rm_supported(9, 4, 32, PFHT) == 1
    assert rmd.rm_supported(9, 2, 64, PFHT) == 1
    assert rmd.rm_supported(10, 2, 64, PFHT) == 0  # 4*L*N bytes of LLRs exceed the LDS of a workgroup
    assert rmd.rm_supported(10, 2, 32, PFHT) == 1
    assert rmd.rm_supported(9, 5, 32, PFHT) == 1
    assert rmd.rm_supported(8, 1, 16, PFHT) == 1
    assert rmd.rm_supported(7, 6, 64, PFHT) == 0   # lists of 64 only for RM(2..4, 8) and RM(2..4, 9)


def test_noiseless_leaf_roots():
    """Leaf roots decode a noiseless codeword exactly, with metric 0."""
    for m, r, L in [(10, 1, 32), (9, 8, 16), (3, 2, 32), (10, 9, 8)]:
        x, _ = synth.frames(m, r, 8, 3.0, seed=19 + m)
        llr = (8.0 * (1.0 - 2.0 * x)).astype(np.float32)
        print(f"case noiseless RM({r},{m}) L={L}", flush=True)
        bits, pm = gpu_decode(m, r, 2, L, 4, PFHT, llr)
        assert np.array_equal(synth.unpack_bits(bits, 1 << m), x)
        assert np.all(pm == 0.0)


def test_leaf_root_sampled_launch():
    """RM(1,10) with L = 32 (one first-order root), 4096 frames in one launch:
    every output a codeword, sampled frames against the oracle."""
    n = 4096
    _, llr = synth.frames(10, 1, n, -3.0, seed=78)
    print("case sampled RM(1,10) P=2 L=32 n=4096", flush=True)
    bits, pm = gpu_decode(10, 1, 2, 32, 6, PFHT, llr)
    h = torch.from_numpy(synth.monomial_table(10, 10 - 1 - 1).astype(np.float32)).cuda()
    xb = torch.from_numpy(synth.unpack_bits(bits, 1024).astype(np.float32)).cuda()
    assert int(torch.remainder(xb @ h.T, 2.0).sum().item()) == 0
    idx = np.sort(np.random.default_rng(8).choice(n, 24, replace=False))
    od = oracle.OracleDecoder(10, 1, 2, 32, seed=6)
    assert_parity((bits[idx], pm[idx]), od.decode_batch(llr[idx], n_threads=THREADS), "sampled")


def test_table5_rm29_l64_plain_and_permuted():
    """Table 5's p-FHT-FSCL-64 on RM(2,9): the list takes 157 KB of LDS."""
    _, llr = synth.frames(9, 2, 16, 1.5, seed=950)
    check(9, 2, 1, 64, PFHT, llr, seed=3)
    check(9, 2, 1, 64, NONE, llr, seed=0)


def test_large_list_sampled_launch():
    """RM(4,9) with L = 32 (Fig. 5(c)'s p-FHT-FSCL-32), 8192 frames in one
    launch: every output a codeword, sampled frames against the oracle."""
    n = 8192
    _, llr = synth.frames(9, 4, n, 2.5, seed=77)
    print("case sampled RM(4,9) P=1 L=32 n=8192", flush=True)
    bits, pm = gpu_decode(9, 4, 1, 32, 0, PFHT, llr)
    h = torch.from_numpy(synth.monomial_table(9, 9 - 4 - 1).astype(np.float32)).cuda()
    xb = torch.from_numpy(synth.unpack_bits(bits, 512).astype(np.float32)).cuda()
    assert int(torch.remainder(xb @ h.T, 2.0).sum().item()) == 0
    idx = np.sort(np.random.default_rng(7).choice(n, 24, replace=False))
    od = oracle.OracleDecoder(9, 4, 1, 32, seed=0)
    assert_parity((bits[idx], pm[idx]), od.decode_batch(llr[idx], n_threads=THREADS), "sampled")


def test_bench_launch_rm38_l64_sampled():
    """The launch the large-list benchmark times: RM(3,8), one decoder with
    L = 64 (Table 5's p-FHT-FSCL-64), 32768 frames at 3.0 dB: every output a
    codeword, sampled frames against the oracle."""
    n = 32768
    _, llr = synth.frames(8, 3, n, 3.0, seed=31)
    print("case sampled RM(3,8) P=1 L=64 n=32768", flush=True)
    bits, pm = gpu_decode(8, 3, 1, 64, 0, PFHT, llr)
    h = torch.from_numpy(synth.monomial_table(8, 8 - 3 - 1).astype(np.float32)).cuda()
    xb = torch.from_numpy(synth.unpack_bits(bits, 256).astype(np.float32)).cuda()
    assert int(torch.remainder(xb @ h.T, 2.0).sum().item()) == 0
    idx = np.sort(np.random.default_rng(31).choice(n, 32, replace=False))
    od = oracle.OracleDecoder(8, 3, 1, 64, seed=0)
    assert_parity((bits[idx], pm[idx]), od.decode_batch(llr[idx], n_threads=THREADS), "bench launch sample")
