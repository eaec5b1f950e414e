"""Parity of the HIP decoder with the CPU oracle, through the C ABI.

Every case decodes the same seeded synthetic frames on the GPU and with the
oracle and requires identical codewords (bit-exact) and final metrics within
1e-5 relative (both follow one operation order, so they are expected to be
equal).  Sizes span several waves and a ragged tail; the full-size launch of
the benchmark is checked on sampled frames and by code membership of every
frame.
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

NONE, PFHT = rmd.RM_PERM_NONE, rmd.RM_PERM_PFHT
THREADS = min(16, os.cpu_count() or 1)
PM_RTOL = 1e-5


def gpu_decode(m, r, P, L, seed, mode, llr, waves=0):
    dec = rmd.Decoder(m, r, P, L, seed=seed, perm_mode=mode, waves_per_block=waves)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    bits, pm = dec.decode(t)
    torch.cuda.synchronize()
    out = bits.cpu().numpy(), pm.cpu().numpy()
    dec.close()
    return out


def oracle_decode(m, r, P, L, seed, mode, llr):
    od = oracle.OracleDecoder(m, r, P, L, seed=seed, perm_mode=mode)
    return od.decode_batch(llr, n_threads=THREADS)


def assert_parity(got, ref, label):
    gb, gp = got
    rb, rp = ref
    bad = np.nonzero(np.any(gb != rb, axis=1))[0]
    assert bad.size == 0, f"{label}: {bad.size} frames differ in bits, first {bad[:8]}"
    rel = np.abs(gp.astype(np.float64) - rp) / np.maximum(1.0, np.abs(rp))
    assert rel.max() <= PM_RTOL, f"{label}: metric rel diff {rel.max()}"


def check(m, r, P, L, mode, llr, seed=0, waves=0):
    label = f"RM({r},{m}) P={P} L={L} mode={mode} seed={seed} n={llr.shape[0]}"
    print("case", label, flush=True)
    assert_parity(gpu_decode(m, r, P, L, seed, mode, llr, waves), oracle_decode(m, r, P, L, seed, mode, llr), label)


# --- the benchmark configurations, at sizes the oracle finishes in seconds ---

def test_plain_fht_fsc_rm27_all_frames():
    _, llr = synth.frames(7, 2, 10000, 3.0, seed=0)
    check(7, 2, 1, 1, NONE, llr)


@pytest.mark.parametrize("ebn0", [2.0, 3.0, 4.0])
def test_rm29_p20_l4(ebn0):
    _, llr = synth.frames(9, 2, 197, ebn0, seed=11)
    check(9, 2, 20, 4, PFHT, llr, seed=5)


def test_rm29_p512_l1():
    _, llr = synth.frames(9, 2, 21, 2.5, seed=12)
    check(9, 2, 512, 1, PFHT, llr, seed=6)


@pytest.mark.parametrize("ebn0", [2.0, 3.5])
def test_rm38_p8_l8(ebn0):
    _, llr = synth.frames(8, 3, 131, ebn0, seed=13)
    check(8, 3, 8, 8, PFHT, llr, seed=7)


@pytest.mark.parametrize("m,P", [(7, 8), (8, 16), (10, 32)])
def test_mixed_codes_l4(m, P):
    n = 67
    e = synth.uniform_ebn0(n, 2.0, 4.0, seed=m)
    _, llr = synth.frames(m, 2, n, e, seed=m)
    check(m, 2, P, 4, PFHT, llr, seed=m)


# --- the tree shapes and list sizes ---

@pytest.mark.parametrize("m,r", [(4, 2), (5, 2), (6, 2), (5, 3), (6, 3), (7, 3), (8, 2), (9, 2), (8, 3), (7, 2)])
@pytest.mark.parametrize("L", [1, 2, 4, 8])
def test_codes_and_lists(m, r, L):
    _, llr = synth.frames(m, r, 70, 1.0, seed=100 + m * 10 + r)
    check(m, r, 3, L, PFHT, llr, seed=L)


@pytest.mark.parametrize("m,r,L", [(3, 1, 1), (3, 1, 4), (4, 1, 4), (5, 1, 1), (6, 1, 4), (3, 2, 1), (3, 2, 4),
                                   (4, 3, 4), (5, 4, 1), (5, 4, 4)])
def test_leaf_roots(m, r, L):
    _, llr = synth.frames(m, r, 65, 0.5, seed=200 + m)
    check(m, r, 2, L, PFHT, llr, seed=3)


# every (m, r, L <= 8) of the domain: leaf roots, higher orders, lists of 2
# and 8 (RM(1,10) and RM(9,10) at L = 8 run one workgroup per frame)
DOMAIN_REST = [(m, r, L) for m in range(3, 11) for r in range(1, m) for L in (1, 2, 4, 8)]


@pytest.mark.parametrize("m,r,L", DOMAIN_REST)
def test_whole_domain(m, r, L):
    """Each built shape against the oracle: 2 decoders, 24 frames at 1.5 dB
    (with frame errors), permuted mode."""
    _, llr = synth.frames(m, r, 24, 1.5, seed=900 + 16 * m + r)
    check(m, r, 2, L, PFHT, llr, seed=L + 3)


@pytest.mark.parametrize("m,r", [(9, 3), (9, 4), (8, 4)])
@pytest.mark.parametrize("L", [1, 2, 4, 8])
def test_higher_order_codes(m, r, L):
    """RM(3,9), RM(4,9), RM(4,8): deeper permutation domains, more SPC leaves."""
    _, llr = synth.frames(m, r, 60, 3.0, seed=500 + m * 10 + r)
    check(m, r, 3, L, PFHT, llr, seed=L + 1)


def test_table5_rm48_p16_l4():
    _, llr = synth.frames(8, 4, 96, 3.5, seed=77)
    check(8, 4, 16, 4, PFHT, llr, seed=2)


@pytest.mark.parametrize("m,r,L", [(7, 2, 2), (7, 2, 4), (9, 2, 4), (9, 2, 8), (8, 3, 4), (8, 3, 8), (10, 2, 4),
                                   (9, 3, 4), (9, 4, 8),
                                   (5, 2, 8), (6, 1, 4), (4, 3, 4)])
def test_plain_list_mode(m, r, L):
    """FHT-FSCL-L without permutations: one active path at the start."""
    _, llr = synth.frames(m, r, 150, 2.0, seed=300 + m * 10 + L)
    check(m, r, 1, L, NONE, llr)


def test_plain_mode_other_codes():
    for m, r in [(5, 2), (8, 3), (9, 2)]:
        _, llr = synth.frames(m, r, 40, 2.0, seed=300 + m)
        check(m, r, 1, 1, NONE, llr)


# --- one decoder per frame (P = 1): the frame-packed kernel runs D frames
# per wave, one per decoder slot; counts leave a ragged last group ---

@pytest.mark.parametrize("m,r,L,mode,n", [
    (7, 2, 1, NONE, 8 * 37 + 5),   # the plain FHT-FSC decoder of RM(2,7): 8 frames per wave
    (9, 2, 1, PFHT, 8 * 13 + 7),
    (9, 2, 4, PFHT, 2 * 41 + 1),   # p-FHT-FSCL-4 (M = 1): 2 frames per wave
    (7, 2, 4, PFHT, 4 * 11 + 3),   # 4 frames per wave
    (8, 3, 2, PFHT, 4 * 20 + 3),   # two permutation-domain nodes
    (6, 1, 4, NONE, 4 * 9 + 2),    # first-order root
    (5, 4, 4, PFHT, 4 * 9 + 1),    # SPC root
    (9, 2, 4, NONE, 2 * 30 + 1),
])
def test_single_decoder_packed(m, r, L, mode, n):
    _, llr = synth.frames(m, r, n, 2.5, seed=600 + 10 * m + L)
    check(m, r, 1, L, mode, llr)


@pytest.mark.parametrize("waves", [1, 2, 4])
def test_single_decoder_packed_tile_invariance(waves):
    _, llr = synth.frames(7, 2, 301, 2.0, seed=610)
    ref = gpu_decode(7, 2, 1, 1, 0, NONE, llr, waves=0)
    got = gpu_decode(7, 2, 1, 1, 0, NONE, llr, waves=waves)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    for k in (0, 7, 8, 300):  # alone: a group of one frame
        one = gpu_decode(7, 2, 1, 1, 0, NONE, llr[k:k + 1], waves=waves)
        assert np.array_equal(one[0][0], ref[0][k]) and one[1][0] == ref[1][k]


# --- ties: integer-valued and all-zero LLRs exercise every tie-break rule ---

@pytest.mark.parametrize("m,r,P,L", [(5, 2, 2, 4), (7, 2, 3, 4), (8, 3, 2, 8), (9, 2, 4, 4), (6, 3, 2, 2),
                                     (9, 2, 3, 1)])
def test_integer_llr_ties(m, r, P, L):
    rng = np.random.default_rng(m * 100 + L)
    llr = rng.integers(-3, 4, size=(50, 1 << m)).astype(np.float32)
    check(m, r, P, L, PFHT, llr, seed=1)


@pytest.mark.parametrize("m,r,P,L", [(8, 3, 4, 8), (9, 2, 6, 4), (7, 2, 4, 8)])
def test_integer_llr_ties_spc_split_stop(m, r, P, L):
    """The SPC splits stop once every flip scores above every keep; with
    LLRs in {-2, ..., 2} flips often tie the largest keep exactly, where
    stopping a split early would go wrong if the rule were not strict."""
    rng = np.random.default_rng(700 + m * 10 + L)
    llr = rng.integers(-2, 3, size=(300, 1 << m)).astype(np.float32)
    check(m, r, P, L, PFHT, llr, seed=5)


def test_misaligned_arrays_rejected():
    """Frames are read in 16-byte and codewords written in 8-byte words: a
    misaligned array is refused before anything is queued."""
    dec = rmd.Decoder(7, 2, 1, 1, seed=0, perm_mode=NONE)
    # 4 frames of RM(2,7): 512 LLRs in, 64 codeword bytes and 4 metrics out;
    # every buffer below holds that much past each pointer used
    buf = torch.zeros(4 * 128 + 4, dtype=torch.float32, device="cuda")
    bits = torch.zeros(4 * 16 + 8, dtype=torch.uint8, device="cuda")
    pm = torch.zeros(5, dtype=torch.float32, device="cuda")
    cases = [(buf[1:].data_ptr(), bits[:64].data_ptr(), pm.data_ptr()),   # llr at 4 bytes
             (buf[:512].data_ptr(), bits[1:].data_ptr(), pm.data_ptr())]  # out_bits at 1 byte
    for llr_p, bits_p, pm_p in cases:
        assert rmd.rm_decode_batch(dec._h, llr_p, 4, bits_p, pm_p) == rmd.RM_E_INVAL
        assert "aligned" in rmd.rm_last_error()
    assert rmd.rm_decode_batch(dec._h, buf[4:].data_ptr(), 4, bits[8:].data_ptr(), pm[1:].data_ptr()) == rmd.RM_OK
    torch.cuda.synchronize()
    dec.close()


def test_all_zero_llr():
    llr = np.zeros((9, 512), np.float32)
    check(9, 2, 4, 4, PFHT, llr, seed=2)


def test_noiseless_frames_decode_to_sent_codeword():
    x, _ = synth.frames(9, 2, 64, 3.0, seed=9)
    llr = (8.0 * (1.0 - 2.0 * x)).astype(np.float32)
    bits, pm = gpu_decode(9, 2, 20, 4, 0, PFHT, llr)
    assert np.array_equal(synth.unpack_bits(bits, 512), x)
    assert np.all(pm == 0.0)


# --- launch shape: results must not depend on waves per block or batch size ---

@pytest.mark.parametrize("waves", [1, 2, 3])
def test_tile_invariance(waves):
    _, llr = synth.frames(9, 2, 37, 2.5, seed=21)
    ref = gpu_decode(9, 2, 20, 4, 4, PFHT, llr, waves=0)
    got = gpu_decode(9, 2, 20, 4, 4, PFHT, llr, waves=waves)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    one = gpu_decode(9, 2, 20, 4, 4, PFHT, llr[5:6], waves=waves)
    assert np.array_equal(one[0][0], ref[0][5]) and one[1][0] == ref[1][5]


def test_empty_batch_is_noop():
    dec = rmd.Decoder(9, 2, 20, 4)
    t = torch.zeros((0, 512), device="cuda")
    bits, pm = dec.decode(t)
    torch.cuda.synchronize()
    assert bits.shape == (0, 64) and pm.shape == (0,)


def test_host_pointer_rejected():
    dec = rmd.Decoder(7, 2, 1, 1, perm_mode=NONE)
    llr = np.zeros((4, 128), np.float32)
    out = np.zeros((4, 16), np.uint8)
    rc = rmd.rm_decode_batch(dec._h, llr.ctypes.data, 4, out.ctypes.data, None)
    assert rc == rmd.RM_E_PTR


# --- the benchmark's full-size launch ---

def test_full_size_rm29_p20_l4_sampled():
    n = 262144
    x, llr = synth.frames(9, 2, n, 3.0, seed=1)
    print("case full-size RM(2,9) P=20 L=4 n=262144", flush=True)
    bits, pm = gpu_decode(9, 2, 20, 4, 0, PFHT, llr)
    # every output is a codeword: its syndrome against RM(m-r-1, m), the dual code, is zero
    h = torch.from_numpy(synth.monomial_table(9, 9 - 2 - 1).astype(np.float32)).cuda()
    xb = torch.from_numpy(synth.unpack_bits(bits, 512).astype(np.float32)).cuda()
    syn = torch.remainder(xb @ h.T, 2.0)
    assert int(syn.sum().item()) == 0
    # sampled frames against the oracle, one by one
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(n, 48, replace=False))
    rb, rp = oracle_decode(9, 2, 20, 4, 0, PFHT, llr[idx])
    assert_parity((bits[idx], pm[idx]), (rb, rp), "full-size sample")


def _full_size_check(m, r, P, L, n, ebn0, seed, samples, label):
    _, llr = synth.frames(m, r, n, ebn0, seed=seed)
    print(f"case full-size {label} n={n}", flush=True)
    bits, pm = gpu_decode(m, r, P, L, 0, PFHT, llr)
    h = torch.from_numpy(synth.monomial_table(m, m - r - 1).astype(np.float32)).cuda()
    for c in range(0, n, 65536):  # syndrome of every frame against the dual code
        xb = torch.from_numpy(synth.unpack_bits(bits[c:c + 65536], 1 << m).astype(np.float32)).cuda()
        assert int(torch.remainder(xb @ h.T, 2.0).sum().item()) == 0
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, samples, replace=False))
    rb, rp = oracle_decode(m, r, P, L, 0, PFHT, llr[idx])
    assert_parity((bits[idx], pm[idx]), (rb, rp), f"full-size {label} sample")


def test_full_size_rm29_p512_l1_sampled():
    """The comparison point RM(2,9) with 512 permuted decoders at L = 1,
    131,072 frames in one launch."""
    _full_size_check(9, 2, 512, 1, 131072, 2.5, 3, 24, "RM(2,9) P=512 L=1")


def test_full_size_rm38_p8_l8_sampled():
    """RM(3,8) with 8 permuted decoders at L = 8, 131,072 frames in one launch."""
    _full_size_check(8, 3, 8, 8, 131072, 2.5, 4, 48, "RM(3,8) P=8 L=8")
