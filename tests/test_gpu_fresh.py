"""Parity of the fresh-permutation mode (maps drawn afresh for every frame)
with the oracle, through the C ABI.

In this mode frame f of a call decodes with its own draw of Alg. 2's initial
maps and of the candidate maps of every permutation-domain node, keyed by
(seed, f, decoder).  The device draws them chunk by chunk; the oracle draws
them on the host from its own implementation of the same generator.  Codewords
must agree bit for bit and metrics within 1e-5 relative, also across chunk
boundaries and at the benchmark's full size (sampled frames).
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

FRESH = rmd.RM_PERM_FRESH
THREADS = min(16, os.cpu_count() or 1)
PM_RTOL = 1e-5


def gpu_decode(m, r, P, L, seed, llr):
    dec = rmd.Decoder(m, r, P, L, seed=seed, perm_mode=FRESH)
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


def check(m, r, P, L, llr, seed):
    label = f"fresh RM({r},{m}) P={P} L={L} seed={seed} n={llr.shape[0]}"
    print("case", label, flush=True)
    od = oracle.OracleDecoder(m, r, P, L, seed=seed, perm_mode=oracle.PERM_FRESH)
    assert_parity(gpu_decode(m, r, P, L, seed, llr), od.decode_batch(llr, n_threads=THREADS), label)


@pytest.mark.parametrize("m,r,P,L,n", [(9, 2, 20, 4, 150), (9, 2, 8, 1, 200), (8, 3, 8, 8, 90), (7, 2, 4, 2, 130),
                                       (10, 2, 4, 4, 40), (9, 3, 3, 4, 60), (9, 4, 2, 8, 40), (8, 4, 16, 4, 50),
                                       (5, 2, 3, 4, 70), (4, 3, 2, 4, 70), (3, 1, 2, 4, 65)])
def test_fresh_parity(m, r, P, L, n):
    _, llr = synth.frames(m, r, n, 2.5, seed=600 + m * 10 + r)
    check(m, r, P, L, llr, seed=L + 11)


def test_fresh_parity_integer_ties():
    rng = np.random.default_rng(5)
    llr = rng.integers(-3, 4, size=(60, 512)).astype(np.float32)
    check(9, 2, 4, 4, llr, seed=2)


def test_fresh_several_chunks():
    """RM(2,9) with 512 decoders at L = 1: the table buffer (2 GiB, 6 maps of
    48 bytes per decoder) holds 14563 frames, so 32000 frames take three
    chunks, the last one ragged."""
    _, llr = synth.frames(9, 2, 32000, 2.5, seed=31)
    dec = rmd.Decoder(9, 2, 512, 1, seed=3, perm_mode=FRESH)
    assert dec.info()["table_bytes"] == 14563 * 512 * 6 * 48
    dec.close()
    print("case fresh RM(2,9) P=512 L=1 n=32000 (sampled)", flush=True)
    bits, pm = gpu_decode(9, 2, 512, 1, 3, llr)
    od = oracle.OracleDecoder(9, 2, 512, 1, seed=3, perm_mode=oracle.PERM_FRESH)
    idx = [0, 1, 14562, 14563, 14564, 29125, 29126, 29127, 31999] + list(range(100, 32000, 1999))
    for f in idx:
        x, p = od.decode(llr[f], frame=f)
        assert np.array_equal(synth.unpack_bits(bits[f:f + 1], 512)[0], x), f"frame {f}"
        assert abs(pm[f] - p) <= PM_RTOL * max(1.0, abs(p)), f"frame {f}"


def test_fresh_frame_index_is_position_in_call():
    """A call numbers its frames from 0: the tail of a batch decoded by itself
    uses the maps of indices 0, 1, ..., not those it had in the whole batch."""
    _, llr = synth.frames(9, 2, 40, 0.5, seed=8)
    whole = gpu_decode(9, 2, 20, 4, 9, llr)
    tail = gpu_decode(9, 2, 20, 4, 9, llr[17:])
    od = oracle.OracleDecoder(9, 2, 20, 4, seed=9, perm_mode=oracle.PERM_FRESH)
    assert_parity(tail, od.decode_batch(llr[17:], n_threads=THREADS), "tail call")
    assert not np.array_equal(whole[1][17:], tail[1])  # at 0.5 dB the draw changes some metrics


def test_fresh_rejected_by_fused_and_server_paths():
    dec = rmd.Decoder(9, 2, 20, 4, perm_mode=FRESH)
    llr = torch.zeros((4, 512), device="cuda")
    bits = torch.zeros((4, 64), dtype=torch.uint8, device="cuda")
    mx = rmd.MixedLauncher()
    with pytest.raises(rmd.RMError) as e:
        mx.decode([(dec, llr, bits, None, 0)])
    assert e.value.code == rmd.RM_E_UNSUPPORTED
    mx.close()
    dec.close()


def test_fresh_full_size_sampled():
    """The benchmark's code and decoder set, 131,072 frames in one call
    (two chunks): every output a codeword, sampled frames against the oracle."""
    n = 131072
    _, llr = synth.frames(9, 2, n, 3.0, seed=41)
    print("case fresh full-size RM(2,9) P=20 L=4 n=131072", flush=True)
    bits, pm = gpu_decode(9, 2, 20, 4, 0, llr)
    h = torch.from_numpy(synth.monomial_table(9, 6).astype(np.float32)).cuda()
    for c in range(0, n, 65536):
        xb = torch.from_numpy(synth.unpack_bits(bits[c:c + 65536], 512).astype(np.float32)).cuda()
        assert int(torch.remainder(xb @ h.T, 2.0).sum().item()) == 0
    od = oracle.OracleDecoder(9, 2, 20, 4, seed=0, perm_mode=oracle.PERM_FRESH)
    rng = np.random.default_rng(41)
    for f in np.sort(rng.choice(n, 40, replace=False)).tolist() + [65535, 65536, n - 1]:
        x, p = od.decode(llr[f], frame=f)
        assert np.array_equal(synth.unpack_bits(bits[f:f + 1], 512)[0], x), f"frame {f}"
        assert abs(pm[f] - p) <= PM_RTOL * max(1.0, abs(p)), f"frame {f}"


def test_fresh_two_streams_in_flight():
    """Two calls of one fresh-mode decoder queued on two streams with no host
    synchronisation between them: the second call's map draw must wait for
    the first call's decode, which still reads the shared table buffer.
    Each result equals the same call made alone."""
    m, r, P, L = 9, 2, 20, 4
    _, a = synth.frames(m, r, 150000, 2.5, seed=91)  # three table chunks
    _, b = synth.frames(m, r, 20000, 2.5, seed=92)
    print("case fresh two streams RM(2,9) P=20 L=4 n=150000+20000", flush=True)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dec = rmd.Decoder(m, r, P, L, seed=4, perm_mode=FRESH)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    ba, pa = dec.decode(ta, stream=s1)
    bb, pb = dec.decode(tb, stream=s2)
    torch.cuda.synchronize()
    got_a, got_b = (ba.cpu().numpy(), pa.cpu().numpy()), (bb.cpu().numpy(), pb.cpu().numpy())
    ra = dec.decode(ta)
    torch.cuda.synchronize()
    rb_ = dec.decode(tb)
    torch.cuda.synchronize()
    dec.close()
    assert np.array_equal(got_a[0], ra[0].cpu().numpy()) and np.array_equal(got_a[1], ra[1].cpu().numpy())
    assert np.array_equal(got_b[0], rb_[0].cpu().numpy()) and np.array_equal(got_b[1], rb_[1].cpu().numpy())
    # and a sample of each against the oracle
    od = oracle.OracleDecoder(m, r, P, L, seed=4, perm_mode=oracle.PERM_FRESH)
    for f in (0, 65535, 65536, 131072, 149999):
        x, p = od.decode(a[f], frame=f)
        assert np.array_equal(synth.pack_bits(x), got_a[0][f])
    for f in (0, 19999):
        x, p = od.decode(b[f], frame=f)
        assert np.array_equal(synth.pack_bits(x), got_b[0][f])
