"""The fused mixed-code launch (rm_mixed_*): one persistent kernel over the
frames of RM(2,7), RM(2,8), RM(2,9) and RM(2,10), list size 4.

Its results must equal, bit for bit (codewords and metrics), those of the
per-code launches, which the parity tests tie to the oracle; sampled frames
are also checked against the oracle directly.  Graph replays are checked one
by one against the eager result, with other GPU work in between.
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

THREADS = min(16, os.cpu_count() or 1)
# (m, P, seed) of the four codes, all r = 2, L = 4
CODES = [(7, 8, 1), (8, 16, 2), (9, 20, 3), (10, 32, 4)]


def make_inputs(counts, ebn0=(2.0, 4.0), seed=100):
    segs = []
    for (m, P, s), n in zip(CODES, counts):
        e = synth.uniform_ebn0(n, *ebn0, seed=seed + m) if n else np.zeros(0)
        _, llr = synth.frames(m, 2, n, e, seed=seed + 10 * m) if n else (None, np.zeros((0, 1 << m), np.float32))
        segs.append((m, P, s, llr))
    return segs


def decoders():
    return {m: rmd.Decoder(m, 2, P, 4, seed=s) for m, P, s in CODES}


def dev_buffers(segs):
    out = []
    for m, P, s, llr in segs:
        n = llr.shape[0]
        t = torch.from_numpy(np.ascontiguousarray(llr)).cuda() if n else torch.empty((0, 1 << m), device="cuda")
        bits = torch.full((n, (1 << m) // 8), 0xAB, dtype=torch.uint8, device="cuda")
        pm = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
        out.append((t, bits, pm))
    return out


def per_code(decs, segs):
    res = []
    for m, P, s, llr in segs:
        if llr.shape[0] == 0:
            res.append((np.zeros((0, (1 << m) // 8), np.uint8), np.zeros(0, np.float32)))
            continue
        b, p = decs[m].decode(torch.from_numpy(np.ascontiguousarray(llr)).cuda())
        torch.cuda.synchronize()
        res.append((b.cpu().numpy(), p.cpu().numpy()))
    return res


def fetch(bufs):
    torch.cuda.synchronize()
    return [(b.cpu().numpy(), p.cpu().numpy()) for _, b, p in bufs]


def assert_same(got, ref, label):
    for k, ((gb, gp), (rb, rp)) in enumerate(zip(got, ref)):
        assert np.array_equal(gb, rb), f"{label}: code {CODES[k]} bits differ"
        assert np.array_equal(gp, rp), f"{label}: code {CODES[k]} metrics differ"


def seg_list(decs, segs, bufs, tiles):
    return [(decs[m], t, b, p, tf) for (m, P, s, _), (t, b, p), tf in zip(segs, bufs, tiles)]


@pytest.mark.parametrize("counts,tiles,grid", [
    ((300, 517, 129, 64), (4, 4, 4, 4), (0, 0)),
    ((300, 517, 129, 64), (1, 7, 64, 3), (0, 0)),
    ((37, 5, 211, 90), (2, 1, 4, 8), (3, 1)),   # few waves: many queue entries each
    ((64, 64, 64, 64), (0, 0, 0, 0), (1000, 4)),
])
def test_mixed_equals_per_code(counts, tiles, grid):
    label = f"counts={counts} tiles={tiles} grid={grid}"
    print("case", label, flush=True)
    decs = decoders()
    segs = make_inputs(counts)
    ref = per_code(decs, segs)
    mx = rmd.MixedLauncher(max_tiles=4096, blocks=grid[0], waves_per_block=grid[1])
    bufs = dev_buffers(segs)
    mx.decode(seg_list(decs, segs, bufs, tiles))
    assert_same(fetch(bufs), ref, label)
    mx.close()


def test_mixed_sampled_frames_match_oracle():
    decs = decoders()
    segs = make_inputs((96, 96, 96, 96), seed=7)
    mx = rmd.MixedLauncher(max_tiles=1024)
    bufs = dev_buffers(segs)
    mx.decode(seg_list(decs, segs, bufs, (4, 4, 4, 4)))
    got = fetch(bufs)
    for (m, P, s, llr), (gb, gp) in zip(segs, got):
        idx = np.arange(0, 96, 13)
        rb, rp = oracle.OracleDecoder(m, 2, P, 4, seed=s).decode_batch(llr[idx], n_threads=THREADS)
        assert np.array_equal(gb[idx], rb), f"RM(2,{m}) bits differ from the oracle"
        assert np.max(np.abs(gp[idx] - rp) / np.maximum(1.0, np.abs(rp))) <= 1e-5


def test_back_to_back_calls_without_sync():
    """Two launches queued one after the other reuse the device queue; the
    second's upload is stream-ordered after the first kernel."""
    decs = decoders()
    s1 = make_inputs((200, 150, 100, 50), seed=21)
    s2 = make_inputs((7, 300, 33, 120), seed=22)
    r1, r2 = per_code(decs, s1), per_code(decs, s2)
    mx = rmd.MixedLauncher(max_tiles=4096)
    b1, b2 = dev_buffers(s1), dev_buffers(s2)
    stream = torch.cuda.Stream()
    mx.decode(seg_list(decs, s1, b1, (1, 1, 1, 1)), stream=stream)
    mx.decode(seg_list(decs, s2, b2, (2, 2, 2, 2)), stream=stream)
    assert_same(fetch(b1), r1, "first")
    assert_same(fetch(b2), r2, "second")


def test_empty_segments():
    decs = decoders()
    segs = make_inputs((0, 77, 0, 13), seed=5)
    ref = per_code(decs, segs)
    mx = rmd.MixedLauncher(max_tiles=64)
    bufs = dev_buffers(segs)
    mx.decode(seg_list(decs, segs, bufs, (4, 4, 4, 4)))
    assert_same(fetch(bufs), ref, "empty segments")
    empty = make_inputs((0, 0, 0, 0))
    mx.decode(seg_list(decs, empty, dev_buffers(empty), (4, 4, 4, 4)))
    torch.cuda.synchronize()


def test_graph_replays_match_eager():
    decs = decoders()
    segs = make_inputs((120, 90, 60, 30), seed=9)
    mx = rmd.MixedLauncher(max_tiles=1024)
    bufs = dev_buffers(segs)
    stream = torch.cuda.Stream()
    sl = seg_list(decs, segs, bufs, (4, 4, 4, 4))
    mx.decode(sl, stream=stream)
    eager = fetch(bufs)
    mx.capture(sl, stream)
    other = make_inputs((50, 50, 50, 50), seed=10)
    other_ref = per_code(decs, other)
    for rep in range(4):
        for _, b, p in bufs:
            b.fill_(0x5A)
            p.fill_(123.0)
        torch.cuda.synchronize()
        mx.replay()
        assert_same(fetch(bufs), eager, f"replay {rep}")
        # eager work between replays: a different eager fused launch on the
        # same launcher (its own queue) and per-code decodes
        ob = dev_buffers(other)
        mx.decode(seg_list(decs, other, ob, (3, 3, 3, 3)), stream=stream)
        assert_same(fetch(ob), other_ref, f"eager between replays {rep}")
    mx.close()


def test_invalid_segments_rejected():
    decs = decoders()
    segs = make_inputs((64, 64, 64, 64), seed=3)
    bufs = dev_buffers(segs)
    mx = rmd.MixedLauncher(max_tiles=16)
    with pytest.raises(rmd.RMError) as e:
        mx.decode(seg_list(decs, segs, bufs, (1, 1, 1, 1)))  # 256 entries > 16
    assert e.value.code == rmd.RM_E_INVAL
    other = rmd.Decoder(9, 2, 4, 1, seed=0)
    with pytest.raises(rmd.RMError) as e:
        mx.decode([(other, bufs[2][0], bufs[2][1], bufs[2][2], 64)])
    assert e.value.code == rmd.RM_E_UNSUPPORTED
    host = torch.from_numpy(np.ascontiguousarray(segs[0][3]))
    seg = rmd.rm_segment(decs[7]._h, host.data_ptr(), 64, bufs[0][1].data_ptr(), None, 64)
    mxh = rmd.rm_mixed_create(16)
    assert rmd.rm_mixed_decode(mxh, [seg]) == rmd.RM_E_PTR
    assert rmd.rm_mixed_decode(mxh, [seg] * 9) == rmd.RM_E_INVAL
    rmd.rm_mixed_destroy(mxh)
    with pytest.raises(rmd.RMError):
        mx.set_grid(0, 5)
    mx.close()


def test_autotuned_launch_equals_per_code():
    decs = decoders()
    segs = make_inputs((256, 256, 128, 64), seed=31)
    ref = per_code(decs, segs)
    mx = rmd.MixedLauncher(max_tiles=4096)
    bufs = dev_buffers(segs)
    stream = torch.cuda.Stream()
    tune = mx.autotune(seg_list(decs, segs, bufs, (0, 0, 0, 0)), stream=stream, reps=1)
    print("tuning", tune, flush=True)
    assert tune["trials"] >= 8 and tune["waves_per_block"] in (1, 2, 4)
    assert all(t in (1, 2, 4, 8, 16) for t in tune["tile_frames"])
    assert_same(fetch(bufs), ref, "after autotune")
    bufs = dev_buffers(segs)
    mx.decode(seg_list(decs, segs, bufs, tune["tile_frames"]), stream=stream)
    assert_same(fetch(bufs), ref, "autotuned launch")


def test_full_size_mixed_graph_sampled():
    """The benchmark's fused launch at full size: 262,144 frames of each code
    (1,048,576 in one launch, Eb/N0 ~ U[2,4] per frame), replayed from its
    graph; every frame is a codeword and sampled frames match the oracle."""
    n = 262144
    decs = decoders()
    segs = make_inputs((n, n, n, n), seed=1234)
    bufs = dev_buffers(segs)
    mx = rmd.MixedLauncher(max_tiles=4 * n + 16)
    stream = torch.cuda.Stream()
    mx.capture(seg_list(decs, segs, bufs, (1, 8, 4, 1)), stream)
    mx.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for (m, P, s, llr), (_, b, p) in zip(segs, bufs):
        print(f"case full-size mixed RM(2,{m})", flush=True)
        h = torch.from_numpy(synth.monomial_table(m, m - 3).astype(np.float32)).cuda()
        for c in range(0, n, 65536):
            xb = torch.from_numpy(synth.unpack_bits(b[c:c + 65536].cpu().numpy(), 1 << m).astype(np.float32)).cuda()
            assert int(torch.remainder(xb @ h.T, 2.0).sum().item()) == 0
        idx = np.sort(rng.choice(n, 12, replace=False))
        rb, rp = oracle.OracleDecoder(m, 2, P, 4, seed=s).decode_batch(np.ascontiguousarray(llr[idx]),
                                                                     n_threads=THREADS)
        assert np.array_equal(b.cpu().numpy()[idx], rb), f"RM(2,{m})"
        assert np.max(np.abs(p.cpu().numpy()[idx] - rp) / np.maximum(1.0, np.abs(rp))) <= 1e-5
    mx.close()
