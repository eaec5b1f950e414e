"""rm_mixed_decode_static: the fused mixed-code launch with no allocation
(queue and head in the library's static device array).

Its results must equal, bit for bit (codewords and metrics), those of
rm_mixed_decode on the same segments, which the mixed-launch tests tie to
the per-code launches and the oracle.  Two calls in a row, the second with
fewer frames, fewer segments and other queue-entry sizes, so that a queue
or head left over from the first call would show; then the same calls on a
stream other than the null stream, and the size limit.
"""
import numpy as np
import pytest

import paper_2108_12550_amd as rmd
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

# (m, P, seed) of the fused kernel's four codes, all r = 2, L = 4
CODES = [(7, 8, 1), (8, 16, 2), (9, 20, 3), (10, 32, 4)]


def make_case(decs, counts, tiles, seed):
    segs, outs = [], []
    for (m, P, s), n, tf in zip(CODES, counts, tiles):
        if n is None:
            continue
        e = synth.uniform_ebn0(n, 2.0, 4.0, seed=seed + m)
        _, llr = synth.frames(m, 2, n, e, seed=seed + 10 * m)
        t = torch.from_numpy(llr).cuda()
        a = (torch.full((n, (1 << m) // 8), 0xAB, dtype=torch.uint8, device="cuda"),
             torch.full((n,), -1.0, dtype=torch.float32, device="cuda"))
        b = (torch.full((n, (1 << m) // 8), 0xCD, dtype=torch.uint8, device="cuda"),
             torch.full((n,), -2.0, dtype=torch.float32, device="cuda"))
        segs.append((decs[m], t, tf))
        outs.append((a, b))
    return segs, outs


def run_both(segs, outs, waves, stream):
    mx = rmd.MixedLauncher(max_tiles=1 << 16)
    mx.decode([(d, t, a[0], a[1], tf) for (d, t, tf), (a, _) in zip(segs, outs)], stream=stream)
    rmd.mixed_decode_static([(d, t, b[0], b[1], tf) for (d, t, tf), (_, b) in zip(segs, outs)],
                            waves_per_block=waves, stream=stream)
    torch.cuda.synchronize()
    mx.close()
    for k, (a, b) in enumerate(outs):
        assert torch.equal(a[0], b[0]), f"segment {k}: codewords differ"
        assert torch.equal(a[1], b[1]), f"segment {k}: metrics differ"


@pytest.mark.parametrize("use_stream", [False, True])
def test_static_launch_equals_launcher(use_stream):
    decs = {m: rmd.Decoder(m, 2, P, 4, seed=s) for m, P, s in CODES}
    stream = torch.cuda.Stream() if use_stream else torch.cuda.default_stream()
    # first call: all four codes, ragged counts, default and mixed entry sizes
    print(f"case static fused launch, call 1, stream={use_stream}", flush=True)
    segs, outs = make_case(decs, [3001, 2050, 1025, 515], [4, 0, 3, 7], seed=11)
    run_both(segs, outs, 2, stream)
    # second call: smaller, two codes, other entry sizes and waves per block
    print(f"case static fused launch, call 2, stream={use_stream}", flush=True)
    segs, outs = make_case(decs, [None, 301, None, 77], [0, 1, 0, 16], seed=12)
    run_both(segs, outs, 1, stream)


def test_static_launch_limits():
    dec = rmd.Decoder(7, 2, 8, 4, seed=1)
    n = rmd.RM_MIXED_STATIC_MAX_TILES + 1
    llr = torch.zeros((n, 128), dtype=torch.float32, device="cuda")
    bits = torch.empty((n, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(rmd.RMError) as ei:
        rmd.mixed_decode_static([(dec, llr, bits, None, 1)])
    assert ei.value.code == rmd.RM_E_INVAL
    with pytest.raises(rmd.RMError) as ei:
        rmd.mixed_decode_static([(dec, llr[:10], bits[:10], None, 1)], waves_per_block=5)
    assert ei.value.code == rmd.RM_E_INVAL
    # an empty segment queues nothing and succeeds
    rmd.mixed_decode_static([(dec, llr[:0], bits[:0], None, 0)])
    torch.cuda.synchronize()
