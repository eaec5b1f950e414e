"""Parity where the decoder is hardest, and its frame error rate against the
paper's curve.

* At 2.0 dB the list and the permutation-domain selections are decided by
  ties and near-ties far more often than at the benchmark's 3.0 dB.  Each
  case decodes a full launch on the GPU and compares with the oracle every
  frame the GPU decodes to a codeword other than the one sent, plus a
  random sample of the rest: bit-exact codewords, metrics within 1e-5
  relative.
* Fig. 7(d) prints the FER of p-FHT-FSCL-4-20 on RM(2,9); 2^21 frames per
  point put the printed value inside a 99.9% Wilson interval of the GPU's
  count.  Both readings of how the permutations are sampled (maps fixed per
  decoder, or drawn afresh for every frame) are run and reported.
"""
import json
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
PM_RTOL = 1e-5
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def wilson(k, n, z):
    p = k / n
    den = 1 + z * z / n
    mid = (p + z * z / (2 * n)) / den
    half = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return mid - half, mid + half


def gpu_decode(dec, llr_dev):
    bits, pm = dec.decode(llr_dev)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), pm.cpu().numpy()


@pytest.mark.parametrize("m,r,P,L,n,n_random,seed", [
    (9, 2, 20, 4, 262144, 2000, 61),   # the benchmark configuration
    (9, 2, 512, 1, 131072, 256, 62),   # RM(2,9) with 512 decoders of list size 1
    (8, 3, 8, 8, 131072, 1000, 63),    # RM(3,8) with 8 decoders of list size 8
])
def test_error_frames_match_oracle(m, r, P, L, n, n_random, seed):
    x, llr = synth.frames(m, r, n, 2.0, seed=seed)
    print(f"case error frames RM({r},{m}) P={P} L={L} n={n} 2.0 dB", flush=True)
    dec = rmd.Decoder(m, r, P, L, seed=0)
    bits, pm = gpu_decode(dec, torch.from_numpy(llr).cuda())
    dec.close()
    wrong = np.nonzero(np.any(synth.unpack_bits(bits, 1 << m) != x, axis=1))[0]
    rng = np.random.default_rng(seed)
    idx = np.union1d(wrong, rng.choice(n, n_random, replace=False))
    print(f"  {wrong.size} frames decoded wrongly; comparing {idx.size} frames with the oracle", flush=True)
    assert wrong.size > 0  # the point is to compare frames the decoder gets wrong
    rb, rp = oracle.OracleDecoder(m, r, P, L, seed=0).decode_batch(llr[idx], n_threads=THREADS)
    bad = np.nonzero(np.any(bits[idx] != rb, axis=1))[0]
    assert bad.size == 0, f"{bad.size} of {idx.size} frames differ from the oracle, first {idx[bad[:8]]}"
    rel = np.abs(pm[idx].astype(np.float64) - rp) / np.maximum(1.0, np.abs(rp))
    assert rel.max() <= PM_RTOL


def test_fresh_mode_error_frames_match_oracle():
    """The same at 2.0 dB with maps drawn afresh for every frame: the maps
    depend on the frame's index in the call, so the oracle decodes each
    sampled frame under its own index."""
    m, r, P, L, n = 9, 2, 20, 4, 65536
    x, llr = synth.frames(m, r, n, 2.0, seed=64)
    print(f"case fresh-mode error frames RM(2,9) P=20 L=4 n={n} 2.0 dB", flush=True)
    dec = rmd.Decoder(m, r, P, L, seed=3, perm_mode=rmd.RM_PERM_FRESH)
    bits, pm = gpu_decode(dec, torch.from_numpy(llr).cuda())
    dec.close()
    wrong = np.nonzero(np.any(synth.unpack_bits(bits, 1 << m) != x, axis=1))[0]
    idx = np.union1d(wrong, np.random.default_rng(64).choice(n, 200, replace=False))
    print(f"  {wrong.size} frames decoded wrongly; comparing {idx.size} frames with the oracle", flush=True)
    od = oracle.OracleDecoder(m, r, P, L, seed=3, perm_mode=oracle.PERM_FRESH)
    for f in idx:
        xb, p = od.decode(llr[f], frame=int(f))
        assert np.array_equal(synth.pack_bits(xb), bits[f]), f"frame {f}"
        assert abs(float(pm[f]) - p) <= PM_RTOL * max(1.0, abs(p)), f"frame {f}"


FER_FRAMES = 1 << 21
FER_BATCH = 1 << 18


@pytest.mark.parametrize("ebn0", ["2.0", "2.5"])
def test_fer_matches_fig7d(ebn0):
    """p-FHT-FSCL-4-20 on RM(2,9) (Fig. 7(d): 2.99e-4 at 2.0 dB, 2.85e-5 at
    2.5 dB): the printed value lies in the 99.9% Wilson interval of the GPU
    decoder's error count over 2^21 frames, with the maps fixed per decoder
    (the benchmark's reading) and with maps drawn afresh for every frame."""
    m, r, P, L = 9, 2, 20, 4
    pub = GOLDEN["fer_rm29_m20"]["p-FHT-FSCL-4-20"][ebn0]
    decs = {"fixed": rmd.Decoder(m, r, P, L, seed=0),
            "fresh": rmd.Decoder(m, r, P, L, seed=0, perm_mode=rmd.RM_PERM_FRESH)}
    errors = {k: 0 for k in decs}
    print(f"case FER RM(2,9) P=20 L=4 {ebn0} dB, {FER_FRAMES} frames", flush=True)
    for b in range(FER_FRAMES // FER_BATCH):
        x, llr = synth.frames(m, r, FER_BATCH, float(ebn0), seed=7000 + 10 * b + int(float(ebn0) * 2))
        t = torch.from_numpy(llr).cuda()
        for k, dec in decs.items():
            bits, _ = gpu_decode(dec, t)
            errors[k] += int(np.any(synth.unpack_bits(bits, 1 << m) != x, axis=1).sum())
    report = {}
    for k, e in errors.items():
        lo, hi = wilson(e, FER_FRAMES, 3.29)
        report[k] = (e / FER_FRAMES, lo, hi)
        print(f"  {k}: FER {e / FER_FRAMES:.3e} ({e} errors), 99.9% interval [{lo:.3e}, {hi:.3e}]; "
              f"Fig. 7(d) {pub:.3e}", flush=True)
    for dec in decs.values():
        dec.close()
    for k, (_, lo, hi) in report.items():
        assert lo <= pub <= hi, (k, report[k], pub)
