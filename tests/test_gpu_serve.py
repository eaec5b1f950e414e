"""The request server (rm_server_*): continuous batching of single-frame
requests of RM(2,7), RM(2,8), RM(2,9), RM(2,10) and RM(3,8) with P in
{8, 20, 32} and L in {1, 4, 8}.

Every request's result must be the same, bit for bit (codeword and metric),
as decoding that frame alone with rm_decode_batch and the request's decoder;
a sample is also checked against the oracle.  Admission refusals are forced
with a tiny batch budget.
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
CODES = [(7, 2), (8, 2), (9, 2), (10, 2), (8, 3)]
WEIGHTS = [0.3, 0.25, 0.2, 0.15, 0.1]
PS = [8, 20, 32]
LS = [1, 4, 8]


class Workload:
    """Seeded requests: per request a code, P, L (decoder) and one frame."""

    def __init__(self, n, seed):
        rng = np.random.default_rng(seed)
        self.code = rng.choice(len(CODES), size=n, p=WEIGHTS)
        self.P = rng.choice(PS, size=n)
        self.L = rng.choice(LS, size=n)
        self.decs = {}
        self.frames = {}  # code index -> (llr array, device tensor)
        self.row = np.zeros(n, dtype=np.int64)
        for k, (m, r) in enumerate(CODES):
            idx = np.nonzero(self.code == k)[0]
            e = synth.uniform_ebn0(max(1, idx.size), 2.0, 4.0, seed=seed + k)
            _, llr = synth.frames(m, r, max(1, idx.size), e, seed=seed + 100 + k)
            self.frames[k] = (llr, torch.from_numpy(llr).cuda())
            self.row[idx] = np.arange(idx.size)
        for i in range(n):
            key = (int(self.code[i]), int(self.P[i]), int(self.L[i]))
            if key not in self.decs:
                m, r = CODES[key[0]]
                self.decs[key] = rmd.Decoder(m, r, key[1], key[2], seed=7 * key[1] + key[2])
        self.n = n

    def key(self, i):
        return (int(self.code[i]), int(self.P[i]), int(self.L[i]))

    def llr_host(self, i):
        return self.frames[int(self.code[i])][0][self.row[i]]

    def llr_dev_ptr(self, i):
        k = int(self.code[i])
        m, _ = CODES[k]
        t = self.frames[k][1]
        return t.data_ptr() + 4 * (1 << m) * int(self.row[i])

    def reference(self):
        """Each request's frame decoded with its decoder by rm_decode_batch."""
        bits = np.zeros((self.n, 128), np.uint8)
        pm = np.zeros(self.n, np.float32)
        for key, dec in self.decs.items():
            idx = np.nonzero((self.code == key[0]) & (self.P == key[1]) & (self.L == key[2]))[0]
            llr = np.ascontiguousarray(self.frames[key[0]][0][self.row[idx]])
            b, p = dec.decode(torch.from_numpy(llr).cuda())
            torch.cuda.synchronize()
            bits[idx, :dec.N // 8] = b.cpu().numpy()
            pm[idx] = p.cpu().numpy()
        return bits, pm


def run_all(srv, wl, on_device, keep_host):
    """Submit every request (retrying refused ones after a poll), poll to the end."""
    got_bits = np.zeros((wl.n, 128), np.uint8)
    got_pm = np.zeros(wl.n, np.float32)
    seen = np.zeros(wl.n, bool)
    refused = 0

    def drain():
        for ticket, tag, bits, metric, ta, tl, td in srv.poll():
            assert not seen[tag]
            seen[tag] = True
            got_bits[tag, :len(bits)] = np.frombuffer(bits, np.uint8)
            got_pm[tag] = metric
            assert ta <= tl <= td

    i = 0
    while i < wl.n:
        dev = bool(on_device[i])
        if dev:
            ptr = wl.llr_dev_ptr(i)
        else:
            h = np.ascontiguousarray(wl.llr_host(i))
            keep_host.append(h)
            ptr = h.ctypes.data
        t = srv.submit(wl.decs[wl.key(i)], ptr, dev, tag=i)
        if t is None:
            refused += 1
            drain()
            continue
        i += 1
        if i % 64 == 0:
            drain()
    while srv.pending() > 0:
        drain()
    drain()
    assert seen.all()
    return got_bits, got_pm, refused


def assert_same(got, ref, label):
    gb, gp = got
    rb, rp = ref
    bad = np.nonzero(np.any(gb != rb, axis=1))[0]
    assert bad.size == 0, f"{label}: {bad.size} requests differ in bits, first {bad[:8]}"
    assert np.array_equal(gp, rp), f"{label}: metrics differ"


@pytest.mark.parametrize("depth,tile,split", [(2, 0, 0), (1, 1, 1), (4, 8, 2), (2, 3, 4), (3, 2, 1)])
def test_mix_equals_alone(depth, tile, split):
    print(f"case depth={depth} tile={tile} split={split}", flush=True)
    wl = Workload(1500, seed=depth * 10 + tile)
    ref = wl.reference()
    srv = rmd.Server(batch_bytes=1 << 20, max_batch=512, depth=depth, tile_frames=tile, split=split)
    for k in wl.frames:
        srv.register_pool(wl.frames[k][1])
    rng = np.random.default_rng(5)
    keep = []
    got_b, got_p, _ = run_all(srv, wl, rng.random(wl.n) < 0.5, keep)
    assert_same((got_b, got_p), ref, f"depth={depth} tile={tile}")
    srv.close()


def test_single_frame_alone_launches_match():
    """A few requests against literally alone decodes (one-frame launches)."""
    wl = Workload(40, seed=77)
    srv = rmd.Server(batch_bytes=1 << 20, max_batch=64, depth=2)
    keep = []
    got_b, got_p, _ = run_all(srv, wl, np.zeros(wl.n, bool), keep)
    for i in range(wl.n):
        dec = wl.decs[wl.key(i)]
        b, p = dec.decode(torch.from_numpy(np.ascontiguousarray(wl.llr_host(i)[None, :])).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(b.cpu().numpy()[0], got_b[i, :dec.N // 8]), f"request {i}"
        assert p.item() == got_p[i]


def test_sampled_requests_match_oracle():
    wl = Workload(300, seed=13)
    srv = rmd.Server(batch_bytes=1 << 20, max_batch=256, depth=2)
    keep = []
    got_b, got_p, _ = run_all(srv, wl, np.zeros(wl.n, bool), keep)
    for key, dec in wl.decs.items():
        idx = np.nonzero((wl.code == key[0]) & (wl.P == key[1]) & (wl.L == key[2]))[0][:2]
        if idx.size == 0:
            continue
        m, r = CODES[key[0]]
        od = oracle.OracleDecoder(m, r, key[1], key[2], seed=7 * key[1] + key[2])
        rb, rp = od.decode_batch(np.ascontiguousarray(wl.frames[key[0]][0][wl.row[idx]]), n_threads=THREADS)
        assert np.array_equal(got_b[idx, :dec.N // 8], rb), f"{key}"
        assert np.max(np.abs(got_p[idx] - rp) / np.maximum(1.0, np.abs(rp))) <= 1e-5


def test_tiny_budget_refuses_then_completes():
    wl = Workload(400, seed=3)
    ref = wl.reference()
    # room for one RM(2,10) frame's LLRs per batch, at most 3 requests, one batch on the device
    srv = rmd.Server(batch_bytes=4096, max_batch=3, depth=1)
    keep = []
    got_b, got_p, refused = run_all(srv, wl, np.zeros(wl.n, bool), keep)
    print("refused", refused, flush=True)
    assert refused > 0
    assert_same((got_b, got_p), ref, "tiny budget")


def test_trace_replay_results_and_latency():
    wl = Workload(4000, seed=21)
    ref = wl.reference()
    srv = rmd.Server(batch_bytes=8 << 20, max_batch=2048, depth=2)
    for k in wl.frames:
        srv.register_pool(wl.frames[k][1])
    rng = np.random.default_rng(1)
    arrival = np.cumsum(rng.exponential(1.0 / 0.5, size=wl.n))  # 0.5 requests per us
    reqs = [(wl.decs[wl.key(i)], wl.llr_dev_ptr(i), True) for i in range(wl.n)]
    ob = np.zeros((wl.n, 128), np.uint8)
    om = np.zeros(wl.n, np.float32)
    lat, st = srv.run_trace(reqs, arrival, ob, om)
    print("trace", st, "p50", np.percentile(lat, 50), "p99", np.percentile(lat, 99), flush=True)
    assert np.all(lat > 0) and np.all(np.isfinite(lat))
    assert st["batches"] >= 1
    assert_same((ob, om), ref, "trace replay")


def test_unsupported_and_foreign_pointers():
    srv = rmd.Server(batch_bytes=1 << 16, max_batch=16, depth=1)
    d2 = rmd.Decoder(9, 2, 4, 2, seed=0)
    x = torch.zeros(512, device="cuda")
    with pytest.raises(rmd.RMError) as e:
        srv.submit(d2, x.data_ptr(), True)
    assert e.value.code == rmd.RM_E_UNSUPPORTED
    d = rmd.Decoder(9, 2, 8, 4, seed=0)
    with pytest.raises(rmd.RMError) as e:
        srv.submit(d, x.data_ptr(), True)  # not in a registered pool
    assert e.value.code == rmd.RM_E_PTR
    srv.register_pool(x)
    assert srv.submit(d, x.data_ptr(), True) is not None
    while srv.pending():
        srv.poll()
    srv.close()


def test_requests_complete_individually():
    """A request is returned as soon as its own outputs are written, not when
    its batch ends: in one batch with a heavy request (RM(2,10), P = 32,
    L = 8) and light ones (RM(2,7), P = 8, L = 1), the light requests are
    returned before the heavy one, and every result is still that of
    rm_decode_batch."""
    heavy = rmd.Decoder(10, 2, 32, 8, seed=3)
    light = rmd.Decoder(7, 2, 8, 1, seed=4)
    _, yh = synth.frames(10, 2, 1, 2.5, seed=91)
    _, yl = synth.frames(7, 2, 200, 2.5, seed=92)
    th, tl = torch.from_numpy(yh).cuda(), torch.from_numpy(yl).cuda()
    ref_h = [a.cpu().numpy() for a in heavy.decode(th)]
    ref_l = [a.cpu().numpy() for a in light.decode(tl)]
    torch.cuda.synchronize()
    srv = rmd.Server(batch_bytes=8 << 20, max_batch=1024, depth=1)
    srv.register_pool(th)
    srv.register_pool(tl)
    # the first request is launched alone; without a poll it stays in flight,
    # so the following ones gather in the next batch
    assert srv.submit(light, tl.data_ptr(), True, tag=1000) is not None
    assert srv.submit(heavy, th.data_ptr(), True, tag=999) is not None
    for i in range(200):
        assert srv.submit(light, tl.data_ptr() + 512 * i, True, tag=i) is not None
    done = {}
    while len(done) < 202:
        for ticket, tag, bits, metric, ta, tlch, td in srv.poll():
            done[tag] = (bits, metric, td)
    t_heavy = done[999][2]
    t_light = np.array([done[i][2] for i in range(200)])
    print(f"  heavy request done at {t_heavy - t_light.min():.0f} us after the first light one; "
          f"light requests before it: {(t_light < t_heavy).sum()} of 200", flush=True)
    assert (t_light < t_heavy).sum() >= 150
    assert np.frombuffer(done[999][0], np.uint8).tobytes() == ref_h[0][0].tobytes() and done[999][1] == ref_h[1][0]
    for i in range(200):
        assert np.frombuffer(done[i][0], np.uint8).tobytes() == ref_l[0][i].tobytes() and done[i][1] == ref_l[1][i]
    srv.close()
