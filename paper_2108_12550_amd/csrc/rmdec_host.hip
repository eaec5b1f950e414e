// rmdec_host.hip -- the C ABI declared in include/rmdec.h: argument checks,
// the permutation draw, the device tables and the kernel launch.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "rmdec.h"
#include "rmdec_internal.hpp"
#include "rmdec_kernels.hpp"

using namespace rmdec;

namespace rmdec {
thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int check_device_ptr(const void *p, const char *name)
{
    hipPointerAttribute_t a;
    memset(&a, 0, sizeof a);
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RM_E_PTR, std::string(name) + " is not device memory");
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(RM_E_PTR, std::string(name) + " is not device memory");
    return RM_OK;
}

// Alignment of the caller's arrays: frames are read in 16-byte words and
// codewords written in 8-byte words (bytes below N = 64).
int check_alignment(int N, const float *llr, const uint8_t *out_bits, const float *out_metric)
{
    const uintptr_t bits_align = N / 8 < 8 ? (uintptr_t)(N / 8) : 8u;
    if ((uintptr_t)llr % 16 != 0)
        return fail(RM_E_INVAL, "llr must be 16-byte aligned");
    if ((uintptr_t)out_bits % bits_align != 0)
        return fail(RM_E_INVAL, "out_bits must be aligned to min(8, N/8) bytes");
    if ((uintptr_t)out_metric % 4 != 0)
        return fail(RM_E_INVAL, "out_metric must be 4-byte aligned");
    return RM_OK;
}

KernelArgs batch_args(const rm_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_metric)
{
    KernelArgs a;
    a.llr = llr;
    a.out_bits = out_bits;
    a.out_pm = out_metric;
    a.maps = d->d_maps;
    a.n_frames = n_frames;
    a.frame_stride = 0;
    a.P = d->cfg.P;
    a.maps_per_dec = d->maps_per_dec;
    a.pfht = d->cfg.perm_mode != RM_PERM_NONE;
    a.waves = d->cfg.waves_per_block;
    return a;
}

hipError_t launch_decoder(const rm_decoder *d, const KernelArgs &a, int64_t n_frames)
{
    const int64_t per_block = (int64_t)a.waves * (d->packed ? d->kern->D : 1);
    const int64_t b = (n_frames + per_block - 1) / per_block;
    const int blocks = (int)(b > (1 << 30) ? (1 << 30) : b);
    return (d->packed ? d->kern->launch_packed : d->kern->launch)(a, blocks, d->stream);
}

// the tables of the instantiation units rmdec_inst_*.hip
KernelTable kernels_codes_a();
KernelTable kernels_codes_b();
KernelTable kernels_codes_c();
KernelTable kernels_codes_d();
KernelTable kernels_codes_e();
KernelTable kernels_codes_f();
KernelTable kernels_codes_g(); // lists of 16, 32 and 64 paths
KernelTable kernels_codes_h(); // lists of 64 paths, N = 512
KernelTable kernels_codes_i(); // the rest of m <= 10, L <= 8, by length
KernelTable kernels_codes_j();
KernelTable kernels_codes_k();
KernelTable kernels_codes_l();
KernelTable kernels_codes_m(); // lists of 16 and 32 paths for the other internal codes
KernelTable kernels_codes_n();
KernelTable kernels_codes_o();
KernelTable kernels_codes_p();
KernelTable kernels_codes_q();
KernelTable kernels_codes_r(); // leaf roots with lists of 8 to 32 paths
KernelTable kernels_codes_s();
KernelTable kernels_codes_t();

} // namespace rmdec

namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): Weyl increment, then mix.
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// Affine map p(i) = A z(i) + b over F2^m; row j of A gives output bit j.
struct Affine {
    int m = 0;
    uint32_t row[16] = {};
    uint32_t b = 0;
    uint32_t apply(uint32_t i) const
    {
        uint32_t z = 0;
        for (int j = 0; j < m; j++)
            z |= (uint32_t)(__builtin_popcount(row[j] & i) & 1) << j;
        return z ^ b;
    }
};

bool invertible(const uint32_t *rows, int m)
{
    uint32_t t[16];
    for (int k = 0; k < m; k++)
        t[k] = rows[k];
    int rank = 0;
    for (int col = 0; col < m && rank < m; col++) {
        int piv = -1;
        for (int k = rank; k < m; k++)
            if ((t[k] >> col) & 1u) {
                piv = k;
                break;
            }
        if (piv < 0)
            continue;
        uint32_t tmp = t[piv];
        t[piv] = t[rank];
        t[rank] = tmp;
        for (int k = 0; k < m; k++)
            if (k != rank && ((t[k] >> col) & 1u))
                t[k] ^= t[rank];
        rank++;
    }
    return rank == m;
}

Affine draw_affine(int m, SplitMix64 &rng)
{
    Affine a;
    a.m = m;
    const uint32_t mask = (1u << m) - 1u;
    do {
        for (int k = 0; k < m; k++)
            a.row[k] = (uint32_t)(rng.next() & mask);
    } while (!invertible(a.row, m));
    a.b = (uint32_t)(rng.next() & mask);
    return a;
}

// The fresh mode's draw: row k of A redrawn until it lies outside the span of
// rows 0..k-1 (tested by reduction against an XOR basis kept by leading
// bit), then b.
Affine draw_affine_rowwise(int m, SplitMix64 &rng)
{
    Affine a;
    a.m = m;
    const uint32_t mask = (1u << m) - 1u;
    uint32_t basis[16] = {}; // basis[h]: a vector of the span whose leading bit is h
    for (int k = 0; k < m; k++) {
        for (;;) {
            const uint32_t r = (uint32_t)(rng.next() & mask);
            uint32_t x = r;
            for (int h = m - 1; h >= 0; h--)
                if (((x >> h) & 1u) && basis[h])
                    x ^= basis[h];
            if (x) {
                basis[31 - __builtin_clz(x)] = x;
                a.row[k] = r;
                break;
            }
        }
    }
    a.b = (uint32_t)(rng.next() & mask);
    return a;
}

Affine identity(int m)
{
    Affine a;
    a.m = m;
    for (int k = 0; k < m; k++)
        a.row[k] = 1u << k;
    return a;
}

int spine_perm_nodes(int m, int r) { return perm_spine(m, r); }

struct Draw {
    std::vector<Affine> init; // [P][L]
    std::vector<Affine> cand; // [P][nperm][2L]
    int nperm = 0;
};

Draw draw_all(int m, int r, int P, int L, uint64_t seed, int pfht)
{
    Draw d;
    d.nperm = pfht ? spine_perm_nodes(m, r) : 0;
    d.init.resize((size_t)P * L);
    d.cand.resize((size_t)P * d.nperm * 2 * L);
    SplitMix64 rng{seed};
    for (int p = 0; p < P; p++) {
        for (int l = 0; l < L; l++)
            d.init[(size_t)p * L + l] = pfht ? draw_affine(m, rng) : identity(m);
        for (int v = 0; v < d.nperm; v++)
            for (int c = 0; c < 2 * L; c++)
                d.cand[((size_t)p * d.nperm + v) * 2 * L + c] = draw_affine(m - v, rng);
    }
    return d;
}

// The fresh mode's draw for one frame: decoder p draws, in the order of the
// fixed tables but row by row, from the SplitMix64 stream whose state is one
// step from seed ^ (frame << 20 | p).
Draw draw_fresh(int m, int r, int P, int L, uint64_t seed, int64_t frame)
{
    Draw d;
    d.nperm = spine_perm_nodes(m, r);
    d.init.resize((size_t)P * L);
    d.cand.resize((size_t)P * d.nperm * 2 * L);
    for (int p = 0; p < P; p++) {
        SplitMix64 key{seed ^ (((uint64_t)frame << 20) | (uint64_t)p)};
        SplitMix64 rng{key.next()};
        for (int l = 0; l < L; l++)
            d.init[(size_t)p * L + l] = draw_affine_rowwise(m, rng);
        for (int v = 0; v < d.nperm; v++)
            for (int c = 0; c < 2 * L; c++)
                d.cand[((size_t)p * d.nperm + v) * 2 * L + c] = draw_affine_rowwise(m - v, rng);
    }
    return d;
}

// A map as the kernel stores it: images of the unit vectors (columns) and b,
// obtained from the full permutation table q[i].
// One stored map: the images of the unit vectors (columns) and the offset,
// each times 4 (byte offsets of float elements, the form the kernels XOR into
// LDS addresses), then the dimension.
void store_table(const std::vector<uint32_t> &q, int m, uint32_t *out)
{
    for (int k = 0; k < kMapWords; k++)
        out[k] = 0;
    for (int k = 0; k < m; k++)
        out[k] = (q[1u << k] ^ q[0]) << 2;
    out[kMapB] = q[0] << 2;
    out[kMapB + 1] = (uint32_t)m;
}

std::vector<uint32_t> table_of(const Affine &a)
{
    std::vector<uint32_t> q((size_t)1 << a.m);
    for (uint32_t i = 0; i < q.size(); i++)
        q[i] = a.apply(i);
    return q;
}

std::vector<uint32_t> inverse_of(const std::vector<uint32_t> &q)
{
    std::vector<uint32_t> r(q.size());
    for (uint32_t i = 0; i < q.size(); i++)
        r[q[i]] = i;
    return r;
}

const KernelEntry *find_kernel(int m, int r, int L)
{
    const KernelTable tabs[] = {kernels_codes_a(), kernels_codes_b(), kernels_codes_c(), kernels_codes_d(),
                                kernels_codes_e(), kernels_codes_f(), kernels_codes_g(), kernels_codes_h(),
                                kernels_codes_i(), kernels_codes_j(), kernels_codes_k(), kernels_codes_l(),
                                kernels_codes_m(), kernels_codes_n(), kernels_codes_o(), kernels_codes_p(),
                                kernels_codes_q(), kernels_codes_r(), kernels_codes_s(), kernels_codes_t()};
    for (const KernelTable &t : tabs)
        for (int i = 0; i < t.count; i++)
            if (t.entries[i].m == m && t.entries[i].r == r && t.entries[i].L == L)
                return &t.entries[i];
    return nullptr;
}

int check_params(int m, int r, int P, int L, int perm_mode)
{
    if (m < 3 || m > 10)
        return fail(RM_E_INVAL, "m must be in [3, 10]");
    if (r < 1 || r > m - 1)
        return fail(RM_E_INVAL, "r must be in [1, m-1]");
    if (P < 1 || P > 1024)
        return fail(RM_E_INVAL, "P must be in [1, 1024]");
    if (!(L == 1 || L == 2 || L == 4 || L == 8 || L == 16 || L == 32 || L == 64))
        return fail(RM_E_INVAL, "L must be 1, 2, 4, 8, 16, 32 or 64");
    if (perm_mode != RM_PERM_NONE && perm_mode != RM_PERM_PFHT && perm_mode != RM_PERM_FRESH)
        return fail(RM_E_INVAL, "unknown perm_mode");
    return RM_OK;
}

int binom_sum(int m, int r)
{
    int k = 0, c = 1;
    for (int i = 0; i <= r; i++) {
        k += c;
        c = c * (m - i) / (i + 1);
    }
    return k;
}

} // namespace


extern "C" {

const char *rm_last_error(void) { return g_err.c_str(); }

int rm_supported(int m, int r, int L, int perm_mode)
{
    if (check_params(m, r, 1, L, perm_mode) != RM_OK)
        return 0;
    return find_kernel(m, r, L) != nullptr;
}

int rm_codeword_to_info(int m, int r, const uint8_t *codewords, int64_t n_frames, uint8_t *info, int64_t *n_invalid)
{
    if (m < 3 || m > 16 || r < 1 || r > m - 1)
        return fail(RM_E_INVAL, "need 3 <= m <= 16 and 1 <= r <= m-1");
    if (n_frames < 0)
        return fail(RM_E_INVAL, "n_frames < 0");
    if (n_frames > 0 && (!codewords || !info))
        return fail(RM_E_INVAL, "null array");
    const int N = 1 << m;
    std::vector<uint8_t> u(N);
    int64_t bad = 0;
    for (int64_t f = 0; f < n_frames; f++) {
        const uint8_t *x = codewords + f * (N / 8);
        for (int i = 0; i < N; i++)
            u[i] = (uint8_t)((x[i >> 3] >> (i & 7)) & 1u);
        // u = x G^{(x)m}: per stage, the first of each pair (i, i + h) takes
        // the XOR of both (G's lower-left 1), the second is kept
        for (int h = 1; h < N; h <<= 1)
            for (int i = 0; i < N; i += 2 * h)
                for (int j = i; j < i + h; j++)
                    u[j] ^= u[j + h];
        uint8_t *o = info + f * binom_sum(m, r);
        int k = 0, frozen = 0;
        for (int i = 0; i < N; i++) {
            if (__builtin_popcount((unsigned)i) >= m - r)
                o[k++] = u[i];
            else
                frozen |= u[i];
        }
        bad += frozen != 0;
    }
    if (n_invalid)
        *n_invalid = bad;
    return RM_OK;
}

int rm_perm_tables(int m, int r, int P, int L, uint64_t seed, int perm_mode, uint16_t *rows, uint16_t *b, int *mdim,
                   int cap)
{
    return rm_perm_tables_frame(m, r, P, L, seed, perm_mode, 0, rows, b, mdim, cap);
}

int rm_perm_tables_frame(int m, int r, int P, int L, uint64_t seed, int perm_mode, int64_t frame, uint16_t *rows,
                         uint16_t *b, int *mdim, int cap)
{
    int rc = check_params(m, r, P, L, perm_mode);
    if (rc != RM_OK)
        return rc;
    if (!rows || !b || !mdim)
        return fail(RM_E_INVAL, "null output array");
    if (frame < 0 || frame >= ((int64_t)1 << 43))
        return fail(RM_E_INVAL, "frame outside [0, 2^43)");
    const Draw d = perm_mode == RM_PERM_FRESH ? draw_fresh(m, r, P, L, seed, frame)
                                              : draw_all(m, r, P, L, seed, perm_mode == RM_PERM_PFHT);
    const int total = P * (L + d.nperm * 2 * L);
    if (cap < total)
        return fail(RM_E_INVAL, "cap too small: need " + std::to_string(total));
    int k = 0;
    auto put = [&](const Affine &a) {
        for (int j = 0; j < 16; j++)
            rows[k * 16 + j] = (uint16_t)(j < a.m ? a.row[j] : 0);
        b[k] = (uint16_t)a.b;
        mdim[k] = a.m;
        k++;
    };
    for (int p = 0; p < P; p++) {
        for (int l = 0; l < L; l++)
            put(d.init[(size_t)p * L + l]);
        for (int v = 0; v < d.nperm; v++)
            for (int c = 0; c < 2 * L; c++)
                put(d.cand[((size_t)p * d.nperm + v) * 2 * L + c]);
    }
    return k;
}

rm_decoder *rm_decoder_create_ex(const rm_config *cfg)
{
    if (!cfg) {
        fail(RM_E_INVAL, "null config");
        return nullptr;
    }
    if (check_params(cfg->m, cfg->r, cfg->P, cfg->L, cfg->perm_mode) != RM_OK)
        return nullptr;
    if (cfg->waves_per_block < 0 || cfg->waves_per_block > 4) {
        fail(RM_E_INVAL, "waves_per_block must be in [0, 4]");
        return nullptr;
    }
    const KernelEntry *k = find_kernel(cfg->m, cfg->r, cfg->L);
    if (!k) {
        fail(RM_E_UNSUPPORTED, "no kernel built for this (m, r, L)");
        return nullptr;
    }
    const int m = cfg->m, r = cfg->r, P = cfg->P, L = cfg->L;
    const int pfht = cfg->perm_mode == RM_PERM_PFHT;
    const int fresh = cfg->perm_mode == RM_PERM_FRESH;
    const Draw d = fresh ? Draw{{}, {}, spine_perm_nodes(m, r)} : draw_all(m, r, P, L, cfg->seed, pfht);
    const int mpd = 2 * L + 4 * L * d.nperm;
    if (mpd > k->maps_per_dec) { // the kernels' LDS holds at most maps_per_dec maps per decoder
        fail(RM_E_UNSUPPORTED, "more maps per decoder than the kernel holds");
        return nullptr;
    }

    // Per decoder: [0,L) initial maps, [L,2L) their inverses; for spine node v:
    // [2L+4Lv, 2L+4Lv+2L) candidate maps (at v = 0 composed after the initial
    // map of path c mod L), then their inverses.
    std::vector<uint32_t> host(fresh ? 0 : (size_t)P * mpd * kMapWords);
    for (int p = 0; p < (fresh ? 0 : P); p++) {
        uint32_t *base = host.data() + (size_t)p * mpd * kMapWords;
        std::vector<std::vector<uint32_t>> init_q(L);
        for (int l = 0; l < L; l++) {
            init_q[l] = table_of(d.init[(size_t)p * L + l]);
            store_table(init_q[l], m, base + (size_t)l * kMapWords);
            store_table(inverse_of(init_q[l]), m, base + (size_t)(L + l) * kMapWords);
        }
        for (int v = 0; v < d.nperm; v++) {
            const int md = m - v;
            for (int c = 0; c < 2 * L; c++) {
                std::vector<uint32_t> q = table_of(d.cand[((size_t)p * d.nperm + v) * 2 * L + c]);
                if (v == 0) {
                    const std::vector<uint32_t> &pi = init_q[c % L];
                    for (uint32_t &e : q)
                        e = pi[e];
                }
                store_table(q, md, base + (size_t)(2 * L + 4 * L * v + c) * kMapWords);
                store_table(inverse_of(q), md, base + (size_t)(2 * L + 4 * L * v + 2 * L + c) * kMapWords);
            }
        }
    }

    rm_decoder *dec = new (std::nothrow) rm_decoder();
    if (!dec) {
        fail(RM_E_NOMEM, "host allocation failed");
        return nullptr;
    }
    dec->cfg = *cfg;
    dec->N = 1 << m;
    dec->K = binom_sum(m, r);
    dec->nperm = d.nperm;
    dec->maps_per_dec = mpd;
    dec->kern = k;
    // one decoder per frame: D frames per wave where a packed kernel exists
    dec->packed = P == 1 && k->launch_packed != nullptr;
    dec->slice_bytes = dec->packed ? (fresh ? k->lds_bytes_packed : k->lds_bytes_packed_shared) : k->lds_bytes_per_wave;
    dec->stream = nullptr;
    dec->table_bytes = host.size() * sizeof(uint32_t);
    dec->fresh_chunk = 0;
    dec->fresh_done = nullptr;
    dec->fresh_pending = false;
    dec->d_maps = nullptr;
    if (fresh) {
        // the tables of up to 65536 frames at a time, at most 2 GiB: the draw
        // kernel runs one thread per (frame, decoder), and the more of them a
        // launch has, the better it hides its latency (RM(2,9) P = 20 L = 4:
        // 14.5 M frames/s with chunks of 16384, 15.3 M with 65536)
        const int64_t per_frame = (int64_t)P * mpd * kMapWords * sizeof(uint32_t);
        int64_t chunk = ((int64_t)2048 << 20) / per_frame;
        chunk = chunk < 1 ? 1 : (chunk > 65536 ? 65536 : chunk);
        dec->fresh_chunk = chunk;
        dec->table_bytes = (size_t)(chunk * per_frame);
    }
    int wpb = cfg->waves_per_block;
    hipError_t e = hipGetDevice(&dec->device);
    if (k->block_lds_bytes > 0) {
        // one workgroup per frame: its LDS must fit the device's per-block limit
        int lds_max = 0;
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dec->device);
        if (e == hipSuccess && (wpb > 1 || k->block_lds_bytes > lds_max)) {
            delete dec;
            fail(RM_E_UNSUPPORTED, wpb > 1 ? "lists of 16 or more paths run one frame per workgroup"
                                           : "the list does not fit the device's LDS per workgroup");
            return nullptr;
        }
        wpb = 1;
    } else {
        if (wpb == 0) {
            // one wave per workgroup where the wave's LDS slice is at most
            // 8 KiB (the finer-grained grid schedules better: RM(2,7) P=8 L=4
            // +12%, RM(2,9) P=20 L=4 +2.5% on MI355X), else as many waves as
            // 64 KiB of slices hold, up to 4 (RM(2,10) and RM(3,8) at L=8,
            // with 12 KiB slices, measured 1-3% slower with one)
            if (dec->slice_bytes <= 8192) {
                wpb = 1;
            } else {
                wpb = 65536 / dec->slice_bytes;
                wpb = wpb < 1 ? 1 : (wpb > 4 ? 4 : wpb);
            }
        }
        if ((size_t)wpb * dec->slice_bytes > 65536) {
            delete dec;
            fail(RM_E_UNSUPPORTED, "LDS slice does not fit the requested waves per block");
            return nullptr;
        }
    }
    dec->cfg.waves_per_block = wpb;
    if (e == hipSuccess)
        e = hipMalloc((void **)&dec->d_maps, dec->table_bytes);
    if (e == hipSuccess && !fresh)
        e = hipMemcpy(dec->d_maps, host.data(), dec->table_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && fresh)
        e = hipEventCreateWithFlags(&dec->fresh_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        fail(RM_E_HIP, std::string("HIP error at create: ") + hipGetErrorString(e));
        if (dec->d_maps)
            (void)hipFree(dec->d_maps);
        if (dec->fresh_done)
            (void)hipEventDestroy(dec->fresh_done);
        delete dec;
        return nullptr;
    }
    g_err.clear();
    return dec;
}

rm_decoder *rm_decoder_create(int m, int r, int P, int L, uint64_t seed)
{
    rm_config c{m, r, P, L, seed, RM_PERM_PFHT, 0};
    return rm_decoder_create_ex(&c);
}

void rm_decoder_destroy(rm_decoder *d)
{
    if (!d)
        return;
    (void)hipStreamSynchronize(d->stream);
    if (d->fresh_done) {
        // the last fresh-mode decode may have run on another stream
        (void)hipEventSynchronize(d->fresh_done);
        (void)hipEventDestroy(d->fresh_done);
    }
    (void)hipFree(d->d_maps);
    delete d;
}

int rm_decoder_set_stream(rm_decoder *d, void *hip_stream)
{
    if (!d)
        return fail(RM_E_INVAL, "null decoder");
    d->stream = (hipStream_t)hip_stream;
    return RM_OK;
}

int rm_decoder_info(const rm_decoder *d, rm_info *out)
{
    if (!d || !out)
        return fail(RM_E_INVAL, "null argument");
    out->m = d->cfg.m;
    out->r = d->cfg.r;
    out->P = d->cfg.P;
    out->L = d->cfg.L;
    out->N = d->N;
    out->K = d->K;
    out->perm_mode = d->cfg.perm_mode;
    out->n_perm_nodes = d->nperm;
    out->maps_per_decoder = d->maps_per_dec;
    out->waves_per_block = d->cfg.waves_per_block;
    out->lds_bytes_per_wave =
        (size_t)(d->kern->block_lds_bytes > 0 ? d->kern->block_lds_bytes : d->slice_bytes);
    out->table_bytes = d->table_bytes;
    return RM_OK;
}

int rm_decode_batch(rm_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_metric)
{
    if (!d)
        return fail(RM_E_INVAL, "null decoder");
    if (n_frames < 0)
        return fail(RM_E_INVAL, "n_frames < 0");
    if (n_frames == 0)
        return RM_OK;
    if (!llr || !out_bits)
        return fail(RM_E_INVAL, "null llr or out_bits");
    int rc = check_device_ptr(llr, "llr");
    if (rc == RM_OK)
        rc = check_device_ptr(out_bits, "out_bits");
    if (rc == RM_OK && out_metric)
        rc = check_device_ptr(out_metric, "out_metric");
    if (rc == RM_OK)
        rc = check_alignment(d->N, llr, out_bits, out_metric);
    if (rc != RM_OK)
        return rc;
    if (d->cfg.perm_mode == RM_PERM_FRESH)
        return fresh_decode(d, llr, n_frames, out_bits, out_metric);
    KernelArgs a = batch_args(d, llr, n_frames, out_bits, out_metric);
    hipError_t e = launch_decoder(d, a, n_frames);
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return RM_OK;
}

} // extern "C"
