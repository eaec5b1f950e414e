// rmdec_device.hpp -- gfx950 device code of the batched p-FHT-FSCL-L-M decoder.
//
// One wavefront decodes one frame at a time: it runs the P decoders of the
// frame one after another (Alg. 5) and keeps the best (smallest final metric)
// codeword.  Each decoder walks the Plotkin tree of RM(r,m) (Alg. 2), fully
// unrolled at compile time from (m, r, L).  Node LLRs and partial codewords
// live in the wave's LDS slice; the heavy per-node arithmetic (FHT, metric
// reductions, top-k selection) runs in registers in a "row layout": the L
// paths of the list occupy L groups of G = 64/L lanes, and element i of a
// path sits in lane (i mod G) of its group, register i div G.
//
// Every floating-point operation that can round is evaluated in the same
// order as the CPU oracle: halving-tree sums (v[i] += v[i+w], w = n/2..1),
// FHT butterflies with strides 2^{s-1}..1 computing (hi - lo, hi + lo),
// g = b +/- a, and the printed metric updates left to right.  Build with
// -ffp-contract=off.  Ties are broken by enumeration order everywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmdec {

constexpr int kWave = 64;

// Words per stored affine map: col[0..11], b at [12], m at [13].
constexpr int kMapWords = 16;
constexpr int kMapB = 12;

struct KernelArgs {
    const float *llr;
    uint8_t *out_bits;
    float *out_pm;
    const uint32_t *maps; // [P][maps_per_dec][kMapWords]
    int64_t n_frames;
    int P;
    int maps_per_dec;
    int pfht; // 1: permutation domain on; 0: identity, no permutation domain
    int waves;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Orders this wave's LDS traffic: every lane's earlier LDS writes are visible
// to every lane's later LDS reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float shfl_xor_f(float v, int mask) { return __shfl_xor(v, mask, kWave); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// min-sum check-node update f(a,b) = sgn(a) sgn(b) min(|a|,|b|): the value
// sgn(a) b clamped to [-|a|, |a|].  Equal to the textbook form except for the
// sign of a zero result, which no later step can observe.
__device__ __forceinline__ float f_minsum(float a, float b)
{
    const float sb = __uint_as_float(__float_as_uint(b) ^ (__float_as_uint(a) & 0x80000000u));
    return __builtin_amdgcn_fmed3f(sb, -fabsf(a), fabsf(a));
}

// bit-node update g(a,b,c) = b + (1-2c) a, one rounding
__device__ __forceinline__ float g_func(float a, float b, uint32_t c) { return c ? (b - a) : (b + a); }

// Affine map stored as columns: p(i) = b ^ XOR_{k: bit k of i} col[k].
template <int MD>
__device__ __forceinline__ uint32_t amap(const uint32_t *mp, uint32_t i)
{
    uint32_t p = mp[kMapB];
#pragma unroll
    for (int k = 0; k < MD; k++)
        p ^= ((i >> k) & 1u) ? mp[k] : 0u;
    return p;
}

// ---------------------------------------------------------------------------
// compile-time shape of a code and of its per-wave LDS slice
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int perm_spine(int m, int r)
{
    int c = 0;
    while (1 < r && r < m - 1) {
        c++;
        r--;
        m--;
    }
    return c;
}

__host__ __device__ constexpr int spc_tau(int L, int n) { return L == 1 ? 0 : (L < n - 1 ? L : n - 1); }

__host__ __device__ constexpr int max_spc_tau(int m, int r, int L)
{
    // SPC nodes RM(s-1, s) of the tree have s <= min(r+1, m); tau grows with s
    return spc_tau(L, 1 << (r + 1 < m ? r + 1 : m));
}

__host__ __device__ constexpr int align16(int x) { return (x + 15) & ~15; }

template <int M, int R, int L>
struct Shape {
    static constexpr int N = 1 << M;
    static constexpr int G = kWave / L;
    static constexpr int NPERM = perm_spine(M, R);
    static constexpr bool ROOT_LEAF = !(1 < R && R < M - 1);
    static constexpr int TAU = max_spc_tau(M, R, L);
    static constexpr int MAPS_PER_DEC = 2 * L + 4 * L * NPERM;

    // level m' < M buffers hold L * 2^{m'} entries, offset L * (2^{m'} - 8)
    static constexpr int LEVEL_ENTRIES = ROOT_LEAF ? 0 : L * (N - 8);
    __host__ __device__ static constexpr int lvl(int m) { return L * ((1 << m) - 8); }

    // byte offsets
    static constexpr int O_Y = 0;
    static constexpr int O_ABUF = align16(O_Y + 4 * N);
    static constexpr int O_AROOT = align16(O_ABUF + 4 * LEVEL_ENTRIES); // leaf roots only
    static constexpr int O_PTMP = align16(O_AROOT + (ROOT_LEAF ? 4 * L * N : 0));
    static constexpr int O_XL = align16(O_PTMP + (NPERM >= 2 ? 4 * L * N / 2 : 0));
    static constexpr int O_XR = align16(O_XL + LEVEL_ENTRIES);
    static constexpr int O_XPERM = align16(O_XR + LEVEL_ENTRIES);
    static constexpr int O_XROOT = align16(O_XPERM + (NPERM >= 2 ? L * N / 2 : 0));
    static constexpr int O_XBEST = align16(O_XROOT + L * N);
    static constexpr int O_MAPS = align16(O_XBEST + N);
    static constexpr int O_PML = align16(O_MAPS + 4 * kMapWords * MAPS_PER_DEC);
    static constexpr int O_PMR = O_PML + 4 * (M + 1) * L;
    static constexpr int O_PPM = O_PMR + 4 * (M + 1) * L;
    static constexpr int O_ANCL = O_PPM + 4 * (M + 1) * L;
    static constexpr int O_ANCR = O_ANCL + 4 * (M + 1) * L;
    static constexpr int O_SEL = O_ANCR + 4 * (M + 1) * L;
    static constexpr int O_LM = O_SEL + 4 * (M + 1) * 2 * L;
    static constexpr int O_PMROOT = O_LM + 4 * 2 * L;
    static constexpr int O_ANCROOT = O_PMROOT + 4 * L;
    static constexpr int O_RMAP = O_ANCROOT + 4 * L;
    static constexpr int O_ZERO = O_RMAP + 4 * L;
    static constexpr int O_CPM = O_ZERO + 4 * L;          // FHTL candidates: L*L metrics
    static constexpr int O_CINF = O_CPM + 4 * L * L;      // (index, sign) of each candidate
    static constexpr int O_SLOT = O_CINF + 4 * L * L;     // survivors
    static constexpr int O_FHTC = O_SLOT + 4 * L;         // per survivor: c word
    static constexpr int O_FHTB = O_FHTC + 4 * L;         // per survivor: b0
    static constexpr int O_ORD = O_FHTB + 4 * L;          // SPC: order[L][TAU+1]
    static constexpr int O_SSRC = O_ORD + 4 * L * (TAU + 1);
    static constexpr int O_SFLIP = O_SSRC + 4 * 2 * L;
    static constexpr int O_SP = O_SFLIP + 4 * 2 * L;
    static constexpr int O_SPM = O_SP + 4 * 2 * L;
    static constexpr int O_CSRC = O_SPM + 4 * 2 * L;
    static constexpr int O_CFLIP = O_CSRC + 4 * 2 * L;
    static constexpr int O_CP = O_CFLIP + 4 * 2 * L;
    static constexpr int O_CSPM = O_CP + 4 * 2 * L;
    static constexpr int O_SFIX = O_CSPM + 4 * 2 * L;
    static constexpr int O_BEST = O_SFIX + 4 * L;         // best metric, best inverse map word offset
    static constexpr int BYTES = align16(O_BEST + 16);
};

// Pointers into one wave's LDS slice.
template <int M, int R, int L>
struct Ws {
    using S = Shape<M, R, L>;
    unsigned char *base;
    __device__ explicit Ws(unsigned char *b) : base(b) {}
    __device__ float *y() const { return (float *)(base + S::O_Y); }
    __device__ float *abuf(int m) const { return (float *)(base + S::O_ABUF) + S::lvl(m); }
    __device__ float *aroot() const { return (float *)(base + S::O_AROOT); }
    __device__ float *ptmp() const { return (float *)(base + S::O_PTMP); }
    __device__ uint8_t *xl(int m) const { return base + S::O_XL + S::lvl(m); }
    __device__ uint8_t *xr(int m) const { return base + S::O_XR + S::lvl(m); }
    __device__ uint8_t *xperm() const { return base + S::O_XPERM; }
    __device__ uint8_t *xroot() const { return base + S::O_XROOT; }
    __device__ uint8_t *xbest() const { return base + S::O_XBEST; }
    __device__ uint32_t *maps() const { return (uint32_t *)(base + S::O_MAPS); }
    __device__ float *pmL(int m) const { return (float *)(base + S::O_PML) + m * L; }
    __device__ float *pmR(int m) const { return (float *)(base + S::O_PMR) + m * L; }
    __device__ float *ppm(int m) const { return (float *)(base + S::O_PPM) + m * L; }
    __device__ int *ancL(int m) const { return (int *)(base + S::O_ANCL) + m * L; }
    __device__ int *ancR(int m) const { return (int *)(base + S::O_ANCR) + m * L; }
    __device__ int *sel(int m) const { return (int *)(base + S::O_SEL) + m * 2 * L; }
    __device__ float *lm() const { return (float *)(base + S::O_LM); }
    __device__ float *pmroot() const { return (float *)(base + S::O_PMROOT); }
    __device__ int *ancroot() const { return (int *)(base + S::O_ANCROOT); }
    __device__ int *rmap() const { return (int *)(base + S::O_RMAP); }
    __device__ float *zero() const { return (float *)(base + S::O_ZERO); }
    __device__ float *cpm() const { return (float *)(base + S::O_CPM); }
    __device__ uint32_t *cinf() const { return (uint32_t *)(base + S::O_CINF); }
    __device__ int *slot() const { return (int *)(base + S::O_SLOT); }
    __device__ uint32_t *fhtc() const { return (uint32_t *)(base + S::O_FHTC); }
    __device__ uint32_t *fhtb() const { return (uint32_t *)(base + S::O_FHTB); }
    __device__ int *ord() const { return (int *)(base + S::O_ORD); }
    __device__ int *ssrc() const { return (int *)(base + S::O_SSRC); }
    __device__ uint32_t *sflip() const { return (uint32_t *)(base + S::O_SFLIP); }
    __device__ int *sp() const { return (int *)(base + S::O_SP); }
    __device__ float *spm() const { return (float *)(base + S::O_SPM); }
    __device__ int *csrc() const { return (int *)(base + S::O_CSRC); }
    __device__ uint32_t *cflip() const { return (uint32_t *)(base + S::O_CFLIP); }
    __device__ int *cp() const { return (int *)(base + S::O_CP); }
    __device__ float *cspm() const { return (float *)(base + S::O_CSPM); }
    __device__ uint32_t *sfix() const { return (uint32_t *)(base + S::O_SFIX); }
    __device__ float *bestpm() const { return (float *)(base + S::O_BEST); }
    __device__ int *bestmap() const { return (int *)(base + S::O_BEST + 4); }
};

// ---------------------------------------------------------------------------
// canonical halving-tree sum of one value per element, row layout.
// v[j] holds element i = lg + G*j (j < RR); the n-element sum ends in lane 0
// of the group.  Lanes whose element is beyond n only feed lanes that are
// never read.
// ---------------------------------------------------------------------------
template <int n, int G, int RR>
__device__ __forceinline__ float tree_sum_rows(float (&v)[RR])
{
#pragma unroll
    for (int w = n / 2; w >= G; w /= 2) {
#pragma unroll
        for (int j = 0; j < w / G; j++)
            v[j] = v[j] + v[j + w / G];
    }
    constexpr int top = (n < G ? n : G) / 2;
#pragma unroll
    for (int w = top; w >= 1; w /= 2)
        v[0] = v[0] + shfl_xor_f(v[0], w);
    return v[0];
}

// ---------------------------------------------------------------------------
// FHTL leaf, node RM(1, s): Alg. 3 over Alg. 4.
// in:  a [L][n] LLRs, pm_in[L];  out: x [L][n] codeword bytes, pm_out, anc_out
// ---------------------------------------------------------------------------
template <int M, int R, int L, int S>
__device__ void fhtl_leaf(const Ws<M, R, L> &w, const float *a, const float *pm_in, uint8_t *x, float *pm_out,
                          int *anc_out)
{
    constexpr int n = 1 << S;
    constexpr int G = kWave / L;
    constexpr int RR = n >= G ? n / G : 1;
    constexpr int K = L < n ? L : n;
    const int lane = lane_id();
    const int g = lane / G;
    const int lg = lane % G;
    const bool valid = (n >= G) || (lg < n);

    float F[RR];
    float v[RR];
#pragma unroll
    for (int j = 0; j < RR; j++) {
        const int i = lg + G * j;
        F[j] = valid ? a[g * n + i] : 0.0f;
        v[j] = fabsf(F[j]);
    }
    // LLR_abs by the halving tree, broadcast from lane 0 of the group
    const float sabs = __shfl(tree_sum_rows<n, G, RR>(v), 0, G);

    // butterflies, stride h = 2^{s-1} .. 1: (lo, hi) <- (hi - lo, hi + lo)
#pragma unroll
    for (int t = 0; t < S; t++) {
        const int h = 1 << (S - t - 1);
        if (h >= G) {
            const int hj = h / G;
#pragma unroll
            for (int j = 0; j < RR; j++)
                if ((j & hj) == 0) {
                    const float lo = F[j], hi = F[j + hj];
                    F[j] = hi - lo;
                    F[j + hj] = hi + lo;
                }
        } else {
            const bool upper = (lg & h) != 0;
#pragma unroll
            for (int j = 0; j < RR; j++) {
                const float p = shfl_xor_f(F[j], h);
                F[j] = upper ? (F[j] + p) : (p - F[j]);
            }
        }
    }

    // keys: |F| bits, then (1024 - i) so that lower indices win ties, then sign
    uint64_t key[RR];
#pragma unroll
    for (int j = 0; j < RR; j++) {
        const uint32_t i = (uint32_t)(lg + G * j);
        key[j] = valid ? (((uint64_t)__float_as_uint(fabsf(F[j])) << 32) | ((1024u - i) << 1) |
                          (F[j] < 0.0f ? 1u : 0u))
                       : 0ull;
    }
    float *cpm = w.cpm();
    uint32_t *cinf = w.cinf();
    const float pmg = pm_in[g];
    for (int t = 0; t < K; t++) {
        uint64_t best = key[0];
#pragma unroll
        for (int j = 1; j < RR; j++)
            best = umax64(best, key[j]);
#pragma unroll
        for (int m = (n < G ? n : G) / 2; m >= 1; m /= 2)
            best = umax64(best, shfl_xor_u64(best, m));
#pragma unroll
        for (int j = 0; j < RR; j++)
            if (key[j] == best)
                key[j] = 0ull;
        if (lg == 0) {
            const float absf = __uint_as_float((uint32_t)(best >> 32));
            const uint32_t lo = (uint32_t)best;
            cpm[g * K + t] = pmg + 0.5f * (sabs - absf);
            cinf[g * K + t] = ((1024u - (lo >> 1)) << 1) | (lo & 1u);
        }
    }
    wave_sync();

    // stable merge of the L*K candidates by metric; keep L
    int *slot = w.slot();
    if (lane < L)
        slot[lane] = 0;
    wave_sync();
    if (lane < L * K) {
        const float my = cpm[lane];
        int rank = 0;
        for (int e = 0; e < L * K; e++) {
            const float o = cpm[e];
            rank += (o < my) || (o == my && e < lane);
        }
        if (rank < L)
            slot[rank] = lane;
    }
    wave_sync();
    uint32_t *fc = w.fhtc();
    uint32_t *fb = w.fhtb();
    if (lane < L) {
        const int e = slot[lane];
        const uint32_t inf = cinf[e];
        const uint32_t idx = inf >> 1;
        const uint32_t c = (uint32_t)(n - 1) - idx;
        // codeword of transform index idx: x(z) = [F<0] ^ parity(c) ^ parity(c & z)
        fc[lane] = c;
        fb[lane] = (inf & 1u) ^ (__popc(c) & 1u);
        pm_out[lane] = cpm[e];
        anc_out[lane] = e / K;
    }
    wave_sync();
    for (int e = lane; e < L * n; e += kWave) {
        const int l = e / n;
        const uint32_t z = (uint32_t)(e % n);
        x[e] = (uint8_t)(fb[l] ^ (__popc(fc[l] & z) & 1u));
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// SPCL leaf, node RM(s-1, s): Eqs. (2)-(6) with tau = min(L, n-1) splits.
// ---------------------------------------------------------------------------
template <int M, int R, int L, int S>
__device__ void spcl_leaf(const Ws<M, R, L> &w, const float *a, const float *pm_in, uint8_t *x, float *pm_out,
                          int *anc_out)
{
    constexpr int n = 1 << S;
    constexpr int tau = spc_tau(L, n);
    constexpr int TS = Shape<M, R, L>::TAU + 1; // stride of the order table
    const int lane = lane_id();
    int *ord = w.ord();
    int *ssrc = w.ssrc();
    uint32_t *sflip = w.sflip();
    int *sp = w.sp();
    float *spm = w.spm();

    if (lane < L) {
        const float *al = a + lane * n;
        uint32_t p = 0;
        for (int i = 0; i < n; i++)
            p ^= al[i] < 0.0f ? 1u : 0u;
        // the tau+1 least reliable positions, |alpha| ascending, ties to the lower index
        float pv = -1.0f;
        int pi = -1;
        for (int t = 0; t <= tau; t++) {
            float bv = 0.0f;
            int bi = -1;
            for (int i = 0; i < n; i++) {
                const float av = fabsf(al[i]);
                const bool after = (av > pv) || (av == pv && i > pi);
                if (after && (bi < 0 || av < bv)) {
                    bv = av;
                    bi = i;
                }
            }
            bi = bi < 0 ? 0 : bi; // only reachable with non-finite input
            ord[lane * TS + t] = bi;
            pv = bv;
            pi = bi;
        }
        float pm = pm_in[lane];
        if (p)
            pm = pm + fabsf(al[ord[lane * TS]]);
        ssrc[lane] = lane;
        sflip[lane] = 0u;
        sp[lane] = (int)p;
        spm[lane] = pm;
    }
    wave_sync();

    int *csrc = w.csrc();
    uint32_t *cflip = w.cflip();
    int *cp = w.cp();
    float *cspm = w.cspm();
    for (int t = 1; t <= tau; t++) {
        if (lane < 2 * L) {
            const int q = lane >> 1;
            int src = ssrc[q];
            uint32_t fl = sflip[q];
            int p = sp[q];
            float pm = spm[q];
            if (lane & 1) {
                const float at = fabsf(a[src * n + ord[src * TS + t]]);
                const float a0 = fabsf(a[src * n + ord[src * TS]]);
                pm = (pm + at) + (p ? -a0 : a0);
                p ^= 1;
                fl |= 1u << t;
            }
            csrc[lane] = src;
            cflip[lane] = fl;
            cp[lane] = p;
            cspm[lane] = pm;
        }
        wave_sync();
        if (lane < 2 * L) {
            const float my = cspm[lane];
            int rank = 0;
            for (int e = 0; e < 2 * L; e++) {
                const float o = cspm[e];
                rank += (o < my) || (o == my && e < lane);
            }
            if (rank < L) {
                ssrc[rank] = csrc[lane];
                sflip[rank] = cflip[lane];
                sp[rank] = cp[lane];
                spm[rank] = cspm[lane];
            }
        }
        wave_sync();
    }

    uint32_t *sfix = w.sfix();
    if (lane < L) {
        const int src = ssrc[lane];
        const int o0 = ord[src * TS];
        // parity of the hard decisions of the source path, flipped once per split taken
        uint32_t p0 = 0;
        for (int i = 0; i < n; i++)
            p0 ^= a[src * n + i] < 0.0f ? 1u : 0u;
        const uint32_t hd0 = a[src * n + o0] < 0.0f ? 1u : 0u;
        sfix[lane] = p0 ^ (__popc(sflip[lane]) & 1u) ^ hd0; // Eq. (6)
        pm_out[lane] = spm[lane];
        anc_out[lane] = src;
    }
    wave_sync();
    for (int e = lane; e < L * n; e += kWave) {
        const int q = e / n;
        const int i = e % n;
        const int src = ssrc[q];
        const uint32_t fl = sflip[q];
        uint32_t bit = a[src * n + i] < 0.0f ? 1u : 0u;
        for (int t = 1; t <= tau; t++)
            if (((fl >> t) & 1u) && ord[src * TS + t] == i)
                bit ^= 1u;
        if (i == ord[src * TS])
            bit = sfix[q];
        x[e] = (uint8_t)bit;
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// permutation-domain selection at a node of size 2^MD (Alg. 2): candidate c
// reads path c mod L through map c; LM_c = sum_i |f|, halving tree; keep the
// L largest (ties to the lower c).  Source element i of path l is src(l, i).
// Writes sel[0..L) (candidate indices, rank order).
// ---------------------------------------------------------------------------
template <int M, int R, int L, int MD, class Src>
__device__ void perm_select(const Ws<M, R, L> &w, const uint32_t *cand_maps, Src src, int *sel)
{
    constexpr int n = 1 << MD;
    constexpr int h = n / 2;
    constexpr int G = kWave / L;
    constexpr int RR = h >= G ? h / G : 1;
    const int lane = lane_id();
    const int g = lane / G;
    const int lg = lane % G;
    const bool valid = (h >= G) || (lg < h);
    float *lm = w.lm();
#pragma unroll
    for (int pass = 0; pass < 2; pass++) {
        const int c = g + L * pass;
        const uint32_t *mp = cand_maps + c * kMapWords;
        const uint32_t colh = mp[MD - 1];
        float v[RR];
#pragma unroll
        for (int j = 0; j < RR; j++) {
            const uint32_t i = (uint32_t)(lg + G * j);
            float t = 0.0f;
            if (valid) {
                const uint32_t p = amap<MD>(mp, i);
                const float x0 = src(g, p);
                const float x1 = src(g, p ^ colh); // image of i + h
                t = fminf(fabsf(x0), fabsf(x1));
            }
            v[j] = t;
        }
        const float s = tree_sum_rows<h, G, RR>(v);
        if (lg == 0)
            lm[c] = s;
    }
    if (lane < L)
        sel[lane] = lane; // keeps every entry a valid candidate even for non-finite LM
    wave_sync();
    if (lane < 2 * L) {
        const float my = lm[lane];
        int rank = 0;
        for (int e = 0; e < 2 * L; e++) {
            const float o = lm[e];
            rank += (o > my) || (o == my && e < lane);
        }
        if (rank < L)
            sel[rank] = lane;
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Alg. 2 on a non-root node RM(RN, MN).  Its LLRs are in abuf(MN); it writes
// its L codewords to x, metrics to pm_out and ancestors to anc_out.
// SPINE: the node is reached from the root by left steps only, so it is in
// the permutation domain if it is an internal node.
// ---------------------------------------------------------------------------
template <int M, int R, int L, int MN, int RN, bool SPINE>
__device__ void node(const Ws<M, R, L> &w, int pfht, const float *pm_in, uint8_t *x, float *pm_out, int *anc_out)
{
    constexpr int n = 1 << MN;
    constexpr int h = n / 2;
    const int lane = lane_id();
    if constexpr (1 < RN && RN < MN - 1) {
        float *A = w.abuf(MN);
        const bool is_per = SPINE && pfht;
        int *sel = w.sel(MN);
        const uint32_t *maps = w.maps();
        constexpr int v = M - MN; // depth on the spine
        constexpr int base = 2 * L + 4 * L * v;
        if (is_per) {
            perm_select<M, R, L, MN>(
                w, maps + base * kMapWords,
                [&](int l, uint32_t i) { return A[l * n + i]; }, sel);
            float *T = w.ptmp();
            for (int e = lane; e < L * n; e += kWave) {
                const int l = e / n;
                const uint32_t i = (uint32_t)(e % n);
                const int c = sel[l];
                T[e] = A[(c % L) * n + amap<MN>(maps + (base + c) * kMapWords, i)];
            }
            if (lane < L)
                w.ppm(MN)[lane] = pm_in[sel[lane] % L];
            wave_sync();
            for (int e = lane; e < L * n; e += kWave)
                A[e] = T[e];
            pm_in = w.ppm(MN);
            wave_sync();
        }
        // left child on f
        float *C = w.abuf(MN - 1);
        for (int e = lane; e < L * h; e += kWave) {
            const int l = e / h, i = e % h;
            C[e] = f_minsum(A[l * n + i], A[l * n + i + h]);
        }
        wave_sync();
        node<M, R, L, MN - 1, RN - 1, SPINE>(w, pfht, pm_in, w.xl(MN - 1), w.pmL(MN - 1), w.ancL(MN - 1));
        // right child on g, reading the surviving ancestor's LLRs
        const uint8_t *XL = w.xl(MN - 1);
        const int *ancL = w.ancL(MN - 1);
        for (int e = lane; e < L * h; e += kWave) {
            const int l = e / h, i = e % h;
            const int k = ancL[l];
            C[e] = g_func(A[k * n + i], A[k * n + i + h], XL[e]);
        }
        wave_sync();
        node<M, R, L, MN - 1, RN, false>(w, pfht, w.pmL(MN - 1), w.xr(MN - 1), w.pmR(MN - 1), w.ancR(MN - 1));
        // combine (x_gamma ^ x_lambda, x_gamma)
        const uint8_t *XR = w.xr(MN - 1);
        const int *ancR = w.ancR(MN - 1);
        uint8_t *XO = is_per ? w.xperm() : x;
        for (int e = lane; e < L * h; e += kWave) {
            const int l = e / h, i = e % h;
            const int k = ancR[l];
            const uint8_t xr = XR[e];
            XO[l * n + i] = (uint8_t)(xr ^ XL[k * h + i]);
            XO[l * n + i + h] = xr;
        }
        if (lane < L) {
            const int a = ancL[ancR[lane]];
            pm_out[lane] = w.pmR(MN - 1)[lane];
            anc_out[lane] = is_per ? (sel[a] % L) : a;
        }
        wave_sync();
        if (is_per) {
            // undo the selected permutation: x[p(i)] = x'[i]  <=>  x[j] = x'[p^{-1}(j)]
            for (int e = lane; e < L * n; e += kWave) {
                const int l = e / n;
                const uint32_t j = (uint32_t)(e % n);
                const int a = ancL[ancR[l]];
                const int c = sel[a];
                x[e] = XO[l * n + amap<MN>(maps + (base + 2 * L + c) * kMapWords, j)];
            }
            wave_sync();
        }
    } else if constexpr (RN == 1) {
        fhtl_leaf<M, R, L, MN>(w, w.abuf(MN), pm_in, x, pm_out, anc_out);
    } else if constexpr (RN == MN - 1) {
        spcl_leaf<M, R, L, MN>(w, w.abuf(MN), pm_in, x, pm_out, anc_out);
    }
}

// ---------------------------------------------------------------------------
// One decoder (Alg. 2 at the root, Alg. 5 loop body).  maps_g: this decoder's
// maps in global memory.  Returns with pmroot/ancroot/xroot filled and
// rmap[l] = forward map index of root path l.
// ---------------------------------------------------------------------------
template <int M, int R, int L>
__device__ void decode_root(const Ws<M, R, L> &w, int pfht)
{
    using Sh = Shape<M, R, L>;
    constexpr int N = Sh::N;
    constexpr int h = N / 2;
    const int lane = lane_id();
    const float *Y = w.y();
    const uint32_t *maps = w.maps();
    int *rmap = w.rmap();
    float *zero = w.zero();
    if (lane < L)
        zero[lane] = 0.0f;

    if constexpr (!Sh::ROOT_LEAF) {
        const bool is_per = pfht != 0;
        if (is_per) {
            // candidate c: composite map (initial map of path c mod L, then candidate c)
            perm_select<M, R, L, M>(
                w, maps + 2 * L * kMapWords, [&](int, uint32_t i) { return Y[i]; }, w.sel(M));
            if (lane < L)
                rmap[lane] = 2 * L + w.sel(M)[lane];
        } else {
            if (lane < L)
                rmap[lane] = lane;
        }
        wave_sync();
        float *C = w.abuf(M - 1);
        for (int e = lane; e < L * h; e += kWave) {
            const int l = e / h, i = e % h;
            const uint32_t *mp = maps + rmap[l] * kMapWords;
            const uint32_t p = amap<M>(mp, (uint32_t)i);
            C[e] = f_minsum(Y[p], Y[p ^ mp[M - 1]]);
        }
        wave_sync();
        node<M, R, L, M - 1, R - 1, true>(w, pfht, zero, w.xl(M - 1), w.pmL(M - 1), w.ancL(M - 1));
        const uint8_t *XL = w.xl(M - 1);
        const int *ancL = w.ancL(M - 1);
        for (int e = lane; e < L * h; e += kWave) {
            const int l = e / h, i = e % h;
            const uint32_t *mp = maps + rmap[ancL[l]] * kMapWords;
            const uint32_t p = amap<M>(mp, (uint32_t)i);
            C[e] = g_func(Y[p], Y[p ^ mp[M - 1]], XL[e]);
        }
        wave_sync();
        node<M, R, L, M - 1, R, false>(w, pfht, w.pmL(M - 1), w.xr(M - 1), w.pmR(M - 1), w.ancR(M - 1));
        const uint8_t *XR = w.xr(M - 1);
        const int *ancR = w.ancR(M - 1);
        uint8_t *XO = w.xroot();
        for (int e = lane; e < L * h; e += kWave) {
            const int l = e / h, i = e % h;
            const uint8_t xr = XR[e];
            XO[l * N + i] = (uint8_t)(xr ^ XL[ancR[l] * h + i]);
            XO[l * N + i + h] = xr;
        }
        if (lane < L) {
            w.pmroot()[lane] = w.pmR(M - 1)[lane];
            w.ancroot()[lane] = ancL[ancR[lane]];
        }
        wave_sync();
    } else {
        // leaf root: the L paths start from y through their initial maps
        if (lane < L)
            rmap[lane] = lane;
        wave_sync();
        float *A = w.aroot();
        for (int e = lane; e < L * N; e += kWave) {
            const int l = e / N;
            A[e] = Y[amap<M>(maps + l * kMapWords, (uint32_t)(e % N))];
        }
        wave_sync();
        if constexpr (R == 1)
            fhtl_leaf<M, R, L, M>(w, A, zero, w.xroot(), w.pmroot(), w.ancroot());
        else
            spcl_leaf<M, R, L, M>(w, A, zero, w.xroot(), w.pmroot(), w.ancroot());
    }
}

// ---------------------------------------------------------------------------
// kernel: one wave per frame (grid-stride), P decoders per frame
// ---------------------------------------------------------------------------
template <int M, int R, int L>
__global__ void __launch_bounds__(256) rm_decode_kernel(KernelArgs args)
{
    using Sh = Shape<M, R, L>;
    constexpr int N = Sh::N;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    Ws<M, R, L> w(smem + wave * Sh::BYTES);
    const int64_t stride = (int64_t)gridDim.x * args.waves;
    for (int64_t f = (int64_t)blockIdx.x * args.waves + wave; f < args.n_frames; f += stride) {
        const float *src = args.llr + f * N;
        for (int i = lane; i < N; i += kWave)
            w.y()[i] = src[i];
        for (int i = lane; i < N; i += kWave)
            w.xbest()[i] = 0;
        if (lane == 0) {
            w.bestpm()[0] = __builtin_inff();
            w.bestmap()[0] = 0;
        }
        wave_sync();
        for (int d = 0; d < args.P; d++) {
            const uint32_t *mg = args.maps + (size_t)d * args.maps_per_dec * kMapWords;
            for (int i = lane; i < args.maps_per_dec * kMapWords; i += kWave)
                w.maps()[i] = mg[i];
            wave_sync();
            decode_root<M, R, L>(w, args.pfht);
            // Alg. 5: first minimum over the list, replace only if strictly smaller
            const float *pmr = w.pmroot();
            int ls = 0;
            for (int l = 1; l < L; l++)
                if (pmr[l] < pmr[ls])
                    ls = l;
            const float pbest = w.bestpm()[0];
            if (pmr[ls] < pbest) {
                const uint8_t *xs = w.xroot() + ls * N;
                for (int i = lane; i < N; i += kWave)
                    w.xbest()[i] = xs[i];
                const int a = w.ancroot()[ls];
                const int inv = w.rmap()[a] + (Sh::ROOT_LEAF || !args.pfht ? L : 2 * L);
                wave_sync();
                if (lane == 0) {
                    w.bestpm()[0] = pmr[ls];
                    w.bestmap()[0] = d * args.maps_per_dec + inv;
                }
            }
            wave_sync();
        }
        // map the winner back to channel order and pack bits
        const uint32_t *mi = args.maps + (size_t)w.bestmap()[0] * kMapWords;
        uint8_t *ob = args.out_bits + f * (N / 8);
        for (int j0 = 0; j0 < N; j0 += kWave) {
            const int j = j0 + lane;
            uint32_t bit = 0;
            if (j < N)
                bit = w.xbest()[amap<M>(mi, (uint32_t)j)];
            const uint64_t mask = __ballot(bit != 0);
            if (N >= kWave) {
                if (lane == 0)
                    *(uint64_t *)(ob + j0 / 8) = mask;
            } else if (lane < N / 8) {
                ob[lane] = (uint8_t)(mask >> (8 * lane));
            }
        }
        if (args.out_pm && lane == 0)
            args.out_pm[f] = w.bestpm()[0];
        wave_sync();
    }
}

} // namespace rmdec
