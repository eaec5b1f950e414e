// rmdec_biglist.hpp -- p-FHT-FSCL / FHT-FSCL with large lists (L = 16, 32,
// 64): one workgroup of 512 threads per frame, the L paths' LLR and codeword
// stacks in LDS.
//
// The register-resident kernels hold a path in 64/L lanes, which cannot hold
// a half-length node vector once L exceeds 8.  Here the paths live in LDS:
// the LLRs of level s (1 <= s < m) take L*2^s floats (L*N floats in all),
// the codeword bits of both children of the node at level s take 2*L*2^s
// bits.  Thread t of a path-parallel step serves path t / G (G = 512 / L
// threads per path); element-parallel steps stride over the path's row.
//
// The operations and their order are those of the batched kernels: Alg. 2
// (candidate maps of the permutation domain, kept by the largest sum of
// |f|, ties to the lower candidate), Alg. 3 and 4 (FHT list decoding with
// the metric of Eq. (10); the min(L, 2^s) largest |F| per path, ties to the
// lower index; candidates merged in the order (metric, path, rank)), the SPC
// list rules of Eqs. (2)-(6), and Alg. 5 over the P decoders.  Sums of
// |alpha| and |f| follow the halving tree v[i] += v[i + w], w = n/2 .. 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmdec_device.hpp"
#include "rmdec_kernels.hpp"

namespace rmdec {
namespace big {

constexpr int kThreads = 512;
// Permutation-domain nodes on the spine the layout holds (r - 1 for
// RM(r, m)): every internal code of length 2^m, except at L = 64, where
// three (r <= 4) keep two workgroups per CU.
constexpr int max_perm(int M, int L) { return (L >= 64 || M < 6) ? 3 : M - 3; }

__host__ __device__ constexpr int words_of(int s) { return s >= 5 ? (1 << (s - 5)) : 1; }
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// LDS layout in 32-bit words.
template <int M, int L>
struct Lay {
    static constexpr int N = 1 << M;
    static constexpr int G = kThreads / L; // threads per path
    static constexpr int Y = 0;             // N floats: the channel LLRs
    static constexpr int A = N;             // level s at A + L*(2^s - 2): L rows of 2^s floats
    static constexpr int A_END = A + L * (N - 2);
    // codeword bits: level s (3..M), side 0 (left child) and 1 (right)
    static constexpr int xb_below(int s)
    {
        int w = 0;
        for (int t = 3; t < s; t++)
            w += 2 * L * words_of(t);
        return w;
    }
    static constexpr int XB = A_END;
    static constexpr int XB_END = XB + xb_below(M) + L * words_of(M); // the root: side 0 only
    // (path and candidate indices are below 256 and kept as bytes, so that
    // two workgroups fit a CU at L*N = 16384)
    // per level s = 3..M: metrics and ancestors of both children's outputs
    static constexpr int PM = XB_END;                   // [M-2][2][L] floats
    static constexpr int ANC = PM + (M - 2) * 2 * L;    // [M-2][2][L] bytes
    // per permutation-domain node (by its depth on the leftmost spine):
    // kept candidates, their source path and metric
    static constexpr int NPM = max_perm(M, L);
    static constexpr int SEL = ANC + (M - 2) * 2 * L / 4; // [NPM][2L] bytes
    static constexpr int ORIG = SEL + NPM * 2 * L / 4;    // [NPM][L] bytes
    static constexpr int PPM = ORIG + NPM * L / 4;        // [NPM][L] floats
    static constexpr int SCR = PPM + NPM * L;             // 2L floats: the candidates' LM values
    static constexpr int PM0 = SCR + 2 * L;                 // L floats: the root's input metrics
    static constexpr int SIDX = PM0 + L;                    // L uint16: FHT survivors' index and sign
    static constexpr int PAR = SIDX + L / 2;                // L bytes: SPC parities of the input paths
    // SPC list state, two copies: source path, parity, metric, flips (2 words,
    // at an even word offset for 8-byte accesses)
    static constexpr int SPC = (PAR + L / 4 + 1) & ~1;
    static constexpr int SPC_ONE = 5 * L;
    static constexpr int BEST = SPC + 2 * SPC_ONE; // the frame's best codeword, N bits
    static constexpr int MISC = BEST + words_of(M);
    static constexpr int WORDS = MISC + 4; // best metric, improved flag, winner
    static constexpr int BYTES = WORDS * 4;

    static constexpr int a_off(int s) { return A + L * ((1 << s) - 2); }
    static constexpr int xb_off(int s, int side) { return XB + xb_below(s) + side * L * words_of(s); }

    // Every array the kernel indexes ends at or before the next one begins,
    // for the largest index its accessors form (row l < L, element i < 2^s,
    // level s, side, permutation-domain depth v < NPM), and the 8-byte
    // accesses of the SPC flip masks are aligned.  Checked for every built
    // shape when the kernel is instantiated.
    static constexpr bool layout_ok()
    {
        if (L % 4 != 0 || L > 256 || M < 4)
            return false;
        for (int s = 1; s < M; s++) // level rows: a_off(s) + l 2^s + i
            if (a_off(s) < A || a_off(s) + L * (1 << s) > A_END)
                return false;
        for (int s = 3; s < M; s++) // both children's codeword bits of level s
            if (xb_off(s, 1) + L * words_of(s) > xb_off(s + 1, 0))
                return false;
        if (XB < A_END || xb_off(3, 0) != XB || xb_off(M, 0) + L * words_of(M) > XB_END)
            return false;
        return PM >= XB_END && PM + (M - 2) * 2 * L <= ANC            // [M-2][2][L] floats
               && ANC + (M - 2) * 2 * L / 4 <= SEL                     // [M-2][2][L] bytes
               && SEL + NPM * 2 * L / 4 <= ORIG                        // [NPM][2L] bytes
               && ORIG + NPM * L / 4 <= PPM                            // [NPM][L] bytes
               && PPM + NPM * L <= SCR                                 // [NPM][L] floats
               && SCR + 2 * L <= PM0 && PM0 + L <= SIDX                // 2L and L floats
               && SIDX + L / 2 <= PAR && PAR + L / 4 <= SPC            // L uint16, L bytes
               && SPC % 2 == 0 && SPC_ONE % 2 == 0 && (3 * L) % 2 == 0 // flip masks: 8-byte aligned
               && SPC + 2 * SPC_ONE <= BEST                            // two copies of 5L words
               && BEST + words_of(M) <= MISC && MISC + 4 <= WORDS;
    }
};

template <int S>
struct MapR {
    uint32_t col[S];
    uint32_t b;
};

// a stored map (columns and offset as byte offsets, times 4) into registers
template <int S>
__device__ __forceinline__ void load_map(const uint32_t *mp, MapR<S> &m)
{
#pragma unroll
    for (int k = 0; k < S; k++)
        m.col[k] = mp[k] >> 2;
    m.b = mp[kMapB] >> 2;
}

template <int S>
__device__ __forceinline__ void identity_map(MapR<S> &m)
{
#pragma unroll
    for (int k = 0; k < S; k++)
        m.col[k] = 1u << k;
    m.b = 0;
}

// Loops over i = t0 + STEP*x (x < NIT, a power of two, t0 < STEP) that need
// p(i) visit x in Gray-code order, x_t = t ^ (t >> 1): consecutive x differ
// in bit ctz(t), so p(i) changes by one column, p_t = p_{t-1} ^ col[log2
// STEP + ctz(t)], one XOR per index instead of one per set bit.  The loops
// are unrolled, so the column index is a constant.
template <int S>
__device__ __forceinline__ uint32_t apply_map(const MapR<S> &m, uint32_t i)
{
    uint32_t p = m.b;
#pragma unroll
    for (int k = 0; k < S; k++)
        p ^= ((i >> k) & 1u) ? m.col[k] : 0u;
    return p;
}

__device__ __forceinline__ float big_fminsum(float a, float b)
{
    const float m = fminf(fabsf(a), fabsf(b));
    return ((__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u) ? -m : m;
}
__device__ __forceinline__ float big_g(float a, float b, uint32_t c) { return b + (1.0f - 2.0f * (float)c) * a; }

// The selection keys are 64-bit patterns whose high word is the bit pattern
// of a non-negative finite or infinite float (a metric or an |x|): read as
// doubles they are finite and non-negative, and for such patterns the order
// of the doubles is the unsigned order of the bits.  So one v_max_f64 /
// v_min_f64 compares and selects a pair of keys.  kKeyPad, the double +inf,
// lies above every key; 0 lies at or below every key.
constexpr uint64_t kKeyPad = 0x7FF0000000000000ull;
__device__ __forceinline__ double key_d(uint64_t k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ uint64_t d_key(double d) { return (uint64_t)__double_as_longlong(d); }
// smallest key over aligned groups of 2W lanes, the same in each lane (DPP
// and swizzle butterflies; bfly_max, the largest, is the batched kernels')
template <int W>
__device__ __forceinline__ double bfly_min(double v)
{
    if constexpr (W >= 1)
        return bfly_min<W / 2>(dmin(v, xor64<span_xor<W>()>(v)));
    else
        return v;
}

// row broadcast (DPP): rows whose bit is set in RM take lane CTRL's value
// from the row below (row_bcast:15 = 0x142, row_bcast:31 = 0x143); the
// other rows keep their own
template <int CTRL, int RM>
__device__ __forceinline__ double row_bcast(double v)
{
    const uint64_t u = d_key(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)u, (int)(uint32_t)u, CTRL, RM, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(u >> 32), (int)(uint32_t)(u >> 32), CTRL, RM, 0xF, false);
    return key_d(((uint64_t)hi << 32) | lo);
}
// the two smallest of two disjoint sets given by their two smallest
// (x1 <= x2, y1 <= y2)
__device__ __forceinline__ void merge_two(double &x1, double &x2, double y1, double y2)
{
    const double s1 = dmin(x1, y1);
    x2 = dmin(dmax(x1, y1), dmin(x2, y2));
    x1 = s1;
}
template <int W>
__device__ __forceinline__ void bfly_min2(double &x1, double &x2)
{
    if constexpr (W >= 1) {
        const double y1 = xor64<span_xor<W>()>(x1), y2 = xor64<span_xor<W>()>(x2);
        merge_two(x1, x2, y1, y2);
        bfly_min2<W / 2>(x1, x2);
    }
}
__device__ __forceinline__ uint64_t lane63(double v)
{
    const uint64_t u = d_key(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}
// The two smallest keys of the whole wave (all 64 lanes active), each lane
// offering its two smallest (v1 <= v2): butterflies within each row of 16
// lanes (the strides 8, 7, 2, 1 pair disjoint sets at every level), then the
// two row broadcasts; lane 63 ends with all four rows (the rows that keep
// their own value in a broadcast merge with themselves, but lane 63 never
// reads them).
__device__ __forceinline__ void wave_umin2(uint64_t v1, uint64_t v2, uint64_t &m1, uint64_t &m2)
{
    double x1 = key_d(v1), x2 = key_d(v2);
    bfly_min2<8>(x1, x2);
    merge_two(x1, x2, row_bcast<0x142, 0xA>(x1), row_bcast<0x142, 0xA>(x2));
    merge_two(x1, x2, row_bcast<0x143, 0xC>(x1), row_bcast<0x143, 0xC>(x2));
    m1 = lane63(x1);
    m2 = lane63(x2);
}

template <int M, int L>
struct BigCtx {
    using Ly = Lay<M, L>;
    static_assert(Ly::layout_ok(), "large-list LDS arrays overlap or leave the slice");
    uint32_t *w;            // LDS words
    const uint32_t *dmaps;  // this decoder's maps
    int tid;
    int pfht;

    __device__ float *f(int off) const { return (float *)(w + off); }
    __device__ int *i(int off) const { return (int *)(w + off); }
    __device__ float *y() const { return f(Ly::Y); }
    __device__ float *a(int s) const { return f(Ly::a_off(s)); } // row l at a(s) + l*2^s
    __device__ uint32_t *xb(int s, int side) const { return w + Ly::xb_off(s, side); }
    __device__ float *pm(int s, int side) const { return f(Ly::PM + ((s - 3) * 2 + side) * L); }
    __device__ uint8_t *b(int off) const { return (uint8_t *)(w + off); }
    __device__ uint8_t *anc(int s, int side) const { return b(Ly::ANC) + ((s - 3) * 2 + side) * L; }
    __device__ uint8_t *sel(int v) const { return b(Ly::SEL) + v * 2 * L; }
    __device__ uint8_t *orig(int v) const { return b(Ly::ORIG) + v * L; }
    __device__ uint16_t *sidx() const { return (uint16_t *)(w + Ly::SIDX); }
    __device__ uint8_t *par() const { return b(Ly::PAR); }
    __device__ float *ppm(int v) const { return f(Ly::PPM + v * L); }
    __device__ const uint32_t *map(int k) const { return dmaps + (size_t)k * kMapWords; }
};

// bit j of path row l at level s (row of words_of(s) words)
template <int S>
__device__ __forceinline__ uint32_t get_bit(const uint32_t *rows, int l, uint32_t j)
{
    return (rows[l * words_of(S) + (j >> 5)] >> (j & 31)) & 1u;
}

// The LLR of element i of the (unpermuted) input row of path l at level S:
// the channel LLRs at the root, else the stored row.
template <int M, int L, int S>
__device__ __forceinline__ float in_llr(const BigCtx<M, L> &c, int l, uint32_t i)
{
    if constexpr (S == M)
        return c.y()[i];
    else
        return c.a(S)[l * (1 << S) + i];
}

// Ascending bitonic sort of NK = 2^k distinct 64-bit keys held by wave 0:
// element i = lane + 64 r sits in register r (two registers for NK = 128);
// afterwards element i holds the key of rank i.  Lanes past NK hold keys of
// their own (sorted among themselves, never mixed with the NK).
template <int NK>
using WaveKeys = uint64_t[NK > kWave ? 2 : 1];

template <int NK, int SZ, int D>
__device__ __forceinline__ void wave_sort_stage(WaveKeys<NK> &k, int lane)
{
    constexpr int NR = NK > kWave ? 2 : 1;
    if constexpr (D == kWave) {
        // between the two registers of a lane (the final merge of 128)
        const uint64_t a = k[0], b = k[1];
        k[0] = a < b ? a : b;
        k[1] = a < b ? b : a;
    } else {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const uint64_t o = xor_lanes<D>(k[r]);
            const int i = lane + kWave * r;
            const bool asc = SZ >= NK || (i & SZ) == 0;
            const bool takemin = ((i & D) == 0) == asc;
            const bool less = k[r] < o;
            k[r] = (less == takemin) ? k[r] : o;
        }
    }
}
template <int NK, int SZ, int D>
__device__ __forceinline__ void wave_sort_run(WaveKeys<NK> &k, int lane)
{
    wave_sort_stage<NK, SZ, D>(k, lane);
    if constexpr (D > 1)
        wave_sort_run<NK, SZ, D / 2>(k, lane);
    else if constexpr (SZ < NK)
        wave_sort_run<NK, SZ * 2, SZ>(k, lane);
}
template <int NK>
__device__ __forceinline__ void wave_sort(WaveKeys<NK> &k, int lane)
{
    wave_sort_run<NK, 2, 1>(k, lane);
}

// Of L sorted lists (row l: metric[l*mstride + j], j < K, non-decreasing)
// keep the L smallest entries in the order (metric, l, j), as a stable merge
// of the lists would: out_pm[q], out_src[q] = l and out_code[q] =
// code[l*cstride + j] for q = 0..L-1 in that order.  A tournament in wave 0:
// lane l holds the next four entries of list l as keys (metric bits, l, j)
// (metrics are non-negative, so their bit patterns order as the values do);
// each of L/2 rounds takes the two smallest keys of the wave (from every
// lane's two smallest remaining entries), which lanes 2r and 2r+1 keep for
// round r, and the winning lanes shift their windows, reloading once fewer
// than two entries are left in a window but not in the list.  The outputs
// are then written by lanes 0..L-1 together.
template <int L, int K>
__device__ __forceinline__ void select_smallest(int tid, const float *metric, int mstride, const uint16_t *code, int cstride,
                                                float *out_pm, uint8_t *out_src, uint16_t *out_code)
{
    static_assert(L <= kWave, "one lane per list");
    if (tid < kWave) {
        const int lane = tid;
        auto key_at = [&](int j) {
            return (lane < L && j < K) ? ((uint64_t)__float_as_uint(metric[lane * mstride + j]) << 32) |
                                             ((uint64_t)lane << 16) | (uint64_t)j
                                       : kKeyPad;
        };
        uint64_t w0 = key_at(0), w1 = key_at(1), w2 = key_at(2), w3 = key_at(3);
        int nxt = 4;             // next entry of the list not yet in the window
        uint64_t mine = kKeyPad; // the winner of round `lane`
        static_assert(L % 2 == 0, "two winners per round");
        for (int q = 0; q < L; q += 2) {
            uint64_t m1, m2;
            wave_umin2(w0, w1, m1, m2);
            mine = lane == q ? m1 : (lane == q + 1 ? m2 : mine);
            const int l1 = (int)((m1 >> 16) & 0xFFFFu), l2 = (int)((m2 >> 16) & 0xFFFFu);
            const bool p1 = lane == l1 || lane == l2; // pops one entry
            const bool p2 = lane == l1 && lane == l2; // pops two
            const uint64_t n0 = p2 ? w2 : (p1 ? w1 : w0);
            const uint64_t n1 = p2 ? w3 : (p1 ? w2 : w1);
            const uint64_t n2 = p2 ? kKeyPad : (p1 ? w3 : w2);
            w3 = p1 ? kKeyPad : w3;
            w0 = n0;
            w1 = n1;
            w2 = n2;
            // padding sits only at the end of a window, so w1 is the padding
            // exactly when fewer than two entries are left in it
            const bool refill = p1 && w1 == kKeyPad && nxt < K;
            if (__any(refill)) {
                if (refill) {
                    if (w0 == kKeyPad) {
                        w0 = key_at(nxt);
                        w1 = key_at(nxt + 1);
                        w2 = key_at(nxt + 2);
                        w3 = key_at(nxt + 3);
                        nxt += 4;
                    } else {
                        w1 = key_at(nxt);
                        w2 = key_at(nxt + 1);
                        w3 = key_at(nxt + 2);
                        nxt += 3;
                    }
                }
            }
        }
        if (lane < L) {
            const int wl = (int)((mine >> 16) & 0xFFFFu), wj = (int)(mine & 0xFFFFu);
            out_pm[lane] = __uint_as_float((uint32_t)(mine >> 32));
            out_src[lane] = (uint8_t)wl;
            out_code[lane] = code[wl * cstride + wj];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// FHTL on a list (Alg. 3 over Alg. 4): L path rows of n = 2^S LLRs, path l's
// at rows + l n.  Per path: the sum of |alpha| (halving tree), the Hadamard
// transform in place, and the K = min(L, n) largest |F| (ties to the lower
// index) as candidates with the metric of Eq. (10) from pm_in[l]; then the L
// smallest of the L K candidates in the order (metric, path, rank): their
// metrics, source paths and (index, sign) codes into out_pm, out_anc,
// out_code, and their codewords into xo ([L][words_of(S)] words).  codes:
// 16-bit scratch, K entries per path at codes + l cstride.  Path l is served
// by the G = 512/L threads l G .., lanes of one wave.
// ---------------------------------------------------------------------------
template <int L, int S>
__device__ __forceinline__ void fht_list(int tid, float *rows, uint16_t *codes, int cstride, const float *pm_in,
                                         float *out_pm, uint8_t *out_anc, uint16_t *out_code, uint32_t *xo)
{
    constexpr int n = 1 << S, K = cmin(L, n), G = kThreads / L;
    constexpr int E = (n + G - 1) / G; // elements per thread of the path's group
    constexpr int GA = G < n ? G : n;  // threads of the group that hold elements
    static_assert(G <= kWave && kWave % G == 0, "a path's threads are lanes of one wave");
    const int l = tid / G, lt = tid % G;
    float *F = rows + l * n;
    // Sum of |alpha|, halving tree: the levels of width >= G within each
    // thread (element lt + G e), the rest a lane butterfly.
    float v[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int i = lt + e * G;
        v[e] = i < n ? fabsf(F[i]) : 0.0f;
    }
#pragma unroll
    for (int wd = E / 2; wd >= 1; wd /= 2)
#pragma unroll
        for (int e = 0; e < wd; e++)
            v[e] = v[e] + v[e + wd];
    const float llr_abs = bfly_sum<GA / 2>(v[0]);
    wave_sync();
    // FHT, strides 2^{S-1} .. 1
    for (int t = 0; t < S; t++) {
        const int hh = 1 << (S - t - 1);
        for (int p = lt; p < n / 2; p += G) {
            const int i = (p / hh) * 2 * hh + (p % hh);
            const float x = F[i], z = F[i + hh];
            F[i] = z - x;
            F[i + hh] = z + x;
        }
        wave_sync();
    }
    // the path's elements in registers as keys: |F| bits, then the index
    // complemented (ties to the lower index), then the sign
    uint64_t key[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int i = lt + e * G;
        if (i < n) {
            const float x = F[i];
            key[e] = ((uint64_t)(__float_as_uint(x) & 0x7FFFFFFFu) << 32) | ((uint64_t)(0xFFFFu - i) << 1) |
                     (x < 0.0f ? 1u : 0u);
        } else {
            key[e] = 0;
        }
    }
    const float pml = pm_in[l];
    wave_sync();
    // K passes: the group's largest remaining key
    float *metric = F;                     // [K] per path, in the path's own row
    uint16_t *cidx = codes + l * cstride; // [K] index << 1 | sign
    // (keys are distinct and above 0, the padding, so exactly one lane holds
    // the group maximum and drops it by equality)
    for (int j = 0; j < K; j++) {
        double b = 0.0;
#pragma unroll
        for (int e = 0; e < E; e++)
            b = dmax(b, key_d(key[e]));
        const uint64_t gb = d_key(bfly_max<G / 2>(b));
#pragma unroll
        for (int e = 0; e < E; e++)
            key[e] = key[e] == gb ? 0ull : key[e];
        if (lt == 0) {
            const float absf = __uint_as_float((uint32_t)(gb >> 32));
            const uint32_t idx = 0xFFFFu - (uint32_t)((gb >> 1) & 0xFFFFu);
            metric[j] = pml + 0.5f * (llr_abs - absf);
            cidx[j] = (uint16_t)((idx << 1) | (uint32_t)(gb & 1u));
        }
    }
    __syncthreads();
    // merge: the L smallest of the L*K candidates in the order (metric, l, j)
    select_smallest<L, K>(tid, rows, n, codes, cstride, out_pm, out_anc, out_code);
    // the survivors' codewords: bit j = sign ^ parity(~(i | j))
    constexpr int W = words_of(S);
    for (int q = tid; q < L * W; q += kThreads) {
        const int ql = q / W, wd = q % W;
        const uint32_t code = (uint32_t)out_code[ql];
        const uint32_t idx = code >> 1, sg = code & 1u;
        uint32_t word = 0;
        for (int bt = 0; bt < cmin(32, n); bt++) {
            const uint32_t j = (uint32_t)(wd * 32 + bt);
            word |= (sg ^ ((uint32_t)__popc(~(idx | j) & (uint32_t)(n - 1)) & 1u)) << bt;
        }
        xo[q] = word;
    }
    __syncthreads();
}

// FHTL leaf RM(1,S) of the tree: its rows are level S, the level below is
// scratch
template <int M, int L, int S, int SIDE>
__device__ __forceinline__ void fhtl_leaf(const BigCtx<M, L> &c, const float *pm_in)
{
    static_assert(S < M, "leaf roots are decoded by rm_bigleaf_kernel");
    fht_list<L, S>(c.tid, c.a(S), (uint16_t *)c.a(S - 1), 1 << S, pm_in, c.pm(S, SIDE), c.anc(S, SIDE), c.sidx(),
                   c.xb(S, SIDE));
}

// The TAU split rounds of the SPC list rule (Eqs. (4), (5)), in wave 0.
// st: two copies of the list state, 5L words each (source path, parity,
// metric, then the 64-bit flip masks), the first holding the state before
// the rounds; ao + p * ostride: path p's |alpha| at o_0 .. o_TAU.  The state
// after the rounds is left in copy TAU & 1.
template <int L, int TAU>
__device__ __forceinline__ void spc_rounds(int tid, int *st, const float *ao, int ostride)
{
    auto SP = [&](int b) { return st + b * 5 * L; };
    auto CP = [&](int b) { return st + b * 5 * L + L; };
    auto CPM = [&](int b) { return (float *)(st + b * 5 * L + 2 * L); };
    auto FL = [&](int b) { return (uint64_t *)(st + b * 5 * L + 3 * L); };
    // Each round: the 2L candidates (keep 2q, flip 2q+1) as keys (metric
    // bits, enumeration position), sorted over the lanes; rank r < L becomes
    // list entry r.  Metrics are non-negative (the flip adds |alpha_{o_t}| >=
    // |alpha_{o_0}| before subtracting |alpha_{o_0}|), so their bit patterns
    // order as the values do.
    if (tid < kWave) {
        constexpr int NK = 2 * L;
        constexpr int NR = NK > kWave ? 2 : 1;
        const int lane = tid;
        int cur = 0;
        for (int t = 1; t <= TAU; t++) {
            if (t > 1) {
                // From the second split on, the list is in ascending metric
                // order.  Once every entry's flip scores strictly above every
                // entry's keep, this split leaves the list as it is, and so
                // does every later one (an entry's flip metric cannot
                // decrease with t while its state is unchanged): stop, with
                // the state in the copy the code after the rounds reads.
                float kv = -__builtin_inff(), fv = __builtin_inff();
                if (lane < L) {
                    const float *aos = ao + SP(cur)[lane] * ostride;
                    kv = CPM(cur)[lane];
                    fv = (kv + aos[t]) + (1.0f - 2.0f * (float)CP(cur)[lane]) * aos[0];
                }
                if (group_reduce<1, kWave, false>(fv) > group_reduce<1, kWave, true>(kv)) {
                    if (cur != (TAU & 1) && lane < L) {
                        SP(cur ^ 1)[lane] = SP(cur)[lane];
                        CP(cur ^ 1)[lane] = CP(cur)[lane];
                        CPM(cur ^ 1)[lane] = CPM(cur)[lane];
                        FL(cur ^ 1)[lane] = FL(cur)[lane];
                    }
                    wave_sync();
                    break;
                }
            }
            WaveKeys<NK> key;
            if (NK > kWave && t > 1) {
                // L = 64: after the first round the list is in metric order,
                // so the keep candidates (lane q: entry q, position 2q) are
                // already sorted.  Sort the L flips alone, then keep the L
                // smallest of the two sorted lists: the minimum of keep q and
                // flip L-1-q is a bitonic sequence holding them, which the
                // half-cleaners sort.
                const int q = lane;
                const int sp = SP(cur)[q];
                const float *aos = ao + sp * ostride;
                const float cpm = CPM(cur)[q];
                const float fv = (cpm + aos[t]) + (1.0f - 2.0f * (float)CP(cur)[q]) * aos[0];
                WaveKeys<kWave> fk, z;
                fk[0] = ((uint64_t)__float_as_uint(fv) << 32) | (uint32_t)(2 * q + 1);
                wave_sort<kWave>(fk, lane);
                const uint64_t kk = ((uint64_t)__float_as_uint(cpm) << 32) | (uint32_t)(2 * q);
                z[0] = d_key(dmin(key_d(kk), xor64<kWave - 1>(key_d(fk[0]))));
                wave_sort_run<kWave, kWave, kWave / 2>(z, lane);
                key[0] = z[0];
#pragma unroll
                for (int r = 1; r < NR; r++)
                    key[r] = kKeyPad; // ranks past L: not used
            } else {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    const int e = lane + kWave * r;
                    if (e < 2 * L) {
                        const int q = e >> 1, fl = e & 1;
                        const int sp = SP(cur)[q];
                        const float *aos = ao + sp * ostride;
                        const float v =
                            fl ? (CPM(cur)[q] + aos[t]) + (1.0f - 2.0f * (float)CP(cur)[q]) * aos[0] : CPM(cur)[q];
                        key[r] = ((uint64_t)__float_as_uint(v) << 32) | (uint32_t)e;
                    } else {
                        key[r] = ~0ull;
                    }
                }
                wave_sort<NK>(key, lane);
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
                const int rank = lane + kWave * r;
                if (rank < L) {
                    const int e = (int)(key[r] & 0xFFFFu), q = e >> 1, fl = e & 1;
                    SP(cur ^ 1)[rank] = SP(cur)[q];
                    CP(cur ^ 1)[rank] = CP(cur)[q] ^ fl;
                    CPM(cur ^ 1)[rank] = __uint_as_float((uint32_t)(key[r] >> 32));
                    FL(cur ^ 1)[rank] = FL(cur)[q] | ((uint64_t)fl << (t - 1));
                }
            }
            wave_sync();
            cur ^= 1;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// SPCL on a list (Eqs. (2)-(6)): L path rows of n = 2^S LLRs, path l's at
// rows + l n.  Hard decisions and parity (into hd, [L][words_of(S)] words,
// and par, [L] bytes), the TAU + 1 least reliable positions of every path
// (positions into ord + l ostride, 16-bit; |alpha| there over the first
// TAU + 1 entries of the row), the TAU split rounds (list state in st: two
// copies of 5L words at an even word offset), then the survivors' metrics,
// source paths and codewords into out_pm, out_anc and xo.
// ---------------------------------------------------------------------------
template <int L, int S>
__device__ __forceinline__ void spc_list(int tid, float *rows, uint32_t *hd, uint16_t *ord, int ostride, uint8_t *par,
                                         int *st, const float *pm_in, float *out_pm, uint8_t *out_anc, uint32_t *xo)
{
    constexpr int n = 1 << S, G = kThreads / L, W = words_of(S);
    constexpr int TAU = cmin(L, n - 1);
    constexpr int E = (n + G - 1) / G;
    static_assert(S >= 3 && TAU <= 64, "flip masks of 64 bits");
    const int l = tid / G, lt = tid % G;
    const float *al = rows + l * n;
    // hard decisions, Eq. (2)
    for (int q = tid; q < L * W; q += kThreads) {
        const int ql = q / W, wd = q % W;
        const float *row = rows + ql * n;
        uint32_t word = 0;
        for (int bt = 0; bt < cmin(32, n); bt++)
            word |= (row[wd * 32 + bt] < 0.0f ? 1u : 0u) << bt;
        hd[q] = word;
    }
    // least reliable positions: keys |alpha| bits, then the index (ties to the lower index)
    uint64_t key[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int i = lt + e * G;
        key[e] = i < n ? (((uint64_t)(__float_as_uint(al[i]) & 0x7FFFFFFFu) << 32) | (uint32_t)i) : kKeyPad;
    }
    __syncthreads();
    if (tid < L) {
        uint32_t p = 0;
        for (int wd = 0; wd < W; wd++)
            p ^= (uint32_t)__popc(hd[tid * W + wd]);
        par[tid] = (uint8_t)(p & 1u);
    }
    float *ao = rows + l * n;          // [TAU+1] |alpha| at o_t
    uint16_t *od = ord + l * ostride; // [TAU+1] o_t
    // (keys are distinct and below the padding, so exactly one lane holds
    // the group minimum and drops it by equality)
    for (int t = 0; t <= TAU; t++) {
        double b = key_d(kKeyPad);
#pragma unroll
        for (int e = 0; e < E; e++)
            b = dmin(b, key_d(key[e]));
        const uint64_t gb = d_key(bfly_min<G / 2>(b));
#pragma unroll
        for (int e = 0; e < E; e++)
            key[e] = key[e] == gb ? kKeyPad : key[e];
        if (lt == 0) {
            ao[t] = __uint_as_float((uint32_t)(gb >> 32));
            od[t] = (uint16_t)(gb & 0xFFFFu);
        }
    }
    __syncthreads();
    // list state: source path, parity, metric, flips (Eq. (3) for the start)
    auto SP = [&](int b) { return st + b * 5 * L; };
    auto CP = [&](int b) { return st + b * 5 * L + L; };
    auto CPM = [&](int b) { return (float *)(st + b * 5 * L + 2 * L); };
    auto FL = [&](int b) { return (uint64_t *)(st + b * 5 * L + 3 * L); };
    if (tid < L) {
        const int q = tid;
        const int p = par[q];
        SP(0)[q] = q;
        CP(0)[q] = p;
        const float a0 = rows[q * n];
        CPM(0)[q] = p ? pm_in[q] + a0 : pm_in[q];
        FL(0)[q] = 0;
    }
    __syncthreads();
    spc_rounds<L, TAU>(tid, st, rows, n);
    constexpr int cur = TAU & 1; // the state after the rounds
    // codewords: hard decisions with the kept flips, o_0 set by Eq. (6)
    for (int q = tid; q < L * W; q += kThreads) {
        const int ql = q / W, wd = q % W;
        const int sp = SP(cur)[ql];
        const uint64_t flips = FL(cur)[ql];
        const uint16_t *os = ord + sp * ostride;
        uint32_t word = hd[sp * W + wd];
        for (int t = 1; t <= TAU; t++)
            if ((flips >> (t - 1)) & 1u) {
                const uint32_t o = os[t];
                if ((int)(o >> 5) == wd)
                    word ^= 1u << (o & 31);
            }
        const uint32_t o0 = os[0];
        if ((int)(o0 >> 5) == wd) {
            const uint32_t hd0 = (hd[sp * W + wd] >> (o0 & 31)) & 1u;
            const uint32_t pr = ((uint32_t)par[sp] ^ (uint32_t)__popcll(flips) ^ hd0) & 1u;
            word = (word & ~(1u << (o0 & 31))) | (pr << (o0 & 31));
        }
        xo[q] = word;
    }
    if (tid < L) {
        out_pm[tid] = CPM(cur)[tid];
        out_anc[tid] = (uint8_t)SP(cur)[tid];
    }
    __syncthreads();
}

// SPCL leaf RM(S-1,S) of the tree: its rows are level S, the two levels
// below are scratch
template <int M, int L, int S, int SIDE>
__device__ __forceinline__ void spcl_leaf(const BigCtx<M, L> &c, const float *pm_in)
{
    using Ly = Lay<M, L>;
    static_assert(S < M && S >= 3, "SPC leaf inside the tree");
    static_assert(Ly::SPC_ONE == 5 * L && Ly::SPC % 2 == 0, "list state layout");
    spc_list<L, S>(c.tid, c.a(S), (uint32_t *)c.a(S - 2), (uint16_t *)c.a(S - 1), 1 << S, c.par(), c.i(Ly::SPC), pm_in,
                   c.pm(S, SIDE), c.anc(S, SIDE), c.xb(S, SIDE));
}

// ---------------------------------------------------------------------------
// internal node RM(R,S) (Alg. 2); V >= 0: depth on the leftmost spine
// ---------------------------------------------------------------------------
template <int M, int L, int R, int S, int V, int SIDE>
__device__ __forceinline__ void big_node(const BigCtx<M, L> &c, const float *pm_in);

// A copy of the context whose thread index the compiler cannot see through:
// the whole tree is inlined into the kernel, and without this the addresses
// and indices derived from the thread index would be computed once and held
// in registers across every node.
template <int M, int L>
__device__ __forceinline__ BigCtx<M, L> node_ctx(const BigCtx<M, L> &c)
{
    BigCtx<M, L> d = c;
    asm volatile("v_mov_b32 %0, %1" : "=v"(d.tid) : "v"(c.tid));
    return d;
}

template <int M, int L, int R, int S, int V, int SIDE>
__device__ __forceinline__ void big_child(const BigCtx<M, L> &c0, const float *pm_in)
{
    const BigCtx<M, L> c = node_ctx(c0);
    if constexpr (R == 1)
        fhtl_leaf<M, L, S, SIDE>(c, pm_in);
    else if constexpr (R == S - 1)
        spcl_leaf<M, L, S, SIDE>(c, pm_in);
    else
        big_node<M, L, R, S, V, SIDE>(c, pm_in);
}

template <int M, int L, int R, int S, int V, int SIDE>
__device__ __forceinline__ void big_node(const BigCtx<M, L> &c, const float *pm_in)
{
    using Ly = Lay<M, L>;
    constexpr int n = 1 << S, h = n / 2, G = Ly::G;
    static_assert(1 < R && R < S - 1, "internal node");
    const bool perm = V >= 0 && c.pfht;
    const int l = c.tid / G, lt = c.tid % G;
    float *ach = c.a(S - 1); // children's LLRs: L rows of h
    constexpr int VP = V >= 0 ? V : 0; // the node's slot among the spine's permutation nodes
    static_assert(VP < Ly::NPM, "permutation domain deeper than the layout holds");
    uint8_t *sel = c.sel(VP);
    uint8_t *orig = c.orig(VP);
    const float *pmL_in = pm_in;
    if (perm) {
        // LM of the 2L candidates: sum of |f| over the pairs that candidate
        // cc's map combines in path cc mod L's LLRs (y at the root, through
        // the composed maps).  An affine map's pairs {p(i), p(i + h)} are the
        // cosets {u, u ^ d} of its column d = p(h) ^ p(0); they are summed in
        // ascending order of u (i with a 0 put in at bit msb(d)) by the
        // halving tree over i, whose first level is taken here
        constexpr int GH = G / 2;
        const int cc = c.tid / GH, ct = c.tid % GH, src = cc % L;
        const uint32_t d = c.map(2 * L + 4 * L * VP + cc)[S - 1] >> 2;
        const uint32_t hi = 0u - (1u << (31 - __builtin_clz(d)));
        float *scr = ach + cc * (h / 2);
        constexpr int NIT = (h / 2 + GH - 1) / GH;
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int i = ct + GH * it;
            if (i < h / 2) {
                const uint32_t i0 = (uint32_t)i, i1 = (uint32_t)(i + h / 2);
                const uint32_t u0 = i0 + (i0 & hi), u1 = i1 + (i1 & hi);
                const float v0 = fabsf(big_fminsum(in_llr<M, L, S>(c, src, u0), in_llr<M, L, S>(c, src, u0 ^ d)));
                const float v1 = fabsf(big_fminsum(in_llr<M, L, S>(c, src, u1), in_llr<M, L, S>(c, src, u1 ^ d)));
                scr[i] = v0 + v1;
            }
        }
        wave_sync(); // a candidate's GH threads are lanes of one wave
        for (int wdt = h / 4; wdt >= 1; wdt /= 2) {
            for (int i = ct; i < wdt; i += GH)
                scr[i] = scr[i] + scr[i + wdt];
            wave_sync();
        }
        float *lm = c.f(Ly::SCR);
        if (ct == 0)
            lm[cc] = scr[0];
        __syncthreads();
        if (c.tid < 2 * L) {
            const float v = lm[c.tid];
            int rank = 0;
            for (int o = 0; o < 2 * L; o++) {
                const float u = lm[o];
                rank += (u > v || (u == v && o < c.tid)) ? 1 : 0;
            }
            sel[rank] = (uint8_t)c.tid;
        }
        __syncthreads();
        if (c.tid < L) {
            orig[c.tid] = (uint8_t)(sel[c.tid] % L);
            c.ppm(VP)[c.tid] = pm_in[sel[c.tid] % L];
        }
        __syncthreads();
        pmL_in = c.ppm(VP);
    }
    // f for the left child
    if constexpr (V >= 0) {
        // the permutation domain: the node's map, or the identity without
        // permutations, walked in Gray-code order
        MapR<S> mp;
        int src = l;
        if (perm) {
            load_map<S>(c.map(2 * L + 4 * L * VP + sel[l]), mp);
            src = orig[l];
        } else {
            identity_map<S>(mp);
        }
        constexpr int NIT = (h + G - 1) / G, LG = ilog2(G);
        uint32_t p = apply_map<S>(mp, (uint32_t)lt);
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            if (it > 0)
                p ^= mp.col[LG + __builtin_ctz(it)];
            const int i = lt + G * (it ^ (it >> 1));
            if (i < h)
                ach[l * h + i] = big_fminsum(in_llr<M, L, S>(c, src, p), in_llr<M, L, S>(c, src, p ^ mp.col[S - 1]));
        }
    } else {
        for (int i = lt; i < h; i += G)
            ach[l * h + i] = big_fminsum(in_llr<M, L, S>(c, l, (uint32_t)i), in_llr<M, L, S>(c, l, (uint32_t)(i + h)));
    }
    __syncthreads();
    big_child<M, L, R - 1, S - 1, (V >= 0 ? V + 1 : -1), 0>(c, pmL_in);
    // g for the right child, from the surviving ancestor's LLRs
    {
        const int k = c.anc(S - 1, 0)[l];
        const uint32_t *xl = c.xb(S - 1, 0);
        if constexpr (V >= 0) {
            MapR<S> mp;
            int src = k;
            if (perm) {
                load_map<S>(c.map(2 * L + 4 * L * VP + sel[k]), mp);
                src = orig[k];
            } else {
                identity_map<S>(mp);
            }
            constexpr int NIT = (h + G - 1) / G, LG = ilog2(G);
            uint32_t p = apply_map<S>(mp, (uint32_t)lt);
#pragma unroll
            for (int it = 0; it < NIT; it++) {
                if (it > 0)
                    p ^= mp.col[LG + __builtin_ctz(it)];
                const int i = lt + G * (it ^ (it >> 1));
                if (i < h)
                    ach[l * h + i] = big_g(in_llr<M, L, S>(c, src, p), in_llr<M, L, S>(c, src, p ^ mp.col[S - 1]),
                                           get_bit<S - 1>(xl, l, (uint32_t)i));
            }
        } else {
            for (int i = lt; i < h; i += G)
                ach[l * h + i] = big_g(in_llr<M, L, S>(c, k, (uint32_t)i), in_llr<M, L, S>(c, k, (uint32_t)(i + h)),
                                       get_bit<S - 1>(xl, l, (uint32_t)i));
        }
    }
    __syncthreads();
    big_child<M, L, R, S - 1, -1, 1>(c, c.pm(S - 1, 0));
    // combine (x_R ^ x_L, x_R), back through the node's permutation
    {
        const uint32_t *xl = c.xb(S - 1, 0);
        const uint32_t *xr = c.xb(S - 1, 1);
        uint32_t *xo = c.xb(S, SIDE);
        constexpr int W = words_of(S);
        for (int q = c.tid; q < L * W; q += kThreads) {
            const int ql = q / W, wd = q % W;
            const int k = c.anc(S - 1, 1)[ql];
            const int a = c.anc(S - 1, 0)[k];
            uint32_t word = 0;
            if (perm) {
                MapR<S> inv;
                load_map<S>(c.map(2 * L + 4 * L * VP + 2 * L + sel[a]), inv);
                constexpr int NB = cmin(32, n);
                uint32_t j = apply_map<S>(inv, (uint32_t)(wd * 32)); // Gray-code walk over the word's bits
#pragma unroll
                for (int it = 0; it < NB; it++) {
                    if (it > 0)
                        j ^= inv.col[__builtin_ctz(it)];
                    const uint32_t bit = j < (uint32_t)h ? (get_bit<S - 1>(xr, ql, j) ^ get_bit<S - 1>(xl, k, j))
                                                         : get_bit<S - 1>(xr, ql, j - h);
                    word |= bit << (it ^ (it >> 1));
                }
            } else if constexpr (S - 1 >= 5) {
                // whole words: the first half x_R ^ x_L, the second x_R
                constexpr int WC = words_of(S - 1);
                word = wd < WC ? (xr[ql * WC + wd] ^ xl[k * WC + wd]) : xr[ql * WC + wd - WC];
            } else {
                // both children's h bits in one word each
                constexpr uint32_t HM = (1u << h) - 1u;
                const uint32_t wr = xr[ql] & HM;
                word = (wr ^ (xl[k] & HM)) | (wr << h);
            }
            xo[q] = word;
        }
        if (c.tid < L) {
            const int k = c.anc(S - 1, 1)[c.tid];
            const int a = c.anc(S - 1, 0)[k];
            c.anc(S, SIDE)[c.tid] = (uint8_t)(perm ? orig[a] : a);
            c.pm(S, SIDE)[c.tid] = c.pm(S - 1, 1)[c.tid];
        }
        __syncthreads();
    }
}

// a frame's codeword (N bits as words_of(M) words in LDS, one partial word
// below N = 32) to its N/8 output bytes
template <int N>
__device__ __forceinline__ void store_codeword(int tid, const uint32_t *x, uint8_t *out)
{
    if constexpr (N >= 32) {
        for (int i = tid; i < N / 32; i += kThreads)
            ((uint32_t *)out)[i] = x[i];
    } else {
        if (tid < N / 8)
            out[tid] = (uint8_t)(x[0] >> (8 * tid));
    }
}

// ---------------------------------------------------------------------------
// the kernel: one workgroup per frame (grid-stride), P decoders per frame
// ---------------------------------------------------------------------------
template <int M, int R, int L>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) rm_biglist_kernel(KernelArgs args)
{
    using Ly = Lay<M, L>;
    constexpr int N = 1 << M, W = words_of(M);
    extern __shared__ __align__(16) uint32_t big_smem[];
    BigCtx<M, L> c;
    c.w = big_smem;
    c.tid = threadIdx.x;
    c.pfht = args.pfht;
    float *misc = c.f(Ly::MISC);
    for (int64_t f = blockIdx.x; f < args.n_frames; f += gridDim.x) {
        const uint32_t *fmaps = args.maps + f * args.frame_stride;
        for (int i = c.tid; i < N; i += kThreads)
            c.y()[i] = args.llr[f * N + i];
        if (c.tid == 0)
            misc[0] = __builtin_inff();
        for (int i = c.tid; i < W; i += kThreads)
            c.w[Ly::BEST + i] = 0u;
        __syncthreads();
        for (int d = 0; d < args.P; d++) {
            c.dmaps = fmaps + (size_t)d * args.maps_per_dec * kMapWords;
            if (c.tid < L)
                c.f(Ly::PM0)[c.tid] = (c.pfht || c.tid == 0) ? 0.0f : __builtin_inff();
            __syncthreads();
            big_node<M, L, R, M, 0, 0>(c, c.f(Ly::PM0));
            // Alg. 5: first minimum over the list; replace only if strictly smaller
            if (c.tid == 0) {
                const float *pm = c.pm(M, 0);
                int ls = 0;
                for (int q = 1; q < L; q++)
                    if (pm[q] < pm[ls])
                        ls = q;
                const int better = pm[ls] < misc[0];
                if (better)
                    misc[0] = pm[ls];
                c.i(Ly::MISC)[1] = better;
                c.i(Ly::MISC)[2] = ls;
            }
            __syncthreads();
            // The root's codewords are in channel order already: with
            // permutations the root's candidate maps include the initial
            // maps, and without them the initial maps are the identity.
            if (c.i(Ly::MISC)[1]) {
                const int ls = c.i(Ly::MISC)[2];
                const uint32_t *x = c.xb(M, 0);
                for (int wd = c.tid; wd < W; wd += kThreads)
                    c.w[Ly::BEST + wd] = x[ls * W + wd];
            }
            __syncthreads();
        }
        store_codeword<N>(c.tid, c.w + Ly::BEST, args.out_bits + f * (N / 8));
        if (c.tid == 0 && args.out_pm)
            args.out_pm[f] = misc[0];
        __syncthreads();
    }
}

// host side: launch (one workgroup per frame) and registry entry
template <int M, int R, int L>
hipError_t launch_big(const KernelArgs &args, int blocks, hipStream_t stream)
{
    constexpr size_t lds = Lay<M, L>::BYTES;
    static const hipError_t attr = hipFuncSetAttribute((const void *)&rm_biglist_kernel<M, R, L>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((rm_biglist_kernel<M, R, L>), dim3(blocks), dim3(kThreads), lds, stream, args);
    return hipGetLastError();
}

template <int M, int R, int L>
constexpr KernelEntry big_entry()
{
    return KernelEntry{M, R, L, 1, 0, 2 * L + 4 * L * perm_spine(M, R), &launch_big<M, R, L>, Lay<M, L>::BYTES};
}

// ---------------------------------------------------------------------------
// Leaf roots: the code is itself RM(1, m) (FHTL) or RM(m-1, m) (SPCL).  Alg. 2
// starts the L paths from the channel LLRs through the decoder's L initial
// maps (y itself for every path without permutations, one path active); the
// leaf's list rule runs on their rows, and the survivor Alg. 5 keeps goes
// back to channel order through the inverse of its path's initial map.
// LDS in 32-bit words: the paths' rows and small per-path arrays, no levels
// below (L N + N + O(L N / 32) words: 134 KB at L = 32, N = 1024).
// ---------------------------------------------------------------------------
template <int M, int L>
struct LeafLay {
    static constexpr int N = 1 << M;
    static constexpr int W = words_of(M);   // codeword words per path
    static constexpr int K = cmin(L, N);    // FHT candidates per path
    static constexpr int TAU = cmin(L, N - 1); // SPC splits
    static constexpr int OW = ((K > TAU + 1 ? K : TAU + 1) + 1) / 2; // words per path of 16-bit codes
    static constexpr int Y = 0;             // N floats: the channel LLRs
    static constexpr int ROW = N;           // [L][N] floats: the paths' rows
    static constexpr int HD = ROW + L * N;  // [L][W] SPC hard decisions
    static constexpr int ORD = HD + L * W;  // [L][OW] FHT (index, sign) codes or SPC positions, 16-bit
    static constexpr int XB = ORD + L * OW; // [L][W] the survivors' codewords
    static constexpr int PMO = XB + L * W;  // [L] floats: their metrics
    static constexpr int ANC = PMO + L;     // [L] bytes: their source paths
    static constexpr int SIDX = ANC + L / 4; // [L] 16-bit: FHT survivors' codes
    static constexpr int PAR = SIDX + L / 2; // [L] bytes: SPC parities
    static constexpr int PM0 = PAR + L / 4;  // [L] floats: the paths' input metrics
    static constexpr int SPC = (PM0 + L + 1) & ~1; // SPC list state: two copies of 5L words
    static constexpr int BEST = SPC + 10 * L; // [W] the frame's best codeword
    static constexpr int MISC = BEST + W;     // best metric, improved flag, winner
    static constexpr int WORDS = MISC + 4;
    static constexpr int BYTES = WORDS * 4;
    static constexpr bool layout_ok()
    {
        return L % 4 == 0 && L <= kWave && kThreads / L <= kWave && 2 * OW >= K && 2 * OW >= TAU + 1 &&
               TAU <= 64 && SPC % 2 == 0 && SPC >= PM0 + L && BEST >= SPC + 10 * L;
    }
};

// Waves per SIMD the registers must allow: four (two workgroups per CU)
// where the LDS allows it; two where one workgroup fills a CU's LDS, which
// leaves room for 64 register-held keys per thread (L = 32 at N = 1024).
template <int M, int L>
constexpr int leaf_wpe()
{
    return 2 * LeafLay<M, L>::BYTES <= 160 * 1024 ? 4 : 2;
}

template <int M, int R, int L, int WPE>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WPE))) rm_bigleaf_kernel(KernelArgs args)
{
    using Ly = LeafLay<M, L>;
    static_assert(Ly::layout_ok(), "leaf-root LDS layout");
    static_assert(R == 1 || R == M - 1, "leaf roots only");
    constexpr int N = 1 << M, W = Ly::W, G = kThreads / L;
    extern __shared__ __align__(16) uint32_t big_smem[];
    uint32_t *w = big_smem;
    const int tid0 = threadIdx.x;
    float *y = (float *)(w + Ly::Y);
    float *row = (float *)(w + Ly::ROW);
    float *pm0 = (float *)(w + Ly::PM0);
    float *pmo = (float *)(w + Ly::PMO);
    uint8_t *anc = (uint8_t *)(w + Ly::ANC);
    float *misc = (float *)(w + Ly::MISC);
    int *imisc = (int *)(w + Ly::MISC);
    for (int64_t f = blockIdx.x; f < args.n_frames; f += gridDim.x) {
        const uint32_t *fmaps = args.maps + f * args.frame_stride;
        for (int i = tid0; i < N; i += kThreads)
            y[i] = args.llr[f * N + i];
        if (tid0 == 0)
            misc[0] = __builtin_inff();
        for (int i = tid0; i < W; i += kThreads)
            w[Ly::BEST + i] = 0u;
        __syncthreads();
        for (int d = 0; d < args.P; d++) {
            // the thread index through an opaque move per decoder: otherwise
            // the per-element constants derived from it are computed once and
            // held in registers (spilled) across the frame loop
            int tid;
            asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(tid0));
            const int l = tid / G, lt = tid % G;
            const uint32_t *dmaps = fmaps + (size_t)d * args.maps_per_dec * kMapWords;
            if (tid < L)
                pm0[tid] = (args.pfht || tid == 0) ? 0.0f : __builtin_inff();
            // path l's row: y through its initial map (map l)
            {
                MapR<M> mp;
                if (args.pfht)
                    load_map<M>(dmaps + (size_t)l * kMapWords, mp);
                else
                    identity_map<M>(mp);
                for (int i = lt; i < N; i += G)
                    row[l * N + i] = y[apply_map<M>(mp, (uint32_t)i)];
            }
            __syncthreads();
            if constexpr (R == 1)
                fht_list<L, M>(tid, row, (uint16_t *)(w + Ly::ORD), 2 * Ly::OW, pm0, pmo, anc,
                               (uint16_t *)(w + Ly::SIDX), w + Ly::XB);
            else
                spc_list<L, M>(tid, row, w + Ly::HD, (uint16_t *)(w + Ly::ORD), 2 * Ly::OW, (uint8_t *)(w + Ly::PAR),
                               (int *)(w + Ly::SPC), pm0, pmo, anc, w + Ly::XB);
            // Alg. 5: first minimum over the list; replace only if strictly smaller
            if (tid == 0) {
                int ls = 0;
                for (int q = 1; q < L; q++)
                    if (pmo[q] < pmo[ls])
                        ls = q;
                const int better = pmo[ls] < misc[0];
                if (better)
                    misc[0] = pmo[ls];
                imisc[1] = better;
                imisc[2] = ls;
            }
            __syncthreads();
            if (imisc[1]) {
                // bit j in channel order is bit inv(j) of the survivor's
                // codeword, inv the inverse of its path's initial map (map
                // L + path); 64 bits per wave and pass, gathered by a ballot
                const int ls = imisc[2];
                MapR<M> inv;
                if (args.pfht)
                    load_map<M>(dmaps + (size_t)(L + anc[ls]) * kMapWords, inv);
                else
                    identity_map<M>(inv);
                const uint32_t *x = w + Ly::XB + ls * W;
                for (int j0 = 0; j0 < N; j0 += kThreads) {
                    const int j = j0 + tid;
                    uint32_t bit = 0;
                    if (j < N) {
                        const uint32_t s = apply_map<M>(inv, (uint32_t)j);
                        bit = (x[s >> 5] >> (s & 31)) & 1u;
                    }
                    const uint64_t mask = __ballot(bit);
                    const int base = j0 + (tid & ~(kWave - 1));
                    if ((tid & (kWave - 1)) == 0 && base < N) {
                        w[Ly::BEST + base / 32] = (uint32_t)mask;
                        if (base + 32 < N)
                            w[Ly::BEST + base / 32 + 1] = (uint32_t)(mask >> 32);
                    }
                }
            }
            __syncthreads();
        }
        store_codeword<N>(tid0, w + Ly::BEST, args.out_bits + f * (N / 8));
        if (tid0 == 0 && args.out_pm)
            args.out_pm[f] = misc[0];
        __syncthreads();
    }
}

template <int M, int R, int L>
hipError_t launch_bigleaf(const KernelArgs &args, int blocks, hipStream_t stream)
{
    constexpr size_t lds = LeafLay<M, L>::BYTES;
    constexpr int WPE = leaf_wpe<M, L>();
    static const hipError_t attr = hipFuncSetAttribute((const void *)&rm_bigleaf_kernel<M, R, L, WPE>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((rm_bigleaf_kernel<M, R, L, WPE>), dim3(blocks), dim3(kThreads), lds, stream, args);
    return hipGetLastError();
}

// a leaf root holds its decoder's L initial maps and their inverses
template <int M, int R, int L>
constexpr KernelEntry bigleaf_entry()
{
    return KernelEntry{M, R, L, 1, 0, 2 * L, &launch_bigleaf<M, R, L>, LeafLay<M, L>::BYTES};
}

} // namespace big
} // namespace rmdec
