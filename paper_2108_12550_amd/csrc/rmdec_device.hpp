// rmdec_device.hpp -- gfx950 device code of the batched p-FHT-FSCL-L-M decoder.
//
// One wavefront decodes one frame at a time: it runs the P decoders of the
// frame one after another (Alg. 5) and keeps the codeword with the smallest
// final metric.  Each decoder walks the Plotkin tree of RM(r,m) (Alg. 2),
// unrolled at compile time from (m, r, L).
//
// Row layout.  The L paths of the list occupy L groups of G = 64/L lanes.
// Element i of a path's node vector sits in lane (i mod G) of the path's
// group, register (i div G); a node of size n < G uses the first n lanes of
// each group.  Node LLRs, FHT values and codeword bits (one bit per register,
// packed in a mask per lane) stay in registers through the tree.  Moving a
// surviving path's data to its list slot is one ds_bpermute per register.
// LDS holds the frame's channel LLRs (read through the affine permutations),
// the decoder's maps and small per-node scratch.
//
// Every rounding operation follows the CPU oracle's order: halving-tree sums
// (v[i] += v[i+w], w = n/2..1; a lane butterfly gives every lane the same
// value), FHT butterflies with strides 2^{s-1}..1 computing (hi - lo, hi + lo),
// g = b -/+ a, and the metric updates left to right.  Build with
// -ffp-contract=off.  Ties are broken by enumeration order everywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rmdec {

constexpr int kWave = 64;

// Words per stored affine map: col[0..9] and b at [10] (both times 4: byte
// offsets of float elements), the dimension m at [11]; three 16-byte words.
constexpr int kMapWords = 12;
constexpr int kMapB = 10;

struct KernelArgs {
    const float *llr;
    uint8_t *out_bits;
    float *out_pm;
    const uint32_t *maps; // [P][maps_per_dec][kMapWords] (per frame when frame_stride > 0)
    int64_t n_frames;
    int64_t frame_stride; // words between frames' tables; 0: one table set for all frames
    int P;
    int maps_per_dec;
    int pfht; // 1: permutation domain on; 0: identity, no permutation domain
    int waves;
};

// ---------------------------------------------------------------------------
// lane primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Orders this wave's LDS traffic: every lane's earlier LDS writes are visible
// to every lane's later LDS reads, and no access moves across it.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    // all patterns used read lanes of the same row, so the bound control never applies
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// max/min of two doubles known to be ordinary (non-NaN) numbers; written as
// instructions so that no quieting of signalling NaNs is added around them
__device__ __forceinline__ double dmax(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmin(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// value held by lane (lane ^ W), W < 64
template <int W>
__device__ __forceinline__ uint32_t xor_lanes_u32(uint32_t v)
{
    if constexpr (W == 1)
        return dpp<0xB1>(v); // quad_perm [1,0,3,2]
    else if constexpr (W == 2)
        return dpp<0x4E>(v); // quad_perm [2,3,0,1]
    else if constexpr (W == 4)
        return dpp<0x1B>(dpp<0x141>(v)); // row_half_mirror (^7), then quad_perm [3,2,1,0] (^3)
    else if constexpr (W == 8)
        return dpp<0x128>(v); // row_ror:8
    else if constexpr (W == 16)
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F); // bit mode: xor 0x10
    else
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ W) << 2, (int)v);
}

// value held by lane (lane ^ W) for any W < 64: the bits of W below 8 are
// one or two DPP moves (row_half_mirror is lane ^ 7 within 8 lanes)
template <int Q>
__device__ __forceinline__ uint32_t xor_quad(uint32_t v)
{
    if constexpr (Q == 0)
        return v;
    else if constexpr (Q == 1)
        return dpp<0xB1>(v);
    else if constexpr (Q == 2)
        return dpp<0x4E>(v);
    else
        return dpp<0x1B>(v);
}
template <int W>
__device__ __forceinline__ uint32_t xor_any(uint32_t v)
{
    if constexpr (W >= 32)
        return xor_any<W - 32>(xor_lanes_u32<32>(v));
    else if constexpr (W >= 16)
        return xor_any<W - 16>(xor_lanes_u32<16>(v));
    else if constexpr (W >= 8)
        return xor_any<W - 8>(xor_lanes_u32<8>(v));
    else if constexpr (W >= 4)
        return xor_quad<W ^ 7>(dpp<0x141>(v));
    else
        return xor_quad<W>(v);
}

// 64-bit value held by lane (lane ^ W)
template <int W>
__device__ __forceinline__ double xor64(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t r = ((uint64_t)xor_any<W>((uint32_t)(u >> 32)) << 32) | xor_any<W>((uint32_t)u);
    return __longlong_as_double((long long)r);
}

template <int W>
__device__ __forceinline__ float xor_lanes(float v)
{
    return __uint_as_float(xor_lanes_u32<W>(__float_as_uint(v)));
}

template <int W>
__device__ __forceinline__ uint64_t xor_lanes(uint64_t v)
{
    const uint32_t lo = xor_lanes_u32<W>((uint32_t)v);
    const uint32_t hi = xor_lanes_u32<W>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int W>
__device__ __forceinline__ double xor_lanes(double v)
{
    return __longlong_as_double((long long)xor_lanes<W>((uint64_t)__double_as_longlong(v)));
}

// The wave's LDS: the dynamic shared segment.  Gathers address it by LDS
// byte address (an address-space-3 pointer made from the integer, so each
// read is one ds_read of the computed address with no base added).  These
// kernels declare no static LDS, so the segment starts at address 0 and the
// per-wave slices, multiples of 4N bytes from it, keep the alignment that
// lets map images be formed by XOR.
extern __shared__ __align__(16) unsigned char rm_smem[];
typedef __attribute__((address_space(3))) unsigned char lds_byte;
__device__ __forceinline__ uint32_t lds_addr(unsigned char *p) { return (uint32_t)(size_t)(lds_byte *)p; }
__device__ __forceinline__ float lds_f32(uint32_t byte_addr)
{
    return *(__attribute__((address_space(3))) const float *)(size_t)byte_addr;
}
__device__ __forceinline__ uint32_t lds_u32(uint32_t byte_addr)
{
    return *(__attribute__((address_space(3))) const uint32_t *)(size_t)byte_addr;
}

// min(|a|, |b|) for ordinary numbers, one instruction
__device__ __forceinline__ float min_abs(float a, float b)
{
    float r;
    asm("v_min_f32_e64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// value held by lane `src`
__device__ __forceinline__ uint32_t from_lane(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ float from_lane(float v, int src) { return __uint_as_float(from_lane(__float_as_uint(v), src)); }
__device__ __forceinline__ int from_lane(int v, int src) { return (int)from_lane((uint32_t)v, src); }
__device__ __forceinline__ uint64_t from_lane(uint64_t v, int src)
{
    return ((uint64_t)from_lane((uint32_t)(v >> 32), src) << 32) | from_lane((uint32_t)v, src);
}
__device__ __forceinline__ double from_lane(double v, int src)
{
    return __longlong_as_double((long long)from_lane((uint64_t)__double_as_longlong(v), src));
}

// forward permute: this lane's value goes to lane `dst` (destinations distinct)
__device__ __forceinline__ double to_lane(double v, int dst)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Partner distance for the level of an order-free butterfly (max, xor) that
// stands for distance W: within 8 lanes, XOR 7 is one DPP move (row half
// mirror) where XOR 4 takes two, and {7, 2, 1} spans the block like
// {4, 2, 1}.  Sums keep the distances of the canonical halving tree.
template <int W>
constexpr int span_xor() { return W == 4 ? 7 : W; }

// butterflies over aligned blocks of 2W lanes (W = 2^k or 0); every lane of
// a block ends with the same value
template <int W>
__device__ __forceinline__ float bfly_sum(float v)
{
    if constexpr (W >= 1)
        return bfly_sum<W / 2>(v + xor_lanes<W>(v));
    else
        return v;
}
template <int W>
__device__ __forceinline__ double bfly_max(double v)
{
    if constexpr (W >= 1)
        return bfly_max<W / 2>(dmax(v, xor64<span_xor<W>()>(v)));
    else
        return v;
}
template <int W>
__device__ __forceinline__ uint64_t bfly_umax(uint64_t v)
{
    if constexpr (W >= 1) {
        const uint64_t o = (uint64_t)__double_as_longlong(xor64<span_xor<W>()>(__longlong_as_double((long long)v)));
        return bfly_umax<W / 2>(o > v ? o : v);
    } else {
        return v;
    }
}
template <int W>
__device__ __forceinline__ uint32_t bfly_xor(uint32_t v)
{
    if constexpr (W >= 1)
        return bfly_xor<W / 2>(v ^ xor_any<span_xor<W>()>(v));
    else
        return v;
}

// ---------------------------------------------------------------------------
// check and bit node updates (Section II-B, min-sum)
// ---------------------------------------------------------------------------
// f(a,b) = sgn(a) sgn(b) min(|a|,|b|), computed as sgn(a) b clamped to
// [-|a|, |a|]; it differs from the textbook form only in the sign of a zero
// result, which no later step can observe.
__device__ __forceinline__ float f_minsum(float a, float b)
{
    const float sb = __uint_as_float(__float_as_uint(b) ^ (__float_as_uint(a) & 0x80000000u));
    return __builtin_amdgcn_fmed3f(sb, -fabsf(a), fabsf(a));
}

// g(a,b,c) = b + (1-2c) a, one rounding
__device__ __forceinline__ float g_func(float a, float b, uint32_t c)
{
    return b + __uint_as_float(__float_as_uint(a) ^ (c << 31));
}

// ---------------------------------------------------------------------------
// compile-time shapes
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

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

template <int n, int G>
struct Lay {
    static constexpr int RR = n >= G ? n / G : 1; // registers per lane
    static constexpr int ACT = n < G ? n : G;     // lanes of a group holding elements
    using Mask = std::conditional_t<(RR > 32), uint64_t, uint32_t>;
    static constexpr Mask FULL = RR >= 64 ? ~(Mask)0 : (Mask)(((uint64_t)1 << RR) - 1);
};

template <int M, int R, int L, int D>
struct Shape {
    static constexpr int N = 1 << M;
    static constexpr int G = kWave / (L * D); // lanes per path; D decoders of L paths per wave
    // the candidate merges hold one candidate per lane of a path's group
    static_assert(L <= G && 2 <= G, "at least max(L, 2) lanes per path");
    static constexpr int LG = ilog2(G);
    static constexpr int NPERM = perm_spine(M, R);
    static constexpr bool ROOT_LEAF = !(1 < R && R < M - 1);
    static constexpr int TAU = max_spc_tau(M, R, L);
    static constexpr int MAPS_PER_DEC = 2 * L + 4 * L * NPERM;

    // byte offsets of the per-wave LDS slice; per-decoder arrays are [D][...]
    // y at the slice start and the staging area (permutation nodes below the
    // root) right after it, both aligned to 4N bytes (slices are a multiple
    // of 4N) so that byte addresses of map images can be formed by XOR; the
    // decoders' maps last, so that a frame-packed slice that needs only the
    // first decoder's copy can end there
    static constexpr int O_Y = 0;
    static constexpr int STAGE_BYTES = NPERM >= 2 ? 4 * D * L * N / 2 : 0;
    static constexpr int O_STAGE = O_Y + 4 * N;
    static constexpr int O_SLOT = align16(O_STAGE + STAGE_BYTES); // survivors of a map selection
    static constexpr int O_SPCA = O_SLOT + 4 * D * L;             // SPC: |alpha| at o_t [D*L][TAU+1]
    static constexpr int O_SPCI = O_SPCA + 4 * D * L * (TAU + 1); // SPC: o_t [D*L][TAU+1]
    static constexpr int O_SPCP = O_SPCI + 4 * D * L * (TAU + 1); // SPC: parity | hd(o_0) << 1
    static constexpr int O_XBEST = align16(O_SPCP + 4 * D * L);   // winner's codeword masks, 2G words
    static constexpr int O_MAPS = align16(O_XBEST + 16 * G);      // [D][MAPS_PER_DEC][kMapWords]
    static constexpr int MAP_BYTES = 4 * kMapWords * MAPS_PER_DEC; // one decoder's maps
    static constexpr int BYTES = ((O_MAPS + MAP_BYTES * D + 4 * N - 1) / (4 * N)) * (4 * N);
};

// Per-wave context.  Lane = (decoder ds, path g, lane-in-group lg); the
// decoder's paths occupy groups gb .. gb+L-1 of the wave.
template <int M, int R, int L, int D>
struct Ctx {
    using S = Shape<M, R, L, D>;
    unsigned char *base;
    uint32_t yoff; // byte offset of this decoder's channel LLRs from O_Y (frame-packed kernels)
    uint32_t moff; // word offset of this decoder's maps from O_MAPS
    int lane, lg;
    int g;  // path within the decoder
    int gb; // first group of this lane's decoder
    int ds; // decoder within the wave
    int pfht;
    __device__ int lane_of(int path) const { return (gb + path) * S::G + lg; } // same element, other path
    __device__ int lead_of(int path) const { return (gb + path) * S::G; }      // first lane of a path
    __device__ float *y() const { return (float *)(base + S::O_Y + yoff); }
    __device__ uint32_t y_addr() const { return lds_addr(base) + S::O_Y + yoff; }
    __device__ uint32_t stage_addr() const { return lds_addr(base) + S::O_STAGE; }
    __device__ uint32_t *maps_all() const { return (uint32_t *)(base + S::O_MAPS); }
    __device__ uint32_t *maps() const { return maps_all() + moff; }
    __device__ float *stage() const { return (float *)(base + S::O_STAGE); }
    __device__ int *slot_all() const { return (int *)(base + S::O_SLOT); }
    __device__ int *slot() const { return slot_all() + ds * L; }
    __device__ float *spca() const { return (float *)(base + S::O_SPCA) + ds * L * (S::TAU + 1); }
    __device__ int *spci() const { return (int *)(base + S::O_SPCI) + ds * L * (S::TAU + 1); }
    __device__ uint32_t *spcp() const { return (uint32_t *)(base + S::O_SPCP) + ds * L; }
    __device__ uint64_t *xbest() const { return (uint64_t *)(base + S::O_XBEST); }
};

template <int n, int G>
struct NodeRes {
    typename Lay<n, G>::Mask x; // codeword bits of the path held by this group
    float pm;                   // its metric
    int anc;                    // input path it descends from
};

// Rank-based stable selection, for each of the D decoders of the wave, of
// the `keep` smallest of its `cnt` metrics in LDS (ties to the lower
// position): slot[t*keep + r] receives
// the position of its rank r (decoder t's metrics start at pm[t*STRIDE]).
// Those slots must already hold valid positions.
template <int cnt, int keep, int D, int STRIDE>
__device__ __forceinline__ void select_smallest(const float *pm, int *slot, int lane)
{
    if (lane < cnt * D) {
        const int seg = lane / cnt;
        const int me = lane - seg * cnt;
        const float *sp = pm + seg * STRIDE;
        const float my = sp[me];
        int rank = 0;
#pragma unroll
        for (int q = 0; q < cnt; q++) {
            const float o = sp[q];
            rank += (o < my) || (o == my && q < me);
        }
        if (rank < keep)
            slot[seg * keep + rank] = me;
    }
}

// Bitonic half-cleaners with strides S, S/2, ..., 1 over lanes: the lower
// lane of each pair keeps the smaller key.  Sorts a bitonic sequence held in
// 2S consecutive lanes.
template <int S>
__device__ __forceinline__ double bitonic_clean(double key, int lg)
{
    if constexpr (S == 0) {
        return key;
    } else {
        // keys are distinct: keep this lane's key if it is on the side the
        // lane wants (the smaller in the lower lane of the pair)
        const double o = xor64<S>(key);
        const bool keep = (key < o) != ((lg & S) != 0);
        return bitonic_clean<S / 2>(keep ? key : o, lg);
    }
}

// Merge of L sorted lists of K keys (list g in lanes g*G + t, t < K, keys
// ascending in t) into the K smallest, ascending, in the lanes of list 0.
// Level LV merges list g with list g ^ 2^LV: the first list against the
// second reversed gives the K smallest of both as a bitonic sequence, which
// the half-cleaners sort.  Keys must be distinct, so the order is total.
template <int LV, int L, int K, int G>
__device__ __forceinline__ double merge_lists(double key, int lg)
{
    if constexpr ((1 << LV) >= L) {
        return key;
    } else {
        const double o = xor64<(1 << LV) * G + (K - 1)>(key);
        return merge_lists<LV + 1, L, K, G>(bitonic_clean<K / 2>(dmin(key, o), lg), lg);
    }
}

// Bitonic sort, ascending, of 2^NB keys held one per lane: key k sits in
// lane (k >> 1) * G + (k & 1) relative to the decoder's first lane, so bit 0
// of k is a lane bit and bit d >= 1 is lane bit log2(G) + d - 1.
template <int NB, int G, int SZ, int ST>
__device__ __forceinline__ double bitonic_sort_step(double key, int k)
{
    constexpr int X = ST == 0 ? 1 : (G << (ST - 1));
    const double o = xor64<X>(key);
    const bool asc = SZ == NB || ((k >> SZ) & 1) == 0;
    const bool lower = ((k >> ST) & 1) == 0;
    // keys are distinct: keep this lane's key if it is on the side the lane wants
    const bool keep = (key < o) == (lower == asc);
    const double r = keep ? key : o;
    if constexpr (ST > 0)
        return bitonic_sort_step<NB, G, SZ, ST - 1>(r, k);
    else if constexpr (SZ < NB)
        return bitonic_sort_step<NB, G, SZ + 1, SZ>(r, k);
    else
        return r;
}
template <int NB, int G>
__device__ __forceinline__ double bitonic_sort(double key, int k)
{
    if constexpr (NB == 0)
        return key;
    else
        return bitonic_sort_step<NB, G, 1, 0>(key, k);
}

// Bitonic sort, ascending, of 2^NB keys held one per lane in consecutive
// lanes: key k in lane base + k (base a multiple of 16, so every partner
// k ^ ST, ST <= 8, is a DPP move within a row; lanes past the keys sort
// copies that nobody reads).
template <int NB, int SZ, int ST>
__device__ __forceinline__ double bitonic_rows_step(double key, int k)
{
    const double o = xor64<ST>(key);
    const bool asc = SZ == (1 << NB) || (k & SZ) == 0;
    const bool lower = (k & ST) == 0;
    // keys are distinct: keep this lane's key if it is on the side the lane wants
    const bool keep = (key < o) == (lower == asc);
    const double r = keep ? key : o;
    if constexpr (ST > 1)
        return bitonic_rows_step<NB, SZ, ST / 2>(r, k);
    else if constexpr (SZ < (1 << NB))
        return bitonic_rows_step<NB, SZ * 2, SZ>(r, k);
    else
        return r;
}

// Byte addresses of elements p(i), i = lg + G j (j < RR), of a vector at
// byte address `base` (aligned to the vector's size, so XOR acts as
// addition), under an affine map on F2^MD stored in LDS as byte-scaled
// columns and offset: the lane part first, then one XOR per register.
template <int MD, int G, int RR>
__device__ __forceinline__ void map_positions(const uint32_t *mp, int lg, uint32_t base, uint32_t (&pos)[RR])
{
    constexpr int LG = ilog2(G);
    uint32_t b = base ^ mp[kMapB];
#pragma unroll
    for (int k = 0; k < LG && k < MD; k++)
        b ^= ((lg >> k) & 1) ? mp[k] : 0u;
    pos[0] = b;
#pragma unroll
    for (int j = 1; j < RR; j++)
        pos[j] = pos[j & (j - 1)] ^ mp[LG + __builtin_ctz(j)];
}

// ---------------------------------------------------------------------------
// canonical halving-tree sum over a node vector in row layout
// ---------------------------------------------------------------------------
template <int n, int G, int RR>
__device__ __forceinline__ float tree_sum(float (&v)[RR])
{
#pragma unroll
    for (int w = n / 2; w >= G; w /= 2) {
#pragma unroll
        for (int j = 0; j < w / G; j++)
            v[j] = v[j] + v[j + w / G];
    }
    return bfly_sum<Lay<n, G>::ACT / 2>(v[0]);
}

// FHT butterflies (Alg. 4): stride h = 2^{s-1} .. 1, (lo, hi) <- (hi - lo, hi + lo)
// f = f + c * (f of the partner lane at XOR distance H), one v_fmac_f32
// with a DPP operand (H = 4: row_half_mirror, then quad_perm [3,2,1,0] on
// the mirrored copy, i.e. lane ^ 7 ^ 3).  NOP: start with two wait states
// (the source may have been written by the instruction just before).
#define RM_DPP_MASKS " row_mask:0xf bank_mask:0xf bound_ctrl:1"
template <int H, bool NOP>
__device__ __forceinline__ void fmac_dpp(float &f, float c)
{
    if constexpr (H == 1) {
        if constexpr (NOP)
            asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 quad_perm:[1,0,3,2]" RM_DPP_MASKS : "+v"(f) : "v"(c));
        else
            asm volatile("v_fmac_f32_dpp %0, %0, %1 quad_perm:[1,0,3,2]" RM_DPP_MASKS : "+v"(f) : "v"(c));
    } else if constexpr (H == 2) {
        if constexpr (NOP)
            asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 quad_perm:[2,3,0,1]" RM_DPP_MASKS : "+v"(f) : "v"(c));
        else
            asm volatile("v_fmac_f32_dpp %0, %0, %1 quad_perm:[2,3,0,1]" RM_DPP_MASKS : "+v"(f) : "v"(c));
    } else if constexpr (H == 8) {
        if constexpr (NOP)
            asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 row_ror:8" RM_DPP_MASKS : "+v"(f) : "v"(c));
        else
            asm volatile("v_fmac_f32_dpp %0, %0, %1 row_ror:8" RM_DPP_MASKS : "+v"(f) : "v"(c));
    } else {
        static_assert(H == 4, "one or two DPP moves");
        float t;
        asm volatile("s_nop 1\n\t"
                     "v_mov_b32_dpp %1, %0 row_half_mirror" RM_DPP_MASKS "\n\t"
                     "s_nop 1\n\t"
                     "v_fmac_f32_dpp %0, %1, %2 quad_perm:[3,2,1,0]" RM_DPP_MASKS
                     : "+v"(f), "=&v"(t)
                     : "v"(c));
    }
}
// two elements at H = 4, the second mirror move filling the first's wait state
template <bool NOP>
__device__ __forceinline__ void fmac_dpp_pair4(float &f0, float &f1, float c)
{
    float t0, t1;
    if constexpr (NOP)
        asm volatile("s_nop 1\n\t"
                     "v_mov_b32_dpp %2, %0 row_half_mirror" RM_DPP_MASKS "\n\t"
                     "v_mov_b32_dpp %3, %1 row_half_mirror" RM_DPP_MASKS "\n\t"
                     "s_nop 0\n\t"
                     "v_fmac_f32_dpp %0, %2, %4 quad_perm:[3,2,1,0]" RM_DPP_MASKS "\n\t"
                     "v_fmac_f32_dpp %1, %3, %4 quad_perm:[3,2,1,0]" RM_DPP_MASKS
                     : "+v"(f0), "+v"(f1), "=&v"(t0), "=&v"(t1)
                     : "v"(c));
    else
        asm volatile("v_mov_b32_dpp %2, %0 row_half_mirror" RM_DPP_MASKS "\n\t"
                     "v_mov_b32_dpp %3, %1 row_half_mirror" RM_DPP_MASKS "\n\t"
                     "s_nop 0\n\t"
                     "v_fmac_f32_dpp %0, %2, %4 quad_perm:[3,2,1,0]" RM_DPP_MASKS "\n\t"
                     "v_fmac_f32_dpp %1, %3, %4 quad_perm:[3,2,1,0]" RM_DPP_MASKS
                     : "+v"(f0), "+v"(f1), "=&v"(t0), "=&v"(t1)
                     : "v"(c));
}

template <int H, int G, int RR>
__device__ __forceinline__ void fht_stages(float (&F)[RR], int lg)
{
    if constexpr (H >= 1) {
        if constexpr (H >= G) {
            constexpr int hj = H / G;
#pragma unroll
            for (int j = 0; j < RR; j++)
                if ((j & hj) == 0) {
                    const float lo = F[j], hi = F[j + hj];
                    F[j] = hi - lo;
                    F[j + hj] = hi + lo;
                }
        } else if constexpr (H == 1 || H == 2 || H == 4 || H == 8) {
            // F = F + c * partner, one v_fmac_f32 with a DPP operand: c = +1
            // in the upper lane (hi + lo), -1 in the lower (lo - hi, the
            // difference negated; exact in magnitude, since the product by
            // +-1 is exact and the sum is rounded once).  The partners of a
            // stage always carry the same sign, so after the stages lane lg
            // holds F times (-1)^(number of zero bits of lg among the
            // cross-lane strides); fht_true_sign restores the sign of the
            // selected entries.  A DPP read must not follow the VALU write of
            // its source by fewer than two wait states.  In the first
            // cross-lane stage the sources were written by compiled code,
            // which may be scheduled right before the statement, so each
            // statement starts with an s_nop; later stages read values their
            // predecessor statement wrote at least two statements earlier
            // (the statements are volatile, hence in order), unless a lane
            // holds fewer than three elements.
            constexpr bool NOP = (H == G / 2) || RR < 3;
            const float cf = (lg & H) ? 1.0f : -1.0f;
            if constexpr (H == 4) {
#pragma unroll
                for (int j = 0; j + 1 < RR; j += 2)
                    fmac_dpp_pair4<NOP>(F[j], F[j + 1], cf);
                if constexpr (RR % 2 == 1)
                    fmac_dpp<4, true>(F[RR - 1], cf);
            } else {
#pragma unroll
                for (int j = 0; j < RR; j++)
                    fmac_dpp<H, NOP>(F[j], cf);
            }
        } else {
            // lower lane: partner - self = hi - lo; upper lane: partner + self = lo + hi
            const uint32_t neg = (lg & H) ? 0u : 0x80000000u;
#pragma unroll
            for (int j = 0; j < RR; j++) {
                const float p = xor_lanes<H>(F[j]);
                F[j] = p + __uint_as_float(__float_as_uint(F[j]) ^ neg);
            }
        }
        fht_stages<H / 2, G, RR>(F, lg);
    }
}

// Walsh mask: bit j (j < RR) = parity(c & j)
template <int RR, class MaskT>
__device__ __forceinline__ MaskT walsh_mask(uint32_t c)
{
    constexpr uint64_t pat[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                                 0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
    MaskT w = 0;
#pragma unroll
    for (int k = 0; k < ilog2(RR); k++)
        w ^= ((c >> k) & 1u) ? (MaskT)pat[k] : (MaskT)0;
    return w;
}

// FHT keys.  A key is a 64-bit pattern read as a double: the bits of F as
// its high word and, as its low word, an index code and the sign of F:
//   lo = ((KB - j) << (LG + 1)) | ((G - 1 - lg) << 1) | [F < 0]
// for element i = lg + G*j (KB = 1024/G), so that lo >> 1 = KI - i with
// KI = 1024 + G - 1.  Doubles of one sign order like their bit patterns, and
// the selection takes |key| (an abs modifier: sign of the high word cleared),
// so max(|key|) orders by |F| (larger first), then by the index (lower
// first).  A lane builds the part without its lane bits with one funnel
// shift; the lane bits are added once to its few retained keys.
__device__ __forceinline__ double fht_key_part(float f, uint32_t jcode)
{
    const uint32_t fb = __float_as_uint(f);
    const uint32_t lo = __builtin_amdgcn_alignbit(jcode, fb, 31u);
    return __longlong_as_double((long long)(((uint64_t)fb << 32) | lo));
}
template <int G>
__device__ __forceinline__ uint32_t fht_jcode(int j)
{
    return (uint32_t)((1024 / G - j) << ilog2(G));
}
__device__ __forceinline__ double key_or_lo(double k, uint32_t bits)
{
    return __longlong_as_double((long long)((uint64_t)__double_as_longlong(k) | bits));
}
// [F < 0] for a selected key (its low bit holds the sign bit of the stored
// F): F was stored times the sign of its lane lg (the cross-lane FHT stages
// of strides in XM, 1 to 8, leave lane lg negated once for every zero bit of
// lg among them); a zero F counts as not negative, as the comparison F < 0
// has it.
template <int G, uint32_t XM>
__device__ __forceinline__ uint32_t fht_true_sign(uint64_t kb)
{
    const uint32_t fb = (uint32_t)(kb >> 32);
    const uint32_t lgw = (uint32_t)(G - 1) - (((uint32_t)kb >> 1) & (uint32_t)(G - 1));
    const uint32_t sneg = (uint32_t)__popc(~lgw & XM) & 1u;
    return (fb & 0x7FFFFFFFu) ? (((uint32_t)kb & 1u) ^ sneg) : 0u;
}
// max/min of |a| and b (b non-negative)
__device__ __forceinline__ double dmax_abs(double b, double a)
{
    double r;
    asm("v_max_f64 %0, %1, |%2|" : "=v"(r) : "v"(b), "v"(a));
    return r;
}
__device__ __forceinline__ double dmin_abs(double b, double a)
{
    double r;
    asm("v_min_f64 %0, %1, |%2|" : "=v"(r) : "v"(b), "v"(a));
    return r;
}

// rank of key k among the n keys of lanes lg ^ W, W < n (larger first; keys
// are distinct)
template <int W, int n>
__device__ __forceinline__ void fht_rank(double k, int &rank)
{
    if constexpr (W < n) {
        rank += xor64<W>(k) > k;
        fht_rank<W + 1, n>(k, rank);
    }
}

// ---------------------------------------------------------------------------
// FHTL leaf RM(1,s): Alg. 3 over Alg. 4 with the metric of Eq. (10).
// A: this group's path LLRs (row layout), pm: its metric.
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D, int S>
__device__ __forceinline__ NodeRes<(1 << S), kWave / (L * D)> fhtl(const Ctx<M, R, L, D> &c,
                                                              float (&A)[Lay<(1 << S), kWave / (L * D)>::RR], float pm)
{
    constexpr int n = 1 << S;
    constexpr int G = kWave / (L * D);
    using Ly = Lay<n, G>;
    constexpr int RR = Ly::RR;
    constexpr int ACT = Ly::ACT;
    constexpr int K = L < n ? L : n;
    using MaskT = typename Ly::Mask;
    const int lg = c.lg;
    const bool valid = lg < ACT;

    float v[RR];
#pragma unroll
    for (int j = 0; j < RR; j++)
        v[j] = valid ? fabsf(A[j]) : 0.0f;
    const float sabs = tree_sum<n, G, RR>(v); // LLR_abs

    fht_stages<n / 2, G, RR>(A, lg);

    const uint32_t lanebits = (uint32_t)(G - 1 - lg) << 1;
    // cross-lane strides of this node's FHT done as v_fmac with a DPP operand
    constexpr uint32_t XM = (uint32_t)((G < n ? G : n) - 1) & 15u;
    float mypm;       // metric of this lane's candidate (Eq. (10))
    uint32_t myinf;   // its index code and sign
    int cand;         // its position t in the path's candidate order
    if constexpr (n <= G && K > 1) {
        // one element per lane: its rank among the node's n keys (larger
        // first) is its position; ranks below K are the candidates
        const double k = valid ? key_or_lo(fht_key_part(A[0], fht_jcode<G>(0)), lanebits) : 0.0;
        const double ka = fabs(k);
        int rank = 0;
        fht_rank<1, n>(ka, rank);
        cand = valid ? rank : lg;
        const uint64_t kb = (uint64_t)__double_as_longlong(k);
        mypm = pm + 0.5f * (sabs - fabsf(__uint_as_float((uint32_t)(kb >> 32))));
        myinf = ((uint32_t)kb & 0xFFEu) | fht_true_sign<G, XM>(kb);
    } else {
        // lane-local three largest keys (without lane bits: one lane, one lg)
        double b1 = 0.0, b2 = 0.0, b3 = 0.0;
#pragma unroll
        for (int j = 0; j < RR; j++) {
            const double k = valid ? fht_key_part(A[j], fht_jcode<G>(j)) : 0.0;
            const double x1 = dmin_abs(b1, k);
            b1 = dmax_abs(b1, k);
            const double x2 = dmin(b2, x1);
            b2 = dmax(b2, x1);
            b3 = dmax(b3, x2);
        }
        if (valid) {
            b1 = key_or_lo(b1, lanebits);
            b2 = key_or_lo(b2, lanebits);
            b3 = key_or_lo(b3, lanebits);
        }
        int left = 3; // keys of this lane known to be its largest below the last pop

        // K rounds: the group's largest remaining key is the next candidate;
        // lane t of the group keeps the key of round t
        double mykey = 0.0;
#pragma unroll
        for (int t = 0; t < K; t++) {
            const double w = bfly_max<ACT / 2>(b1);
            if (K == 1 || lg == t) // one round: every lane of the group holds the winner
                mykey = w;
            if (t + 1 < K) {
                // (b3 need not be cleared: once `left` reaches 0 the lane rescans)
                const bool own = valid && (b1 == w);
                if (own) {
                    b1 = b2;
                    b2 = b3;
                    left--;
                }
                const bool need = own && left == 0;
                if (__any(need)) {
                    // the owner used up its known keys: rescan below w
                    double n1 = 0.0, n2 = 0.0, n3 = 0.0;
#pragma unroll
                    for (int j = 0; j < RR; j++) {
                        double k = valid ? key_or_lo(fht_key_part(A[j], fht_jcode<G>(j)), lanebits) : 0.0;
                        k = fabs(k) < w ? k : 0.0;
                        const double x1 = dmin_abs(n1, k);
                        n1 = dmax_abs(n1, k);
                        const double x2 = dmin(n2, x1);
                        n2 = dmax(n2, x1);
                        n3 = dmax(n3, x2);
                    }
                    if (need) {
                        b1 = n1;
                        b2 = n2;
                        b3 = n3;
                        left = 3;
                    }
                }
            }
        }

        // the candidate's metric (Eq. (10)) and its index and sign
        const uint64_t kb = (uint64_t)__double_as_longlong(mykey);
        mypm = pm + 0.5f * (sabs - __uint_as_float((uint32_t)(kb >> 32)));
        myinf = ((uint32_t)kb & 0xFFEu) | fht_true_sign<G, XM>(kb);
        cand = lg;
    }

    // stable merge of the L*K candidates by metric, keep L (Alg. 3).  Each
    // path's K candidates are already in metric order (the metric does not
    // decrease as |F| decreases), so the lists are merged by a bitonic
    // network over lanes.  Merge key: the metric's bits (metrics are
    // non-negative, since |F| <= sum |alpha| holds in floating point: both
    // sums follow the same pairing tree) over (e = g*K + t, index, sign),
    // so ties go to the lower enumeration position e.
    static_assert(K == L, "list merge assumes min(L, 2^s) = L");
    int e;
    float opm;
    uint32_t inf;
    if constexpr (L == 1) {
        e = 0;
        opm = mypm;
        inf = myinf;
    } else {
        const uint32_t mlo = ((uint32_t)(c.g * K + cand) << 12) | myinf;
        double mk = __longlong_as_double((long long)(((uint64_t)__float_as_uint(mypm) << 32) | mlo));
        if constexpr (n <= G) // to lane t of the group for candidate t
            mk = to_lane(mk, c.lead_of(c.g) + cand);
        mk = merge_lists<0, L, K, G>(mk, lg);
        // survivor l sits in lane l of the decoder's first group
        const uint64_t sk = (uint64_t)__double_as_longlong(from_lane(mk, c.lead_of(0) + c.g));
        e = (int)((uint32_t)sk >> 12);
        opm = __uint_as_float((uint32_t)(sk >> 32));
        inf = (uint32_t)sk & 0xFFFu;
    }

    // codeword of transform index idx: x(z) = [F<0] ^ parity(cw) ^ parity(cw & z), cw = n-1-idx
    const uint32_t idx = (uint32_t)(1024 + G - 1) - (inf >> 1);
    const uint32_t cw = (uint32_t)(n - 1) - idx;
    const uint32_t b0 = (inf & 1u) ^ (__popc(cw) & 1u);
    const uint32_t lbit = b0 ^ (__popc(cw & (uint32_t)lg) & 1u);
    MaskT x;
    if constexpr (n >= G)
        x = (walsh_mask<RR, MaskT>(cw >> ilog2(G)) ^ (lbit ? ~(MaskT)0 : (MaskT)0)) & Ly::FULL;
    else
        x = (MaskT)lbit;
    return {x, opm, (int)((uint32_t)e / K)};
}

// maximum (MAX) or minimum of v over the lanes lane ^ w, w a multiple of W
// below E (W, E powers of two): over the path groups of a decoder for W = G,
// E = G L
template <int W, int E, bool MAX>
__device__ __forceinline__ float group_reduce(float v)
{
    if constexpr (W >= E) {
        return v;
    } else {
        const float o = xor_lanes<W>(v);
        return group_reduce<2 * W, E, MAX>(MAX ? fmaxf(v, o) : fminf(v, o));
    }
}

// rank of this lane's value among the n values of its group (smaller first,
// ties to the lower element index); partner element lg ^ w sits in lane ^ w
template <int W, int n>
__device__ __forceinline__ void spc_rank(uint32_t me, int lg, int &rank)
{
    if constexpr (W < n) {
        const uint32_t o = xor_any<W>(me);
        rank += (o < me) || (o == me && (lg ^ W) < lg);
        spc_rank<W + 1, n>(me, lg, rank);
    }
}

// ---------------------------------------------------------------------------
// SPCL leaf RM(s-1,s): Eqs. (2)-(6), tau = min(L, 2^s - 1) splits (0 if L = 1)
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D, int S>
__device__ __forceinline__ NodeRes<(1 << S), kWave / (L * D)> spcl(const Ctx<M, R, L, D> &c,
                                                              float (&A)[Lay<(1 << S), kWave / (L * D)>::RR], float pm)
{
    constexpr int n = 1 << S;
    constexpr int G = kWave / (L * D);
    using Ly = Lay<n, G>;
    constexpr int RR = Ly::RR;
    constexpr int ACT = Ly::ACT;
    constexpr int tau = spc_tau(L, n);
    constexpr int TS = Shape<M, R, L, D>::TAU + 1;
    using MaskT = typename Ly::Mask;
    const int lg = c.lg;
    const int g = c.g;
    const bool valid = lg < ACT;

    // hard decisions and parity (Eq. (2))
    MaskT hd = 0;
#pragma unroll
    for (int j = 0; j < RR; j++)
        hd |= (valid && A[j] < 0.0f) ? ((MaskT)1 << j) : (MaskT)0;
    const uint32_t par = bfly_xor<ACT / 2>((uint32_t)(__popcll((uint64_t)hd) & 1));

    if constexpr (tau == 0 && n <= G) {
        // Wagner decoding (no splits): the least reliable position o_0 is the
        // group minimum of (|alpha|, index), one element per lane; its key
        // also carries the element's hard decision.  Metric Eq. (3); the
        // parity is restored at o_0 (Eq. (6)).
        const uint64_t key = valid ? (((uint64_t)__float_as_uint(fabsf(A[0])) << 32) | ((uint32_t)lg << 1) | (uint32_t)hd)
                                   : ~0ull;
        const uint64_t mn = ~bfly_umax<ACT / 2>(~key);
        const uint32_t o0 = ((uint32_t)mn >> 1) & 0xFFu;
        const float cur0 = par ? pm + __uint_as_float((uint32_t)(mn >> 32)) : pm;
        const MaskT x = (uint32_t)lg == o0 ? (MaskT)(par ^ ((uint32_t)mn & 1u)) : hd;
        return {x, cur0, g};
    }

    // o_0 .. o_tau: |alpha| ascending, ties to the lower index
    float *spca = c.spca();
    int *spci = c.spci();
    if constexpr (n <= G) {
        // one element per lane: its rank among the node's n elements
        const uint32_t me = __float_as_uint(fabsf(A[0]));
        int rank = 0;
        spc_rank<1, n>(me, lg, rank);
        if (valid && rank <= tau) {
            spca[g * TS + rank] = __uint_as_float(me);
            spci[g * TS + rank] = lg;
        }
    } else {
    uint64_t key[RR];
#pragma unroll
    for (int j = 0; j < RR; j++) {
        const uint32_t i = (uint32_t)(lg + G * j);
        key[j] = valid ? (((uint64_t)(0x7FFFFFFFu - __float_as_uint(fabsf(A[j]))) << 32) | (1024u - i)) : 0ull;
    }
#pragma unroll
    for (int t = 0; t <= tau; t++) {
        uint64_t b = key[0];
#pragma unroll
        for (int j = 1; j < RR; j++)
            b = key[j] > b ? key[j] : b;
        const uint64_t w = bfly_umax<ACT / 2>(b);
#pragma unroll
        for (int j = 0; j < RR; j++)
            key[j] = key[j] == w ? 0ull : key[j];
        if (lg == 0) {
            spca[g * TS + t] = __uint_as_float(0x7FFFFFFFu - (uint32_t)(w >> 32));
            spci[g * TS + t] = (int)(1024u - (uint32_t)w);
        }
    }
    }
    uint32_t *spcp = c.spcp();
    wave_sync();
    const int o0 = spci[g * TS];
    const float a0 = spca[g * TS];
    const uint32_t hd_o0 = (uint32_t)(from_lane((uint64_t)hd, c.lead_of(g) + (int)((uint32_t)o0 % G)) >> ((uint32_t)o0 / G)) & 1u;
    if (lg == 0)
        spcp[g] = par | (hd_o0 << 1);
    float cur = pm;
    if (par) // Eq. (3)
        cur = pm + a0;

    // state of the path held by this group
    int src = g;
    uint32_t flips = 0;
    uint32_t p = par;
    wave_sync();
#pragma unroll
    for (int t = 1; t <= tau; t++) {
        // (keep, flip o_t) for every path in list order, Eqs. (4) and (5):
        // candidate e = 2g + lg (lg < 2).  Stable selection of the L
        // smallest: bitonic sort of the 2L keys (metric bits over e, then
        // the candidate's state as payload; metrics are non-negative).
        const float at = spca[src * TS + t];
        const float as0 = spca[src * TS];
        const float fpm = (cur + at) + (p ? -as0 : as0);
        if (t >= 2) {
            // From the second split on, the list is in ascending (metric,
            // position) order.  Once every path's flip scores strictly above
            // every path's keep, this split leaves the list as it is, and so
            // does every later one: a path's flip metric cannot decrease with
            // t while its state is unchanged (|alpha| at o_t is
            // non-decreasing in t, and rounding is monotone).  The wave stops
            // when that holds for each of its decoders.
            const float kmax = group_reduce<G, G * L, true>(cur);
            const float fmin = group_reduce<G, G * L, false>(fpm);
            if (__builtin_amdgcn_ballot_w64(!(fmin > kmax)) == 0)
                break;
        }
        uint64_t sk;
        if constexpr (L >= 8) {
            static_assert((L * G) % 16 == 0, "the decoder's lanes start at a multiple of 16");
            // 2L >= 16 candidates: candidate e in lane base + e of the
            // decoder's lanes, where every exchange of the sort is a DPP move
            // (in the path groups' own lanes, the strides 4 and 8 of the
            // candidate index would be lane distances 16 and 32)
            const int kc = c.lane - c.lead_of(0);
            const int e = kc & (2 * L - 1);
            const int from = c.lead_of(e >> 1);
            const uint32_t stw = (flips << 8) | ((uint32_t)src << 1) | p;
            const float mc = from_lane(cur, from), mf = from_lane(fpm, from);
            const uint32_t sc = from_lane(stw, from);
            const uint32_t st = (e & 1) ? sc ^ ((1u << (t + 8)) | 1u) : sc;
            double key = __longlong_as_double(
                (long long)(((uint64_t)__float_as_uint((e & 1) ? mf : mc) << 32) | ((uint32_t)e << 24) | st));
            key = bitonic_rows_step<ilog2(2 * L), 2, 1>(key, kc);
            // this group's path takes rank g
            sk = (uint64_t)__double_as_longlong(from_lane(key, c.lead_of(0) + g));
        } else {
            const int e = 2 * g + (lg & 1);
            const uint32_t st = (lg & 1) ? ((flips | (1u << t)) << 8) | ((uint32_t)src << 1) | (p ^ 1u)
                                         : (flips << 8) | ((uint32_t)src << 1) | p;
            double key = __longlong_as_double(
                (long long)(((uint64_t)__float_as_uint((lg & 1) ? fpm : cur) << 32) | ((uint32_t)e << 24) | st));
            key = bitonic_sort<ilog2(2 * L), G>(key, e);
            // this group's path takes rank g
            sk = (uint64_t)__double_as_longlong(from_lane(key, c.lead_of(g >> 1) + (g & 1)));
        }
        cur = __uint_as_float((uint32_t)(sk >> 32));
        p = (uint32_t)sk & 1u;
        src = (int)(((uint32_t)sk >> 1) & 0x7Fu);
        flips = ((uint32_t)sk >> 8) & 0xFFFFu;
    }

    // codeword: hard decisions of the source path, the taken flips, then the
    // parity of o_0 (Eq. (6))
    MaskT x = (MaskT)from_lane((uint64_t)hd, c.lane_of(src));
    const uint32_t sp = spcp[src];
    const int so0 = spci[src * TS];
    const uint32_t fix = (sp & 1u) ^ (__popc(flips) & 1u) ^ ((sp >> 1) & 1u);
#pragma unroll
    for (int t = 1; t <= tau; t++) {
        const int pos = spci[src * TS + t];
        if (((flips >> t) & 1u) && (int)((uint32_t)pos % G) == lg)
            x ^= (MaskT)1 << ((uint32_t)pos / G);
    }
    if ((int)((uint32_t)so0 % G) == lg)
        x = (x & ~((MaskT)1 << ((uint32_t)so0 / G))) | ((MaskT)fix << ((uint32_t)so0 / G));
    wave_sync();
    return {x, cur, src};
}

// ---------------------------------------------------------------------------
// f and g steps in row layout: node of size n -> child of size n/2
// ---------------------------------------------------------------------------
template <int n, int G>
__device__ __forceinline__ void f_step(const float (&A)[Lay<n, G>::RR], float (&C)[Lay<n / 2, G>::RR])
{
    constexpr int RR = Lay<n, G>::RR;
    if constexpr (n / 2 >= G) {
#pragma unroll
        for (int j = 0; j < RR / 2; j++)
            C[j] = f_minsum(A[j], A[j + RR / 2]);
    } else {
        C[0] = f_minsum(A[0], xor_lanes<n / 2>(A[0]));
    }
}

template <int n, int G>
__device__ __forceinline__ void g_step(const float (&A)[Lay<n, G>::RR], typename Lay<n / 2, G>::Mask xl,
                                       float (&C)[Lay<n / 2, G>::RR])
{
    constexpr int RR = Lay<n, G>::RR;
    if constexpr (n / 2 >= G) {
#pragma unroll
        for (int j = 0; j < RR / 2; j++)
            C[j] = g_func(A[j], A[j + RR / 2], (uint32_t)(xl >> j) & 1u);
    } else {
        C[0] = g_func(A[0], xor_lanes<n / 2>(A[0]), (uint32_t)xl & 1u);
    }
}

// x_nu = (x_gamma ^ x_lambda, x_gamma)
template <int n, int G>
__device__ __forceinline__ typename Lay<n, G>::Mask combine(typename Lay<n / 2, G>::Mask xl,
                                                            typename Lay<n / 2, G>::Mask xr, int lg)
{
    using MaskT = typename Lay<n, G>::Mask;
    if constexpr (n / 2 >= G) {
        constexpr int H = Lay<n / 2, G>::RR;
        return (MaskT)(xl ^ xr) | ((MaskT)xr << H);
    } else {
        const uint32_t up = xor_lanes_u32<n / 2>((uint32_t)xr);
        return (MaskT)(lg < n / 2 ? ((uint32_t)(xl ^ xr) & 1u) : (up & 1u));
    }
}

// ---------------------------------------------------------------------------
// Permutation-domain selection at a node of size 2^MD (Alg. 2): candidate c
// reads path c mod L through map c; LM_c = sum of |f| over the pairs the
// map's f combines; the L largest survive (ties to the lower c).  src(path)
// is the LDS byte address of that path's node LLRs (y at the root, whose
// candidate maps are stored composed with the paths' initial maps).  Returns
// the candidate that becomes this group's path.
//
// An affine map's pairs {p(i), p(i + h)} are the cosets {u, u ^ d} of its
// column d = p(h) ^ p(0): the LM is summed over those cosets in ascending
// order of their smaller element u (u = i with a 0 put in at bit msb(d)),
// by the halving tree over i.  Read that way the pairs need no map: a path
// group's lanes read consecutive words of the node vector and the same
// words XOR d, with no bank conflicts among them.
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D, int MD, class Src>
__device__ __forceinline__ int perm_select(const Ctx<M, R, L, D> &c, const uint32_t *cand_maps, Src src)
{
    constexpr int n = 1 << MD;
    constexpr int h = n / 2;
    constexpr int G = kWave / (L * D);
    using Lh = Lay<h, G>;
    constexpr int RR = Lh::RR;
    const bool valid = c.lg < Lh::ACT;
    float lm[2];
#pragma unroll
    for (int pass = 0; pass < 2; pass++) {
        // d as a byte offset; element i = lg + G j of the sum list is u(i),
        // the positions at and above msb(d) moved up by one: byte address
        // x + (x & -top) for x = 4i, top = the byte value of msb(d)
        const uint32_t colh = cand_maps[(c.g + L * pass) * kMapWords + MD - 1];
        const uint32_t hi = 0u - (1u << (31 - __builtin_clz(colh)));
        const uint32_t x4 = valid ? 4u * (uint32_t)c.lg : 0u;
        const uint32_t b = src(c.g) + x4 + (x4 & hi);
        uint32_t pos[RR];
#pragma unroll
        for (int j = 0; j < RR; j++)
            pos[j] = b + (uint32_t)(4 * G * j) + ((uint32_t)(4 * G * j) & hi);
        float v[RR];
#pragma unroll
        for (int j = 0; j < RR; j++)
            v[j] = valid ? min_abs(lds_f32(pos[j]), lds_f32(pos[j] ^ colh)) : 0.0f;
        lm[pass] = tree_sum<h, G, RR>(v);
    }
    // rank of candidates g and g+L among all 2L (larger LM first, ties to lower index)
    int r0 = 0, r1 = 0;
#pragma unroll
    for (int q = 0; q < L; q++) {
        const float o0 = from_lane(lm[0], c.lead_of(q));
        const float o1 = from_lane(lm[1], c.lead_of(q));
        r0 += (o0 > lm[0]) || (o0 == lm[0] && q < c.g);
        r0 += (o1 > lm[0]);
        r1 += (o0 > lm[1]) || (o0 == lm[1]);
        r1 += (o1 > lm[1]) || (o1 == lm[1] && q < c.g);
    }
    int *slot = c.slot();
    if (c.lane < L * D)
        c.slot_all()[c.lane] = (int)((uint32_t)c.lane % L);
    wave_sync();
    if (c.lg == 0) {
        if (r0 < L)
            slot[r0] = c.g;
        if (r1 < L)
            slot[r1] = c.g + L;
    }
    wave_sync();
    const int sel = slot[c.g];
    wave_sync();
    return sel;
}

// ---------------------------------------------------------------------------
// Alg. 2 on a node RM(RN, MN) below the root; A holds this group's path LLRs.
// SPINE: reached from the root by left steps only, so an internal node is in
// the permutation domain.
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D, int MN, int RN, bool SPINE>
__device__ __forceinline__ NodeRes<(1 << MN), kWave / (L * D)> node(const Ctx<M, R, L, D> &c,
                                                               float (&A)[Lay<(1 << MN), kWave / (L * D)>::RR], float pm)
{
    constexpr int n = 1 << MN;
    constexpr int G = kWave / (L * D);
    using Ly = Lay<n, G>;
    constexpr int RR = Ly::RR;
    if constexpr (1 < RN && RN < MN - 1) {
        using Lc = Lay<n / 2, G>;
        int sel = 0;
        bool is_per = false;
        constexpr int v = M - MN;
        constexpr int mbase = 2 * L + 4 * L * v; // candidate maps of this spine node
        float *stage = c.stage();
        if constexpr (SPINE) {
            if (c.pfht) {
                is_per = true;
                if (c.lg < Ly::ACT) {
#pragma unroll
                    for (int j = 0; j < RR; j++)
                        stage[(c.gb + c.g) * n + c.lg + G * j] = A[j];
                }
                wave_sync();
                sel = perm_select<M, R, L, D, MN>(c, c.maps() + mbase * kMapWords,
                                                  [&](int path) { return c.stage_addr() + (uint32_t)((c.gb + path) * n * 4); });
                const int org = (int)((uint32_t)sel % L);
                uint32_t pos[RR];
                map_positions<MN, G, RR>(c.maps() + (mbase + sel) * kMapWords, c.lg,
                                         c.stage_addr() + (uint32_t)((c.gb + org) * n * 4), pos);
#pragma unroll
                for (int j = 0; j < RR; j++)
                    A[j] = lds_f32(pos[j]);
                pm = from_lane(pm, c.lead_of(org));
                wave_sync();
            }
        }
        float C[Lc::RR];
        f_step<n, G>(A, C);
        const auto rl = node<M, R, L, D, MN - 1, RN - 1, SPINE>(c, C, pm);
        float Aa[RR];
#pragma unroll
        for (int j = 0; j < RR; j++)
            Aa[j] = from_lane(A[j], c.lane_of(rl.anc));
        g_step<n, G>(Aa, rl.x, C);
        const auto rr = node<M, R, L, D, MN - 1, RN, false>(c, C, rl.pm);
        const auto xl = (typename Lc::Mask)from_lane((uint64_t)rl.x, c.lane_of(rr.anc));
        int anc = from_lane(rl.anc, c.lead_of(rr.anc));
        auto x = combine<n, G>(xl, rr.x, c.lg);
        if constexpr (SPINE) {
            if (is_per) {
                // back to the node's input order: x[p(i)] = x'[i], read as x[j] = x'[p^{-1}(j)]
                const int csel = from_lane(sel, c.lead_of(anc));
                uint32_t *sb = (uint32_t *)stage;
                if (c.lg < Ly::ACT) {
#pragma unroll
                    for (int j = 0; j < RR; j++)
                        sb[(c.gb + c.g) * n + c.lg + G * j] = (uint32_t)(x >> j) & 1u;
                }
                wave_sync();
                uint32_t pos[RR];
                map_positions<MN, G, RR>(c.maps() + (mbase + 2 * L + csel) * kMapWords, c.lg,
                                         c.stage_addr() + (uint32_t)((c.gb + c.g) * n * 4), pos);
                typename Ly::Mask y = 0;
#pragma unroll
                for (int j = 0; j < RR; j++)
                    y |= (typename Ly::Mask)(lds_u32(pos[j]) & 1u) << j;
                x = c.lg < Ly::ACT ? y : (typename Ly::Mask)0;
                anc = (int)((uint32_t)csel % L);
                wave_sync();
            }
        }
        return {x, rr.pm, anc};
    } else if constexpr (RN == 1) {
        return fhtl<M, R, L, D, MN>(c, A, pm);
    } else {
        static_assert(RN == MN - 1, "leaf must be RM(1,s) or RM(s-1,s)");
        return spcl<M, R, L, D, MN>(c, A, pm);
    }
}

// Result of one decoder at the root for the path held by this group.
template <int M, int R, int L, int D>
struct RootRes {
    uint64_t xlo, xhi; // codeword masks (internal root: first and second half)
    float pm;
    int invmap; // index of the inverse map back to channel order
};

// ---------------------------------------------------------------------------
// Alg. 2 at the root of one decoder: the L paths start from the channel LLRs
// through their initial maps; at an internal root in p-FHT mode the 2L
// candidates are composed maps (initial map of path c mod L, then candidate c).
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D>
__device__ __forceinline__ RootRes<M, R, L, D> decode_root(const Ctx<M, R, L, D> &c)
{
    using Sh = Shape<M, R, L, D>;
    constexpr int N = Sh::N;
    constexpr int G = Sh::G;
    const uint32_t *maps = c.maps();
    // Alg. 2 starts its L paths from L permutations; without permutations the
    // list starts from one path, the other entries inactive (infinite metric)
    const float pm0 = (c.pfht || c.g == 0) ? 0.0f : __builtin_inff();
    if constexpr (!Sh::ROOT_LEAF) {
        constexpr int h = N / 2;
        using Lc = Lay<h, G>;
        constexpr int RC = Lc::RR;
        int rmap = c.g;
        if (c.pfht)
            rmap = 2 * L + perm_select<M, R, L, D, M>(c, maps + 2 * L * kMapWords, [&](int) { return c.y_addr(); });
        float C[RC];
        {
            const uint32_t *mp = maps + rmap * kMapWords;
            uint32_t pos[RC];
            map_positions<M - 1, G, RC>(mp, c.lg, c.y_addr(), pos);
            const uint32_t colh = mp[M - 1];
#pragma unroll
            for (int j = 0; j < RC; j++)
                C[j] = f_minsum(lds_f32(pos[j]), lds_f32(pos[j] ^ colh));
        }
        const auto rl = node<M, R, L, D, M - 1, R - 1, true>(c, C, pm0);
        {
            const uint32_t *mp = maps + from_lane(rmap, c.lead_of(rl.anc)) * kMapWords;
            uint32_t pos[RC];
            map_positions<M - 1, G, RC>(mp, c.lg, c.y_addr(), pos);
            const uint32_t colh = mp[M - 1];
#pragma unroll
            for (int j = 0; j < RC; j++)
                C[j] = g_func(lds_f32(pos[j]), lds_f32(pos[j] ^ colh), (uint32_t)(rl.x >> j) & 1u);
        }
        const auto rr = node<M, R, L, D, M - 1, R, false>(c, C, rl.pm);
        const auto xl = (typename Lc::Mask)from_lane((uint64_t)rl.x, c.lane_of(rr.anc));
        const int anc = from_lane(rl.anc, c.lead_of(rr.anc));
        const int inv = from_lane(rmap, c.lead_of(anc)) + (c.pfht ? 2 * L : L);
        return {(uint64_t)(xl ^ rr.x), (uint64_t)rr.x, rr.pm, inv};
    } else {
        using Ly = Lay<N, G>;
        constexpr int RN = Ly::RR;
        float A[RN];
        {
            uint32_t pos[RN];
            map_positions<M, G, RN>(maps + c.g * kMapWords, c.lg, c.y_addr(), pos);
#pragma unroll
            for (int j = 0; j < RN; j++)
                A[j] = lds_f32(pos[j]);
        }
        NodeRes<N, G> res;
        if constexpr (R == 1)
            res = fhtl<M, R, L, D, M>(c, A, pm0);
        else
            res = spcl<M, R, L, D, M>(c, A, pm0);
        return {(uint64_t)res.x, 0ull, res.pm, L + res.anc};
    }
}

// ---------------------------------------------------------------------------
// One frame: the P decoders of Alg. 5, then the winner back in channel order.
// decode_decoders runs decoders [d_begin, d_end) of the frame whose N channel
// LLRs are at `src` and keeps, in decoder order, the first strictly smaller
// final metric (Alg. 5); the winner's codeword masks stay in the LDS slice.
// emit_codeword writes that codeword (N/8 bytes at `ob`) and the metric (to
// `opm`, if not null).  The calling wavefront owns the LDS slice at `slice`;
// `lane` is its lane id.  From `args` only the decoder set (maps, P, mode) is
// used.
// ---------------------------------------------------------------------------
struct FrameBest {
    float best;  // smallest final metric (+inf if no decoder ran)
    int bestmap; // index of the map that takes the winner back to channel order
};

template <int M, int R, int L, int D>
__device__ __forceinline__ Ctx<M, R, L, D> frame_ctx(const KernelArgs &args, unsigned char *slice, int lane)
{
    using Sh = Shape<M, R, L, D>;
    constexpr int G = Sh::G;
    Ctx<M, R, L, D> c;
    c.base = slice;
    c.yoff = 0;
    c.lane = lane;
    // lane is in [0, 64): unsigned division and remainder are shifts and masks
    const uint32_t ul = (uint32_t)lane, gw = ul / G;
    c.g = (int)(gw % L);
    c.gb = (int)(gw - gw % L);
    c.ds = (int)(gw / L);
    c.moff = (uint32_t)c.ds * (Sh::MAPS_PER_DEC * kMapWords);
    c.lg = (int)(ul % G);
    c.pfht = args.pfht;
    return c;
}

template <int M, int R, int L, int D>
__device__ __forceinline__ FrameBest decode_decoders(const KernelArgs &args, const uint32_t *maps, const float *src,
                                                     unsigned char *slice, int lane, int d_begin, int d_end)
{
    using Sh = Shape<M, R, L, D>;
    constexpr int N = Sh::N;
    constexpr int G = Sh::G;
    const Ctx<M, R, L, D> c = frame_ctx<M, R, L, D>(args, slice, lane);
    wave_sync();
    for (int i = c.lane; i < N; i += kWave)
        c.y()[i] = src[i];
    float best = __builtin_inff();
    int bestmap = 0;
    uint64_t *xb = c.xbest();
    if (c.lane < 2 * G)
        xb[c.lane] = 0ull;
    for (int d0 = d_begin; d0 < d_end; d0 += D) {
        // the maps of decoders d0 .. d0+D-1 (past d_end: a copy of the last, result unused)
        wave_sync();
#pragma unroll
        for (int t = 0; t < D; t++) {
            const int dd = d0 + t < d_end ? d0 + t : d_end - 1;
            // stored with columns and offset as byte offsets of float elements
            const uint4 *mg = (const uint4 *)(maps + (size_t)dd * args.maps_per_dec * kMapWords);
            uint4 *ml = (uint4 *)(c.maps_all() + t * Sh::MAPS_PER_DEC * kMapWords);
            for (int i = c.lane; i < args.maps_per_dec * (kMapWords / 4); i += kWave)
                ml[i] = mg[i];
        }
        wave_sync();
        // lane-derived constants recomputed per pass (an opaque copy of the
        // lane id), rather than hoisted to the frame and spilled
        int dlane;
        asm volatile("v_mov_b32 %0, %1" : "=v"(dlane) : "v"(lane));
        const RootRes<M, R, L, D> r = decode_root<M, R, L, D>(frame_ctx<M, R, L, D>(args, slice, dlane));
        // Alg. 5 in decoder order: first minimum over the list, replace only if strictly smaller
#pragma unroll
        for (int t = 0; t < D; t++) {
            if (d0 + t >= d_end)
                break;
            float pmin = from_lane(r.pm, (t * L) * G);
            int lstar = 0;
#pragma unroll
            for (int q = 1; q < L; q++) {
                const float o = from_lane(r.pm, (t * L + q) * G);
                if (o < pmin) {
                    pmin = o;
                    lstar = q;
                }
            }
            if (pmin < best) {
                best = pmin;
                bestmap = (d0 + t) * args.maps_per_dec + from_lane(r.invmap, (t * L + lstar) * G);
                if ((int)((uint32_t)c.lane / G) == t * L + lstar) {
                    xb[c.lg] = r.xlo;
                    xb[G + c.lg] = r.xhi;
                }
            }
        }
    }
    wave_sync();
    return {best, bestmap};
}

// Writes the codeword whose masks (row layout of the root, 2G words) are at
// xb, taken back to channel order by the map at mi, and the metric `best`.
template <int M, int R, int L, int D>
__device__ __forceinline__ void emit_masks(const uint32_t *mi, float best, const uint64_t *xb, uint8_t *ob, float *opm,
                                           int lane)
{
    using Sh = Shape<M, R, L, D>;
    constexpr int N = Sh::N;
    constexpr int G = Sh::G;
    // the winner back in channel order, packed
    uint32_t col[M + 1];
#pragma unroll
    for (int k = 0; k < M; k++)
        col[k] = mi[k] >> 2;
    col[M] = mi[kMapB] >> 2;
    // image of position j = j0 + lane: the lane's bits folded once, the bits
    // of j0 (a multiple of 64, known at compile time) per block
    uint32_t el = col[M];
#pragma unroll
    for (int k = 0; k < M && k < 6; k++)
        el ^= (((uint32_t)lane >> k) & 1u) ? col[k] : 0u;
#pragma unroll
    for (int j0 = 0; j0 < N; j0 += kWave) {
        const uint32_t j = (uint32_t)(j0 + lane);
        uint32_t eh = 0;
#pragma unroll
        for (int k = 6; k < M; k++)
            eh ^= ((j0 >> k) & 1) ? col[k] : 0u;
        uint32_t e = el ^ eh;
        uint32_t bit = 0;
        if (j < (uint32_t)N) {
            e &= (uint32_t)(N - 1);
            if constexpr (!Sh::ROOT_LEAF) {
                constexpr uint32_t h = N / 2;
                const uint32_t ee = e < h ? e : e - h;
                const uint64_t w = xb[(e < h ? 0 : G) + (ee % G)];
                bit = (uint32_t)(w >> (ee / G)) & 1u;
            } else {
                bit = (uint32_t)(xb[e % G] >> (e / G)) & 1u;
            }
        }
        const uint64_t mask = __ballot(bit != 0);
        if constexpr (N >= kWave) {
            if (lane == 0)
                *(uint64_t *)(ob + j0 / 8) = mask;
        } else {
            if (lane < N / 8)
                ob[lane] = (uint8_t)(mask >> (8 * lane));
        }
    }
    if (opm && lane == 0)
        *opm = best;
}

template <int M, int R, int L, int D>
__device__ __forceinline__ void emit_codeword(const KernelArgs &args, const uint32_t *maps, FrameBest fb, uint8_t *ob,
                                              float *opm, unsigned char *slice, int lane)
{
    const Ctx<M, R, L, D> c = frame_ctx<M, R, L, D>(args, slice, lane);
    emit_masks<M, R, L, D>(maps + (size_t)fb.bestmap * kMapWords, fb.best, c.xbest(), ob, opm, lane);
    wave_sync();
}

template <int M, int R, int L, int D>
__device__ __forceinline__ void decode_frame(const KernelArgs &args, const uint32_t *maps, const float *src, uint8_t *ob,
                                             float *opm, unsigned char *slice, int lane)
{
    const FrameBest fb = decode_decoders<M, R, L, D>(args, maps, src, slice, lane, 0, args.P);
    emit_codeword<M, R, L, D>(args, maps, fb, ob, opm, slice, lane);
}

// frame f of a contiguous batch
template <int M, int R, int L, int D>
__device__ __forceinline__ void decode_batch_frame(const KernelArgs &args, int64_t f, unsigned char *slice, int lane)
{
    constexpr int N = 1 << M;
    decode_frame<M, R, L, D>(args, args.maps + f * args.frame_stride, args.llr + f * N, args.out_bits + f * (N / 8),
                             args.out_pm ? args.out_pm + f : nullptr, slice, lane);
}

// Workgroups are dealt round-robin over the 8 XCDs.  Numbered this way, the
// workgroups of one XCD take consecutive frames, whose codewords and metrics
// then fill 128-byte lines in one L2 instead of being written back in parts
// by several (a bijection on [0, nb) whatever the dispatch order).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    constexpr int64_t X = 8;
    const int64_t q = nb / X, r = nb % X, x = b % X, i = b / X;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---------------------------------------------------------------------------
// batched kernel: one wave per frame (grid-stride)
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) rm_decode_kernel(KernelArgs args)
{
    using Sh = Shape<M, R, L, D>;
    const int wave = (int)(threadIdx.x / kWave);
    const int64_t stride = (int64_t)gridDim.x * args.waves;
    for (int64_t f = xcd_block(blockIdx.x, gridDim.x) * args.waves + wave; f < args.n_frames; f += stride) {
        uint32_t tid; // opaque per frame: see rm_mixed_kernel
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(threadIdx.x));
        decode_batch_frame<M, R, L, D>(args, f, rm_smem + (tid / kWave) * Sh::BYTES, (int)(tid & (kWave - 1)));
    }
}

// ---------------------------------------------------------------------------
// Frame-packed kernel for one decoder per frame (P = 1): the D decoder slots
// of a wave decode D consecutive frames, one each, instead of one frame with
// D - 1 idle slots.  Slot 0 keeps the slice's own copy of y; the copies of
// slots 1 .. D-1 and the D winners' codeword masks follow the slice.
// ---------------------------------------------------------------------------
template <int M, int R, int L, int D>
struct Packed {
    using S = Shape<M, R, L, D>;
    static constexpr int N = S::N;
    static_assert(D > 1, "frame packing needs several decoder slots per wave");
    // After the standard slice's y, staging, small arrays and the maps of
    // one decoder (SHARED: every frame uses the same tables) or of all D
    // slots: the y of slots 1 .. D-1, 4N bytes each.  The D winners' masks
    // ([D][2G] words, written once the decoding has stopped reading y)
    // overlay those copies of y where they fit.
    static constexpr int yx(bool shared)
    {
        return ((S::O_MAPS + S::MAP_BYTES * (shared ? 1 : D) + 4 * N - 1) / (4 * N)) * (4 * N);
    }
    static constexpr int XB_BYTES = 16 * S::G * D;
    static constexpr int xb(bool shared)
    {
        return XB_BYTES <= 4 * N * (D - 1) ? yx(shared) : yx(shared) + 4 * N * (D - 1);
    }
    static constexpr int bytes(bool shared)
    {
        return ((xb(shared) + XB_BYTES > yx(shared) + 4 * N * (D - 1) ? xb(shared) + XB_BYTES
                                                                       : yx(shared) + 4 * N * (D - 1)) +
                4 * N - 1) /
               (4 * N) * (4 * N);
    }
    static constexpr int BYTES = bytes(false);        // maps per slot (fresh tables per frame)
    static constexpr int BYTES_SHARED = bytes(true);  // one copy of the maps
    __host__ __device__ static constexpr uint32_t yoff(uint32_t ds, bool shared)
    {
        return ds == 0 ? 0u : (uint32_t)yx(shared) + 4u * N * (ds - 1);
    }
};

// 8 x 8 bit transpose: bit 8b + l of the result is bit 8l + b of x
__device__ __forceinline__ uint64_t transpose8x8(uint64_t x)
{
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    return x ^ t ^ (t << 28);
}

// frames f0 .. f0+D-1 (those below n_frames) of a contiguous batch
template <int M, int R, int L, int D>
__device__ __forceinline__ void decode_packed(const KernelArgs &args, int64_t f0, unsigned char *slice, int lane)
{
    using Sh = Shape<M, R, L, D>;
    using Pk = Packed<M, R, L, D>;
    constexpr int N = Sh::N;
    constexpr int G = Sh::G;
    const int64_t left = args.n_frames - f0;
    const int nf = left < D ? (int)left : D;
    const bool shared = args.frame_stride == 0;
    wave_sync();
    // each slot's frame (16-byte moves; slots past the last frame repeat
    // frame f0 and their results are not written)
    constexpr int QF = N / 4; // 16-byte words per frame
#pragma unroll
    for (int q0 = 0; q0 < D * QF; q0 += kWave) {
        const int q = q0 + lane;
        if (D * QF % kWave == 0 || q < D * QF) {
            const int t = q / QF;
            const int64_t f = f0 + (t < nf ? t : 0);
            const uint4 v = ((const uint4 *)(args.llr + f * N))[q % QF];
            *(uint4 *)(slice + Sh::O_Y + Pk::yoff((uint32_t)t, shared) + 16 * (q % QF)) = v;
        }
    }
    // the decoder's maps: one copy shared by all slots when every frame
    // uses the same tables, else each slot's frame's own
    const int nmap = shared ? 1 : D;
    for (int t = 0; t < nmap; t++) {
        const uint4 *mg = (const uint4 *)(args.maps + (f0 + (t < nf ? t : 0)) * args.frame_stride);
        uint4 *ml = (uint4 *)(slice + Sh::O_MAPS) + t * Sh::MAPS_PER_DEC * (kMapWords / 4);
        for (int i = lane; i < args.maps_per_dec * (kMapWords / 4); i += kWave)
            ml[i] = mg[i];
    }
    wave_sync();
    int dlane; // opaque copy of the lane id, as in decode_decoders
    asm volatile("v_mov_b32 %0, %1" : "=v"(dlane) : "v"(lane));
    Ctx<M, R, L, D> c = frame_ctx<M, R, L, D>(args, slice, dlane);
    c.yoff = Pk::yoff((uint32_t)c.ds, shared);
    if (shared)
        c.moff = 0;
    const RootRes<M, R, L, D> r = decode_root<M, R, L, D>(c);
    // Alg. 5 with one decoder: the first minimum over the list; a frame
    // whose metrics are all +inf keeps the all-zero codeword
    float pmin = from_lane(r.pm, (c.ds * L) * G);
    int lstar = 0;
#pragma unroll
    for (int q = 1; q < L; q++) {
        const float o = from_lane(r.pm, (c.ds * L + q) * G);
        if (o < pmin) {
            pmin = o;
            lstar = q;
        }
    }
    const bool found = pmin < __builtin_inff();
    if constexpr (L == 1 && G == 8 && N >= 128) {
        if (!args.pfht) {
            // Plain mode: every map is the identity, so the codeword in
            // channel order is the root's row layout read out directly.
            // Element i of a half sits in lane i % 8 of the slot's group, bit
            // i / 8 of that lane's mask; a 64-bit output word gathers one byte
            // of each of the 8 lanes and transposes the 8 x 8 bits.
            constexpr int NH = Sh::ROOT_LEAF ? N : N / 2;
            const int64_t f = f0 + c.ds;
            const bool mine = c.lg == 0 && c.ds < nf;
#pragma unroll
            for (int h = 0; h < N / NH; h++) {
                const uint64_t mask = found ? (h == 0 ? r.xlo : r.xhi) : 0ull;
#pragma unroll
                for (int w = 0; w < NH / 64; w++) {
                    uint64_t v = ((mask >> (8 * w)) & 0xFFull) << (8 * c.lg);
                    v |= xor_lanes<1>(v);
                    v |= xor_lanes<2>(v);
                    v |= xor_lanes<4>(v);
                    v = transpose8x8(v);
                    if (mine)
                        *(uint64_t *)(args.out_bits + f * (N / 8) + (h * NH + 64 * w) / 8) = v;
                }
            }
            if (args.out_pm && mine)
                args.out_pm[f] = pmin;
            wave_sync();
            return;
        }
    }
    const int invmap = from_lane(r.invmap, (c.ds * L + lstar) * G);
    uint64_t *xb = (uint64_t *)(slice + Pk::xb(shared)) + c.ds * 2 * G;
    if (c.g == lstar) {
        xb[c.lg] = found ? r.xlo : 0ull;
        xb[G + c.lg] = found ? r.xhi : 0ull;
    }
    wave_sync();
    for (int t = 0; t < nf; t++) {
        const int64_t f = f0 + t;
        const int bm = __builtin_amdgcn_readlane(invmap, t * L * G);
        const float best = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pmin), t * L * G));
        // the winner's inverse map, from the slot's copy in LDS (a frame
        // without a finite metric has all-zero masks, which every map keeps all-zero)
        const uint32_t *mi = (const uint32_t *)(slice + Sh::O_MAPS) +
                             (shared ? 0 : t * Sh::MAPS_PER_DEC * kMapWords) + bm * kMapWords;
        emit_masks<M, R, L, D>(mi, best, (const uint64_t *)(slice + Pk::xb(shared)) + t * 2 * G,
                               args.out_bits + f * (N / 8), args.out_pm ? args.out_pm + f : nullptr, lane);
    }
    wave_sync();
}

template <int M, int R, int L, int D, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) rm_decode_packed_kernel(KernelArgs args)
{
    using Pk = Packed<M, R, L, D>;
    const int wave = (int)(threadIdx.x / kWave);
    const int64_t groups = (args.n_frames + D - 1) / D;
    const int64_t stride = (int64_t)gridDim.x * args.waves;
    const int sbytes = args.frame_stride == 0 ? Pk::BYTES_SHARED : Pk::BYTES;
    for (int64_t gi = xcd_block(blockIdx.x, gridDim.x) * args.waves + wave; gi < groups; gi += stride) {
        uint32_t tid; // opaque per frame group: see rm_mixed_kernel
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(threadIdx.x));
        decode_packed<M, R, L, D>(args, gi * D, rm_smem + (tid / kWave) * sbytes, (int)(tid & (kWave - 1)));
    }
}

// ---------------------------------------------------------------------------
// Fused mixed-code launch: a persistent grid drains a queue of tiles, each a
// run of frames of one segment (one code, one decoder set); the code of a
// segment selects which compiled decoder runs.
// ---------------------------------------------------------------------------
constexpr int kMaxSegments = 8;

struct Tile {
    uint32_t seg;   // segment index
    uint32_t first; // first frame of the run
    uint32_t count; // frames in the run
    uint32_t pad;
};

struct MixedArgs {
    KernelArgs seg[kMaxSegments]; // per segment: its frames, outputs and decoder tables
    int code[kMaxSegments];       // index of the segment's code in the kernel's code list
    const Tile *tiles;
    uint32_t n_tiles;
    uint32_t *head; // next tile to take; reset to 0 before every launch
    int waves;
};

template <int M_, int R_, int L_, int D_>
struct Code {
    static constexpr int M = M_, R = R_, L = L_, D = D_;
    using Sh = Shape<M_, R_, L_, D_>;
};

// LDS slice of one wave in the fused kernel: the largest footprint of the
// codes, rounded up to a multiple of the largest 4N, so that every code's
// slice base stays aligned to its own 4N (the XOR-folded gathers need it).
template <class... Codes>
struct MaxBytes {
    static constexpr int cmax(int a, int b) { return a > b ? a : b; }
    template <class... T>
    static constexpr int vmax(T... v)
    {
        int r = 0;
        ((r = cmax(r, v)), ...);
        return r;
    }
    static constexpr int align = vmax(4 * Codes::Sh::N...);
    static constexpr int value = (vmax(Codes::Sh::BYTES...) + align - 1) / align * align;
};

template <class C>
__device__ __forceinline__ void run_tile(const KernelArgs &a, const Tile &t, unsigned char *slice, int lane)
{
    for (uint32_t k = 0; k < t.count; k++)
        decode_batch_frame<C::M, C::R, C::L, C::D>(a, (int64_t)t.first + k, slice, lane);
}

template <int WPE, class... Codes>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) rm_mixed_kernel(MixedArgs a)
{
    while (true) {
        uint32_t t = 0;
        if (lane_id() == 0)
            t = atomicAdd(a.head, 1u);
        t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
        if (t >= a.n_tiles)
            break; // every wave ends once the queue is drained
        // The thread id is re-read through an opaque move on every tile, so
        // that values derived from it stay inside each code's branch instead
        // of being hoisted out of the loop, where those of all codes would
        // be live at once.
        uint32_t tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(threadIdx.x));
        const int lane = (int)(tid & (kWave - 1));
        unsigned char *slice = rm_smem + (tid / kWave) * MaxBytes<Codes...>::value;
        const Tile tile = a.tiles[t];
        const int code = a.code[tile.seg];
        const KernelArgs &ka = a.seg[tile.seg];
        int idx = 0;
        ((code == idx++ ? (run_tile<Codes>(ka, tile, slice, lane), 0) : 0), ...);
    }
}

} // namespace rmdec

namespace rmdec {

// ---------------------------------------------------------------------------
// Serving launch: like the fused kernel, but every frame is a separate
// request with its own input address and output slot, and the decoder sets
// of a step are a table in device memory.
// ---------------------------------------------------------------------------
struct Job {
    const float *llr; // the request's N channel LLRs (device)
    uint32_t out;     // output slot: bits at out * kServeBitsStride, metric at out
    uint32_t pad;
};

constexpr int kServeBitsStride = 128; // bytes per output slot (N/8 <= 128)

struct ServeArgs {
    const KernelArgs *segs; // per decoder set of the step: maps, P, mode (llr/out fields unused)
    const int *seg_code;    // index of each set's code in the kernel's code list
    const Tile *tiles;      // runs of jobs of one set: seg, first job, count
    const Job *jobs;
    uint32_t n_tiles;
    uint32_t *head; // next tile to take; zero when the step starts
    uint8_t *out_bits;
    float *out_pm;
    uint32_t *done; // per output slot: set to `epoch` once its codeword and metric are written
    uint32_t epoch;
};

// A request's outputs are complete: after the wave's writes to them (all by
// lane 0) are visible system-wide, its completion word takes the step's
// epoch, so that a host thread polling the word may read the outputs.
__device__ __forceinline__ void signal_done(const ServeArgs &a, uint32_t slot, int lane)
{
    if (lane == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __hip_atomic_store(a.done + slot, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <class C>
__device__ __forceinline__ void serve_tile(const ServeArgs &a, const KernelArgs &ka, const Tile &t, unsigned char *slice,
                                           int lane)
{
    static_assert(C::Sh::N >= kWave, "signal_done orders lane 0's writes: every output word must come from lane 0");
    for (uint32_t k = 0; k < t.count; k++) {
        const Job j = a.jobs[t.first + k];
        decode_frame<C::M, C::R, C::L, C::D>(ka, ka.maps, j.llr, a.out_bits + (size_t)j.out * kServeBitsStride, a.out_pm + j.out,
                                             slice, lane);
        signal_done(a, j.out, lane);
    }
}

template <int WPE, class... Codes>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) rm_serve_kernel(ServeArgs a)
{
    while (true) {
        uint32_t t = 0;
        if (lane_id() == 0)
            t = atomicAdd(a.head, 1u);
        t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
        if (t >= a.n_tiles)
            break; // every wave ends once the step's queue is drained
        uint32_t tid; // opaque per tile: see rm_mixed_kernel
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(threadIdx.x));
        const int lane = (int)(tid & (kWave - 1));
        unsigned char *slice = rm_smem + (tid / kWave) * MaxBytes<Codes...>::value;
        const Tile tile = a.tiles[t];
        const int code = a.seg_code[tile.seg];
        const KernelArgs ka = a.segs[tile.seg];
        int idx = 0;
        ((code == idx++ ? (serve_tile<Codes>(a, ka, tile, slice, lane), 0) : 0), ...);
    }
}

// Serving launch with a request's decoders split over the waves of a
// workgroup: the workgroup takes one queue entry at a time; for each request
// wave w runs decoders [P*w/W, P*(w+1)/W) (W waves), the waves exchange their
// best metrics through LDS, and the wave holding the first minimum in
// decoder order writes the codeword -- the result of Alg. 5 over all P, with
// the request's latency divided by about W.
// The workgroup's exchange area follows its W wave slices in the dynamic
// segment (kSplitXBytes more than W slices), since static LDS would move the
// slices off address 0.
constexpr int kSplitXBytes = 64;

template <int WPE, class... Codes>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) rm_serve_split_kernel(ServeArgs a)
{
    const int W = (int)(blockDim.x / kWave);
    unsigned char *xa = rm_smem + (size_t)W * MaxBytes<Codes...>::value;
    uint32_t &s_tile = *(uint32_t *)xa;
    float *s_best = (float *)(xa + 16); // [W], W <= 4
    int *s_map = (int *)(xa + 32);      // [W]
    while (true) {
        if (threadIdx.x == 0)
            s_tile = atomicAdd(a.head, 1u);
        __syncthreads();
        const uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_tile);
        if (t >= a.n_tiles)
            break; // the same entry for every wave: all leave together
        const Tile tile = a.tiles[t];
        const int code = a.seg_code[tile.seg];
        const KernelArgs ka = a.segs[tile.seg];
        for (uint32_t k = 0; k < tile.count; k++) {
            uint32_t tid; // opaque per request: see rm_mixed_kernel
            asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(threadIdx.x));
            const int lane = (int)(tid & (kWave - 1));
            const int w = (int)(tid / kWave);
            unsigned char *slice = rm_smem + w * MaxBytes<Codes...>::value;
            const int d_begin = ka.P * w / W, d_end = ka.P * (w + 1) / W;
            const Job j = a.jobs[tile.first + k];
            FrameBest fb = {__builtin_inff(), 0};
            int idx = 0;
            ((code == idx++ ? (fb = decode_decoders<Codes::M, Codes::R, Codes::L, Codes::D>(ka, ka.maps, j.llr, slice, lane,
                                                                                           d_begin, d_end),
                               0)
                            : 0),
             ...);
            if (lane == 0) {
                s_best[w] = fb.best;
                s_map[w] = fb.bestmap;
            }
            __syncthreads();
            int win = 0;
            for (int q = 1; q < W; q++)
                win = s_best[q] < s_best[win] ? q : win;
            if (w == win) {
                const FrameBest wb = {s_best[win], s_map[win]};
                idx = 0;
                ((code == idx++ ? (emit_codeword<Codes::M, Codes::R, Codes::L, Codes::D>(
                                       ka, ka.maps, wb, a.out_bits + (size_t)j.out * kServeBitsStride,
                                       a.out_pm + j.out, slice, lane),
                                   0)
                                : 0),
                 ...);
                signal_done(a, j.out, lane);
            }
            __syncthreads();
        }
    }
}

} // namespace rmdec
