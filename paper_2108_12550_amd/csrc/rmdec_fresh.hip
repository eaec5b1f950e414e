// rmdec_fresh.hip -- the fresh-permutation mode (RM_PERM_FRESH): every frame
// draws its own affine maps, so that each received vector is decoded with
// permutations sampled for it alone (the initialisation of Alg. 2 done per
// received vector).  A generation kernel writes the maps of a chunk of frames
// into a device buffer, in the layout of the fixed tables, and the batched
// kernel then reads frame f's tables at f times the per-frame stride.
#include <hip/hip_runtime.h>

#include <string>

#include "rmdec.h"
#include "rmdec_internal.hpp"

namespace rmdec {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kDim = 10; // largest map dimension (m <= 10)

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): Weyl step, then mix
__device__ __forceinline__ uint64_t smx_next(uint64_t &s)
{
    s += kGamma;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// An affine map over F2^md held by columns: col[k] = A e_k, and b.  Entries
// at and beyond md are zero, so every loop below runs over all kDim entries
// (fully unrolled, register resident) without changing the result.
struct CMap {
    uint32_t col[kDim];
    uint32_t b;
};

// bit matrix transpose: out[k] bit j = in[j] bit k
__device__ __forceinline__ void transpose(const uint32_t (&in)[kDim], uint32_t (&out)[kDim])
{
#pragma unroll
    for (int k = 0; k < kDim; k++) {
        uint32_t w = 0;
#pragma unroll
        for (int j = 0; j < kDim; j++)
            w |= ((in[j] >> k) & 1u) << j;
        out[k] = w;
    }
}

// A v for A given by columns: XOR of the columns at the set bits of v
__device__ __forceinline__ uint32_t apply(const uint32_t (&col)[kDim], uint32_t v)
{
    uint32_t y = 0;
#pragma unroll
    for (int k = 0; k < kDim; k++)
        y ^= ((v >> k) & 1u) ? col[k] : 0u;
    return y;
}

// one uniform element of AGL(md, 2) and its inverse, built row by row: row k
// of A (low md bits of one output) is redrawn until it lies outside the span
// of rows 0..k-1, then b.  Independence is tested by reducing the candidate
// against an XOR basis indexed by leading bit.  One loop trip per drawn
// candidate, whichever row it is for, so that the lanes of a wave diverge
// only by their total number of redraws.
//
// Each basis vector also records which rows it is the sum of (comb, a mask
// over row indices).  Once all md rows are in, reducing the basis to the
// identity (clearing bit h of every higher vector with vector h, in
// increasing h) leaves comb[h] = the rows that sum to e_h, i.e. row h of
// A^{-1} (C A = I for the matrix C of the comb rows).
__device__ __forceinline__ void draw_map(int md, uint64_t &st, CMap &a, CMap &ai)
{
    const uint32_t mask = (1u << md) - 1u;
    uint32_t row[kDim], basis[kDim], comb[kDim];
#pragma unroll
    for (int j = 0; j < kDim; j++) {
        row[j] = 0;
        basis[j] = 0;
        comb[j] = 0;
    }
    for (int k = 0; k < md;) {
        const uint32_t r = (uint32_t)(smx_next(st) & mask);
        uint32_t x = r, cx = 1u << k;
#pragma unroll
        for (int h = kDim - 1; h >= 0; h--) {
            const bool hit = (x >> h) & 1u;
            x ^= hit ? basis[h] : 0u;
            cx ^= hit ? comb[h] : 0u;
        }
        if (x) {
            const int lead = 31 - __builtin_clz(x);
#pragma unroll
            for (int j = 0; j < kDim; j++) {
                basis[j] = j == lead ? x : basis[j];
                comb[j] = j == lead ? cx : comb[j];
                row[j] = j == k ? r : row[j];
            }
            k++;
        }
    }
    a.b = (uint32_t)(smx_next(st) & mask);
    // reduce the basis (vector h has leading bit h) to the identity
#pragma unroll
    for (int h = 0; h < kDim; h++)
#pragma unroll
        for (int h2 = h + 1; h2 < kDim; h2++) {
            const bool hit = (basis[h2] >> h) & 1u;
            basis[h2] ^= hit ? basis[h] : 0u;
            comb[h2] ^= hit ? comb[h] : 0u;
        }
    transpose(row, a.col);
    transpose(comb, ai.col); // comb[h] is row h of A^{-1}
    ai.b = apply(ai.col, a.b); // p^{-1}(y) = A^{-1} y + A^{-1} b
}

// the stored form: columns and b, both times 4, then the dimension
__device__ __forceinline__ void store_map(const CMap &a, int md, uint32_t *out)
{
    uint4 *o = (uint4 *)out;
    o[0] = make_uint4(a.col[0] << 2, a.col[1] << 2, a.col[2] << 2, a.col[3] << 2);
    o[1] = make_uint4(a.col[4] << 2, a.col[5] << 2, a.col[6] << 2, a.col[7] << 2);
    o[2] = make_uint4(a.col[8] << 2, a.col[9] << 2, a.b << 2, (uint32_t)md);
}

__device__ __forceinline__ void load_map(const uint32_t *in, CMap &a)
{
    const uint4 *s = (const uint4 *)in;
    const uint4 w0 = s[0], w1 = s[1], w2 = s[2];
    a.col[0] = w0.x >> 2;
    a.col[1] = w0.y >> 2;
    a.col[2] = w0.z >> 2;
    a.col[3] = w0.w >> 2;
    a.col[4] = w1.x >> 2;
    a.col[5] = w1.y >> 2;
    a.col[6] = w1.z >> 2;
    a.col[7] = w1.w >> 2;
    a.col[8] = w2.x >> 2;
    a.col[9] = w2.y >> 2;
    a.b = w2.z >> 2;
}

// (p o q)(i) = A_p (A_q i + b_q) + b_p
__device__ __forceinline__ void compose(const CMap &p, const CMap &q, CMap &r)
{
#pragma unroll
    for (int k = 0; k < kDim; k++)
        r.col[k] = apply(p.col, q.col[k]);
    r.b = apply(p.col, q.b) ^ p.b;
}

struct FreshArgs {
    uint32_t *maps; // [frames][P][maps_per_dec][kMapWords]
    uint64_t seed;
    int64_t frame0; // index of the chunk's first frame in the call
    int frames, P, L, m, nperm, maps_per_dec;
};

// One thread per (frame, decoder): that decoder's maps for that frame, drawn
// row by row from the SplitMix64 stream whose state is one step from
// seed ^ (frame << 20 | decoder), in the fixed draw order (the L initial
// maps, then 2L candidates per permutation-domain node in preorder), stored
// as the fixed tables are: initial maps, their inverses, then per node the
// candidates and their inverses.  At the root a candidate q of path c is
// stored composed after that path's initial map p (read back from this
// thread's own stores), p o q, with inverse q^{-1} o p^{-1}.
__global__ void __launch_bounds__(256) rm_fresh_maps_kernel(FreshArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.frames * a.P)
        return;
    const int64_t f = t / a.P;
    const int d = (int)(t % a.P);
    uint64_t st = a.seed ^ (((uint64_t)(a.frame0 + f) << 20) | (uint64_t)d);
    st = smx_next(st);
    uint32_t *base = a.maps + (size_t)t * a.maps_per_dec * kMapWords;
    const int L = a.L, m = a.m;
    for (int l = 0; l < L; l++) {
        CMap q, qi;
        draw_map(m, st, q, qi);
        store_map(q, m, base + (size_t)l * kMapWords);
        store_map(qi, m, base + (size_t)(L + l) * kMapWords);
    }
    for (int v = 0; v < a.nperm; v++) {
        const int md = m - v;
        uint32_t *node = base + (size_t)(2 * L + 4 * L * v) * kMapWords;
        for (int c = 0; c < 2 * L; c++) {
            CMap q, qi;
            draw_map(md, st, q, qi);
            if (v == 0) {
                CMap p, pi, r, ri;
                load_map(base + (size_t)(c % L) * kMapWords, p);
                load_map(base + (size_t)(L + c % L) * kMapWords, pi);
                compose(p, q, r);
                compose(qi, pi, ri);
                store_map(r, md, node + (size_t)c * kMapWords);
                store_map(ri, md, node + (size_t)(2 * L + c) * kMapWords);
            } else {
                store_map(q, md, node + (size_t)c * kMapWords);
                store_map(qi, md, node + (size_t)(2 * L + c) * kMapWords);
            }
        }
    }
}

} // namespace

int fresh_decode(rm_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_metric)
{
    const int64_t per_frame = (int64_t)d->cfg.P * d->maps_per_dec * kMapWords;
    // The table buffer is shared by every call: a decode queued earlier on
    // another stream may still read it, so the first draw waits for the last
    // decode that used it (within a call, stream order does the same).
    if (d->fresh_pending) {
        const hipError_t w = hipStreamWaitEvent(d->stream, d->fresh_done, 0);
        if (w != hipSuccess)
            return fail(RM_E_HIP, std::string("fresh-mode stream wait: ") + hipGetErrorString(w));
    }
    for (int64_t f0 = 0; f0 < n_frames; f0 += d->fresh_chunk) {
        const int64_t nf = n_frames - f0 < d->fresh_chunk ? n_frames - f0 : d->fresh_chunk;
        FreshArgs g;
        g.maps = d->d_maps;
        g.seed = d->cfg.seed;
        g.frame0 = f0;
        g.frames = (int)nf;
        g.P = d->cfg.P;
        g.L = d->cfg.L;
        g.m = d->cfg.m;
        g.nperm = d->nperm;
        g.maps_per_dec = d->maps_per_dec;
        const int64_t threads = nf * d->cfg.P;
        hipLaunchKernelGGL(rm_fresh_maps_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, d->stream, g);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) {
            KernelArgs a = batch_args(d, llr + f0 * d->N, nf, out_bits + f0 * (d->N / 8),
                                      out_metric ? out_metric + f0 : nullptr);
            a.frame_stride = per_frame;
            e = launch_decoder(d, a, nf);
        }
        if (e == hipSuccess) {
            e = hipEventRecord(d->fresh_done, d->stream);
            d->fresh_pending = d->fresh_pending || e == hipSuccess;
        }
        if (e != hipSuccess)
            return fail(RM_E_HIP, std::string("fresh-mode launch: ") + hipGetErrorString(e));
    }
    return RM_OK;
}

} // namespace rmdec
