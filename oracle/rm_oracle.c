/*
 * rm_oracle.c -- TEST INFRASTRUCTURE, not product code.
 *
 * Plain CPU oracle for the permuted FHT-FSCL decoder of Reed-Muller codes
 * (Doan, Hashemi, Gross, arXiv 2108.12550).  It is written to be read next to
 * the paper: every function follows one passage and keeps its order of steps.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load it; it shares nothing with the HIP decoder.
 *
 * Arithmetic is scalar IEEE binary32 (the decoder's working precision), built
 * with -O2 -ffp-contract=off and no fast-math, so that every decision (sorts,
 * arg-max, hard decisions) is taken on the same values as a GPU path that
 * follows the same operation order.  Where the paper leaves an order or a tie
 * open, the choice made here is stated in a comment and listed as a reading.
 *
 * Pins (tests/test_oracle_pins.py): code tables against printed values; FHT
 * and SPC decoding against brute force; the decoder against exact
 * invariants (codeword membership, final metric = correlation metric,
 * noiseless input, sign-flip equivariance, ML at r = 1 roots, Wagner at
 * r = m-1 roots, exhaustive ML on RM(2,5)); FER against Fig. 5(a).
 * Parity unpinned: tie-break order among equal values and the permutation
 * draw (fixed by contract; the draw is checked only for being an
 * automorphism and against the library's independent implementation).
 */
#include "rm_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define MAXM 10          /* N <= 1024 */
#define MAXL 64

/* ------------------------------------------------------------------------ */
/* SplitMix64, from its published definition (Steele, Lea and Flood,        */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014): a Weyl    */
/* sequence with increment 0x9E3779B97F4A7C15 passed through a 64-bit mix.    */
/* ------------------------------------------------------------------------ */
uint64_t rmo_splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* Affine maps z -> A z + b over F2^m (the full symmetry group of RM(r,m)   */
/* for 1 <= r <= m-2).  Position i is the point z(i) with z_k = bit k of i.  */
/* Row j of A gives output bit j: (A z)_j = parity(row_j & i).               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int m;
    uint32_t row[MAXM];
    uint32_t b;
} amap;

static int parity32(uint32_t v)
{
    int p = 0;
    while (v) {
        p ^= 1;
        v &= v - 1;
    }
    return p;
}

static uint32_t amap_apply(const amap *a, uint32_t i)
{
    uint32_t z = 0;
    for (int j = 0; j < a->m; j++)
        z |= (uint32_t)parity32(a->row[j] & i) << j;
    return z ^ a->b;
}

/* Gaussian elimination over GF(2). */
static int gf2_full_rank(const uint32_t *rows, int m)
{
    uint32_t t[MAXM];
    memcpy(t, rows, (size_t)m * sizeof *t);
    int rank = 0;
    for (int col = 0; col < m; col++) {
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

/* One uniform element of AGL(m,2): draw the m rows of A (low m bits of one
 * SplitMix64 output each) until A is invertible, then draw b. */
static void amap_draw(amap *a, int m, uint64_t *st)
{
    const uint32_t mask = (1u << m) - 1u;
    a->m = m;
    do {
        for (int k = 0; k < m; k++)
            a->row[k] = (uint32_t)(rmo_splitmix64_next(st) & mask);
    } while (!gf2_full_rank(a->row, m));
    a->b = (uint32_t)(rmo_splitmix64_next(st) & mask);
}

/* Do the n rows (m columns) have rank n?  Gaussian elimination over GF(2). */
static int gf2_rows_independent(const uint32_t *rows, int n, int m)
{
    uint32_t t[MAXM];
    memcpy(t, rows, (size_t)n * sizeof *t);
    int rank = 0;
    for (int col = 0; col < m && rank < n; col++) {
        int piv = -1;
        for (int k = rank; k < n; k++)
            if ((t[k] >> col) & 1u) {
                piv = k;
                break;
            }
        if (piv < 0)
            continue;
        uint32_t tmp = t[piv];
        t[piv] = t[rank];
        t[rank] = tmp;
        for (int k = 0; k < n; k++)
            if (k != rank && ((t[k] >> col) & 1u))
                t[k] ^= t[rank];
        rank++;
    }
    return rank == n;
}

/* The fresh mode's draw of one uniform element of AGL(m,2), built row by
 * row: row k of A is drawn (low m bits of one SplitMix64 output) until rows
 * 0..k are linearly independent, so every ordered basis of F2^m, hence every
 * invertible A, is equally likely; then b. */
static void amap_draw_rowwise(amap *a, int m, uint64_t *st)
{
    const uint32_t mask = (1u << m) - 1u;
    a->m = m;
    for (int k = 0; k < m; k++)
        do
            a->row[k] = (uint32_t)(rmo_splitmix64_next(st) & mask);
        while (!gf2_rows_independent(a->row, k + 1, m));
    a->b = (uint32_t)(rmo_splitmix64_next(st) & mask);
}

/* ------------------------------------------------------------------------ */
/* Code construction (Section II-A): x = u G^{(x)m}, G = [[1,0],[1,1]];      */
/* u_i is frozen iff the weight w_i of row i of G^{(x)m} is below            */
/* d = 2^{m-r}.  The Kronecker powers are built explicitly.                  */
/* ------------------------------------------------------------------------ */
static uint8_t *gkron[MAXM + 1];
static pthread_mutex_t gkron_lock = PTHREAD_MUTEX_INITIALIZER;

static const uint8_t *kron_power(int s)
{
    pthread_mutex_lock(&gkron_lock);
    if (!gkron[0]) {
        gkron[0] = malloc(1);
        gkron[0][0] = 1;
        for (int t = 1; t <= MAXM; t++) {
            int n = 1 << t, h = n / 2;
            uint8_t *g = calloc((size_t)n * n, 1);
            const uint8_t *p = gkron[t - 1];
            /* G (x) P = [[P, 0], [P, P]] */
            for (int i = 0; i < h; i++)
                for (int j = 0; j < h; j++) {
                    g[(size_t)i * n + j] = p[(size_t)i * h + j];
                    g[(size_t)(i + h) * n + j] = p[(size_t)i * h + j];
                    g[(size_t)(i + h) * n + j + h] = p[(size_t)i * h + j];
                }
            gkron[t] = g;
        }
    }
    pthread_mutex_unlock(&gkron_lock);
    return gkron[s];
}

int rmo_info_set(int m, int r, uint8_t *is_info)
{
    if (m < 0 || m > MAXM || r < 0 || r > m)
        return -1;
    const int n = 1 << m;
    const uint8_t *g = kron_power(m);
    const long d = 1L << (m - r);
    for (int i = 0; i < n; i++) {
        long w = 0;
        for (int j = 0; j < n; j++)
            w += g[(size_t)i * n + j];
        is_info[i] = (uint8_t)(w >= d);
    }
    return 0;
}

int rmo_encode(int m, const uint8_t *u, uint8_t *x)
{
    if (m < 0 || m > MAXM)
        return -1;
    const int n = 1 << m;
    const uint8_t *g = kron_power(m);
    for (int j = 0; j < n; j++)
        x[j] = 0;
    for (int k = 0; k < n; k++)
        if (u[k])
            for (int j = 0; j < n; j++)
                x[j] ^= g[(size_t)k * n + j];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Processing element (Section II-B), min-sum form.                          */
/* ------------------------------------------------------------------------ */
static float sgnf(float a) { return a < 0.0f ? -1.0f : 1.0f; } /* sgn(0) reads +1 */

static float f_minsum(float a, float b) { return sgnf(a) * sgnf(b) * fminf(fabsf(a), fabsf(b)); }

static float g_func(float a, float b, uint8_t c) { return b + (1.0f - 2.0f * (float)c) * a; }

/* Sum of n values by the halving tree v[i] += v[i+w], w = n/2, n/4, ..., 1.
 * The paper fixes no summation order; this one is the decoder's contract. */
static float tree_sum(const float *v, int n)
{
    float *t = malloc((size_t)n * sizeof *t);
    memcpy(t, v, (size_t)n * sizeof *t);
    for (int w = n / 2; w >= 1; w /= 2)
        for (int i = 0; i < w; i++)
            t[i] = t[i] + t[i + w];
    float s = t[0];
    free(t);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2's reliability of a candidate permutation (LM): the sum of |f| over */
/* the pairs of positions that the candidate's f step combines, where       */
/* |f(a, b)| = min(|a|, |b|).  Under an affine map p the pairs              */
/* {p(i), p(i + n/2)}, i < n/2, are the cosets {u, u ^ d} of               */
/* d = p(n/2) ^ p(0), so the metric depends on the map through d alone.     */
/* The paper fixes no order for the sum.  Here the cosets are taken in      */
/* ascending order of their smaller element u in the array v that holds the */
/* LLRs (u runs over the positions whose bit msb(d) is 0), and the halving  */
/* tree sums that list: the order in which a decoder reads the pairs        */
/* straight from the array, without going through the map.                  */
/* ------------------------------------------------------------------------ */
float rmo_lm(int m, const float *v, uint32_t d)
{
    const int h = 1 << (m - 1);
    int k = 0;
    while ((d >> (k + 1)) != 0)
        k++;
    float *fv = malloc((size_t)h * sizeof *fv);
    for (int i = 0; i < h; i++) {
        const uint32_t lo = (uint32_t)i & ((1u << k) - 1u);
        const uint32_t u = (((uint32_t)i >> k) << (k + 1)) | lo; /* i with a 0 put in at bit k */
        fv[i] = fabsf(f_minsum(v[u], v[u ^ d]));
    }
    const float s = tree_sum(fv, h);
    free(fv);
    return s;
}

/* Stable ascending insertion sort of the index array ord[] by key[]. */
static void stable_sort_asc(int *ord, const float *key, int n)
{
    for (int a = 1; a < n; a++) {
        int v = ord[a], b = a - 1;
        while (b >= 0 && key[ord[b]] > key[v]) {
            ord[b + 1] = ord[b];
            b--;
        }
        ord[b + 1] = v;
    }
}

/* Stable descending insertion sort of ord[] by key[]. */
static void stable_sort_desc(int *ord, const float *key, int n)
{
    for (int a = 1; a < n; a++) {
        int v = ord[a], b = a - 1;
        while (b >= 0 && key[ord[b]] < key[v]) {
            ord[b + 1] = ord[b];
            b--;
        }
        ord[b + 1] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* Walsh-Hadamard transform by the Plotkin split (Section II-C): the halves  */
/* lo = F[0..n/2), hi = F[n/2..n) become (hi - lo, hi + lo), then each half  */
/* is transformed on its own.  F[i] ends as the correlation of alpha with    */
/* the +-1 image of the first-order codeword that index i stands for.        */
/* ------------------------------------------------------------------------ */
static void hadamard(float *F, int n)
{
    if (n < 2)
        return;
    const int h = n / 2;
    for (int i = 0; i < h; i++) {
        const float lo = F[i], hi = F[i + h];
        F[i] = hi - lo;
        F[i + h] = hi + lo;
    }
    hadamard(F, h);
    hadamard(F + h, h);
}

/* The k largest of key[0..n) as indices, largest first, ties to the lower */
/* index: k scans, each taking the largest entry not yet taken.             */
static void largest_k(const float *key, int n, int k, int *out)
{
    uint8_t *taken = calloc((size_t)n, 1);
    for (int j = 0; j < k; j++) {
        int best = -1;
        for (int i = 0; i < n; i++)
            if (!taken[i] && (best < 0 || key[i] > key[best]))
                best = i;
        taken[best] = 1;
        out[j] = best;
    }
    free(taken);
}

/* Message word of the first-order codeword selected by transform index i   */
/* and the sign of F[i] (Section II-C, Alg. 4): the sign gives the constant */
/* term m_s; the s linear terms are the binary digits of 2^s - 1 - i, the   */
/* least significant digit first (m_t = bit s-1-t).                          */
static void first_order_message(int s, int i, int negative, uint8_t *msg)
{
    const unsigned c = (unsigned)((1 << s) - 1 - i);
    for (int t = 0; t < s; t++)
        msg[t] = (uint8_t)((c >> (s - 1 - t)) & 1u);
    msg[s] = (uint8_t)negative;
}

/* ------------------------------------------------------------------------ */
/* FHT decoding of one path at a first-order node RM(1,s) (Alg. 4), with   */
/* the metric of Eq. (10).  The k = min(L, 2^s) candidates are the indices  */
/* of the k largest |F| (ties to the lower index); each gives a codeword    */
/* (its message through G^{(x)s}) and the metric pm_in + (sum|alpha| -      */
/* |F[i]|) / 2.  Writes cw[j*n..], pm[j], idx[j] for j < k; returns k.      */
/* ------------------------------------------------------------------------ */
int rmo_fht(int s, int L, const float *alpha, float pm_in, uint8_t *cw, float *pm, int *idx)
{
    if (s < 1 || s > MAXM || L < 1)
        return -1;
    const int n = 1 << s;
    const int k = L < n ? L : n;
    float *F = malloc((size_t)n * sizeof *F);
    float *mag = malloc((size_t)n * sizeof *mag);
    int *ord = malloc((size_t)n * sizeof *ord);
    uint8_t *info = malloc((size_t)n);
    uint8_t *u = malloc((size_t)n);
    rmo_info_set(s, 1, info);

    for (int i = 0; i < n; i++)
        mag[i] = fabsf(alpha[i]);
    const float sum_abs = tree_sum(mag, n);

    memcpy(F, alpha, (size_t)n * sizeof *F);
    hadamard(F, n);

    for (int i = 0; i < n; i++)
        mag[i] = fabsf(F[i]);
    largest_k(mag, n, k, ord); /* largest |F| first, ties to the lower index */

    for (int j = 0; j < k; j++) {
        const int i = ord[j];
        uint8_t msg[MAXM + 1];
        first_order_message(s, i, F[i] < 0.0f, msg);
        /* information positions of RM(1,s) in increasing order: the s rows
         * of weight 2^(s-1) carry m_0 .. m_(s-1), the all-ones row m_s */
        int t = 0;
        for (int q = 0; q < n; q++)
            u[q] = info[q] ? msg[t++] : 0;
        rmo_encode(s, u, cw + (size_t)j * n);
        idx[j] = i;
        pm[j] = pm_in + 0.5f * (sum_abs - mag[i]);
    }
    free(F);
    free(mag);
    free(ord);
    free(info);
    free(u);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Alg. 3: FHTL.  Every path contributes min(L,2^s) candidates to E, listed  */
/* path by path; E is sorted stably by metric (merge sort in the paper) and  */
/* the first L survive.  anc[l] is the input path of survivor l.             */
/* ------------------------------------------------------------------------ */
static void fhtl_node(int s, int L, float *const *alpha, const float *pm_in, uint8_t **x, float *pm_out,
                      int *anc)
{
    const int n = 1 << s;
    const int k = L < n ? L : n;
    const int ne = L * k;
    uint8_t *cw = malloc((size_t)ne * n);
    float *pe = malloc((size_t)ne * sizeof *pe);
    int *src = malloc((size_t)ne * sizeof *src);
    int *ord = malloc((size_t)ne * sizeof *ord);
    int idx[MAXL];
    for (int l = 0; l < L; l++) {
        rmo_fht(s, L, alpha[l], pm_in[l], cw + (size_t)l * k * n, pe + (size_t)l * k, idx);
        for (int j = 0; j < k; j++)
            src[l * k + j] = l;
    }
    for (int e = 0; e < ne; e++)
        ord[e] = e;
    stable_sort_asc(ord, pe, ne);
    for (int l = 0; l < L; l++) {
        memcpy(x[l], cw + (size_t)ord[l] * n, (size_t)n);
        pm_out[l] = pe[ord[l]];
        anc[l] = src[ord[l]];
    }
    free(cw);
    free(pe);
    free(src);
    free(ord);
}

int rmo_fhtl(int s, int L, const float *alpha, const float *pm_in, uint8_t *x, float *pm, int *anc)
{
    if (s < 1 || s > MAXM || L < 1 || L > MAXL)
        return -1;
    const int n = 1 << s;
    float *ap[MAXL];
    uint8_t *xp[MAXL];
    for (int l = 0; l < L; l++) {
        ap[l] = (float *)alpha + (size_t)l * n;
        xp[l] = x + (size_t)l * n;
    }
    fhtl_node(s, L, ap, pm_in, xp, pm, anc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SPCL: fast list decoding of a single-parity-check node RM(s-1,s),         */
/* Eqs. (2)-(6).  Per path: hard decisions, parity p, the least reliable      */
/* positions o_0, o_1, ... (|alpha| ascending, ties to the lower index) and   */
/* PM += |alpha_{o_0}| when p = 1.  Then tau splits on o_1..o_tau; each path  */
/* is listed as (keep, flip), the list is sorted stably by metric and cut to  */
/* L.  Last, o_0 is set so that the parity check holds.                       */
/* tau = min(L, 2^s - 1), and tau = 0 for L = 1 (a split there can never win). */
/* ------------------------------------------------------------------------ */
static void spcl_node(int s, int L, float *const *alpha, const float *pm_in, uint8_t **x, float *pm_out,
                      int *anc)
{
    const int n = 1 << s;
    const int tau = (L == 1) ? 0 : (L < n - 1 ? L : n - 1);
    int *order = malloc((size_t)L * (tau + 1) * sizeof *order);
    uint8_t *hd = malloc((size_t)L * n);
    uint8_t *taken = malloc((size_t)n);
    /* path list: source path, hard decisions, parity, metric */
    int *csrc = malloc((size_t)2 * L * sizeof *csrc);
    uint8_t *ch = malloc((size_t)2 * L * n);
    int *cp = malloc((size_t)2 * L * sizeof *cp);
    float *cpm = malloc((size_t)2 * L * sizeof *cpm);
    int *nsrc = malloc((size_t)2 * L * sizeof *nsrc);
    uint8_t *nh = malloc((size_t)2 * L * n);
    int *np = malloc((size_t)2 * L * sizeof *np);
    float *npm = malloc((size_t)2 * L * sizeof *npm);
    int *ord = malloc((size_t)2 * L * sizeof *ord);

    for (int l = 0; l < L; l++) {
        int p = 0;
        for (int i = 0; i < n; i++) {
            hd[(size_t)l * n + i] = (uint8_t)(alpha[l][i] < 0.0f); /* Eq. (2) */
            p ^= hd[(size_t)l * n + i];
        }
        memset(taken, 0, (size_t)n);
        for (int t = 0; t <= tau; t++) {
            int best = -1;
            for (int i = 0; i < n; i++)
                if (!taken[i] && (best < 0 || fabsf(alpha[l][i]) < fabsf(alpha[l][best])))
                    best = i;
            taken[best] = 1;
            order[l * (tau + 1) + t] = best;
        }
        csrc[l] = l;
        memcpy(ch + (size_t)l * n, hd + (size_t)l * n, (size_t)n);
        cp[l] = p;
        cpm[l] = pm_in[l];
        if (p) /* Eq. (3) */
            cpm[l] = pm_in[l] + fabsf(alpha[l][order[l * (tau + 1)]]);
    }

    for (int t = 1; t <= tau; t++) {
        for (int q = 0; q < L; q++) {
            const int sp = csrc[q];
            const int ot = order[sp * (tau + 1) + t];
            const int o0 = order[sp * (tau + 1)];
            /* keep */
            nsrc[2 * q] = sp;
            memcpy(nh + (size_t)(2 * q) * n, ch + (size_t)q * n, (size_t)n);
            np[2 * q] = cp[q];
            npm[2 * q] = cpm[q];
            /* flip o_t: Eq. (4) with the path's current parity, then Eq. (5) */
            nsrc[2 * q + 1] = sp;
            memcpy(nh + (size_t)(2 * q + 1) * n, ch + (size_t)q * n, (size_t)n);
            nh[(size_t)(2 * q + 1) * n + ot] ^= 1;
            npm[2 * q + 1] = (cpm[q] + fabsf(alpha[sp][ot])) + (1.0f - 2.0f * (float)cp[q]) * fabsf(alpha[sp][o0]);
            np[2 * q + 1] = cp[q] ^ 1;
        }
        for (int e = 0; e < 2 * L; e++)
            ord[e] = e;
        stable_sort_asc(ord, npm, 2 * L);
        for (int q = 0; q < L; q++) {
            const int e = ord[q];
            csrc[q] = nsrc[e];
            memcpy(ch + (size_t)q * n, nh + (size_t)e * n, (size_t)n);
            cp[q] = np[e];
            cpm[q] = npm[e];
        }
    }

    for (int q = 0; q < L; q++) {
        const int o0 = order[csrc[q] * (tau + 1)];
        uint8_t *h = ch + (size_t)q * n;
        int par = 0;
        for (int i = 0; i < n; i++)
            if (i != o0)
                par ^= h[i];
        h[o0] = (uint8_t)par; /* Eq. (6) */
        memcpy(x[q], h, (size_t)n);
        pm_out[q] = cpm[q];
        anc[q] = csrc[q];
    }
    free(order);
    free(hd);
    free(taken);
    free(csrc);
    free(ch);
    free(cp);
    free(cpm);
    free(nsrc);
    free(nh);
    free(np);
    free(npm);
    free(ord);
}

int rmo_spcl(int s, int L, const float *alpha, const float *pm_in, uint8_t *x, float *pm, int *anc)
{
    if (s < 1 || s > MAXM || L < 1 || L > MAXL)
        return -1;
    const int n = 1 << s;
    float *ap[MAXL];
    uint8_t *xp[MAXL];
    for (int l = 0; l < L; l++) {
        ap[l] = (float *)alpha + (size_t)l * n;
        xp[l] = x + (size_t)l * n;
    }
    spcl_node(s, L, ap, pm_in, xp, pm, anc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Decoder object: code parameters and the random permutations, drawn once  */
/* from the seed in a fixed order: for each decoder d, the L initial maps,   */
/* then 2L candidate maps for every permutation-domain node in preorder.     */
/* ------------------------------------------------------------------------ */
struct rmo_decoder {
    int m, r, P, L, mode;
    uint64_t seed;
    int n_perm_nodes; /* internal nodes visited while isPermutation holds */
    amap *init;       /* [P][L] */
    amap *cand;       /* [P][n_perm_nodes][2L] */
};

/* Draw one decoder's maps for one frame of the fresh mode from the stream
 * st: the L initial maps, then 2L candidate maps for every
 * permutation-domain node in preorder, each built row by row. */
static void draw_decoder_maps(int m, int L, int nperm, uint64_t *st, amap *init, amap *cand)
{
    for (int l = 0; l < L; l++)
        amap_draw_rowwise(&init[l], m, st);
    for (int v = 0; v < nperm; v++)
        for (int c = 0; c < 2 * L; c++)
            amap_draw_rowwise(&cand[(size_t)v * 2 * L + c], m - v, st);
}

/* Stream of decoder dd for frame f in the fresh mode: one SplitMix64 step
 * from seed ^ (f << 20 | dd) gives the starting state. */
static uint64_t fresh_stream(uint64_t seed, int64_t f, int dd)
{
    uint64_t st = seed ^ (((uint64_t)f << 20) | (uint64_t)dd);
    return rmo_splitmix64_next(&st);
}

/* The permutation domain covers the internal nodes reached from the root by
 * left steps before the first first-order node (Alg. 2: isPermutation is set
 * at the root and cleared at the first r = 1 node, which is the leftmost). */
static int count_perm_nodes(int m, int r, int mode)
{
    if (mode == RMO_PERM_NONE)
        return 0;
    int c = 0;
    while (1 < r && r < m - 1) {
        c++;
        r--;
        m--;
    }
    return c;
}

rmo_decoder *rmo_create(int m, int r, int P, int L, int perm_mode, uint64_t seed)
{
    if (m < 2 || m > MAXM || r < 1 || r > m - 1 || P < 1 || L < 1 || L > MAXL)
        return NULL;
    if (perm_mode != RMO_PERM_NONE && perm_mode != RMO_PERM_PFHT && perm_mode != RMO_PERM_FRESH)
        return NULL;
    if (perm_mode == RMO_PERM_FRESH && P > (1 << 20))
        return NULL;
    rmo_decoder *d = calloc(1, sizeof *d);
    d->m = m;
    d->r = r;
    d->P = P;
    d->L = L;
    d->mode = perm_mode;
    d->seed = seed;
    d->n_perm_nodes = count_perm_nodes(m, r, perm_mode);
    d->init = calloc((size_t)P * L, sizeof *d->init);
    d->cand = calloc((size_t)P * (d->n_perm_nodes ? d->n_perm_nodes : 1) * 2 * L, sizeof *d->cand);
    kron_power(0);
    uint64_t st = seed;
    for (int p = 0; p < P; p++) {
        for (int l = 0; l < L; l++) {
            amap *a = &d->init[(size_t)p * L + l];
            if (perm_mode != RMO_PERM_NONE) {
                amap_draw(a, m, &st);
            } else { /* identity */
                a->m = m;
                for (int k = 0; k < m; k++)
                    a->row[k] = 1u << k;
                a->b = 0;
            }
        }
        for (int v = 0; v < d->n_perm_nodes; v++)
            for (int c = 0; c < 2 * L; c++)
                amap_draw(&d->cand[((size_t)p * d->n_perm_nodes + v) * 2 * L + c], m - v, &st);
    }
    return d;
}

void rmo_destroy(rmo_decoder *d)
{
    if (!d)
        return;
    free(d->init);
    free(d->cand);
    free(d);
}

int rmo_perm_count(const rmo_decoder *d) { return d->P * (d->L + d->n_perm_nodes * 2 * d->L); }

int rmo_perm_export(const rmo_decoder *d, uint16_t *rows, uint16_t *b, int *mdim, int cap)
{
    int k = 0;
    for (int p = 0; p < d->P; p++) {
        for (int l = 0; l < d->L; l++) {
            const amap *a = &d->init[(size_t)p * d->L + l];
            if (k >= cap)
                return -1;
            for (int j = 0; j < 16; j++)
                rows[k * 16 + j] = (uint16_t)(j < a->m ? a->row[j] : 0);
            b[k] = (uint16_t)a->b;
            mdim[k] = a->m;
            k++;
        }
        for (int v = 0; v < d->n_perm_nodes; v++)
            for (int c = 0; c < 2 * d->L; c++) {
                const amap *a = &d->cand[((size_t)p * d->n_perm_nodes + v) * 2 * d->L + c];
                if (k >= cap)
                    return -1;
                for (int j = 0; j < 16; j++)
                    rows[k * 16 + j] = (uint16_t)(j < a->m ? a->row[j] : 0);
                b[k] = (uint16_t)a->b;
                mdim[k] = a->m;
                k++;
            }
    }
    return k;
}

int rmo_perm_export_frame(const rmo_decoder *d, int64_t frame, uint16_t *rows, uint16_t *b, int *mdim, int cap)
{
    if (d->mode != RMO_PERM_FRESH)
        return rmo_perm_export(d, rows, b, mdim, cap);
    const int L = d->L, nperm = d->n_perm_nodes;
    amap *init = calloc((size_t)L, sizeof *init);
    amap *cand = calloc((size_t)(nperm ? nperm : 1) * 2 * L, sizeof *cand);
    int k = 0;
    for (int p = 0; p < d->P && k >= 0; p++) {
        uint64_t st = fresh_stream(d->seed, frame, p);
        draw_decoder_maps(d->m, L, nperm, &st, init, cand);
        for (int q = 0; q < L + nperm * 2 * L && k >= 0; q++) {
            const amap *a = q < L ? &init[q] : &cand[q - L];
            if (k >= cap) {
                k = -1;
                break;
            }
            for (int j = 0; j < 16; j++)
                rows[k * 16 + j] = (uint16_t)(j < a->m ? a->row[j] : 0);
            b[k] = (uint16_t)a->b;
            mdim[k] = a->m;
            k++;
        }
    }
    free(init);
    free(cand);
    return k;
}

/* Preorder node list as (kind, r, m) triples, following Alg. 2's tests in
 * their order: 1<r<m-1 internal, then r=1 FHTL, then r=m-1 SPCL. */
static int sched_walk(int m, int r, int *is_perm, int *out, int cap, int k)
{
    if (1 < r && r < m - 1) {
        if (k + 3 <= cap) {
            out[k] = *is_perm ? RMO_NODE_PERM : RMO_NODE_INTERNAL;
            out[k + 1] = r;
            out[k + 2] = m;
        }
        k += 3;
        k = sched_walk(m - 1, r - 1, is_perm, out, cap, k);
        k = sched_walk(m - 1, r, is_perm, out, cap, k);
    } else if (r == 1) {
        *is_perm = 0;
        if (k + 3 <= cap) {
            out[k] = RMO_NODE_FHTL;
            out[k + 1] = r;
            out[k + 2] = m;
        }
        k += 3;
    } else if (r == m - 1) {
        if (k + 3 <= cap) {
            out[k] = RMO_NODE_SPCL;
            out[k + 1] = r;
            out[k + 2] = m;
        }
        k += 3;
    }
    return k;
}

int rmo_schedule(int m, int r, int perm_mode, int *out, int cap)
{
    if (m < 2 || m > MAXM || r < 1 || r > m - 1)
        return -1;
    int is_perm = (perm_mode == RMO_PERM_PFHT);
    return sched_walk(m, r, &is_perm, out, cap, 0) / 3;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2: p-FHT-FSCL on node RM(r,m) with L paths.                          */
/* In:  alpha[l] (n = 2^m LLRs), pm_in[l].                                    */
/* Out: x[l] (n bits as bytes), pm_out[l], anc[l] = input path from which    */
/*      output path l descends (the surviving ancestor).                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    const rmo_decoder *dec;
    const amap *cand; /* this decoder's candidate maps: [n_perm_nodes][2L] */
    int is_perm;      /* isPermutation */
    int perm_node;    /* index of the next permutation-domain node */
    const float *y;   /* the received vector, read by the root's LM */
    const amap *init; /* the paths' initial maps: path l's root LLRs are y[init_l(i)] */
} ctx_t;

static float **alloc_fvecs(int L, int n)
{
    float **v = malloc((size_t)L * sizeof *v);
    for (int l = 0; l < L; l++)
        v[l] = malloc((size_t)n * sizeof **v);
    return v;
}

static uint8_t **alloc_bvecs(int L, int n)
{
    uint8_t **v = malloc((size_t)L * sizeof *v);
    for (int l = 0; l < L; l++)
        v[l] = malloc((size_t)n);
    return v;
}

static void free_vecs(void **v, int L)
{
    for (int l = 0; l < L; l++)
        free(v[l]);
    free(v);
}

static void node_decode(ctx_t *c, int r, int m, float *const *alpha, const float *pm_in, uint8_t **x,
                        float *pm_out, int *anc)
{
    const int L = c->dec->L;
    const int n = 1 << m;
    const int h = n / 2;

    if (1 < r && r < m - 1) {
        float *const *wa = alpha; /* the LLR vectors the children are built from */
        const float *wpm = pm_in;
        float **pa = NULL;
        float ppm[MAXL];
        int is_per = 0;
        int sel[2 * MAXL];
        int origin[MAXL];
        const amap *cands = NULL;

        if (c->is_perm) {
            /* Permutation domain: 2L candidates, candidate cc permutes the LLRs
             * of path cc mod L; LM = sum |f(permuted)| (rmo_lm); keep the L
             * largest.  At the root path l's LLRs are y read through its
             * initial map, so the pairs are read from y, through the
             * candidate's map composed after that initial map. */
            is_per = 1;
            cands = &c->cand[(size_t)c->perm_node * 2 * L];
            c->perm_node++;
            float lm[2 * MAXL];
            for (int cc = 0; cc < 2 * L; cc++) {
                const int src = cc % L;
                const amap *pc = &cands[cc];
                if (m == c->dec->m) {
                    const amap *pi = &c->init[src];
                    const uint32_t d = amap_apply(pi, amap_apply(pc, (uint32_t)h)) ^ amap_apply(pi, amap_apply(pc, 0));
                    lm[cc] = rmo_lm(m, c->y, d);
                } else {
                    const uint32_t d = amap_apply(pc, (uint32_t)h) ^ amap_apply(pc, 0);
                    lm[cc] = rmo_lm(m, alpha[src], d);
                }
            }
            for (int cc = 0; cc < 2 * L; cc++)
                sel[cc] = cc;
            stable_sort_desc(sel, lm, 2 * L); /* largest reliability first, ties to lower cc */
            pa = alloc_fvecs(L, n);
            for (int l = 0; l < L; l++) {
                origin[l] = sel[l] % L;
                for (int i = 0; i < n; i++)
                    pa[l][i] = alpha[origin[l]][amap_apply(&cands[sel[l]], (uint32_t)i)];
                ppm[l] = pm_in[origin[l]];
            }
            wa = pa;
            wpm = ppm;
        }

        /* left child RM(r-1, m-1) on f */
        float **aL = alloc_fvecs(L, h);
        uint8_t **xL = alloc_bvecs(L, h);
        float pmL[MAXL];
        int ancL[MAXL];
        for (int l = 0; l < L; l++)
            for (int i = 0; i < h; i++)
                aL[l][i] = f_minsum(wa[l][i], wa[l][i + h]);
        node_decode(c, r - 1, m - 1, aL, wpm, xL, pmL, ancL);

        /* right child RM(r, m-1) on g, reading the surviving ancestor's LLRs */
        float **aR = alloc_fvecs(L, h);
        uint8_t **xR = alloc_bvecs(L, h);
        float pmR[MAXL];
        int ancR[MAXL];
        for (int l = 0; l < L; l++)
            for (int i = 0; i < h; i++)
                aR[l][i] = g_func(wa[ancL[l]][i], wa[ancL[l]][i + h], xL[l][i]);
        node_decode(c, r, m - 1, aR, pmL, xR, pmR, ancR);

        /* combine (x_gamma xor x_lambda, x_gamma) and undo the node's permutation */
        uint8_t *xv = malloc((size_t)n);
        for (int l = 0; l < L; l++) {
            const int k = ancR[l];
            for (int i = 0; i < h; i++) {
                xv[i] = (uint8_t)(xR[l][i] ^ xL[k][i]);
                xv[i + h] = xR[l][i];
            }
            const int a = ancL[k];
            if (is_per) {
                for (int i = 0; i < n; i++)
                    x[l][amap_apply(&cands[sel[a]], (uint32_t)i)] = xv[i];
                anc[l] = origin[a];
            } else {
                memcpy(x[l], xv, (size_t)n);
                anc[l] = a;
            }
            pm_out[l] = pmR[l];
        }
        free(xv);
        free_vecs((void **)aL, L);
        free_vecs((void **)xL, L);
        free_vecs((void **)aR, L);
        free_vecs((void **)xR, L);
        if (pa)
            free_vecs((void **)pa, L);
    } else if (r == 1) {
        c->is_perm = 0;
        fhtl_node(m, L, alpha, pm_in, x, pm_out, anc);
    } else if (r == m - 1) {
        spcl_node(m, L, alpha, pm_in, x, pm_out, anc);
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. 5: M decoders on the same y; keep the codeword of the smallest final */
/* metric (a later decoder replaces it only if strictly smaller).  Each      */
/* decoder starts its L paths from y permuted by its initial maps, and the   */
/* surviving codeword is mapped back through the inverse at the root.        */
/* If no metric is ever below +inf (non-finite input) x is all zero.          */
/* ------------------------------------------------------------------------ */
int rmo_decode(const rmo_decoder *d, const float *y, uint8_t *xhat, float *pm)
{
    return rmo_decode_frame(d, y, 0, xhat, pm);
}

int rmo_decode_frame(const rmo_decoder *d, const float *y, int64_t frame, uint8_t *xhat, float *pm)
{
    const int m = d->m, L = d->L, n = 1 << m;
    float best = INFINITY;
    memset(xhat, 0, (size_t)n);
    float **a = alloc_fvecs(L, n);
    uint8_t **x = alloc_bvecs(L, n);
    uint8_t *xo = malloc((size_t)n);
    float pm0[MAXL], pmo[MAXL];
    int anc[MAXL];
    const int fresh = d->mode == RMO_PERM_FRESH;
    amap *finit = fresh ? calloc((size_t)L, sizeof *finit) : NULL;
    amap *fcand = fresh ? calloc((size_t)(d->n_perm_nodes ? d->n_perm_nodes : 1) * 2 * L, sizeof *fcand) : NULL;
    for (int p = 0; p < d->P; p++) {
        const amap *init = &d->init[(size_t)p * L];
        const amap *cand = &d->cand[(size_t)p * d->n_perm_nodes * 2 * L];
        if (fresh) { /* this frame's own maps for decoder p */
            uint64_t st = fresh_stream(d->seed, frame, p);
            draw_decoder_maps(m, L, d->n_perm_nodes, &st, finit, fcand);
            init = finit;
            cand = fcand;
        }
        for (int l = 0; l < L; l++) {
            const amap *ai = &init[l];
            for (int i = 0; i < n; i++)
                a[l][i] = y[amap_apply(ai, (uint32_t)i)];
            /* Alg. 2 starts its L paths from L different permutations.
             * Plain FHT-FSCL (no permutations) starts from one path: list
             * entries 1..L-1 begin inactive, with an infinite metric, so
             * they never displace a finite candidate and the list fills
             * through the path splits alone. */
            pm0[l] = (d->mode != RMO_PERM_NONE || l == 0) ? 0.0f : INFINITY;
        }
        ctx_t c = {d, cand, d->mode != RMO_PERM_NONE, 0, y, init};
        node_decode(&c, d->r, m, a, pm0, x, pmo, anc);
        int ls = 0;
        for (int l = 1; l < L; l++)
            if (pmo[l] < pmo[ls])
                ls = l;
        if (pmo[ls] < best) {
            best = pmo[ls];
            const amap *ai = &init[anc[ls]];
            for (int i = 0; i < n; i++)
                xo[amap_apply(ai, (uint32_t)i)] = x[ls][i];
            memcpy(xhat, xo, (size_t)n);
        }
    }
    *pm = best;
    free_vecs((void **)a, L);
    free_vecs((void **)x, L);
    free(xo);
    free(finit);
    free(fcand);
    return 0;
}

typedef struct {
    const rmo_decoder *d;
    const float *llr;
    int64_t f0, f1, frame0;
    uint8_t *out_bits;
    float *out_pm;
} job_t;

static void *batch_worker(void *arg)
{
    job_t *j = arg;
    const int n = 1 << j->d->m;
    uint8_t *x = malloc((size_t)n);
    for (int64_t f = j->f0; f < j->f1; f++) {
        float pm;
        rmo_decode_frame(j->d, j->llr + f * n, j->frame0 + f, x, &pm);
        uint8_t *ob = j->out_bits + f * (n / 8);
        memset(ob, 0, (size_t)n / 8);
        for (int i = 0; i < n; i++)
            ob[i >> 3] |= (uint8_t)(x[i] << (i & 7));
        if (j->out_pm)
            j->out_pm[f] = pm;
    }
    free(x);
    return NULL;
}

int rmo_decode_batch(const rmo_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_pm,
                     int n_threads)
{
    return rmo_decode_batch_at(d, llr, n_frames, 0, out_bits, out_pm, n_threads);
}

int rmo_decode_batch_at(const rmo_decoder *d, const float *llr, int64_t n_frames, int64_t frame0,
                        uint8_t *out_bits, float *out_pm, int n_threads)
{
    if (!d || n_frames < 0 || frame0 < 0 || (1 << d->m) < 8)
        return -1;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > 256)
        n_threads = 256;
    pthread_t th[256];
    job_t jobs[256];
    const int64_t per = (n_frames + n_threads - 1) / n_threads;
    int started = 0;
    for (int t = 0; t < n_threads; t++) {
        int64_t f0 = t * per, f1 = f0 + per;
        if (f0 >= n_frames)
            break;
        if (f1 > n_frames)
            f1 = n_frames;
        jobs[t] = (job_t){d, llr, f0, f1, frame0, out_bits, out_pm};
        pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
        started++;
    }
    for (int t = 0; t < started; t++)
        pthread_join(th[t], NULL);
    return 0;
}
