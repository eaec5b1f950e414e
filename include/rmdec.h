/*
 * rmdec.h -- C ABI of the MI355X (gfx950) batched decoder for Reed-Muller
 * codes: permuted fast successive-cancellation list decoding with the fast
 * Hadamard transform, run as M parallel decoders per frame (p-FHT-FSCL-L-M).
 *
 * The operation follows Doan, Hashemi and Gross, "Successive-Cancellation
 * Decoding of Reed-Muller Codes with Fast Hadamard Transform" (arXiv
 * 2108.12550): Alg. 5 (M decoders, minimum final metric) over Alg. 2
 * (permutation-domain path extension until the first order-1 node), Alg. 3
 * and Alg. 4 (FHT list decoding of RM(1,s) nodes with the metric of
 * Eq. (10)) and the SPC list rules of Eqs. (2)-(6).
 *
 * Naming: the paper writes RM(r, m) with order r and length N = 2^m; every
 * function here takes m and r as separately named arguments.  "P" below is
 * the number of parallel decoders (the paper's M).
 *
 * Memory: every array argument of rm_decode_batch is DEVICE memory owned by
 * the caller.  The library owns its permutation tables (device memory,
 * allocated at create, freed at destroy) and nothing else; it keeps no
 * reference to caller buffers after the work it queued has completed.
 *
 * Errors: functions returning int give RM_OK (0) or a negative code; a
 * thread-local message is available from rm_last_error().
 */
#ifndef RMDEC_H
#define RMDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RM_OK 0
#define RM_E_INVAL (-1)       /* argument outside the documented domain          */
#define RM_E_NOMEM (-2)       /* host or device allocation failed                */
#define RM_E_HIP (-3)         /* a HIP runtime call failed (message has details) */
#define RM_E_UNSUPPORTED (-4) /* no kernel built for this (m, r, L, mode)        */
#define RM_E_PTR (-5)         /* a host pointer was passed where device memory is required */
/* RM_E_AGAIN (-6) is defined with the request server below */

/* Permutation mode. */
#define RM_PERM_NONE 0 /* FHT-FSCL: identity, no permutation domain; the list starts
                          from one path, the other L-1 entries inactive            */
#define RM_PERM_PFHT 1 /* p-FHT-FSCL: random affine permutations (Alg. 2)         */
#define RM_PERM_FRESH 2 /* p-FHT-FSCL with maps drawn afresh for every frame: the
                           initialisation of Alg. 2 applied per received vector.
                           Frame f of a call (f = 0, 1, ...) decodes with the maps
                           of rm_perm_tables_frame(..., frame = f, ...); the draw
                           runs on the device, chunk by chunk, inside
                           rm_decode_batch (results depend on f)                  */

typedef struct rm_decoder rm_decoder;

typedef struct rm_config {
    int m;               /* 3 <= m <= 10, N = 2^m                                  */
    int r;               /* 1 <= r <= m-1                                          */
    int P;               /* parallel decoders per frame (paper's M), 1..1024      */
    int L;               /* list size per decoder: 1, 2, 4, 8, 16, 32 or 64       */
    uint64_t seed;       /* seed of the permutation draw (SplitMix64)             */
    int perm_mode;       /* RM_PERM_PFHT, RM_PERM_NONE or RM_PERM_FRESH           */
    int waves_per_block; /* 0 = library choice; else 1..4 wavefronts per block   */
} rm_config;

typedef struct rm_info {
    int m, r, P, L, N, K;
    int perm_mode;
    int n_perm_nodes;       /* internal nodes decoded in the permutation domain  */
    int maps_per_decoder;   /* affine maps stored per decoder                    */
    int waves_per_block;
    size_t lds_bytes_per_wave;
    size_t table_bytes;     /* device bytes of the permutation tables            */
} rm_info;

/*
 * Create a decoder for RM(r, m) with P parallel decoders of list size L in
 * the p-FHT-FSCL mode.  The random permutations (Alg. 2's initial maps and
 * the 2L candidate maps of every permutation-domain node) are drawn once,
 * here, from `seed`, as uniform elements of the affine group AGL(m, 2), the
 * full symmetry group of the code.  Draw order, per decoder d = 0..P-1: the
 * L initial maps, then 2L candidate maps per permutation-domain node in
 * preorder; each map draws the m rows of A (low m bits of one SplitMix64
 * output each, redrawn as a whole until A is invertible), then b.
 * Returns NULL on error (see rm_last_error()); needs a HIP device.
 */
rm_decoder *rm_decoder_create(int m, int r, int P, int L, uint64_t seed);

/* As rm_decoder_create, with a permutation mode and a launch override. */
rm_decoder *rm_decoder_create_ex(const rm_config *cfg);

/*
 * Decode n_frames received frames (Alg. 5 per frame).
 *   llr        device, n_frames x N float32, frame-major; LLR = ln P(0)/P(1)
 *              (positive means bit 0).  Values must be finite.
 *   out_bits   device, n_frames x N/8 bytes: the decoded codeword x_hat,
 *              bit i of frame f at byte f*N/8 + (i>>3), bit (i&7).
 *   out_metric device, n_frames float32 final path metrics, or NULL.
 * llr must be 16-byte aligned, out_bits aligned to min(8, N/8) bytes and
 * out_metric to 4 (RM_E_INVAL otherwise): the kernels move frames in 16-byte
 * and codewords in 8-byte words.  Work is queued on the decoder's stream (rm_decoder_set_stream; default the
 * null stream) and the call returns without waiting.  n_frames = 0 is a
 * no-op.  Results depend only on (m, r, P, L, seed, perm_mode, llr), and in
 * RM_PERM_FRESH mode also on each frame's index within the call.
 */
int rm_decode_batch(rm_decoder *d, const float *llr, int64_t n_frames, uint8_t *out_bits, float *out_metric);
/* In RM_PERM_FRESH mode the decoder keeps one device buffer of map tables,
 * redrawn for every chunk of frames; a call made on another stream than the
 * previous call's first waits (on the device) for that call's decodes. */

/* Release the decoder after the work queued on its stream completes.  NULL-safe. */
void rm_decoder_destroy(rm_decoder *d);

/* Bind a hipStream_t (passed as void*) for later rm_decode_batch calls. */
int rm_decoder_set_stream(rm_decoder *d, void *hip_stream);

/* Report the decoder's sizes and launch shape. */
int rm_decoder_info(const rm_decoder *d, rm_info *out);

/*
 * Host only (no device needed): run the permutation draw of
 * rm_decoder_create_ex for (m, r, P, L, seed, perm_mode) and return every
 * drawn map in draw order: rows[k*16 + j] = row j of A_k (bit i of the row
 * multiplies bit i of the position index), b[k], mdim[k] = its dimension.
 * Returns the number of maps, or a negative code if cap is too small.
 * For cross-checking the draw against an independent implementation.
 */
int rm_perm_tables(int m, int r, int P, int L, uint64_t seed, int perm_mode, uint16_t *rows, uint16_t *b,
                   int *mdim, int cap);

/*
 * Host only: as rm_perm_tables, for frame `frame` (0 <= frame < 2^43) of a
 * call.  In RM_PERM_FRESH mode decoder d of frame f draws, in the order of
 * rm_decoder_create, from the SplitMix64 generator whose state is the first
 * output of the generator seeded with seed ^ (f << 20 | d); each map builds
 * A row by row (row k: low bits of one output, redrawn until it lies outside
 * the span of rows 0..k-1; again uniform over invertible A), then b.  The
 * other modes ignore `frame`.
 */
int rm_perm_tables_frame(int m, int r, int P, int L, uint64_t seed, int perm_mode, int64_t frame, uint16_t *rows,
                         uint16_t *b, int *mdim, int cap);

/* 1 if a kernel is built for (m, r, L, perm_mode), else 0.  Host only.
 * Built: every 3 <= m <= 10, 1 <= r <= m-1 at L = 1, 2, 4, 8, 16 and 32 (lists
 * of 16 and 32, and RM(1,10) and RM(9,10) at L = 8, run one workgroup of 512
 * threads per frame), and L = 64 for RM(2..4, 8) and RM(2..4, 9). */
int rm_supported(int m, int r, int L, int perm_mode);

/*
 * Host only: information bits of decoded codewords (Section II-A).  A
 * codeword of RM(r, m) is x = u G^{(x)m}, G = [[1,0],[1,1]], with u_i = 0 off
 * the information set I = {i : popcount(i) >= m - r} (row weights 2^popcount(i)
 * of at least the minimum distance 2^(m-r)); G^{(x)m} is its own inverse over
 * GF(2), so u = x G^{(x)m}.  For each of n_frames codewords in the packed
 * layout of rm_decode_batch's out_bits (host memory, N/8 bytes per frame)
 * this writes u_I to `info` (host, K bytes per frame, one 0/1 value per
 * byte, I in increasing order, K = sum_{i<=r} C(m, i)).  If `n_invalid` is
 * not NULL it receives the number of frames whose u is not zero off I (not
 * codewords of RM(r, m)); their info bytes are still written.  Returns RM_OK,
 * or RM_E_INVAL for m, r outside 3 <= m <= 16, 1 <= r <= m-1, n_frames < 0 or
 * a NULL array with n_frames > 0.
 */
int rm_codeword_to_info(int m, int r, const uint8_t *codewords, int64_t n_frames, uint8_t *info, int64_t *n_invalid);

/* Message of the last error on this thread ("" if none). */
const char *rm_last_error(void);

/*
 * Fused mixed-code launch: frames of several codes (decoders created above)
 * decoded by ONE persistent kernel launch.  The host cuts every segment into
 * runs of `tile_frames` frames and queues the segments' runs in descending
 * order of the work of one of their frames (P decoders of L paths over
 * N log2 N), so that the most expensive entries are taken first; the last
 * frames of the last (cheapest) segment, up to twice the persistent grid's
 * wavefronts and as far as max_tiles leaves room, get one entry each, so
 * that the waves run out of work together.  A launch needs
 * sum_i ceil(n_frames_i / tile_frames_i) <= max_tiles entries.  The
 * persistent grid drains the queue.  Per frame the result is exactly that
 * of rm_decode_batch with the segment's decoder (Alg. 5 over Alg. 2-4 and
 * the SPC rules).
 */
typedef struct rm_mixed rm_mixed;

typedef struct rm_segment {
    const rm_decoder *dec; /* decoder of this segment's code (its tables, P, L)  */
    const float *llr;      /* device, n_frames x N float32, frame-major          */
    int64_t n_frames;      /* >= 0                                               */
    uint8_t *out_bits;     /* device, n_frames x N/8 bytes (as rm_decode_batch)  */
    float *out_metric;     /* device, n_frames float32, or NULL                  */
    int tile_frames;       /* frames per queue entry, 1..64; 0 = library default */
} rm_segment;

#define RM_MIXED_MAX_SEGMENTS 8

/*
 * Create a mixed launcher on the current device: a device work queue of up to
 * max_tiles entries (16 bytes each) and a pinned host staging copy of it.
 * Returns NULL on error (see rm_last_error()).
 */
rm_mixed *rm_mixed_create(int64_t max_tiles);

/* 1 if (m, r, L) is compiled into the fused kernel, else 0.  Host only. */
int rm_mixed_supported(int m, int r, int L);

/* Bind a hipStream_t (as void*) for later launches and graph captures. */
int rm_mixed_set_stream(rm_mixed *mx, void *hip_stream);

/* Persistent grid size: blocks and waves per block (0 = library choice). */
int rm_mixed_set_grid(rm_mixed *mx, int blocks, int waves_per_block);

/*
 * Queue the segments (1..RM_MIXED_MAX_SEGMENTS) on the bound stream: an
 * asynchronous upload of the queue entries, a reset of the queue head and
 * one persistent launch.  Returns without waiting (it waits only for the
 * previous call's upload to have left the staging buffer).  Successive calls
 * reuse one device queue, so all calls on one launcher must go to one stream
 * (or be ordered by the caller).  Segments whose code is not compiled into
 * the fused kernel give RM_E_UNSUPPORTED; more entries than max_tiles give
 * RM_E_INVAL, as do arrays aligned below rm_decode_batch's rule; host
 * pointers give RM_E_PTR.  Nothing is queued on error.
 */
int rm_mixed_decode(rm_mixed *mx, const rm_segment *segs, int n_segs);

/*
 * Record the launch of rm_mixed_decode for these segments (same pointers
 * and sizes) as a hipGraph on the bound stream, which must not be the null
 * stream; rm_mixed_replay launches it again on the bound stream.  The graph
 * owns a device queue of its own, filled once at capture (a synchronous
 * copy), so later rm_mixed_decode calls do not disturb it.  The recorded
 * steps are: reset of the queue head (a kernel, not a memset) and the
 * persistent decode kernel.  Re-capturing replaces the graph.  The segments'
 * buffers and decoders must stay valid while the graph may be replayed.
 */
int rm_mixed_capture(rm_mixed *mx, const rm_segment *segs, int n_segs);
int rm_mixed_replay(rm_mixed *mx);

/* Launch choices of the fused kernel found by rm_mixed_autotune. */
typedef struct rm_mixed_tuning {
    int blocks;                                /* persistent grid (0 = from occupancy)   */
    int waves_per_block;                       /* chosen wavefronts per block            */
    int tile_frames[RM_MIXED_MAX_SEGMENTS];    /* chosen frames per queue entry, per segment */
    float ms;                                  /* average launch time of the best choice */
    int trials;                                /* configurations timed                   */
} rm_mixed_tuning;

/*
 * Autotuner: time rm_mixed_decode on these segments (their outputs are
 * overwritten) for waves per block in {1, 2, 4} and frames per queue entry
 * in {1, 2, 4, 8, 16} -- first one value for all segments, then each
 * segment's own value with the others held -- one warm-up and `reps` timed
 * launches (1..100) per choice.  Blocks on the bound stream.  Sets the
 * launcher's waves per block to the best choice and returns all choices in
 * *out; the caller puts out->tile_frames[i] into segment i.  The decoded
 * results do not depend on any of these choices.
 */
int rm_mixed_autotune(rm_mixed *mx, const rm_segment *segs, int n_segs, int reps, rm_mixed_tuning *out);

/* Release after the work queued on its stream completes.  NULL-safe. */
void rm_mixed_destroy(rm_mixed *mx);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fused
 * launch of rm_mixed_decode with no launcher object and no allocation.  The
 * queue entries and the queue head live in a static device array of the
 * library (256 B + 16 B x RM_MIXED_STATIC_MAX_TILES = 8 MiB, held on every
 * device the library runs on until the process ends).  Queues on
 * `hip_stream` (a hipStream_t as void*, NULL = null stream) one small kernel
 * that writes the queue and clears the head, then the persistent decode
 * kernel (waves_per_block 0..4, 0 = 2; the grid is the occupancy limit).
 * Per frame the result is exactly that of rm_mixed_decode and of
 * rm_decode_batch.  Segments follow rm_mixed_decode's rules; more queue
 * entries than RM_MIXED_STATIC_MAX_TILES give RM_E_INVAL and nothing is
 * queued.  Every call on one device shares that device's array: calls that
 * may overlap on one device (other streams, or another host thread) race and
 * must be ordered by the caller.  Calls no hipMalloc or hipFree.
 */
#define RM_MIXED_STATIC_MAX_TILES (1 << 19)
int rm_mixed_decode_static(const rm_segment *segs, int n_segs, int waves_per_block, void *hip_stream);

/*
 * Request server: continuous batching of single-frame requests of any code,
 * P and L that a serving kernel is built for (rm_server_supported).
 *
 * Each admitted request is copied into the open batch (its LLRs into the
 * batch's pinned staging area, or, for device-resident LLRs, only its
 * address).  The open batch is launched as soon as fewer than `depth`
 * batches are on the device; until then it keeps admitting requests, so
 * batches grow with the load.  A launch is one upload, one persistent
 * kernel per list size present (each frame decoded exactly as by
 * rm_decode_batch with the request's decoder: Alg. 5 over Alg. 2-4 and the
 * SPC rules) and one download; up to `depth` batches run concurrently on
 * their own streams.  Admission is by memory footprint: a request is
 * refused with RM_E_AGAIN when the open batch has no room for its LLRs
 * (4N bytes of `batch_bytes`), no free request slot, or when no batch
 * buffer is free to open; it can be submitted again after rm_server_poll
 * has retired finished batches.  All device and pinned memory is allocated
 * at create: (depth + 1) batch buffers.
 *
 * Results are identical to decoding the same frame alone with
 * rm_decode_batch (they do not depend on batch composition).  Not
 * thread-safe: one host thread at a time per server.
 */
#define RM_E_AGAIN (-6) /* not admitted now: retry after rm_server_poll */

typedef struct rm_server rm_server;

typedef struct rm_server_config {
    int64_t batch_bytes;    /* LLR bytes one batch can hold (>= 4096)                   */
    int max_batch;          /* requests per batch, 1..65536                             */
    int depth;              /* batches on the device at once, 1..4                      */
    int tile_frames;        /* requests per queue entry of a kernel, 1..64 (0 = 2)      */
    int split;              /* waves sharing one request's P decoders: 1, 2 or 4 (0 = 4);
                               the waves of a workgroup each run P/split decoders of the
                               same request (Alg. 5 over all P is kept: the first
                               minimum in decoder order wins), dividing its latency   */
} rm_server_config;

typedef struct rm_request {
    const rm_decoder *dec;  /* decoder of the request (code, P, L, tables)              */
    const float *llr;       /* the frame's N float32 LLRs                               */
    int llr_on_device;      /* 0: host memory, copied at submit; 1: device memory that
                               must stay valid until the request completes            */
    uint64_t tag;           /* caller's value, returned in the completion               */
    double t_arrival_us;    /* arrival time on rm_server_now_us()'s clock; 0 = now      */
    uint8_t *out_bits;      /* optional host destination of the N/8 codeword bytes     */
    float *out_metric;      /* optional host destination of the final metric           */
} rm_request;

typedef struct rm_completion {
    uint64_t ticket, tag;
    int status;             /* RM_OK                                                    */
    int n_bytes;            /* N/8                                                      */
    float metric;           /* final path metric                                        */
    uint8_t bits[128];      /* codeword, bit i at byte i>>3, bit i&7                    */
    double t_arrival_us, t_launch_us, t_done_us; /* rm_server_now_us() clock           */
} rm_completion;

/* Create a server on the current device.  NULL on error (rm_last_error()). */
rm_server *rm_server_create(const rm_server_config *cfg);

/* 1 if requests of (m, r, L) can be served, else 0.  Host only. */
int rm_server_supported(int m, int r, int L);

/* Microseconds on the server's monotonic clock. */
double rm_server_now_us(void);

/*
 * Declare device memory [base, base + bytes) that device-resident requests
 * (llr_on_device = 1) may point into; checked once here (RM_E_PTR if it is
 * not device memory), so that submit only checks ranges.  Up to 16 pools.
 */
int rm_server_register_pool(rm_server *s, const void *base, int64_t bytes);

/*
 * Admit one request: RM_OK and *ticket set (tickets count up from 1), or
 * RM_E_AGAIN (not admitted: nothing kept), RM_E_UNSUPPORTED (no serving
 * kernel for its code and L), RM_E_PTR (device-resident LLRs outside every
 * registered pool), RM_E_INVAL.  May launch the open batch.
 */
int rm_server_submit(rm_server *s, const rm_request *req, uint64_t *ticket);

/*
 * Non-blocking progress: retire finished batches, write up to `max`
 * completions (oldest batch first) and launch the open batch if a device
 * slot is free.  Returns the number of completions written (>= 0) or an
 * error code.  Completions not written stay queued for the next call.
 */
int rm_server_poll(rm_server *s, rm_completion *out, int max);

/* Admitted requests whose completion has not yet been returned by poll. */
int64_t rm_server_pending(const rm_server *s);

/*
 * Open-loop trace replay (load generator, runs on the calling thread):
 * request i is submitted at t0 + arrival_us[i] (t0 = call time; arrival
 * times non-decreasing), or as soon after as it is admitted; the call polls
 * until every request has completed and writes latency_us[i] = completion
 * time - (t0 + arrival_us[i]).  Requests' t_arrival_us fields are ignored.
 * stats (may be NULL) receives: [0] elapsed us, [1] batches launched,
 * [2] refused submit attempts, [3] largest batch.
 */
int rm_server_run_trace(rm_server *s, const rm_request *reqs, const double *arrival_us, int64_t n,
                        double *latency_us, double *stats);

/* Release after all device work completes; pending completions are dropped.  NULL-safe. */
void rm_server_destroy(rm_server *s);

#ifdef __cplusplus
}
#endif
#endif
