// rmdec_mixed.hip -- fused mixed-code launch: one persistent kernel decodes
// the frames of several codes from a device work queue (C ABI in rmdec.h).
#include <hip/hip_runtime.h>

#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rmdec.h"
#include "rmdec_internal.hpp"

using namespace rmdec;

namespace {

// The codes compiled into the fused kernel: RM(2,7), RM(2,8), RM(2,9) and
// RM(2,10), list size 4; four decoders per wavefront for RM(2,7) and
// RM(2,8), two for RM(2,9), one for RM(2,10) (the per-code kernels make the
// same choices).  The four bodies are held to 128 VGPRs, 4 waves per SIMD
// like the per-code kernels (left to the cap of 3 they take 132 and run 3).
constexpr int kWPE = 4;

constexpr int kFused[][3] = {{7, 2, 4}, {8, 2, 4}, {9, 2, 4}, {10, 2, 4}};
constexpr int kNumFused = 4;
constexpr int kFusedBytes = MaxBytes<Code<7, 2, 4, 4>, Code<8, 2, 4, 4>, Code<9, 2, 4, 2>, Code<10, 2, 4, 1>>::value;

const void *fused_kernel()
{
    return (const void *)&rm_mixed_kernel<kWPE, Code<7, 2, 4, 4>, Code<8, 2, 4, 4>, Code<9, 2, 4, 2>, Code<10, 2, 4, 1>>;
}

hipError_t launch_fused(const MixedArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((rm_mixed_kernel<kWPE, Code<7, 2, 4, 4>, Code<8, 2, 4, 4>, Code<9, 2, 4, 2>, Code<10, 2, 4, 1>>),
                       dim3(blocks), dim3(kWave * a.waves), (size_t)a.waves * kFusedBytes, s, a);
    return hipGetLastError();
}

// Clears the queue head before each fused launch (a kernel rather than a
// memset, so that the step can sit in a captured graph).
__global__ void rm_reset_head(uint32_t *head) { *head = 0u; }

int fused_slot(int m, int r, int L)
{
    for (int i = 0; i < kNumFused; i++)
        if (kFused[i][0] == m && kFused[i][1] == r && kFused[i][2] == L)
            return i;
    return -1;
}

} // namespace

// A device work queue: the entries and the head counter the waves claim
// entries with.
struct Queue {
    Tile *tiles = nullptr;
    uint32_t *head = nullptr;
    int64_t cap = 0;
};

struct rm_mixed {
    hipStream_t stream = nullptr;
    int device = 0;
    Queue q;                     // queue of rm_mixed_decode
    Tile *h_stage = nullptr;     // pinned staging of q's entries
    hipEvent_t staged = nullptr; // recorded once the last upload has read h_stage
    int blocks = 0, waves = 0;
    Queue gq; // queue owned by the captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_queue(Queue &q)
{
    if (q.tiles)
        (void)hipFree(q.tiles);
    if (q.head)
        (void)hipFree(q.head);
    q = Queue{};
}

hipError_t alloc_queue(Queue &q, int64_t cap)
{
    hipError_t e = hipMalloc((void **)&q.tiles, (size_t)cap * sizeof(Tile));
    if (e == hipSuccess)
        e = hipMalloc((void **)&q.head, sizeof(uint32_t));
    if (e != hipSuccess)
        free_queue(q);
    else
        q.cap = cap;
    return e;
}

void drop_graph(rm_mixed *mx)
{
    if (mx->exec)
        (void)hipGraphExecDestroy(mx->exec);
    if (mx->graph)
        (void)hipGraphDestroy(mx->graph);
    mx->exec = nullptr;
    mx->graph = nullptr;
    free_queue(mx->gq);
}

// Queue of one launch.  The segments are taken in descending order of the
// work of one of their frames (P decoders of L paths over N log N), so that
// the most expensive entries are claimed first and the cheapest last
// (longest processing time first); each is cut into runs of its tile_frames
// frames, except that the last `tail` frames of the last segment in that
// order get one entry each, so the waves run out of work within about one
// of its frames of each other.  Segments without frames come first and add
// no entries.  Entry k of the queue is a function of k (tile_at), which the
// host and the no-alloc path's fill kernel both evaluate.
struct QueuePlan {
    int n_segs;
    int order[kMaxSegments];          // segment at queue position j
    int64_t n_frames[kMaxSegments];   // by segment index
    uint32_t tf[kMaxSegments];        // by segment index
    int64_t split;                    // frames of the last position cut into runs; the rest one per entry
    int64_t start[kMaxSegments + 1];  // first entry of position j; start[n_segs] = entries in all
};

__host__ __device__ inline Tile tile_at(const QueuePlan &p, int64_t k)
{
    int j = 0;
    while (j + 1 < p.n_segs && k >= p.start[j + 1])
        j++;
    const int i = p.order[j];
    const int64_t tf = p.tf[i];
    const int64_t lim = j == p.n_segs - 1 ? p.split : p.n_frames[i];
    const int64_t runs = (lim + tf - 1) / tf;
    const int64_t r = k - p.start[j];
    if (r < runs) {
        const int64_t first = r * tf;
        return Tile{(uint32_t)i, (uint32_t)first, (uint32_t)(lim - first < tf ? lim - first : tf), 0u};
    }
    return Tile{(uint32_t)i, (uint32_t)(lim + (r - runs)), 1u, 0u};
}

// Segment order and entry counts, for a persistent grid of `waves` waves and
// a queue of `cap` entries: the single-frame tail is at most 2 * waves frames
// and only as long as the queue has room for (none if even the plain runs
// exceed cap, which the callers then reject).
void plan_queue(QueuePlan &p, const MixedArgs &a, int64_t waves, int64_t cap)
{
    double cost[kMaxSegments];
    for (int i = 0; i < p.n_segs; i++) {
        const int m = kFused[a.code[i]][0];
        cost[i] = p.n_frames[i] > 0 ? (double)a.seg[i].P * kFused[a.code[i]][2] * (double)(1 << m) * m : -1.0;
        p.order[i] = i;
    }
    for (int i = 1; i < p.n_segs; i++) // stable insertion sort, empty segments first, then most expensive first
        for (int j = i; j > 0; j--) {
            const int x = p.order[j], y = p.order[j - 1];
            const bool before = cost[x] < 0.0 ? cost[y] >= 0.0 : (cost[y] >= 0.0 && cost[x] > cost[y]);
            if (!before)
                break;
            p.order[j] = y;
            p.order[j - 1] = x;
        }
    const int last = p.order[p.n_segs - 1];
    const int64_t n = p.n_frames[last], tf = p.tf[last];
    int64_t others = 0;
    for (int j = 0; j + 1 < p.n_segs; j++)
        others += (p.n_frames[p.order[j]] + p.tf[p.order[j]] - 1) / p.tf[p.order[j]];
    // entries with the last t frames one per entry: non-decreasing in t
    auto entries = [&](int64_t t) { return others + (n - t + tf - 1) / tf + t; };
    int64_t lo = 0, hi = 2 * waves < n ? 2 * waves : n;
    if (entries(0) > cap)
        hi = 0;
    while (lo < hi) { // largest t <= hi with entries(t) <= cap
        const int64_t mid = (lo + hi + 1) / 2;
        if (entries(mid) <= cap)
            lo = mid;
        else
            hi = mid - 1;
    }
    p.split = n - lo;
    p.start[0] = 0;
    for (int j = 0; j < p.n_segs; j++) {
        const int i = p.order[j];
        const int64_t lim = j == p.n_segs - 1 ? p.split : p.n_frames[i];
        p.start[j + 1] = p.start[j] + (lim + p.tf[i] - 1) / p.tf[i] + (p.n_frames[i] - lim);
    }
}

// Validate the segments and fill the per-segment kernel arguments and the
// plan's frame counts and run lengths.
int check_segments(const rm_segment *segs, int n_segs, MixedArgs &a, QueuePlan &p)
{
    if (!segs)
        return fail(RM_E_INVAL, "null argument");
    if (n_segs < 1 || n_segs > RM_MIXED_MAX_SEGMENTS)
        return fail(RM_E_INVAL, "n_segs must be in [1, RM_MIXED_MAX_SEGMENTS]");
    memset(&a, 0, sizeof a);
    memset(&p, 0, sizeof p);
    p.n_segs = n_segs;
    uint32_t *tf = p.tf;
    for (int i = 0; i < n_segs; i++) {
        const rm_segment &g = segs[i];
        if (!g.dec)
            return fail(RM_E_INVAL, "segment without decoder");
        if (g.n_frames < 0)
            return fail(RM_E_INVAL, "n_frames < 0");
        if (g.n_frames > 0xFFFFFFFFll)
            return fail(RM_E_INVAL, "segment too long for one launch");
        if (g.dec->cfg.perm_mode == RM_PERM_FRESH)
            return fail(RM_E_UNSUPPORTED, "fresh-permutation decoders run through rm_decode_batch only");
        const int slot = fused_slot(g.dec->cfg.m, g.dec->cfg.r, g.dec->cfg.L);
        if (slot < 0)
            return fail(RM_E_UNSUPPORTED, "code not compiled into the fused kernel");
        if (g.tile_frames < 0 || g.tile_frames > 64)
            return fail(RM_E_INVAL, "tile_frames must be in [1, 64] (0: library default)");
        tf[i] = g.tile_frames == 0 ? 4u : (uint32_t)g.tile_frames;
        if (g.n_frames > 0) {
            if (!g.llr || !g.out_bits)
                return fail(RM_E_INVAL, "null llr or out_bits");
            int rc = check_device_ptr(g.llr, "llr");
            if (rc == RM_OK)
                rc = check_device_ptr(g.out_bits, "out_bits");
            if (rc == RM_OK && g.out_metric)
                rc = check_device_ptr(g.out_metric, "out_metric");
            if (rc == RM_OK)
                rc = check_alignment(g.dec->N, g.llr, g.out_bits, g.out_metric);
            if (rc != RM_OK)
                return rc;
        }
        a.seg[i] = batch_args(g.dec, g.llr, g.n_frames, g.out_bits, g.out_metric);
        a.code[i] = slot;
        p.n_frames[i] = g.n_frames;
    }
    return RM_OK;
}

// persistent grid: the blocks the device holds at once
int occupancy_blocks(int device, int waves)
{
    int per_cu = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel(), kWave * waves,
                                                                (size_t)waves * kFusedBytes);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || per_cu < 1 || cus < 1)
        return 256 * 4;
    return per_cu * cus;
}

int grid_blocks(rm_mixed *mx, int waves)
{
    return mx->blocks ? mx->blocks : occupancy_blocks(mx->device, waves);
}

// Validate, fill the kernel arguments and build the queue entries on the host.
int prepare(rm_mixed *mx, const rm_segment *segs, int n_segs, MixedArgs &a, std::vector<Tile> &tiles)
{
    if (!mx)
        return fail(RM_E_INVAL, "null launcher");
    QueuePlan p;
    int rc = check_segments(segs, n_segs, a, p);
    if (rc != RM_OK)
        return rc;
    a.waves = mx->waves ? mx->waves : 2;
    plan_queue(p, a, (int64_t)grid_blocks(mx, a.waves) * a.waves, mx->q.cap);
    const int64_t total = p.start[n_segs];
    if (total > mx->q.cap)
        return fail(RM_E_INVAL, "more queue entries than the launcher was created for");
    tiles.resize((size_t)total);
    for (int64_t k = 0; k < total; k++)
        tiles[(size_t)k] = tile_at(p, k);
    a.n_tiles = (uint32_t)total;
    return RM_OK;
}

// Queue the head reset and the persistent kernel on the launcher's stream.
int enqueue(rm_mixed *mx, const MixedArgs &a, int blocks)
{
    hipLaunchKernelGGL(rm_reset_head, dim3(1), dim3(1), 0, mx->stream, a.head);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && a.n_tiles > 0)
        e = launch_fused(a, blocks, mx->stream);
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("fused launch: ") + hipGetErrorString(e));
    return RM_OK;
}

} // namespace

extern "C" {

int rm_mixed_supported(int m, int r, int L) { return fused_slot(m, r, L) >= 0; }

rm_mixed *rm_mixed_create(int64_t max_tiles)
{
    if (max_tiles < 1 || max_tiles > (int64_t)1 << 30) {
        fail(RM_E_INVAL, "max_tiles must be in [1, 2^30]");
        return nullptr;
    }
    rm_mixed *mx = new (std::nothrow) rm_mixed();
    if (!mx) {
        fail(RM_E_NOMEM, "host allocation failed");
        return nullptr;
    }
    hipError_t e = hipGetDevice(&mx->device);
    if (e == hipSuccess)
        e = alloc_queue(mx->q, max_tiles);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&mx->h_stage, (size_t)max_tiles * sizeof(Tile), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&mx->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        fail(RM_E_HIP, std::string("HIP error at create: ") + hipGetErrorString(e));
        rm_mixed_destroy(mx);
        return nullptr;
    }
    g_err.clear();
    return mx;
}

int rm_mixed_set_stream(rm_mixed *mx, void *hip_stream)
{
    if (!mx)
        return fail(RM_E_INVAL, "null launcher");
    mx->stream = (hipStream_t)hip_stream;
    return RM_OK;
}

int rm_mixed_set_grid(rm_mixed *mx, int blocks, int waves_per_block)
{
    if (!mx)
        return fail(RM_E_INVAL, "null launcher");
    if (blocks < 0 || waves_per_block < 0 || waves_per_block > 4)
        return fail(RM_E_INVAL, "blocks >= 0 and waves_per_block in [0, 4]");
    if ((size_t)(waves_per_block ? waves_per_block : 2) * kFusedBytes > 65536)
        return fail(RM_E_UNSUPPORTED, "LDS slices do not fit the requested waves per block");
    mx->blocks = blocks;
    mx->waves = waves_per_block;
    return RM_OK;
}

int rm_mixed_decode(rm_mixed *mx, const rm_segment *segs, int n_segs)
{
    MixedArgs a;
    std::vector<Tile> tiles;
    int rc = prepare(mx, segs, n_segs, a, tiles);
    if (rc != RM_OK)
        return rc;
    // The upload is ordered on the stream after the previous launch that
    // read the queue; the staging buffer is reused once that upload is done.
    hipError_t e = hipEventSynchronize(mx->staged);
    if (e == hipSuccess && !tiles.empty()) {
        memcpy(mx->h_stage, tiles.data(), tiles.size() * sizeof(Tile));
        e = hipMemcpyAsync(mx->q.tiles, mx->h_stage, tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                           mx->stream);
        if (e == hipSuccess)
            e = hipEventRecord(mx->staged, mx->stream);
    }
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("queue upload: ") + hipGetErrorString(e));
    a.tiles = mx->q.tiles;
    a.head = mx->q.head;
    return enqueue(mx, a, grid_blocks(mx, a.waves));
}

int rm_mixed_capture(rm_mixed *mx, const rm_segment *segs, int n_segs)
{
    MixedArgs a;
    std::vector<Tile> tiles;
    int rc = prepare(mx, segs, n_segs, a, tiles);
    if (rc != RM_OK)
        return rc;
    if (!mx->stream)
        return fail(RM_E_INVAL, "graph capture needs a non-null stream");
    drop_graph(mx);
    // the graph gets a queue of its own, filled once, here
    hipError_t e = alloc_queue(mx->gq, tiles.empty() ? 1 : (int64_t)tiles.size());
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(mx->gq.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        drop_graph(mx);
        return fail(RM_E_HIP, std::string("graph queue: ") + hipGetErrorString(e));
    }
    a.tiles = mx->gq.tiles;
    a.head = mx->gq.head;
    const int blocks = grid_blocks(mx, a.waves);
    e = hipStreamBeginCapture(mx->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        drop_graph(mx);
        return fail(RM_E_HIP, std::string("begin capture: ") + hipGetErrorString(e));
    }
    rc = enqueue(mx, a, blocks);
    e = hipStreamEndCapture(mx->stream, &mx->graph);
    if (rc != RM_OK) {
        drop_graph(mx);
        return rc;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&mx->exec, mx->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(mx);
        return fail(RM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    return RM_OK;
}

int rm_mixed_replay(rm_mixed *mx)
{
    if (!mx)
        return fail(RM_E_INVAL, "null launcher");
    if (!mx->exec)
        return fail(RM_E_INVAL, "nothing captured");
    hipError_t e = hipGraphLaunch(mx->exec, mx->stream);
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
    return RM_OK;
}

// ---------------------------------------------------------------------------
// autotuner: times the fused launch on the caller's segments and keeps the
// fastest waves per block and frames per queue entry (per segment)
// ---------------------------------------------------------------------------
namespace {

int time_config(rm_mixed *mx, const rm_segment *segs, int n_segs, const int *tf, int waves, int reps,
                hipEvent_t e0, hipEvent_t e1, float *ms)
{
    rm_segment local[RM_MIXED_MAX_SEGMENTS];
    for (int i = 0; i < n_segs; i++) {
        local[i] = segs[i];
        local[i].tile_frames = tf[i];
    }
    const int saved = mx->waves;
    mx->waves = waves;
    int rc = rm_mixed_decode(mx, local, n_segs); // warm-up
    hipError_t e = hipSuccess;
    if (rc == RM_OK)
        e = hipEventRecord(e0, mx->stream);
    for (int k = 0; rc == RM_OK && e == hipSuccess && k < reps; k++)
        rc = rm_mixed_decode(mx, local, n_segs);
    if (rc == RM_OK && e == hipSuccess)
        e = hipEventRecord(e1, mx->stream);
    if (rc == RM_OK && e == hipSuccess)
        e = hipEventSynchronize(e1);
    if (rc == RM_OK && e == hipSuccess)
        e = hipEventElapsedTime(ms, e0, e1);
    mx->waves = saved;
    if (rc != RM_OK)
        return rc;
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("autotune timing: ") + hipGetErrorString(e));
    *ms /= (float)reps;
    return RM_OK;
}

} // namespace

int rm_mixed_autotune(rm_mixed *mx, const rm_segment *segs, int n_segs, int reps, rm_mixed_tuning *out)
{
    if (!mx || !segs || !out)
        return fail(RM_E_INVAL, "null argument");
    if (n_segs < 1 || n_segs > RM_MIXED_MAX_SEGMENTS)
        return fail(RM_E_INVAL, "n_segs must be in [1, RM_MIXED_MAX_SEGMENTS]");
    if (reps < 1 || reps > 100)
        return fail(RM_E_INVAL, "reps must be in [1, 100]");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return fail(RM_E_HIP, std::string("autotune events: ") + hipGetErrorString(e));
    }
    static const int kTiles[] = {1, 2, 4, 8, 16};
    static const int kWaves[] = {1, 2, 4};
    int tf[RM_MIXED_MAX_SEGMENTS];
    int best_tf[RM_MIXED_MAX_SEGMENTS];
    for (int i = 0; i < n_segs; i++)
        tf[i] = best_tf[i] = 4;
    int best_w = 0, trials = 0, rc = RM_OK;
    float best = 3.4e38f, ms = 0.f;
    auto trial = [&](int w) {
        rc = time_config(mx, segs, n_segs, tf, w, reps, e0, e1, &ms);
        trials++;
        if (rc == RM_OK && ms < best) {
            best = ms;
            best_w = w;
            for (int i = 0; i < n_segs; i++)
                best_tf[i] = tf[i];
        }
    };
    // 1: waves per block, 4 frames per entry
    for (int w : kWaves) {
        if ((size_t)w * kFusedBytes > 65536)
            continue;
        trial(w);
        if (rc != RM_OK)
            break;
    }
    // 2: one frames-per-entry value for all segments
    for (int k = 0; rc == RM_OK && k < 5; k++) {
        if (kTiles[k] == 4)
            continue;
        for (int i = 0; i < n_segs; i++)
            tf[i] = kTiles[k];
        trial(best_w);
    }
    // 3: each segment's own value, the others held at the best so far
    for (int i = 0; rc == RM_OK && n_segs > 1 && i < n_segs; i++) {
        for (int k = 0; rc == RM_OK && k < 5; k++) {
            for (int j = 0; j < n_segs; j++)
                tf[j] = best_tf[j];
            if (kTiles[k] == best_tf[i])
                continue;
            tf[i] = kTiles[k];
            trial(best_w);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != RM_OK)
        return rc;
    mx->waves = best_w;
    memset(out, 0, sizeof *out);
    out->blocks = mx->blocks;
    out->waves_per_block = best_w;
    for (int i = 0; i < n_segs; i++)
        out->tile_frames[i] = best_tf[i];
    out->ms = best;
    out->trials = trials;
    return RM_OK;
}

void rm_mixed_destroy(rm_mixed *mx)
{
    if (!mx)
        return;
    (void)hipStreamSynchronize(mx->stream);
    drop_graph(mx);
    free_queue(mx->q);
    if (mx->h_stage)
        (void)hipHostFree(mx->h_stage);
    if (mx->staged)
        (void)hipEventDestroy(mx->staged);
    delete mx;
}

} // extern "C"

// ---------------------------------------------------------------------------
// Fused launch that allocates nothing: the queue entries and the queue head
// live in one statically sized device array instead of a launcher's buffers.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kStaticTiles = RM_MIXED_STATIC_MAX_TILES;
constexpr int kHeadWords = 64; // the head counter, alone in the first 256 bytes
// [head, pad .. ][Tile x kStaticTiles]: 256 B + 8 MiB on every device the library runs on
__device__ __align__(256) uint32_t scratch[kHeadWords + kStaticTiles * (sizeof(Tile) / 4)];

// Writes the queue entries of the plan (thread k: entry k) and clears the
// head, so the fill and the decode can sit in a captured graph.
__global__ void rm_fill_static_queue(QueuePlan p, Tile *tiles, uint32_t *head)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0)
        *head = 0u;
    if (k < p.start[p.n_segs])
        tiles[k] = tile_at(p, k);
}

// Device address of `scratch` on each device, looked up once per device with
// that device current (each device holds its own copy of the array).
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
uint32_t *g_static_ptr[kMaxDevices];
int g_static_blocks[kMaxDevices][5];

int static_scratch(int device, int waves, uint32_t **ptr, int *blocks)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(RM_E_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RM_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
        g_static_ptr[device] = (uint32_t *)p;
    }
    if (!g_static_blocks[device][waves])
        g_static_blocks[device][waves] = occupancy_blocks(device, waves);
    *ptr = g_static_ptr[device];
    *blocks = g_static_blocks[device][waves];
    return RM_OK;
}

} // namespace

extern "C" int rm_mixed_decode_static(const rm_segment *segs, int n_segs, int waves_per_block, void *hip_stream)
{
    if (waves_per_block < 0 || waves_per_block > 4)
        return fail(RM_E_INVAL, "waves_per_block must be in [0, 4]");
    const int waves = waves_per_block ? waves_per_block : 2;
    if ((size_t)waves * kFusedBytes > 65536)
        return fail(RM_E_UNSUPPORTED, "LDS slices do not fit the requested waves per block");
    MixedArgs a;
    QueuePlan p;
    int rc = check_segments(segs, n_segs, a, p);
    if (rc != RM_OK)
        return rc;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("current device: ") + hipGetErrorString(e));
    uint32_t *base = nullptr;
    int blocks = 0;
    rc = static_scratch(device, waves, &base, &blocks);
    if (rc != RM_OK)
        return rc;
    plan_queue(p, a, (int64_t)blocks * waves, kStaticTiles);
    const int64_t total = p.start[n_segs];
    if (total > kStaticTiles)
        return fail(RM_E_INVAL, "more queue entries than RM_MIXED_STATIC_MAX_TILES (use larger tile_frames)");
    if (total == 0)
        return RM_OK;
    Tile *tiles = (Tile *)(base + kHeadWords);
    const hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(rm_fill_static_queue, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, p, tiles, base);
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("queue fill: ") + hipGetErrorString(e));
    a.tiles = tiles;
    a.head = base;
    a.n_tiles = (uint32_t)total;
    a.waves = waves;
    e = launch_fused(a, blocks, s);
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("fused launch: ") + hipGetErrorString(e));
    return RM_OK;
}
