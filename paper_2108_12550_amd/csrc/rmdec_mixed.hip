// rmdec_mixed.hip -- fused mixed-code launch: one persistent kernel decodes
// the frames of several codes from a device work queue (C ABI in rmdec.h).
#include <hip/hip_runtime.h>

#include <string.h>

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
// same choices).  Under the cap of 3 waves per SIMD the four bodies
// together hold 128 VGPRs, so the kernel runs 4 waves per SIMD.
constexpr int kWPE = 3;

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

// Validate the segments, fill the per-segment kernel arguments and build the
// queue entries: every segment cut into runs of tile_frames frames, the runs
// of all segments interleaved round-robin.
int prepare(rm_mixed *mx, const rm_segment *segs, int n_segs, MixedArgs &a, std::vector<Tile> &tiles)
{
    if (!mx || !segs)
        return fail(RM_E_INVAL, "null argument");
    if (n_segs < 1 || n_segs > RM_MIXED_MAX_SEGMENTS)
        return fail(RM_E_INVAL, "n_segs must be in [1, RM_MIXED_MAX_SEGMENTS]");
    memset(&a, 0, sizeof a);
    std::vector<int64_t> runs(n_segs);
    std::vector<int> tf(n_segs);
    int64_t total = 0, longest = 0;
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
        tf[i] = g.tile_frames == 0 ? 4 : g.tile_frames;
        if (tf[i] < 1 || tf[i] > 64)
            return fail(RM_E_INVAL, "tile_frames must be in [1, 64]");
        if (g.n_frames > 0) {
            if (!g.llr || !g.out_bits)
                return fail(RM_E_INVAL, "null llr or out_bits");
            int rc = check_device_ptr(g.llr, "llr");
            if (rc == RM_OK)
                rc = check_device_ptr(g.out_bits, "out_bits");
            if (rc == RM_OK && g.out_metric)
                rc = check_device_ptr(g.out_metric, "out_metric");
            if (rc != RM_OK)
                return rc;
        }
        a.seg[i] = batch_args(g.dec, g.llr, g.n_frames, g.out_bits, g.out_metric);
        a.code[i] = slot;
        runs[i] = (g.n_frames + tf[i] - 1) / tf[i];
        total += runs[i];
        longest = runs[i] > longest ? runs[i] : longest;
    }
    if (total > mx->q.cap)
        return fail(RM_E_INVAL, "more queue entries than the launcher was created for");
    tiles.clear();
    tiles.reserve((size_t)total);
    for (int64_t q = 0; q < longest; q++)
        for (int i = 0; i < n_segs; i++)
            if (q < runs[i]) {
                const int64_t first = q * tf[i];
                const int64_t cnt = segs[i].n_frames - first < tf[i] ? segs[i].n_frames - first : tf[i];
                tiles.push_back(Tile{(uint32_t)i, (uint32_t)first, (uint32_t)cnt, 0u});
            }
    a.n_tiles = (uint32_t)tiles.size();
    a.waves = mx->waves ? mx->waves : 2;
    return RM_OK;
}

int grid_blocks(rm_mixed *mx, int waves)
{
    if (mx->blocks)
        return mx->blocks;
    int per_cu = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel(), kWave * waves,
                                                                (size_t)waves * kFusedBytes);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, mx->device);
    if (e != hipSuccess || per_cu < 1 || cus < 1)
        return 256 * 4;
    return per_cu * cus;
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
