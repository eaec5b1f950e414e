// rmdec_serve.hip -- request server (C ABI in rmdec.h): continuous batching
// of single-frame requests over the serving kernels of rmdec_serve.hpp.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "rmdec.h"
#include "rmdec_internal.hpp"
#include "rmdec_serve.hpp"

using namespace rmdec;

namespace {

constexpr int kMaxSegs = 64;   // distinct decoders in one batch
constexpr int kGroups = 3;     // serving kernels: list sizes 1, 4, 8
constexpr int kMaxPools = 16;

int group_of(int L) { return L == 1 ? 0 : L == 4 ? 1 : L == 8 ? 2 : -1; }

const ServeGroup &group(int g)
{
    static const ServeGroup gs[kGroups] = {serve_group_l1(), serve_group_l4(), serve_group_l8()};
    return gs[g];
}

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct ReqMeta {
    uint64_t ticket, tag;
    double t_arrival;
    int seg;
    int n_bytes; // N/8
    const float *llr_dev; // device address the kernel reads
    uint8_t *out_bits;
    float *out_metric;
};

// One batch buffer: pinned host staging and device copies of the tables,
// LLRs and outputs of up to max_batch requests.
struct Batch {
    enum State { FREE, OPEN, INFLIGHT, DONE } state = FREE;
    hipStream_t stream = nullptr;          // upload, list-size-1 kernel, download
    hipStream_t side[2] = {nullptr, nullptr}; // list-size-4 and -8 kernels, concurrent with the first
    hipEvent_t uploaded = nullptr, side_done[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    unsigned char *h_tab = nullptr, *d_tab = nullptr; // heads | segs | codes | jobs | tiles
    unsigned char *h_llr = nullptr, *d_llr = nullptr;
    // outputs in coherent host memory that the kernels write directly:
    // bits [max_batch][128] | metrics [max_batch] | completion words [max_batch]
    unsigned char *h_out = nullptr, *d_out = nullptr; // host address, device address
    uint32_t epoch = 0;       // value of the completion words of this launch
    int64_t llr_used = 0;
    std::vector<ReqMeta> reqs;
    // requests not yet returned by poll, per serving kernel, in the order
    // that kernel takes them
    std::vector<int> unreported[kGroups];
    const rm_decoder *seg_dec[kMaxSegs];
    int n_segs = 0;
    double t_launch = 0, t_done = 0;
};

} // namespace

struct rm_server {
    rm_server_config cfg;
    int device = 0;
    int waves = 2;                      // waves per block, one request per wave (split = 1)
    int grid_max[kGroups] = {0, 0, 0};  // resident blocks of each serving kernel
    size_t off_segs = 0, off_codes = 0, off_jobs = 0, tab_bytes = 0, out_pm_off = 0, out_done_off = 0;
    uint32_t epochs = 0;        // launches so far (each launch's completion words take the next value)
    std::vector<Batch> batches;
    int open = -1;              // index of the open batch, or -1
    int inflight = 0;           // batches launched and not yet finished
    std::deque<int> order;      // launched batches, oldest first
    uint64_t next_ticket = 0;
    int64_t pending = 0;
    int64_t launches = 0;
    int64_t largest = 0;
    const unsigned char *pool_lo[kMaxPools];
    const unsigned char *pool_hi[kMaxPools];
    int n_pools = 0;
};

namespace {

void free_batch(Batch &b)
{
    if (b.stream)
        (void)hipStreamSynchronize(b.stream);
    for (hipEvent_t ev : {b.done, b.uploaded, b.side_done[0], b.side_done[1]})
        if (ev)
            (void)hipEventDestroy(ev);
    for (hipStream_t st : {b.stream, b.side[0], b.side[1]})
        if (st)
            (void)hipStreamDestroy(st);
    for (unsigned char *p : {b.h_tab, b.h_llr, b.h_out})
        if (p)
            (void)hipHostFree(p);
    for (unsigned char *p : {b.d_tab, b.d_llr})
        if (p)
            (void)hipFree(p);
}

hipError_t alloc_batch(rm_server *s, Batch &b)
{
    const size_t out_bytes = s->out_done_off + (size_t)s->cfg.max_batch * 4;
    hipError_t e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; i++)
        e = hipStreamCreateWithFlags(&b.side[i], hipStreamNonBlocking);
    for (hipEvent_t *ev : {&b.done, &b.uploaded, &b.side_done[0], &b.side_done[1]})
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&b.h_tab, s->tab_bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&b.h_llr, (size_t)s->cfg.batch_bytes, hipHostMallocDefault);
    // coherent and mapped: the kernels' writes reach it while they run
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&b.h_out, out_bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        memset(b.h_out, 0, out_bytes); // completion words start below every epoch
        e = hipHostGetDevicePointer((void **)&b.d_out, b.h_out, 0);
    }
    if (e == hipSuccess)
        e = hipMalloc((void **)&b.d_tab, s->tab_bytes);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b.d_llr, (size_t)s->cfg.batch_bytes);
    b.reqs.reserve((size_t)s->cfg.max_batch);
    return e;
}

// Take a free batch buffer as the open batch; false if none is free.
bool open_batch(rm_server *s)
{
    if (s->open >= 0)
        return true;
    for (size_t i = 0; i < s->batches.size(); i++) {
        Batch &b = s->batches[i];
        if (b.state == Batch::FREE) {
            b.state = Batch::OPEN;
            b.llr_used = 0;
            b.reqs.clear();
            for (auto &u : b.unreported)
                u.clear();
            b.n_segs = 0;
            s->open = (int)i;
            return true;
        }
    }
    return false;
}

// Upload the open batch, launch one serving kernel per list size present
// (concurrently, on the batch's three streams) and queue the download.
int launch_open(rm_server *s)
{
    Batch &b = s->batches[s->open];
    const int n = (int)b.reqs.size();
    // tables: decoder sets, their codes, jobs grouped by list size and set
    // (sets of larger work first), tiles of up to tile_frames jobs
    KernelArgs *segs = (KernelArgs *)(b.h_tab + s->off_segs);
    int *codes = (int *)(b.h_tab + s->off_codes);
    Job *jobs = (Job *)(b.h_tab + s->off_jobs);
    Tile *tiles = (Tile *)(jobs + n);
    int count[kMaxSegs] = {0};
    for (const ReqMeta &r : b.reqs)
        count[r.seg]++;
    int seg_order[kMaxSegs];
    for (int i = 0; i < b.n_segs; i++) {
        const rm_decoder *d = b.seg_dec[i];
        segs[i] = batch_args(d, nullptr, 0, nullptr, nullptr);
        codes[i] = serve_code_index(d->cfg.m, d->cfg.r);
        seg_order[i] = i;
    }
    auto work = [&](int i) { return (int64_t)b.seg_dec[i]->N * b.seg_dec[i]->cfg.P * b.seg_dec[i]->cfg.L; };
    std::sort(seg_order, seg_order + b.n_segs, [&](int x, int y) {
        const int gx = group_of(b.seg_dec[x]->cfg.L), gy = group_of(b.seg_dec[y]->cfg.L);
        return gx != gy ? gx < gy : work(x) > work(y);
    });
    int first_job[kMaxSegs];
    int cursor = 0;
    for (int k = 0; k < b.n_segs; k++) {
        first_job[seg_order[k]] = cursor;
        cursor += count[seg_order[k]];
    }
    int fill[kMaxSegs];
    memcpy(fill, first_job, sizeof fill);
    for (int i = 0; i < n; i++) {
        const ReqMeta &r = b.reqs[i];
        jobs[fill[r.seg]++] = Job{r.llr_dev, (uint32_t)i, 0u};
    }
    // poll scans each kernel's requests in the order the kernel takes them
    for (int k = 0; k < n; k++) {
        const int i = (int)jobs[k].out;
        b.unreported[group_of(b.seg_dec[b.reqs[(size_t)i].seg]->cfg.L)].push_back(i);
    }
    b.epoch = ++s->epochs == 0 ? ++s->epochs : s->epochs; // never 0, the words' initial value
    const int tf = s->cfg.tile_frames;
    int n_tiles = 0;
    int g_first[kGroups] = {0, 0, 0}, g_count[kGroups] = {0, 0, 0};
    for (int k = 0; k < b.n_segs; k++) {
        const int i = seg_order[k];
        const int g = group_of(b.seg_dec[i]->cfg.L);
        if (g_count[g] == 0)
            g_first[g] = n_tiles;
        for (int q = 0; q < count[i]; q += tf) {
            tiles[n_tiles++] = Tile{(uint32_t)i, (uint32_t)(first_job[i] + q), (uint32_t)std::min(tf, count[i] - q), 0u};
            g_count[g]++;
        }
    }
    memset(b.h_tab, 0, 16); // queue heads, one per serving kernel
    const size_t tab_used = (size_t)((unsigned char *)(tiles + n_tiles) - b.h_tab);
    hipError_t e = hipMemcpyAsync(b.d_tab, b.h_tab, tab_used, hipMemcpyHostToDevice, b.stream);
    if (e == hipSuccess && b.llr_used > 0)
        e = hipMemcpyAsync(b.d_llr, b.h_llr, (size_t)b.llr_used, hipMemcpyHostToDevice, b.stream);
    if (e == hipSuccess && (g_count[1] || g_count[2]))
        e = hipEventRecord(b.uploaded, b.stream);
    // the heaviest list size first
    for (int g = kGroups - 1; e == hipSuccess && g >= 0; g--) {
        if (g_count[g] == 0)
            continue;
        hipStream_t st = g == 0 ? b.stream : b.side[g - 1];
        if (g > 0)
            e = hipStreamWaitEvent(st, b.uploaded, 0);
        if (e != hipSuccess)
            break;
        ServeArgs a;
        a.segs = (const KernelArgs *)(b.d_tab + s->off_segs);
        a.seg_code = (const int *)(b.d_tab + s->off_codes);
        a.jobs = (const Job *)(b.d_tab + s->off_jobs);
        a.tiles = (const Tile *)(b.d_tab + ((unsigned char *)(tiles + g_first[g]) - b.h_tab));
        a.n_tiles = (uint32_t)g_count[g];
        a.head = (uint32_t *)b.d_tab + g;
        a.out_bits = b.d_out;
        a.out_pm = (float *)(b.d_out + s->out_pm_off);
        a.done = (uint32_t *)(b.d_out + s->out_done_off);
        a.epoch = b.epoch;
        if (s->cfg.split > 1) {
            // one queue entry per workgroup at a time, its requests split over the waves
            e = group(g).launch_split(a, std::min(g_count[g], s->grid_max[g]), s->cfg.split, st);
        } else {
            const int want = (g_count[g] + s->waves - 1) / s->waves;
            e = group(g).launch(a, std::min(want, s->grid_max[g]), s->waves, st);
        }
        if (e == hipSuccess && g > 0)
            e = hipEventRecord(b.side_done[g - 1], st);
    }
    for (int g = 1; e == hipSuccess && g < kGroups; g++)
        if (g_count[g])
            e = hipStreamWaitEvent(b.stream, b.side_done[g - 1], 0);
    if (e == hipSuccess)
        e = hipEventRecord(b.done, b.stream);
    if (e != hipSuccess)
        return fail(RM_E_HIP, std::string("serving launch: ") + hipGetErrorString(e));
    b.state = Batch::INFLIGHT;
    b.t_launch = now_us();
    s->order.push_back(s->open);
    s->open = -1;
    s->inflight++;
    s->launches++;
    s->largest = std::max<int64_t>(s->largest, n);
    return RM_OK;
}

int maybe_launch(rm_server *s)
{
    if (s->open >= 0 && !s->batches[s->open].reqs.empty() && s->inflight < s->cfg.depth)
        return launch_open(s);
    return RM_OK;
}

// Mark finished batches; returns RM_OK or an error.
int retire(rm_server *s)
{
    for (int i : s->order) {
        Batch &b = s->batches[i];
        if (b.state != Batch::INFLIGHT)
            continue;
        const hipError_t e = hipEventQuery(b.done);
        if (e == hipErrorNotReady)
            continue;
        if (e != hipSuccess)
            return fail(RM_E_HIP, std::string("serving batch: ") + hipGetErrorString(e));
        b.state = Batch::DONE;
        b.t_done = now_us();
        s->inflight--;
    }
    return RM_OK;
}

} // namespace

extern "C" {

double rm_server_now_us(void) { return now_us(); }

int rm_server_supported(int m, int r, int L) { return serve_code_index(m, r) >= 0 && group_of(L) >= 0; }

rm_server *rm_server_create(const rm_server_config *cfg)
{
    if (!cfg) {
        fail(RM_E_INVAL, "null config");
        return nullptr;
    }
    rm_server_config c = *cfg;
    if (c.tile_frames == 0)
        c.tile_frames = 2;
    if (c.split == 0)
        c.split = 4;
    if (c.batch_bytes < 4096 || c.batch_bytes > ((int64_t)1 << 34) || c.max_batch < 1 || c.max_batch > 65536 ||
        c.depth < 1 || c.depth > 4 || c.tile_frames < 1 || c.tile_frames > 64 ||
        (c.split != 1 && c.split != 2 && c.split != 4)) {
        fail(RM_E_INVAL, "config outside batch_bytes [4096, 2^34], max_batch [1, 65536], depth [1, 4], "
                         "tile_frames [1, 64], split in {1, 2, 4}");
        return nullptr;
    }
    rm_server *s = new (std::nothrow) rm_server();
    if (!s) {
        fail(RM_E_NOMEM, "host allocation failed");
        return nullptr;
    }
    s->cfg = c;
    s->off_segs = 64;
    s->off_codes = s->off_segs + kMaxSegs * sizeof(KernelArgs);
    s->off_jobs = align_up(s->off_codes + kMaxSegs * sizeof(int), 16);
    s->tab_bytes = s->off_jobs + (size_t)c.max_batch * (sizeof(Job) + sizeof(Tile));
    s->out_pm_off = (size_t)c.max_batch * kServeBitsStride;
    s->out_done_off = s->out_pm_off + (size_t)c.max_batch * 4;
    hipError_t e = hipGetDevice(&s->device);
    int cus = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    const int bw = c.split > 1 ? c.split : s->waves; // waves per block
    for (int g = 0; e == hipSuccess && g < kGroups; g++) {
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c.split > 1 ? group(g).split_kernel : group(g).kernel,
                                                         kWave * bw,
                                                         (size_t)bw * group(g).lds_bytes_per_wave + (c.split > 1 ? kSplitXBytes : 0));
        s->grid_max[g] = std::max(1, per_cu * cus);
    }
    s->batches.resize((size_t)c.depth + 1);
    for (size_t i = 0; e == hipSuccess && i < s->batches.size(); i++)
        e = alloc_batch(s, s->batches[i]);
    if (e != hipSuccess) {
        fail(RM_E_HIP, std::string("HIP error at server create: ") + hipGetErrorString(e));
        rm_server_destroy(s);
        return nullptr;
    }
    g_err.clear();
    return s;
}

int rm_server_register_pool(rm_server *s, const void *base, int64_t bytes)
{
    if (!s || !base || bytes <= 0)
        return fail(RM_E_INVAL, "null server, null base or empty pool");
    if (s->n_pools == kMaxPools)
        return fail(RM_E_INVAL, "too many pools");
    int rc = check_device_ptr(base, "pool");
    if (rc == RM_OK)
        rc = check_device_ptr((const unsigned char *)base + bytes - 1, "pool end");
    if (rc != RM_OK)
        return rc;
    s->pool_lo[s->n_pools] = (const unsigned char *)base;
    s->pool_hi[s->n_pools] = (const unsigned char *)base + bytes;
    s->n_pools++;
    return RM_OK;
}

int rm_server_submit(rm_server *s, const rm_request *req, uint64_t *ticket)
{
    if (!s || !req || !req->dec || !req->llr)
        return fail(RM_E_INVAL, "null server, request, decoder or llr");
    const rm_decoder *d = req->dec;
    if (!rm_server_supported(d->cfg.m, d->cfg.r, d->cfg.L))
        return fail(RM_E_UNSUPPORTED, "no serving kernel for this code and list size");
    if (d->cfg.perm_mode == RM_PERM_FRESH)
        return fail(RM_E_UNSUPPORTED, "fresh-permutation decoders run through rm_decode_batch only");
    const int N = d->N;
    const int64_t need = req->llr_on_device ? 0 : 4 * (int64_t)N;
    if (req->llr_on_device) {
        const unsigned char *lo = (const unsigned char *)req->llr, *hi = lo + 4 * (size_t)N;
        bool inside = false;
        for (int i = 0; i < s->n_pools && !inside; i++)
            inside = lo >= s->pool_lo[i] && hi <= s->pool_hi[i];
        if (!inside)
            return fail(RM_E_PTR, "device-resident LLRs outside every registered pool");
    }
    if (!open_batch(s))
        return RM_E_AGAIN;
    Batch *b = &s->batches[s->open];
    int seg = -1;
    for (int i = 0; i < b->n_segs; i++)
        if (b->seg_dec[i] == d)
            seg = i;
    const bool full = (int)b->reqs.size() == s->cfg.max_batch || b->llr_used + need > s->cfg.batch_bytes ||
                      (seg < 0 && b->n_segs == kMaxSegs);
    if (full) {
        // the open batch has no room: launch it if the device can take it
        if (s->inflight >= s->cfg.depth)
            return RM_E_AGAIN;
        const int rc = launch_open(s);
        if (rc != RM_OK)
            return rc;
        if (!open_batch(s))
            return RM_E_AGAIN;
        b = &s->batches[s->open];
        seg = -1;
    }
    if (seg < 0) {
        seg = b->n_segs++;
        b->seg_dec[seg] = d;
    }
    ReqMeta r;
    r.ticket = ++s->next_ticket;
    r.tag = req->tag;
    r.t_arrival = req->t_arrival_us > 0 ? req->t_arrival_us : now_us();
    r.seg = seg;
    r.n_bytes = N / 8;
    r.out_bits = req->out_bits;
    r.out_metric = req->out_metric;
    if (req->llr_on_device) {
        r.llr_dev = req->llr;
    } else {
        memcpy(b->h_llr + b->llr_used, req->llr, (size_t)need);
        r.llr_dev = (const float *)(b->d_llr + b->llr_used);
        b->llr_used += need;
    }
    b->reqs.push_back(r);
    s->pending++;
    if (ticket)
        *ticket = r.ticket;
    return maybe_launch(s);
}

int rm_server_poll(rm_server *s, rm_completion *out, int max)
{
    if (!s || (max > 0 && !out) || max < 0)
        return fail(RM_E_INVAL, "null server or output");
    int rc = retire(s);
    if (rc != RM_OK)
        return rc;
    // Every request whose completion word holds its launch's epoch is done
    // (the kernel wrote its outputs before the word); launched batches are
    // scanned oldest first, each in the order its kernels take the requests.
    // A kernel takes its queue entries in order, so once kMissRun requests in
    // a row are not done the rest of that list is left for a later poll.
    constexpr int kMissRun = 2048;
    int k = 0;
    for (int bi : s->order) {
        Batch &b = s->batches[bi];
        const volatile uint32_t *done = (const volatile uint32_t *)(b.h_out + s->out_done_off);
        const float *pm = (const float *)(b.h_out + s->out_pm_off);
        const double t_seen = now_us();
        for (std::vector<int> &un : b.unreported) {
            size_t keep = 0;
            int miss = 0;
            for (size_t q = 0; q < un.size(); q++) {
                const int i = un[q];
                if (k == max || miss >= kMissRun || done[i] != b.epoch) {
                    un[keep++] = i;
                    miss++;
                    continue;
                }
                miss = 0;
                std::atomic_thread_fence(std::memory_order_acquire);
                const ReqMeta &r = b.reqs[(size_t)i];
                rm_completion &c = out[k++];
                c.ticket = r.ticket;
                c.tag = r.tag;
                c.status = RM_OK;
                c.n_bytes = r.n_bytes;
                c.metric = pm[i];
                memcpy(c.bits, b.h_out + (size_t)i * kServeBitsStride, (size_t)r.n_bytes);
                c.t_arrival_us = r.t_arrival;
                c.t_launch_us = b.t_launch;
                c.t_done_us = t_seen;
                if (r.out_bits)
                    memcpy(r.out_bits, c.bits, (size_t)r.n_bytes);
                if (r.out_metric)
                    *r.out_metric = c.metric;
                s->pending--;
            }
            un.resize(keep);
        }
    }
    // a batch is reused once all its requests are returned and its kernels
    // have finished
    while (!s->order.empty()) {
        Batch &b = s->batches[s->order.front()];
        bool all = true;
        for (const auto &u : b.unreported)
            all = all && u.empty();
        if (b.state != Batch::DONE || !all)
            break;
        b.state = Batch::FREE;
        s->order.pop_front();
    }
    rc = maybe_launch(s);
    return rc != RM_OK ? rc : k;
}

int64_t rm_server_pending(const rm_server *s) { return s ? s->pending : 0; }

int rm_server_run_trace(rm_server *s, const rm_request *reqs, const double *arrival_us, int64_t n,
                        double *latency_us, double *stats)
{
    if (!s || n < 0 || (n > 0 && (!reqs || !arrival_us || !latency_us)))
        return fail(RM_E_INVAL, "null argument");
    if (s->pending != 0)
        return fail(RM_E_INVAL, "trace replay needs an idle server");
    std::vector<rm_completion> buf(1024);
    const int64_t launches0 = s->launches;
    s->largest = 0;
    double refused = 0;
    const double t0 = now_us();
    int64_t next = 0, done = 0;
    while (done < n) {
        const double t = now_us() - t0;
        while (next < n && arrival_us[next] <= t) {
            rm_request r = reqs[next];
            r.tag = (uint64_t)next;
            r.t_arrival_us = t0 + arrival_us[next];
            const int rc = rm_server_submit(s, &r, nullptr);
            if (rc == RM_E_AGAIN) {
                refused += 1;
                break;
            }
            if (rc != RM_OK)
                return rc;
            next++;
        }
        const int k = rm_server_poll(s, buf.data(), (int)buf.size());
        if (k < 0)
            return k;
        for (int i = 0; i < k; i++) {
            latency_us[buf[i].tag] = buf[i].t_done_us - buf[i].t_arrival_us;
            done++;
        }
    }
    if (stats) {
        stats[0] = now_us() - t0;
        stats[1] = (double)(s->launches - launches0);
        stats[2] = refused;
        stats[3] = (double)s->largest;
    }
    return RM_OK;
}

void rm_server_destroy(rm_server *s)
{
    if (!s)
        return;
    for (Batch &b : s->batches)
        free_batch(b);
    delete s;
}

} // extern "C"
