// Host runtime behind the C ABI declared in include/perch.h: contexts, the
// resident mesh and scene registry with its HBM budget, per-stream work
// buffers, argument validation and kernel launches.

#include "perch.h"
#include "perch_internal.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace perch;

namespace {

thread_local std::string g_last_error;

// Scratch of perch_score_poses_noalloc: launch descriptors, per-pose work,
// class lists, counters and the device-memory slots of the two largest
// footprint classes, in one array that each device holds for the life of
// the process.  Host code uses only the device address that
// hipGetSymbolAddress returns for it (kept per device), never the name.
constexpr size_t kNoAllocScratchBytes = (size_t)48 << 20;
constexpr int kNoAllocMaxPoses = 65536;
constexpr int kNoAllocMaxPixels = 640 * 480;
constexpr int kNoAllocGrid2 = 8, kNoAllocGrid3 = 4;   // work-groups of the device-memory classes
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_addr;

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
    *out = p;
    return hipSuccess;
}

perch_status fail(perch_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

perch_status ok()
{
    g_last_error.clear();
    return PERCH_OK;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? PERCH_ENOMEM : PERCH_EDEVICE, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                                    \
    } while (0)

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Events recorded after the last launch on each stream that read a buffer;
// a released buffer is reused only once all of them have completed.
struct Fence {
    std::vector<hipEvent_t> ev;
};
using FenceRef = std::shared_ptr<Fence>;

struct CachedBlock {
    void *ptr = nullptr;
    size_t bytes = 0;
    FenceRef fence;
};

// Last-use events of a resident mesh or scene, one per stream.
using Uses = std::map<hipStream_t, hipEvent_t>;

struct MeshRec {
    DevBuf verts, tris, rgb;
    MeshDev dev{};
    size_t bytes = 0;
    Uses uses;
};

struct SceneRec {
    DevBuf depth, rgb, labels, opt, olab, kx, ky, ax, ay, thdr, tnn, hstart, hpts;
    SceneDev dev{};
    long long table_entries = 0;        // entries of the nearest-neighbour table (0 with the voxel hash)
    bool table_on_host = false;         // its size counted on the host (a batch was running)
    std::vector<int32_t> host_labels;
    std::vector<uint16_t> host_depth;   // kept with labels: per-label depth ranges (pose proposals)
    std::map<int32_t, std::vector<int>> label_boxes;
    size_t bytes = 0;
    Uses uses;
};

// Allocation granule: 4 KiB up to 1 MiB, then an eighth of the leading
// power of two, so that buffers of similar size can reuse each other.
size_t round_alloc(size_t bytes)
{
    if (bytes <= ((size_t)1 << 20)) return (bytes + 4095) & ~(size_t)4095;
    const int lg = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t g = (size_t)1 << (lg - 3);
    return (bytes + g - 1) / g * g;
}

// Device buffers of one launch: descriptors, per-pose work, device-memory
// slots of the large footprint classes, per-item minima.
struct LaunchBufs {
    DevBuf desc, info, lists, counts, scratch, best, lab;
};

// Pinned staging of descriptors for asynchronous uploads: a ring of slots,
// each reused only after the copy that read it has executed.
struct Staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};

struct StreamBufs {
    LaunchBufs lb;
    DevBuf tmp;               // J_r / J_o of perch_best_poses
    DevBuf icp;               // ICP: pose cursor, per-work-group tiles and point lists
    DevBuf msg;               // tree: cursor, flag, raster keys, poses, per-work-group tiles, outputs
    DevBuf msg_states[2];     // tree: the planes of the states of two consecutive levels
    DevBuf knn1, knn1_dist;   // kNN I: keys, points, colours, observed list, marks, counts; the distance array
    Staging ring[8];
    int next = 0;
    int32_t last_n = 0;       // poses of the last scoring launch on this stream
};

}  // namespace

struct perch_batch;

struct perch_ctx {
    int device = 0;
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    size_t lds_max = 0;
    int next_mesh = 1, next_scene = 1;
    std::map<int32_t, MeshRec> meshes;
    std::map<int32_t, SceneRec> scenes;
    std::map<hipStream_t, StreamBufs> work;
    std::vector<perch_batch *> batches;
    std::recursive_mutex mu;
    perch_tuning tune{};                  // zeros: defaults
    int static_lds[3] = {0, 0, 0};        // static LDS bytes of the 256-, 512- and 1024-thread scoring kernels
    std::vector<Staging *> scene_stage;   // free pinned staging areas of scene uploads
    int icp_lds_words = 0;                // dynamic LDS words of the ICP kernel
    int msg_lds_words = 0;                // dynamic LDS words of the tree's successor kernel
    void *noalloc = nullptr;              // this device's address of the allocation-free path's scratch

    // released device blocks awaiting reuse, and recycled use-tracking events
    std::vector<CachedBlock> cache;
    size_t cached = 0;
    std::vector<hipEvent_t> ev_pool;

    // profiler: HIP events around each launch, on the launch stream
    bool prof = false;
    struct Rec {
        int slot;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[kNumProfSlots] = {};
    int launches[kNumProfSlots] = {};

    hipEvent_t event()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    template <class F>
    hipError_t timed(int slot, hipStream_t st, F &&launch)
    {
        if (!prof) return launch();
        Rec r{slot, event(), event()};
        (void)hipEventRecord(r.a, st);
        hipError_t e = launch();
        (void)hipEventRecord(r.b, st);
        pending.push_back(r);
        return e;
    }
    void collect()
    {
        for (Rec &r : pending) {
            (void)hipEventSynchronize(r.b);
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                total_ms[r.slot] += ms;
                launches[r.slot] += 1;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }

    hipEvent_t use_event()
    {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
        return e;
    }
    // record "read by work queued so far on st" for a mesh or scene
    void mark_use(Uses &u, hipStream_t st)
    {
        hipEvent_t &e = u[st];
        if (!e) e = use_event();
        (void)hipEventRecord(e, st);
    }
    FenceRef fence_of(Uses &u)
    {
        auto f = std::make_shared<Fence>();
        for (auto &kv : u) f->ev.push_back(kv.second);
        u.clear();
        return f;
    }
    bool fence_done(const FenceRef &f)
    {
        if (!f) return true;
        for (hipEvent_t e : f->ev)
            if (hipEventQuery(e) != hipSuccess) return false;
        for (hipEvent_t e : f->ev) ev_pool.push_back(e);
        f->ev.clear();
        return true;
    }
    // Free every cached block; waits for the device first.
    void trim()
    {
        if (cache.empty()) return;
        (void)hipDeviceSynchronize();
        for (CachedBlock &c : cache) {
            (void)hipFree(c.ptr);
            if (c.fence) fence_done(c.fence);
        }
        cache.clear();
        cached = 0;
    }
    perch_status alloc(DevBuf &b, size_t bytes)
    {
        bytes = round_alloc(bytes == 0 ? 256 : bytes);
        if (budget && used + bytes > budget)
            return fail(PERCH_ENOMEM, "HBM budget exceeded: %zu + %zu > %zu bytes", used, bytes, budget);
        // the smallest released block of at most twice the size whose readers are done
        int pick = -1;
        for (int i = 0; i < (int)cache.size(); ++i) {
            const CachedBlock &c = cache[i];
            if (c.bytes < bytes || c.bytes > 2 * bytes) continue;
            if (pick >= 0 && cache[pick].bytes <= c.bytes) continue;
            if (!fence_done(c.fence)) continue;
            pick = i;
        }
        if (pick >= 0) {
            b.ptr = cache[pick].ptr;
            b.bytes = cache[pick].bytes;
            cached -= b.bytes;
            cache.erase(cache.begin() + pick);
            used += b.bytes;
            return PERCH_OK;
        }
        if (budget && used + cached + bytes > budget) trim();
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipErrorOutOfMemory && !cache.empty()) {
            trim();
            e = hipMalloc(&p, bytes);
        }
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? PERCH_ENOMEM : PERCH_EDEVICE, "hipMalloc(%zu): %s", bytes,
                        hipGetErrorString(e));
        b.ptr = p;
        b.bytes = bytes;
        used += bytes;
        return PERCH_OK;
    }
    // Return a block to the cache; it is reused once `fence` has completed.
    void release(DevBuf &b, FenceRef fence = nullptr)
    {
        if (b.ptr) {
            cache.push_back(CachedBlock{b.ptr, b.bytes, fence});
            cached += b.bytes;
            used -= b.bytes;
        }
        b.ptr = nullptr;
        b.bytes = 0;
        if (cached > kCacheMax) trim();
    }
    static constexpr size_t kCacheMax = (size_t)16 << 30;
    // grow a per-stream buffer; waits for the device first so no queued
    // kernel still reads the old allocation
    perch_status ensure(DevBuf &b, size_t bytes)
    {
        if (b.bytes >= bytes && b.ptr) return PERCH_OK;
        if (b.ptr) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return fail(PERCH_EDEVICE, "hipDeviceSynchronize: %s", hipGetErrorString(e));
            release(b);
        }
        return alloc(b, bytes);
    }
};

// A prepared batch: device buffers, pinned descriptors and results, and a
// captured graph (descriptor upload, classification, scoring, per-item
// argmin, result download) whose kernels read everything through the
// descriptors, so new work only needs new descriptors.
struct perch_batch {
    perch_ctx *ctx = nullptr;
    int cap_items = 0, cap_poses = 0;
    size_t cap_pixels = 0, desc_cap = 0;
    LaunchCfg cfg{};
    LaunchBufs lb;
    void *pin_desc = nullptr, *pin_best = nullptr;
    hipStream_t cap = nullptr;
    // the launch captured twice: [1] with the paper's variants (J_o by
    // nearest-neighbour marking, the kNN II scan) compiled in, [0] without
    // them (the set's scenes pick one)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    // launched and not yet waited for: written by the launching and waiting
    // threads, read under the context lock by scene preparation and release
    std::atomic<bool> pending{false};
    bool valid = false, any_pv = false;
    int n_req = 0;
    std::vector<int32_t> scene_ids, mesh_ids;
    std::vector<int> item_of_req;
};

namespace {

// A batch that references a scene or mesh: EBUSY while its launch is
// pending, otherwise the batch is invalidated.
perch_status release_check(perch_ctx *ctx, bool scene, int32_t id)
{
    for (perch_batch *b : ctx->batches) {
        const std::vector<int32_t> &ids = scene ? b->scene_ids : b->mesh_ids;
        if (std::find(ids.begin(), ids.end(), id) == ids.end()) continue;
        if (b->pending && hipEventQuery(b->done) == hipErrorNotReady)
            return fail(PERCH_EBUSY, "%s %d is used by a batch still running", scene ? "scene" : "mesh", id);
        b->valid = false;
    }
    return PERCH_OK;
}

perch_status enter(perch_ctx *ctx)
{
    if (!ctx) return fail(PERCH_EINVAL, "null context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(PERCH_EDEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
    return PERCH_OK;
}

// NULL is the HIP null stream (the default stream of PyTorch and of plain HIP code).
hipStream_t pick_stream(perch_ctx *, void *s) { return (hipStream_t)s; }

// sRGB8 -> linear (IEC 61966-2-1), computed in binary64 and rounded.
void colour_table(float out[256])
{
    for (int v = 0; v < 256; ++v) {
        const double c = (double)v / 255.0;
        out[v] = (float)(c <= 0.04045 ? c / 12.92 : std::pow((c + 0.055) / 1.055, 2.4));
    }
}

// Launch configuration from the context's tuning.  At 128 VGPRs a CU keeps
// 16 waves resident: four 256-thread, two 512-thread or one 1024-thread
// scoring work-group, and each gets that share of the CU's LDS.
LaunchCfg launch_cfg(const perch_ctx *ctx)
{
    const perch_tuning &t = ctx->tune;
    const long long lds = (long long)ctx->lds_max;
    LaunchCfg c{};
    c.small_block = t.small_block == 256 ? 256 : 512;
    const int per_cu = 1024 / c.small_block;
    c.cap_large = (int)std::min<long long>((lds - ctx->static_lds[2]) / 4, 65535);
    const int fit = (int)std::min<long long>((lds / per_cu - ctx->static_lds[c.small_block == 256 ? 0 : 1]) / 4,
                                             c.cap_large);
    c.cap_small = t.small_words > 0 ? std::min(t.small_words, fit) : fit;
    const int def[kNumClasses] = {ctx->n_cu * per_cu, ctx->n_cu, ctx->n_cu, std::min(ctx->n_cu, 64)};
    for (int k = 0; k < kNumClasses; ++k)
        c.grid[k] = t.grid[k] > 0 ? std::min(t.grid[k], 16 * ctx->n_cu) : def[k];
    c.sort = t.order != 1;
    c.key_bands = t.key_bands != 1;
    return c;
}

bool finite3(const float *p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

}  // namespace

namespace {

// The label's pixels: {x0, y0, w, h} of their bounding box (all 0 when
// there are none), then the least and greatest valid depth among them (mm;
// 1, 0 when none has a reading).
std::vector<int> label_box(SceneRec &r, int32_t label)
{
    auto it = r.label_boxes.find(label);
    if (it != r.label_boxes.end()) return it->second;
    const int W = r.dev.W, H = r.dev.H;
    int x0 = W, y0 = H, x1 = -1, y1 = -1, zmin = 65536, zmax = 0;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i)
            if (r.host_labels[(size_t)j * W + i] == label) {
                x0 = std::min(x0, i);
                x1 = std::max(x1, i);
                y0 = std::min(y0, j);
                y1 = std::max(y1, j);
                const int d = r.host_depth.empty() ? 0 : r.host_depth[(size_t)j * W + i];
                if (d > 0) {
                    zmin = std::min(zmin, d);
                    zmax = std::max(zmax, d);
                }
            }
    std::vector<int> b = x1 < 0 ? std::vector<int>{0, 0, 0, 0} : std::vector<int>{x0, y0, x1 - x0 + 1, y1 - y0 + 1};
    b.push_back(zmax > 0 ? zmin : 1);
    b.push_back(zmax);
    r.label_boxes[label] = b;
    return b;
}

size_t align64(size_t x) { return (x + 63) & ~(size_t)63; }

// Host image of a launch's descriptors: header | items | scenes | meshes.
struct Built {
    std::vector<char> bytes;
    size_t items_off = 64, scenes_off = 0, meshes_off = 0;
    int n_items = 0, n_poses = 0;
    size_t max_pixels = 0;
    bool any_rgb = false;
    bool any_pv = false;   // some scene takes one of the paper's variants (NN marking, kNN II)
    std::vector<int32_t> scene_ids, mesh_ids;
    std::vector<int> item_of_req;   // item index of each request, -1 if it has no poses
};

size_t desc_capacity(int items)
{
    return 64 + align64((size_t)items * sizeof(ItemDev)) + align64((size_t)items * sizeof(SceneDev))
           + align64((size_t)items * sizeof(MeshDev));
}

perch_status build_descriptors(perch_ctx *ctx, const perch_work *req, int32_t n_req, Built &b, int cap_items = 0,
                               uint8_t *rflag = nullptr, uint8_t *oflag = nullptr)
{
    if (n_req < 0) return fail(PERCH_EINVAL, "negative item count");
    if (n_req > 0 && !req) return fail(PERCH_EINVAL, "null items");
    std::vector<ItemDev> items;
    std::vector<SceneDev> scenes;
    std::vector<MeshDev> meshes;
    std::map<int32_t, int> sidx, midx;
    long long total = 0;
    b.item_of_req.assign((size_t)n_req, -1);
    for (int32_t r = 0; r < n_req; ++r) {
        const perch_work &q = req[r];
        auto si = ctx->scenes.find(q.scene_id);
        if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "item %d: unknown scene id %d", r, q.scene_id);
        auto mi = ctx->meshes.find(q.mesh_id);
        if (mi == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "item %d: unknown mesh id %d", r, q.mesh_id);
        if ((si->second.dev.flags & PERCH_USE_RGB) && !mi->second.dev.vrgb)
            return fail(PERCH_EINVAL, "item %d: scene uses the RGB term but mesh %d has no vertex colours", r,
                        q.mesh_id);
        if (q.n_poses < 0) return fail(PERCH_EINVAL, "item %d: n_poses must be >= 0", r);
        if (q.n_poses == 0) continue;
        if (!q.poses_dev || !q.jr_dev || !q.jo_dev) return fail(PERCH_EINVAL, "item %d: null poses, jr or jo", r);
        if (!sidx.count(q.scene_id)) {
            sidx[q.scene_id] = (int)scenes.size();
            scenes.push_back(si->second.dev);
            b.scene_ids.push_back(q.scene_id);
        }
        if (!midx.count(q.mesh_id)) {
            midx[q.mesh_id] = (int)meshes.size();
            meshes.push_back(mi->second.dev);
            b.mesh_ids.push_back(q.mesh_id);
        }
        const SceneDev &sd = si->second.dev;
        ItemDev it{};
        it.scene = sidx[q.scene_id];
        it.mesh = midx[q.mesh_id];
        it.label = q.label;
        it.n = q.n_poses;
        it.first = (int)total;
        it.key32 = sd.dq2 < 65536;
        if ((sd.flags & PERCH_VOL_MASK) == PERCH_VOL_LABEL) {
            std::vector<int> box = label_box(si->second, q.label);
            for (int k = 0; k < 4; ++k) it.vbox[k] = box[k];
        }
        it.poses = q.poses_dev;
        it.jr = q.jr_dev;
        it.jo = q.jo_dev;
        it.nr = q.nr_dev;
        it.nq = q.nq_dev;
        it.rflag = rflag;
        it.oflag = oflag;
        b.item_of_req[r] = (int)items.size();
        items.push_back(it);
        total += q.n_poses;
        b.max_pixels = std::max(b.max_pixels, (size_t)sd.W * sd.H);
        b.any_rgb |= (sd.flags & PERCH_USE_RGB) != 0;
        b.any_pv |= (sd.flags & (PERCH_JO_NN | PERCH_KNN2 | PERCH_HASH)) != 0;
        if (sd.flags & PERCH_KNN1)
            return fail(PERCH_EINVAL, "PERCH_KNN1 scenes are scored by perch_score_poses only");
    }
    if (total >= (1LL << 30)) return fail(PERCH_EINVAL, "too many poses in one launch (%lld)", total);
    b.n_items = (int)items.size();
    b.n_poses = (int)total;
    // tables sized for the capacity of a prepared batch, else for this launch
    const size_t slots = cap_items > 0 ? (size_t)cap_items : std::max(items.size(), (size_t)1);
    if (cap_items > 0 && items.size() > (size_t)cap_items)
        return fail(PERCH_EINVAL, "%zu items exceed the batch capacity %d", items.size(), cap_items);
    b.scenes_off = 64 + align64(slots * sizeof(ItemDev));
    b.meshes_off = b.scenes_off + align64(slots * sizeof(SceneDev));
    b.bytes.assign(b.meshes_off + align64(slots * sizeof(MeshDev)), 0);
    LaunchHdr h{b.n_items, b.n_poses, (int)b.scene_ids.size()};
    std::memcpy(b.bytes.data(), &h, sizeof h);
    if (!items.empty()) std::memcpy(b.bytes.data() + 64, items.data(), items.size() * sizeof(ItemDev));
    if (!scenes.empty()) std::memcpy(b.bytes.data() + b.scenes_off, scenes.data(), scenes.size() * sizeof(SceneDev));
    if (!meshes.empty()) std::memcpy(b.bytes.data() + b.meshes_off, meshes.data(), meshes.size() * sizeof(MeshDev));
    return PERCH_OK;
}

// Device-memory slot sizes (32-bit words) of the large footprint classes:
// class 2 holds 64-bit keys over at most the image, class 3 also the tile.
void slot_layout(const LaunchCfg &cfg, size_t max_pixels, size_t slot_words[kNumClasses],
                 size_t slot_base[kNumClasses], size_t *total_words, size_t *tile_words)
{
    *tile_words = (max_pixels + 1) & ~(size_t)1;
    slot_words[0] = slot_words[1] = 0;
    slot_words[2] = 2 * max_pixels;
    slot_words[3] = *tile_words + 2 * max_pixels;
    *total_words = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        slot_base[c] = *total_words;
        *total_words += slot_words[c] * (size_t)cfg.grid[c];
    }
}

// Per-work-group CIELAB slots of the RGB term: one entry per pixel of the
// class's largest tile.
void lab_layout(const LaunchCfg &cfg, size_t max_pixels, size_t lab_px[kNumClasses], size_t lab_base[kNumClasses],
                size_t *total)
{
    lab_px[0] = (size_t)cfg.cap_small;
    lab_px[1] = lab_px[2] = (size_t)cfg.cap_large;
    lab_px[3] = max_pixels;
    *total = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        lab_base[c] = *total;
        *total += lab_px[c] * (size_t)cfg.grid[c];
    }
}

perch_status ensure_bufs(perch_ctx *ctx, LaunchBufs &lb, size_t desc_bytes, int cap_poses, int cap_items,
                         size_t max_pixels, const LaunchCfg &cfg, bool rgb)
{
    size_t sw[kNumClasses], sb[kNumClasses], total = 0, tile = 0;
    slot_layout(cfg, max_pixels, sw, sb, &total, &tile);
    size_t lp[kNumClasses], lb0[kNumClasses], lab_total = 0;
    lab_layout(cfg, max_pixels, lp, lb0, &lab_total);
    perch_status s;
    if ((s = ctx->ensure(lb.desc, desc_bytes))) return s;
    if ((s = ctx->ensure(lb.info, (size_t)std::max(cap_poses, 1) * sizeof(PoseInfo)))) return s;
    if ((s = ctx->ensure(lb.lists, (size_t)kNumClasses * std::max(cap_poses, 1) * sizeof(int)))) return s;
    if ((s = ctx->ensure(lb.counts, kCounterInts * 4))) return s;
    if ((s = ctx->ensure(lb.scratch, total * 4))) return s;
    if ((s = ctx->ensure(lb.best, (size_t)std::max(cap_items, 1) * 8))) return s;
    if (rgb && (s = ctx->ensure(lb.lab, lab_total * sizeof(float4)))) return s;
    return PERCH_OK;
}

Work make_work(const LaunchBufs &lb, const Built &b, int cap_poses, const LaunchCfg &cfg, size_t max_pixels,
               bool want_best)
{
    Work w{};
    const char *d = (const char *)lb.desc.ptr;
    w.hdr = (const LaunchHdr *)d;
    w.items = (const ItemDev *)(d + 64);
    w.scenes = (const SceneDev *)(d + b.scenes_off);
    w.meshes = (const MeshDev *)(d + b.meshes_off);
    w.cap_poses = cap_poses;
    w.info = (PoseInfo *)lb.info.ptr;
    w.lists = (int *)lb.lists.ptr;
    w.counts = (int *)lb.counts.ptr;
    w.gscratch = (uint32_t *)lb.scratch.ptr;
    size_t total = 0;
    slot_layout(cfg, max_pixels, w.slot_words, w.slot_base, &total, &w.dev_tile_words);
    w.cap_small = cfg.cap_small;
    w.cap_large = cfg.cap_large;
    w.sort = cfg.sort;
    w.key_bands = cfg.key_bands;
    w.best = want_best ? (int32_t *)lb.best.ptr : nullptr;
    size_t lab_total = 0;
    lab_layout(cfg, max_pixels, w.lab_px, w.lab_base, &lab_total);
    w.lab = lb.lab.bytes >= lab_total * sizeof(float4) ? (float4 *)lb.lab.ptr : nullptr;
    return w;
}

// Enqueue a launch: classify, score the four footprint classes, and the
// per-item argmin when w.best is set.
hipError_t enqueue(perch_ctx *ctx, const Work &w, const LaunchCfg &cfg, int poses_grid, int items_grid, bool any_rgb,
                   bool any_pv, hipStream_t st, bool timed)
{
    auto T = [&](int slot, auto &&f) { return timed ? ctx->timed(slot, st, f) : f(); };
    hipError_t e = T(kProfSetup, [&] { return launch_setup(w, poses_grid, st); });
    for (int cls = 0; cls < kNumClasses && e == hipSuccess; ++cls)
        e = T(kProfClass0 + cls, [&] { return launch_score_class(w, cfg, cls, any_rgb, any_pv, st); });
    if (e == hipSuccess && w.best) e = T(kProfArgmin, [&] { return launch_item_argmin(w, items_grid, st); });
    return e;
}

// Copy descriptors to the device through a pinned staging slot, asynchronously.
perch_status upload(StreamBufs &sb, const Built &b, void *dev, hipStream_t st)
{
    Staging &slot = sb.ring[sb.next];
    sb.next = (sb.next + 1) % 8;
    if (slot.done) HIP_TRY(hipEventSynchronize(slot.done));
    else HIP_TRY(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    if (slot.bytes < b.bytes.size()) {
        if (slot.host) HIP_TRY(hipHostFree(slot.host));
        slot.host = nullptr;
        slot.bytes = 0;
        HIP_TRY(hipHostMalloc(&slot.host, b.bytes.size(), hipHostMallocDefault));
        slot.bytes = b.bytes.size();
    }
    std::memcpy(slot.host, b.bytes.data(), b.bytes.size());
    HIP_TRY(hipMemcpyAsync(dev, slot.host, b.bytes.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(slot.done, st));
    return PERCH_OK;
}

void mark_uses(perch_ctx *ctx, const std::vector<int32_t> &scene_ids, const std::vector<int32_t> &mesh_ids,
               hipStream_t st)
{
    for (int32_t id : scene_ids) ctx->mark_use(ctx->scenes[id].uses, st);
    for (int32_t id : mesh_ids) ctx->mark_use(ctx->meshes[id].uses, st);
}

// Direct (non-graph) launch of a list of work items on a stream (caller
// holds the context lock).  With want_best, the per-item minima are left in
// the stream's buffers: *n_items_out and item_of_req say where.
perch_status run_direct(perch_ctx *ctx, const perch_work *req, int32_t n_req, hipStream_t st, bool want_best,
                        int *n_items_out = nullptr, std::vector<int> *item_of_req = nullptr,
                        uint8_t *rflag = nullptr, uint8_t *oflag = nullptr)
{
    Built b;
    if (perch_status s = build_descriptors(ctx, req, n_req, b, 0, rflag, oflag)) return s;
    if (n_items_out) *n_items_out = b.n_items;
    if (item_of_req) *item_of_req = b.item_of_req;
    if (b.n_poses == 0) return PERCH_OK;
    StreamBufs &sb = ctx->work[st];
    const LaunchCfg cfg = launch_cfg(ctx);
    if (perch_status s = ensure_bufs(ctx, sb.lb, b.bytes.size(), b.n_poses, b.n_items, b.max_pixels, cfg, b.any_rgb))
        return s;
    if (perch_status s = upload(sb, b, sb.lb.desc.ptr, st)) return s;
    const Work w = make_work(sb.lb, b, b.n_poses, cfg, b.max_pixels, want_best);
    sb.last_n = b.n_poses;
    hipError_t e = enqueue(ctx, w, cfg, b.n_poses, b.n_items, b.any_rgb, b.any_pv, st, true);
    if (e != hipSuccess) return fail(PERCH_EDEVICE, "score launch: %s", hipGetErrorString(e));
    mark_uses(ctx, b.scene_ids, b.mesh_ids, st);
    return PERCH_OK;
}

}  // namespace

namespace {

// A roctx range over one entry point (named as the entry point), seen by
// rocprofv3 --marker-trace; without a profiler attached it is a call that
// returns at once.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

}  // namespace

extern "C" {

const char *perch_last_error(void) { return g_last_error.c_str(); }

perch_status perch_create(int device, size_t hbm_budget_bytes, perch_ctx **out)
{
    if (!out) return fail(PERCH_EINVAL, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(PERCH_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(PERCH_EINVAL, "device %d out of range [0, %d)", device, n);
    HIP_TRY(hipSetDevice(device));
    auto *ctx = new perch_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device);
    ctx->n_cu = (e == hipSuccess && v > 0) ? v : 256;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    ctx->lds_max = (e == hipSuccess && v > 0) ? (size_t)v : 65536;
    float lin[256];
    colour_table(lin);
    e = upload_colour_table(lin);
    if (e == hipSuccess) e = prepare_score_kernels((int)ctx->lds_max, ctx->static_lds);
    if (e == hipSuccess) e = prepare_icp_kernel((int)ctx->lds_max, &ctx->icp_lds_words);
    if (e == hipSuccess) e = upload_msg_colour_table(lin);
    if (e == hipSuccess) e = upload_knn1_colour_table(lin);
    if (e == hipSuccess) e = prepare_msg_kernel((int)ctx->lds_max, &ctx->msg_lds_words);
    if (e == hipSuccess) e = scratch_address(device, &ctx->noalloc);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete ctx;
        return fail(PERCH_EDEVICE, "context set-up: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return ok();
}

perch_status perch_destroy(perch_ctx *ctx)
{
    if (!ctx) return ok();
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->meshes) {
        FenceRef f = ctx->fence_of(kv.second.uses);
        ctx->release(kv.second.verts, f);
        ctx->release(kv.second.tris, f);
        ctx->release(kv.second.rgb, f);
    }
    for (auto &kv : ctx->scenes) {
        SceneRec &r = kv.second;
        FenceRef f = ctx->fence_of(r.uses);
        for (DevBuf *b : {&r.depth, &r.rgb, &r.labels, &r.opt, &r.olab, &r.kx, &r.ky, &r.ax, &r.ay, &r.thdr,
                          &r.tnn, &r.hstart, &r.hpts})
            ctx->release(*b, f);
    }
    while (!ctx->batches.empty()) perch_batch_destroy(ctx->batches.back());
    for (auto &kv : ctx->work) {
        StreamBufs &w = kv.second;
        for (DevBuf *b : {&w.lb.desc, &w.lb.info, &w.lb.lists, &w.lb.counts, &w.lb.scratch, &w.lb.best, &w.lb.lab,
                          &w.tmp, &w.icp})
            ctx->release(*b);
        for (Staging &g : w.ring) {
            if (g.host) (void)hipHostFree(g.host);
            if (g.done) (void)hipEventDestroy(g.done);
        }
    }
    for (Staging *g : ctx->scene_stage) {
        if (g->host) (void)hipHostFree(g->host);
        delete g;
    }
    ctx->scene_stage.clear();
    ctx->collect();
    ctx->trim();
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return ok();
}

perch_status perch_load_mesh(perch_ctx *ctx, const float *xyz, int32_t n_verts, const int32_t *tri,
                             int32_t n_tris, const uint8_t *rgb, int32_t *mesh_id)
{
    const Range range_("perch_load_mesh");
    if (perch_status st = enter(ctx)) return st;
    if (!xyz || !tri || !mesh_id) return fail(PERCH_EINVAL, "null xyz, tri or mesh_id");
    if (n_verts < 1) return fail(PERCH_EINVAL, "n_verts must be >= 1 (got %d)", n_verts);
    if (n_tris < 1 || n_tris > kMaxTris)
        return fail(PERCH_EINVAL, "n_tris must be in [1, %d] (got %d)", kMaxTris, n_tris);
    std::vector<float4> v((size_t)n_verts);
    float lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
    for (int32_t k = 0; k < n_verts; ++k) {
        const float *p = xyz + 3 * (size_t)k;
        if (!finite3(p)) return fail(PERCH_EINVAL, "vertex %d is not finite", k);
        v[k] = make_float4(p[0], p[1], p[2], 0.0f);
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    std::vector<int4> t((size_t)n_tris);
    for (int32_t k = 0; k < n_tris; ++k) {
        const int32_t *q = tri + 3 * (size_t)k;
        for (int a = 0; a < 3; ++a)
            if (q[a] < 0 || q[a] >= n_verts) return fail(PERCH_EINVAL, "triangle %d index %d out of range", k, q[a]);
        t[k] = make_int4(q[0], q[1], q[2], 0);
    }
    std::vector<uint32_t> c;
    if (rgb) {
        c.resize((size_t)n_verts);
        for (int32_t k = 0; k < n_verts; ++k)
            c[k] = (uint32_t)rgb[3 * (size_t)k] | ((uint32_t)rgb[3 * (size_t)k + 1] << 8)
                   | ((uint32_t)rgb[3 * (size_t)k + 2] << 16);
    }
    MeshRec r;
    auto cleanup = [&]() {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        ctx->release(r.verts);
        ctx->release(r.tris);
        ctx->release(r.rgb);
    };
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        perch_status st;
        if ((st = ctx->alloc(r.verts, v.size() * sizeof(float4))) || (st = ctx->alloc(r.tris, t.size() * sizeof(int4)))
            || (rgb && (st = ctx->alloc(r.rgb, c.size() * sizeof(uint32_t))))) {
            std::string msg = g_last_error;
            cleanup();
            return fail(st, "%s", msg.c_str());
        }
    }
    hipError_t e = hipMemcpy(r.verts.ptr, v.data(), v.size() * sizeof(float4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r.tris.ptr, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess && rgb) e = hipMemcpy(r.rgb.ptr, c.data(), c.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cleanup();
        return fail(PERCH_EDEVICE, "mesh upload: %s", hipGetErrorString(e));
    }
    r.dev.verts = (const float4 *)r.verts.ptr;
    r.dev.tris = (const int4 *)r.tris.ptr;
    r.dev.vrgb = (const uint32_t *)r.rgb.ptr;
    r.dev.nv = n_verts;
    r.dev.nt = n_tris;
    for (int a = 0; a < 3; ++a) {
        r.dev.lo[a] = lo[a];
        r.dev.hi[a] = hi[a];
    }
    r.bytes = r.verts.bytes + r.tris.bytes + r.rgb.bytes;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    const int32_t id = ctx->next_mesh++;
    ctx->meshes[id] = r;
    *mesh_id = id;
    return ok();
}

perch_status perch_unload_mesh(perch_ctx *ctx, int32_t mesh_id)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->meshes.find(mesh_id);
    if (it == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", mesh_id);
    if (perch_status st = release_check(ctx, false, mesh_id)) return st;
    FenceRef f = ctx->fence_of(it->second.uses);
    ctx->release(it->second.verts, f);
    ctx->release(it->second.tris, f);
    ctx->release(it->second.rgb, f);
    ctx->meshes.erase(it);
    return ok();
}

namespace {

// Entries of a scene's neighbour table counted on the host: per pixel the
// depths [min - dzmm, max + dzmm] (kept inside [1, 65534]) of the valid
// observed depths in its (2 wtx + 1) x (2 wty + 1) window, the count the
// ranges kernels reach (row pass, then column pass, over the same clipped
// windows).  -1 when the windows are too wide for this pass to pay.
long long table_entries_host(const uint16_t *depth, int W, int H, int wtx, int wty, int dzmm)
{
    if (wtx > 48 || wty > 48) return -1;
    const size_t N = (size_t)W * H;
    std::vector<uint16_t> mn(N), mx(N), smn(W), smx(W);
    for (int j = 0; j < H; ++j) {
        const uint16_t *row = depth + (size_t)j * W;
        uint16_t *a = mn.data() + (size_t)j * W, *b = mx.data() + (size_t)j * W;
        for (int i = 0; i < W; ++i) {
            smn[i] = row[i] ? row[i] : (uint16_t)0xFFFF;     // an empty pixel takes part in neither extreme
            smx[i] = row[i];
            a[i] = smn[i];
            b[i] = smx[i];
        }
        for (int o = 1; o <= wtx && o < W; ++o) {
            for (int i = 0; i + o < W; ++i) {
                a[i] = std::min(a[i], smn[i + o]);
                b[i] = std::max(b[i], smx[i + o]);
            }
            for (int i = o; i < W; ++i) {
                a[i] = std::min(a[i], smn[i - o]);
                b[i] = std::max(b[i], smx[i - o]);
            }
        }
    }
    std::vector<uint16_t> cmn(W), cmx(W);
    long long total = 0;
    for (int j = 0; j < H; ++j) {
        std::fill(cmn.begin(), cmn.end(), (uint16_t)0xFFFF);
        std::fill(cmx.begin(), cmx.end(), (uint16_t)0);
        for (int jj = std::max(j - wty, 0); jj <= std::min(j + wty, H - 1); ++jj) {
            const uint16_t *a = mn.data() + (size_t)jj * W, *b = mx.data() + (size_t)jj * W;
            for (int i = 0; i < W; ++i) {
                cmn[i] = std::min(cmn[i], a[i]);
                cmx[i] = std::max(cmx[i], b[i]);
            }
        }
        for (int i = 0; i < W; ++i)
            if (cmx[i] > 0)
                total += std::min(65534, (int)cmx[i] + dzmm) - std::max(1, (int)cmn[i] - dzmm) + 1;
    }
    return total;
}

// True while a batch of this context is still running (caller holds the lock).
bool batches_busy(perch_ctx *ctx)
{
    for (perch_batch *b : ctx->batches)
        if (b->pending && hipEventQuery(b->done) == hipErrorNotReady) return true;
    return false;
}

}  // namespace

perch_status perch_table_entries(const uint16_t *depth_mm, int32_t w, int32_t h, int32_t wx, int32_t wy,
                                 int32_t dzmm, int64_t *entries)
{
    if (!depth_mm || !entries) return fail(PERCH_EINVAL, "null depth or output");
    if (w < 1 || h < 1 || wx < 0 || wy < 0 || dzmm < 0) return fail(PERCH_EINVAL, "bad image size or window");
    *entries = table_entries_host(depth_mm, w, h, wx, wy, dzmm);
    return ok();
}

perch_status perch_set_scene(perch_ctx *ctx, const perch_scene_desc *d, int32_t *scene_id)
{
    const Range range_("perch_set_scene");
    if (perch_status st = enter(ctx)) return st;
    if (!d || !scene_id) return fail(PERCH_EINVAL, "null descriptor or scene_id");
    const perch_intrinsics &K = d->K;
    if (K.width < 1 || K.width > 4096 || K.height < 1 || K.height > 4096)
        return fail(PERCH_EINVAL, "image size %dx%d outside [1, 4096]", K.width, K.height);
    if (!(K.fx > 0.0f) || !(K.fy > 0.0f) || !std::isfinite(K.fx) || !std::isfinite(K.fy) || !std::isfinite(K.cx)
        || !std::isfinite(K.cy))
        return fail(PERCH_EINVAL, "intrinsics must be finite with fx, fy > 0");
    if (!d->depth_mm) return fail(PERCH_EINVAL, "depth_mm is required");
    if (!(d->delta_mm > 0.0f) || !(d->delta_mm <= 500.0f)) return fail(PERCH_EINVAL, "delta_mm must be in (0, 500]");
    if (!(d->tau_c >= 0.0f) || !std::isfinite(d->tau_c)) return fail(PERCH_EINVAL, "tau_c must be finite and >= 0");
    if (d->stride < 1) return fail(PERCH_EINVAL, "stride must be >= 1");
    const uint32_t known =
        PERCH_USE_RGB | PERCH_MARK_OCCLUDERS | PERCH_VOL_MASK | PERCH_JO_NN | PERCH_KNN2 | PERCH_KNN1 | PERCH_HASH;
    if (d->flags & ~known) return fail(PERCH_EINVAL, "unknown flag bits 0x%x", d->flags & ~known);
    if (((d->flags & PERCH_KNN1) != 0) + ((d->flags & PERCH_KNN2) != 0) + ((d->flags & PERCH_HASH) != 0) > 1)
        return fail(PERCH_EINVAL, "PERCH_KNN1, PERCH_KNN2 and PERCH_HASH are three searches; pass one");
    const uint32_t vol = d->flags & PERCH_VOL_MASK;
    if (vol != PERCH_VOL_AABB && vol != PERCH_VOL_CYL && vol != PERCH_VOL_LABEL)
        return fail(PERCH_EINVAL, "unsupported volume mode");
    if ((d->flags & PERCH_USE_RGB) && !d->rgb) return fail(PERCH_EINVAL, "PERCH_USE_RGB needs scene rgb");
    if (vol == PERCH_VOL_LABEL && !d->labels) return fail(PERCH_EINVAL, "PERCH_VOL_LABEL needs labels");
    const int W = K.width, H = K.height;
    const size_t N = (size_t)W * H;
    const bool use_rgb = (d->flags & PERCH_USE_RGB) != 0;

    std::vector<double> kx(W), ky(H);
    for (int i = 0; i < W; ++i) kx[i] = (((double)i - (double)K.cx) * 16.0) / (double)K.fx;
    for (int j = 0; j < H; ++j) ky[j] = (((double)j - (double)K.cy) * 16.0) / (double)K.fy;
    // Window factors: a point at pixel column i and depth z has every point
    // within delta inside ax[i] / (z - delta) + 1 columns (rows: ay).
    std::vector<float> ax(W), ay(H);
    auto up = [](double v) {
        float f = (float)v;
        return (double)f < v ? std::nextafter(f, INFINITY) : f;
    };
    const double dl4 = (double)d->delta_mm + 0.25;
    for (int i = 0; i < W; ++i) {
        const double r = ((double)i - (double)K.cx) / (double)K.fx;
        ax[i] = up((double)K.fx * dl4 * std::sqrt(1.0 + r * r));
    }
    for (int j = 0; j < H; ++j) {
        const double r = ((double)j - (double)K.cy) / (double)K.fy;
        ay[j] = up((double)K.fy * dl4 * std::sqrt(1.0 + r * r));
    }

    SceneRec r;
    const bool hashed = (d->flags & PERCH_HASH) != 0;
    // voxel hash: cells of edge 2^hshift >= dq, 2^hbits >= 2 N buckets
    int hshift = 0, hbits = 10;
    {
        const int dq = (int)std::nearbyint(16.0 * (double)d->delta_mm);
        while ((1 << hshift) < dq) ++hshift;
        while (((size_t)1 << hbits) < 2 * N) ++hbits;
    }
    const size_t n_buckets = (size_t)1 << hbits;
    DevBuf tmp;   // table: row pass (N words), the table total, the scan's block sums; hash: bucket counts, sums
    const size_t tmp_main = hashed ? n_buckets * 4 : (N * 4 + 7) & ~(size_t)7;
    const int scan_blocks = table_scan_blocks(hashed ? (int)n_buckets : (int)N);
    // host images staged in one pinned area: depth | rgb | labels | kx | ky | ax | ay | table total
    auto up8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
    const size_t o_depth = 0, o_rgb = up8(N * 2), o_lab = o_rgb + (use_rgb ? up8(N * 3) : 0);
    const size_t o_kx = o_lab + (d->labels ? up8(N * 4) : 0), o_ky = o_kx + (size_t)W * 8, o_ax = o_ky + (size_t)H * 8;
    const size_t o_ay = o_ax + up8((size_t)W * 4), o_total = o_ay + up8((size_t)H * 4), stage_bytes = o_total + 8;
    // Window half-sizes that hold every neighbour pair of this scene: a
    // rendered point with an observed neighbour has depth >= dmin - dzmm,
    // and the pixel window shrinks with depth.
    const int dq = (int)std::nearbyint(16.0 * (double)d->delta_mm), dzmm = dq / 16;
    int wtx = W, wty = H;
    {
        int dmin = 65535;
        for (size_t k = 0; k < N; ++k)
            if (d->depth_mm[k] > 0 && d->depth_mm[k] < dmin) dmin = d->depth_mm[k];
        const double dl = (double)d->delta_mm + 0.25;
        const double z = (double)dmin - (double)dzmm;
        const double rx = std::max(std::fabs(0.0 - K.cx), std::fabs((double)(W - 1) - K.cx)) / K.fx;
        const double ry = std::max(std::fabs(0.0 - K.cy), std::fabs((double)(H - 1) - K.cy)) / K.fy;
        if (dmin < 65535 && z - dl > 1.0) {
            wtx = std::min(W, (int)(K.fx * dl * std::sqrt(1.0 + rx * rx) / (z - dl)) + 2);
            wty = std::min(H, (int)(K.fy * dl * std::sqrt(1.0 + ry * ry) / (z - dl)) + 2);
        }
    }
    // The table's size decides its allocation.  While this context's batches
    // keep the device busy, waiting for the ranges kernels' count would wait
    // behind them (a scoring launch holds every compute unit): the host
    // counts it instead, the device's count is checked against it at the end.
    long long host_total = -1;
    if (!hashed) {
        bool busy;
        {
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            busy = batches_busy(ctx);
        }
        if (busy) host_total = table_entries_host(d->depth_mm, W, H, wtx, wty, dzmm);
        if (host_total >= (1LL << 31) - 1)
            return fail(PERCH_ENOMEM, "scene neighbour table too large (%lld entries)", host_total);
    }
    Staging *stg = nullptr;
    // allocation and kernel launches under the context lock; the waits outside it, so scoring on other streams
    // is not held up
    auto cleanup = [&]() {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        for (DevBuf *b : {&r.depth, &r.rgb, &r.labels, &r.opt, &r.olab, &r.kx, &r.ky, &r.ax, &r.ay, &r.thdr,
                          &r.tnn, &r.hstart, &r.hpts, &tmp})
            ctx->release(*b);
        if (stg) ctx->scene_stage.push_back(stg);
    };
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        perch_status st = PERCH_OK;
        auto A = [&](DevBuf &b, size_t n) {
            if (st == PERCH_OK) st = ctx->alloc(b, n);
        };
        A(r.depth, N * 2);
        A(r.opt, N * sizeof(int4));
        A(r.kx, W * 8);
        A(r.ky, H * 8);
        A(r.ax, W * 4);
        A(r.ay, H * 4);
        if (use_rgb) {
            A(r.rgb, N * 3);
            A(r.olab, N * sizeof(float4));
        }
        if (d->labels) A(r.labels, N * 4);
        if (hashed) {
            A(r.hstart, (n_buckets + 1) * 4);
            A(r.hpts, N * sizeof(int4));
        } else {
            A(r.thdr, N * sizeof(int2));
            if (host_total >= 0) A(r.tnn, (size_t)std::max(host_total, 1LL) * 4);
        }
        A(tmp, tmp_main + 64 + (size_t)(scan_blocks + 1) * 8);
        if (st == PERCH_OK) {
            if (!ctx->scene_stage.empty()) {
                stg = ctx->scene_stage.back();
                ctx->scene_stage.pop_back();
            } else {
                stg = new Staging();
            }
        }
        if (st != PERCH_OK) {
            std::string msg = g_last_error;
            cleanup();
            return fail(st, "%s", msg.c_str());
        }
    }
    hipError_t e = hipSuccess;
    if (stg->bytes < stage_bytes) {
        if (stg->host) e = hipHostFree(stg->host);
        stg->host = nullptr;
        stg->bytes = 0;
        if (e == hipSuccess) e = hipHostMalloc(&stg->host, stage_bytes, hipHostMallocDefault);
        if (e == hipSuccess) stg->bytes = stage_bytes;
    }
    if (e != hipSuccess) {
        cleanup();
        return fail(PERCH_ENOMEM, "pinned staging of %zu bytes: %s", stage_bytes, hipGetErrorString(e));
    }
    char *hs = (char *)stg->host;
    std::memcpy(hs + o_depth, d->depth_mm, N * 2);
    if (use_rgb) std::memcpy(hs + o_rgb, d->rgb, N * 3);
    if (d->labels) std::memcpy(hs + o_lab, d->labels, N * 4);
    std::memcpy(hs + o_kx, kx.data(), W * 8);
    std::memcpy(hs + o_ky, ky.data(), H * 8);
    std::memcpy(hs + o_ax, ax.data(), W * 4);
    std::memcpy(hs + o_ay, ay.data(), H * 4);
    SceneDev &s = r.dev;
    s.depth = (const uint16_t *)r.depth.ptr;
    s.opt = (const int4 *)r.opt.ptr;
    s.olab = (const float4 *)r.olab.ptr;
    s.labels = (const int32_t *)r.labels.ptr;
    s.kx = (const double *)r.kx.ptr;
    s.ky = (const double *)r.ky.ptr;
    s.ax = (const float *)r.ax.ptr;
    s.ay = (const float *)r.ay.ptr;
    s.thdr = (const int2 *)r.thdr.ptr;
    s.hstart = (const int *)r.hstart.ptr;
    s.hpts = (const int4 *)r.hpts.ptr;
    s.hshift = hshift;
    s.hbits = hbits;
    s.W = W;
    s.H = H;
    s.fx = K.fx;
    s.fy = K.fy;
    s.cx = K.cx;
    s.cy = K.cy;
    s.dq = dq;
    s.dq2 = s.dq * s.dq;
    s.dzmm = dzmm;
    s.delta = d->delta_mm;
    s.tau = d->tau_c;
    s.flags = d->flags;
    s.stride = d->stride;
    s.wtx = wtx;
    s.wty = wty;
    // uploads from the pinned area, then points, colours and the search structure, all on the context stream
    long long *total_dev = (long long *)((char *)tmp.ptr + tmp_main);
    long long *blk_dev = (long long *)((char *)tmp.ptr + tmp_main + 64);
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        hipStream_t cs = ctx->stream;
        auto H2D = [&](DevBuf &b, size_t off, size_t n) {
            if (e == hipSuccess) e = hipMemcpyAsync(b.ptr, hs + off, n, hipMemcpyHostToDevice, cs);
        };
        H2D(r.depth, o_depth, N * 2);
        if (use_rgb) H2D(r.rgb, o_rgb, N * 3);
        if (d->labels) H2D(r.labels, o_lab, N * 4);
        H2D(r.kx, o_kx, W * 8);
        H2D(r.ky, o_ky, H * 8);
        H2D(r.ax, o_ax, W * 4);
        H2D(r.ay, o_ay, H * 4);
        if (e == hipSuccess)
            e = ctx->timed(kProfScenePrep, cs, [&] {
                hipError_t e2 = launch_scene_prep(s, (const uint8_t *)r.rgb.ptr, (int4 *)r.opt.ptr,
                                                  (float4 *)r.olab.ptr, cs);
                if (e2 != hipSuccess) return e2;
                if (hashed) return launch_hash_build(s, (int *)tmp.ptr, blk_dev, cs);
                return launch_table_ranges(s, (uint32_t *)tmp.ptr, (int2 *)r.thdr.ptr, total_dev, blk_dev, cs);
            });
        if (e == hipSuccess && !hashed)
            e = hipMemcpyAsync(hs + o_total, total_dev, 8, hipMemcpyDeviceToHost, cs);
        if (e == hipSuccess && host_total >= 0) {
            s.tnn = (const int32_t *)r.tnn.ptr;
            r.table_entries = host_total;
            r.table_on_host = true;
            e = ctx->timed(kProfScenePrep, cs,
                           [&] { return launch_table_fill(s, (int32_t *)r.tnn.ptr, host_total, cs); });
        }
    }
    if (!hashed && host_total < 0) {
        // the table's size decides its allocation: one wait for it
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        long long total = 0;
        std::memcpy(&total, hs + o_total, 8);
        if (e != hipSuccess) {
            cleanup();
            return fail(PERCH_EDEVICE, "scene upload / preparation: %s", hipGetErrorString(e));
        }
        if (total >= (1LL << 31) - 1) {
            cleanup();
            return fail(PERCH_ENOMEM, "scene neighbour table too large (%lld entries)", total);
        }
        r.table_entries = total;
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        if (perch_status st = ctx->alloc(r.tnn, (size_t)std::max(total, 1LL) * 4)) {
            std::string msg = g_last_error;
            cleanup();
            return fail(st, "%s", msg.c_str());
        }
        s.tnn = (const int32_t *)r.tnn.ptr;
        e = ctx->timed(kProfScenePrep, ctx->stream,
                       [&] { return launch_table_fill(s, (int32_t *)r.tnn.ptr, total, ctx->stream); });
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        cleanup();
        return fail(PERCH_EDEVICE, "scene preparation: %s", hipGetErrorString(e));
    }
    if (host_total >= 0) {
        long long dev_total = 0;
        std::memcpy(&dev_total, hs + o_total, 8);
        if (dev_total != host_total) {
            cleanup();
            return fail(PERCH_EDEVICE, "neighbour table counted %lld entries on the host, %lld on the device", host_total,
                        dev_total);
        }
    }
    if (d->labels) {
        r.host_labels.assign(d->labels, d->labels + N);
        r.host_depth.assign(d->depth_mm, d->depth_mm + N);
    }
    r.bytes = r.depth.bytes + r.rgb.bytes + r.labels.bytes + r.opt.bytes + r.olab.bytes + r.kx.bytes
              + r.ky.bytes + r.ax.bytes + r.ay.bytes + r.thdr.bytes + r.tnn.bytes + r.hstart.bytes + r.hpts.bytes;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->release(tmp);
    ctx->scene_stage.push_back(stg);
    const int32_t id = ctx->next_scene++;
    ctx->scenes[id] = std::move(r);
    *scene_id = id;
    return ok();
}

perch_status perch_drop_scene(perch_ctx *ctx, int32_t scene_id)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    if (perch_status st = release_check(ctx, true, scene_id)) return st;
    SceneRec &r = it->second;
    FenceRef f = ctx->fence_of(r.uses);
    for (DevBuf *b : {&r.depth, &r.rgb, &r.labels, &r.opt, &r.olab, &r.kx, &r.ky, &r.ax, &r.ay, &r.thdr, &r.tnn})
        ctx->release(*b, f);
    ctx->scenes.erase(it);
    return ok();
}

namespace {

// kNN I: one pose at a time, every (rendered, observed) distance in one array.
perch_status score_knn1(perch_ctx *ctx, SceneRec &sr, const MeshRec &mr, int32_t label, const float *poses_dev,
                        int32_t n, int32_t *jr_dev, int32_t *jo_dev, int32_t *nr_dev, int32_t *nq_dev, hipStream_t st)
{
    if (n < 0) return fail(PERCH_EINVAL, "n must be >= 0");
    if (n > 0 && (!poses_dev || !jr_dev || !jo_dev)) return fail(PERCH_EINVAL, "null poses or output");
    if (n == 0) return PERCH_OK;
    StreamBufs &b = ctx->work[st];
    const SceneDev &s = sr.dev;
    const size_t N = (size_t)s.W * s.H;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const bool nnm = (s.flags & PERCH_JO_NN) != 0;
    const size_t o_keys = 256, o_pts = o_keys + up(N * 4), o_pcol = o_pts + up(N * 16), o_obs = o_pcol + up(N * 4),
                 o_mark = o_obs + up(N * 4), bytes = o_mark + up(nnm ? N : 1);
    if (perch_status e = ctx->ensure(b.knn1, bytes)) return e;
    char *base = (char *)b.knn1.ptr;
    Knn1Args a{};
    a.s = s;
    a.m = mr.dev;
    a.poses = poses_dev;
    a.label = label;
    a.keys = (uint32_t *)(base + o_keys);
    a.pts = (int4 *)(base + o_pts);
    a.pcol = (uint32_t *)(base + o_pcol);
    a.obs = (const int *)(base + o_obs);
    a.marked = nnm ? (uint8_t *)(base + o_mark) : nullptr;
    a.counts = (int *)base;
    a.jr = jr_dev;
    a.jo = jo_dev;
    a.nr = nr_dev;
    a.nq = nq_dev;
    int *n_obs_dev = (int *)base + 16;
    HIP_TRY(hipMemsetAsync(n_obs_dev, 0, sizeof(int), st));
    HIP_TRY(knn1_observed(s, (int *)(base + o_obs), n_obs_dev, st));
    int host[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&host[1], n_obs_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    a.n_obs = host[1];
    for (int32_t p = 0; p < n; ++p) {
        HIP_TRY(ctx->timed(kProfRender, st, [&] { return knn1_render(a, p, st); }));
        HIP_TRY(hipMemcpyAsync(&host[0], a.counts, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const int L = host[0];
        const size_t need = (size_t)L * (size_t)a.n_obs * 4;
        if (ctx->ensure(b.knn1_dist, std::max(need, (size_t)256)) != PERCH_OK)
            return fail(PERCH_ENOMEM, "kNN I: the %d x %d distance array of pose %d (%zu bytes) does not fit", L,
                        a.n_obs, p, need);
        a.dist = (uint32_t *)b.knn1_dist.ptr;
        HIP_TRY(ctx->timed(kProfKnn1, st, [&] { return knn1_score(a, p, L, st); }));
    }
    ctx->mark_use(sr.uses, st);
    return PERCH_OK;
}

}  // namespace

perch_status perch_score_poses(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                               const float *poses_dev, int32_t n, int32_t *jr_dev, int32_t *jo_dev,
                               int32_t *nr_dev, int32_t *nq_dev, void *hip_stream)
{
    const Range range_("perch_score_poses");
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    {
        auto si = ctx->scenes.find(scene_id);
        if (si != ctx->scenes.end() && (si->second.dev.flags & PERCH_KNN1)) {
            auto mi = ctx->meshes.find(mesh_id);
            if (mi == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", mesh_id);
            perch_status s = score_knn1(ctx, si->second, mi->second, label, poses_dev, n, jr_dev, jo_dev, nr_dev,
                                        nq_dev, pick_stream(ctx, hip_stream));
            if (s == PERCH_OK) ctx->mark_use(mi->second.uses, pick_stream(ctx, hip_stream));
            return s ? s : ok();
        }
    }
    const perch_work item{scene_id, mesh_id, label, n, poses_dev, jr_dev, jo_dev, nr_dev, nq_dev};
    perch_status s = run_direct(ctx, &item, 1, pick_stream(ctx, hip_stream), false);
    return s ? s : ok();
}

perch_status perch_score_detail(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                const float *poses_dev, int32_t n, int32_t *jr_dev, int32_t *jo_dev,
                                int32_t *nr_dev, int32_t *nq_dev, uint8_t *rflag_dev, uint8_t *oflag_dev,
                                void *hip_stream)
{
    const Range range_("perch_score_detail");
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    if (si->second.dev.flags & PERCH_KNN1) return fail(PERCH_EINVAL, "PERCH_KNN1 scenes have no class images");
    if (n < 1 || n > 256) return fail(PERCH_EINVAL, "n must be in [1, 256]");
    if (!rflag_dev || !oflag_dev) return fail(PERCH_EINVAL, "null class images");
    hipStream_t st = pick_stream(ctx, hip_stream);
    const size_t bytes = (size_t)n * si->second.dev.W * si->second.dev.H;
    HIP_TRY(hipMemsetAsync(rflag_dev, 0, bytes, st));
    HIP_TRY(hipMemsetAsync(oflag_dev, 0, bytes, st));
    const perch_work item{scene_id, mesh_id, label, n, poses_dev, jr_dev, jo_dev, nr_dev, nq_dev};
    perch_status s = run_direct(ctx, &item, 1, st, false, nullptr, nullptr, rflag_dev, oflag_dev);
    return s ? s : ok();
}

perch_status perch_score_poses_noalloc(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                       const float *poses_dev, int32_t n, int32_t *jr_dev, int32_t *jo_dev,
                                       int32_t *nr_dev, int32_t *nq_dev, void *hip_stream)
{
    const Range range_("perch_score_poses_noalloc");
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!ctx->noalloc) return fail(PERCH_EDEVICE, "no scratch address on device %d", ctx->device);
    if (n < 0 || n > kNoAllocMaxPoses)
        return fail(PERCH_EINVAL, "n = %d: the allocation-free path scores 0 to %d poses per call", n,
                    kNoAllocMaxPoses);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    const SceneDev &sd = si->second.dev;
    if (sd.flags & PERCH_KNN1)
        return fail(PERCH_EINVAL, "PERCH_KNN1 scenes need a distance array per pose; use perch_score_poses");
    if ((long long)sd.W * sd.H > kNoAllocMaxPixels)
        return fail(PERCH_EINVAL, "scene of %d x %d pixels: the allocation-free path takes at most %d pixels", sd.W,
                    sd.H, kNoAllocMaxPixels);
    const perch_work item{scene_id, mesh_id, label, n, poses_dev, jr_dev, jo_dev, nr_dev, nq_dev};
    Built b;
    if (perch_status s = build_descriptors(ctx, &item, 1, b)) return s;
    if (b.n_poses == 0) return ok();
    if (b.bytes.size() > (size_t)kDescArgBytes)
        return fail(PERCH_EINVAL, "descriptor block of %zu bytes exceeds %d", b.bytes.size(), kDescArgBytes);
    LaunchCfg cfg = launch_cfg(ctx);
    cfg.grid[2] = std::min(cfg.grid[2], kNoAllocGrid2);
    cfg.grid[3] = std::min(cfg.grid[3], kNoAllocGrid3);
    size_t sw[kNumClasses], sb[kNumClasses], slot_words = 0, tile_words = 0;
    slot_layout(cfg, b.max_pixels, sw, sb, &slot_words, &tile_words);
    // carve the scratch: descriptors | pose info | class lists | counters | slots
    LaunchBufs lb;
    size_t off = 0;
    auto carve = [&](DevBuf &d, size_t bytes) {
        d.ptr = (char *)ctx->noalloc + off;
        d.bytes = bytes;
        off += (bytes + 255) & ~(size_t)255;
    };
    carve(lb.desc, kDescArgBytes);
    carve(lb.info, (size_t)b.n_poses * sizeof(PoseInfo));
    carve(lb.lists, (size_t)kNumClasses * b.n_poses * sizeof(int));
    carve(lb.counts, kCounterInts * 4);
    carve(lb.scratch, slot_words * 4);
    if (off > kNoAllocScratchBytes)
        return fail(PERCH_EINVAL, "launch needs %zu scratch bytes, more than %zu", off, kNoAllocScratchBytes);
    hipStream_t st = pick_stream(ctx, hip_stream);
    hipError_t e = launch_desc_write(b.bytes.data(), b.bytes.size(), lb.desc.ptr, st);
    if (e != hipSuccess) return fail(PERCH_EDEVICE, "descriptor write: %s", hipGetErrorString(e));
    // no CIELAB slots (lb.lab is empty): the J_o colour tests recompute the rendered colours
    const Work w = make_work(lb, b, b.n_poses, cfg, b.max_pixels, false);
    e = enqueue(ctx, w, cfg, b.n_poses, b.n_items, b.any_rgb, b.any_pv, st, false);
    if (e != hipSuccess) return fail(PERCH_EDEVICE, "score launch: %s", hipGetErrorString(e));
    mark_uses(ctx, b.scene_ids, b.mesh_ids, st);
    return ok();
}

perch_status perch_score_batch(perch_ctx *ctx, const perch_work *items, int32_t n_items, void *hip_stream)
{
    const Range range_("perch_score_batch");
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    perch_status s = run_direct(ctx, items, n_items, pick_stream(ctx, hip_stream), false);
    return s ? s : ok();
}

perch_status perch_best_poses(perch_ctx *ctx, int32_t scene_id, int32_t n_obj, const int32_t *mesh_ids,
                              const int32_t *labels, const float *const *poses_dev, const int32_t *n_poses,
                              int32_t *best_idx_host, int32_t *best_cost_host, void *hip_stream)
{
    const Range range_("perch_best_poses");
    if (perch_status st = enter(ctx)) return st;
    if (n_obj < 1) return fail(PERCH_EINVAL, "n_obj must be >= 1");
    if (!mesh_ids || !labels || !poses_dev || !n_poses || !best_idx_host || !best_cost_host)
        return fail(PERCH_EINVAL, "null argument");
    for (int32_t k = 0; k < n_obj; ++k)
        if (n_poses[k] < 1) return fail(PERCH_EINVAL, "object %d has no poses", k);
    hipStream_t st = pick_stream(ctx, hip_stream);
    int n_items = 0;
    std::vector<int> item_of_req;
    const int32_t *best_dev = nullptr;
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        // J_r / J_o land in a per-stream scratch area; only the minima return
        StreamBufs &sb = ctx->work[st];
        size_t need = 0;
        for (int32_t k = 0; k < n_obj; ++k) need += (size_t)n_poses[k] * 8;
        if (perch_status s0 = ctx->ensure(sb.tmp, need)) return s0;
        std::vector<perch_work> items((size_t)n_obj);
        int32_t *base = (int32_t *)sb.tmp.ptr;
        size_t off = 0;
        for (int32_t k = 0; k < n_obj; ++k) {
            items[k] = perch_work{scene_id, mesh_ids[k], labels[k], n_poses[k], poses_dev[k], base + off,
                                  base + off + n_poses[k], nullptr, nullptr};
            off += 2 * (size_t)n_poses[k];
        }
        if (perch_status s = run_direct(ctx, items.data(), n_obj, st, true, &n_items, &item_of_req)) return s;
        best_dev = (const int32_t *)sb.lb.best.ptr;
    }
    // wait without the lock, then fetch the minima
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int32_t> res((size_t)2 * n_items);
    HIP_TRY(hipMemcpy(res.data(), best_dev, res.size() * 4, hipMemcpyDeviceToHost));
    for (int32_t k = 0; k < n_obj; ++k) {
        const int it = item_of_req[k];
        best_idx_host[k] = it >= 0 ? res[2 * it] : -1;
        best_cost_host[k] = it >= 0 ? res[2 * it + 1] : -1;
    }
    return ok();
}

perch_status perch_render(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, const float *poses_dev, int32_t n,
                          uint16_t *depth_dev, uint8_t *rgb_dev, int32_t *tri_dev, void *hip_stream)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    auto mi = ctx->meshes.find(mesh_id);
    if (mi == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", mesh_id);
    if (n < 1 || n > 256) return fail(PERCH_EINVAL, "n must be in [1, 256]");
    if (!poses_dev || !depth_dev) return fail(PERCH_EINVAL, "null poses or depth");
    if (rgb_dev && !mi->second.dev.vrgb) return fail(PERCH_EINVAL, "mesh %d has no vertex colours", mesh_id);
    hipStream_t st = pick_stream(ctx, hip_stream);
    StreamBufs &b = ctx->work[st];
    const SceneDev &s = si->second.dev;
    if (perch_status e = ctx->ensure(b.lb.scratch, (size_t)n * s.W * s.H * 4)) return e;
    HIP_TRY(ctx->timed(kProfRender, st, [&] {
        return launch_render(s, mi->second.dev, poses_dev, n, (uint32_t *)b.lb.scratch.ptr, depth_dev, rgb_dev,
                             tri_dev, st);
    }));
    ctx->mark_use(si->second.uses, st);
    ctx->mark_use(mi->second.uses, st);
    return ok();
}

perch_status perch_refine_poses(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                const float *poses_dev, int32_t n, const perch_icp_params *prm, float *refined_dev,
                                int32_t *iters_dev, int32_t *matched_dev, void *hip_stream)
{
    const Range range_("perch_refine_poses");
    if (perch_status st = enter(ctx)) return st;
    if (!prm) return fail(PERCH_EINVAL, "null ICP parameters");
    if (prm->iterations < 1 || prm->iterations > 1000) return fail(PERCH_EINVAL, "iterations must be in [1, 1000]");
    if (!(prm->max_corr_mm > 0.0f && prm->max_corr_mm <= 100.0f))
        return fail(PERCH_EINVAL, "max_corr_mm must be in (0, 100]");
    if (prm->stride < 1) return fail(PERCH_EINVAL, "stride must be >= 1");
    if (prm->dof != 3 && prm->dof != 6) return fail(PERCH_EINVAL, "dof must be 3 or 6");
    if (prm->min_points < 3) return fail(PERCH_EINVAL, "min_points must be >= 3");
    if (prm->method != PERCH_ICP_POINT && prm->method != PERCH_ICP_PLANE)
        return fail(PERCH_EINVAL, "method must be PERCH_ICP_POINT or PERCH_ICP_PLANE");
    if (prm->method == PERCH_ICP_PLANE && prm->dof != 6) return fail(PERCH_EINVAL, "GICP (PERCH_ICP_PLANE) is 6-DoF");
    if (n < 0) return fail(PERCH_EINVAL, "n must be >= 0");
    if (n > 0 && (!poses_dev || !refined_dev)) return fail(PERCH_EINVAL, "null poses or output");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    auto mi = ctx->meshes.find(mesh_id);
    if (mi == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", mesh_id);
    if (n == 0) return ok();
    hipStream_t st = pick_stream(ctx, hip_stream);
    StreamBufs &b = ctx->work[st];
    const SceneDev &s = si->second.dev;
    const int grid = std::min(n, std::max(ctx->n_cu, 1));
    const size_t px = (size_t)s.W * s.H;
    const size_t tiles_off = 256, pts_off = tiles_off + (size_t)grid * px * 4;
    const int slots = prm->method == PERCH_ICP_PLANE ? 3 : 2;   // source, mapped (+ normals for GICP)
    const size_t bytes = pts_off + (size_t)grid * slots * px * sizeof(int4);
    if (perch_status e = ctx->ensure(b.icp, bytes)) return e;
    IcpArgs a{};
    a.s = s;
    a.m = mi->second.dev;
    a.poses = poses_dev;
    a.n = n;
    a.label = label;
    a.iterations = prm->iterations;
    a.stride = prm->stride;
    a.dof = prm->dof;
    a.min_points = prm->min_points;
    a.method = prm->method;
    a.rq = (int)std::nearbyint(16.0 * (double)prm->max_corr_mm);
    a.rq2 = a.rq * a.rq;
    a.box[0] = 0;
    a.box[1] = 0;
    a.box[2] = s.W - 1;
    a.box[3] = s.H - 1;
    if ((s.flags & PERCH_VOL_MASK) == PERCH_VOL_LABEL) {   // only the label's pixels can match
        const std::vector<int> lb = label_box(si->second, label);
        a.box[0] = lb[0];
        a.box[1] = lb[1];
        a.box[2] = lb[0] + lb[2] - 1;
        a.box[3] = lb[1] + lb[3] - 1;
    }
    a.lds_words = ctx->icp_lds_words;
    a.refined = refined_dev;
    a.iters = iters_dev;
    a.matched = matched_dev;
    char *base = (char *)b.icp.ptr;
    a.cursor = (int *)base;
    a.tiles = (uint32_t *)(base + tiles_off);
    a.pts = (int4 *)(base + pts_off);
    a.pts_cap = px;
    HIP_TRY(ctx->timed(kProfIcp, st, [&] { return launch_icp(a, grid, st); }));
    ctx->mark_use(si->second.uses, st);
    ctx->mark_use(mi->second.uses, st);
    return ok();
}

namespace {

// Layout of a stream's tree buffer: cursor and flag, then the raster keys of
// a composition, the placed poses, the per-work-group tiles and the scores.
struct MsgLayout {
    size_t keys, poses, tiles, out, bytes;
};
static MsgLayout msg_layout(size_t px, int grid, size_t n_poses, size_t n_out)
{
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    MsgLayout l;
    l.keys = 512;
    l.poses = l.keys + up(px * 4);
    l.tiles = l.poses + up(n_poses * 12 * sizeof(float));
    l.out = l.tiles + up((size_t)grid * px * 4);
    l.bytes = l.out + up(n_out * 3 * sizeof(int32_t));
    return l;
}

static perch_status msg_check_scene(const SceneRec &sr)
{
    if (sr.dev.flags & PERCH_JO_NN) return fail(PERCH_EINVAL, "the tree search does not take PERCH_JO_NN");
    if (sr.dev.flags & PERCH_KNN1) return fail(PERCH_EINVAL, "the tree search does not take PERCH_KNN1");
    return PERCH_OK;
}

static MsgArgs msg_args(perch_ctx *ctx, SceneRec &sr, const MeshRec &mr, int32_t label, const MsgState &st,
                 const float *poses_dev, int n, char *base, const MsgLayout &l)
{
    MsgArgs a{};
    a.s = sr.dev;
    a.m = mr.dev;
    a.poses = poses_dev;
    a.n = n;
    a.label = label;
    if ((sr.dev.flags & PERCH_VOL_MASK) == PERCH_VOL_LABEL) {
        const std::vector<int> lb = label_box(sr, label);
        for (int c = 0; c < 4; ++c) a.vbox[c] = lb[c];
    }
    a.st = st;
    a.lds_words = ctx->msg_lds_words;
    a.tiles = (uint32_t *)(base + l.tiles);
    a.cursor = (int *)base;
    return a;
}

}  // namespace

perch_status perch_msg_expand(perch_ctx *ctx, int32_t scene_id, const perch_placed *state, int32_t n_state,
                              int32_t mesh_id, int32_t label, const float *poses_dev, int32_t n,
                              int32_t *valid_dev, int32_t *jr_dev, int32_t *jo_dev, int32_t *nr_dev,
                              int32_t *nq_dev, void *hip_stream)
{
    const Range range_("perch_msg_expand");
    if (perch_status st = enter(ctx)) return st;
    if (n < 0 || n_state < 0 || n_state > 32) return fail(PERCH_EINVAL, "n must be >= 0 and n_state in [0, 32]");
    if (n_state > 0 && !state) return fail(PERCH_EINVAL, "null state");
    if (n > 0 && (!poses_dev || !valid_dev || !jr_dev || !jo_dev)) return fail(PERCH_EINVAL, "null poses or output");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    SceneRec &sr = si->second;
    if (perch_status e = msg_check_scene(sr)) return e;
    auto mi = ctx->meshes.find(mesh_id);
    if (mi == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", mesh_id);
    for (int k = 0; k < n_state; ++k) {
        if (!ctx->meshes.count(state[k].mesh_id)) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", state[k].mesh_id);
        for (int c = 0; c < 12; ++c)
            if (!std::isfinite(state[k].pose[c])) return fail(PERCH_EINVAL, "state pose %d is not finite", k);
    }
    hipStream_t st = pick_stream(ctx, hip_stream);
    StreamBufs &b = ctx->work[st];
    const SceneDev &s = sr.dev;
    const size_t px = (size_t)s.W * s.H;
    const int grid = std::max(1, std::min(n, std::max(ctx->n_cu, 1)));
    const MsgLayout l = msg_layout(px, grid, (size_t)n_state, 0);
    if (perch_status e = ctx->ensure(b.msg, l.bytes)) return e;
    if (perch_status e = ctx->ensure(b.msg_states[0], msg_state_bytes(px))) return e;
    char *base = (char *)b.msg.ptr;
    const bool rgb = (s.flags & PERCH_USE_RGB) != 0;
    const MsgState ms = msg_state_at(b.msg_states[0].ptr, px, rgb);
    int *flag = (int *)(base + 256);
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
    HIP_TRY(msg_state_clear(s, ms, st));
    if (n_state > 0) {
        std::vector<float> hp((size_t)n_state * 12);
        for (int k = 0; k < n_state; ++k) std::memcpy(&hp[(size_t)k * 12], state[k].pose, 12 * sizeof(float));
        float *dp = (float *)(base + l.poses);
        HIP_TRY(hipMemcpyAsync(dp, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice, st));
        for (int k = 0; k < n_state; ++k) {
            MsgAddArgs a{};
            a.s = s;
            a.m = ctx->meshes[state[k].mesh_id].dev;
            a.pose = dp + 12 * (size_t)k;
            a.label = state[k].label;
            a.st = ms;
            a.keys = (uint32_t *)(base + l.keys);
            a.flag = flag;
            HIP_TRY(msg_state_add(a, st));
        }
        HIP_TRY(msg_state_near(s, ms, st));
        int hflag = 0;
        HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (hflag) return fail(PERCH_EINVAL, "the state is not monotone: an object occludes one placed before it");
    }
    if (n > 0) {
        MsgArgs a = msg_args(ctx, sr, mi->second, label, ms, poses_dev, n, base, l);
        a.valid = valid_dev;
        a.jr = jr_dev;
        a.jo = jo_dev;
        a.nr = nr_dev;
        a.nq = nq_dev;
        HIP_TRY(ctx->timed(kProfMsg, st, [&] { return launch_msg(a, grid, st); }));
    }
    ctx->mark_use(sr.uses, st);
    ctx->mark_use(mi->second.uses, st);
    for (int k = 0; k < n_state; ++k) ctx->mark_use(ctx->meshes[state[k].mesh_id].uses, st);
    return ok();
}

perch_status perch_msg_search(perch_ctx *ctx, int32_t scene_id, const perch_msg_object *objects, int32_t n_obj,
                              int32_t beam, int32_t *order_host, int32_t *pose_host, int64_t *cost_host,
                              int64_t *scored_host, void *hip_stream)
{
    const Range range_("perch_msg_search");
    if (perch_status st = enter(ctx)) return st;
    if (n_obj < 1 || n_obj > 32) return fail(PERCH_EINVAL, "n_obj must be in [1, 32]");
    if (!objects || !order_host || !pose_host || !cost_host) return fail(PERCH_EINVAL, "null argument");
    if (beam < 0) return fail(PERCH_EINVAL, "beam must be >= 0");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    SceneRec &sr = si->second;
    if (perch_status e = msg_check_scene(sr)) return e;
    size_t max_n = 0;
    for (int o = 0; o < n_obj; ++o) {
        if (!ctx->meshes.count(objects[o].mesh_id))
            return fail(PERCH_ENOTFOUND, "unknown mesh id %d", objects[o].mesh_id);
        if (objects[o].n_poses < 0 || (objects[o].n_poses > 0 && !objects[o].poses_dev))
            return fail(PERCH_EINVAL, "object %d: bad poses", o);
        max_n = std::max(max_n, (size_t)objects[o].n_poses);
    }
    for (int l = 0; l < n_obj; ++l) order_host[l] = pose_host[l] = -1;
    *cost_host = -1;
    if (scored_host) *scored_host = 0;
    hipStream_t st = pick_stream(ctx, hip_stream);
    StreamBufs &b = ctx->work[st];
    const SceneDev &s = sr.dev;
    const size_t px = (size_t)s.W * s.H;
    const size_t sb = msg_state_bytes(px);
    const bool rgb = (s.flags & PERCH_USE_RGB) != 0;
    const int grid = std::max(1, std::min((int)std::max<size_t>(max_n, 1), std::max(ctx->n_cu, 1)));

    struct Node {
        int64_t cost;
        std::vector<std::pair<int, int>> seq;   // (object, pose index) in placement order
        uint32_t placed;
    };
    std::vector<Node> cur(1, Node{0, {}, 0u});
    int cur_buf = 0;
    if (perch_status e = ctx->ensure(b.msg_states[cur_buf], sb)) return e;
    HIP_TRY(msg_state_clear(s, msg_state_at(b.msg_states[cur_buf].ptr, px, rgb), st));
    int64_t scored = 0;
    for (int level = 0; level < n_obj; ++level) {
        // every successor of every state, scored into one output array
        size_t total = 0;
        for (const Node &nd : cur)
            for (int o = 0; o < n_obj; ++o)
                if (!(nd.placed >> o & 1u)) total += (size_t)objects[o].n_poses;
        const MsgLayout l = msg_layout(px, grid, 0, total);
        if (perch_status e = ctx->ensure(b.msg, l.bytes)) return e;
        char *base = (char *)b.msg.ptr;
        int32_t *outd = (int32_t *)(base + l.out);
        size_t off = 0;
        for (size_t c = 0; c < cur.size(); ++c) {
            const MsgState ms = msg_state_at((char *)b.msg_states[cur_buf].ptr + c * sb, px, rgb);
            for (int o = 0; o < n_obj; ++o) {
                if (cur[c].placed >> o & 1u) continue;
                const int n = objects[o].n_poses;
                if (n == 0) continue;
                MsgArgs a = msg_args(ctx, sr, ctx->meshes[objects[o].mesh_id], objects[o].label, ms,
                                     objects[o].poses_dev, n, base, l);
                a.valid = outd + off;
                a.jr = outd + total + off;
                a.jo = outd + 2 * total + off;
                HIP_TRY(ctx->timed(kProfMsg, st, [&] { return launch_msg(a, std::min(grid, n), st); }));
                off += (size_t)n;
            }
        }
        std::vector<int32_t> h(3 * total);
        if (total > 0) HIP_TRY(hipMemcpyAsync(h.data(), outd, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        scored += (int64_t)total;
        // the states' lexicographic ranks; children compare as (cost, parent rank, object, pose)
        std::vector<int> idx(cur.size()), rank(cur.size());
        for (size_t c = 0; c < cur.size(); ++c) idx[c] = (int)c;
        std::sort(idx.begin(), idx.end(), [&](int x, int y) { return cur[x].seq < cur[y].seq; });
        for (size_t r = 0; r < idx.size(); ++r) rank[idx[r]] = (int)r;
        struct Cand {
            int64_t cost;
            int prank, o, k, parent;
        };
        std::vector<Cand> cand;
        off = 0;
        for (size_t c = 0; c < cur.size(); ++c)
            for (int o = 0; o < n_obj; ++o) {
                if (cur[c].placed >> o & 1u) continue;
                for (int k = 0; k < objects[o].n_poses; ++k, ++off)
                    if (h[off]) cand.push_back(Cand{cur[c].cost + h[total + off] + h[2 * total + off], rank[c], o, k, (int)c});
            }
        auto less = [](const Cand &x, const Cand &y) {
            if (x.cost != y.cost) return x.cost < y.cost;
            if (x.prank != y.prank) return x.prank < y.prank;
            if (x.o != y.o) return x.o < y.o;
            return x.k < y.k;
        };
        const size_t keep = beam > 0 ? std::min(cand.size(), (size_t)beam) : cand.size();
        std::partial_sort(cand.begin(), cand.begin() + keep, cand.end(), less);
        cand.resize(keep);
        if (cand.empty()) break;                       // every state is a dead end
        std::vector<Node> next(keep);
        for (size_t c = 0; c < keep; ++c) {
            const Node &par = cur[cand[c].parent];
            next[c].cost = cand[c].cost;
            next[c].seq = par.seq;
            next[c].seq.emplace_back(cand[c].o, cand[c].k);
            next[c].placed = par.placed | (1u << cand[c].o);
        }
        if (level == n_obj - 1) {
            for (int q = 0; q < n_obj; ++q) {
                order_host[q] = next[0].seq[q].first;
                pose_host[q] = next[0].seq[q].second;
            }
            *cost_host = next[0].cost;
            break;
        }
        // the kept states' planes: the parent's, with the new object appended
        const int nb = 1 - cur_buf;
        if (beam == 0 && ctx->budget && ctx->used + keep * sb > ctx->budget)
            return fail(PERCH_ENOMEM, "exhaustive search: %zu states of %zu bytes exceed the budget", keep, sb);
        if (perch_status e = ctx->ensure(b.msg_states[nb], keep * sb)) return e;
        char *base2 = (char *)b.msg.ptr;
        for (size_t c = 0; c < keep; ++c) {
            char *dst = (char *)b.msg_states[nb].ptr + c * sb;
            HIP_TRY(hipMemcpyAsync(dst, (char *)b.msg_states[cur_buf].ptr + (size_t)cand[c].parent * sb, sb,
                                   hipMemcpyDeviceToDevice, st));
            const MsgState ms = msg_state_at(dst, px, rgb);
            MsgAddArgs a{};
            a.s = s;
            a.m = ctx->meshes[objects[cand[c].o].mesh_id].dev;
            a.pose = objects[cand[c].o].poses_dev + 12 * (size_t)cand[c].k;
            a.label = objects[cand[c].o].label;
            a.st = ms;
            a.keys = (uint32_t *)(base2 + l.keys);
            a.flag = (int *)(base2 + 256);
            HIP_TRY(msg_state_add(a, st));
            HIP_TRY(msg_state_near(s, ms, st));
        }
        cur.swap(next);
        cur_buf = nb;
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (scored_host) *scored_host = scored;
    ctx->mark_use(sr.uses, st);
    for (int o = 0; o < n_obj; ++o) ctx->mark_use(ctx->meshes[objects[o].mesh_id].uses, st);
    return ok();
}

perch_status perch_propose_poses(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                 const perch_proposal_params *prm, float *poses_dev, int32_t capacity, int32_t *n_out,
                                 void *hip_stream)
{
    const Range range_("perch_propose_poses");
    if (perch_status st = enter(ctx)) return st;
    if (!prm || !n_out) return fail(PERCH_EINVAL, "null parameters or count");
    if (prm->viewpoints < 1 || prm->inplane < 1 || prm->max_depths < 1)
        return fail(PERCH_EINVAL, "viewpoints, inplane and max_depths must be >= 1");
    if (!(prm->z_step_mm > 0.0f)) return fail(PERCH_EINVAL, "z_step_mm must be > 0");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto si = ctx->scenes.find(scene_id);
    if (si == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    if (si->second.host_labels.empty()) return fail(PERCH_EINVAL, "scene %d has no labels", scene_id);
    auto mi = ctx->meshes.find(mesh_id);
    if (mi == ctx->meshes.end()) return fail(PERCH_ENOTFOUND, "unknown mesh id %d", mesh_id);
    const std::vector<int> lb = label_box(si->second, label);
    *n_out = 0;
    if (lb[2] == 0 || lb[5] < lb[4]) return ok();      // no labelled pixel with a depth reading
    long long T = (long long)std::floor((double)(lb[5] - lb[4]) / (double)prm->z_step_mm) + 1;
    const bool spread = T > prm->max_depths;
    if (spread) T = prm->max_depths;
    const long long n = (long long)prm->viewpoints * prm->inplane * T;
    if (n > (1LL << 30)) return fail(PERCH_EINVAL, "too many proposals (%lld)", n);
    *n_out = (int32_t)n;
    if (!poses_dev) return ok();                       // count only
    if (capacity < n) return fail(PERCH_EINVAL, "capacity %d < %lld proposals", capacity, n);
    const SceneDev &s = si->second.dev;
    ProposalArgs a{};
    a.M = prm->viewpoints;
    a.N = prm->inplane;
    a.T = (int)T;
    a.zmin = (double)lb[4];
    a.zmax = (double)lb[5];
    a.step = spread ? (T > 1 ? (a.zmax - a.zmin) / (double)(T - 1) : 0.0) : (double)prm->z_step_mm;
    a.uc = (double)lb[0] + (double)(lb[2] - 1) / 2.0;
    a.vc = (double)lb[1] + (double)(lb[3] - 1) / 2.0;
    a.fx = s.fx;
    a.fy = s.fy;
    a.cx = s.cx;
    a.cy = s.cy;
    for (int c = 0; c < 3; ++c)
        a.centre[c] = ((double)mi->second.dev.lo[c] + (double)mi->second.dev.hi[c]) / 2.0;
    a.out = poses_dev;
    a.n = (int)n;
    HIP_TRY(launch_proposals(a, pick_stream(ctx, hip_stream)));
    return ok();
}

perch_status perch_profile_enable(perch_ctx *ctx, int32_t enable)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->collect();
    for (int k = 0; k < kNumProfSlots; ++k) {
        ctx->total_ms[k] = 0.0;
        ctx->launches[k] = 0;
    }
    ctx->prof = enable != 0;
    return ok();
}

perch_status perch_profile_read(perch_ctx *ctx, int32_t n_slots, double *total_ms, int32_t *launches)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (n_slots < 0 || (n_slots > 0 && (!total_ms || !launches))) return fail(PERCH_EINVAL, "bad output arrays");
    ctx->collect();
    for (int k = 0; k < n_slots; ++k) {
        total_ms[k] = k < kNumProfSlots ? ctx->total_ms[k] : 0.0;
        launches[k] = k < kNumProfSlots ? ctx->launches[k] : 0;
    }
    return ok();
}

perch_status perch_set_tuning(perch_ctx *ctx, const perch_tuning *t)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!t) {
        ctx->tune = perch_tuning{};
        return ok();
    }
    if (t->small_block != 0 && t->small_block != 256 && t->small_block != 512)
        return fail(PERCH_EINVAL, "small_block must be 0, 256 or 512 (got %d)", t->small_block);
    if (t->small_words < 0) return fail(PERCH_EINVAL, "small_words must be >= 0");
    for (int k = 0; k < kNumClasses; ++k)
        if (t->grid[k] < 0) return fail(PERCH_EINVAL, "grid[%d] must be >= 0", k);
    if (t->order < 0 || t->order > 2) return fail(PERCH_EINVAL, "order must be 0, 1 or 2");
    if (t->key_bands < 0 || t->key_bands > 2) return fail(PERCH_EINVAL, "key_bands must be 0, 1 or 2");
    ctx->tune = *t;
    return ok();
}

perch_status perch_get_tuning(perch_ctx *ctx, perch_tuning *out)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!out) return fail(PERCH_EINVAL, "null output");
    const LaunchCfg c = launch_cfg(ctx);
    out->small_block = c.small_block;
    out->small_words = c.cap_small;
    for (int k = 0; k < kNumClasses; ++k) out->grid[k] = c.grid[k];
    out->order = c.sort ? 2 : 1;
    out->key_bands = c.key_bands ? 2 : 1;
    return ok();
}

perch_status perch_scene_info_get(perch_ctx *ctx, int32_t scene_id, perch_scene_info *out)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!out) return fail(PERCH_EINVAL, "null output");
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(PERCH_ENOTFOUND, "unknown scene id %d", scene_id);
    const SceneRec &r = it->second;
    const LaunchCfg c = launch_cfg(ctx);
    out->device_bytes = r.bytes;
    out->table_entries = (int64_t)r.table_entries;
    out->window_x = r.dev.wtx;
    out->window_y = r.dev.wty;
    out->tile_cap_small = c.cap_small;
    out->tile_cap_large = c.cap_large;
    out->table_counted_on_host = r.table_on_host ? 1 : 0;
    out->reserved = 0;
    return ok();
}

perch_status perch_last_classes(perch_ctx *ctx, void *hip_stream, int32_t n, int32_t *class_host)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t st = pick_stream(ctx, hip_stream);
    auto it = ctx->work.find(st);
    if (it == ctx->work.end() || it->second.last_n <= 0) return fail(PERCH_ENOTFOUND, "no scoring call on this stream");
    StreamBufs &b = it->second;
    if (n != b.last_n || !class_host) return fail(PERCH_EINVAL, "n must equal the last call's %d poses", b.last_n);
    std::vector<int32_t> counts(kNumClasses), lists((size_t)kNumClasses * n);
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(counts.data(), b.lb.counts.ptr, kNumClasses * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(lists.data(), b.lb.lists.ptr, lists.size() * 4, hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < n; ++i) class_host[i] = -1;
    for (int c = 0; c < kNumClasses; ++c)
        for (int32_t k = 0; k < counts[c] && k < n; ++k) {
            const int32_t p = lists[(size_t)c * n + k];
            if (p >= 0 && p < n) class_host[p] = c;
        }
    return ok();
}

perch_status perch_batch_create(perch_ctx *ctx, int32_t max_items, int32_t max_poses, int32_t max_image_pixels,
                               perch_batch **out)
{
    if (perch_status st = enter(ctx)) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!out) return fail(PERCH_EINVAL, "null output pointer");
    *out = nullptr;
    if (max_items < 1 || max_poses < 1 || max_image_pixels < 1 || max_poses >= (1 << 30))
        return fail(PERCH_EINVAL, "capacities must be positive (max_poses < 2^30)");
    auto *b = new perch_batch();
    b->ctx = ctx;
    b->cap_items = max_items;
    b->cap_poses = max_poses;
    b->cap_pixels = (size_t)max_image_pixels;
    b->desc_cap = desc_capacity(max_items);
    b->cfg = launch_cfg(ctx);
    auto cleanup = [&](perch_status st, const char *what, hipError_t e) {
        std::string msg = e != hipSuccess ? std::string(what) + ": " + hipGetErrorString(e) : g_last_error;
        for (DevBuf *d : {&b->lb.desc, &b->lb.info, &b->lb.lists, &b->lb.counts, &b->lb.scratch, &b->lb.best,
                          &b->lb.lab})
            ctx->release(*d);
        if (b->pin_desc) (void)hipHostFree(b->pin_desc);
        if (b->pin_best) (void)hipHostFree(b->pin_best);
        for (int g = 0; g < 2; ++g) {
            if (b->exec[g]) (void)hipGraphExecDestroy(b->exec[g]);
            if (b->graph[g]) (void)hipGraphDestroy(b->graph[g]);
        }
        if (b->cap) (void)hipStreamDestroy(b->cap);
        if (b->done) (void)hipEventDestroy(b->done);
        delete b;
        return fail(st, "%s", msg.c_str());
    };
    if (perch_status st = ensure_bufs(ctx, b->lb, b->desc_cap, max_poses, max_items, b->cap_pixels, b->cfg, true))
        return cleanup(st, "", hipSuccess);
    hipError_t e = hipHostMalloc(&b->pin_desc, b->desc_cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&b->pin_best, (size_t)8 * max_items, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) return cleanup(PERCH_EDEVICE, "batch set-up", e);
    std::memset(b->pin_desc, 0, b->desc_cap);   // header: no items, no poses
    Built layout;
    layout.scenes_off = 64 + align64((size_t)max_items * sizeof(ItemDev));
    layout.meshes_off = layout.scenes_off + align64((size_t)max_items * sizeof(SceneDev));
    const Work w = make_work(b->lb, layout, max_poses, b->cfg, b->cap_pixels, true);
    for (int g = 0; g < 2 && e == hipSuccess; ++g) {
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t c = hipMemcpyAsync(b->lb.desc.ptr, b->pin_desc, b->desc_cap, hipMemcpyHostToDevice, b->cap);
            if (c == hipSuccess) c = enqueue(ctx, w, b->cfg, max_poses, max_items, true, g == 1, b->cap, false);
            if (c == hipSuccess)
                c = hipMemcpyAsync(b->pin_best, b->lb.best.ptr, (size_t)8 * max_items, hipMemcpyDeviceToHost, b->cap);
            e = hipStreamEndCapture(b->cap, &b->graph[g]);
            if (c != hipSuccess) e = c;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[g], b->graph[g], nullptr, nullptr, 0);
    }
    if (e != hipSuccess) return cleanup(PERCH_EDEVICE, "batch graph capture", e);
    ctx->batches.push_back(b);
    *out = b;
    return ok();
}

perch_status perch_batch_set(perch_batch *b, const perch_work *items, int32_t n_items)
{
    if (!b) return fail(PERCH_EINVAL, "null batch");
    perch_ctx *ctx = b->ctx;
    if (perch_status st = enter(ctx)) return st;
    if (b->pending) {
        HIP_TRY(hipEventSynchronize(b->done));
        b->pending = false;
    }
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Built d;
    if (perch_status s = build_descriptors(ctx, items, n_items, d, b->cap_items)) {
        b->valid = false;
        return s;
    }
    if (d.n_poses > b->cap_poses || d.max_pixels > b->cap_pixels) {
        b->valid = false;
        return fail(PERCH_EINVAL, "batch capacity exceeded (%d poses of %d, %zu pixels of %zu)", d.n_poses,
                    b->cap_poses, d.max_pixels, b->cap_pixels);
    }
    std::memcpy(b->pin_desc, d.bytes.data(), std::min(d.bytes.size(), b->desc_cap));
    b->scene_ids = d.scene_ids;
    b->mesh_ids = d.mesh_ids;
    b->item_of_req = d.item_of_req;
    b->n_req = n_items;
    b->any_pv = d.any_pv;
    b->valid = true;
    return ok();
}

perch_status perch_batch_launch(perch_batch *b, void *hip_stream)
{
    const Range range_("perch_batch_launch");
    if (!b) return fail(PERCH_EINVAL, "null batch");
    perch_ctx *ctx = b->ctx;
    if (perch_status st = enter(ctx)) return st;
    if (b->pending) HIP_TRY(hipEventSynchronize(b->done));
    b->pending = false;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (!b->valid) return fail(PERCH_EINVAL, "batch has no valid work (set it again)");
    hipStream_t st = pick_stream(ctx, hip_stream);
    HIP_TRY(ctx->timed(kProfGraph, st, [&] { return hipGraphLaunch(b->exec[b->any_pv ? 1 : 0], st); }));
    HIP_TRY(hipEventRecord(b->done, st));
    b->pending = true;
    mark_uses(ctx, b->scene_ids, b->mesh_ids, st);
    return ok();
}

perch_status perch_batch_wait(perch_batch *b, int32_t *best_idx_host, int32_t *best_cost_host)
{
    if (!b) return fail(PERCH_EINVAL, "null batch");
    perch_ctx *ctx = b->ctx;
    if (perch_status st = enter(ctx)) return st;
    if (!b->pending) return fail(PERCH_EINVAL, "batch was not launched");
    HIP_TRY(hipEventSynchronize(b->done));
    b->pending = false;
    const int32_t *res = (const int32_t *)b->pin_best;
    for (int32_t r = 0; r < b->n_req; ++r) {
        const int it = b->item_of_req[r];
        if (best_idx_host) best_idx_host[r] = it >= 0 ? res[2 * it] : -1;
        if (best_cost_host) best_cost_host[r] = it >= 0 ? res[2 * it + 1] : -1;
    }
    return ok();
}

perch_status perch_batch_query(perch_batch *b)
{
    if (!b) return fail(PERCH_EINVAL, "null batch");
    if (!b->pending) return ok();
    const hipError_t e = hipEventQuery(b->done);
    if (e == hipSuccess) return ok();
    if (e == hipErrorNotReady) {
        g_last_error = "batch still running";
        return PERCH_EBUSY;
    }
    return fail(PERCH_EDEVICE, "hipEventQuery: %s", hipGetErrorString(e));
}

perch_status perch_batch_destroy(perch_batch *b)
{
    if (!b) return ok();
    perch_ctx *ctx = b->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    if (b->pending) (void)hipEventSynchronize(b->done);
    for (int g = 0; g < 2; ++g) {
        (void)hipGraphExecDestroy(b->exec[g]);
        (void)hipGraphDestroy(b->graph[g]);
    }
    (void)hipStreamDestroy(b->cap);
    (void)hipEventDestroy(b->done);
    (void)hipHostFree(b->pin_desc);
    (void)hipHostFree(b->pin_best);
    for (DevBuf *d : {&b->lb.desc, &b->lb.info, &b->lb.lists, &b->lb.counts, &b->lb.scratch, &b->lb.best, &b->lb.lab})
        ctx->release(*d);
    ctx->batches.erase(std::find(ctx->batches.begin(), ctx->batches.end(), b));
    delete b;
    return ok();
}

}  // extern "C"
