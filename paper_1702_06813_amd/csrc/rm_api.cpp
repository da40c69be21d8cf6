// Host runtime of the rendermap C ABI: context, argument validation, scratch
// arena, batch descriptors, tile autotuner and stream capture helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "rm_internal.h"

using namespace rm;

struct rm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;
    size_t scratch_size = 0;
    int32_t* pinned = nullptr;        // small host readback buffer
    std::string err;
    int tile_w = 0, tile_h = 0;       // 0 = automatic
    int schedule = 0;                 // 0 automatic (= 2), 1 one workgroup per item, 2 persistent longest-first
    bool autotune = false;
    // tuned tile per launch shape: {mode, n_tris, n_scans, then width, height,
    // pose count of every scan}
    std::map<std::vector<int64_t>, std::pair<int, int>> tuned;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool profiling = false;
    // timed launches of the rasterizer ([0]) and of the binning kernel ([1])
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events[2];
    size_t prof_used[2] = {0, 0};
    // tile-bin capacity, adapted from the largest bins of earlier calls, unless
    // fixed by rm_set_bin_cap (then never grown), and the part of it for large
    // footprints (at most half), adapted from the largest large fill
    int32_t bin_cap = 1024;
    int32_t big_cap = 256;
    int32_t small_want = 0;           // learned slots for small footprints
    int32_t bin_cap_fixed = 0;
    int64_t bin_budget = (int64_t)32 << 30;   // bins and overflow together: a quarter of the device memory
    // overflow (spill list and regions): -1 adaptive, 0 none, > 0 fixed
    // entries (rm_set_bin_pool); adaptively it takes part in calls once a bin
    // has outgrown its capacity, sized from what earlier calls spilled
    int64_t pool_mode = -1;
    int64_t list_want = 0;            // spill-list entries learned (adaptive)
    int64_t region_want = 0;          // overflow-region entries learned (adaptive)
    // launch shapes (records, tile, triangles, poses) whose bins have outgrown
    // a capacity that could not grow: their calls bin with the spilling kernel
    // (which also measures what overflow must hold) and get overflow room
    std::set<std::tuple<int64_t, int, int, int64_t, int>> track_shapes;
    std::tuple<int64_t, int, int, int64_t, int> pending_shape;   // of the pending readback
    hipEvent_t bin_ev = nullptr;      // recorded after the readback of the largest bins
    bool bin_pending = false;
    bool pool_pending = false;        // the pending readback includes what the call spilled
    int32_t last_cap_s = 0, last_cap_b = 0;   // bin parts of the call whose readback is pending
    // launch shapes whose bins were sized by a synchronous check after binning
    std::set<std::tuple<int64_t, int, int, int64_t, int>> bin_checked;
    // once a graph has been captured, scratch that it may reference is never freed early
    bool captured = false;
    std::vector<void*> retired;
};

namespace {

thread_local std::string g_err;

int fail(rm_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_err = buf;
    return code;
}

#define RM_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, RM_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool capturing(rm_ctx* ctx) {
    hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &s) != hipSuccess) return false;
    return s != hipStreamCaptureStatusNone;
}

// Bump allocator over the context scratch; sizes first, then carve.
struct Carve {
    size_t off = 0;
    template <typename T>
    size_t take(int64_t n) {
        const size_t o = off;
        off += ((size_t)std::max<int64_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
        return o;
    }
};

int ensure_scratch(rm_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->scratch_size) return RM_OK;
    if (capturing(ctx))
        return fail(ctx, RM_ERR_CAPACITY, "scratch must grow to %zu bytes during stream capture; "
                                          "run the call once before capturing", bytes);
    RM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->scratch) {
        if (ctx->captured) ctx->retired.push_back(ctx->scratch);
        else RM_HIP(ctx, hipFree(ctx->scratch));
    }
    ctx->scratch = nullptr;
    ctx->scratch_size = 0;
    // a quarter more for later calls that need a little more, at most 2 GiB
    const size_t sz = std::max(bytes + std::min(bytes / 4, (size_t)2 << 30), (size_t)1 << 20);
    if (hipMalloc(&ctx->scratch, sz) != hipSuccess) {
        ctx->scratch = nullptr;
        (void)hipGetLastError();
        return fail(ctx, RM_ERR_OOM, "could not allocate %zu bytes of scratch", sz);
    }
    ctx->scratch_size = sz;
    return RM_OK;
}

template <typename T>
T* at(rm_ctx* ctx, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ctx->scratch) + off); }

int check_camera(rm_ctx* ctx, const rm_camera& c) {
    if (c.width < 1 || c.height < 1 || c.width > 4096 || c.height > 4096)
        return fail(ctx, RM_ERR_INVALID_ARG, "image size %dx%d outside 1..4096", c.width, c.height);
    if (!(std::isfinite(c.fx) && std::isfinite(c.fy) && c.fx != 0.0f && c.fy != 0.0f &&
          std::isfinite(c.cx) && std::isfinite(c.cy)))
        return fail(ctx, RM_ERR_INVALID_ARG, "camera intrinsics must be finite with fx, fy != 0");
    if (std::fabs(c.cx) > 8192.0f || std::fabs(c.cy) > 8192.0f)
        return fail(ctx, RM_ERR_INVALID_ARG, "principal point beyond 8192 px");
    if (!(c.z_near > 0.0f && c.z_far > c.z_near && std::isfinite(c.z_far)))
        return fail(ctx, RM_ERR_INVALID_ARG, "need 0 < z_near < z_far < inf (got %g, %g)", c.z_near, c.z_far);
    return RM_OK;
}

int check_mesh(rm_ctx* ctx, const rm_mesh* m) {
    if (!m) return fail(ctx, RM_ERR_INVALID_ARG, "mesh is NULL");
    if (m->n_tris < 0 || m->n_tris >= ((int64_t)1 << 31) || m->n_vertices < 0 || m->n_vertices >= ((int64_t)1 << 31))
        return fail(ctx, RM_ERR_INVALID_ARG, "mesh sizes out of range (V=%lld, T=%lld)",
                    (long long)m->n_vertices, (long long)m->n_tris);
    if (m->n_tris > 0 && (!m->xyz || !m->tri || !m->cls || m->n_vertices < 1))
        return fail(ctx, RM_ERR_INVALID_ARG, "mesh arrays must be non-NULL and n_vertices >= 1 when n_tris > 0");
    return RM_OK;
}

bool valid_tile(int w, int h) {
    return (w == 8 && h == 8) || (w == 16 && h == 16) || (w == 32 && h == 32) || (w == 64 && h == 32);
}

// Autotune candidates, largest first: each step down quadruples or doubles
// the per-pose tile records and bins, so the search stops at the first shape
// that is clearly slower than the best so far.
constexpr int kNumTiles = 4;
const int kTiles[kNumTiles][2] = {{64, 32}, {32, 32}, {16, 16}, {8, 8}};

// Fills the scan descriptors and counts items and partial records.
void plan(BatchDesc& bd, int tw, int th) {
    bd.tile_w = tw;
    bd.tile_h = th;
    int64_t items = 0, recs = 0;
    for (int s = 0; s < bd.n_scans; ++s) {
        ScanDesc& d = bd.s[s];
        d.tiles_x = (d.width + tw - 1) / tw;
        d.tiles_y = (d.height + th - 1) / th;
        d.item_off = items;
        d.rec_off = recs;
        const int64_t n = (int64_t)d.n_poses * d.tiles_x * d.tiles_y;
        items += n;
        recs += n;
    }
    bd.n_items = items;
}

int64_t total_records(const BatchDesc& bd) {
    int64_t r = 0;
    for (int s = 0; s < bd.n_scans; ++s) r += (int64_t)bd.s[s].n_poses * bd.s[s].tiles_x * bd.s[s].tiles_y;
    return r;
}

// Whether a batch can run with tile tw x th: at most kMaxTileGrid tiles per
// image row and column (tile rectangles are packed in 8-bit fields) and fewer
// than 2^31 (pose, tile) records in the call.  Empty on success, otherwise
// the reason.
std::string tile_limit(const BatchDesc& bd0, int tw, int th) {
    BatchDesc bd = bd0;
    plan(bd, tw, th);
    char buf[160];
    for (int s = 0; s < bd.n_scans; ++s)
        if (bd.s[s].tiles_x > kMaxTileGrid || bd.s[s].tiles_y > kMaxTileGrid) {
            snprintf(buf, sizeof(buf), "%dx%d image needs more than %d tiles of %dx%d per row or column",
                     bd.s[s].width, bd.s[s].height, kMaxTileGrid, tw, th);
            return buf;
        }
    if (total_records(bd) >= ((int64_t)1 << 31)) {
        snprintf(buf, sizeof(buf), "%lld (pose, tile) records of %dx%d tiles exceed 2^31 - 1",
                 (long long)total_records(bd), tw, th);
        return buf;
    }
    return std::string();
}

constexpr int64_t kMinBinCap = 64;                     // the budget never shrinks a bin below this

// Pinned readback slots: [1] and [4] largest small and large bin of the last
// call, [2..3] largest small and large fills of a sizing pass; int64 pairs:
// [6..7] and [12..13] list and region entries the last call asked for,
// [8..9], [10..11] and [14..15] list entries, records and region entries of a
// sizing pass.
int64_t pinned64(const rm_ctx* ctx, int i) {
    int64_t v;
    memcpy(&v, ctx->pinned + i, sizeof(v));
    return v;
}

// Overflow entries to learn from a demand of `need`: a quarter more, for the
// poses of later calls.
int64_t pool_margin(int64_t need) { return need > 0 ? need + need / 4 + 4096 : 0; }

// Slots for large footprints to learn from a largest large fill of `fb`.
int64_t big_margin(int64_t fb) { return (fb + fb / 4 + 63) & ~(int64_t)63; }

// Learns bin capacity and large part from the largest small and large fills
// seen (fs, fb), as far as the bins of n_records fit the budget; true if
// either grew.
bool learn_bins(rm_ctx* ctx, int64_t n_records, int64_t fs, int64_t fb) {
    const int64_t want_b = std::min<int64_t>(big_margin(fb), (int64_t)1 << 23);
    const int64_t want_s = std::min<int64_t>(fs + fs / 4, (int64_t)1 << 24);
    int64_t cap = ctx->bin_cap;
    while (cap < want_s + want_b && cap < ((int64_t)1 << 24)) cap *= 2;
    while (cap > 1024 && n_records * cap * 4 > ctx->bin_budget) cap /= 2;
    const bool grew = cap > ctx->bin_cap || want_b > ctx->big_cap || want_s > ctx->small_want;
    ctx->bin_cap = (int32_t)std::max<int64_t>(cap, ctx->bin_cap);
    ctx->big_cap = (int32_t)std::max<int64_t>(want_b, ctx->big_cap);
    ctx->small_want = (int32_t)std::max<int64_t>(want_s, ctx->small_want);
    return grew;
}

// The part of a capacity of cap for large footprints: what was learned when
// both parts fit, else at most an eighth (small footprints are the bulk of
// the entries), and never more than half.
int64_t big_part(const rm_ctx* ctx, int64_t cap) {
    const int64_t b = std::min<int64_t>(ctx->big_cap, cap / 2);
    return (int64_t)ctx->small_want + ctx->big_cap <= cap ? b : std::min<int64_t>(b, cap / 8);
}

// The capacity a call of n_records gets: the fixed one, or the learned one
// halved until its bins fit the budget.
int64_t call_cap(const rm_ctx* ctx, int64_t n_records) {
    if (ctx->bin_cap_fixed > 0) return ctx->bin_cap_fixed;
    int64_t cap = ctx->bin_cap;
    while (cap > kMinBinCap && n_records * cap * 4 > ctx->bin_budget) cap /= 2;
    return cap;
}

// Grows the bins when the largest bins of an earlier call (read back
// asynchronously) did not fit their parts, and the overflow when what the
// call spilled did not; never while capturing.
void adapt_bin_cap(rm_ctx* ctx, int64_t n_records) {
    if (!ctx->bin_pending || capturing(ctx)) return;
    if (hipEventQuery(ctx->bin_ev) != hipSuccess) { (void)hipGetLastError(); return; }
    ctx->bin_pending = false;
    const int32_t fs = ctx->pinned[1], fb = ctx->pinned[4];
    if (ctx->pool_pending) {
        ctx->pool_pending = false;
        ctx->list_want = std::max(ctx->list_want, pool_margin(pinned64(ctx, 6)));
        ctx->region_want = std::max(ctx->region_want, pool_margin(pinned64(ctx, 12)));
    }
    if (ctx->bin_cap_fixed == 0) learn_bins(ctx, n_records, fs, fb);
    if (fs <= ctx->last_cap_s && fb <= ctx->last_cap_b) return;
    // bins that would still overflow at the capacity of their shape's next call spill from then on
    const int64_t cap = call_cap(ctx, std::get<0>(ctx->pending_shape)), cap_b = big_part(ctx, cap);
    if ((fs > cap - cap_b || fb > cap_b) && ctx->pool_mode < 0) ctx->track_shapes.insert(ctx->pending_shape);
}

// Starts the timing of one launch of kernel k (0 rasterizer, 1 binning) when
// profiling (not under capture or for the allocation-free call); *stop
// receives the event to record after it, or null.
int prof_begin(rm_ctx* ctx, int k, bool fixed, hipEvent_t* stop) {
    *stop = nullptr;
    if (!ctx->profiling || capturing(ctx) || fixed) return RM_OK;
    if (ctx->prof_used[k] == ctx->prof_events[k].size()) {
        hipEvent_t x, y;
        RM_HIP(ctx, hipEventCreate(&x));
        RM_HIP(ctx, hipEventCreate(&y));
        ctx->prof_events[k].emplace_back(x, y);
    }
    RM_HIP(ctx, hipEventRecord(ctx->prof_events[k][ctx->prof_used[k]].first, ctx->stream));
    *stop = ctx->prof_events[k][ctx->prof_used[k]].second;
    ++ctx->prof_used[k];
    return RM_OK;
}

// Overflow room of a call with n_records bins of capacity cap: the fixed
// size, or for a shape that tracks overflow what was learned, scaled down
// to what the budget leaves beside the bins (list entries 12 bytes, region
// entries 4), the list in whole segments below 2^32 - 1 entries.
void overflow_caps(const rm_ctx* ctx, int64_t n_records, int64_t cap, bool fixed_arena, bool track,
                   int64_t* spill_cap, int64_t* pool_cap) {
    int64_t sc = 0, pc = 0;
    if (!fixed_arena && ctx->pool_mode > 0) {
        sc = pc = ctx->pool_mode;
    } else if (!fixed_arena && ctx->pool_mode < 0 && track) {
        const double room = (double)std::max<int64_t>(0, ctx->bin_budget - n_records * cap * 4);
        const double want = 12.0 * (double)ctx->list_want + 4.0 * (double)ctx->region_want;
        const double f = want > room ? room / want : 1.0;
        sc = (int64_t)((double)ctx->list_want * f);
        pc = (int64_t)((double)ctx->region_want * f);
    }
    *spill_cap = std::min<int64_t>(sc, 0xfffffffell) / kSpillLists * kSpillLists;
    *pool_cap = pc;
}

// One scoring pass: cull, near-to-far cluster order, bin, rasterize (+ fused
// comparison), reduce.
int run_pass(rm_ctx* ctx, const rm_mesh* mesh, BatchDesc& bd, int tw, int th, int mode, const double* T_wc,
             float eps, double* out, float* depth_out, int32_t* tri_out, uint8_t* cls_out, const float* vnrm,
             const Arena& arena) {
    {
        const std::string why = tile_limit(bd, tw, th);
        if (!why.empty()) return fail(ctx, RM_ERR_UNSUPPORTED, "%s", why.c_str());
    }
    plan(bd, tw, th);
    const int P = bd.n_poses;
    const int64_t C = (mesh->n_tris + kClusterTris - 1) / kClusterTris;
    const int64_t R = total_records(bd);
    const bool fixed_cap = ctx->bin_cap_fixed > 0;
    adapt_bin_cap(ctx, R);
    // The first uncaptured call of a launch shape reads the largest bin fills
    // back right after binning and, if the bins were too small, grows them
    // (or, where the budget stops that, sizes the overflow) and bins again,
    // so that no call of that shape takes the slow every-cluster path of an
    // overflowing bin; later calls adapt asynchronously.  A fixed capacity
    // (rm_set_bin_cap) is never grown, a fixed overflow never resized, and
    // the allocation-free call has neither growth nor overflow.
    const auto shape = std::make_tuple(R, tw, th, mesh->n_tris, P);
    const bool pool_adaptive = ctx->pool_mode < 0 && !arena.fixed;
    const bool log = getenv("RM_LOG") != nullptr;  // the sizing pass then also reports fixed settings
    const bool check = !arena.fixed && !capturing(ctx) && ctx->bin_checked.count(shape) == 0 &&
                       (!fixed_cap || pool_adaptive || log);
    const bool persistent = ctx->schedule != 1;
    RasterArgs a;
    int32_t* vis_count = nullptr;
    int32_t* vis_tris = nullptr;
    int32_t* bin_max = nullptr;
    int64_t cap = 0, cap_b = 0;
    for (int attempt = 0;; ++attempt) {
        // the capacity learned so far (or fixed), limited to what this call's records may take
        cap = call_cap(ctx, R);
        // overflow: spill-list entries (12 bytes) and region entries (4
        // bytes), as learned, scaled down to what the budget leaves beside the bins
        const bool shape_track = pool_adaptive && ctx->track_shapes.count(shape) > 0;
        int64_t spill_cap = 0, pool_cap = 0;
        overflow_caps(ctx, R, cap, arena.fixed != nullptr, shape_track, &spill_cap, &pool_cap);
        // the spilling kernel also measures what overflow must hold: always in a sizing pass
        const bool track = !arena.fixed && (check || ctx->pool_mode > 0 || shape_track);
        Carve cv;
        // vis_count, vis_tris, bin_max[2], bin_fill[2], bin fills, order histogram and cursors, queue
        const int64_t n_cnt = 2 * (int64_t)P + 4 + 2 * R + 65;
        const size_t o_cnt = cv.take<int32_t>(n_cnt);
        const size_t o_ord = cv.take<int32_t>(persistent ? R : 1);
        const size_t o_vis = cv.take<uint2>((int64_t)P * C);
        const size_t o_visz = cv.take<float>((int64_t)P * C);
        const size_t o_rec = cv.take<float>(mode == kRender ? 1 : R * kRecFields);
        const size_t o_cb = cv.take<char>(mesh->clusters ? 1 : rm_mesh_clusters_size(mesh->n_tris));
        // spill counters (u64) and lost flags [R], zeroed; region offsets; spilled
        // records; spill list; regions
        const int64_t n_cnt64 = kSpillTops + 2 * kSpillLists;
        const int64_t n_sz = track ? 2 * n_cnt64 + R : 0;
        const size_t o_sz = track ? cv.take<int32_t>(n_sz) : 0;
        const size_t o_poff = track ? cv.take<int64_t>(R) : 0;
        const size_t o_srec = track ? cv.take<int32_t>(R) : 0;
        const size_t o_spill = spill_cap > 0 ? cv.take<uint3>(spill_cap) : 0;
        const size_t o_pool = pool_cap > 0 ? cv.take<uint32_t>(pool_cap) : 0;
        const size_t o_bin = cv.off;
        char* base = nullptr;
        if (arena.fixed) {
            // bins take what the fixed buffer leaves; a bin that overflows a
            // smaller capacity is rasterized from every visible cluster (same result)
            if (o_bin + 256 > arena.fixed_size)
                return fail(ctx, RM_ERR_CAPACITY, "the call needs %zu bytes of scratch besides its bins; the "
                                                  "allocation-free buffer holds %zu", o_bin + 256, arena.fixed_size);
            cap = std::min<int64_t>(cap, (int64_t)((arena.fixed_size - o_bin) / 4) / std::max<int64_t>(R, 1));
            cv.take<uint32_t>(R * cap);
            base = arena.fixed;
        } else {
            cv.take<uint32_t>(R * cap);
            int rc = ensure_scratch(ctx, cv.off);
            if (rc) return rc;
            base = static_cast<char*>(ctx->scratch);
        }
        cap_b = big_part(ctx, cap);
        auto at = [&](size_t off) { return base + off; };
        vis_count = reinterpret_cast<int32_t*>(at(o_cnt));
        vis_tris = vis_count + P;
        bin_max = vis_tris + P;
        int32_t* bin_fill = bin_max + 2;
        int32_t* bin_small = bin_fill + 2;
        int32_t* bin_big = bin_small + R;
        int32_t* hist = bin_big + R;
        const void* prep = mesh->clusters;
        if (!prep && C > 0) {
            void* w = at(o_cb);
            RM_HIP(ctx, launch_prepare(ctx->stream, mesh->xyz, mesh->n_vertices, mesh->tri, mesh->n_tris, w));
            prep = w;
        }
        const ClusterBounds* cb = static_cast<const ClusterBounds*>(prep);
        const float* nrm = prep ? reinterpret_cast<const float*>(static_cast<const char*>(prep) +
                                                                 prepared_normals_offset(mesh->n_tris))
                                : nullptr;
        RM_HIP(ctx, launch_zero_i32(ctx->stream, vis_count, n_cnt));
        if (track) RM_HIP(ctx, launch_zero_i32(ctx->stream, reinterpret_cast<int32_t*>(at(o_sz)), n_sz));
        uint2* vis = reinterpret_cast<uint2*>(at(o_vis));
        float* vis_z = reinterpret_cast<float*>(at(o_visz));
        RM_HIP(ctx, launch_cull(ctx->stream, bd, cb, (int32_t)C, T_wc, vis, vis_z, vis_count, vis_tris));
        RM_HIP(ctx, launch_vis_sort(ctx->stream, bd, (int32_t)C, vis_count, vis_z, vis));
        a.xyz = mesh->xyz;
        a.tri = mesh->tri;
        a.cls = mesh->cls;
        a.nrm = nrm;
        a.n_tris = mesh->n_tris;
        a.vmax = mesh->n_vertices > 0 ? (uint32_t)(mesh->n_vertices - 1) : 0u;
        a.n_clusters = (int32_t)C;
        a.T_wc = T_wc;
        a.vis = vis;
        a.vis_count = vis_count;
        a.bins = reinterpret_cast<uint32_t*>(at(o_bin));
        a.bin_small = bin_small;
        a.bin_big = bin_big;
        a.bin_max = bin_max;
        a.bin_fill = check ? bin_fill : nullptr;
        a.bin_cap = (int32_t)cap;
        a.bin_big_cap = (int32_t)cap_b;
        a.spill_top = track ? reinterpret_cast<unsigned long long*>(at(o_sz)) : nullptr;
        a.spill_lost = track ? reinterpret_cast<int32_t*>(at(o_sz)) + 2 * n_cnt64 : nullptr;
        a.spill_recs = track ? reinterpret_cast<int32_t*>(at(o_srec)) : nullptr;
        a.pool_off = track ? reinterpret_cast<int64_t*>(at(o_poff)) : nullptr;
        // (a list without regions would place nothing: keep neither)
        a.spill = spill_cap > 0 && pool_cap > 0 ? reinterpret_cast<uint3*>(at(o_spill)) : nullptr;
        a.pool = spill_cap > 0 && pool_cap > 0 ? reinterpret_cast<uint32_t*>(at(o_pool)) : nullptr;
        a.spill_cap = a.spill ? spill_cap : 0;
        a.pool_cap = a.pool ? pool_cap : 0;
        a.order = nullptr;
        a.queue = hist + 64;
        a.n_order = (int32_t)R;
        a.rec = reinterpret_cast<float*>(at(o_rec));
        a.eps = eps;
        a.vnrm = vnrm;
        a.tri_color = mode == kCost || mode == kGrad ? mesh->color : nullptr;
        a.color_tol = bd.color_tol;
        a.depth_out = depth_out;
        a.tri_out = tri_out;
        a.cls_out = cls_out;
        hipEvent_t be1;
        int prc = prof_begin(ctx, 1, arena.fixed != nullptr, &be1);
        if (prc) return prc;
        RM_HIP(ctx, launch_bin(ctx->stream, bd, a));
        if (track) RM_HIP(ctx, launch_overflow(ctx->stream, a, R));
        if (be1) RM_HIP(ctx, hipEventRecord(be1, ctx->stream));
        if (persistent) {
            int32_t* order = reinterpret_cast<int32_t*>(at(o_ord));
            RM_HIP(ctx, launch_order(ctx->stream, bd, bin_small, bin_big, R, hist, order));
            a.order = order;
        }
        if (!check) break;
        RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 2, bin_fill, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 8, a.spill_top, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 10, a.spill_top + 2, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 14, a.spill_top + 4, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        RM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        ctx->bin_checked.insert(shape);
        const int64_t fs = ctx->pinned[2], fb = ctx->pinned[3];
        const int64_t spilled = pinned64(ctx, 8), spill_recs = pinned64(ctx, 10), filled = pinned64(ctx, 14);
        if (log)
            fprintf(stderr,
                    "[rendermap] plan: %d scans, %d poses, %lld triangles (%lld clusters), tile %dx%d, %lld tile "
                    "records, %s schedule, bin capacity %lld (%lld for large footprints; largest fills %lld "
                    "small, %lld large), overflow list %lld and regions %lld entries (%lld bins spill; they need "
                    "%lld list and %lld region entries), %zu bytes of scratch\n",
                    bd.n_scans, P, (long long)mesh->n_tris, (long long)C, tw, th, (long long)R,
                    persistent ? "persistent longest-first" : "one workgroup per item", (long long)cap,
                    (long long)cap_b, (long long)fs, (long long)fb, (long long)a.spill_cap, (long long)a.pool_cap,
                    (long long)spill_recs, (long long)spilled, (long long)filled, cv.off);
        if ((fs <= cap - cap_b && fb <= cap_b) || attempt >= 2) break;
        if (!fixed_cap && learn_bins(ctx, R, fs, fb)) {
            const int64_t c2 = call_cap(ctx, R), b2 = big_part(ctx, c2);
            if (c2 > cap || b2 != cap_b) {
                if (log)
                    fprintf(stderr, "[rendermap] bins grown to %lld entries (%lld large); binning again\n",
                            (long long)c2, (long long)b2);
                if (pool_adaptive && (fs > c2 - b2 || fb > b2)) ctx->track_shapes.insert(shape);
                continue;
            }
        }
        // the bins cannot grow: what outgrows them spills
        if (pool_adaptive) ctx->track_shapes.insert(shape);
        const bool placed = spilled <= a.spill_cap && filled <= a.pool_cap;
        if (placed || !pool_adaptive) {
            if (!placed && log)
                fprintf(stderr, "[rendermap] bins whose overflow does not fit take the every-cluster path\n");
            break;
        }
        ctx->list_want = std::max(ctx->list_want, pool_margin(spilled));
        ctx->region_want = std::max(ctx->region_want, pool_margin(filled));
        int64_t next_spill = 0, next_pool = 0;
        overflow_caps(ctx, R, cap, false, true, &next_spill, &next_pool);
        if (next_spill <= a.spill_cap && next_pool <= a.pool_cap) {
            if (log) fprintf(stderr, "[rendermap] the budget leaves the overflow no more room\n");
            break;
        }
        if (log)
            fprintf(stderr, "[rendermap] overflow sized to %lld list and %lld region entries; binning again\n",
                    (long long)next_spill, (long long)next_pool);
    }
    hipEvent_t pe1;
    {
        int prc = prof_begin(ctx, 0, arena.fixed != nullptr, &pe1);
        if (prc) return prc;
    }
    RM_HIP(ctx, launch_raster(ctx->stream, bd, a, mode));
    if (pe1) RM_HIP(ctx, hipEventRecord(pe1, ctx->stream));
    if (mode != kRender)
        RM_HIP(ctx, launch_reduce(ctx->stream, bd, a.rec, vis_tris, eps, mode, out));
    if (!capturing(ctx) && !ctx->bin_pending && !arena.fixed) {
        if (!ctx->bin_ev) RM_HIP(ctx, hipEventCreateWithFlags(&ctx->bin_ev, hipEventDisableTiming));
        RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 1, bin_max, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
        RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 4, bin_max + 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        if (a.spill_top) {
            RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 6, a.spill_top, sizeof(int64_t), hipMemcpyDeviceToHost,
                                       ctx->stream));
            RM_HIP(ctx, hipMemcpyAsync(ctx->pinned + 12, a.spill_top + 4, sizeof(int64_t), hipMemcpyDeviceToHost,
                                       ctx->stream));
        }
        RM_HIP(ctx, hipEventRecord(ctx->bin_ev, ctx->stream));
        ctx->bin_pending = true;
        ctx->pool_pending = a.spill_top != nullptr;
        ctx->last_cap_s = (int32_t)(cap - cap_b);
        ctx->last_cap_b = (int32_t)cap_b;
        ctx->pending_shape = shape;
    }
    return RM_OK;
}

// Tuning key of a launch shape: mode, triangle count, and every scan's image
// size and pose count.
std::vector<int64_t> tune_key(const BatchDesc& bd, int64_t n_tris, int mode) {
    std::vector<int64_t> k = {mode, n_tris, bd.n_scans};
    for (int s = 0; s < bd.n_scans; ++s) {
        k.push_back(bd.s[s].width);
        k.push_back(bd.s[s].height);
        k.push_back(bd.s[s].n_poses);
    }
    return k;
}

// Chooses the tile shape (explicit, cached autotune result, or default) and runs.
int run_scored(rm_ctx* ctx, const rm_mesh* mesh, BatchDesc& bd, int mode, const double* T_wc, float eps,
               double* out, float* depth_out, int32_t* tri_out, uint8_t* cls_out, const float* vnrm,
               const Arena& arena) {
    if (ctx->tile_w) return run_pass(ctx, mesh, bd, ctx->tile_w, ctx->tile_h, mode, T_wc, eps, out, depth_out,
                                     tri_out, cls_out, vnrm, arena);
    if (arena.fixed)
        return run_pass(ctx, mesh, bd, 64, 32, mode, T_wc, eps, out, depth_out, tri_out, cls_out, vnrm, arena);
    const std::vector<int64_t> key = tune_key(bd, mesh->n_tris, mode);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end())
        return run_pass(ctx, mesh, bd, it->second.first, it->second.second, mode, T_wc, eps, out, depth_out,
                        tri_out, cls_out, vnrm, arena);
    if (!ctx->autotune || capturing(ctx))
        return run_pass(ctx, mesh, bd, 64, 32, mode, T_wc, eps, out, depth_out, tri_out, cls_out, vnrm, arena);
    if (!ctx->ev0) {
        RM_HIP(ctx, hipEventCreate(&ctx->ev0));
        RM_HIP(ctx, hipEventCreate(&ctx->ev1));
    }
    float best = 1e30f;
    int bi = -1;
    for (int k = 0; k < kNumTiles; ++k) {
        if (!tile_limit(bd, kTiles[k][0], kTiles[k][1]).empty()) continue;   // not possible for this batch
        // one warm-up and one timed pass per shape; the warm-up's largest bin
        // is read back first so that the timed pass runs with bins that fit
        for (int rep = 0; rep < 2; ++rep) {
            if (rep == 1) {
                if (ctx->bin_pending) RM_HIP(ctx, hipEventSynchronize(ctx->bin_ev));
                RM_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
            }
            int rc = run_pass(ctx, mesh, bd, kTiles[k][0], kTiles[k][1], mode, T_wc, eps, out, depth_out, tri_out,
                              cls_out, vnrm, arena);
            if (rc) return rc;
        }
        RM_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
        RM_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0.0f;
        RM_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        if (ms < best) { best = ms; bi = k; }
        else if (ms > 1.25f * best) break;
    }
    if (bi < 0) {
        const std::string why = tile_limit(bd, kTiles[kNumTiles - 1][0], kTiles[kNumTiles - 1][1]);
        return fail(ctx, RM_ERR_UNSUPPORTED, "no tile shape fits this batch: %s", why.c_str());
    }
    ctx->tuned[key] = {kTiles[bi][0], kTiles[bi][1]};
    if (getenv("RM_LOG"))
        fprintf(stderr, "[rendermap] autotune: %d scans, %d poses, %lld triangles: tile %dx%d (%.3f ms)\n",
                bd.n_scans, bd.n_poses, (long long)mesh->n_tris, kTiles[bi][0], kTiles[bi][1], best);
    return run_pass(ctx, mesh, bd, kTiles[bi][0], kTiles[bi][1], mode, T_wc, eps, out, depth_out, tri_out, cls_out,
                    vnrm, arena);
}

int fill_scan(rm_ctx* ctx, ScanDesc& d, const rm_camera& c) {
    int rc = check_camera(ctx, c);
    if (rc) return rc;
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    d.width = c.width; d.height = c.height;
    d.z_near = c.z_near; d.z_far = c.z_far;
    return RM_OK;
}

}  // namespace

int rm::align_common(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t S, const int32_t* pose_off,
                     const double* T_wc, rm_cost_params params, double* out, int mode, const float* vnrm,
                     const Arena* arena) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    int rc = check_mesh(ctx, mesh);
    if (rc) return rc;
    if (!scans || !pose_off) return fail(ctx, RM_ERR_INVALID_ARG, "scans and pose_off must be non-NULL");
    if (S < 1 || S > RM_MAX_SCANS) return fail(ctx, RM_ERR_INVALID_ARG, "n_scans %d outside 1..%d", S, RM_MAX_SCANS);
    if (!(params.eps > 0.0f) || !std::isfinite(params.eps))
        return fail(ctx, RM_ERR_INVALID_ARG, "eps must be positive and finite");
    if (params.flags != 0) return fail(ctx, RM_ERR_INVALID_ARG, "flags must be 0");
    if (!(params.color_tol >= 0.0f) || !std::isfinite(params.color_tol))
        return fail(ctx, RM_ERR_INVALID_ARG, "color_tol must be finite and >= 0");
    if (pose_off[0] != 0) return fail(ctx, RM_ERR_INVALID_ARG, "pose_off[0] must be 0");
    BatchDesc bd;
    std::memset(&bd, 0, sizeof(bd));
    bd.n_scans = S;
    bd.color_tol = params.color_tol;
    for (int s = 0; s < S; ++s) {
        if (pose_off[s + 1] < pose_off[s]) return fail(ctx, RM_ERR_INVALID_ARG, "pose_off must be non-decreasing");
        if (!scans[s].depth || !scans[s].cls)
            return fail(ctx, RM_ERR_INVALID_ARG, "scan %d has NULL depth or cls", s);
        rc = fill_scan(ctx, bd.s[s], scans[s].cam);
        if (rc) return rc;
        bd.s[s].depth = scans[s].depth;
        bd.s[s].cls = scans[s].cls;
        bd.s[s].mask = scans[s].mask;
        bd.s[s].color = scans[s].color;
        bd.s[s].pose_off = pose_off[s];
        bd.s[s].n_poses = pose_off[s + 1] - pose_off[s];
    }
    const int P = pose_off[S];
    if (P > 65535) return fail(ctx, RM_ERR_INVALID_ARG, "at most 65535 poses per call (got %d)", P);
    if (P == 0) return RM_OK;
    if (!T_wc || !out) return fail(ctx, RM_ERR_INVALID_ARG, "T_wc and out must be non-NULL");
    bd.n_poses = P;
    DeviceGuard g(ctx->device);
    const Arena none;
    return run_scored(ctx, mesh, bd, mode, T_wc, params.eps, out, nullptr, nullptr, nullptr, vnrm,
                      arena ? *arena : none);
}

int rm::ctx_fail(rm_ctx* ctx, int code, const char* msg) { return fail(ctx, code, "%s", msg); }

int rm::ctx_device(const rm_ctx* ctx) { return ctx->device; }

namespace {

}  // namespace

extern "C" {

int rm_ctx_create(int32_t device, rm_ctx** out) {
    if (!out) return fail(nullptr, RM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return fail(nullptr, RM_ERR_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n) return fail(nullptr, RM_ERR_INVALID_ARG, "device %d outside 0..%d", device, n - 1);
    rm_ctx* c = new rm_ctx();
    c->device = device;
    DeviceGuard g(device);
    noalloc_setup(device);
    size_t mem_free = 0, mem_total = 0;
    if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess)
        c->bin_budget = std::max<int64_t>((int64_t)4 << 30, (int64_t)(mem_total / 4));
    else
        (void)hipGetLastError();
    if (hipHostMalloc((void**)&c->pinned, 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(nullptr, RM_ERR_DEVICE, "hipHostMalloc failed");
    }
    *out = c;
    return RM_OK;
}

int rm_ctx_destroy(rm_ctx* ctx) {
    if (!ctx) return RM_OK;
    {
        DeviceGuard g(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream); else (void)hipDeviceSynchronize();
        if (ctx->scratch) (void)hipFree(ctx->scratch);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
        if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
        for (auto& e : ctx->prof_events[0]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        for (auto& e : ctx->prof_events[1]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        if (ctx->bin_ev) (void)hipEventDestroy(ctx->bin_ev);
        for (void* r : ctx->retired) (void)hipFree(r);
    }
    delete ctx;
    return RM_OK;
}

int rm_ctx_set_stream(rm_ctx* ctx, void* stream) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(stream);
    return RM_OK;
}

const char* rm_last_error(const rm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int rm_set_tile(rm_ctx* ctx, int32_t tile_w, int32_t tile_h) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    if (tile_w == 0 && tile_h == 0) { ctx->tile_w = ctx->tile_h = 0; return RM_OK; }
    if (!valid_tile(tile_w, tile_h)) return fail(ctx, RM_ERR_INVALID_ARG, "tile %dx%d not supported", tile_w, tile_h);
    ctx->tile_w = tile_w;
    ctx->tile_h = tile_h;
    return RM_OK;
}

int rm_set_schedule(rm_ctx* ctx, int32_t mode) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (mode < 0 || mode > 2) return fail(ctx, RM_ERR_INVALID_ARG, "schedule %d outside 0..2", mode);
    ctx->schedule = mode;
    return RM_OK;
}

int rm_autotune(rm_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->autotune = enable != 0;
    return RM_OK;
}

int rm_set_bin_cap(rm_ctx* ctx, int32_t cap) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (cap < 0 || cap > (1 << 24)) return fail(ctx, RM_ERR_INVALID_ARG, "bin capacity %d outside 0..2^24", cap);
    ctx->bin_cap_fixed = cap;
    ctx->bin_checked.clear();         // the next call of each shape sizes its bins again
    ctx->track_shapes.clear();
    return RM_OK;
}

int rm_set_bin_pool(rm_ctx* ctx, int64_t entries) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (entries < -1 || entries > ((int64_t)1 << 40))
        return fail(ctx, RM_ERR_INVALID_ARG, "overflow pool of %lld entries outside -1..2^40", (long long)entries);
    ctx->pool_mode = entries;
    ctx->bin_checked.clear();
    ctx->track_shapes.clear();
    return RM_OK;
}

int rm_get_tile(rm_ctx* ctx, int32_t width, int32_t height, int32_t n_poses, int64_t n_tris, int32_t* tile_w,
                int32_t* tile_h) {
    if (!ctx || !tile_w || !tile_h) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    if (ctx->tile_w) { *tile_w = ctx->tile_w; *tile_h = ctx->tile_h; return RM_OK; }
    for (int mode = kCost; mode <= kIcp; ++mode) {
        const std::vector<int64_t> key = {mode, n_tris, 1, width, height, n_poses};
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) { *tile_w = it->second.first; *tile_h = it->second.second; return RM_OK; }
    }
    *tile_w = 64;
    *tile_h = 32;
    return RM_OK;
}

int rm_profile(rm_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->profiling = enable != 0;
    return RM_OK;
}

namespace {
int profile_read(rm_ctx* ctx, int k, int64_t* n_launches, double* total_ms) {
    if (!ctx || !n_launches || !total_ms) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    for (size_t i = 0; i < ctx->prof_used[k]; ++i) {
        float ms = 0.0f;
        RM_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_events[k][i].first, ctx->prof_events[k][i].second));
        tot += ms;
    }
    *n_launches = (int64_t)ctx->prof_used[k];
    *total_ms = tot;
    ctx->prof_used[k] = 0;
    return RM_OK;
}
}  // namespace

int rm_profile_read(rm_ctx* ctx, int64_t* n_launches, double* total_ms) {
    return profile_read(ctx, 0, n_launches, total_ms);
}

int rm_profile_read_binning(rm_ctx* ctx, int64_t* n_launches, double* total_ms) {
    return profile_read(ctx, 1, n_launches, total_ms);
}

int rm_graph_begin(rm_ctx* ctx) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    if (!ctx->stream) return fail(ctx, RM_ERR_INVALID_ARG, "capture needs a non-null stream");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    return RM_OK;
}

int rm_graph_end(rm_ctx* ctx, void** graph_exec) {
    if (!ctx || !graph_exec) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard g(ctx->device);
    hipGraph_t graph = nullptr;
    RM_HIP(ctx, hipStreamEndCapture(ctx->stream, &graph));
    hipGraphExec_t ex = nullptr;
    ctx->captured = true;
    hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(ctx, RM_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    *graph_exec = ex;
    return RM_OK;
}

int rm_graph_launch(rm_ctx* ctx, void* graph_exec) {
    if (!ctx || !graph_exec) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), ctx->stream));
    return RM_OK;
}

int rm_graph_destroy(void* graph_exec) {
    if (graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec));
    return RM_OK;
}

int rm_scan_image(rm_ctx* ctx, const float* depth, int32_t height, int32_t width, float z_min, float z_max,
                  float* d_out, uint8_t* c_out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (!depth || !d_out || !c_out) return fail(ctx, RM_ERR_INVALID_ARG, "NULL image pointer");
    if (height < 1 || width < 1 || (int64_t)height * width > ((int64_t)1 << 26))
        return fail(ctx, RM_ERR_INVALID_ARG, "bad image size %dx%d", width, height);
    if (!(z_min >= 0.0f && z_max > z_min && std::isfinite(z_max)))
        return fail(ctx, RM_ERR_INVALID_ARG, "need 0 <= z_min < z_max < inf");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_scan_image(ctx->stream, depth, height, width, z_min, z_max, d_out, c_out));
    return RM_OK;
}

int rm_mesh_from_range(rm_ctx* ctx, const float* depth, rm_camera cam, const double* T_wc, int32_t stride,
                       int32_t smooth_radius, float z_min, float z_max, float max_edge, float* xyz_out, int32_t* tri_out,
                       uint8_t* cls_out, int64_t cap_t, int64_t* n_v_out, int64_t* n_t_out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    int rc = check_camera(ctx, cam);
    if (rc) return rc;
    if (!depth || !T_wc || !xyz_out || !tri_out || !cls_out || !n_v_out || !n_t_out)
        return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    if (stride < 1 || stride > 256) return fail(ctx, RM_ERR_INVALID_ARG, "stride %d outside 1..256", stride);
    if (smooth_radius < 0 || smooth_radius > RM_MAX_SMOOTH_RADIUS)
        return fail(ctx, RM_ERR_INVALID_ARG, "smooth_radius %d outside 0..%d", smooth_radius, RM_MAX_SMOOTH_RADIUS);
    if (!(z_min >= 0.0f && z_max > z_min && std::isfinite(z_max)))
        return fail(ctx, RM_ERR_INVALID_ARG, "need 0 <= z_min < z_max < inf");
    if (!(max_edge > 0.0f)) return fail(ctx, RM_ERR_INVALID_ARG, "max_edge must be positive");
    if (cap_t < 0) return fail(ctx, RM_ERR_INVALID_ARG, "cap_t must be >= 0");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(T_wc[k])) return fail(ctx, RM_ERR_INVALID_ARG, "pose has a non-finite entry");
    if (capturing(ctx)) return fail(ctx, RM_ERR_UNSUPPORTED, "rm_mesh_from_range synchronizes; not capturable");
    DeviceGuard g(ctx->device);
    const int32_t gh = (cam.height + stride - 1) / stride, gw = (cam.width + stride - 1) / stride;
    const int64_t nn = (int64_t)gh * gw;
    const int64_t nb = meshify_blocks(cam.height, cam.width, stride);
    Carve cv;
    const size_t o_kind = cv.take<uint8_t>(nn);
    const size_t o_cnt = cv.take<int32_t>(nb);
    const size_t o_off = cv.take<int32_t>(nb);
    const size_t o_tot = cv.take<int32_t>(1);
    rc = ensure_scratch(ctx, cv.off);
    if (rc) return rc;
    RM_HIP(ctx, launch_meshify(ctx->stream, depth, cam, T_wc, stride, smooth_radius, z_min, z_max, max_edge, xyz_out, tri_out,
                               cls_out, cap_t, at<uint8_t>(ctx, o_kind), at<int32_t>(ctx, o_cnt),
                               at<int32_t>(ctx, o_off), at<int32_t>(ctx, o_tot)));
    RM_HIP(ctx, hipMemcpyAsync(ctx->pinned, at<int32_t>(ctx, o_tot), sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    RM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *n_v_out = nn;
    *n_t_out = ctx->pinned[0];
    if (ctx->pinned[0] > cap_t)
        return fail(ctx, RM_ERR_CAPACITY, "mesh has %d triangles, capacity %lld", ctx->pinned[0], (long long)cap_t);
    return RM_OK;
}

int64_t rm_mesh_clusters_size(int64_t n_tris) {
    if (n_tris <= 0) return 0;
    return prepared_normals_offset(n_tris) + n_tris * 3 * (int64_t)sizeof(float);
}

int rm_mesh_clusters(rm_ctx* ctx, const rm_mesh* mesh, void* out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    int rc = check_mesh(ctx, mesh);
    if (rc) return rc;
    if (!out && mesh->n_tris > 0) return fail(ctx, RM_ERR_INVALID_ARG, "out is NULL");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_prepare(ctx->stream, mesh->xyz, mesh->n_vertices, mesh->tri, mesh->n_tris, out));
    return RM_OK;
}

int rm_render_depth(rm_ctx* ctx, const rm_mesh* mesh, rm_camera cam, const double* T_wc, int32_t n_poses,
                    float* depth_out, int32_t* tri_out, uint8_t* cls_out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    int rc = check_mesh(ctx, mesh);
    if (rc) return rc;
    if (n_poses < 0 || n_poses > 65535) return fail(ctx, RM_ERR_INVALID_ARG, "n_poses %d outside 0..65535", n_poses);
    if (n_poses == 0) return RM_OK;
    if (!T_wc) return fail(ctx, RM_ERR_INVALID_ARG, "T_wc is NULL");
    BatchDesc bd;
    std::memset(&bd, 0, sizeof(bd));
    bd.n_scans = 1;
    bd.n_poses = n_poses;
    rc = fill_scan(ctx, bd.s[0], cam);
    if (rc) return rc;
    bd.s[0].pose_off = 0;
    bd.s[0].n_poses = n_poses;
    DeviceGuard g(ctx->device);
    const int tw = ctx->tile_w ? ctx->tile_w : 64, th = ctx->tile_w ? ctx->tile_h : 32;
    return run_pass(ctx, mesh, bd, tw, th, kRender, T_wc, 1.0f, nullptr, depth_out, tri_out, cls_out, nullptr,
                    Arena());
}

int rm_align_cost(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t n_scans, const int32_t* pose_off,
                  const double* T_wc, rm_cost_params params, double* out) {
    return align_common(ctx, mesh, scans, n_scans, pose_off, T_wc, params, out, kCost, nullptr, nullptr);
}

int rm_align_cost_grad(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t n_scans,
                       const int32_t* pose_off, const double* T_wc, rm_cost_params params, double* out) {
    return align_common(ctx, mesh, scans, n_scans, pose_off, T_wc, params, out, kGrad, nullptr, nullptr);
}

int rm_depth_downsample(rm_ctx* ctx, const float* depth, int32_t height, int32_t width, int32_t factor, float z_max,
                        float* out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (!depth || !out) return fail(ctx, RM_ERR_INVALID_ARG, "NULL image pointer");
    if (height < 1 || width < 1 || (int64_t)height * width > ((int64_t)1 << 26))
        return fail(ctx, RM_ERR_INVALID_ARG, "bad image size %dx%d", width, height);
    if (factor < 1 || factor > 64) return fail(ctx, RM_ERR_INVALID_ARG, "factor %d outside 1..64", factor);
    if (!(z_max > 0.0f)) return fail(ctx, RM_ERR_INVALID_ARG, "z_max must be positive");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_downsample(ctx->stream, depth, height, width, factor, z_max, out));
    return RM_OK;
}

int rm_depth_normals(rm_ctx* ctx, const float* depth, int32_t height, int32_t width, float fx, float fy, float sigma,
                     int32_t radius, float* normals) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (!depth || !normals) return fail(ctx, RM_ERR_INVALID_ARG, "NULL image pointer");
    if (height < 1 || width < 1 || (int64_t)height * width > ((int64_t)1 << 26))
        return fail(ctx, RM_ERR_INVALID_ARG, "bad image size %dx%d", width, height);
    if (!(fx > 0.0f) || !(fy > 0.0f) || !std::isfinite(fx) || !std::isfinite(fy))
        return fail(ctx, RM_ERR_INVALID_ARG, "fx and fy must be positive and finite");
    if (!(sigma > 0.0f) || !std::isfinite(sigma)) return fail(ctx, RM_ERR_INVALID_ARG, "sigma must be positive");
    if (radius < 0 || radius > RM_MAX_NORMAL_RADIUS)
        return fail(ctx, RM_ERR_INVALID_ARG, "radius %d outside 0..%d", radius, RM_MAX_NORMAL_RADIUS);
    GaussW gw;
    std::memset(&gw, 0, sizeof(gw));
    gw.radius = radius;
    double sum = 0.0;
    for (int k = -radius; k <= radius; ++k) {
        gw.w[k + radius] = std::exp(-(double)k * k / (2.0 * (double)sigma * (double)sigma));
        sum += gw.w[k + radius];
    }
    for (int k = 0; k <= 2 * radius; ++k) gw.w[k] /= sum;
    DeviceGuard g(ctx->device);
    int rc = ensure_scratch(ctx, (size_t)height * width * sizeof(double));
    if (rc) return rc;
    RM_HIP(ctx, launch_depth_normals(ctx->stream, depth, height, width, (double)fx, (double)fy, gw, at<double>(ctx, 0),
                                     normals));
    return RM_OK;
}

int rm_vertex_normals(rm_ctx* ctx, const float* normals, int32_t height, int32_t width, int32_t stride,
                      const double* T_wc, float* out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (!normals || !out || !T_wc) return fail(ctx, RM_ERR_INVALID_ARG, "NULL pointer");
    if (height < 1 || width < 1 || (int64_t)height * width > ((int64_t)1 << 26))
        return fail(ctx, RM_ERR_INVALID_ARG, "bad image size %dx%d", width, height);
    if (stride < 1) return fail(ctx, RM_ERR_INVALID_ARG, "stride must be >= 1");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(T_wc[k])) return fail(ctx, RM_ERR_INVALID_ARG, "T_wc is not finite");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_vertex_normals(ctx->stream, normals, height, width, stride, T_wc, out));
    return RM_OK;
}

int rm_icp_cost_grad(rm_ctx* ctx, const rm_mesh* mesh, const float* vertex_normals, const rm_scan* scans,
                     int32_t n_scans, const int32_t* pose_off, const double* T_wc, float tol, double* out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (!vertex_normals) return fail(ctx, RM_ERR_INVALID_ARG, "vertex_normals is NULL");
    if (!(tol > 0.0f) || !std::isfinite(tol)) return fail(ctx, RM_ERR_INVALID_ARG, "tol must be positive and finite");
    rm_cost_params p;
    p.eps = tol;
    p.flags = 0;
    p.color_tol = 0.0f;
    return align_common(ctx, mesh, scans, n_scans, pose_off, T_wc, p, out, kIcp, vertex_normals, nullptr);
}

int rm_gn_step(rm_ctx* ctx, const double* out, int32_t n_poses, double lambda, double* T_wc, double* delta_out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (n_poses < 0) return fail(ctx, RM_ERR_INVALID_ARG, "n_poses < 0");
    if (n_poses == 0) return RM_OK;
    if (!out || !T_wc) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ctx, RM_ERR_INVALID_ARG, "lambda must be >= 0");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_gn_step(ctx->stream, out, n_poses, lambda, T_wc, delta_out));
    return RM_OK;
}

int rm_table_cost_weighted(rm_ctx* ctx, const double* out, int32_t n_poses, const double* weights, double* cost_out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (n_poses < 0) return fail(ctx, RM_ERR_INVALID_ARG, "n_poses < 0");
    if (n_poses == 0) return RM_OK;
    if (!out || !weights || !cost_out) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    for (int k = 0; k < RM_N_WEIGHTS; ++k)
        if (!std::isfinite(weights[k])) return fail(ctx, RM_ERR_INVALID_ARG, "weights must be finite");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_weighted(ctx->stream, out, n_poses, weights, cost_out));
    return RM_OK;
}

int rm_adam_step(rm_ctx* ctx, const double* out, int32_t n_poses, double lr, double beta1, double beta2, int32_t step,
                 double* m, double* v, double* T_wc) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (n_poses < 0) return fail(ctx, RM_ERR_INVALID_ARG, "n_poses < 0");
    if (n_poses == 0) return RM_OK;
    if (!out || !m || !v || !T_wc) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || step < 1)
        return fail(ctx, RM_ERR_INVALID_ARG, "need lr > 0, 0 <= beta < 1, step >= 1");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_adam_step(ctx->stream, out, n_poses, lr, beta1, beta2, step, m, v, T_wc));
    return RM_OK;
}

int rm_se3_retract(rm_ctx* ctx, const double* T_in, const double* delta, int32_t n_poses, double* T_out) {
    if (!ctx) return fail(nullptr, RM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->err.clear();
    if (n_poses < 0) return fail(ctx, RM_ERR_INVALID_ARG, "n_poses < 0");
    if (n_poses == 0) return RM_OK;
    if (!T_in || !delta || !T_out) return fail(ctx, RM_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard g(ctx->device);
    RM_HIP(ctx, launch_retract(ctx->stream, T_in, delta, n_poses, T_out));
    return RM_OK;
}

}  // extern "C"
