// Host runtime behind the C ABI in include/lucidraster.h: context, device
// arena sub-allocator, resident scenes, per-frame plan and launches, stats.
#include "lucidraster.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lr_internal.h"

namespace {

thread_local std::string g_last_error = "";

// First-fit allocator over [0, size) of a device arena (256-byte aligned).
class Arena {
public:
    void init(uint64_t size) { free_.clear(); free_[0] = size; }
    bool alloc(uint64_t bytes, uint64_t &off)
    {
        bytes = (bytes + 255) & ~uint64_t(255);
        if (bytes == 0)
            bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                uint64_t rest = it->second - bytes;
                free_.erase(it);
                if (rest)
                    free_[off + bytes] = rest;
                used_[off] = bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end())
            return;
        uint64_t bytes = u->second;
        used_.erase(u);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (auto &f : free_)
            m = std::max(m, f.second);
        return m;
    }

private:
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
    std::map<uint64_t, uint64_t> used_;
};

struct SceneRec {
    uint32_t n;
    uint64_t off;  // v[12][n] floats then rgba[n]
};

struct Workspace {
    uint64_t off = 0, bytes = 0;
    bool valid = false;
};

}  // namespace

struct lr_context_s {
    int device = 0;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    bool own_arena = false;
    lr_config cfg{};
    Arena alloc;
    std::map<lr_scene, SceneRec> scenes;
    lr_scene next_scene = 1;
    Workspace ws;
    uint64_t ws_ctr_off = 0;       // FrameCounters of the last frame (inside ws)
    uint32_t pair_hint = 0;        // capacity learnt from an overflow
    hipStream_t last_stream = nullptr;
    hipEvent_t ws_free = nullptr;  // recorded after each frame that used ws
    // stage timing: one set of 8 events per frame in a ring
    std::vector<hipEvent_t> ring;  // kRing * 8
    uint32_t ring_head = 0, ring_count = 0;
    bool timing = false;
    bool have_frame = false;
    uint64_t last_quads = 0;
    std::string err;
    std::mutex mu;
    lr::FrameCounters *host_ctr = nullptr;  // pinned
};

namespace {

lr_status fail(lr_context ctx, lr_status s, const std::string &msg)
{
    g_last_error = msg;
    if (ctx)
        ctx->err = msg;
    return s;
}

lr_status hip_fail(lr_context ctx, hipError_t e, const char *what)
{
    return fail(ctx, LR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define LR_HIP(ctx, call)                                 \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess)                             \
            return hip_fail((ctx), e_, #call);            \
    } while (0)

uint32_t log2u(uint32_t x)
{
    uint32_t s = 0;
    while ((1u << s) < x)
        s++;
    return s;
}

// Byte layout of a frame workspace.
struct Plan {
    uint32_t n, W, H, bin, shift, nbx, nby, nbins, unit_quads, nunits, ntiles, pair_cap, nblk_x, nblk_y,
        match_bits, qcap_blocks;
    uint64_t o_rec, o_xy, o_bbox, o_cull, o_table, o_tiles, o_start, o_count, o_pairs, o_fb, o_ecode, o_emask, o_eid, o_ctr,
        total;
};

Plan make_plan(uint32_t n, uint32_t W, uint32_t H, uint32_t bin, uint32_t pair_hint)
{
    Plan p{};
    p.n = n;
    p.W = W;
    p.H = H;
    p.bin = bin;
    p.shift = log2u(bin);
    p.nbx = (W + bin - 1) / bin;
    p.nby = (H + bin - 1) / bin;
    p.nbins = p.nbx * p.nby;
    // about 1024 binning units, each a multiple of 64 quads, at least 512
    uint32_t uq = (uint32_t)std::max<uint64_t>(512, (((uint64_t)n + 1023) / 1024 + 63) / 64 * 64);
    p.unit_quads = uq;
    p.nunits = std::max<uint32_t>(1, (n + uq - 1) / uq);
    p.ntiles = (p.nunits + 63) / 64;
    // first guess; an overflow is reported and the next frame is planned larger
    uint64_t cap = 5ull * n / 2 + 4ull * p.nbins + 65536;
    cap = std::max<uint64_t>(cap, pair_hint);
    p.pair_cap = (uint32_t)std::min<uint64_t>(cap, 0xF0000000ull);
    p.nblk_x = (W + 7) / 8;
    p.nblk_y = (H + 7) / 8;
    p.match_bits = std::max<uint32_t>(1, log2u(p.nbins));
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t r = o;
        o += (bytes + 255) & ~uint64_t(255);
        return r;
    };
    p.o_rec = take((uint64_t)n * sizeof(lr::QuadRec));
    p.o_xy = take((uint64_t)n * sizeof(lr::QuadXY));
    p.o_bbox = take((uint64_t)n * 8);
    p.o_cull = take((uint64_t)n);
    p.o_table = take((uint64_t)p.nunits * p.nbins * 4);
    p.o_tiles = take((uint64_t)p.ntiles * p.nbins * 4);
    p.o_start = take(((uint64_t)p.nbins + 1) * 4);
    p.o_count = take((uint64_t)p.nbins * 4);
    p.o_pairs = take((uint64_t)p.pair_cap * 4);
    p.qcap_blocks = (p.nblk_x * p.nblk_y + lr::kQueues - 1) / lr::kQueues;
    p.o_fb = take((uint64_t)lr::kQueues * p.qcap_blocks * 64 * 4);
    p.o_ecode = take((uint64_t)lr::kRasterWaves * p.pair_cap * 4);
    p.o_emask = take((uint64_t)lr::kRasterWaves * p.pair_cap * 8);
    p.o_eid = take((uint64_t)lr::kRasterWaves * p.pair_cap * 4);
    p.o_ctr = take(sizeof(lr::FrameCounters));
    p.total = o;
    return p;
}

// Frames whose stage times are kept when timing is on.
constexpr uint32_t kRing = 1024;

// The binning kernels keep one 32-bit counter per bin in LDS (64 KiB).
constexpr uint32_t kMaxBins = 16384;

bool valid_bin(uint32_t b) { return b == 16 || b == 32 || b == 64; }

lr_status ensure_workspace(lr_context ctx, uint64_t bytes)
{
    if (ctx->ws.valid && ctx->ws.bytes >= bytes)
        return LR_OK;
    if (ctx->ws.valid) {
        // in-flight frames may still read the old workspace
        LR_HIP(ctx, hipDeviceSynchronize());
        ctx->alloc.release(ctx->ws.off);
        ctx->ws.valid = false;
    }
    uint64_t want = bytes + bytes / 4;
    uint64_t off;
    if (!ctx->alloc.alloc(want, off)) {
        if (!ctx->alloc.alloc(bytes, off))
            return fail(ctx, LR_ERR_OUT_OF_MEMORY,
                        "arena too small for the frame workspace (" + std::to_string(bytes) + " bytes)");
        want = bytes;
    }
    ctx->ws.off = off;
    ctx->ws.bytes = want;
    ctx->ws.valid = true;
    return LR_OK;
}

struct DebugOut {
    float *rgba = nullptr;
    uint32_t *count = nullptr;
    uint8_t *flag = nullptr;
    const uint32_t *off = nullptr;
    uint32_t *ids = nullptr;
    uint32_t cap = 0;
};

lr_status build_args(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t W, uint32_t H,
                     uint8_t *out, uint32_t bin, lr::FrameArgs &a, Plan &plan)
{
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end())
        return fail(ctx, LR_ERR_NOT_FOUND, "unknown scene handle");
    if (!cam)
        return fail(ctx, LR_ERR_INVALID_ARG, "camera is NULL");
    if (W < 1 || H < 1 || W > 16384 || H > 16384)
        return fail(ctx, LR_ERR_INVALID_ARG, "width and height must be in [1, 16384]");
    if (!valid_bin(bin))
        return fail(ctx, LR_ERR_INVALID_ARG, "bin size must be 16, 32 or 64");
    if (!std::isfinite(cam->fov_y) || !(cam->fov_y > 0.0f) || !(cam->fov_y < 3.14159f))
        return fail(ctx, LR_ERR_INVALID_ARG, "fov_y must be in (0, pi)");
    const SceneRec &sc = it->second;
    plan = make_plan(sc.n, W, H, bin, ctx->pair_hint);
    if (plan.nbins > kMaxBins)
        return fail(ctx, LR_ERR_INVALID_ARG,
                    "too many bins for this frame size (at most 16384; use a larger bin size)");
    lr_status st = ensure_workspace(ctx, plan.total);
    if (st != LR_OK)
        return st;
    char *base = ctx->arena + ctx->ws.off;
    std::memset(&a, 0, sizeof(a));
    a.v = reinterpret_cast<const float *>(ctx->arena + sc.off);
    a.rgba_in = reinterpret_cast<const uint32_t *>(ctx->arena + sc.off + 48ull * sc.n);
    a.n = sc.n;
    for (int k = 0; k < 3; k++)
        a.pos[k] = cam->pos[k];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            a.rot[3 * r + c] = cam->rot[r][c];
    a.z_near = cam->z_near;
    // focal length in pixels, on the host
    a.f = (0.5 * (double)H) / std::tan(0.5 * (double)cam->fov_y);
    a.cx = 0.5 * (double)W;
    a.cy = 0.5 * (double)H;
    a.W = W;
    a.H = H;
    a.rec = reinterpret_cast<lr::QuadRec *>(base + plan.o_rec);
    a.xy = reinterpret_cast<lr::QuadXY *>(base + plan.o_xy);
    a.bbox = reinterpret_cast<uint2 *>(base + plan.o_bbox);
    a.cull = reinterpret_cast<uint8_t *>(base + plan.o_cull);
    a.bin_shift = plan.shift;
    a.nbx = plan.nbx;
    a.nby = plan.nby;
    a.nbins = plan.nbins;
    a.unit_quads = plan.unit_quads;
    a.nunits = plan.nunits;
    a.ntiles = plan.ntiles;
    a.table = reinterpret_cast<uint32_t *>(base + plan.o_table);
    a.tile_sums = reinterpret_cast<uint32_t *>(base + plan.o_tiles);
    a.bin_start = reinterpret_cast<uint32_t *>(base + plan.o_start);
    a.bin_count = reinterpret_cast<uint32_t *>(base + plan.o_count);
    a.pairs = reinterpret_cast<uint32_t *>(base + plan.o_pairs);
    a.pair_cap = plan.pair_cap;
    a.match_bits = plan.match_bits;
    a.nblk_x = plan.nblk_x;
    a.nblk_y = plan.nblk_y;
    a.qcap_blocks = plan.qcap_blocks;
    a.fb_queue = reinterpret_cast<uint32_t *>(base + plan.o_fb);
    a.ent_code = reinterpret_cast<uint32_t *>(base + plan.o_ecode);
    a.ent_mask = reinterpret_cast<unsigned long long *>(base + plan.o_emask);
    a.ent_id = reinterpret_cast<uint32_t *>(base + plan.o_eid);
    a.ctr = reinterpret_cast<lr::FrameCounters *>(base + plan.o_ctr);
    a.out = out;
    ctx->ws_ctr_off = ctx->ws.off + plan.o_ctr;
    return LR_OK;
}

hipStream_t pick_stream(lr_context ctx, void *stream)
{
    return stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
}

// Frames share the context workspace: a frame on another stream waits for
// the previous frame to release it.
lr_status order_after_previous(lr_context ctx, hipStream_t s)
{
    if (ctx->have_frame && ctx->last_stream != s)
        LR_HIP(ctx, hipStreamWaitEvent(s, ctx->ws_free, 0));
    return LR_OK;
}

lr_status render_impl(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t W, uint32_t H,
                      uint8_t *out, void *stream, int unsorted, const DebugOut *dbg, uint32_t bin,
                      uint32_t k)
{
    if (!out)
        return fail(ctx, LR_ERR_INVALID_ARG, "output pointer is NULL");
    if (!lr::sorter_depth_supported((int)k))
        return fail(ctx, LR_ERR_INVALID_ARG, "sorter depth must be one of 2, 4, 8, 12, 16, 24, 32");
    lr::FrameArgs a;
    Plan plan;
    lr_status st = build_args(ctx, scene, cam, W, H, out, bin, a, plan);
    if (st != LR_OK)
        return st;
    if (dbg) {
        a.dbg_rgba = dbg->rgba;
        a.dbg_count = dbg->count;
        a.dbg_flag = dbg->flag;
        a.dbg_off = dbg->off;
        a.dbg_ids = dbg->ids;
        a.dbg_cap = dbg->cap;
    }
    hipStream_t s = pick_stream(ctx, stream);
    st = order_after_previous(ctx, s);
    if (st != LR_OK)
        return st;
    hipEvent_t *ev = nullptr;
    if (ctx->timing) {
        ev = &ctx->ring[(size_t)ctx->ring_head * 8];
        ctx->ring_head = (ctx->ring_head + 1) % kRing;
        ctx->ring_count = std::min(ctx->ring_count + 1, kRing);
    }
    hipError_t e = lr::launch_frame(a, (int)k, unsorted, s, ev);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "kernel launch");
    LR_HIP(ctx, hipEventRecord(ctx->ws_free, s));
    ctx->last_stream = s;
    ctx->have_frame = true;
    ctx->last_quads = a.n;
    return LR_OK;
}

void stage_times(lr_context ctx, uint32_t slot, float *us)
{
    hipEvent_t *ev = &ctx->ring[(size_t)slot * 8];
    float ms = 0.0f;
    for (int i = 0; i < 7; i++)
        us[i] = hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess ? ms * 1000.0f : 0.0f;
    us[7] = hipEventElapsedTime(&ms, ev[0], ev[7]) == hipSuccess ? ms * 1000.0f : 0.0f;
}

lr_status sync_impl(lr_context ctx, bool clear)
{
    LR_HIP(ctx, hipDeviceSynchronize());
    if (!ctx->have_frame)
        return LR_OK;
    LR_HIP(ctx, hipMemcpy(ctx->host_ctr, ctx->arena + ctx->ws_ctr_off, sizeof(lr::FrameCounters),
                          hipMemcpyDeviceToHost));
    const uint32_t err = ctx->host_ctr->error;
    if (err & lr::kErrPairs) {
        uint64_t want = (uint64_t)ctx->host_ctr->pairs_total + ctx->host_ctr->pairs_total / 4 + 1024;
        ctx->pair_hint = (uint32_t)std::min<uint64_t>(want, 0xF0000000ull);
        if (clear)
            ctx->host_ctr->error &= ~lr::kErrPairs;
        return fail(ctx, LR_ERR_CAPACITY,
                    "bin lists overflowed (" + std::to_string(ctx->host_ctr->pairs_total) +
                        " pairs); capacity raised, render again");
    }
    if (err & lr::kErrFallback)
        return fail(ctx, LR_ERR_CAPACITY, "a pixel had more fragments than the exact per-pixel sort holds");
    return LR_OK;
}

}  // namespace

extern "C" {

const char *lr_status_string(lr_status s)
{
    switch (s) {
    case LR_OK: return "LR_OK";
    case LR_ERR_INVALID_ARG: return "LR_ERR_INVALID_ARG";
    case LR_ERR_OUT_OF_MEMORY: return "LR_ERR_OUT_OF_MEMORY";
    case LR_ERR_DEVICE: return "LR_ERR_DEVICE";
    case LR_ERR_CAPACITY: return "LR_ERR_CAPACITY";
    case LR_ERR_NOT_FOUND: return "LR_ERR_NOT_FOUND";
    case LR_ERR_BUSY: return "LR_ERR_BUSY";
    default: return "LR_ERR_UNKNOWN";
    }
}

const char *lr_last_error(lr_context ctx)
{
    if (ctx)
        return ctx->err.c_str();
    return g_last_error.c_str();
}

lr_status lr_create(const lr_config *cfg, lr_context *out)
{
    if (!cfg || !out)
        return fail(nullptr, LR_ERR_INVALID_ARG, "config or output is NULL");
    lr_config c = *cfg;
    if (c.bin_size == 0)
        c.bin_size = 32;
    if (c.block_h == 0)
        c.block_h = 8;
    if (c.sorter_depth == 0)
        c.sorter_depth = 8;
    if (!valid_bin(c.bin_size))
        return fail(nullptr, LR_ERR_INVALID_ARG, "bin_size must be 16, 32 or 64");
    if (c.block_h != 8)
        return fail(nullptr, LR_ERR_INVALID_ARG, "block_h must be 8 (8x8 blocks)");
    if (!lr::sorter_depth_supported((int)c.sorter_depth))
        return fail(nullptr, LR_ERR_INVALID_ARG, "sorter_depth must be one of 2, 4, 8, 12, 16, 24, 32");
    if (c.arena && c.arena_bytes < (1u << 20))
        return fail(nullptr, LR_ERR_INVALID_ARG, "arena must be at least 1 MiB");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0)
        return fail(nullptr, LR_ERR_DEVICE, "no HIP device available");
    if (c.device < 0 || c.device >= ndev)
        return fail(nullptr, LR_ERR_INVALID_ARG, "device ordinal out of range");
    lr_context ctx = new (std::nothrow) lr_context_s();
    if (!ctx)
        return fail(nullptr, LR_ERR_OUT_OF_MEMORY, "host allocation failed");
    ctx->cfg = c;
    ctx->device = c.device;
    e = hipSetDevice(c.device);
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(nullptr, e, "hipSetDevice");
    }
    ctx->stream = reinterpret_cast<hipStream_t>(c.stream);
    if (c.arena) {
        ctx->arena = reinterpret_cast<char *>(c.arena);
        ctx->arena_bytes = c.arena_bytes;
    } else {
        ctx->arena_bytes = c.arena_bytes ? c.arena_bytes : (1ull << 30);
        void *p = nullptr;
        e = hipMalloc(&p, ctx->arena_bytes);
        if (e != hipSuccess) {
            delete ctx;
            return fail(nullptr, LR_ERR_OUT_OF_MEMORY, "hipMalloc of the arena failed");
        }
        ctx->arena = reinterpret_cast<char *>(p);
        ctx->own_arena = true;
    }
    ctx->alloc.init(ctx->arena_bytes);
    ctx->timing = (c.flags & LR_FLAG_TIMING) != 0;
    bool ok = hipEventCreateWithFlags(&ctx->ws_free, hipEventDisableTiming) == hipSuccess;
    if (ctx->timing) {
        ctx->ring.assign((size_t)kRing * 8, nullptr);
        for (auto &ev : ctx->ring)
            if (ok)
                ok = hipEventCreate(&ev) == hipSuccess;
    }
    ok = ok && hipHostMalloc((void **)&ctx->host_ctr, sizeof(lr::FrameCounters), hipHostMallocDefault) ==
                   hipSuccess;
    if (!ok) {
        lr_destroy(ctx);
        return fail(nullptr, LR_ERR_DEVICE, "HIP event or pinned allocation failed");
    }
    std::memset(ctx->host_ctr, 0, sizeof(lr::FrameCounters));
    *out = ctx;
    return LR_OK;
}

lr_status lr_destroy(lr_context ctx)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    (void)hipDeviceSynchronize();
    if (ctx->ws_free)
        (void)hipEventDestroy(ctx->ws_free);
    for (auto &e : ctx->ring)
        if (e)
            (void)hipEventDestroy(e);
    if (ctx->host_ctr)
        (void)hipHostFree(ctx->host_ctr);
    if (ctx->own_arena && ctx->arena)
        (void)hipFree(ctx->arena);
    delete ctx;
    return LR_OK;
}

lr_status lr_upload_scene(lr_context ctx, const lr_quad *q, uint32_t n, int q_on_device, lr_scene *out)
{
    if (!ctx || !q || !out)
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || n > (1u << 24))
        return fail(ctx, LR_ERR_INVALID_ARG, "quad count must be in [1, 2^24]");
    std::lock_guard<std::mutex> lock(ctx->mu);
    uint64_t off;
    if (!ctx->alloc.alloc(52ull * n, off))
        return fail(ctx, LR_ERR_OUT_OF_MEMORY, "arena full");
    float *v = reinterpret_cast<float *>(ctx->arena + off);
    uint32_t *rgba = reinterpret_cast<uint32_t *>(ctx->arena + off + 48ull * n);
    if (q_on_device) {
        hipError_t e = lr::launch_transpose_scene(q, n, v, rgba, ctx->stream);
        if (e != hipSuccess) {
            ctx->alloc.release(off);
            return hip_fail(ctx, e, "scene transpose");
        }
    } else {
        std::vector<float> hv((size_t)12 * n);
        std::vector<uint32_t> hc(n);
        for (uint32_t i = 0; i < n; i++) {
            for (int k = 0; k < 4; k++)
                for (int r = 0; r < 3; r++)
                    hv[(size_t)(k * 3 + r) * n + i] = q[i].v[k][r];
            hc[i] = q[i].rgba;
        }
        hipError_t e = hipMemcpyAsync(v, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rgba, hc.data(), hc.size() * 4, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            ctx->alloc.release(off);
            return hip_fail(ctx, e, "scene upload");
        }
    }
    lr_scene id = ctx->next_scene++;
    ctx->scenes[id] = SceneRec{n, off};
    *out = id;
    return LR_OK;
}

lr_status lr_release_scene(lr_context ctx, lr_scene scene)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end())
        return fail(ctx, LR_ERR_NOT_FOUND, "unknown scene handle");
    LR_HIP(ctx, hipDeviceSynchronize());
    ctx->alloc.release(it->second.off);
    ctx->scenes.erase(it);
    return LR_OK;
}

lr_status lr_render(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width, uint32_t height,
                    uint8_t *out_rgba8, void *stream)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::unique_lock<std::mutex> lock(ctx->mu, std::try_to_lock);
    if (!lock.owns_lock())
        return fail(ctx, LR_ERR_BUSY, "context in use by another thread");
    return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 0, nullptr, ctx->cfg.bin_size,
                       ctx->cfg.sorter_depth);
}

lr_status lr_render_debug(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                          uint32_t height, uint8_t *out_rgba8, void *stream, float *rgba_f32, uint32_t *counts,
                          uint8_t *flagged, const uint32_t *order_offsets, uint32_t *order_ids,
                          uint32_t order_cap)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    if ((order_ids != nullptr) != (order_offsets != nullptr))
        return fail(ctx, LR_ERR_INVALID_ARG, "order_ids and order_offsets go together");
    std::unique_lock<std::mutex> lock(ctx->mu, std::try_to_lock);
    if (!lock.owns_lock())
        return fail(ctx, LR_ERR_BUSY, "context in use by another thread");
    DebugOut d;
    d.rgba = rgba_f32;
    d.count = counts;
    d.flag = flagged;
    d.off = order_offsets;
    d.ids = order_ids;
    d.cap = order_cap;
    if (!rgba_f32 && !counts && !flagged && !order_ids)
        return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 0, nullptr, ctx->cfg.bin_size,
                           ctx->cfg.sorter_depth);
    return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 0, &d, ctx->cfg.bin_size,
                       ctx->cfg.sorter_depth);
}

lr_status lr_render_unsorted(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                             uint32_t height, uint8_t *out_rgba8, void *stream, float *rgba_f32)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::unique_lock<std::mutex> lock(ctx->mu, std::try_to_lock);
    if (!lock.owns_lock())
        return fail(ctx, LR_ERR_BUSY, "context in use by another thread");
    DebugOut d;
    d.rgba = rgba_f32;
    return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 1, rgba_f32 ? &d : nullptr,
                       ctx->cfg.bin_size, ctx->cfg.sorter_depth);
}

lr_status lr_render_batch(lr_context ctx, const lr_request *reqs, uint32_t n, void *stream)
{
    if (!ctx || (!reqs && n))
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lock(ctx->mu, std::try_to_lock);
    if (!lock.owns_lock())
        return fail(ctx, LR_ERR_BUSY, "context in use by another thread");
    for (uint32_t i = 0; i < n; i++) {
        const lr_request &r = reqs[i];
        uint32_t bin = r.bin_size ? r.bin_size : ctx->cfg.bin_size;
        uint32_t k = r.sorter_depth ? r.sorter_depth : ctx->cfg.sorter_depth;
        lr_status st = render_impl(ctx, r.scene, &r.camera, r.width, r.height, r.out_rgba8, stream, 0, nullptr,
                                   bin, k);
        if (st != LR_OK)
            return st;
    }
    return LR_OK;
}

lr_status lr_sync(lr_context ctx)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    return sync_impl(ctx, true);
}

lr_status lr_get_stats(lr_context ctx, lr_stats *out)
{
    if (!ctx || !out)
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(ctx->mu);
    lr_status st = sync_impl(ctx, false);
    std::memset(out, 0, sizeof(*out));
    if (!ctx->have_frame)
        return st;
    const lr::FrameCounters &c = *ctx->host_ctr;
    unsigned long long sum[lr::ST_COUNT] = {};
    for (uint32_t k = 0; k < lr::kStripes; k++)
        for (uint32_t i = 0; i < lr::ST_COUNT; i++)
            sum[i] += c.stripe[k].v[i];
    out->quads = ctx->last_quads;
    out->visible = sum[lr::ST_CULL0 + lr::VISIBLE];
    for (int r = 1; r < 6; r++)
        out->culled[r] = sum[lr::ST_CULL0 + r];
    out->bin_pairs = c.pairs_total;
    out->block_entries = sum[lr::ST_ENTRIES];
    out->fragments = sum[lr::ST_FRAGMENTS];
    for (uint32_t k = 0; k < lr::kQueues; k++) {
        out->flagged_pixels += c.stripe[k].flag_n;
        out->dense_blocks += c.stripe[k].dense_n;
    }
    out->error_word = c.error;
    if (ctx->timing && ctx->ring_count) {
        const uint32_t last = (ctx->ring_head + kRing - 1) % kRing;
        stage_times(ctx, last, out->stage_us);
    }
    return st;
}

lr_status lr_get_stage_times(lr_context ctx, uint32_t max_frames, float *us, uint32_t *n_out)
{
    if (!ctx || !n_out || (max_frames && !us))
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(ctx->mu);
    *n_out = 0;
    if (!ctx->timing)
        return fail(ctx, LR_ERR_INVALID_ARG, "the context was created without LR_FLAG_TIMING");
    LR_HIP(ctx, hipDeviceSynchronize());
    const uint32_t n = std::min(max_frames, ctx->ring_count);
    for (uint32_t f = 0; f < n; f++) {
        const uint32_t slot = (ctx->ring_head + kRing - n + f) % kRing;
        stage_times(ctx, slot, us + 8 * (size_t)f);
    }
    *n_out = n;
    return LR_OK;
}

lr_status lr_debug_setup(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                         uint32_t height, int32_t *X, int32_t *Y, int32_t *bbox, double *plane, uint8_t *cull)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    lr::FrameArgs a;
    Plan plan;
    lr_status st = build_args(ctx, scene, cam, width, height, nullptr, ctx->cfg.bin_size, a, plan);
    if (st != LR_OK)
        return st;
    LR_HIP(ctx, hipDeviceSynchronize());
    LR_HIP(ctx, lr::launch_setup_only(a, ctx->stream));
    LR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const uint32_t n = a.n;
    std::vector<lr::QuadRec> rec(n);
    std::vector<lr::QuadXY> xy(n);
    std::vector<uint8_t> cl(n);
    LR_HIP(ctx, hipMemcpy(rec.data(), a.rec, (size_t)n * sizeof(lr::QuadRec), hipMemcpyDeviceToHost));
    LR_HIP(ctx, hipMemcpy(xy.data(), a.xy, (size_t)n * sizeof(lr::QuadXY), hipMemcpyDeviceToHost));
    LR_HIP(ctx, hipMemcpy(cl.data(), a.cull, n, hipMemcpyDeviceToHost));
    for (uint32_t i = 0; i < n; i++) {
        const bool vis = cl[i] == lr::VISIBLE;
        const bool snapped = cl[i] == lr::VISIBLE || cl[i] == lr::DEGENERATE || cl[i] == lr::NO_SAMPLE ||
                             cl[i] == lr::EDGE_ON;
        for (int k = 0; k < 4; k++) {
            if (X)
                X[4 * (size_t)i + k] = snapped ? xy[i].X[k] : 0;
            if (Y)
                Y[4 * (size_t)i + k] = snapped ? xy[i].Y[k] : 0;
        }
        if (bbox) {
            bbox[4 * (size_t)i + 0] = vis ? (int32_t)(rec[i].bb_i & 0xffff) : 1;
            bbox[4 * (size_t)i + 1] = vis ? (int32_t)(rec[i].bb_i >> 16) : 0;
            bbox[4 * (size_t)i + 2] = vis ? (int32_t)(rec[i].bb_j & 0xffff) : 1;
            bbox[4 * (size_t)i + 3] = vis ? (int32_t)(rec[i].bb_j >> 16) : 0;
        }
        if (plane) {
            plane[3 * (size_t)i + 0] = vis ? rec[i].A : 0.0;
            plane[3 * (size_t)i + 1] = vis ? rec[i].B : 0.0;
            plane[3 * (size_t)i + 2] = vis ? rec[i].C0 : 0.0;
        }
        if (cull)
            cull[i] = cl[i];
    }
    return LR_OK;
}

lr_status lr_debug_bins(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width, uint32_t height,
                        uint32_t bin_size, uint32_t *counts, uint32_t *ids, uint64_t ids_cap, uint64_t *total)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (bin_size == 0)
        bin_size = ctx->cfg.bin_size;
    lr::FrameArgs a;
    Plan plan;
    lr_status st = build_args(ctx, scene, cam, width, height, nullptr, bin_size, a, plan);
    if (st != LR_OK)
        return st;
    LR_HIP(ctx, hipDeviceSynchronize());
    LR_HIP(ctx, lr::launch_binning_only(a, ctx->stream));
    LR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    lr::FrameCounters c;
    LR_HIP(ctx, hipMemcpy(&c, a.ctr, sizeof(c), hipMemcpyDeviceToHost));
    if (total)
        *total = c.pairs_total;
    if (counts)
        LR_HIP(ctx, hipMemcpy(counts, a.bin_count, (size_t)a.nbins * 4, hipMemcpyDeviceToHost));
    if (c.error & lr::kErrPairs) {
        uint64_t want = (uint64_t)c.pairs_total + c.pairs_total / 4 + 1024;
        ctx->pair_hint = (uint32_t)std::min<uint64_t>(want, 0xF0000000ull);
        return fail(ctx, LR_ERR_CAPACITY, "bin lists overflowed; capacity raised, call again");
    }
    if (ids) {
        if (c.pairs_total > ids_cap)
            return fail(ctx, LR_ERR_CAPACITY, "ids_cap smaller than the number of pairs");
        LR_HIP(ctx, hipMemcpy(ids, a.pairs, (size_t)c.pairs_total * 4, hipMemcpyDeviceToHost));
    }
    return LR_OK;
}

}  // extern "C"
