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
#include <tuple>
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
    uint64_t off;       // v[12][n] floats, rgba[n], then (vertex colours) vc[4][n]
    bool vcol = false;  // per-vertex colours
};

struct Workspace {
    uint64_t off = 0, bytes = 0;
    bool valid = false;
};

// A batch workspace: frame table + per-frame workspaces of one launch group.
struct BatchSlot {
    uint64_t off = 0, bytes = 0;
    bool valid = false, used = false;
    hipEvent_t done = nullptr;   // recorded after the last group that used it
    hipStream_t last = nullptr;
    uint64_t stamp = 0;
};

// A frame of the last render call (for statistics).
struct FrameRef {
    const char *ctr;  // device address of its counter set
    uint64_t quads;
    int slot;  // batch slot holding its counters, -1: the context workspace
};

// Frame tags remembered for the error log (tag % kTagRing).
constexpr uint32_t kTagRing = 4096;

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t stamp = 0;
};

// Resolved tuning of one frame.
struct Tune {
    uint32_t bin, half, k;
};

using HintKey = std::tuple<lr_scene, uint32_t, uint32_t, uint32_t>;  // scene, W, H, bin

// Pinned frame-table buffers in flight at once (host side of the batch table).
constexpr uint32_t kTabRing = 8;

// Frame workspace of lr_render_noalloc: a fixed device array, so that call
// allocates nothing.  Each device that loads the library holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in;
// the device address comes from hipGetSymbolAddress (scratch_address).
constexpr uint64_t kScratchBytes = 128ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (it is current in lr_create).
hipError_t scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct lr_context_s {
    int device = 0;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    lr_config cfg{};
    Arena alloc;
    std::map<lr_scene, SceneRec> scenes;
    lr_scene next_scene = 1;
    Workspace ws;
    uint32_t ws_set = 0;                     // counter set (0/1) the next single frame uses
    std::map<HintKey, uint32_t> pair_hints;  // bin-list capacity learnt from overflows
    std::vector<FrameRef> last_frames;       // frames of the last render call
    lr_stats acc{};                          // stats of its frames whose counters were reused
    lr::ErrLog *elog = nullptr;              // device, in the arena
    uint64_t elog_off = 0;
    uint32_t next_tag = 0;
    std::vector<HintKey> tag_keys;           // kTagRing
    std::vector<lr_tune_rule> rules;
    // batches
    std::vector<BatchSlot> slots;
    uint32_t max_slots = 2;
    uint64_t slot_stamp = 0;
    lr::FrameArgs *host_tab = nullptr;       // pinned, kTabRing x kMaxBatch
    hipEvent_t tab_ev[kTabRing] = {};
    bool tab_used[kTabRing] = {};
    uint32_t tab_head = 0;
    hipStream_t capture_stream = nullptr;
    bool use_graphs = true;
    std::map<std::vector<uint64_t>, GraphEntry> graphs;
    uint64_t graph_stamp = 0;
    hipStream_t last_stream = nullptr;
    hipEvent_t ws_free = nullptr;  // recorded after each frame that used ws
    // stage timing: one set of 8 events per frame in a ring
    std::vector<hipEvent_t> ring;  // kRing * 8
    uint32_t ring_head = 0, ring_count = 0;
    bool timing = false;
    bool cut = false;  // LR_FLAG_ALPHA_CUTOFF
    bool have_frame = false;
    std::string err;
    std::mutex mu;
    lr::FrameCounters *host_ctr = nullptr;  // pinned
    // lr_render_noalloc: this device's `scratch` and an event after the last
    // call of this context that used it
    char *scratch = nullptr;
    hipEvent_t scratch_free = nullptr;
    hipStream_t scratch_stream = nullptr;
    bool scratch_used = false;
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
    uint32_t n, W, H, bin, half, shift, nbx, nby, nbins, unit_quads, nunits, bin_waves, pair_cap, nblk_x, nblk_y,
        qcap_blocks;
    uint64_t o_cov, o_plane, o_extra, o_xy, o_bbox, o_cull, o_table, o_start, o_count, o_pairs, o_fb, o_ecode, o_emask, o_eid, o_ctr,
        o_femask, o_feid, o_blkent, o_ebound, o_binpx, o_highlist, o_binclass, o_large, o_vcrec, total;
    uint32_t fe_cap;
    uint32_t cut;  // transmittance cutoff: entries carry a bound code
    bool vcol;     // vertex-colour records
};

Plan make_plan(uint32_t n, uint32_t W, uint32_t H, uint32_t bin, uint32_t half, uint32_t pair_hint, uint32_t cut,
               bool vcol)
{
    Plan p{};
    p.cut = cut;
    p.n = n;
    p.W = W;
    p.H = H;
    p.bin = bin;
    p.half = half;
    p.shift = log2u(bin);
    p.nbx = (W + bin - 1) / bin;
    p.nby = (H + bin - 1) / bin;
    p.nbins = p.nbx * p.nby;
    // Binning units.  With at most 8192 bins four waves share a unit; each
    // unit's scatter first builds its offsets for every bin, so a unit gets
    // about nbins / 2 quads (512 to 4096), and there are at most about 1024
    // units.  More bins: one wave per unit of at least 256 quads.
    p.bin_waves = p.nbins <= 8192 ? 4u : 1u;
    uint64_t uq = (((uint64_t)n + 1023) / 1024 + 255) / 256 * 256;
    if (p.bin_waves == 4)
        uq = std::max<uint64_t>(uq, std::min<uint64_t>(4096, std::max<uint64_t>(512, (p.nbins / 2 + 511) / 512 * 512)));
    else
        uq = std::max<uint64_t>(uq, 256);
    p.unit_quads = (uint32_t)uq;
    p.nunits = std::max<uint32_t>(1, (n + uq - 1) / uq);
    // first guess; an overflow is reported and the next frame is planned larger
    uint64_t cap = 5ull * n / 2 + 4ull * p.nbins + 65536;
    cap = std::max<uint64_t>(cap, pair_hint);
    p.pair_cap = (uint32_t)std::min<uint64_t>(cap, 0xF0000000ull);
    p.nblk_x = (W + 7) / 8;
    p.nblk_y = (H + 7) / 8;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t r = o;
        o += (bytes + 255) & ~uint64_t(255);
        return r;
    };
    // two counter sets first, at the same place for every plan: a single frame
    // uses one and zeroes the other for the next frame
    p.o_ctr = take(2 * sizeof(lr::FrameCounters));
    p.o_cov = take((uint64_t)n * sizeof(lr::CovRec));
    p.o_plane = take((uint64_t)n * sizeof(lr::PlaneRec));
    p.o_extra = take((uint64_t)n * sizeof(lr::ExtraRec));
    p.o_xy = take((uint64_t)n * sizeof(lr::QuadXY));
    p.o_bbox = take((uint64_t)n * 8);
    p.o_cull = take((uint64_t)n);
    p.o_large = take((uint64_t)n * 4);
    p.o_vcrec = vcol ? take((uint64_t)n * sizeof(lr::VColRec)) : 0;
    p.vcol = vcol;
    p.o_table = take((uint64_t)p.nunits * p.nbins * 4);
    p.o_start = take(((uint64_t)p.nbins + 1) * 4);
    p.o_count = take((uint64_t)p.nbins * 4);
    p.o_binpx = take((uint64_t)p.nbins * 8);
    p.o_highlist = take((uint64_t)p.nbins * 4);
    p.o_binclass = take((uint64_t)p.nbins);
    p.o_pairs = take((uint64_t)p.pair_cap * 4);
    p.qcap_blocks = (p.nblk_x * p.nblk_y + lr::kQueues - 1) / lr::kQueues;
    p.o_fb = take((uint64_t)lr::kQueues * p.qcap_blocks * 64 * 4);
    // block entries: a region per (bin, wave) as long as the bin list, twice
    // that with half-blocks
    const uint64_t ents = (uint64_t)lr::raster_waves(p.shift) * p.pair_cap * (half ? 2 : 1);
    p.o_ecode = take(ents * 4);
    p.o_emask = take(ents * 8);
    p.o_eid = take(ents * 4);
    p.o_ebound = cut ? take(ents * 4) : 0;
    // entries kept for the exact pass (blocks past this capacity walk their bin list)
    p.fe_cap = std::max<uint32_t>(p.pair_cap, 65536u);
    p.o_femask = take((uint64_t)p.fe_cap * 8);
    p.o_feid = take((uint64_t)p.fe_cap * 4);
    p.o_blkent = take((uint64_t)p.nblk_x * p.nblk_y * 8);
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
    // both counter sets start at zero
    LR_HIP(ctx, hipMemset(ctx->arena + off, 0, 2 * sizeof(lr::FrameCounters)));
    ctx->ws_set = 0;
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

uint32_t pair_hint(lr_context ctx, lr_scene scene, uint32_t W, uint32_t H, uint32_t bin)
{
    auto it = ctx->pair_hints.find(HintKey(scene, W, H, bin));
    return it == ctx->pair_hints.end() ? 0u : it->second;
}

bool valid_k(uint32_t k) { return lr::sorter_depth_supported((int)k); }
bool valid_block_h(uint32_t b) { return b == 4 || b == 8; }

// Checks shared by every render entry point; fills the plan.
lr_status check_frame(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t W, uint32_t H,
                      const Tune &t, Plan &plan)
{
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end())
        return fail(ctx, LR_ERR_NOT_FOUND, "unknown scene handle");
    if (!cam)
        return fail(ctx, LR_ERR_INVALID_ARG, "camera is NULL");
    if (W < 1 || H < 1 || W > 16384 || H > 16384)
        return fail(ctx, LR_ERR_INVALID_ARG, "width and height must be in [1, 16384]");
    if (!valid_bin(t.bin))
        return fail(ctx, LR_ERR_INVALID_ARG, "bin size must be 16, 32 or 64");
    if (!valid_k(t.k))
        return fail(ctx, LR_ERR_INVALID_ARG, "sorter depth must be one of 2, 4, 8, 12, 16, 24, 32");
    if (!std::isfinite(cam->fov_y) || !(cam->fov_y > 0.0f) || !(cam->fov_y < 3.14159f))
        return fail(ctx, LR_ERR_INVALID_ARG, "fov_y must be in (0, pi)");
    if (it->second.vcol && ctx->cut)
        return fail(ctx, LR_ERR_INVALID_ARG, "the transmittance cutoff is defined for flat colours only");
    plan = make_plan(it->second.n, W, H, t.bin, t.half, pair_hint(ctx, scene, W, H, t.bin), ctx->cut ? 1u : 0u,
                     it->second.vcol);
    if (plan.nbins > kMaxBins)
        return fail(ctx, LR_ERR_INVALID_ARG,
                    "too many bins for this frame size (at most 16384; use a larger bin size)");
    return LR_OK;
}

// Frame arguments for a planned frame of the n quads at scene (SoA: 12
// vertex planes, then the colours) whose workspace starts at base.
void fill_frame(const char *scene, uint32_t n, const lr_camera *cam, uint8_t *out, const Plan &plan, char *base,
                lr::ErrLog *elog, lr::FrameArgs &a)
{
    std::memset(&a, 0, sizeof(a));
    a.v = reinterpret_cast<const float *>(scene);
    a.rgba_in = reinterpret_cast<const uint32_t *>(scene + 48ull * n);
    a.n = n;
    if (plan.vcol) {
        a.vcol_in = reinterpret_cast<const uint32_t *>(scene + 52ull * n);
        a.vcrec = reinterpret_cast<lr::VColRec *>(base + plan.o_vcrec);
    }
    for (int k = 0; k < 3; k++)
        a.pos[k] = cam->pos[k];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            a.rot[3 * r + c] = cam->rot[r][c];
    a.z_near = cam->z_near;
    // focal length in pixels, on the host
    a.f = (0.5 * (double)plan.H) / std::tan(0.5 * (double)cam->fov_y);
    a.cx = 0.5 * (double)plan.W;
    a.cy = 0.5 * (double)plan.H;
    a.W = plan.W;
    a.H = plan.H;
    a.cov = reinterpret_cast<lr::CovRec *>(base + plan.o_cov);
    a.plane = reinterpret_cast<lr::PlaneRec *>(base + plan.o_plane);
    a.extra = reinterpret_cast<lr::ExtraRec *>(base + plan.o_extra);
    a.xy = reinterpret_cast<lr::QuadXY *>(base + plan.o_xy);
    a.bbox = reinterpret_cast<uint2 *>(base + plan.o_bbox);
    a.cull = reinterpret_cast<uint8_t *>(base + plan.o_cull);
    a.bin_shift = plan.shift;
    a.nbx = plan.nbx;
    a.nby = plan.nby;
    a.nbins = plan.nbins;
    a.unit_quads = plan.unit_quads;
    a.bin_waves = plan.bin_waves;
    a.nunits = plan.nunits;
    a.table = reinterpret_cast<uint32_t *>(base + plan.o_table);
    a.bin_start = reinterpret_cast<uint32_t *>(base + plan.o_start);
    a.bin_count = reinterpret_cast<uint32_t *>(base + plan.o_count);
    a.pairs = reinterpret_cast<uint32_t *>(base + plan.o_pairs);
    a.pair_cap = plan.pair_cap;
    a.half_blocks = plan.half;
    a.nblk_x = plan.nblk_x;
    a.nblk_y = plan.nblk_y;
    a.qcap_blocks = plan.qcap_blocks;
    a.fb_queue = reinterpret_cast<uint32_t *>(base + plan.o_fb);
    a.ent_code = reinterpret_cast<uint32_t *>(base + plan.o_ecode);
    a.ent_mask = reinterpret_cast<unsigned long long *>(base + plan.o_emask);
    a.ent_id = reinterpret_cast<uint32_t *>(base + plan.o_eid);
    a.ent_bound = plan.cut ? reinterpret_cast<uint32_t *>(base + plan.o_ebound) : nullptr;
    // density classes (switched on per frame by set_classes)
    a.bin_px = plan.bin_waves == 4 ? reinterpret_cast<unsigned long long *>(base + plan.o_binpx) : nullptr;
    a.high_list = reinterpret_cast<uint32_t *>(base + plan.o_highlist);
    a.bin_class = reinterpret_cast<uint8_t *>(base + plan.o_binclass);
    a.k_low = 0;
    a.bbox_binning = 0;
    a.large_list = reinterpret_cast<uint32_t *>(base + plan.o_large);
    a.alpha_cut = plan.cut;
    a.fe_mask = reinterpret_cast<unsigned long long *>(base + plan.o_femask);
    a.fe_id = reinterpret_cast<uint32_t *>(base + plan.o_feid);
    a.fe_cap = plan.fe_cap;
    a.blk_ent = reinterpret_cast<uint2 *>(base + plan.o_blkent);
    a.ctr = reinterpret_cast<lr::FrameCounters *>(base + plan.o_ctr);
    a.elog = elog;
    a.out = out;
}

// The same for a resident scene of the context.
void fill_args(lr_context ctx, const SceneRec &sc, const lr_camera *cam, uint8_t *out, const Plan &plan,
               char *base, lr::FrameArgs &a)
{
    fill_frame(ctx->arena + sc.off, sc.n, cam, out, plan, base, ctx->elog, a);
    a.bbox_binning = (ctx->cfg.flags & LR_FLAG_BBOX_BINNING) ? 1u : 0u;
    a.cull_back = (ctx->cfg.flags & LR_FLAG_CULL_BACKFACES) ? 1u : 0u;
}

// Density classes of a frame rendered at sorter depth k (0: unsorted), with
// LR_FLAG_DENSITY_CLASSES: when k is deeper than kLowDepth and the binning
// can gather its density estimate (the four-wave kernels), the raster takes
// the dense bins first and the sparse ones at kLowDepth.
void set_classes(lr_context ctx, uint32_t k, lr::FrameArgs &a)
{
    const bool on = (ctx->cfg.flags & LR_FLAG_DENSITY_CLASSES) && a.bin_px && k > lr::kLowDepth;
    a.k_low = on ? lr::kLowDepth : 0u;
    if (!on)
        a.bin_px = nullptr;  // nothing to estimate
}

// Tags a frame for the error log.
void tag_frame(lr_context ctx, lr_scene scene, const Plan &plan, lr::FrameArgs &a)
{
    a.tag = ctx->next_tag++;
    ctx->tag_keys[a.tag % kTagRing] = HintKey(scene, plan.W, plan.H, plan.bin);
}

// A single frame in the context workspace.
lr_status build_args(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t W, uint32_t H,
                     uint8_t *out, const Tune &t, lr::FrameArgs &a, Plan &plan)
{
    lr_status st = check_frame(ctx, scene, cam, W, H, t, plan);
    if (st != LR_OK)
        return st;
    st = ensure_workspace(ctx, plan.total);
    if (st != LR_OK)
        return st;
    char *base = ctx->arena + ctx->ws.off;
    fill_args(ctx, ctx->scenes[scene], cam, out, plan, base, a);
    a.ctr = reinterpret_cast<lr::FrameCounters *>(base + plan.o_ctr) + ctx->ws_set;
    a.ctr_next = reinterpret_cast<lr::FrameCounters *>(base + plan.o_ctr) + (ctx->ws_set ^ 1u);
    tag_frame(ctx, scene, plan, a);
    return LR_OK;
}

Tune default_tune(lr_context ctx)
{
    return Tune{ctx->cfg.bin_size, ctx->cfg.block_h == 4 ? 1u : 0u, ctx->cfg.sorter_depth};
}

// Tuning of a request: its own fields, else the first matching rule, else
// the context defaults.
Tune resolve_tune(lr_context ctx, const lr_request &r)
{
    Tune t = default_tune(ctx);
    auto sc = ctx->scenes.find(r.scene);
    const uint64_t px = (uint64_t)r.width * r.height;
    if (sc != ctx->scenes.end() && px) {
        const double qpp = (double)sc->second.n / (double)px;
        for (const lr_tune_rule &u : ctx->rules) {
            if (px <= u.max_pixels && qpp <= (double)u.max_quads_per_pixel) {
                t = Tune{u.bin_size, u.block_h == 4 ? 1u : 0u, u.sorter_depth};
                break;
            }
        }
    }
    if (r.bin_size)
        t.bin = r.bin_size;
    if (r.sorter_depth)
        t.k = r.sorter_depth;
    if (r.block_h)
        t.half = r.block_h == 4 ? 1u : (r.block_h == 8 ? 0u : 2u);  // 2: invalid
    // Vertex-colour frames sort at depth 16 at most: deeper queues beside the
    // colour planes outgrow the register file.  The depth never changes the
    // image (pixels past the queue take the exact pass).
    if (sc != ctx->scenes.end() && sc->second.vcol && t.k > 16)
        t.k = 16;
    return t;
}

// Tuning of a single render: the first matching rule, else the defaults.
Tune frame_tune(lr_context ctx, lr_scene scene, uint32_t W, uint32_t H)
{
    lr_request r;
    std::memset(&r, 0, sizeof(r));
    r.scene = scene;
    r.width = W;
    r.height = H;
    return resolve_tune(ctx, r);
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
                      uint8_t *out, void *stream, int unsorted, const DebugOut *dbg, const Tune &t)
{
    if (!out)
        return fail(ctx, LR_ERR_INVALID_ARG, "output pointer is NULL");
    lr::FrameArgs a;
    Plan plan;
    lr_status st = build_args(ctx, scene, cam, W, H, out, t, a, plan);
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
    set_classes(ctx, unsorted ? 0u : t.k, a);
    if (unsorted)
        a.bbox_binning = 1;  // the unsorted blend needs every bin list in quad order
    hipError_t e = lr::launch_frame(a, (int)t.k, unsorted, s, ev);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "kernel launch");
    LR_HIP(ctx, hipEventRecord(ctx->ws_free, s));
    ctx->last_stream = s;
    ctx->have_frame = true;
    ctx->last_frames.clear();
    ctx->last_frames.push_back(FrameRef{reinterpret_cast<const char *>(a.ctr), a.n, -1});
    ctx->ws_set ^= 1u;
    std::memset(&ctx->acc, 0, sizeof(ctx->acc));
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

// Adds one frame's counters to *sum.
lr_status add_frame_stats(lr_context ctx, const FrameRef &fr, lr_stats *sum)
{
    LR_HIP(ctx, hipMemcpy(ctx->host_ctr, fr.ctr, sizeof(lr::FrameCounters),
                          hipMemcpyDeviceToHost));
    const lr::FrameCounters &c = *ctx->host_ctr;
    unsigned long long v[lr::ST_COUNT] = {};
    for (uint32_t k = 0; k < lr::kStripes; k++)
        for (uint32_t i = 0; i < lr::ST_COUNT; i++)
            v[i] += c.stripe[k].v[i];
    sum->quads += fr.quads;
    sum->visible += v[lr::ST_CULL0 + lr::VISIBLE];
    for (uint32_t r = 1; r < lr::kCullReasons; r++)
        sum->culled[r] += v[lr::ST_CULL0 + r];
    sum->bin_pairs += c.pairs_total;
    sum->block_entries += v[lr::ST_ENTRIES];
    sum->fragments += v[lr::ST_FRAGMENTS];
    for (uint32_t k = 0; k < lr::kQueues; k++) {
        sum->flagged_pixels += c.stripe[k].flag_n;
        sum->dense_blocks += c.stripe[k].dense_n;
    }
    sum->error_word |= c.error;
    return LR_OK;
}

// Waits for the device and reads the error log: every frame since the last
// clear whose bin lists overflowed raises its capacity hint, and the call
// reports LR_ERR_CAPACITY.  clear empties the log.
lr_status sync_impl(lr_context ctx, bool clear)
{
    LR_HIP(ctx, hipDeviceSynchronize());
    uint32_t n = 0;
    LR_HIP(ctx, hipMemcpy(&n, ctx->elog, sizeof(n), hipMemcpyDeviceToHost));
    if (n == 0)
        return LR_OK;
    const uint32_t m = std::min(n, lr::kErrLogCap);
    std::vector<lr::ErrLog::Entry> e(m);
    LR_HIP(ctx, hipMemcpy(e.data(), ctx->elog->e, m * sizeof(lr::ErrLog::Entry), hipMemcpyDeviceToHost));
    uint32_t worst = 0;
    for (const auto &x : e) {
        const uint64_t want = (uint64_t)x.pairs + x.pairs / 4 + 1024;
        uint32_t &h = ctx->pair_hints[ctx->tag_keys[x.tag % kTagRing]];
        h = std::max<uint32_t>(h, (uint32_t)std::min<uint64_t>(want, 0xF0000000ull));
        worst = std::max(worst, x.pairs);
    }
    if (clear)
        LR_HIP(ctx, hipMemset(ctx->elog, 0, sizeof(uint32_t)));
    return fail(ctx, LR_ERR_CAPACITY,
                std::to_string(n) + " frame(s) overflowed their bin lists (up to " + std::to_string(worst) +
                    " pairs); capacity raised, render again");
}

// ------------------------------------------------------------------ batches

// A slot for a launch group of `bytes` on stream s; the stream is ordered
// after the slot's previous group.  Sets *slot_out, or fails with
// LR_ERR_OUT_OF_MEMORY when no slot of that size can be had.
lr_status acquire_slot(lr_context ctx, hipStream_t s, uint64_t bytes, BatchSlot **slot_out,
                       std::vector<FrameRef> &call_frames)
{
    BatchSlot *pick = nullptr;
    for (auto &sl : ctx->slots)
        if (sl.used && sl.last == s)
            pick = &sl;
    if (!pick)
        for (auto &sl : ctx->slots)
            if (!sl.used || hipEventQuery(sl.done) == hipSuccess) {
                pick = &sl;
                break;
            }
    if (!pick && ctx->slots.size() < ctx->max_slots) {
        BatchSlot ns;
        LR_HIP(ctx, hipEventCreateWithFlags(&ns.done, hipEventDisableTiming));
        ctx->slots.push_back(ns);
        pick = &ctx->slots.back();
    }
    if (!pick) {
        pick = &ctx->slots[0];
        for (auto &sl : ctx->slots)
            if (sl.stamp < pick->stamp)
                pick = &sl;
    }
    // frames of this call still counted in the slot: fold their statistics in
    // before the slot is overwritten
    const int idx = (int)(pick - ctx->slots.data());
    bool waited = false;
    for (size_t i = 0; i < call_frames.size();) {
        if (call_frames[i].slot == idx) {
            if (!waited)
                LR_HIP(ctx, hipEventSynchronize(pick->done));
            waited = true;
            lr_status st = add_frame_stats(ctx, call_frames[i], &ctx->acc);
            if (st != LR_OK)
                return st;
            call_frames.erase(call_frames.begin() + (long)i);
        } else {
            i++;
        }
    }
    if (!pick->valid || pick->bytes < bytes) {
        if (pick->valid) {
            if (pick->used)
                LR_HIP(ctx, hipEventSynchronize(pick->done));
            ctx->alloc.release(pick->off);
            pick->valid = false;
        }
        uint64_t want = bytes + bytes / 4, off;
        if (!ctx->alloc.alloc(want, off)) {
            want = bytes;
            if (!ctx->alloc.alloc(want, off))
                return LR_ERR_OUT_OF_MEMORY;
        }
        pick->off = off;
        pick->bytes = want;
        pick->valid = true;
    }
    if (pick->used && pick->last != s)
        LR_HIP(ctx, hipStreamWaitEvent(s, pick->done, 0));
    *slot_out = pick;
    return LR_OK;
}

constexpr uint64_t kTableBytes = ((uint64_t)lr::kMaxBatch * sizeof(lr::FrameArgs) + 255) & ~uint64_t(255);

uint64_t group_bytes(const std::vector<Plan> &plans, uint32_t i0, uint32_t i1)
{
    uint64_t b = kTableBytes;
    for (uint32_t i = i0; i < i1; i++)
        b += (plans[i].total + 255) & ~uint64_t(255);
    return b;
}

// Launches one group through a cached hipGraph (captured on first use of
// this launch geometry), or directly.
lr_status launch_group(lr_context ctx, const lr::FrameArgs *host, const lr::FrameArgs *dev, const int *ks,
                       uint32_t nf, hipStream_t s)
{
    if (!ctx->use_graphs) {
        hipError_t e = lr::launch_batch(host, dev, ks, nf, s);
        return e == hipSuccess ? LR_OK : hip_fail(ctx, e, "batch launch");
    }
    // everything else the kernels read comes from the frame table
    std::vector<uint64_t> key;
    key.reserve(2 + 8 * (size_t)nf);
    key.push_back(reinterpret_cast<uint64_t>(dev));
    key.push_back(nf);
    for (uint32_t f = 0; f < nf; f++) {
        key.push_back(host[f].n);
        key.push_back(host[f].nunits);
        key.push_back(host[f].nbins);
        key.push_back(host[f].bin_shift);  // raster waves per workgroup and binning kernels
        key.push_back(host[f].bin_waves);
        key.push_back((uint64_t)ks[f]);
        key.push_back(host[f].alpha_cut);
        key.push_back(host[f].k_low);
    }
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 64) {
            // evict the least recently used; wait so no replay of it is pending
            auto old = ctx->graphs.begin();
            for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
                if (g->second.stamp < old->second.stamp)
                    old = g;
            LR_HIP(ctx, hipDeviceSynchronize());
            (void)hipGraphExecDestroy(old->second.exec);
            ctx->graphs.erase(old);
        }
        hipGraph_t g = nullptr;
        LR_HIP(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = lr::launch_batch(host, dev, ks, nf, ctx->capture_stream);
        hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return hip_fail(ctx, e != hipSuccess ? e : e2, "batch graph capture");
        }
        GraphEntry ge;
        e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "hipGraphInstantiate");
        it = ctx->graphs.emplace(key, ge).first;
    }
    it->second.stamp = ++ctx->graph_stamp;
    LR_HIP(ctx, hipGraphLaunch(it->second.exec, s));
    return LR_OK;
}

lr_status batch_impl(lr_context ctx, const lr_request *reqs, uint32_t n, hipStream_t s)
{
    std::vector<Plan> plans(n);
    std::vector<Tune> tunes(n);
    for (uint32_t i = 0; i < n; i++) {
        const lr_request &r = reqs[i];
        tunes[i] = resolve_tune(ctx, r);
        if (tunes[i].half > 1)
            return fail(ctx, LR_ERR_INVALID_ARG, "block_h must be 4 or 8");
        if (!r.out_rgba8)
            return fail(ctx, LR_ERR_INVALID_ARG, "output pointer is NULL");
        lr_status st = check_frame(ctx, r.scene, &r.camera, r.width, r.height, tunes[i], plans[i]);
        if (st != LR_OK)
            return st;
    }
    std::vector<FrameRef> frames;
    frames.reserve(n);
    std::memset(&ctx->acc, 0, sizeof(ctx->acc));
    std::vector<int> ks(lr::kMaxBatch);
    uint32_t i0 = 0;
    while (i0 < n) {
        uint32_t i1 = std::min<uint32_t>(n, i0 + lr::kMaxBatch);
        BatchSlot *slot = nullptr;
        for (;;) {
            lr_status st = acquire_slot(ctx, s, group_bytes(plans, i0, i1), &slot, frames);
            if (st == LR_OK)
                break;
            if (st != LR_ERR_OUT_OF_MEMORY)
                return st;
            if (i1 - i0 == 1)
                return fail(ctx, LR_ERR_OUT_OF_MEMORY,
                            "arena too small for one frame of the batch (" +
                                std::to_string(group_bytes(plans, i0, i1)) + " bytes)");
            i1 = i0 + (i1 - i0) / 2;
        }
        const uint32_t nf = i1 - i0;
        // host frame table (pinned ring; waits only if its previous copy is pending)
        const uint32_t h = ctx->tab_head;
        ctx->tab_head = (h + 1) % kTabRing;
        if (ctx->tab_used[h])
            LR_HIP(ctx, hipEventSynchronize(ctx->tab_ev[h]));
        lr::FrameArgs *host = ctx->host_tab + (size_t)h * lr::kMaxBatch;
        char *base = ctx->arena + slot->off;
        lr::FrameArgs *dev = reinterpret_cast<lr::FrameArgs *>(base);
        uint64_t o = kTableBytes;
        for (uint32_t f = 0; f < nf; f++) {
            const lr_request &r = reqs[i0 + f];
            const Plan &pl = plans[i0 + f];
            fill_args(ctx, ctx->scenes[r.scene], &r.camera, r.out_rgba8, pl, base + o, host[f]);
            host[f].status = r.status;
            tag_frame(ctx, r.scene, pl, host[f]);
            ks[f] = (int)tunes[i0 + f].k;
            set_classes(ctx, tunes[i0 + f].k, host[f]);
            frames.push_back(FrameRef{base + o + pl.o_ctr, pl.n, (int)(slot - ctx->slots.data())});
            o += (pl.total + 255) & ~uint64_t(255);
        }
        LR_HIP(ctx, hipMemcpyAsync(dev, host, nf * sizeof(lr::FrameArgs), hipMemcpyHostToDevice, s));
        LR_HIP(ctx, hipEventRecord(ctx->tab_ev[h], s));
        ctx->tab_used[h] = true;
        lr_status st = launch_group(ctx, host, dev, ks.data(), nf, s);
        if (st != LR_OK)
            return st;
        LR_HIP(ctx, hipEventRecord(slot->done, s));
        slot->used = true;
        slot->last = s;
        slot->stamp = ++ctx->slot_stamp;
        i0 = i1;
    }
    // copied, not moved: the vector keeps its capacity (reserved at creation),
    // so a later single-frame call adds no host allocation
    ctx->last_frames.assign(frames.begin(), frames.end());
    ctx->have_frame = n > 0;
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
    if (!valid_block_h(c.block_h))
        return fail(nullptr, LR_ERR_INVALID_ARG, "block_h must be 4 (8x4 half-blocks) or 8 (8x8 blocks)");
    if (c.batch_slots == 0)
        c.batch_slots = 2;
    if (c.batch_slots > 8)
        return fail(nullptr, LR_ERR_INVALID_ARG, "batch_slots must be at most 8");
    if (!lr::sorter_depth_supported((int)c.sorter_depth))
        return fail(nullptr, LR_ERR_INVALID_ARG, "sorter_depth must be one of 2, 4, 8, 12, 16, 24, 32");
    if (!c.arena)
        return fail(nullptr, LR_ERR_INVALID_ARG, "arena is NULL: the caller provides the device arena");
    if (c.arena_bytes < (1u << 20))
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
    ctx->arena = reinterpret_cast<char *>(c.arena);
    ctx->arena_bytes = c.arena_bytes;
    ctx->alloc.init(ctx->arena_bytes);
    ctx->timing = (c.flags & LR_FLAG_TIMING) != 0;
    ctx->use_graphs = (c.flags & LR_FLAG_NO_GRAPH) == 0;
    ctx->cut = (c.flags & LR_FLAG_ALPHA_CUTOFF) != 0;
    ctx->max_slots = c.batch_slots;
    ctx->slots.reserve(8);  // slot addresses stay fixed (at most 8 slots)
    bool ok = hipEventCreateWithFlags(&ctx->ws_free, hipEventDisableTiming) == hipSuccess;
    for (uint32_t i = 0; i < kTabRing; i++)
        ok = ok && hipEventCreateWithFlags(&ctx->tab_ev[i], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ctx->scratch_free, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&ctx->host_tab, sizeof(lr::FrameArgs) * lr::kMaxBatch * kTabRing,
                             hipHostMallocDefault) == hipSuccess;
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
    ctx->tag_keys.assign(kTagRing, HintKey(0, 0, 0, 0));
    ctx->last_frames.reserve(lr::kMaxBatch);
    {
        void *p = nullptr;
        e = scratch_address(c.device, &p);
        if (e != hipSuccess) {
            lr_destroy(ctx);
            return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
        }
        ctx->scratch = static_cast<char *>(p);
    }
    if (!ctx->alloc.alloc(sizeof(lr::ErrLog), ctx->elog_off)) {
        lr_destroy(ctx);
        return fail(nullptr, LR_ERR_OUT_OF_MEMORY, "arena too small");
    }
    ctx->elog = reinterpret_cast<lr::ErrLog *>(ctx->arena + ctx->elog_off);
    if (hipMemset(ctx->elog, 0, sizeof(lr::ErrLog)) != hipSuccess) {
        lr_destroy(ctx);
        return fail(nullptr, LR_ERR_DEVICE, "hipMemset of the error log failed");
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
    for (auto &g : ctx->graphs)
        (void)hipGraphExecDestroy(g.second.exec);
    for (auto &sl : ctx->slots)
        if (sl.done)
            (void)hipEventDestroy(sl.done);
    for (uint32_t i = 0; i < kTabRing; i++)
        if (ctx->tab_ev[i])
            (void)hipEventDestroy(ctx->tab_ev[i]);
    if (ctx->capture_stream)
        (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->host_tab)
        (void)hipHostFree(ctx->host_tab);
    if (ctx->ws_free)
        (void)hipEventDestroy(ctx->ws_free);
    if (ctx->scratch_free)
        (void)hipEventDestroy(ctx->scratch_free);
    for (auto &e : ctx->ring)
        if (e)
            (void)hipEventDestroy(e);
    if (ctx->host_ctr)
        (void)hipHostFree(ctx->host_ctr);
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
        // waits, so q may be freed on return and renders on any stream see
        // the scene
        hipError_t e = lr::launch_transpose_scene(q, n, v, rgba, ctx->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(ctx->stream);
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
    SceneRec rec;
    rec.n = n;
    rec.off = off;
    ctx->scenes[id] = rec;
    *out = id;
    return LR_OK;
}

lr_status lr_upload_scene_vertex_colors(lr_context ctx, const lr_quad_vc *q, uint32_t n, lr_scene *out)
{
    if (!ctx || !q || !out)
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || n > (1u << 24))
        return fail(ctx, LR_ERR_INVALID_ARG, "quad count must be in [1, 2^24]");
    std::lock_guard<std::mutex> lock(ctx->mu);
    uint64_t off;
    if (!ctx->alloc.alloc(68ull * n, off))
        return fail(ctx, LR_ERR_OUT_OF_MEMORY, "arena full");
    // v[12][n] fp32, rgba[n] (vertex 0's colour), vc[4][n]
    std::vector<float> hv((size_t)12 * n);
    std::vector<uint32_t> hc((size_t)5 * n);
    for (uint32_t i = 0; i < n; i++) {
        for (int k = 0; k < 4; k++) {
            for (int r = 0; r < 3; r++)
                hv[(size_t)(k * 3 + r) * n + i] = q[i].v[k][r];
            hc[(size_t)(1 + k) * n + i] = q[i].rgba[k];
        }
        hc[i] = q[i].rgba[0];
    }
    char *base = ctx->arena + off;
    hipError_t e = hipMemcpyAsync(base, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + 48ull * n, hc.data(), hc.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        ctx->alloc.release(off);
        return hip_fail(ctx, e, "scene upload");
    }
    lr_scene id = ctx->next_scene++;
    SceneRec rec;
    rec.n = n;
    rec.off = off;
    rec.vcol = true;
    ctx->scenes[id] = rec;
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
    return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 0, nullptr, frame_tune(ctx, scene, width, height));
}

lr_status lr_render_noalloc(lr_context ctx, lr_scene scene, const lr_camera *cam, uint32_t width,
                            uint32_t height, uint8_t *out_rgba8, void *stream)
{
    if (!ctx)
        return fail(nullptr, LR_ERR_INVALID_ARG, "context is NULL");
    std::unique_lock<std::mutex> lock(ctx->mu, std::try_to_lock);
    if (!lock.owns_lock())
        return fail(ctx, LR_ERR_BUSY, "context in use by another thread");
    if (!out_rgba8)
        return fail(ctx, LR_ERR_INVALID_ARG, "output pointer is NULL");
    if (!ctx->scratch)
        return fail(ctx, LR_ERR_DEVICE, "the static scratch of this device was not found");
    const Tune t = frame_tune(ctx, scene, width, height);
    Plan plan;
    lr_status st = check_frame(ctx, scene, cam, width, height, t, plan);
    if (st != LR_OK)
        return st;
    if (plan.total > kScratchBytes)
        return fail(ctx, LR_ERR_OUT_OF_MEMORY,
                    "frame workspace of " + std::to_string(plan.total) +
                        " bytes exceeds the static scratch of lr_render_noalloc (" +
                        std::to_string(kScratchBytes) + " bytes); use lr_render");
    lr::FrameArgs a;
    fill_args(ctx, ctx->scenes.find(scene)->second, cam, out_rgba8, plan, ctx->scratch, a);
    // no counter set is zeroed ahead: the frame's first kernel clears its own
    a.ctr = reinterpret_cast<lr::FrameCounters *>(ctx->scratch + plan.o_ctr);
    a.ctr_next = nullptr;
    tag_frame(ctx, scene, plan, a);
    hipStream_t s = pick_stream(ctx, stream);
    // this context's previous call on another stream may still use scratch
    if (ctx->scratch_used && ctx->scratch_stream != s)
        LR_HIP(ctx, hipStreamWaitEvent(s, ctx->scratch_free, 0));
    hipEvent_t *ev = nullptr;
    if (ctx->timing) {
        ev = &ctx->ring[(size_t)ctx->ring_head * 8];
        ctx->ring_head = (ctx->ring_head + 1) % kRing;
        ctx->ring_count = std::min(ctx->ring_count + 1, kRing);
    }
    set_classes(ctx, t.k, a);
    hipError_t e = lr::launch_frame(a, (int)t.k, 0, s, ev);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "kernel launch");
    LR_HIP(ctx, hipEventRecord(ctx->scratch_free, s));
    ctx->scratch_stream = s;
    ctx->scratch_used = true;
    ctx->have_frame = true;
    ctx->last_frames.clear();
    ctx->last_frames.push_back(FrameRef{reinterpret_cast<const char *>(a.ctr), a.n, -1});
    std::memset(&ctx->acc, 0, sizeof(ctx->acc));
    return LR_OK;
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
        return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 0, nullptr, frame_tune(ctx, scene, width, height));
    return render_impl(ctx, scene, cam, width, height, out_rgba8, stream, 0, &d, frame_tune(ctx, scene, width, height));
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
                       frame_tune(ctx, scene, width, height));
}

lr_status lr_render_batch(lr_context ctx, const lr_request *reqs, uint32_t n, void *stream)
{
    if (!ctx || (!reqs && n))
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lock(ctx->mu, std::try_to_lock);
    if (!lock.owns_lock())
        return fail(ctx, LR_ERR_BUSY, "context in use by another thread");
    if (n == 0)
        return LR_OK;
    return batch_impl(ctx, reqs, n, pick_stream(ctx, stream));
}

lr_status lr_set_tuning(lr_context ctx, const lr_tune_rule *rules, uint32_t n)
{
    if (!ctx || (!rules && n))
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    for (uint32_t i = 0; i < n; i++) {
        const lr_tune_rule &u = rules[i];
        if (!u.max_pixels || !valid_bin(u.bin_size) || !valid_block_h(u.block_h) || !valid_k(u.sorter_depth) ||
            !(u.max_quads_per_pixel > 0.0f))
            return fail(ctx, LR_ERR_INVALID_ARG, "tuning rule " + std::to_string(i) + " is invalid");
    }
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->rules.assign(rules, rules + n);
    return LR_OK;
}

lr_status lr_request_bytes(lr_context ctx, const lr_request *req, uint64_t *bytes)
{
    if (!ctx || !req || !bytes)
        return fail(ctx, LR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(ctx->mu);
    const Tune t = resolve_tune(ctx, *req);
    if (t.half > 1)
        return fail(ctx, LR_ERR_INVALID_ARG, "block_h must be 4 or 8");
    Plan plan;
    lr_status st = check_frame(ctx, req->scene, &req->camera, req->width, req->height, t, plan);
    if (st != LR_OK)
        return st;
    *bytes = (plan.total + 255) & ~uint64_t(255);
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
    std::memset(out, 0, sizeof(*out));
    lr_status st = sync_impl(ctx, false);
    if (ctx->have_frame) {
        *out = ctx->acc;
        for (const FrameRef &fr : ctx->last_frames) {
            lr_status s2 = add_frame_stats(ctx, fr, out);
            if (s2 != LR_OK)
                return s2;
        }
    }
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
    lr_status st = build_args(ctx, scene, cam, width, height, nullptr, default_tune(ctx), a, plan);
    if (st != LR_OK)
        return st;
    LR_HIP(ctx, hipDeviceSynchronize());
    a.want_xy = 1;
    LR_HIP(ctx, lr::launch_setup_only(a, ctx->stream));
    LR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // the next frame expects its counter set zeroed
    LR_HIP(ctx, hipMemset(a.ctr, 0, sizeof(lr::FrameCounters)));
    const uint32_t n = a.n;
    std::vector<lr::CovRec> cov(n);
    std::vector<lr::PlaneRec> pl(n);
    std::vector<lr::QuadXY> xy(n);
    std::vector<uint8_t> cl(n);
    LR_HIP(ctx, hipMemcpy(cov.data(), a.cov, (size_t)n * sizeof(lr::CovRec), hipMemcpyDeviceToHost));
    LR_HIP(ctx, hipMemcpy(pl.data(), a.plane, (size_t)n * sizeof(lr::PlaneRec), hipMemcpyDeviceToHost));
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
            bbox[4 * (size_t)i + 0] = vis ? (int32_t)(cov[i].bb_i & 0xffff) : 1;
            bbox[4 * (size_t)i + 1] = vis ? (int32_t)(cov[i].bb_i >> 16) : 0;
            bbox[4 * (size_t)i + 2] = vis ? (int32_t)(cov[i].bb_j & 0xffff) : 1;
            bbox[4 * (size_t)i + 3] = vis ? (int32_t)(cov[i].bb_j >> 16) : 0;
        }
        if (plane) {
            plane[3 * (size_t)i + 0] = vis ? pl[i].A : 0.0;
            plane[3 * (size_t)i + 1] = vis ? pl[i].B : 0.0;
            plane[3 * (size_t)i + 2] = vis ? pl[i].C0 : 0.0;
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
    Tune t = default_tune(ctx);
    t.bin = bin_size;
    lr_status st = build_args(ctx, scene, cam, width, height, nullptr, t, a, plan);
    if (st != LR_OK)
        return st;
    LR_HIP(ctx, hipDeviceSynchronize());
    LR_HIP(ctx, lr::launch_binning_only(a, ctx->stream));
    LR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    lr::FrameCounters c;
    LR_HIP(ctx, hipMemcpy(&c, a.ctr, sizeof(c), hipMemcpyDeviceToHost));
    // the next frame expects its counter set zeroed
    LR_HIP(ctx, hipMemset(a.ctr, 0, sizeof(lr::FrameCounters)));
    if (total)
        *total = c.pairs_total;
    if (counts)
        LR_HIP(ctx, hipMemcpy(counts, a.bin_count, (size_t)a.nbins * 4, hipMemcpyDeviceToHost));
    if (c.error & lr::kErrPairs)
        return sync_impl(ctx, true);  // raises the capacity hint; call again
    if (ids) {
        if (c.pairs_total > ids_cap)
            return fail(ctx, LR_ERR_CAPACITY, "ids_cap smaller than the number of pairs");
        LR_HIP(ctx, hipMemcpy(ids, a.pairs, (size_t)c.pairs_total * 4, hipMemcpyDeviceToHost));
    }
    return LR_OK;
}

}  // extern "C"
