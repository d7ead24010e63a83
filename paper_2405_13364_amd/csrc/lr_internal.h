// Internal layouts shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lr {

// Cull reasons, in the order the setup stage tests them.
enum Cull : uint8_t { VISIBLE = 0, NEAR = 1, GUARD = 2, DEGENERATE = 3, NO_SAMPLE = 4, EDGE_ON = 5, BACKFACE = 6 };
constexpr uint32_t kCullReasons = 7;

// Quads whose snapped vertex extent stays within 2^18 sub-pixel units (1024
// px) in x and y use 32-bit half-plane tests; wider quads take an exact fp64
// path.  Bound: |a*di + b*dj| <= 2*ext^2/256 + 16*ext < 2^30 for ext <= 2^18.
constexpr int32_t kNarrowExtent = 1 << 18;

// Per visible quad, what the raster stage reads, split by when it is read
// (attributes read together are stored together, as the paper's setup
// stage does with its per-triangle storages, Stage 1, Phase 2).
//
// Half-plane h of triangle T (h = 3T + e) holds (a, b, t): the sample of pixel
// (imin + di, jmin + dj) is inside edge e iff a*di + b*dj >= t.  A zero-area
// triangle stores (0, 0, 1), which no sample satisfies.  This is the
// top-left rule made integral: with E the edge function in sub-pixel units
// and R the sample of pixel (imin, jmin), E(S) = E(R) + 256 (a di + b dj), and
// E(S) >= bias (bias 0 on top-left edges, 1 otherwise) iff
// a di + b dj >= ceil((bias - E(R)) / 256).
//
// CovRec: read for every (block, candidate quad) pair to build the coverage
// mask: the first four half-planes (all of a convex quad's), bbox, flags,
// colour.  64 bytes.
struct alignas(64) CovRec {
    int32_t hp[12];   // half-planes 0..3 (a, b, t)           bytes 0..47
    uint32_t bb_i;    // imin | imax << 16                    48
    uint32_t bb_j;    // jmin | jmax << 16                    52
    uint32_t flags;   // kWide | kConvex | triangle bits      56
    uint32_t rgba;    //                                      60
};
static_assert(sizeof(CovRec) == 64, "CovRec is 64 bytes");

// PlaneRec: read for every non-empty entry and by the per-pixel walk: the
// reciprocal-depth plane (fp64) relative to the bbox origin, that origin and
// the colour.  32 bytes.
struct alignas(32) PlaneRec {
    double A, B, C0;
    uint32_t ij;      // imin | jmin << 16
    uint32_t rgba;
};
static_assert(sizeof(PlaneRec) == 32, "PlaneRec is 32 bytes");

// ExtraRec: half-planes 4 and 5, written and read only for quads that are
// not strictly convex (two triangles of three edges each).
struct alignas(32) ExtraRec {
    int32_t hp[6];
    uint32_t pad[2];
};
static_assert(sizeof(ExtraRec) == 32, "ExtraRec is 32 bytes");

// VColRec: per-vertex colours of a visible quad (scenes uploaded with vertex
// colours), for each of its triangles T0 = (P0, P1, P2) and T1 = (P0, P2,
// P3): five planes (a, b, c) in fp64, relative to the bbox origin ij --
// the sum of the barycentric weights (pl[t][0..2]) and the weighted sums of
// R, G, B and A (pl[t][3 + 3 ch ..]).  At pixel (imin + di, jmin + dj),
// channel ch is plane(3 + 3 ch) / plane(0), each plane fma(a, di, fma(b, dj,
// c)).  256 bytes.
struct alignas(32) VColRec {
    double pl[2][15];
    uint32_t ij;       // imin | jmin << 16
    uint32_t pad[3];
};
static_assert(sizeof(VColRec) == 256, "VColRec is 256 bytes");

constexpr uint32_t kWide = 1u;       // use the fp64 coverage path
constexpr uint32_t kT0Valid = 2u;    // triangle (P0, P1, P2) has non-zero area
constexpr uint32_t kT0Swap = 4u;     // ... and is stored as (P0, P2, P1)
constexpr uint32_t kT1Valid = 8u;    // triangle (P0, P2, P3)
constexpr uint32_t kT1Swap = 16u;
// Strictly convex quad with consistent winding: hp[0..11] hold its four
// outer edges (P0P1, P1P2, P2P3, P3P0, oriented to positive area) and a
// sample is covered iff it is inside all four.  This equals the union of
// the two triangles under the top-left rule: both triangles then have the
// quad's orientation, and a sample moved by the rule's infinitesimal shift
// (eps, eps^2) never lies on the shared diagonal.
constexpr uint32_t kConvex = 32u;

// The small/large split of Stage 1, Phase 1: a quad whose bbox meets more
// than kLargeBins bins of 32 x 32 pixels is large (whatever the frame's bin
// size).
constexpr uint32_t kLargeBins = 4;

// Snapped vertices (sub-pixel units) of a quad.
struct alignas(32) QuadXY {
    int32_t X[4];
    int32_t Y[4];
};

// Statistics are accumulated in kStripes copies, one 128-byte line each,
// picked by workgroup index: device-scope atomics on one address serialize
// across the XCDs, atomics on different lines do not.  The host sums them.
constexpr uint32_t kStripes = 256;
enum Stat { ST_CULL0 = 0, ST_ENTRIES = 7, ST_FRAGMENTS = 8, ST_COUNT = 9 };  // ST_CULL0 + reason

// The queue of flagged pixels is split the same way into kQueues stripes (by
// block index), each with its counter in the stripe's line; a stripe holds at
// most 64 x qcap_blocks pixels.  dense_n counts blocks done in depth slices.
constexpr uint32_t kQueues = 64;

struct alignas(128) StatStripe {
    unsigned long long v[ST_COUNT];
    uint32_t dense_n;   // blocks processed in depth slices
    uint32_t flag_n;    // pixels in flagged-queue stripe
    uint32_t pad[12];
};
static_assert(sizeof(StatStripe) == 128, "one line per stripe");

// Device counters of one frame (zeroed by the first kernel of the frame).
struct FrameCounters {
    uint32_t pairs_total;      // (bin, quad) pairs found by the scan
    uint32_t error;            // kErr* bits
    uint32_t fe_n;             // entries kept for the exact pass (may exceed fe_cap)
    uint32_t n_high;           // bins in high_list
    uint32_t n_large;          // quads in large_list
    uint32_t pad[27];
    StatStripe stripe[kStripes];
};

// blk_ent of a flagged block whose entries were not kept
constexpr uint32_t kNoEntries = 0xFFFFFFFFu;

constexpr uint32_t kErrPairs = 1u;      // bin lists overflowed their capacity
constexpr uint32_t kErrDense = 4u;      // a block could not be sliced to fit its list (pixels sent to the exact sort)

// Context-wide log of frames whose bin lists overflowed, kept until the host
// reads and clears it (frame workspaces, and their counters, are reused by
// later frames before the host looks).
constexpr uint32_t kErrLogCap = 480;
struct ErrLog {
    uint32_t n;          // overflows logged (may exceed kErrLogCap)
    uint32_t pad[31];
    struct Entry {
        uint32_t tag;    // FrameArgs::tag of the frame
        uint32_t pairs;  // pairs the frame needed
    } e[kErrLogCap];
};

// Waves per raster workgroup (one bin, one 8x8 block per wave at a time):
// 4 for a 16-pixel bin (its 4 blocks in one round), 8 for 32 pixels (2
// rounds of 16 blocks), 16 for 64 pixels (4 rounds of 64 blocks); measured
// on the 1280x720 and 1920x1080 workloads.
__host__ __device__ constexpr uint32_t raster_waves(uint32_t bin_shift)
{
    return bin_shift <= 4 ? 4u : (bin_shift == 5 ? 8u : 16u);
}

// The same for a sorter depth: 16-wave workgroups leave 128 VGPRs per lane,
// too few for the deeper sorters, which keep 8 waves.
__host__ __device__ constexpr uint32_t raster_waves_for(uint32_t bin_shift, int sorter_depth)
{
    return (raster_waves(bin_shift) == 16 && sorter_depth > 12) ? 8u : raster_waves(bin_shift);
}

// Bands of bin rows of the four-wave scatter: each unit's scatter is split
// over workgroups that own one band each, so that the band's per-wave
// offsets (four rows of at most kBandBins words) leave room for several
// workgroups per CU.  Bands double until one holds at most kBandBins bins
// (or is a single row).
constexpr uint32_t kBandBins = 2048;

__host__ __device__ constexpr uint32_t scatter_bands(uint32_t nbx, uint32_t nby)
{
    uint32_t s = 1;
    while (2 * s <= nby && ((nby + s - 1) / s) * nbx > kBandBins)
        s *= 2;
    return s;
}

// Bins of the largest band.
__host__ __device__ constexpr uint32_t band_bins(uint32_t nbx, uint32_t nby)
{
    return (nby + scatter_bands(nbx, nby) - 1) / scatter_bands(nbx, nby) * nbx;
}

// Everything one frame's kernels need (passed by value).
struct FrameArgs {
    // scene (SoA): v[(k*3 + r) * n + q] for vertex k, component r; rgba[n]
    const float *v;
    const uint32_t *rgba_in;
    uint32_t n;
    // per-vertex colours vcol_in[k * n + q] of vertex k (null: flat colours),
    // and the interpolation records setup writes for them
    const uint32_t *vcol_in;
    VColRec *vcrec;
    // camera
    float pos[3];
    float rot[9];
    float z_near;
    double f, cx, cy;
    uint32_t W, H;
    // setup outputs
    CovRec *cov;
    PlaneRec *plane;
    ExtraRec *extra;
    QuadXY *xy;
    uint2 *bbox;      // (imin | imax << 16, jmin | jmax << 16); culled: (0xffff, 0xffff)
    uint8_t *cull;
    uint32_t want_xy;  // write snapped vertices of every snapped quad (parity dump); else wide quads only
    uint32_t cull_back;  // cull back-facing quads (dd < 0: clockwise on the display)
    // binning
    uint32_t bin_shift;     // log2(bin size)
    uint32_t nbx, nby, nbins;
    uint32_t unit_quads;    // quads per binning unit (multiple of 256)
    uint32_t nunits;
    uint32_t bin_waves;     // waves per binning workgroup (1, or 4 for at most 8192 bins)
    uint32_t *table;        // [nunits][nbins]
    uint32_t *bin_start;    // [nbins + 1]
    uint32_t *bin_count;    // [nbins]
    uint32_t *pairs;        // [pair_cap]
    uint32_t pair_cap;
    // density classes (the paper's Section 4 suggests adapting bins to the
    // density and running low- and high-density rasterizers together): per
    // bin, the sum over its pairs of the quad bbox's pixels inside the bin,
    // a depth-complexity estimate d; the scan lists the dense bins (d above
    // kDenseDepth, ctr->n_high of them, rasterized first) and marks each
    // bin's class (kSparse: d at most kSparseDepth, rasterized with a
    // kLowDepth sorter).  Null / 0 when the frame has one class.
    unsigned long long *bin_px;  // [nbins]
    uint32_t *high_list;         // [nbins]
    uint8_t *bin_class;          // [nbins]
    uint32_t k_low;              // sorter depth of sparse bins (0: one class)
    // large quads (bbox over more than kLargeBins bins of 32 px) are binned
    // to the bins their half-planes do not trivially reject, with their
    // bins spread over a wave's lanes; 1: every quad by its whole bbox
    uint32_t bbox_binning;
    // the frame's large quads, listed by setup (ctr->n_large of them, in no
    // particular order); every binning workgroup takes a strided share
    uint32_t *large_list;    // [n]
    // raster
    uint32_t half_blocks;     // 1: block lists are sorted per 8x4 half-block
    uint32_t nblk_x, nblk_y;  // 8x8 blocks
    uint32_t qcap_blocks;     // blocks per queue stripe: ceil(nblk_x*nblk_y / kQueues)
    uint32_t *fb_queue;       // flagged pixels [kQueues][qcap_blocks * 64]
    // block entries of the raster stage, per (bin, wave) region of the bin's
    // length at entry (NW * bin_start[bin] + wave * bin_count[bin], NW the
    // raster waves per workgroup)
    // ((1 + half_blocks) times those sizes with half-blocks)
    uint32_t *ent_code;       // block depth code
    unsigned long long *ent_mask;  // 64-sample coverage mask
    uint32_t *ent_id;         // quad index
    uint32_t *ent_bound;      // with the cutoff: nearest possible order code of the entry's fragments
    // transmittance cutoff: a pixel stops after the fragment that brings its
    // fp32 transmittance below 2^-20 (0: exact blend of every fragment)
    uint32_t alpha_cut;
    // entries of blocks with flagged pixels, kept for the exact pass: each
    // block's entries that cover one of its flagged pixels, their masks
    // restricted to those pixels, and the quad indices
    unsigned long long *fe_mask;
    uint32_t *fe_id;
    uint32_t fe_cap;
    uint2 *blk_ent;           // per 8x8 block with flagged pixels: (first, count) in fe_*,
                              // or (kNoEntries, 0) when they did not fit (the bin list is walked)
    FrameCounters *ctr;
    // single frames: the other of the workspace's two counter sets, zeroed by
    // this frame's last kernel for the next frame (null: k_frame_begin zeroes ctr)
    FrameCounters *ctr_next;
    ErrLog *elog;
    uint32_t tag;             // host-assigned frame tag for the error log
    uint8_t *out;             // RGBA8
    // debug outputs (may be null)
    float *dbg_rgba;
    uint32_t *dbg_count;
    uint8_t *dbg_flag;
    const uint32_t *dbg_off;
    uint32_t *dbg_ids;
    uint32_t dbg_cap;
    // device word receiving the frame's error bits (may be null)
    uint32_t *status;
};

// Frames per batched launch: the frame map travels in the kernel arguments.
constexpr uint32_t kMaxBatch = 64;

// Source of a workgroup's frame.  OneFrame: a single frame, its arguments by
// value.  FrameMap: frames of a batch whose arguments sit in device memory;
// for one launch, wg0[f] is the first workgroup of frame f and wg0[nf] the
// grid size (a frame with no work in the launch has wg0[f] == wg0[f + 1]).
struct OneFrame {
    FrameArgs a;
};

struct FrameMap {
    const FrameArgs *tab;
    uint32_t nf;
    uint32_t wg0[kMaxBatch + 1];
};

// Density classes of a bin by its depth estimate d (the pixels of its pairs'
// bboxes inside it, per pixel of the bin): dense above kDenseDepth, sparse
// at most kSparseDepth, mid between.
enum BinClass : uint8_t { kSparse = 0, kMid = 1, kDense = 2 };
constexpr uint32_t kDenseDepth = 32;
constexpr uint32_t kSparseDepth = 2;
// Sorter depth of sparse bins when the frame's depth is larger.
constexpr uint32_t kLowDepth = 4;


// Kernel launches (lr_kernels.hip).
hipError_t launch_frame(const FrameArgs &a, int sorter_depth, int unsorted, hipStream_t s,
                        hipEvent_t *ev /* 8 events or null */);
hipError_t launch_setup_only(const FrameArgs &a, hipStream_t s);
hipError_t launch_binning_only(const FrameArgs &a, hipStream_t s);
hipError_t launch_transpose_scene(const void *quads_dev, uint32_t n, float *v, uint32_t *rgba,
                                  hipStream_t s);
bool sorter_depth_supported(int k);

// A batch of nf <= kMaxBatch frames: host copies of their arguments (for the
// launch geometry), the same arguments already in device memory (dev), and
// each frame's sorter depth.  One launch per stage covers every frame (one
// per distinct sorter depth for the raster stage).
hipError_t launch_batch(const FrameArgs *host, const FrameArgs *dev, const int *sorter_depth, uint32_t nf,
                        hipStream_t s);


}  // namespace lr
