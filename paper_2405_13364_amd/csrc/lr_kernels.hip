// gfx950 kernels of the exact-transparency rasterizer.
//
// Stages (paper Section 2, "Pipeline description"):
//   setup    one lane per quad: cull, project, snap, bbox, half-planes, depth
//            plane (Stage 1);
//   binning  per-bin lists of quad indices by counting, prefix sums and a
//            stable scatter, so every list is in ascending quad index (Stage 2);
//   raster   one wave per 8x8 block of a bin: coverage masks of the bin's
//            quads, a block-level depth sort, then one lane per pixel walks
//            the sorted entries through a K-deep per-pixel sorter and blends
//            front to back (Stage 3).  A pixel whose sorter would emit an
//            out-of-order fragment is detected and recomputed by an exact
//            per-pixel sort.
// The exactness contract: coverage and fragment keys are integer or exactly
// specified IEEE operations (built with -ffp-contract=off; fma only where
// written), and every pixel's blend sequence is its fragments in ascending
// (~bits(key), quad index) order.
#include "lr_internal.h"

#include <math.h>

#include <algorithm>

namespace lr {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

// v of lane (this lane ^ m), for a constant power of two m.  Within a row of
// 16 lanes the exchange is a DPP move (quad permutes for 1 and 2, row
// rotations for 4 and 8); across rows and halves it is gfx950's
// permlane16 / permlane32 swap.  All are VALU operations: no LDS round
// trip, so chains of them (sorting networks, transposes, reductions) carry
// no LDS latency.  Every lane must be active.
__device__ __forceinline__ uint32_t shfl_xor(uint32_t v, int m)
{
    const uint32_t lane = lane_id();
    switch (m) {
    case 1:
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);  // quad_perm 1,0,3,2
    case 2:
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);  // quad_perm 2,3,0,1
    case 4: {
        const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false);  // row_ror 4
        const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x12C, 0xf, 0xf, false);  // row_ror 12
        return (lane & 4) ? dn : up;
    }
    case 8:
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);  // row_ror 8
    case 16: {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    case 32: {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
    default:
        return (uint32_t)__shfl_xor((int)v, m, 64);
    }
}

// Inclusive prefix sum over the wave: a Hillis-Steele scan within each row
// of 16 lanes by DPP row shifts, then the row totals carried across rows by
// the row broadcasts of lanes 15 and 31.  Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr 1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr 2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr 4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr 8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast 15 -> rows 1, 3
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast 31 -> rows 2, 3
    return v;
}

// Transpose a 64x64 bit matrix held one row per lane (lane e holds row e as
// lo | hi << 32).  Afterwards lane p holds column p: bit e set iff row e has
// bit p.  Each level swaps one bit of the row index with the same bit of the
// column index.
__device__ __forceinline__ uint64_t transpose64(uint64_t m, uint32_t lane)
{
    uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
    {
        // lanes 0-31 take hi from lane + 32's lo, lanes 32-63 lo from lane - 32's hi
        const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        lo = r[0];
        hi = r[1];
    }
#define LR_TRANSPOSE_LEVEL(S, MASK)                                                  \
    {                                                                                \
        const bool up = lane & (S);                                                  \
        uint32_t plo = shfl_xor(lo, (S)), phi = shfl_xor(hi, (S));                   \
        lo = up ? ((lo & ~(MASK)) | ((plo >> (S)) & (MASK))) : ((lo & (MASK)) | ((plo & (MASK)) << (S))); \
        hi = up ? ((hi & ~(MASK)) | ((phi >> (S)) & (MASK))) : ((hi & (MASK)) | ((phi & (MASK)) << (S))); \
    }
    LR_TRANSPOSE_LEVEL(16, 0x0000FFFFu)
    LR_TRANSPOSE_LEVEL(8, 0x00FF00FFu)
    LR_TRANSPOSE_LEVEL(4, 0x0F0F0F0Fu)
    LR_TRANSPOSE_LEVEL(2, 0x33333333u)
    LR_TRANSPOSE_LEVEL(1, 0x55555555u)
#undef LR_TRANSPOSE_LEVEL
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Orders LDS accesses among the lanes of one wave (a wavefront-scope fence:
// no wait for outstanding global memory operations).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fragment order code: ascending code = nearer first (the high word of the
// total order; the quad index is the low word).  k >= +0 always.
__device__ __forceinline__ float frag_key(double A, double B, double C0, int di, int dj)
{
    double v = fma(A, (double)di, fma(B, (double)dj, C0));
    float k = (float)v;
    return (k > 0.0f) ? k : 0.0f;
}

__device__ __forceinline__ uint32_t order_code(float k) { return ~__float_as_uint(k); }

// A colour as the blend uses it: alpha and the three channels, each byte /
// 255 in fp32.
__device__ __forceinline__ float4 decode_rgba(uint32_t c)
{
    const float s = 1.0f / 255.0f;
    return make_float4((float)(c >> 24) * s, (float)(c & 255u) * s, (float)((c >> 8) & 255u) * s,
                       (float)((c >> 16) & 255u) * s);
}

// Front-to-back blend step (fp32) of a decoded colour (x = alpha), shared by
// every sorted path so that their results are bit-identical.
__device__ __forceinline__ void blend_ftb_dec(float4 d, float &T, float &R, float &G, float &B)
{
    const float w = T * d.x;
    R = fmaf(w, d.y, R);
    G = fmaf(w, d.z, G);
    B = fmaf(w, d.w, B);
    T = T * (1.0f - d.x);
}


// Transmittance below which a pixel stops when the cutoff is on (the
// tolerance-safe form of the alpha threshold of Stage 3, "Sample blending":
// what is left out weighs less than 2^-20 per channel).
constexpr float kCutT = 0x1p-20f;

// Front-to-back step with the cutoff: the same arithmetic as blend_ftb_dec
// until a fragment brings T below kCutT; from then on the pixel is stopped
// and later fragments blend nothing.  T keeps its value at the stop, so
// "stopped" is T < kCutT (T starts at 1).
__device__ __forceinline__ void blend_ftb_cut(float4 d, float &T, float &R, float &G, float &B)
{
    const bool stopped = T < kCutT;
    const float w = stopped ? 0.0f : T * d.x;
    R = fmaf(w, d.y, R);
    G = fmaf(w, d.z, G);
    B = fmaf(w, d.w, B);
    const float Tn = T * (1.0f - d.x);
    T = stopped ? T : Tn;
}

// "Over" step of the unsorted baseline (fp32) for a blend operand d
// (alpha, R, G, B).
__device__ __forceinline__ void blend_over_dec(float4 d, float &R, float &G, float &B, float &Al)
{
    const float om = 1.0f - d.x;
    R = fmaf(d.x, d.y, om * R);
    G = fmaf(d.x, d.z, om * G);
    B = fmaf(d.x, d.w, om * B);
    Al = fmaf(om, Al, d.x);
}

__device__ __forceinline__ uint32_t to_u8(float x)
{
    float y = floorf(x * 255.0f + 0.5f);
    y = fminf(fmaxf(y, 0.0f), 255.0f);
    return (uint32_t)y;
}

__device__ __forceinline__ uint32_t pack_rgba8(float R, float G, float B, float A)
{
    return to_u8(R) | (to_u8(G) << 8) | (to_u8(B) << 16) | (to_u8(A) << 24);
}

// ------------------------------------------------------- frame resolution
//
// Every kernel runs either for one frame (arguments by value) or for a batch
// of frames (one grid covering all of them): frame_of gives the workgroup's
// frame and its workgroup index within that frame.

__device__ __forceinline__ const FrameArgs *frame_of(const OneFrame &src, uint32_t &blk)
{
    blk = blockIdx.x;
    return &src.a;
}

__device__ __forceinline__ const FrameArgs *frame_of(const FrameMap &m, uint32_t &blk)
{
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = m.nf;  // wg0[lo] <= b < wg0[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (m.wg0[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    blk = b - m.wg0[lo];
    return m.tab + lo;
}

// The small/large split of Stage 1, Phase 1: a quad whose pixel bbox meets
// more than kLargeBins bins of 32 x 32 pixels is large.
__device__ __forceinline__ bool quad_is_large(uint2 bb)
{
    const uint32_t imin = bb.x & 0xffffu, imax = bb.x >> 16, jmin = bb.y & 0xffffu, jmax = bb.y >> 16;
    if (imin > imax || jmin > jmax)
        return false;
    return ((imax >> 5) - (imin >> 5) + 1) * ((jmax >> 5) - (jmin >> 5) + 1) > kLargeBins;
}

// ------------------------------------------------------------- frame begin

template <class Src>
__global__ __launch_bounds__(256) void k_frame_begin(Src src)
{
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    uint4 *p = reinterpret_cast<uint4 *>(a.ctr);
    for (uint32_t i = threadIdx.x; i < sizeof(FrameCounters) / 16; i += blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

__device__ __forceinline__ void add_stat(FrameCounters *c, uint32_t stat, unsigned long long v)
{
    atomicAdd(&c->stripe[blockIdx.x % kStripes].v[stat], v);
}

// ------------------------------------------------------------------- setup

// Integer geometry of snapped vertices in fp64.  A guarded vertex lies
// within 32768 px of the origin, so its sub-pixel coordinates are integers
// below 2^23 in magnitude, differences of them below 2^24, and every
// product below and difference of products below 2^50: all exact in fp64,
// whose multiply runs at full rate where a 64-bit integer multiply takes
// several quarter-rate ones.  The values are the integer ones.
__device__ __forceinline__ double edge_fn(double ax, double ay, double bx, double by, double px, double py)
{
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

// Threshold t of an edge from (sx, sy) along (dx, dy) for the pixel-centre
// sample R: with E the edge function in sub-pixel units, a sample is inside
// iff E(S) >= bias (0 on top-left edges, 1 otherwise), and E(S) = E(R) +
// 256 (a di + b dj), so t = ceil((bias - E(R)) / 256), clamped to int32.
__device__ __forceinline__ int32_t edge_threshold(double sx, double sy, double dx, double dy, double Rx, double Ry)
{
    const bool top_left = (dy < 0.0) || (dy == 0.0 && dx > 0.0);
    const double er = dx * (Ry - sy) - dy * (Rx - sx);
    const double t = ceil(((top_left ? 0.0 : 1.0) - er) * (1.0 / 256.0));
    return (int32_t)fmin(fmax(t, (double)INT32_MIN), (double)INT32_MAX);
}

// Half-planes of triangle (ia, ib, ic) relative to sample R = (Rx, Ry).
__device__ void tri_halfplanes(const int32_t *X, const int32_t *Y, int ia, int ib, int ic, double Rx, double Ry,
                               int32_t *hp, uint32_t &flags, uint32_t valid_bit, uint32_t swap_bit)
{
    double vx[3] = {(double)X[ia], (double)X[ib], (double)X[ic]};
    double vy[3] = {(double)Y[ia], (double)Y[ib], (double)Y[ic]};
    const double area2 = edge_fn(vx[0], vy[0], vx[1], vy[1], vx[2], vy[2]);
    if (area2 == 0.0) {
        for (int e = 0; e < 3; e++) {
            hp[3 * e] = 0;
            hp[3 * e + 1] = 0;
            hp[3 * e + 2] = 1;
        }
        return;
    }
    flags |= valid_bit;
    if (area2 < 0.0) {
        flags |= swap_bit;
        const double tx = vx[1], ty = vy[1];
        vx[1] = vx[2];
        vy[1] = vy[2];
        vx[2] = tx;
        vy[2] = ty;
    }
    for (int e = 0; e < 3; e++) {
        const double sx = vx[e], sy = vy[e];
        const double dx = vx[(e + 1) % 3] - sx, dy = vy[(e + 1) % 3] - sy;
        hp[3 * e] = (int32_t)(-dy);
        hp[3 * e + 1] = (int32_t)dx;
        hp[3 * e + 2] = edge_threshold(sx, sy, dx, dy, Rx, Ry);
    }
}

// A strictly convex quad (all four corner turns of one sign) gets its four
// outer edges, oriented to positive area, in hp[0..11] and kConvex.
__device__ void convex_halfplanes(const int32_t *X, const int32_t *Y, double Rx, double Ry, int32_t *hp,
                                  uint32_t &flags)
{
    double fx[4], fy[4];
    for (int k = 0; k < 4; k++) {
        fx[k] = (double)X[k];
        fy[k] = (double)Y[k];
    }
    int sgn[4];
    for (int k = 0; k < 4; k++) {
        const int p = k, q = (k + 1) & 3, r = (k + 2) & 3;
        const double t = edge_fn(fx[p], fy[p], fx[q], fy[q], fx[r], fy[r]);
        sgn[k] = (t > 0.0) - (t < 0.0);
    }
    const bool pos = sgn[0] > 0 && sgn[1] > 0 && sgn[2] > 0 && sgn[3] > 0;
    const bool neg = sgn[0] < 0 && sgn[1] < 0 && sgn[2] < 0 && sgn[3] < 0;
    if (!pos && !neg)
        return;
    int32_t h[12];
    for (int e = 0; e < 4; e++) {
        // positive orientation: P0 P1 P2 P3, or reversed P0 P3 P2 P1
        const int s0 = pos ? e : (4 - e) & 3;
        const int s1 = pos ? (e + 1) & 3 : (3 - e) & 3;
        const double sx = fx[s0], sy = fy[s0], dx = fx[s1] - sx, dy = fy[s1] - sy;
        h[3 * e] = (int32_t)(-dy);
        h[3 * e + 1] = (int32_t)dx;
        h[3 * e + 2] = edge_threshold(sx, sy, dx, dy, Rx, Ry);
    }
    for (int k = 0; k < 12; k++)
        hp[k] = h[k];
    flags |= kConvex;
}

// A visible quad's setup results, held in registers; k_setup stores them
// as the quad's CovRec, PlaneRec and, when it is not strictly convex, its
// ExtraRec.
// Interpolation planes of a quad's vertex colours (Stage 3, "Sample
// shading": per-vertex attributes interpolated per sample).  For a triangle
// with camera-space vertices (A, B, C), the ray through pixel centre (px,
// py), r = ((px - cx)/f, -(py - cy)/f, 1), meets the triangle's plane at
// barycentric weights proportional to r.(BxC), r.(CxA), r.(AxB): affine in
// the pixel, so each weight, their sum and the weighted colour sums are
// planes over (di, dj) = (px - 0.5 - imin, py - 0.5 - jmin).
__device__ void vertex_colour_planes(const FrameArgs &a, uint32_t q, const double (*c)[3], int imin, int jmin)
{
    VColRec rec;
    const double u0 = ((double)imin + 0.5) - a.cx, w0 = ((double)jmin + 0.5) - a.cy;
    for (int t = 0; t < 2; t++) {
        const int idx[3] = {0, t ? 2 : 1, t ? 3 : 2};
        double pl[15];
        for (int k = 0; k < 15; k++)
            pl[k] = 0.0;
        for (int k = 0; k < 3; k++) {
            const double *P = c[idx[(k + 1) % 3]], *Q = c[idx[(k + 2) % 3]];
            double n[3], p, s;
            p = P[1] * Q[2]; s = P[2] * Q[1]; n[0] = p - s;
            p = P[2] * Q[0]; s = P[0] * Q[2]; n[1] = p - s;
            p = P[0] * Q[1]; s = P[1] * Q[0]; n[2] = p - s;
            // the weight w_k(di, dj) = wa di + wb dj + wc
            const double wa = n[0] / a.f, wb = -n[1] / a.f;
            const double wc = (u0 * n[0] - w0 * n[1]) / a.f + n[2];
            const uint32_t col = a.vcol_in[(size_t)idx[k] * a.n + q];
            pl[0] += wa;
            pl[1] += wb;
            pl[2] += wc;
            for (int ch = 0; ch < 4; ch++) {
                const double v = (double)((col >> (8 * ch)) & 255u) / 255.0;
                pl[3 + 3 * ch] += v * wa;
                pl[4 + 3 * ch] += v * wb;
                pl[5 + 3 * ch] += v * wc;
            }
        }
        for (int k = 0; k < 15; k++)
            rec.pl[t][k] = pl[k];
    }
    rec.ij = (uint32_t)imin | ((uint32_t)jmin << 16);
    rec.pad[0] = rec.pad[1] = rec.pad[2] = 0;
    a.vcrec[q] = rec;
}

// Whether triangle (P0, P_ib, P_ic) of the snapped vertices covers the centre
// of pixel (px, py) under the top-left rule (exact: products below 2^50 in
// fp64); a zero-area triangle covers nothing.
__device__ bool snapped_tri_covers(const QuadXY &xy, int ib, int ic, int px, int py)
{
    const double Sx = 256.0 * (double)px + 128.0, Sy = 256.0 * (double)py + 128.0;
    double vx[3] = {(double)xy.X[0], (double)xy.X[ib], (double)xy.X[ic]};
    double vy[3] = {(double)xy.Y[0], (double)xy.Y[ib], (double)xy.Y[ic]};
    const double area2 = (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vy[1] - vy[0]) * (vx[2] - vx[0]);
    if (area2 == 0.0)
        return false;
    if (area2 < 0.0) {
        const double tx = vx[1], ty = vy[1];
        vx[1] = vx[2];
        vy[1] = vy[2];
        vx[2] = tx;
        vy[2] = ty;
    }
    for (int e = 0; e < 3; e++) {
        const double dx = vx[(e + 1) % 3] - vx[e], dy = vy[(e + 1) % 3] - vy[e];
        const double E = dx * (Sy - vy[e]) - dy * (Sx - vx[e]);
        const bool tl = (dy < 0.0) || (dy == 0.0 && dx > 0.0);
        if (!(E > 0.0 || (E == 0.0 && tl)))
            return false;
    }
    return true;
}

// The colour of quad q at pixel (px, py), which it covers: interpolated over
// T0 if T0 covers the sample, else over T1; as a blend operand (alpha, R, G,
// B), like decode_rgba.
__device__ float4 vertex_colour(const FrameArgs &a, uint32_t q, int px, int py)
{
    const QuadXY xy = a.xy[q];
    const int t = snapped_tri_covers(xy, 1, 2, px, py) ? 0 : 1;
    const VColRec &r = a.vcrec[q];
    const double di = (double)(px - (int)(r.ij & 0xffffu)), dj = (double)(py - (int)(r.ij >> 16));
    const double *pl = r.pl[t];
    const double den = fma(pl[0], di, fma(pl[1], dj, pl[2]));
    float ch[4];
    for (int k = 0; k < 4; k++)
        ch[k] = (float)(fma(pl[3 + 3 * k], di, fma(pl[4 + 3 * k], dj, pl[5 + 3 * k])) / den);
    return make_float4(ch[3], ch[0], ch[1], ch[2]);
}

struct QuadSetup {
    int32_t hp[18];
    uint32_t bb_i, bb_j, rgba, flags;
    double A, B, C0;
};

// Setup of quad q (Stage 1): writes its snapped vertices, bbox and cull
// reason, leaves the records of a visible quad in r (the caller stores
// them); returns the reason (VISIBLE = 0).
__device__ __forceinline__ uint32_t setup_quad(const FrameArgs &a, uint32_t q, QuadSetup &r)
{
    uint32_t reason = 0xff;
    {
        const uint32_t n = a.n;
        double c[4][3];
        for (int k = 0; k < 4; k++) {
            double d0 = (double)a.v[(k * 3 + 0) * (size_t)n + q] - (double)a.pos[0];
            double d1 = (double)a.v[(k * 3 + 1) * (size_t)n + q] - (double)a.pos[1];
            double d2 = (double)a.v[(k * 3 + 2) * (size_t)n + q] - (double)a.pos[2];
            for (int r = 0; r < 3; r++)
                c[k][r] = fma((double)a.rot[3 * r + 2], d2,
                              fma((double)a.rot[3 * r + 1], d1, (double)a.rot[3 * r + 0] * d0));
        }
        uint2 bb = make_uint2(0xffffu, 0xffffu);
        bool near = false;
        for (int k = 0; k < 4; k++)
            if (!(c[k][2] > (double)a.z_near))
                near = true;
        if (near) {
            reason = NEAR;
        } else {
            double sx[4], sy[4];
            bool guard = false;
            for (int k = 0; k < 4; k++) {
                double qx = c[k][0] / c[k][2];
                double qy = c[k][1] / c[k][2];
                sx[k] = fma(a.f, qx, a.cx);
                sy[k] = fma(-a.f, qy, a.cy);
                if (!(fabs(sx[k]) < 32768.0) || !(fabs(sy[k]) < 32768.0))
                    guard = true;
            }
            if (guard) {
                reason = GUARD;
            } else {
                QuadXY xy;
                for (int k = 0; k < 4; k++) {
                    xy.X[k] = (int32_t)rint(sx[k] * 256.0);
                    xy.Y[k] = (int32_t)rint(sy[k] * 256.0);
                }
                // snapped vertices are kept for the fp64 path of wide quads and
                // for the parity dump
                bool keep_xy = a.want_xy != 0;
                const double X0 = xy.X[0], Y0 = xy.Y[0], X1 = xy.X[1], Y1 = xy.Y[1];
                const double X2 = xy.X[2], Y2 = xy.Y[2], X3 = xy.X[3], Y3 = xy.Y[3];
                const double a0 = edge_fn(X0, Y0, X1, Y1, X2, Y2);
                const double a1 = edge_fn(X0, Y0, X2, Y2, X3, Y3);
                if (a0 == 0.0 && a1 == 0.0) {
                    reason = DEGENERATE;
                } else {
                    // |X|, |Y| < 2^23: 32-bit integer arithmetic is exact here
                    int32_t xmin = xy.X[0], xmax = xy.X[0], ymin = xy.Y[0], ymax = xy.Y[0];
                    for (int k = 1; k < 4; k++) {
                        xmin = min(xmin, xy.X[k]);
                        xmax = max(xmax, xy.X[k]);
                        ymin = min(ymin, xy.Y[k]);
                        ymax = max(ymax, xy.Y[k]);
                    }
                    int32_t imin = (xmin - 128 + 255) >> 8, imax = (xmax - 128) >> 8;
                    int32_t jmin = (ymin - 128 + 255) >> 8, jmax = (ymax - 128) >> 8;
                    imin = max(imin, 0);
                    jmin = max(jmin, 0);
                    imax = min(imax, (int32_t)a.W - 1);
                    jmax = min(jmax, (int32_t)a.H - 1);
                    if (imin > imax || jmin > jmax) {
                        reason = NO_SAMPLE;
                    } else {
                        double e1[3], e2[3], nn[3], m[3];
                        for (int r = 0; r < 3; r++) {
                            e1[r] = c[2][r] - c[0][r];
                            e2[r] = c[3][r] - c[1][r];
                        }
                        {
                            double p, s;
                            p = e1[1] * e2[2]; s = e1[2] * e2[1]; nn[0] = p - s;
                            p = e1[2] * e2[0]; s = e1[0] * e2[2]; nn[1] = p - s;
                            p = e1[0] * e2[1]; s = e1[1] * e2[0]; nn[2] = p - s;
                        }
                        for (int r = 0; r < 3; r++)
                            m[r] = ((c[0][r] + c[1][r]) + (c[2][r] + c[3][r])) * 0.25;
                        double dd = (nn[0] * m[0] + nn[1] * m[1]) + nn[2] * m[2];
                        double g = a.f * dd;
                        double A = nn[0] / g;
                        double B = (-nn[1]) / g;
                        double u0 = ((double)imin + 0.5) - a.cx;
                        double w0 = ((double)jmin + 0.5) - a.cy;
                        double t1 = nn[0] * u0, t2 = nn[1] * w0;
                        double C0 = ((t1 - t2) + nn[2] * a.f) / g;
                        if (dd == 0.0 || !isfinite(dd) || !isfinite(A) || !isfinite(B) ||
                            !isfinite(C0)) {
                            reason = EDGE_ON;
                        } else if (a.cull_back && dd < 0.0) {
                            // facing away: n . m < 0 is clockwise on the display
                            reason = BACKFACE;
                        } else {
                            reason = VISIBLE;
                            uint32_t flags = 0;
                            if (xmax - xmin > kNarrowExtent || ymax - ymin > kNarrowExtent)
                                flags |= kWide;
                            const double Rx = 256.0 * imin + 128.0, Ry = 256.0 * jmin + 128.0;
                            // a narrow strictly convex quad needs its four outer
                            // edges only; the others their triangles' six
                            if (!(flags & kWide))
                                convex_halfplanes(xy.X, xy.Y, Rx, Ry, r.hp, flags);
                            if (flags & kConvex) {
                                for (int k = 12; k < 18; k++)
                                    r.hp[k] = 0;
                            } else {
                                tri_halfplanes(xy.X, xy.Y, 0, 1, 2, Rx, Ry, r.hp, flags, kT0Valid, kT0Swap);
                                tri_halfplanes(xy.X, xy.Y, 0, 2, 3, Rx, Ry, r.hp + 9, flags, kT1Valid,
                                               kT1Swap);
                            }
                            keep_xy = keep_xy || (flags & kWide) != 0;
                            r.bb_i = (uint32_t)imin | ((uint32_t)imax << 16);
                            r.bb_j = (uint32_t)jmin | ((uint32_t)jmax << 16);
                            r.rgba = a.rgba_in[q];
                            r.flags = flags;
                            r.A = A;
                            r.B = B;
                            r.C0 = C0;
                            bb = make_uint2(r.bb_i, r.bb_j);
                            if (a.vcol_in) {
                                vertex_colour_planes(a, q, c, imin, jmin);
                                keep_xy = true;  // the triangle choice reads the snapped vertices
                            }
                        }
                    }
                }
                if (keep_xy)
                    a.xy[q] = xy;
            }
        }
        a.bbox[q] = bb;
        a.cull[q] = (uint8_t)reason;
    }
    return reason;
}

// Quads per lane of the setup kernel (each workgroup takes 256 quads).
constexpr uint32_t kSetupQPL = 1;

// The workgroup's 256 coverage and plane records are contiguous in HBM
// (indexed by quad).  A lane storing its own records would issue stores
// whose lanes sit 64 or 32 bytes apart, partial lines each; instead the
// records are staged in LDS and written as consecutive 16-byte chunks, whole
// lines per group of lanes.  In LDS, chunk c of row t sits at slot c ^ (t &
// (chunks - 1)), so the staging writes of neighbouring rows fall in
// different banks.  Rows of culled quads are written as zeros (nothing reads
// them).  The two extra half-planes of a quad that is not strictly convex
// (rare) are stored by its own lane.
constexpr uint32_t kCovChunks = sizeof(CovRec) / 16;
constexpr uint32_t kPlaneChunks = sizeof(PlaneRec) / 16;

template <class Src>
__global__ __launch_bounds__(256 / kSetupQPL) void k_setup(Src src)
{
    static_assert(kSetupQPL == 1, "record staging assumes one quad per lane");
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    if (a.bin_px) {
        // the density estimate is summed by the binning count that follows
        const uint32_t nblk = (a.n + 255) / 256;
        for (uint32_t b = blk * blockDim.x + threadIdx.x; b < a.nbins; b += nblk * blockDim.x)
            a.bin_px[b] = 0;
    }
    __shared__ uint4 s_cov[256 * kCovChunks];
    __shared__ uint4 s_pl[256 * kPlaneChunks];
    uint32_t reasons[kSetupQPL];
    uint2 my_bb = make_uint2(0xffffu, 0xffffu);  // the lane's pixel bbox (visible quads)
    {
        const uint32_t t = threadIdx.x;
        const uint32_t q = blk * 256 + t;
        QuadSetup r;
        reasons[0] = q < a.n ? setup_quad(a, q, r) : 0xffu;
        if (reasons[0] == VISIBLE)
            my_bb = make_uint2(r.bb_i, r.bb_j);
        uint4 cc[kCovChunks], pc[kPlaneChunks];
        if (reasons[0] == VISIBLE) {
            cc[0] = make_uint4(r.hp[0], r.hp[1], r.hp[2], r.hp[3]);
            cc[1] = make_uint4(r.hp[4], r.hp[5], r.hp[6], r.hp[7]);
            cc[2] = make_uint4(r.hp[8], r.hp[9], r.hp[10], r.hp[11]);
            cc[3] = make_uint4(r.bb_i, r.bb_j, r.flags, r.rgba);
            const unsigned long long ua = __double_as_longlong(r.A);
            const unsigned long long ub = __double_as_longlong(r.B);
            const unsigned long long uc = __double_as_longlong(r.C0);
            pc[0] = make_uint4((uint32_t)ua, (uint32_t)(ua >> 32), (uint32_t)ub, (uint32_t)(ub >> 32));
            pc[1] = make_uint4((uint32_t)uc, (uint32_t)(uc >> 32), (r.bb_i & 0xffffu) | (r.bb_j << 16), r.rgba);
            if (!(r.flags & kConvex)) {
                uint4 *ex = reinterpret_cast<uint4 *>(a.extra + q);
                ex[0] = make_uint4(r.hp[12], r.hp[13], r.hp[14], r.hp[15]);
                ex[1] = make_uint4(r.hp[16], r.hp[17], 0u, 0u);
            }
        } else {
#pragma unroll
            for (uint32_t c = 0; c < kCovChunks; c++)
                cc[c] = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (uint32_t c = 0; c < kPlaneChunks; c++)
                pc[c] = make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (uint32_t c = 0; c < kCovChunks; c++)
            s_cov[t * kCovChunks + (c ^ (t & (kCovChunks - 1)))] = cc[c];
#pragma unroll
        for (uint32_t c = 0; c < kPlaneChunks; c++)
            s_pl[t * kPlaneChunks + (c ^ (t & (kPlaneChunks - 1)))] = pc[c];
    }
    // cull statistics: one atomic per workgroup and reason, striped
    __shared__ uint32_t s_cull[kCullReasons];
    if (threadIdx.x < kCullReasons)
        s_cull[threadIdx.x] = 0;
    __syncthreads();
    {
        const uint32_t q0 = blk * 256;
        const uint32_t rows = q0 < a.n ? min(256u, a.n - q0) : 0u;
        uint4 *dc = reinterpret_cast<uint4 *>(a.cov + q0);
#pragma unroll
        for (uint32_t i = 0; i < kCovChunks; i++) {
            const uint32_t idx = i * 256 + threadIdx.x, row = idx / kCovChunks, c = idx % kCovChunks;
            if (row < rows)
                dc[idx] = s_cov[row * kCovChunks + (c ^ (row & (kCovChunks - 1)))];
        }
        uint4 *dp = reinterpret_cast<uint4 *>(a.plane + q0);
#pragma unroll
        for (uint32_t i = 0; i < kPlaneChunks; i++) {
            const uint32_t idx = i * 256 + threadIdx.x, row = idx / kPlaneChunks, c = idx % kPlaneChunks;
            if (row < rows)
                dp[idx] = s_pl[row * kPlaneChunks + (c ^ (row & (kPlaneChunks - 1)))];
        }
    }
    const uint32_t lane = lane_id();
    if (!a.bbox_binning) {
        // the frame's list of large quads (binned by every binning workgroup)
        const uint32_t q = blk * 256 + threadIdx.x;
        const bool large = reasons[0] == VISIBLE && quad_is_large(my_bb);
        const uint64_t lm = ballot(large);
        uint32_t base = 0;
        if (lane == 0 && lm)
            base = atomicAdd(&a.ctr->n_large, (uint32_t)__popcll(lm));
        base = lane_value(base, 0);
        if (large)
            a.large_list[base + rank_below(lm)] = q;
    }
    for (uint32_t r = 0; r < kCullReasons; r++) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t k = 0; k < kSetupQPL; k++)
            c += (uint32_t)__popcll(ballot(reasons[k] == r));
        if (c && lane == 0)
            atomicAdd(&s_cull[r], c);
    }
    __syncthreads();
    if (threadIdx.x < kCullReasons && s_cull[threadIdx.x])
        add_stat(a.ctr, ST_CULL0 + threadIdx.x, s_cull[threadIdx.x]);
}

// ----------------------------------------------------------------- binning
//
// The quads are split into units of a.unit_quads consecutive indices; one
// wave owns a unit.  Count: a per-unit LDS histogram over bins, written as
// one row of table[unit][bin].  Scan: per bin, an exclusive prefix over
// units (in tiles of 64), then over bins.  Scatter: the same unit walks its
// quads in order and ranks equal bins within each group of 64 pairs with
// ballots, so each bin list ends up in ascending quad index.

__device__ __forceinline__ bool quad_bins(uint2 bb, uint32_t shift, uint32_t &bx0, uint32_t &by0,
                                          uint32_t &bw, uint32_t &np)
{
    uint32_t imin = bb.x & 0xffffu, imax = bb.x >> 16, jmin = bb.y & 0xffffu, jmax = bb.y >> 16;
    if (imin > imax || jmin > jmax) {
        np = 0;
        return false;
    }
    bx0 = imin >> shift;
    by0 = jmin >> shift;
    bw = (imax >> shift) - bx0 + 1;
    np = bw * ((jmax >> shift) - by0 + 1);
    return true;
}

// The rows [r0, r1) of a bin rectangle (bx0, by0, bw wide, np bins): by0
// becomes its first kept row relative to r0, np its kept bins.
__device__ __forceinline__ void clip_rows(uint32_t &by0, uint32_t bw, uint32_t &np, uint32_t r0, uint32_t r1)
{
    if (!np)
        return;
    const uint32_t ya = max(by0, r0), yb = min(by0 + np / bw, r1);
    np = ya < yb ? (yb - ya) * bw : 0u;
    by0 = ya < yb ? ya - r0 : 0u;
}

// Calls f(i, bx, by) for the np bins of a rectangle bw bins wide whose
// first bin is (bx0, by0), row by row (i = by * nbx + bx): steps instead of
// a division per bin.
template <typename F>
__device__ __forceinline__ void for_rect_bins(uint32_t bx0, uint32_t by0, uint32_t bw, uint32_t np, uint32_t nbx,
                                              F &&f)
{
    uint32_t bx = bx0, by = by0, i = by0 * nbx + bx0;
    for (uint32_t j = 0; j < np; j++) {
        f(i, bx, by);
        if (++bx == bx0 + bw) {
            bx = bx0;
            by++;
            i += nbx - bw + 1;
        } else {
            i++;
        }
    }
}

// Groups of 64 quads (and of 64 bins) whose loads a binning wave issues
// together.
constexpr uint32_t kBinPrefetch = 8;

// Pixels of bbox bb inside bin (bx, by): the bin's share of the quad's
// bbox, summed per bin as a depth-complexity estimate.
__device__ __forceinline__ uint32_t bin_overlap_px(uint2 bb, uint32_t bx, uint32_t by, uint32_t shift)
{
    const int x0 = (int)(bx << shift), y0 = (int)(by << shift), s1 = (1 << shift) - 1;
    const int w = min((int)(bb.x >> 16), x0 + s1) - max((int)(bb.x & 0xffffu), x0) + 1;
    const int h = min((int)(bb.y >> 16), y0 + s1) - max((int)(bb.y & 0xffffu), y0) + 1;
    return (uint32_t)(w * h);
}

// ----- large quads (Stage 1, Phase 1 split; Stage 2, "Triangle
// rasterization": bins of a large primitive found by a bin-level scan with
// a trivial-reject test)


// Whether bin (bx, by) may hold a covered sample of the quad: the bin is
// rejected when, for the convex quad or for each of its two triangles, some
// edge stays below its threshold on every pixel centre of the bin inside
// the quad's bbox (a linear function peaks at a corner of that rectangle),
// so no sample there can be covered.  The test is conservative: a kept bin
// may still hold no sample.  Quads on the fp64 coverage path keep every bin.
__device__ __forceinline__ bool bin_maybe_covered(const CovRec &r, const ExtraRec &ex, uint32_t bx, uint32_t by,
                                                  uint32_t shift)
{
    if (r.flags & kWide)
        return true;
    const int imin = (int)(r.bb_i & 0xffffu), imax = (int)(r.bb_i >> 16);
    const int jmin = (int)(r.bb_j & 0xffffu), jmax = (int)(r.bb_j >> 16);
    const int x0 = (int)(bx << shift), y0 = (int)(by << shift), s1 = (1 << shift) - 1;
    const int di0 = max(x0, imin) - imin, di1 = min(x0 + s1, imax) - imin;
    const int dj0 = max(y0, jmin) - jmin, dj1 = min(y0 + s1, jmax) - jmin;
    auto out = [&](int a, int b, int t) { return a * (a >= 0 ? di1 : di0) + b * (b >= 0 ? dj1 : dj0) < t; };
    const int32_t *h = r.hp;
    if (r.flags & kConvex)
        return !(out(h[0], h[1], h[2]) || out(h[3], h[4], h[5]) || out(h[6], h[7], h[8]) ||
                 out(h[9], h[10], h[11]));
    const bool t0 = out(h[0], h[1], h[2]) || out(h[3], h[4], h[5]) || out(h[6], h[7], h[8]);
    const bool t1 = out(h[9], h[10], h[11]) || out(ex.hp[0], ex.hp[1], ex.hp[2]) || out(ex.hp[3], ex.hp[4], ex.hp[5]);
    return !(t0 && t1);
}

// A large quad's records for the bin test (wave-uniform loads).
__device__ __forceinline__ void large_records(const FrameArgs &a, uint32_t q, CovRec &r, ExtraRec &ex)
{
    r = a.cov[q];
    ex = ExtraRec{};
    if (!(r.flags & (kConvex | kWide)))
        ex = a.extra[q];
}

// Counts the kept bins of one large quad q (wave-uniform), its bbox bins
// spread over the lanes; only bins in rows [r0, r1), indexed from row r0.
__device__ __forceinline__ void count_one_large(const FrameArgs &a, uint32_t q, uint32_t *s_hist, uint32_t *s_px,
                                                uint32_t r0 = 0, uint32_t r1 = 0xFFFFu)
{
    const uint32_t lane = lane_id();
    const uint2 bb = a.bbox[q];
    CovRec r;
    ExtraRec ex;
    large_records(a, q, r, ex);
    uint32_t bx0, by0, bw, np;
    quad_bins(bb, a.bin_shift, bx0, by0, bw, np);
    clip_rows(by0, bw, np, r0, r1);
    for (uint32_t j = lane; j < np; j += 64) {
        const uint32_t by = by0 + j / bw, bx = bx0 + j % bw;
        if (bin_maybe_covered(r, ex, bx, by + r0, a.bin_shift)) {
            atomicAdd(&s_hist[by * a.nbx + bx], 1u);
            if (s_px)
                atomicAdd(&s_px[by * a.nbx + bx], bin_overlap_px(bb, bx, by + r0, a.bin_shift));
        }
    }
}

// Calls f(q) for the large quads that wave w (of nw) of binning unit u
// takes: list entries u + nunits * (w + nw * m), so they spread over every
// unit whatever their indices (the count and the scatter take the same).
template <typename F>
__device__ __forceinline__ void for_large_share(const FrameArgs &a, uint32_t u, uint32_t w, uint32_t nw, F &&f)
{
    if (a.bbox_binning)
        return;
    const uint32_t nl = uniform(a.ctr->n_large);
    for (uint32_t i = u + a.nunits * w; i < nl; i += a.nunits * nw)
        f(uniform(a.large_list[i]));
}

template <class Src>
__global__ __launch_bounds__(64) void k_bin_count(Src src)
{
    extern __shared__ uint32_t s_hist[];
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    const uint2 *__restrict__ bbox = a.bbox;
    const uint32_t lane = threadIdx.x, u = blk;
    for (uint32_t b = lane; b < a.nbins; b += 64)
        s_hist[b] = 0;
    __syncthreads();
    const uint32_t q0 = u * a.unit_quads, q1 = min(q0 + a.unit_quads, a.n);
    // bboxes of 8 groups of 64 quads are loaded before any is used
    for (uint32_t base = q0; base < q1; base += 64 * kBinPrefetch) {
        uint2 bb[kBinPrefetch];
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const uint32_t q = base + 64 * k + lane;
            bb[k] = q < q1 ? bbox[q] : make_uint2(0xffffu, 0xffffu);  // (0xffff, 0xffff): no pixel
        }
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const bool large = !a.bbox_binning && quad_is_large(bb[k]);  // binned from the large list
            uint32_t bx0, by0, bw, np;
            if (!large && quad_bins(bb[k], a.bin_shift, bx0, by0, bw, np))
                for_rect_bins(bx0, by0, bw, np, a.nbx, [&](uint32_t i, uint32_t, uint32_t) { atomicAdd(&s_hist[i], 1u); });
        }
    }
    for_large_share(a, u, 0, 1, [&](uint32_t q) { count_one_large(a, q, s_hist, nullptr); });
    __syncthreads();
    uint32_t *row = a.table + (size_t)u * a.nbins;
    for (uint32_t b = lane; b < a.nbins; b += 64)
        row[b] = s_hist[b];
}

// Workgroups of the bin scan: one per group of 64 bins.
__host__ __device__ __forceinline__ uint32_t scan_groups(uint32_t nbins) { return (nbins + 63) / 64; }

// Bin scan over units.  A workgroup owns 64 bins (one per lane) and walks
// their whole columns of table[u][b]; its 16 waves split the units.  Pass 1
// sums each wave's share, each lane adds up the shares of the waves before
// its own for its base, and pass 2 rewrites the column as exclusive prefixes
// over units; the column total is the bin's count.  (The prefix over bins is
// taken by the scatter, which needs it first.)
constexpr uint32_t kScanWaves = 16;

// Column values a lane keeps in registers between the two passes (when its
// wave's share of the units is no longer, pass 2 reads nothing again).
constexpr uint32_t kScanKeep = 32;

template <class Src>
__global__ __launch_bounds__(kScanWaves * 64) void k_bin_scan(Src src)
{
    __shared__ uint32_t s_share[kScanWaves][64];
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const uint32_t b = blk * 64 + lane;
    const bool on = b < a.nbins;
    const uint32_t per = (a.nunits + kScanWaves - 1) / kScanWaves;
    const uint32_t u0 = min(wave * per, a.nunits), u1 = min(u0 + per, a.nunits);
    const bool kept = per <= kScanKeep;
    uint32_t keep[kScanKeep];
    uint32_t sum = 0;
    if (on) {
        if (kept) {
#pragma unroll
            for (uint32_t k = 0; k < kScanKeep; k++)
                keep[k] = (u0 + k < u1) ? a.table[(size_t)(u0 + k) * a.nbins + b] : 0u;
#pragma unroll
            for (uint32_t k = 0; k < kScanKeep; k++)
                sum += keep[k];
        } else {
            // loads of a group are issued before they are summed
            for (uint32_t g = u0; g < u1; g += 16) {
                uint32_t v[16];
#pragma unroll
                for (int k = 0; k < 16; k++)
                    v[k] = (g + k < u1) ? a.table[(size_t)(g + k) * a.nbins + b] : 0;
#pragma unroll
                for (int k = 0; k < 16; k++)
                    sum += v[k];
            }
        }
    }
    s_share[wave][lane] = sum;
    __syncthreads();
    // this wave's base: the shares of the waves before it; the total is the
    // bin's count
    uint32_t run = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kScanWaves; w++) {
        const uint32_t v = s_share[w][lane];
        run += w < wave ? v : 0u;
        total += v;
    }
    if (wave == 0) {
        if (on)
            a.bin_count[b] = total;
        if (a.k_low) {
            // density class by the depth estimate; dense bins go to the
            // list the raster takes first (one atomic per workgroup)
            bool high = false;
            if (on) {
                const uint32_t bx = b % a.nbx, by = b / a.nbx;
                const uint32_t w = min(a.W - (bx << a.bin_shift), 1u << a.bin_shift);
                const uint32_t h = min(a.H - (by << a.bin_shift), 1u << a.bin_shift);
                const unsigned long long px = a.bin_px[b], area = (unsigned long long)w * h;
                high = px > kDenseDepth * area;
                a.bin_class[b] = high ? kDense : (px > kSparseDepth * area ? kMid : kSparse);
            }
            const uint64_t hm = ballot(high);
            uint32_t base = 0;
            if (lane == 0 && hm)
                base = atomicAdd(&a.ctr->n_high, (uint32_t)__popcll(hm));
            base = lane_value(base, 0);
            if (high)
                a.high_list[base + rank_below(hm)] = b;
        }
    }
    if (on) {
        if (kept) {
#pragma unroll
            for (uint32_t k = 0; k < kScanKeep; k++) {
                if (u0 + k < u1)
                    a.table[(size_t)(u0 + k) * a.nbins + b] = run;
                run += keep[k];
            }
        } else {
            for (uint32_t g = u0; g < u1; g += 16) {
                uint32_t v[16];
#pragma unroll
                for (int k = 0; k < 16; k++)
                    v[k] = (g + k < u1) ? a.table[(size_t)(g + k) * a.nbins + b] : 0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (g + k < u1)
                        a.table[(size_t)(g + k) * a.nbins + b] = run;
                    run += v[k];
                }
            }
        }
    }
}

// Zeroes the next frame's counter set (single frames), spread over the
// calling kernel's workgroups.
__device__ __forceinline__ void clear_next_counters(const FrameArgs &a, uint32_t blk, uint32_t nblk)
{
    if (!a.ctr_next)
        return;
    uint4 *p = reinterpret_cast<uint4 *>(a.ctr_next);
    const uint32_t n = sizeof(FrameCounters) / 16;
    for (uint32_t i = blk * blockDim.x + threadIdx.x; i < n; i += nblk * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

// Quads whose bboxes the scatter stages in LDS at a time: all loads of a
// group are issued before its stores, so no wait for earlier stores (loads
// and stores share one completion counter) sits inside the scatter loop.
constexpr uint32_t kScatterGroup = 512;

// Scatters the pairs of one group of 64 consecutive quads (lane l holds the
// bbox of quad base + l) into their bin lists, 64 pairs at a time: the
// group's pairs are numbered quad by quad (exclusive prefix of the pair
// counts), each quad's lane marks the window slots of its own pairs, and
// each lane then takes the pair of its slot; lanes whose pairs share a bin
// take consecutive slots in lane order from one LDS atomic on offs[bin], so
// every bin list stays in ascending quad order.
__device__ __forceinline__ void scatter_small(const FrameArgs &a, uint2 cur, uint32_t base, uint32_t *offs,
                                              uint32_t *s_pref, uint32_t (*s_rect)[3], uint32_t *s_own, uint32_t lane,
                                              uint32_t lo_lane, uint32_t hi_lane, uint32_t r0, uint32_t r1)
{
    // bits that tell the band's bins apart
    const uint32_t rows = min(r1, a.nby) - r0;
    const uint32_t mbits = rows * a.nbx > 1 ? 32u - (uint32_t)__builtin_clz(rows * a.nbx - 1) : 1u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t bx0 = 0, by0 = 0, bw = 1, np = 0;
    quad_bins(cur, a.bin_shift, bx0, by0, bw, np);
    clip_rows(by0, bw, np, r0, r1);  // bins of the band, rows from r0
    if (lane < lo_lane || lane >= hi_lane)
        np = 0;  // lanes of this run only
    // exclusive prefix of np over the wave: the chunk's pair pre .. pre + np - 1
    // belong to this lane's quad
    const uint32_t incl = wave_incl_scan(np);
    const uint32_t total = lane_value(incl, 63), pre = incl - np;
    s_pref[lane] = pre;
    s_rect[lane][0] = bx0;
    s_rect[lane][1] = by0;
    s_rect[lane][2] = bw;
    for (uint32_t w = 0; w < total; w += 64) {
        // owners of the window's 64 pairs, marked by the quads' lanes
        for (uint32_t p = max(pre, w); p < min(pre + np, w + 64); p++)
            s_own[p - w] = lane;
        wave_sync();
        const uint32_t p = w + lane;
        const bool valid = p < total;
        uint32_t bin = 0, qv = 0;
        if (valid) {
            const uint32_t lo = s_own[lane];
            const uint32_t k = p - s_pref[lo];
            const uint32_t rbw = s_rect[lo][2];
            bin = (s_rect[lo][1] + k / rbw) * a.nbx + s_rect[lo][0] + k % rbw;
            qv = base + lo;
        }
        // lanes holding the same bin: AND over the bits of the bin index
        uint64_t peers = ballot(valid);
        for (uint32_t bit = 0; bit < mbits; bit++) {
            const bool set = (bin >> bit) & 1u;
            const uint64_t bm = ballot(set);
            peers &= set ? bm : ~bm;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t leader = peers ? (uint32_t)__builtin_ctzll(peers) : lane;
        uint32_t base_off = 0;
        if (valid && rank == 0)
            base_off = atomicAdd(&offs[bin], (uint32_t)__popcll(peers));
        // every lane reads its group leader's base offset
        const uint32_t pos = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(leader << 2), (int)base_off) + rank;
        if (valid && pos < a.pair_cap)
            a.pairs[pos] = qv;
        wave_sync();  // the window's owners are read before the next window marks its own
    }
    wave_sync();
}

// Places the kept bins of one large quad q (bbox bb), its bbox bins spread
// over the lanes; every lane holds a different bin, so each takes its slot
// with one LDS atomic.
__device__ __forceinline__ void scatter_large(const FrameArgs &a, uint32_t q, uint2 bb, uint32_t *offs, uint32_t lane,
                                              uint32_t r0, uint32_t r1)
{
    CovRec r;
    ExtraRec ex;
    large_records(a, q, r, ex);
    uint32_t bx0, by0, bw, np;
    quad_bins(bb, a.bin_shift, bx0, by0, bw, np);
    clip_rows(by0, bw, np, r0, r1);  // bins of the band, rows from r0
    for (uint32_t j = lane; j < np; j += 64) {
        const uint32_t by = by0 + j / bw, bx = bx0 + j % bw;
        if (bin_maybe_covered(r, ex, bx, by + r0, a.bin_shift)) {
            const uint32_t pos = atomicAdd(&offs[by * a.nbx + bx], 1u);
            if (pos < a.pair_cap)
                a.pairs[pos] = q;
        }
    }
    wave_sync();
}

// The pairs of 64 consecutive quads (lane l holds the bbox of quad base +
// l); large quads are left to the large list.
__device__ __forceinline__ void scatter_chunk(const FrameArgs &a, uint2 cur, uint32_t base, uint32_t *offs,
                                              uint32_t *s_pref, uint32_t (*s_rect)[3], uint32_t *s_own, uint32_t lane,
                                              uint32_t r0 = 0, uint32_t r1 = 0xFFFFu)
{
    const bool large = !a.bbox_binning && quad_is_large(cur);
    scatter_small(a, large ? make_uint2(0xffffu, 0xffffu) : cur, base, offs, s_pref, s_rect, s_own, lane, 0u, 64u, r0,
                  r1);
}

// Publishes a frame's bin offsets (bin_start) and total, and logs a
// capacity overflow; done by the first scatter workgroup.
__device__ __forceinline__ void publish_total(const FrameArgs &a, uint32_t total)
{
    a.bin_start[a.nbins] = total;
    a.ctr->pairs_total = total;
    if (total > a.pair_cap) {
        a.ctr->error |= kErrPairs;
        const uint32_t i = atomicAdd(&a.elog->n, 1u);
        if (i < kErrLogCap) {
            a.elog->e[i].tag = a.tag;
            a.elog->e[i].pairs = total;
        }
    }
}

template <class Src>
__global__ __launch_bounds__(64) void k_bin_scatter(Src src)
{
    extern __shared__ uint32_t s_off[];
    __shared__ uint32_t s_pref[64];
    __shared__ uint32_t s_rect[64][3];
    __shared__ uint32_t s_own[64];
    __shared__ uint2 s_bb[kScatterGroup];
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    const uint2 *__restrict__ bbox = a.bbox;
    const uint32_t lane = threadIdx.x, u = blk;
    const uint32_t *row = a.table + (size_t)u * a.nbins;
    // every workgroup takes the exclusive prefix over the bin counts itself
    // (the first one also publishes it as bin_start); its offset in bin b is
    // that plus its own row of the scanned table
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < a.nbins; b0 += 64 * kBinPrefetch) {
        uint32_t c[kBinPrefetch], r[kBinPrefetch];
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const uint32_t b = b0 + 64 * k + lane;
            c[k] = b < a.nbins ? a.bin_count[b] : 0;
            r[k] = b < a.nbins ? row[b] : 0;
        }
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const uint32_t b = b0 + 64 * k + lane;
            const uint32_t incl = wave_incl_scan(c[k]);
            const uint32_t start = carry + incl - c[k];
            carry += lane_value(incl, 63);
            if (b < a.nbins) {
                s_off[b] = start + r[k];
                if (u == 0)
                    a.bin_start[b] = start;
            }
        }
    }
    if (u == 0 && lane == 0)
        publish_total(a, carry);
    wave_sync();  // one wave per workgroup
    const uint32_t q0 = u * a.unit_quads, q1 = min(q0 + a.unit_quads, a.n);
    for (uint32_t base = q0; base < q1; base += 64) {
        const uint32_t q = base + lane;
        if ((base - q0) % kScatterGroup == 0) {
            uint2 bb[kScatterGroup / 64];
#pragma unroll
            for (uint32_t k = 0; k < kScatterGroup / 64; k++) {
                const uint32_t qq = base + 64 * k + lane;
                bb[k] = make_uint2(0xffffu, 0xffffu);  // no pixel
                if (qq < q1)
                    bb[k] = bbox[qq];
            }
#pragma unroll
            for (uint32_t k = 0; k < kScatterGroup / 64; k++)
                s_bb[64 * k + lane] = bb[k];
            wave_sync();
        }
        scatter_chunk(a, s_bb[(base - q0) % kScatterGroup + lane], base, s_off, s_pref, s_rect, s_own, lane);
        wave_sync();  // one wave per workgroup
    }
    for_large_share(a, u, 0, 1, [&](uint32_t q) { scatter_large(a, q, bbox[q], s_off, lane, 0u, 0xFFFFu); });
}


// Binning with four waves per unit (frames of at most kBin4MaxBins bins).
// Count: the unit's quads are split over 1,024 lanes into one LDS
// histogram.  Scatter: one workgroup per unit and band of bin rows; wave w
// takes the w-th quarter of the unit and counts its pairs in the band into
// its own histogram; the bin's start (a prefix over the bin counts each
// workgroup takes), the unit's scanned table entry and a per-bin prefix
// over the four quarters give each wave
// its own offsets, so the quarters scatter concurrently and every bin list
// still comes out in ascending quad order.
constexpr uint32_t kBin4MaxBins = 8192;  // the count's histogram: 32 KiB
constexpr uint32_t kBin4Waves = 4;
// The count's workgroup: sixteen waves share the histogram of a unit of
// 2048 quads or more (each lane counts a few of them instead of up to
// sixteen), four waves that of a smaller unit (more workgroups per CU).
__host__ __device__ constexpr uint32_t count4_waves(uint32_t unit_quads) { return unit_quads >= 2048 ? 16u : 4u; }

template <class Src, uint32_t NW>
__global__ __launch_bounds__(NW * 64) void k_bin_count4(Src src)
{
    extern __shared__ uint32_t s_hist[];  // [nbins] counts, then [nbins] overlap pixels when gathered
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    const uint2 *__restrict__ bbox = a.bbox;
    const uint32_t t = threadIdx.x, u = blk;
    const bool px = a.bin_px != nullptr;
    uint32_t *s_px = s_hist + a.nbins;
    for (uint32_t b = t; b < a.nbins; b += NW * 64) {
        s_hist[b] = 0;
        if (px)
            s_px[b] = 0;
    }
    __syncthreads();
    const uint32_t q0 = u * a.unit_quads, q1 = min(q0 + a.unit_quads, a.n);
    for (uint32_t base = q0; base < q1; base += NW * 64 * kBinPrefetch) {
        uint2 bb[kBinPrefetch];
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const uint32_t q = base + NW * 64 * k + t;
            bb[k] = make_uint2(0xffffu, 0xffffu);  // no pixel
            if (q < q1)
                bb[k] = bbox[q];
        }
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const bool large = !a.bbox_binning && quad_is_large(bb[k]);  // binned from the large list
            uint32_t bx0, by0, bw, np;
            if (!large && quad_bins(bb[k], a.bin_shift, bx0, by0, bw, np)) {
                for_rect_bins(bx0, by0, bw, np, a.nbx, [&](uint32_t i, uint32_t bx, uint32_t by) {
                    atomicAdd(&s_hist[i], 1u);
                    if (px)
                        atomicAdd(&s_px[i], bin_overlap_px(bb[k], bx, by, a.bin_shift));
                });
            }
        }
    }
    for_large_share(a, u, t >> 6, NW,
                    [&](uint32_t q) { count_one_large(a, q, s_hist, px ? s_px : nullptr); });
    __syncthreads();
    uint32_t *row = a.table + (size_t)u * a.nbins;
    for (uint32_t b = t; b < a.nbins; b += NW * 64) {
        row[b] = s_hist[b];
        if (px && s_px[b])
            atomicAdd(&a.bin_px[b], (unsigned long long)s_px[b]);
    }
}

// Workgroups are dispatched to the eight XCDs in turn (workgroup i to XCD
// i mod 8).  xcd_order(i, n) numbers the n workgroups of a launch XCD by
// XCD instead: the ones XCD 0 receives get 0 .. n0 - 1, XCD 1's the next,
// and so on -- a bijection of [0, n), so consecutive indices share an XCD
// and its L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_order(uint32_t i, uint32_t n)
{
    const uint32_t k = i % kXcds, j = i / kXcds, q = n / kXcds, r = n % kXcds;
    return k < r ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j;
}

template <class Src>
__device__ __forceinline__ constexpr bool is_one_frame() { return false; }
template <>
__device__ __forceinline__ constexpr bool is_one_frame<OneFrame>() { return true; }

// Groups of 64 quads whose bboxes a scatter wave loads into registers at
// once: with loads and stores counted by one completion counter, a load
// inside the scatter loop would also wait for every scattered store before
// it, so all loads of a run of groups are issued up front.
constexpr uint32_t kScatterRegGroups = 16;

// bb[k] = bbox of quad c0 + 64 k + lane (no pixel past w1).
__device__ __forceinline__ void load_groups(const uint2 *__restrict__ bbox, uint32_t c0, uint32_t w1, uint32_t lane,
                                            uint2 (&bb)[kScatterRegGroups])
{
#pragma unroll
    for (uint32_t k = 0; k < kScatterRegGroups; k++) {
        const uint32_t q = c0 + 64 * k + lane;
        bb[k] = make_uint2(0xffffu, 0xffffu);
        if (q < w1)
            bb[k] = bbox[q];
    }
}

// Moves group k + 1 to bb[k]: the group in hand is always bb[0], so the
// loops over groups index the array statically (register moves, no dynamic
// register indexing).
__device__ __forceinline__ void shift_groups(uint2 (&bb)[kScatterRegGroups])
{
#pragma unroll
    for (uint32_t k = 0; k + 1 < kScatterRegGroups; k++)
        bb[k] = bb[k + 1];
}

template <class Src>
__global__ __launch_bounds__(kBin4Waves * 64) void k_bin_scatter4(Src src)
{
    extern __shared__ uint32_t s_offs[];  // [kBin4Waves][bins of the band]
    __shared__ uint32_t s_pref[kBin4Waves][64];
    __shared__ uint32_t s_rect[kBin4Waves][64][3];
    __shared__ uint32_t s_own[kBin4Waves][64];
    __shared__ uint32_t s_part[2][kBin4Waves];
    uint32_t blk;
    const FrameArgs &a = *frame_of(src, blk);
    const uint2 *__restrict__ bbox = a.bbox;
    const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63;
    // workgroup = (unit u, band h of bin rows r0 .. r1 - 1)
    const uint32_t nb = scatter_bands(a.nbx, a.nby), rows = (a.nby + nb - 1) / nb;
    // consecutive units of a band on one XCD (single frames): their runs in
    // each bin list are adjacent, so that XCD's L2 merges their scattered
    // 4-byte stores into whole lines
    const uint32_t v = is_one_frame<Src>() ? xcd_order(blk, a.nunits * nb) : blk;
    const uint32_t u = v % a.nunits, h = v / a.nunits;
    const uint32_t r0 = min(h * rows, a.nby), r1 = min(r0 + rows, a.nby);
    const uint32_t b0 = r0 * a.nbx, nbins = (r1 - r0) * a.nbx;  // the band's bins: b0 .. b0 + nbins - 1
    uint32_t *offs = s_offs + wave * nbins;
    // this wave's quarter of the unit, in groups of 64 quads
    const uint32_t q0 = u * a.unit_quads, q1 = min(q0 + a.unit_quads, a.n);
    const uint32_t per = (a.unit_quads / kBin4Waves + 63) / 64 * 64;
    const uint32_t w0 = min(q0 + wave * per, q1), w1 = min(w0 + per, q1);
    for (uint32_t b = lane; b < nbins; b += 64)
        offs[b] = 0;
    wave_sync();
    for (uint32_t c0 = w0; c0 < w1; c0 += 64 * kScatterRegGroups) {
        uint2 bb[kScatterRegGroups];
        load_groups(bbox, c0, w1, lane, bb);
        // the same pairs as the count kernel, in the band: bbox bins of the
        // small quads, then the kept bins of this wave's share of the large
        // list
        for (uint32_t base = c0; base < min(c0 + 64 * kScatterRegGroups, w1); base += 64) {
            const bool large = !a.bbox_binning && quad_is_large(bb[0]);
            uint32_t bx0, by0, bw, np;
            if (!large && quad_bins(bb[0], a.bin_shift, bx0, by0, bw, np)) {
                clip_rows(by0, bw, np, r0, r1);
                for_rect_bins(bx0, by0, bw, np, a.nbx, [&](uint32_t i, uint32_t, uint32_t) { atomicAdd(&offs[i], 1u); });
            }
            shift_groups(bb);
        }
    }
    for_large_share(a, u, wave, kBin4Waves, [&](uint32_t q) { count_one_large(a, q, offs, nullptr, r0, r1); });
    __syncthreads();
    // the bins before the band: their total is where the band's lists start
    uint32_t before = 0;
    for (uint32_t c0 = 0; c0 < b0; c0 += kBin4Waves * 64 * kBinPrefetch) {
        uint32_t c[kBinPrefetch];
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const uint32_t b = c0 + kBin4Waves * 64 * k + t;
            c[k] = b < b0 ? a.bin_count[b] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++)
            before += c[k];
    }
    before = lane_value(wave_incl_scan(before), 63);
    if (lane == 0)
        s_part[1][wave] = before;
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kBin4Waves; w++)
        total += s_part[1][w];
    // exclusive prefix over the band's bins, 256 consecutive bins per step:
    // the lanes of a wave touch consecutive LDS words, so the per-wave offset
    // rows are read and rewritten without bank conflicts; the first unit
    // also publishes bin_start
    const uint32_t *row = a.table + (size_t)u * a.nbins;
    uint32_t step = 0;
    for (uint32_t c0 = 0; c0 < nbins; c0 += kBin4Waves * 64 * kBinPrefetch) {
        uint32_t c[kBinPrefetch], r[kBinPrefetch];
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++) {
            const uint32_t b = c0 + kBin4Waves * 64 * k + t;
            c[k] = b < nbins ? a.bin_count[b0 + b] : 0u;
            r[k] = b < nbins ? row[b0 + b] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kBinPrefetch; k++, step++) {
            const uint32_t b = c0 + kBin4Waves * 64 * k + t;
            if (c0 + kBin4Waves * 64 * k >= nbins)
                break;
            // wave sums go to alternating rows (the row above was read before
            // the barrier ending the previous step): a row is rewritten two
            // steps later, after every wave has passed the barrier in between
            const uint32_t incl = wave_incl_scan(c[k]);
            if (lane == 63)
                s_part[step & 1][wave] = incl;
            __syncthreads();
            uint32_t start = total + incl - c[k];
#pragma unroll
            for (uint32_t w = 0; w < kBin4Waves; w++) {
                const uint32_t ws = s_part[step & 1][w];
                start += w < wave ? ws : 0u;
                total += ws;
            }
            if (b < nbins) {
                if (u == 0)
                    a.bin_start[b0 + b] = start;
                uint32_t run = start + r[k];
#pragma unroll
                for (uint32_t w = 0; w < kBin4Waves; w++) {
                    const uint32_t cw = s_offs[w * nbins + b];
                    s_offs[w * nbins + b] = run;
                    run += cw;
                }
            }
        }
    }
    // the last band ends at the last row: its total is the frame's
    if (u == 0 && h == nb - 1 && t == 0)
        publish_total(a, total);
    __syncthreads();
    for (uint32_t c0 = w0; c0 < w1; c0 += 64 * kScatterRegGroups) {
        uint2 bb[kScatterRegGroups];
        load_groups(bbox, c0, w1, lane, bb);
        for (uint32_t base = c0; base < min(c0 + 64 * kScatterRegGroups, w1); base += 64) {
            scatter_chunk(a, bb[0], base, offs, s_pref[wave], s_rect[wave], s_own[wave], lane, r0, r1);
            shift_groups(bb);
        }
    }
    for_large_share(a, u, wave, kBin4Waves, [&](uint32_t q) { scatter_large(a, q, bbox[q], offs, lane, r0, r1); });
}

// ------------------------------------------------------------------ raster
//
// One workgroup per bin (Stage 3: a workgroup rasterizes a bin, its
// subgroups work on blocks).  Each wave owns one 8x8 block at a time.  The
// bin's quad list is read in chunks shared by the workgroup; each wave picks
// from a chunk, by ballot, the quads whose bbox meets its block and gathers
// them into batches of 64.  A batch is processed one candidate per lane:
// gather the quad's record, build its 64-sample coverage mask of the block,
// keep the non-empty ones.

// Exact coverage of the quad's triangle pair at pixel (px, py) with fp64
// edge functions (all products stay below 2^50).  For quads wider than
// kNarrowExtent.
__device__ bool wide_covers(uint32_t flags, const QuadXY &xy, int px, int py)
{
    const double Sx = 256.0 * (double)px + 128.0, Sy = 256.0 * (double)py + 128.0;
    bool in = false;
    for (int T = 0; T < 2; T++) {
        const uint32_t vb = T ? kT1Valid : kT0Valid, sb = T ? kT1Swap : kT0Swap;
        if (!(flags & vb))
            continue;
        int ib = T ? 2 : 1, ic = T ? 3 : 2;
        if (flags & sb) {
            int t = ib;
            ib = ic;
            ic = t;
        }
        const int idx[3] = {0, ib, ic};
        bool inside = true;
        for (int e = 0; e < 3; e++) {
            const int s = idx[e], t = idx[(e + 1) % 3];
            const double dx = (double)xy.X[t] - (double)xy.X[s];
            const double dy = (double)xy.Y[t] - (double)xy.Y[s];
            const double E = dx * (Sy - (double)xy.Y[s]) - dy * (Sx - (double)xy.X[s]);
            const bool tl = (dy < 0.0) || (dy == 0.0 && dx > 0.0);
            if (!(E > 0.0 || (E == 0.0 && tl)))
                inside = false;
        }
        in = in || inside;
    }
    return in;
}

// The same for a wide quad (rare): per sample, out of line.
__device__ __noinline__ uint64_t wide_block_mask(uint32_t flags, QuadXY xy, int px0, int py0)
{
    uint64_t m = 0;
#pragma unroll 1
    for (int k = 0; k < 64; k++)
        if (wide_covers(flags, xy, px0 + (k & 7), py0 + (k >> 3)))
            m |= 1ull << k;
    return m;
}

// Sign bits of edge values shifted into an accumulator: (acc << 1) | (v >> 31).
__device__ __forceinline__ uint32_t shift_in_sign(uint32_t acc, int v)
{
    return __builtin_amdgcn_alignbit(acc, (uint32_t)v, 31);
}

// Coverage of one 8-sample row by a narrow quad, exact under the top-left
// rule: e[h] holds the integer edge value E = a*di + b*dj - t of half-plane
// h at the row's last sample (x = 7) and a[h] its step in x; the values are
// stepped from x = 7 down so the sign bits land in order, bit x set when
// the sample is inside (E >= 0 on every edge of a convex quad's four, or of
// one of the two triangles' three).  |a*di + b*dj| < 2^30 and |t| < 2^30
// for narrow quads, so E never overflows.
template <int NE>
__device__ __forceinline__ uint32_t row_walk(const int *a, const int *e0)
{
    int e[NE];
#pragma unroll
    for (int h = 0; h < NE; h++)
        e[h] = e0[h];
    uint32_t bits = 0;
#pragma unroll
    for (int x = 0; x < 8; x++) {
        if constexpr (NE == 4) {
            bits = shift_in_sign(bits, e[0] | e[1] | e[2] | e[3]);  // 1: outside some edge
            asm volatile("" : "+v"(e[0]), "+v"(e[1]), "+v"(e[2]), "+v"(e[3]));
        } else {
            // outside iff both triangles have a negative edge value
            bits = shift_in_sign(bits, (e[0] | e[1] | e[2]) & (e[3] | e[4] | e[5]));
            asm volatile("" : "+v"(e[0]), "+v"(e[1]), "+v"(e[2]), "+v"(e[3]), "+v"(e[4]), "+v"(e[5]));
        }
#pragma unroll
        for (int h = 0; h < NE; h++)
            e[h] -= a[h];
    }
    return ~bits & 0xffu;
}

// A wave's scratch for the coverage masks of one batch.
struct RowWork {
    uint16_t item[512];           // (candidate << 3) | row, candidate by candidate
    unsigned long long mask[64];  // candidate masks, filled one row byte at a time
};

__device__ __forceinline__ int lane_int(int v, uint32_t src_lane)
{
    return __builtin_amdgcn_ds_bpermute((int)(src_lane << 2), v);
}

// Row passes up to which a batch spreads its rows over the lanes; denser
// batches (large quads, most rows covered) walk eight rows per candidate.
constexpr uint32_t kRowPasses = 4;

// Coverage masks of a batch of candidates (lanes with `has`: quad q, its
// record r already in registers) over the 8x8 block at (px0, py0), bit
// 8y + x for pixel (px0 + x, py0 + y).
// Only the rows that a candidate's bbox meets can be covered.  When those
// (candidate, row) pairs fill at most kRowPasses waves' worth, they are
// listed and spread over the lanes, one row walk each, with each
// candidate's edge values fetched from its own lane; otherwise every
// candidate's lane walks the eight rows itself.  The four edges of a convex
// quad stay in registers; the two more of a triangle pair (rare) are read
// again from its record.  A wide quad (rarer) is done sample by sample by
// its own lane.  Returns this lane's mask.
__device__ __forceinline__ uint64_t batch_masks(const CovRec &r, bool has, const ExtraRec *__restrict__ extra,
                                                const QuadXY *__restrict__ xyp, uint32_t q, RowWork &W, int px0,
                                                int py0, uint32_t lane)
{
    // candidate lane: per edge h < 4 the step a, the row step b and the value
    // at (x = 7, y = 0) of the block; di, dj of that sample
    int ca[4] = {0, 0, 0, 0}, cb[4] = {0, 0, 0, 0}, cv[4] = {0, 0, 0, 0};
    int di = 0, dj = 0;
    uint32_t nr = 0, y0 = 0, cvx = 1;
    bool wide = false;
    if (has) {
        wide = (r.flags & kWide) != 0;
        cvx = (r.flags & kConvex) ? 1u : 0u;
        if (!wide) {
            di = px0 + 7 - (int)(r.bb_i & 0xffffu);
            dj = py0 - (int)(r.bb_j & 0xffffu);
#pragma unroll
            for (int h = 0; h < 4; h++) {
                ca[h] = r.hp[3 * h];
                cb[h] = r.hp[3 * h + 1];
                cv[h] = ca[h] * di + cb[h] * dj - r.hp[3 * h + 2];
            }
            // the bbox meets the block, so rows y0..y1 are within 0..7
            const int y1 = min((int)(r.bb_j >> 16) - py0, 7);
            y0 = (uint32_t)max(-dj, 0);
            nr = y1 >= (int)y0 ? (uint32_t)y1 - y0 + 1 : 0u;
        }
    }
    // exclusive prefix of the row counts (at most 8: four bit planes)
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        const uint64_t bm = ballot(((nr >> b) & 1u) != 0);
        pre += rank_below(bm) << b;
        tot += (uint32_t)__popcll(bm) << b;
    }
    const bool any6 = ballot(nr != 0 && !cvx) != 0;
    uint64_t mk = 0;
    if (tot > kRowPasses * 64) {
        if (nr) {
            int a6[6], b6[6], v6[6];
#pragma unroll
            for (int h = 0; h < 4; h++) {
                a6[h] = ca[h];
                b6[h] = cb[h];
                v6[h] = cv[h];
            }
            a6[4] = a6[5] = b6[4] = b6[5] = v6[4] = v6[5] = 0;
            if (!cvx) {
                const int *hp = extra[q].hp;
#pragma unroll
                for (int h = 4; h < 6; h++) {
                    a6[h] = hp[3 * h - 12];
                    b6[h] = hp[3 * h - 11];
                    v6[h] = a6[h] * di + b6[h] * dj - hp[3 * h - 10];
                }
            }
            uint32_t lo = 0, hi = 0;
#pragma unroll 1
            for (uint32_t y = 0; y < 8; y++) {
                int e[6];
#pragma unroll
                for (int h = 0; h < 6; h++)
                    e[h] = v6[h] + b6[h] * (int)y;
                const uint32_t bits = cvx ? row_walk<4>(a6, e) : row_walk<6>(a6, e);
                if (y < 4)
                    lo |= bits << (8 * y);
                else
                    hi |= bits << (8 * (y - 4));
            }
            mk = (uint64_t)lo | ((uint64_t)hi << 32);
        }
    } else if (tot) {
        if (nr)
            W.mask[lane] = 0;
        for (uint32_t k = 0; k < nr; k++)
            W.item[pre + k] = (uint16_t)((lane << 3) | (y0 + k));
        wave_sync();
        uint8_t *rows = reinterpret_cast<uint8_t *>(W.mask);
        for (uint32_t base = 0; base < tot; base += 64) {
            const uint32_t i = base + lane;
            const uint32_t it = i < tot ? W.item[i] : 0u, c = it >> 3, y = it & 7u;
            // every lane takes part in the fetches
            int a[6], e[6];
#pragma unroll
            for (int h = 0; h < 4; h++) {
                a[h] = lane_int(ca[h], c);
                e[h] = lane_int(cv[h], c) + lane_int(cb[h], c) * (int)y;
            }
            bool c4 = true;
            if (any6) {
                const uint32_t qc = (uint32_t)lane_int((int)q, c);
                const int dic = lane_int(di, c), djc = lane_int(dj, c) + (int)y;
                c4 = lane_int((int)cvx, c) != 0;
                a[4] = a[5] = e[4] = e[5] = 0;
                if (i < tot && !c4) {
                    const int *hp = extra[qc].hp;
#pragma unroll
                    for (int h = 4; h < 6; h++) {
                        a[h] = hp[3 * h - 12];
                        e[h] = a[h] * dic + hp[3 * h - 11] * djc - hp[3 * h - 10];
                    }
                }
            }
            if (i < tot)
                rows[8 * c + y] = (uint8_t)(c4 ? row_walk<4>(a, e) : row_walk<6>(a, e));
        }
        wave_sync();
        if (nr)
            mk = W.mask[lane];
    }
    if (wide)
        mk = wide_block_mask(r.flags, xyp[q], px0, py0);
    return mk;
}

// Single-sample coverage (one lane, one quad), same rule.
__device__ __forceinline__ bool pixel_coverage(const CovRec &r, const ExtraRec *__restrict__ extra,
                                               const QuadXY *__restrict__ xyp, uint32_t q, int px, int py)
{
    if (r.flags & kWide)
        return wide_covers(r.flags, xyp[q], px, py);
    const int di = px - (int)(r.bb_i & 0xffffu);
    const int dj = py - (int)(r.bb_j & 0xffffu);
    const int *hp = r.hp;
    if (r.flags & kConvex) {
        bool in = true;
        for (int h = 0; h < 4; h++)
            in = in && (__mul24(hp[3 * h], di) + __mul24(hp[3 * h + 1], dj) >= hp[3 * h + 2]);
        return in;
    }
    const bool t0 = (__mul24(hp[0], di) + __mul24(hp[1], dj) >= hp[2]) &&
                    (__mul24(hp[3], di) + __mul24(hp[4], dj) >= hp[5]) &&
                    (__mul24(hp[6], di) + __mul24(hp[7], dj) >= hp[8]);
    const int *ex = extra[q].hp;
    const bool t1 = (__mul24(hp[9], di) + __mul24(hp[10], dj) >= hp[11]) &&
                    (__mul24(ex[0], di) + __mul24(ex[1], dj) >= ex[2]) &&
                    (__mul24(ex[3], di) + __mul24(ex[4], dj) >= ex[5]);
    return t0 || t1;
}

// Block key: the quad's depth at the centroid of its covered samples in the
// block (Stage 3, phase 2), fp32; smaller code = nearer.  A heuristic only:
// the per-pixel sorter and its exact fallback decide the final order.
__device__ __forceinline__ uint32_t block_depth_code(const PlaneRec &r, uint64_t m, int px0, int py0)
{
    const float cnt = (float)__popcll(m);
    const float sx = (float)(__popcll(m & 0xAAAAAAAAAAAAAAAAull) + 2 * __popcll(m & 0xCCCCCCCCCCCCCCCCull) +
                             4 * __popcll(m & 0xF0F0F0F0F0F0F0F0ull));
    const float sy = (float)(__popcll(m & 0xFF00FF00FF00FF00ull) + 2 * __popcll(m & 0xFFFF0000FFFF0000ull) +
                             4 * __popcll(m & 0xFFFFFFFF00000000ull));
    const float inv = 1.0f / cnt;
    const float cx = (float)(px0 - (int)(r.ij & 0xffffu)) + sx * inv;
    const float cy = (float)(py0 - (int)(r.ij >> 16)) + sy * inv;
    // the plane rounded to fp32
    float k = (float)r.A * cx + (float)r.B * cy + (float)r.C0;
    k = (k > 0.0f) ? k : 0.0f;  // NaN -> 0
    return 0x7F800000u - min(__float_as_uint(k), 0x7F800000u);  // < 2^31
}

// Ascending bitonic sort of n keys in wave-private LDS by one wave.
template <typename KeyT>
__device__ void wave_bitonic_sort(KeyT *keys, uint32_t n, KeyT pad, uint32_t lane)
{
    if (n < 2)
        return;
    uint32_t P = 2;
    while (P < n)
        P <<= 1;
    for (uint32_t i = n + lane; i < P; i += 64)
        keys[i] = pad;
    wave_sync();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = lane; t < P / 2; t += 64) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t ixj = i | j;
                const KeyT x = keys[i], y = keys[ixj];
                const bool up = (i & k) == 0;
                if ((x > y) == up) {
                    keys[i] = y;
                    keys[ixj] = x;
                }
            }
            wave_sync();
        }
    }
}

// v of lane (this lane ^ m) for sort keys of 32 or 64 bits.
__device__ __forceinline__ uint32_t shfl_xor_key(uint32_t v, int m) { return shfl_xor(v, m); }
__device__ __forceinline__ unsigned long long shfl_xor_key(unsigned long long v, int m)
{
    const uint32_t lo = shfl_xor((uint32_t)v, m), hi = shfl_xor((uint32_t)(v >> 32), m);
    return ((unsigned long long)hi << 32) | lo;
}

// Ascending bitonic sort of the 64 R keys v[r] at index lane * R + r, in
// registers: partners in the same lane (the first log2 R steps of every
// merge) are compared directly, partners in other lanes exchanged with
// shfl_xor.  Every lane must be active.
template <int R, typename KeyT>
__device__ __forceinline__ void wave_sort_regs(KeyT (&v)[R], uint32_t lane)
{
#pragma unroll
    for (uint32_t k = 2; k <= 64u * R; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (j < (uint32_t)R) {
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)R; r++) {
                    if (r & j)
                        continue;
                    const bool up = ((lane * R + r) & k) == 0;
                    const KeyT x = v[r], y = v[r | j];
                    const bool sw = (x > y) == up;
                    v[r] = sw ? y : x;
                    v[r | j] = sw ? x : y;
                }
            } else {
                const uint32_t m = j / R;  // the partner lane is lane ^ m
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)R; r++) {
                    const KeyT o = shfl_xor_key(v[r], (int)m);
                    const bool up = ((lane * R + r) & k) == 0;
                    const bool lower = (lane & m) == 0;  // this lane holds the lower index of the pair
                    v[r] = (lower == up) ? min(v[r], o) : max(v[r], o);
                }
            }
        }
    }
}

// Sorts keys[0 .. n - 1] of a wave's LDS ascending through registers
// (n <= 64 R; keys[n .. 64 R - 1] must be in bounds, their values are not
// read).
template <int R, typename KeyT>
__device__ __forceinline__ void sort_keys_regs(KeyT *keys, uint32_t n, KeyT pad, uint32_t lane)
{
    KeyT v[R];
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)R; r++) {
        const uint32_t i = lane * R + r;
        v[r] = keys[i];
        v[r] = i < n ? v[r] : pad;
    }
    wave_sort_regs<R>(v, lane);
    wave_sync();
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)R; r++) {
        const uint32_t i = lane * R + r;
        if (i < n)
            keys[i] = v[r];
    }
    wave_sync();
}

// An entry's plane, bbox origin and colour as the per-pixel walk reads them
// (the quad's PlaneRec).
using Stage = PlaneRec;

// Entries one on-chip sort takes; longer block lists are cut into slices.
constexpr uint32_t kSortCap = 1024;

// A block with at most kFast entries keeps everything its walk needs on
// chip, in slot order: sort keys, codes, masks and each entry's depth plane
// and colour; it writes no entry to global memory.  When a block's list
// grows past kFast, its on-chip entries are copied out once and every later
// entry goes to global memory; the keys of the longer list then overwrite
// this storage, which they share.
constexpr uint32_t kFast = 64;
struct FastEntries {
    uint32_t key[kFast];                // the first kFast sort keys
    uint32_t code[kFast];
    unsigned long long mask[kFast];
    Stage st[kFast];
    uint32_t id[kFast];
    uint32_t bound[kFast];              // with the cutoff: nearest possible order code
};
union WaveKeys {
    uint32_t key[kSortCap];
    FastEntries f;
};
static_assert(sizeof(FastEntries) <= sizeof(uint32_t) * kSortCap, "fast entries alias the key array");

// Per-wave LDS of the sorted raster: candidate batch, sort keys of the
// current slice (also the slicing histogram) or the fast entries, and the
// phase-3 staging in sorted order, whose space the coverage pass of each
// phase-1 batch borrows.
struct WalkStage {
    Stage st[64];
    uint32_t sid[64];
};
struct WaveLds {
    uint32_t cand[128];
    uint32_t seg_after[kSortCap / 64];  // cutoff: smallest bound code after each segment
    WaveKeys k;
    union {
        WalkStage w;  // phase 3
        RowWork rw;   // phase 1: coverage masks of a batch
    } s;
};

// A workgroup's window on its bin list: the whole list when it has at most
// list_cap(NW) quads (loaded once for every round of blocks), else one chunk
// of NW * 64 at a time.
constexpr uint32_t kListCap = 512;
__host__ __device__ constexpr uint32_t list_cap(uint32_t nw) { return nw * 64 > kListCap ? nw * 64 : kListCap; }
template <int NW>
struct BinChunk {
    uint32_t q[list_cap(NW)];
    uint2 bb[list_cap(NW)];
};

struct BlockGeom {
    int px0, py0, px1, py1;  // block pixel rect clipped to the screen
    int px, py;              // this lane's pixel
    uint32_t blk, pix;
    uint64_t onmask;
    bool active, on;
};

__device__ __forceinline__ BlockGeom block_geom(const FrameArgs &a, uint32_t bxk, uint32_t byk, bool valid,
                                                uint32_t lane)
{
    BlockGeom g;
    g.active = valid && bxk < a.nblk_x && byk < a.nblk_y;
    g.px0 = (int)bxk * 8;
    g.py0 = (int)byk * 8;
    g.px1 = min(g.px0 + 7, (int)a.W - 1);
    g.py1 = min(g.py0 + 7, (int)a.H - 1);
    g.px = g.px0 + (int)(lane & 7);
    g.py = g.py0 + (int)(lane >> 3);
    g.on = g.active && g.px < (int)a.W && g.py < (int)a.H;
    g.onmask = ballot(g.on);
    g.blk = byk * a.nblk_x + bxk;
    g.pix = g.on ? (uint32_t)g.py * a.W + (uint32_t)g.px : 0;
    return g;
}

// Phase 1 of a block: walks the bin list; every batch of up to 64
// candidates (quads whose bbox meets the block, in list = ascending quad
// order) goes to on_batch(m): lane e < m holds cand[e].  All waves of the
// workgroup call this together (the chunk loads are shared).
template <int NW, typename Lds, typename F>
__device__ void scan_bin(const uint2 *__restrict__ bbox, const uint32_t *__restrict__ pairs, BinChunk<NW> &C,
                         Lds &L, uint32_t start, uint32_t cnt, bool cached, const BlockGeom &g, F &&on_batch)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    uint32_t nc = 0;
    // a long list comes in windows of list_cap(NW) quads, every thread
    // loading its share of a window's indices, then of their bboxes, at once
    constexpr uint32_t kPer = list_cap(NW) / (NW * 64);
    const uint32_t step = cached ? cnt : list_cap(NW);
    for (uint32_t base = 0; base < cnt; base += step) {
        if (!cached) {
            uint32_t qw[kPer];
            uint2 bw[kPer];
#pragma unroll
            for (uint32_t k = 0; k < kPer; k++) {
                const uint32_t t = base + k * NW * 64 + tid;
                qw[k] = t < cnt ? pairs[start + t] : 0u;
            }
#pragma unroll
            for (uint32_t k = 0; k < kPer; k++) {
                const uint32_t t = base + k * NW * 64 + tid;
                bw[k] = t < cnt ? bbox[qw[k]] : make_uint2(0xffffu, 0u);
            }
#pragma unroll
            for (uint32_t k = 0; k < kPer; k++) {
                C.q[k * NW * 64 + tid] = qw[k];
                C.bb[k * NW * 64 + tid] = bw[k];
            }
            __syncthreads();
        }
        const uint32_t m = min(cnt - base, step);
        if (g.active) {
            for (uint32_t c = 0; c < m; c += 64) {
                const uint32_t e = c + lane;
                bool ov = false;
                uint32_t q = 0;
                if (e < m) {
                    q = C.q[e];
                    const uint2 bb = C.bb[e];
                    ov = (int)(bb.x & 0xffffu) <= g.px1 && (int)(bb.x >> 16) >= g.px0 &&
                         (int)(bb.y & 0xffffu) <= g.py1 && (int)(bb.y >> 16) >= g.py0;
                }
                const uint64_t b = ballot(ov);
                if (ov)
                    L.cand[nc + rank_below(b)] = q;
                nc += (uint32_t)__popcll(b);
                if (nc >= 64) {
                    wave_sync();
                    on_batch(64u);
                    wave_sync();
                    // carry the overflow to the front of the batch buffer
                    if (lane + 64 < nc)
                        L.cand[lane] = L.cand[lane + 64];
                    nc -= 64;
                    wave_sync();
                }
            }
        }
        if (!cached)
            __syncthreads();
    }
    if (g.active && nc) {
        wave_sync();
        on_batch(nc);
        wave_sync();
    }
}

// Loads a bin list of at most kListCap quads into the workgroup's window.
template <int NW>
__device__ __forceinline__ void load_bin_list(const uint2 *__restrict__ bbox, const uint32_t *__restrict__ pairs,
                                              BinChunk<NW> &C, uint32_t start, uint32_t cnt)
{
    for (uint32_t t = threadIdx.x; t < cnt; t += NW * 64) {
        const uint32_t q = pairs[start + t];
        C.q[t] = q;
        C.bb[t] = bbox[q];
    }
    __syncthreads();
}

// Queue a block's pixels for the exact per-pixel sort (wave-aggregated, on
// the block's queue stripe).
__device__ __forceinline__ void push_flagged(const FrameArgs &a, bool flag, const BlockGeom &g, uint32_t lane)
{
    const uint64_t m = ballot(flag);
    if (!m)
        return;
    const uint32_t s = g.blk % kQueues;
    uint32_t base = 0;
    if (lane == 0)
        base = atomicAdd(&a.ctr->stripe[s].flag_n, (uint32_t)__popcll(m));
    base = lane_value(base, 0);
    if (flag)
        a.fb_queue[(size_t)s * a.qcap_blocks * 64 + base + rank_below(m)] = g.pix;
}

// Per-pixel state of phase 3: the K-deep sorter (codes ascending, filled
// with placeholder code 0 that is emitted first and blends nothing), the
// last emitted code, and the front-to-back blend.
template <int K, bool DEBUG, bool CUT, bool VCOL>
struct PixelSorter {
    uint32_t qk[K], qc[K], qi[DEBUG ? K : 1];
    uint32_t last, nfrag, npop, obase;
    bool flagged;
    bool done;     // CUT: stopped, and no fragment left can precede the ones emitted
    float T, R, G, B;
    int px, py;    // VCOL: the pixel (queued colours are quad indices)

    // CUT: the transmittance is below kCutT: nothing more is blended
    __device__ __forceinline__ bool stopped() const { return T < kCutT; }

    __device__ __forceinline__ void init(uint32_t ob)
    {
#pragma unroll
        for (int j = 0; j < K; j++) {
            qk[j] = 0;
            qc[j] = 0;
            if (DEBUG)
                qi[j] = 0;
        }
        last = nfrag = npop = 0;
        obase = ob;
        flagged = false;
        done = false;
        T = 1.0f;
        R = G = B = 0.0f;
    }

    __device__ __forceinline__ void emit(const FrameArgs &a, bool on, uint32_t pk, uint32_t pc, uint32_t pi)
    {
        flagged |= (pk - 1u) < last;  // emitted codes must strictly increase (placeholders excepted)
        last = pk;
        const bool live = !CUT || !stopped();  // this fragment is blended
        // with vertex colours pc is the quad (placeholders blend nothing)
        const float4 d = VCOL ? (pk ? vertex_colour(a, pc, px, py) : make_float4(0.0f, 0.0f, 0.0f, 0.0f))
                              : decode_rgba(pc);
        if (CUT)
            blend_ftb_cut(d, T, R, G, B);
        else
            blend_ftb_dec(d, T, R, G, B);
        if (DEBUG && pk != 0 && live) {
            if (a.dbg_ids && on && obase + npop < a.dbg_cap)
                a.dbg_ids[obase + npop] = pi;
            npop++;
        }
    }

    // insert x and emit the smallest of queue + x
    __device__ __forceinline__ void push(const FrameArgs &a, bool on, uint32_t x, uint32_t xc, uint32_t xi)
    {
        nfrag++;
        flagged |= (x == 0xFFFFFFFFu);  // zero key: leave it to the exact path
        bool lt[K];
#pragma unroll
        for (int j = 0; j < K; j++)
            lt[j] = x < qk[j];
        const uint32_t pk = lt[0] ? x : qk[0];
        const uint32_t pc = lt[0] ? xc : qc[0];
        uint32_t pi = 0;
        if (DEBUG)
            pi = lt[0] ? xi : qi[0];
#pragma unroll
        for (int j = 0; j < K - 1; j++) {
            qk[j] = lt[j + 1] ? (lt[j] ? qk[j] : x) : qk[j + 1];
            qc[j] = lt[j + 1] ? (lt[j] ? qc[j] : xc) : qc[j + 1];
            if (DEBUG)
                qi[j] = lt[j + 1] ? (lt[j] ? qi[j] : xi) : qi[j + 1];
        }
        qk[K - 1] = lt[K - 1] ? qk[K - 1] : x;
        qc[K - 1] = lt[K - 1] ? qc[K - 1] : xc;
        if (DEBUG)
            qi[K - 1] = lt[K - 1] ? qi[K - 1] : xi;
        emit(a, on, pk, pc, pi);
    }

    // every fragment still queued comes strictly after the last emitted one
    // (placeholders excepted)
    __device__ __forceinline__ bool queue_after_last() const
    {
        bool ok = true;
#pragma unroll
        for (int j = 0; j < K; j++)
            ok = ok && (qk[j] == 0u || qk[j] > last);
        return ok;
    }

    __device__ __forceinline__ void flush(const FrameArgs &a, bool on)
    {
#pragma unroll
        for (int j = 0; j < K; j++)
            emit(a, on, qk[j], qc[j], DEBUG ? qi[j] : 0);
    }
};

// Phase 1 of the sorted path for one batch: each lane takes a candidate,
// its coverage mask of the block comes from batch_masks and, if not empty,
// the lane builds its block key; non-empty entries take slot n + rank, on
// chip while the block has at most kFast of them and in the wave's global
// entry region beyond, and the first kSortCap also go to the LDS sort keys
// (key bits above the slot index).
//
// With half-blocks, the rows 0-3 and 4-7 of a mask become separate entries,
// each keyed at the centroid of its own samples: one sort then orders both
// 8x4 halves, and a pixel only sees the entries of its half.
template <bool CUT>
__device__ __forceinline__ void put_entry(const FrameArgs &a, WaveLds &L, uint32_t ebase, uint32_t sb,
                                          uint32_t slot, uint32_t code, uint64_t mask, uint32_t q,
                                          const PlaneRec &pl, bool to_global, uint32_t bound)
{
    if (to_global) {
        a.ent_code[ebase + slot] = code;
        a.ent_mask[ebase + slot] = mask;
        a.ent_id[ebase + slot] = q;
        if (CUT)
            a.ent_bound[ebase + slot] = bound;
    } else {  // slot < kFast
        L.k.f.code[slot] = code;
        L.k.f.mask[slot] = mask;
        L.k.f.st[slot] = pl;
        L.k.f.id[slot] = q;
        if (CUT)
            L.k.f.bound[slot] = bound;
    }
    if (slot < kSortCap)
        L.k.key[slot] = ((code >> (sb - 1)) << sb) | slot;  // code: 31 bits
}

// Nearest order code any fragment of an entry can have (with the cutoff):
// the plane's largest value over the part of the pixel rectangle [i0, i1] x
// [j0, j1] inside the quad's bbox (an affine function peaks at a corner),
// rounded to fp32 and raised by one ulp, which bounds every fragment key of
// the entry from above (their fp64 values differ from the true plane by far
// less than half an fp32 ulp).  0 (no bound) when that value is not positive.
__device__ __forceinline__ uint32_t entry_bound_code(const PlaneRec &pl, const CovRec &r, int i0, int i1, int j0,
                                                     int j1)
{
    const int imin = (int)(pl.ij & 0xffffu), jmin = (int)(pl.ij >> 16);
    i0 = max(i0, imin);
    i1 = min(i1, (int)(r.bb_i >> 16));
    j0 = max(j0, jmin);
    j1 = min(j1, (int)(r.bb_j >> 16));
    const int di = (pl.A >= 0.0 ? i1 : i0) - imin;
    const int dj = (pl.B >= 0.0 ? j1 : j0) - jmin;
    const float k = (float)fma(pl.A, (double)di, fma(pl.B, (double)dj, pl.C0));
    if (!(k > 1e-30f))
        return 0u;
    const uint32_t kb = __float_as_uint(k);
    return ~(kb >= 0x7F800000u ? 0x7F800000u : kb + 1u);
}

template <bool CUT>
__device__ __forceinline__ void sorted_batch(const FrameArgs &a, const QuadXY *__restrict__ xyp, WaveLds &L,
                                             uint32_t m, const BlockGeom &g, uint32_t lane, uint32_t ebase,
                                             uint32_t sb, bool half, uint32_t &n)
{
    uint64_t m0 = 0, m1 = 0;  // entries: m0 (whole block, or rows 0-3), m1 (rows 4-7)
    uint32_t q = 0, c0 = 0, c1 = 0;
    // the candidate's coverage record and plane, loaded at once (one memory
    // latency for the masks, the block keys and the entries)
    CovRec r;
    PlaneRec pl;
    const bool has = lane < m;
    if (has) {
        q = L.cand[lane];
        r = a.cov[q];
        pl = a.plane[q];
    }
    const uint64_t mk = batch_masks(r, has, a.extra, xyp, q, L.s.rw, g.px0, g.py0, lane) & g.onmask;
    uint32_t d0 = 0, d1 = 0;  // CUT: entry bounds
    if (has) {
        m0 = half ? (mk & 0xFFFFFFFFull) : mk;
        m1 = half ? (mk & ~0xFFFFFFFFull) : 0;
        if (m0) {
            c0 = block_depth_code(pl, m0, g.px0, g.py0);
            if (CUT)
                d0 = entry_bound_code(pl, r, g.px0, g.px1, g.py0, half ? g.py0 + 3 : g.py1);
        }
        if (m1) {
            c1 = block_depth_code(pl, m1, g.px0, g.py0);
            if (CUT)
                d1 = entry_bound_code(pl, r, g.px0, g.px1, g.py0 + 4, g.py1);
        }
    }
    const uint64_t b0 = ballot(m0 != 0);
    const uint64_t b1 = half ? ballot(m1 != 0) : 0;
    const uint32_t n0 = (uint32_t)__popcll(b0);
    const bool to_global = n + n0 + (uint32_t)__popcll(b1) > kFast;
    if (to_global && n <= kFast && lane < n) {
        // the list leaves the fast path: copy its on-chip entries out first
        a.ent_code[ebase + lane] = L.k.f.code[lane];
        a.ent_mask[ebase + lane] = L.k.f.mask[lane];
        a.ent_id[ebase + lane] = L.k.f.id[lane];
        if (CUT)
            a.ent_bound[ebase + lane] = L.k.f.bound[lane];
    }
    if (m0)
        put_entry<CUT>(a, L, ebase, sb, n + rank_below(b0), c0, m0, q, pl, to_global, d0);
    if (m1)
        put_entry<CUT>(a, L, ebase, sb, n + n0 + rank_below(b1), c1, m1, q, pl, to_global, d1);
    n += n0 + (uint32_t)__popcll(b1);
}

// Phases 2 and 3 for n sorted-key entries in L.key (entry = low sb bits,
// an index into the wave's global entry region): depth-sort them, then one
// lane per pixel walks them in 64-entry segments whose coverage masks are
// transposed to per-pixel bit sets, feeding each pixel's sorter.
//
// With the cutoff, a pixel whose transmittance has dropped below kCutT is
// done -- it skips the rest of the list -- once no fragment left can come
// before the ones it emitted: every entry after the current segment
// (rest_after covers entries walked after this list) has a bound code above
// its last emitted code, and so has everything still in its queue.  Then
// the fragments it blended are exactly the first ones of the full order.
// A wave stops walking when all its pixels are done or flagged.
template <int K, bool DEBUG, bool CUT, bool VCOL>
__device__ void walk_entries(const FrameArgs &a, WaveLds &L, uint32_t n, uint32_t ebase, uint32_t sb,
                             const BlockGeom &g, uint32_t lane, PixelSorter<K, DEBUG, CUT, VCOL> &ps,
                             uint32_t rest_after = 0xFFFFFFFFu)
{
    wave_sync();
    // the block's keys: in registers up to 256 (flat colours: the cutoff and
    // vertex-colour kernels have no registers to spare), else the LDS network
    if (!CUT && !VCOL && n <= 128)
        sort_keys_regs<2, uint32_t>(L.k.key, n, 0xFFFFFFFFu, lane);
    else if (!CUT && !VCOL && n <= 256)
        sort_keys_regs<4, uint32_t>(L.k.key, n, 0xFFFFFFFFu, lane);
    else
        wave_bitonic_sort<uint32_t>(L.k.key, n, 0xFFFFFFFFu, lane);
    // CUT: seg_after[s] is the smallest bound code of the entries after segment s
    if (CUT) {
        // segments from the back, four at a time (their loads issued together)
        const uint32_t nseg = (n + 63) / 64;
        uint32_t run = rest_after;
        for (int g4 = (int)((nseg + 3) / 4) - 1; g4 >= 0; g4--) {
            uint32_t bm[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t e = (uint32_t)(g4 * 4 + k) * 64 + lane;
                bm[k] = e < n ? a.ent_bound[ebase + (L.k.key[e] & ((1u << sb) - 1))] : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int k = 3; k >= 0; k--) {
                const uint32_t sg = (uint32_t)(g4 * 4 + k);
                if (sg < nseg && lane == 0)
                    L.seg_after[sg] = run;
                if (sg < nseg) {
                    uint32_t v = bm[k];
                    for (int off = 32; off > 0; off >>= 1)
                        v = min(v, shfl_xor(v, off));
                    run = min(run, v);
                }
            }
        }
    }
    for (uint32_t seg = 0; seg < n; seg += 64) {
        const uint32_t e = seg + lane;
        uint64_t m = 0;
        if (e < n) {
            const uint32_t slot = ebase + (L.k.key[e] & ((1u << sb) - 1));
            m = a.ent_mask[slot];
            const uint32_t q = a.ent_id[slot];
            L.s.w.st[lane] = a.plane[q];
            if (DEBUG || VCOL)
                L.s.w.sid[lane] = q;
        }
        wave_sync();
        uint64_t col = transpose64(m, lane);
        if (!g.on || ps.flagged || ps.done)
            col = 0;
        while (col) {
            const uint32_t k = (uint32_t)__builtin_ctzll(col);
            col &= col - 1;
            const Stage st = L.s.w.st[k];
            const float kf =
                frag_key(st.A, st.B, st.C0, g.px - (int)(st.ij & 0xffffu), g.py - (int)(st.ij >> 16));
            const uint32_t sid = (DEBUG || VCOL) ? L.s.w.sid[k] : 0u;
            ps.push(a, g.on, order_code(kf), VCOL ? sid : st.rgba, sid);
            if (ps.flagged)
                col = 0;
        }
        wave_sync();
        if (CUT) {
            const uint32_t rest = L.seg_after[seg >> 6];
            ps.done = ps.done || (ps.stopped() && !ps.flagged && rest > ps.last && ps.queue_after_last());
            if (!ballot(g.on && !ps.flagged && !ps.done))
                break;
        }
    }
}

// Ascending sort of one 32-bit key per lane across the wave (bitonic network
// over lane indices, exchanges by cross-lane permutes).
__device__ __forceinline__ uint32_t wave_sort_reg(uint32_t v, uint32_t lane)
{
    // an opaque copy of the lane index: the network's per-step lane masks are
    // then formed where they are used instead of being hoisted to the kernel
    // start, where they would hold 21 scalar register pairs for its lifetime
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            const uint32_t o = shfl_xor(v, (int)j);
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            v = keep_min ? min(v, o) : max(v, o);
        }
    }
    return v;
}

// Phases 2 and 3 for a block of n <= kFast entries, all on chip: the keys
// are sorted in registers and each entry's mask, plane and colour come from
// the fast entries written during phase 1.
template <int K, bool DEBUG, bool CUT, bool VCOL>
__device__ void walk_fast(const FrameArgs &a, WaveLds &L, uint32_t n, uint32_t sb, const BlockGeom &g,
                          uint32_t lane, PixelSorter<K, DEBUG, CUT, VCOL> &ps)
{
    wave_sync();
    uint32_t key = lane < n ? L.k.f.key[lane] : 0xFFFFFFFFu;
    key = wave_sort_reg(key, lane);
    uint64_t m = 0;
    if (lane < n) {
        const uint32_t slot = key & ((1u << sb) - 1);
        m = L.k.f.mask[slot];
        L.s.w.st[lane] = L.k.f.st[slot];
        if (DEBUG || VCOL)
            L.s.w.sid[lane] = L.k.f.id[slot];
    }
    wave_sync();
    uint64_t col = transpose64(m, lane);
    if (!g.on)
        col = 0;
    while (col) {
        const uint32_t k = (uint32_t)__builtin_ctzll(col);
        col &= col - 1;
        const Stage st = L.s.w.st[k];
        const float kf = frag_key(st.A, st.B, st.C0, g.px - (int)(st.ij & 0xffffu), g.py - (int)(st.ij >> 16));
        const uint32_t sid = (DEBUG || VCOL) ? L.s.w.sid[k] : 0u;
        ps.push(a, g.on, order_code(kf), VCOL ? sid : st.rgba, sid);
        if (ps.flagged)
            col = 0;
    }
    wave_sync();
}

// A block with n > kSortCap entries: a 256-bucket histogram of its block
// keys over [kmin, kmax] splits the key range into slices of at most
// kSortCap entries (whole buckets, nearest first); each slice is gathered
// from the global entry region into the LDS keys and walked.  The pixel
// sorters carry over from slice to slice, so they see the same entry order
// as one sort of the whole list.  Returns false when one bucket alone holds
// more than kSortCap entries.  With the cutoff, each slice is walked knowing
// the smallest bound code of the slices after it, and the walk ends when
// every pixel of the block is done or flagged.
template <int K, bool DEBUG, bool CUT, bool VCOL>
__device__ bool walk_sliced(const FrameArgs &a, WaveLds &L, uint32_t n, uint32_t ebase, uint32_t sb,
                            const BlockGeom &g, uint32_t lane, PixelSorter<K, DEBUG, CUT, VCOL> &ps)
{
    // the key range of the block's entries
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0;
    for (uint32_t e = lane; e < n; e += 64) {
        const uint32_t c = a.ent_code[ebase + e];
        kmin = min(kmin, c);
        kmax = max(kmax, c);
    }
    for (int off = 32; off > 0; off >>= 1) {
        kmin = min(kmin, shfl_xor(kmin, off));
        kmax = max(kmax, shfl_xor(kmax, off));
    }
    const uint32_t span = kmax - kmin;  // < 2^31
    const uint32_t bits = span ? 32 - __builtin_clz(span) : 1;
    const uint32_t hs = bits > 8 ? bits - 8 : 0;  // bucket = (code - kmin) >> hs, in [0, 256)
    uint32_t *hist = L.k.key;  // reused: 256 counters, then the slice keys
    uint32_t *bmin = L.k.key + 256;  // CUT: smallest bound code per bucket
    for (uint32_t b = lane; b < 256; b += 64) {
        hist[b] = 0;
        if (CUT)
            bmin[b] = 0xFFFFFFFFu;
    }
    wave_sync();
    for (uint32_t e = lane; e < n; e += 64) {
        const uint32_t bk = (a.ent_code[ebase + e] - kmin) >> hs;
        atomicAdd(&hist[bk], 1u);
        if (CUT)
            atomicMin(&bmin[bk], a.ent_bound[ebase + e]);
    }
    wave_sync();
    uint32_t counts[4], sfx[4];
    for (int k = 0; k < 4; k++)
        counts[k] = hist[lane * 4 + k];  // lane holds buckets 4*lane .. 4*lane+3
    if (CUT) {
        // sfx[k]: smallest bound code of the buckets from 4*lane+k on
        for (int k = 0; k < 4; k++)
            sfx[k] = bmin[lane * 4 + k];
        for (int k = 2; k >= 0; k--)
            sfx[k] = min(sfx[k], sfx[k + 1]);
        uint32_t run = 0xFFFFFFFFu;
        for (int l = 63; l >= 0; l--) {
            const uint32_t v = lane_value(sfx[0], (uint32_t)l);
            if (lane == (uint32_t)l)
                for (int k = 0; k < 4; k++)
                    sfx[k] = min(sfx[k], run);
            run = min(run, v);
        }
    }
    wave_sync();
    // code resolution inside a slice: 32 - sb bits for the (code - lo) part
    const uint32_t room = 32 - sb;
    uint32_t b0 = 0;
    while (b0 < 256) {
        // greedy: the longest run of buckets from b0 holding at most kSortCap entries
        uint32_t take = 0, sum = 0;
        for (uint32_t b = b0; b < 256; b++) {
            const uint32_t c = lane_value(counts[b & 3], b >> 2);
            if (sum + c > kSortCap)
                break;
            sum += c;
            take++;
        }
        if (take == 0)
            return false;
        const uint32_t b1 = b0 + take;
        const uint32_t lo = kmin + (b0 << hs);
        const uint32_t hi = (b1 >= 256) ? kmax + 1 : kmin + (b1 << hs);
        const uint32_t w = hi - lo - 1;
        const uint32_t wb = w ? 32 - __builtin_clz(w) : 1;
        const uint32_t sh = wb > room ? wb - room : 0;
        uint32_t ns = 0;
        for (uint32_t base = 0; base < n; base += 64) {
            const uint32_t e = base + lane;
            uint32_t code = 0;
            bool in = false;
            if (e < n) {
                code = a.ent_code[ebase + e];
                in = code >= lo && code < hi;
            }
            const uint64_t bm = ballot(in);
            if (in)
                L.k.key[ns + rank_below(bm)] = (((code - lo) >> sh) << sb) | e;
            ns += (uint32_t)__popcll(bm);
        }
        uint32_t rest = 0xFFFFFFFFu;
        if (CUT && b1 < 256) {
            const uint32_t k = b1 & 3u;
            const uint32_t v = k == 0 ? sfx[0] : (k == 1 ? sfx[1] : (k == 2 ? sfx[2] : sfx[3]));
            rest = lane_value(v, b1 >> 2);
        }
        walk_entries<K, DEBUG, CUT, VCOL>(a, L, ns, ebase, sb, g, lane, ps, rest);
        if (CUT && !ballot(g.on && !ps.flagged && !ps.done))
            break;
        b0 = b1;
    }
    return true;
}

// Keeps, for the exact pass, the block's entries that cover one of its
// flagged pixels F (the n entries sit in slot order on chip when n <=
// kFast, else in the wave's global region): masks restricted to F, and quad
// indices, contiguous at blk_ent[block].  When the frame's capacity for
// them is used up, the block is marked and the exact pass walks its bin
// list instead.
__device__ void keep_flagged_entries(const FrameArgs &a, const WaveLds &L, const BlockGeom &g, uint64_t F,
                                     uint32_t n, uint32_t ebase, uint32_t lane)
{
    const bool fast = n <= kFast;
    uint32_t total = 0;
    for (uint32_t e0 = 0; e0 < n; e0 += 64) {
        const uint32_t e = e0 + lane;
        uint64_t m = 0;
        if (e < n)
            m = (fast ? L.k.f.mask[e] : a.ent_mask[ebase + e]) & F;
        total += (uint32_t)__popcll(ballot(m != 0));
    }
    uint32_t first = 0;
    if (lane == 0)
        first = atomicAdd(&a.ctr->fe_n, total);
    first = lane_value(first, 0);
    if ((uint64_t)first + total > a.fe_cap) {
        if (lane == 0)
            a.blk_ent[g.blk] = make_uint2(kNoEntries, 0u);
        return;
    }
    uint32_t run = first;
    for (uint32_t e0 = 0; e0 < n; e0 += 64) {
        const uint32_t e = e0 + lane;
        uint64_t m = 0;
        uint32_t q = 0;
        if (e < n) {
            m = (fast ? L.k.f.mask[e] : a.ent_mask[ebase + e]) & F;
            q = fast ? L.k.f.id[e] : a.ent_id[ebase + e];
        }
        const uint64_t b = ballot(m != 0);
        if (m) {
            a.fe_mask[run + rank_below(b)] = m;
            a.fe_id[run + rank_below(b)] = q;
        }
        run += (uint32_t)__popcll(b);
    }
    if (lane == 0)
        a.blk_ent[g.blk] = make_uint2(first, total);
}

// Outputs of a finished block: the pixel, flagged pixels to the exact
// queue (with the block's entries kept for them), and the wave's running
// statistics.
template <int K, bool DEBUG, bool CUT, bool VCOL>
__device__ void finish_block(const FrameArgs &a, const WaveLds &L, const BlockGeom &g, uint32_t lane,
                             PixelSorter<K, DEBUG, CUT, VCOL> &ps, uint32_t entries, uint32_t ebase)
{
    if (g.on && !ps.flagged)
        ps.flush(a, g.on);
    const uint64_t F = ballot(g.on && ps.flagged);
    if (F)
        keep_flagged_entries(a, L, g, F, entries, ebase, lane);
    push_flagged(a, g.on && ps.flagged, g, lane);
    const bool write = g.on && !ps.flagged;
    if (write) {
        reinterpret_cast<uint32_t *>(a.out)[g.pix] = pack_rgba8(ps.R, ps.G, ps.B, 1.0f - ps.T);
        if (DEBUG && a.dbg_rgba)
            reinterpret_cast<float4 *>(a.dbg_rgba)[g.pix] = make_float4(ps.R, ps.G, ps.B, 1.0f - ps.T);
    }
    if (DEBUG && g.on) {
        if (a.dbg_count)
            a.dbg_count[g.pix] = CUT ? ps.npop : ps.nfrag;  // with the cutoff: fragments blended
        if (a.dbg_flag)
            a.dbg_flag[g.pix] = ps.flagged ? 1 : 0;
    }
    // statistics (flagged pixels are counted by the exact path)
    uint32_t wsum = write ? ps.nfrag : 0;
    for (int off = 32; off > 0; off >>= 1)
        wsum += shfl_xor(wsum, off);
    // added per block: per-wave totals would hold registers through the walk
    if (lane == 0) {
        if (entries)
            add_stat(a.ctr, ST_ENTRIES, entries);
        if (wsum)
            add_stat(a.ctr, ST_FRAGMENTS, wsum);
    }
}

// Phases 2 and 3 of one block whose n entries phase 1 has built, with a
// K-deep per-pixel sorter, and the block's outputs.
template <int K, bool DEBUG, bool CUT, bool VCOL>
__device__ __forceinline__ void walk_block(const FrameArgs &a, WaveLds &L, const BlockGeom &g, uint32_t lane,
                                           uint32_t n, uint32_t ebase, uint32_t sb)
{
    PixelSorter<K, DEBUG, CUT, VCOL> ps;
    ps.init((DEBUG && g.on && a.dbg_off) ? a.dbg_off[g.pix] : 0);
    ps.px = g.px;
    ps.py = g.py;
    if (n <= kFast) {
        walk_fast<K, DEBUG, CUT, VCOL>(a, L, n, sb, g, lane, ps);
    } else {
        // entries written by other lanes of this wave are read back below
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (n <= kSortCap) {
            walk_entries<K, DEBUG, CUT, VCOL>(a, L, n, ebase, sb, g, lane, ps);
        } else {
            if (lane == 0)
                atomicAdd(&a.ctr->stripe[g.blk % kQueues].dense_n, 1u);
            if (!walk_sliced<K, DEBUG, CUT, VCOL>(a, L, n, ebase, sb, g, lane, ps)) {
                // no slice fits: the exact path takes the block
                ps.flagged = true;
                if (lane == 0)
                    atomicOr(&a.ctr->error, kErrDense);
            }
        }
    }
    finish_block<K, DEBUG, CUT, VCOL>(a, L, g, lane, ps, n, ebase);
}

// Sorted raster: one workgroup of NW waves per bin, one 8x8 block per wave
// per round.  With density classes the launch takes the dense bins first
// (their long workgroups start at once instead of at their place in screen
// order) and the other bins alongside them, sparse ones with a
// kLowDepth-deep sorter (the paper's Section 4 proposes adapting to density
// and running its low- and high-density rasterizers at the same time).
template <int K, bool DEBUG, class Src, int NW, bool CUT, bool VCOL>
__global__ __launch_bounds__(NW * 64, (!DEBUG && (K <= 8 || (K <= 16 && !CUT && !VCOL))) ? 4 : 2) void k_raster(Src src)
{
    __shared__ BinChunk<NW> C;
    __shared__ WaveLds Lw[NW];
    uint32_t bin;
    const FrameArgs &a = *frame_of(src, bin);
    const QuadXY *__restrict__ xyp = a.xy;
    const uint2 *__restrict__ bbox = a.bbox;
    const uint32_t *__restrict__ pairs = a.pairs;
    if (a.ctr->error & kErrPairs)
        return;  // bin lists are incomplete: the frame is reported as failed
    // with density classes the grid is twice the bins: first the dense bins,
    // then every other bin in screen order, sparse ones with the shallower
    // sorter
    bool low = false;
    if (a.k_low) {
        if (bin < a.nbins) {
            if (bin >= uniform(a.ctr->n_high))
                return;
            bin = uniform(a.high_list[bin]);
        } else {
            bin -= a.nbins;
            const uint32_t cls = a.bin_class[bin];
            if (cls == kDense)
                return;
            low = cls == kSparse;
        }
    }
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t bpb = 1u << (a.bin_shift - 3), nb = bpb * bpb;
    const uint32_t start = uniform(a.bin_start[bin]), cnt = uniform(a.bin_count[bin]);
    const uint32_t bx_bin = (bin % a.nbx) * bpb, by_bin = (bin / a.nbx) * bpb;
    // this wave's entry region: cnt entries per block, twice that with half-blocks
    const bool half = a.half_blocks != 0;
    const uint32_t ecap = half ? 2 * cnt : cnt;
    const uint32_t ebase = NW * (half ? 2 * start : start) + wave * ecap;
    // entry index bits in a sort key: enough for kSortCap and for ecap
    const uint32_t sb = max(10u, ecap > 1 ? 32 - __builtin_clz(ecap - 1) : 1u);
    WaveLds &L = Lw[wave];
    const bool cached = cnt <= list_cap(NW);
    if (cached)
        load_bin_list<NW>(bbox, pairs, C, start, cnt);
    const uint32_t nrounds = (nb + NW - 1) / NW;
    for (uint32_t ri = 0; ri < nrounds; ri++) {
        const uint32_t k = ri * NW + wave;
        const BlockGeom g = block_geom(a, bx_bin + k % bpb, by_bin + k / bpb, k < nb, lane);
        uint32_t n = 0;
        scan_bin<NW>(bbox, pairs, C, L, start, cnt, cached, g, [&](uint32_t m) {
            sorted_batch<CUT>(a, xyp, L, m, g, lane, ebase, sb, half, n);
        });
        if (g.active) {
            if constexpr (K > (int)kLowDepth) {
                if (low)
                    walk_block<(int)kLowDepth, DEBUG, CUT, VCOL>(a, L, g, lane, n, ebase, sb);
                else
                    walk_block<K, DEBUG, CUT, VCOL>(a, L, g, lane, n, ebase, sb);
            } else {
                walk_block<K, DEBUG, CUT, VCOL>(a, L, g, lane, n, ebase, sb);
            }
        }
    }
}

// --------------------------------------------------------- exact per pixel
//
// One wave per flagged pixel: the candidates are the entries the raster
// kept for the pixel's block (whose masks already say which quads cover the
// pixel), or, when the frame ran out of room for them, every quad of the
// pixel's bin tested on the single sample.  Covering fragments are sorted
// by their full (code, index) key in LDS and blended in order with the
// raster's blend routine, so the pixel comes out as an unbounded per-pixel
// sorter would give it ("Sample blending": the slower exact algorithm for
// the pixels the fixed-size sorter cannot order).  Pixels deeper than the LDS buffer are
// done in rounds: each round keeps only keys above the last blended key and,
// when the buffer fills, sorts it and keeps its lower half (raising an upper
// cut), so a round blends the smallest keys left, at least half a buffer.

constexpr uint32_t kFallbackBuf = 2048;
constexpr uint32_t kFallbackStep = 8;
// Groups of 64 sorted fragments whose colours the blend loads at once.
constexpr uint32_t kFallbackColours = 8;
// The exact pass runs one workgroup per CU, each with kFallbackWaves waves
// working on their own pixels with their own 16 KiB key buffer.
constexpr uint32_t kFallbackWaves = 8;
constexpr uint32_t kFallbackGrid = 256;
constexpr size_t kFallbackLds = (size_t)kFallbackWaves * kFallbackBuf * 8;

// Sorts a wave's n keys in LDS ascending: in registers up to 512 keys, else
// the LDS network.
__device__ __noinline__ void sort_keys(unsigned long long *keys, uint32_t n, uint32_t lane)
{
    if (n <= 64)
        sort_keys_regs<1>(keys, n, ~0ull, lane);
    else if (n <= 128)
        sort_keys_regs<2>(keys, n, ~0ull, lane);
    else if (n <= 256)
        sort_keys_regs<4>(keys, n, ~0ull, lane);
    else if (n <= 512)
        sort_keys_regs<8>(keys, n, ~0ull, lane);
    else
        wave_bitonic_sort<unsigned long long>(keys, n, ~0ull, lane);
}

// Lane s's value of v, as a wave-uniform value.
__device__ __forceinline__ float lane_float(float v, uint32_t s)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)s));
}

// A record in one go: its 16-byte chunks issued together, so the coverage
// test and the key wait once per record instead of once per field they
// branch on.
template <typename R>
__device__ __forceinline__ R load_whole(const R *__restrict__ p, uint32_t q)
{
    const uint4 *c = reinterpret_cast<const uint4 *>(p + q);
    uint4 d[sizeof(R) / 16];
#pragma unroll
    for (uint32_t k = 0; k < sizeof(R) / 16; k++)
        d[k] = c[k];
    R r;
    __builtin_memcpy(&r, d, sizeof(R));
    return r;
}

// Frames of a launch source, for kernels that walk them in turn.
__device__ __forceinline__ uint32_t frame_count(const OneFrame &) { return 1; }
__device__ __forceinline__ const FrameArgs &frame_at(const OneFrame &src, uint32_t) { return src.a; }
__device__ __forceinline__ uint32_t frame_count(const FrameMap &m) { return m.nf; }
__device__ __forceinline__ const FrameArgs &frame_at(const FrameMap &m, uint32_t f) { return m.tab[f]; }

// A persistent grid (kFallbackGrid workgroups of kFallbackWaves waves) walks
// the frames in order; in each frame wave g of the grid takes flagged pixels
// g, g + (waves of the grid), ..., so any number of flagged pixels spreads
// over the whole GPU.
template <bool DEBUG, class Src>
__global__ __launch_bounds__(kFallbackWaves * 64) void k_fallback(Src src)
{
    extern __shared__ unsigned long long s_fb[];  // [kFallbackWaves][kFallbackBuf] keys
    const uint32_t blk = blockIdx.x, nblk = gridDim.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long *s_key = s_fb + (size_t)wave * kFallbackBuf;
    for (uint32_t fi = 0; fi < frame_count(src); fi++) {
        const FrameArgs &a = frame_at(src, fi);
        const QuadXY *__restrict__ xyp = a.xy;
        const uint2 *__restrict__ bbox = a.bbox;
        const uint32_t *__restrict__ pairs = a.pairs;
        clear_next_counters(a, blk, nblk);
        // every error bit of the frame is set by the earlier kernels
        if (a.status && blk == 0 && threadIdx.x == 0)
            *a.status = a.ctr->error;
        if (a.ctr->error & kErrPairs)
            continue;
        // the frame's flagged pixels: one queue stripe per lane (kQueues == 64)
        const uint32_t cq = a.ctr->stripe[lane].flag_n;
        const uint32_t incl = wave_incl_scan(cq);
        const uint32_t count = lane_value(incl, 63);
        for (uint32_t item = blk * kFallbackWaves + wave; item < count; item += nblk * kFallbackWaves) {
            // stripe sq holds items [incl[sq - 1], incl[sq])
            const uint32_t sq = (uint32_t)__popcll(ballot(incl <= item));
            const uint32_t t = item - (sq ? lane_value(incl, sq - 1) : 0);
            const uint32_t p = uniform(a.fb_queue[(size_t)sq * a.qcap_blocks * 64 + t]);
            const int i = (int)(p % a.W), j = (int)(p / a.W);
            const uint32_t bin = ((uint32_t)j >> a.bin_shift) * a.nbx + ((uint32_t)i >> a.bin_shift);
            const uint32_t start = uniform(a.bin_start[bin]);
            const uint32_t cnt = uniform(a.bin_count[bin]);
            // candidates: the entries the raster kept for the pixel's block
            // (those covering one of its flagged pixels), else the bin list
            const uint2 ent = a.blk_ent[((uint32_t)j >> 3) * a.nblk_x + ((uint32_t)i >> 3)];
            const bool kept = uniform(ent.x) != kNoEntries;
            const uint32_t ncand = kept ? uniform(ent.y) : cnt;
            const uint32_t bit = (((uint32_t)j & 7u) << 3) | ((uint32_t)i & 7u);
            const uint32_t obase = (DEBUG && a.dbg_off) ? a.dbg_off[p] : 0;
            float T = 1.0f, R = 0.0f, G2 = 0.0f, B = 0.0f;
            const bool cut = a.alpha_cut != 0;
            unsigned long long lo = 0;  // keys <= lo are blended already (real keys are > 0)
            uint32_t total = 0, done = 0;
            uint32_t blended = 0;
            for (bool more = true; more;) {
                unsigned long long hi = ~0ull;  // the buffer holds every key in (lo, hi]
                bool cut_round = false;  // the buffer overflowed: keys above hi wait for a later round
                uint32_t n = 0, seen = 0;
                // kFallbackStep chunks of 64 candidates per step: each stage's loads
                // (list entries, then bboxes, then records) are issued together
                for (uint32_t base = 0; base < ncand; base += 64 * kFallbackStep) {
                    if (n + 64 * kFallbackStep > kFallbackBuf) {
                        // keep the lower half of the buffer
                        wave_bitonic_sort<unsigned long long>(s_key, n, ~0ull, lane);
                        n = kFallbackBuf / 2;
                        hi = s_key[n - 1];
                        cut_round = true;
                        wave_sync();
                    }
                    uint32_t q[kFallbackStep];
                    bool ov[kFallbackStep];
                    if (kept) {
                        // the block's kept entries: coverage is the pixel's mask bit
#pragma unroll
                        for (uint32_t c = 0; c < kFallbackStep; c++) {
                            const uint32_t l = base + 64 * c + lane;
                            const bool in = l < ncand;
                            const unsigned long long m = in ? a.fe_mask[ent.x + l] : 0ull;
                            q[c] = in ? a.fe_id[ent.x + l] : 0u;
                            ov[c] = (m >> bit) & 1ull;
                        }
                    } else {
                        // the bin list: bbox, then exact coverage of the sample
#pragma unroll
                        for (uint32_t c = 0; c < kFallbackStep; c++) {
                            const uint32_t l = base + 64 * c + lane;
                            q[c] = l < ncand ? pairs[start + l] : 0xFFFFFFFFu;
                        }
#pragma unroll
                        for (uint32_t c = 0; c < kFallbackStep; c++) {
                            const uint2 bb = q[c] != 0xFFFFFFFFu ? bbox[q[c]] : make_uint2(0xffffu, 0u);
                            ov[c] = (int)(bb.x & 0xffffu) <= i && (int)(bb.x >> 16) >= i &&
                                    (int)(bb.y & 0xffffu) <= j && (int)(bb.y >> 16) >= j;
                        }
                    }
#pragma unroll
                    for (uint32_t c = 0; c < kFallbackStep; c++) {
                        bool cov = false;
                        unsigned long long key = 0;
                        if (ov[c]) {
                            const PlaneRec pl = load_whole(a.plane, q[c]);
                            if (kept || pixel_coverage(load_whole(a.cov, q[c]), a.extra, xyp, q[c], i, j)) {
                                cov = true;
                                const float kf = frag_key(pl.A, pl.B, pl.C0, i - (int)(pl.ij & 0xffffu),
                                                          j - (int)(pl.ij >> 16));
                                key = ((unsigned long long)order_code(kf) << 32) | q[c];
                            }
                        }
                        seen += (uint32_t)__popcll(ballot(cov));
                        const bool keep = cov && key > lo && key <= hi;
                        const uint64_t m = ballot(keep);
                        if (keep)
                            s_key[n + rank_below(m)] = key;
                        n += (uint32_t)__popcll(m);
                    }
                    wave_sync();
                }
                if (total == 0)
                    total = seen;
                sort_keys(s_key, n, lane);
                uint32_t cpre[kFallbackColours];  // colours of the next kFallbackColours groups, loaded together
                for (uint32_t base = 0; base < n && !(cut && T < kCutT); base += 64) {
                    const uint32_t e = base + lane;
                    const uint32_t g = (base / 64) % kFallbackColours;
                    if (g == 0) {
#pragma unroll
                        for (uint32_t k = 0; k < kFallbackColours; k++) {
                            const uint32_t ek = e + 64 * k;
                            cpre[k] = ek < n ? a.plane[(uint32_t)(s_key[ek] & 0xffffffffu)].rgba : 0u;
                        }
                    }
                    uint32_t c = cpre[0];
#pragma unroll
                    for (uint32_t k = 0; k + 1 < kFallbackColours; k++)
                        cpre[k] = cpre[k + 1];
                    const uint32_t q = e < n ? (uint32_t)(s_key[e] & 0xffffffffu) : 0u;
                    // colours decoded (or interpolated) by all lanes, then blended
                    // in order, each read from its lane as a uniform value
                    const float4 dl = (a.vcol_in && e < n) ? vertex_colour(a, q, i, j) : decode_rgba(c);
                    const uint32_t lim = min(64u, n - base);
                    uint32_t nb = lim;  // fragments of this group blended
                    if (cut) {
                        nb = 0;
#pragma unroll
                        for (uint32_t s = 0; s < 64; s++) {
                            if (s >= lim || T < kCutT)
                                break;
                            const float4 d = make_float4(lane_float(dl.x, s), lane_float(dl.y, s),
                                                         lane_float(dl.z, s), lane_float(dl.w, s));
                            blend_ftb_cut(d, T, R, G2, B);
                            nb++;
                        }
                    } else {
#pragma unroll
                        for (uint32_t s = 0; s < 64; s++) {
                            if (s >= lim)
                                break;
                            const float4 d = make_float4(lane_float(dl.x, s), lane_float(dl.y, s),
                                                         lane_float(dl.z, s), lane_float(dl.w, s));
                            blend_ftb_dec(d, T, R, G2, B);
                        }
                    }
                    if (DEBUG && a.dbg_ids && lane < nb && obase + done + e < a.dbg_cap)
                        a.dbg_ids[obase + done + e] = q;
                    blended += nb;
                    wave_sync();
                }
                done += n;
                if (n)
                    lo = s_key[n - 1];
                more = cut_round && !(cut && T < kCutT);
                wave_sync();
            }
            if (lane == 0) {
                add_stat(a.ctr, ST_FRAGMENTS, total);
                reinterpret_cast<uint32_t *>(a.out)[p] = pack_rgba8(R, G2, B, 1.0f - T);
                if (DEBUG) {
                    if (a.dbg_rgba)
                        reinterpret_cast<float4 *>(a.dbg_rgba)[p] = make_float4(R, G2, B, 1.0f - T);
                    if (a.dbg_count)
                        a.dbg_count[p] = cut ? blended : total;
                }
            }
            wave_sync();
        }
    }
}

// ------------------------------------------------------ unsorted baseline
//
// Same bins, waves, batches and coverage; each pixel blends its fragments in
// list (= quad index) order with "over", one transposed batch at a time.

struct UnsortedLds {
    uint32_t cand[128];
    uint32_t col[64];
    RowWork rw;
};

template <int NW, bool DEBUG, class Src>
__global__ __launch_bounds__(NW * 64) void k_unsorted(Src src)
{
    __shared__ BinChunk<NW> C;
    __shared__ UnsortedLds Uw[NW];
    uint32_t bin;
    const FrameArgs &a = *frame_of(src, bin);
    const QuadXY *__restrict__ xyp = a.xy;
    const uint2 *__restrict__ bbox = a.bbox;
    const uint32_t *__restrict__ pairs = a.pairs;
    clear_next_counters(a, bin, a.nbins);
    if (a.ctr->error & kErrPairs)
        return;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t bpb = 1u << (a.bin_shift - 3), nb = bpb * bpb;
    const uint32_t start = uniform(a.bin_start[bin]), cnt = uniform(a.bin_count[bin]);
    const uint32_t bx_bin = (bin % a.nbx) * bpb, by_bin = (bin / a.nbx) * bpb;
    UnsortedLds &U = Uw[wave];
    const bool cached = cnt <= list_cap(NW);
    if (cached)
        load_bin_list<NW>(bbox, pairs, C, start, cnt);
    unsigned long long st_ent = 0, st_frag = 0;
    const uint32_t nrounds = (nb + NW - 1) / NW;
    for (uint32_t ri = 0; ri < nrounds; ri++) {
        const uint32_t k = ri * NW + wave;
        const BlockGeom g = block_geom(a, bx_bin + k % bpb, by_bin + k / bpb, k < nb, lane);
        float R = 0.0f, G = 0.0f, B = 0.0f, Al = 0.0f;
        uint32_t nfrag = 0, ntot = 0;
        scan_bin<NW>(bbox, pairs, C, U, start, cnt, cached, g, [&](uint32_t m) {
            CovRec r;
            uint32_t q = 0;
            const bool has = lane < m;
            if (has) {
                q = U.cand[lane];
                r = a.cov[q];
            }
            const uint64_t mk = batch_masks(r, has, a.extra, xyp, q, U.rw, g.px0, g.py0, lane) & g.onmask;
            if (has)
                U.col[lane] = r.rgba;
            ntot += (uint32_t)__popcll(ballot(mk != 0));
            wave_sync();
            uint64_t bits = transpose64(mk, lane);
            if (!g.on)
                bits = 0;
            while (bits) {
                const uint32_t kk = (uint32_t)__builtin_ctzll(bits);
                bits &= bits - 1;
                blend_over_dec(a.vcol_in ? vertex_colour(a, U.cand[kk], g.px, g.py) : decode_rgba(U.col[kk]), R, G,
                               B, Al);
                nfrag++;
            }
            wave_sync();
        });
        if (g.active) {
            if (g.on) {
                reinterpret_cast<uint32_t *>(a.out)[g.pix] = pack_rgba8(R, G, B, Al);
                if (DEBUG) {
                    if (a.dbg_rgba)
                        reinterpret_cast<float4 *>(a.dbg_rgba)[g.pix] = make_float4(R, G, B, Al);
                    if (a.dbg_count)
                        a.dbg_count[g.pix] = nfrag;
                }
            }
            uint32_t wsum = nfrag;
            for (int off = 32; off > 0; off >>= 1)
                wsum += shfl_xor(wsum, off);
            st_ent += ntot;
            st_frag += wsum;
        }
    }
    if (lane == 0) {
        if (st_ent)
            add_stat(a.ctr, ST_ENTRIES, st_ent);
        if (st_frag)
            add_stat(a.ctr, ST_FRAGMENTS, st_frag);
    }
}
// ---------------------------------------------------------- scene upload

__global__ __launch_bounds__(256) void k_transpose_scene(const uint32_t *__restrict__ in, uint32_t n,
                                                         float *__restrict__ v, uint32_t *__restrict__ rgba)
{
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n)
        return;
    const uint32_t *r = in + 13 * (size_t)q;
    for (int c = 0; c < 12; c++)
        v[(size_t)c * n + q] = __uint_as_float(r[c]);
    rgba[q] = r[12];
}

// ---------------------------------------------------------------- launches


static hipError_t launch_setup_and_bins(const FrameArgs &a, hipStream_t s, hipEvent_t *ev, bool bins)
{
    const OneFrame f{a};
    // single frames find their counters zeroed by the previous frame
    if (!a.ctr_next)
        hipLaunchKernelGGL(k_frame_begin<OneFrame>, dim3(1), dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_setup<OneFrame>, dim3((a.n + 255) / 256), dim3(256 / kSetupQPL), 0, s, f);
    if (ev)
        (void)hipEventRecord(ev[1], s);
    if (!bins)
        return hipGetLastError();
    if (a.bin_waves == kBin4Waves) {
        if (count4_waves(a.unit_quads) == 16)
            hipLaunchKernelGGL((k_bin_count4<OneFrame, 16>), dim3(a.nunits), dim3(16 * 64),
                               a.nbins * 4 * (a.bin_px ? 2 : 1), s, f);
        else
            hipLaunchKernelGGL((k_bin_count4<OneFrame, 4>), dim3(a.nunits), dim3(4 * 64),
                               a.nbins * 4 * (a.bin_px ? 2 : 1), s, f);
    } else {
        hipLaunchKernelGGL(k_bin_count<OneFrame>, dim3(a.nunits), dim3(64), a.nbins * 4, s, f);
    }
    if (ev)
        (void)hipEventRecord(ev[2], s);
    hipLaunchKernelGGL(k_bin_scan<OneFrame>, dim3(scan_groups(a.nbins)), dim3(kScanWaves * 64), 0, s, f);
    if (ev)
        (void)hipEventRecord(ev[3], s);
    if (a.bin_waves == kBin4Waves)
        hipLaunchKernelGGL(k_bin_scatter4<OneFrame>, dim3(a.nunits * scatter_bands(a.nbx, a.nby)),
                           dim3(kBin4Waves * 64), kBin4Waves * band_bins(a.nbx, a.nby) * 4, s, f);
    else
        hipLaunchKernelGGL(k_bin_scatter<OneFrame>, dim3(a.nunits), dim3(64), a.nbins * 4, s, f);
    if (ev)
        (void)hipEventRecord(ev[4], s);
    return hipGetLastError();
}

hipError_t launch_setup_only(const FrameArgs &a, hipStream_t s)
{
    return launch_setup_and_bins(a, s, nullptr, false);
}

hipError_t launch_binning_only(const FrameArgs &a, hipStream_t s)
{
    return launch_setup_and_bins(a, s, nullptr, true);
}

bool sorter_depth_supported(int k)
{
    return k == 2 || k == 4 || k == 8 || k == 12 || k == 16 || k == 24 || k == 32;
}

// Raster (one workgroup per bin), then the exact pass.
// Raster workgroups of a frame: one per bin, twice that with density classes.
static uint32_t raster_grid(const FrameArgs &a) { return a.k_low ? 2 * a.nbins : a.nbins; }

// Raster (one workgroup per bin), then the exact pass.
template <int K, bool DEBUG, bool CUT, bool VCOL>
static void launch_sorted(const FrameArgs &a, hipStream_t s, hipEvent_t *ev)
{
    const OneFrame f{a};
    // the parity dump keeps one more id per sorter slot: past depth 4 (and
    // with the cutoff or vertex colours) its kernels do not fit 16 waves'
    // registers and take 8, as do cutoff and vertex-colour kernels past depth
    // 8 (the image is the same)
    constexpr bool wide_dbg = (DEBUG && (K > 4 || CUT || VCOL)) || ((CUT || VCOL) && K > 8);
    const uint32_t nw = min(raster_waves_for(a.bin_shift, K), wide_dbg ? 8u : 16u);
    if (nw == 4)
        hipLaunchKernelGGL((k_raster<K, DEBUG, OneFrame, 4, CUT, VCOL>), dim3(raster_grid(a)), dim3(4 * 64), 0, s, f);
    else if (nw == 8)
        hipLaunchKernelGGL((k_raster<K, DEBUG, OneFrame, 8, CUT, VCOL>), dim3(raster_grid(a)), dim3(8 * 64), 0, s, f);
    else if constexpr (K <= 12 && !wide_dbg)
        hipLaunchKernelGGL((k_raster<K, DEBUG, OneFrame, 16, CUT, VCOL>), dim3(raster_grid(a)), dim3(16 * 64), 0, s, f);
    if (ev) {
        (void)hipEventRecord(ev[5], s);
        (void)hipEventRecord(ev[6], s);
    }
    hipLaunchKernelGGL((k_fallback<DEBUG, OneFrame>), dim3(kFallbackGrid), dim3(kFallbackWaves * 64),
                       kFallbackLds, s, f);
    if (ev)
        (void)hipEventRecord(ev[7], s);
}

template <bool DEBUG, bool CUT, bool VCOL>
static void launch_sorted_k(const FrameArgs &a, int k, hipStream_t s, hipEvent_t *ev)
{
    switch (k) {
    case 2: launch_sorted<2, DEBUG, CUT, VCOL>(a, s, ev); break;
    case 4: launch_sorted<4, DEBUG, CUT, VCOL>(a, s, ev); break;
    case 8: launch_sorted<8, DEBUG, CUT, VCOL>(a, s, ev); break;
    case 12: launch_sorted<12, DEBUG, CUT, VCOL>(a, s, ev); break;
    case 16: launch_sorted<16, DEBUG, CUT, VCOL>(a, s, ev); break;
    case 24: launch_sorted<VCOL ? 16 : 24, DEBUG, CUT, VCOL>(a, s, ev); break;
    default: launch_sorted<VCOL ? 16 : 32, DEBUG, CUT, VCOL>(a, s, ev); break;
    }
}

template <bool DEBUG>
static void launch_unsorted(const FrameArgs &a, hipStream_t s)
{
    const OneFrame f{a};
    switch (raster_waves(a.bin_shift)) {
    case 4: hipLaunchKernelGGL((k_unsorted<4, DEBUG, OneFrame>), dim3(a.nbins), dim3(4 * 64), 0, s, f); break;
    case 8: hipLaunchKernelGGL((k_unsorted<8, DEBUG, OneFrame>), dim3(a.nbins), dim3(8 * 64), 0, s, f); break;
    default: hipLaunchKernelGGL((k_unsorted<16, DEBUG, OneFrame>), dim3(a.nbins), dim3(16 * 64), 0, s, f); break;
    }
}

hipError_t launch_frame(const FrameArgs &a, int sorter_depth, int unsorted, hipStream_t s, hipEvent_t *ev)
{
    if (ev)
        (void)hipEventRecord(ev[0], s);
    hipError_t e = launch_setup_and_bins(a, s, ev, true);
    if (e != hipSuccess)
        return e;
    const bool dbg = a.dbg_rgba || a.dbg_count || a.dbg_flag || a.dbg_ids;
    if (unsorted) {
        if (dbg)
            launch_unsorted<true>(a, s);
        else
            launch_unsorted<false>(a, s);
        if (ev) {
            (void)hipEventRecord(ev[5], s);
            (void)hipEventRecord(ev[6], s);
            (void)hipEventRecord(ev[7], s);
        }
    } else if (dbg) {
        if (a.vcol_in)
            launch_sorted_k<true, false, true>(a, sorter_depth, s, ev);
        else if (a.alpha_cut)
            launch_sorted_k<true, true, false>(a, sorter_depth, s, ev);
        else
            launch_sorted_k<true, false, false>(a, sorter_depth, s, ev);
    } else if (a.vcol_in) {
        launch_sorted_k<false, false, true>(a, sorter_depth, s, ev);
    } else if (a.alpha_cut) {
        launch_sorted_k<false, true, false>(a, sorter_depth, s, ev);
    } else {
        launch_sorted_k<false, false, false>(a, sorter_depth, s, ev);
    }
    return hipGetLastError();
}

// --------------------------------------------------------- batched launches

// A frame map for one stage: wg(f) workgroups for frame f (0 to skip it).
template <typename F>
static FrameMap stage_map(const FrameArgs *dev, uint32_t nf, F &&wg)
{
    FrameMap m{};
    m.tab = dev;
    m.nf = nf;
    uint32_t t = 0;
    for (uint32_t f = 0; f < nf; f++) {
        m.wg0[f] = t;
        t += wg(f);
    }
    m.wg0[nf] = t;
    return m;
}

template <int K, bool CUT, bool VCOL>
static void launch_raster_group(const FrameMap &m, uint32_t nw, hipStream_t s)
{
    // cutoff and vertex-colour kernels past depth 8 do not fit 16 waves'
    // registers: they take 8 (the frames' entry regions hold 16)
    constexpr bool narrow = (CUT || VCOL) && K > 8;
    if (narrow && nw == 16)
        nw = 8;
    if (nw == 4)
        hipLaunchKernelGGL((k_raster<K, false, FrameMap, 4, CUT, VCOL>), dim3(m.wg0[m.nf]), dim3(4 * 64), 0, s, m);
    else if (nw == 8)
        hipLaunchKernelGGL((k_raster<K, false, FrameMap, 8, CUT, VCOL>), dim3(m.wg0[m.nf]), dim3(8 * 64), 0, s, m);
    else if constexpr (K <= 12 && !narrow)
        hipLaunchKernelGGL((k_raster<K, false, FrameMap, 16, CUT, VCOL>), dim3(m.wg0[m.nf]), dim3(16 * 64), 0, s, m);
}

template <bool CUT, bool VCOL>
static void raster_group_k(int K, const FrameMap &mr, uint32_t nw, hipStream_t s)
{
    switch (K) {
    case 2: launch_raster_group<2, CUT, VCOL>(mr, nw, s); break;
    case 4: launch_raster_group<4, CUT, VCOL>(mr, nw, s); break;
    case 8: launch_raster_group<8, CUT, VCOL>(mr, nw, s); break;
    case 12: launch_raster_group<12, CUT, VCOL>(mr, nw, s); break;
    case 16: launch_raster_group<16, CUT, VCOL>(mr, nw, s); break;
    case 24: launch_raster_group<VCOL ? 16 : 24, CUT, VCOL>(mr, nw, s); break;
    default: launch_raster_group<VCOL ? 16 : 32, CUT, VCOL>(mr, nw, s); break;
    }
}

hipError_t launch_batch(const FrameArgs *host, const FrameArgs *dev, const int *sorter_depth, uint32_t nf,
                        hipStream_t s)
{
    if (nf == 0)
        return hipSuccess;
    if (nf > kMaxBatch)
        return hipErrorInvalidValue;
    uint32_t max_bins = 0;
    for (uint32_t f = 0; f < nf; f++)
        max_bins = std::max(max_bins, host[f].nbins);
    const FrameMap one = stage_map(dev, nf, [](uint32_t) { return 1u; });
    hipLaunchKernelGGL(k_frame_begin<FrameMap>, dim3(nf), dim3(256), 0, s, one);
    const FrameMap ms = stage_map(dev, nf, [&](uint32_t f) { return (host[f].n + 255) / 256; });
    hipLaunchKernelGGL(k_setup<FrameMap>, dim3(ms.wg0[nf]), dim3(256 / kSetupQPL), 0, s, ms);
    // binning: frames with few bins use the four-wave kernels (one launch
    // each over those frames), the others the one-wave kernels
    uint32_t max_bins4 = 0;
    for (uint32_t f = 0; f < nf; f++)
        if (host[f].bin_waves == kBin4Waves)
            max_bins4 = std::max(max_bins4, host[f].nbins);
    const FrameMap mu = stage_map(dev, nf, [&](uint32_t f) { return host[f].bin_waves == 1 ? host[f].nunits : 0u; });
    const FrameMap mu4 =
        stage_map(dev, nf, [&](uint32_t f) { return host[f].bin_waves == kBin4Waves ? host[f].nunits : 0u; });
    // the scatter: one workgroup per unit and band of bin rows
    uint32_t max_band4 = 0;
    for (uint32_t f = 0; f < nf; f++)
        if (host[f].bin_waves == kBin4Waves)
            max_band4 = std::max(max_band4, band_bins(host[f].nbx, host[f].nby));
    const FrameMap mb4 = stage_map(dev, nf, [&](uint32_t f) {
        return host[f].bin_waves == kBin4Waves ? host[f].nunits * scatter_bands(host[f].nbx, host[f].nby) : 0u;
    });
    if (mu.wg0[nf])
        hipLaunchKernelGGL(k_bin_count<FrameMap>, dim3(mu.wg0[nf]), dim3(64), max_bins * 4, s, mu);
    if (mu4.wg0[nf]) {
        uint32_t max_uq = 0;
        for (uint32_t f = 0; f < nf; f++)
            if (host[f].bin_waves == kBin4Waves)
                max_uq = std::max(max_uq, host[f].unit_quads);
        if (count4_waves(max_uq) == 16)
            hipLaunchKernelGGL((k_bin_count4<FrameMap, 16>), dim3(mu4.wg0[nf]), dim3(16 * 64), max_bins4 * 8, s, mu4);
        else
            hipLaunchKernelGGL((k_bin_count4<FrameMap, 4>), dim3(mu4.wg0[nf]), dim3(4 * 64), max_bins4 * 8, s, mu4);
    }
    const FrameMap mt =
        stage_map(dev, nf, [&](uint32_t f) { return scan_groups(host[f].nbins); });
    hipLaunchKernelGGL(k_bin_scan<FrameMap>, dim3(mt.wg0[nf]), dim3(kScanWaves * 64), 0, s, mt);
    if (mu.wg0[nf])
        hipLaunchKernelGGL(k_bin_scatter<FrameMap>, dim3(mu.wg0[nf]), dim3(64), max_bins * 4, s, mu);
    if (mb4.wg0[nf])
        hipLaunchKernelGGL(k_bin_scatter4<FrameMap>, dim3(mb4.wg0[nf]), dim3(kBin4Waves * 64),
                           kBin4Waves * max_band4 * 4, s, mb4);
    static const int kDepths[] = {2, 4, 8, 12, 16, 24, 32};
    static const uint32_t kWaveCounts[] = {4, 8, 16};
    // raster launches, one per (depth, waves, cutoff) present
    for (int K : kDepths) {
        for (uint32_t nw : kWaveCounts) {
            for (uint32_t mode = 0; mode < 3; mode++) {  // flat, flat with the cutoff, vertex colours
                auto in_group = [&](uint32_t f) {
                    const uint32_t fm = host[f].vcol_in ? 2u : (host[f].alpha_cut ? 1u : 0u);
                    return sorter_depth[f] == K && raster_waves_for(host[f].bin_shift, K) == nw && fm == mode;
                };
                bool any = false;
                for (uint32_t f = 0; f < nf; f++)
                    any = any || in_group(f);
                if (!any)
                    continue;
                const FrameMap mr =
                    stage_map(dev, nf, [&](uint32_t f) { return in_group(f) ? raster_grid(host[f]) : 0u; });
                if (mode == 1)
                    raster_group_k<true, false>(K, mr, nw, s);
                else if (mode == 2)
                    raster_group_k<false, true>(K, mr, nw, s);
                else
                    raster_group_k<false, false>(K, mr, nw, s);
            }
        }
    }
    const FrameMap mf = stage_map(dev, nf, [&](uint32_t) { return 0u; });  // frames walked in turn
    hipLaunchKernelGGL((k_fallback<false, FrameMap>), dim3(kFallbackGrid), dim3(kFallbackWaves * 64), kFallbackLds,
                       s, mf);
    return hipGetLastError();
}

hipError_t launch_transpose_scene(const void *quads_dev, uint32_t n, float *v, uint32_t *rgba, hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose_scene, dim3((n + 255) / 256), dim3(256), 0, s,
                       (const uint32_t *)quads_dev, n, v, rgba);
    return hipGetLastError();
}

}  // namespace lr
