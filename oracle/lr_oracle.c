/*
 * CPU oracle for exact order-independent transparency of planar quads
 * (LucidRaster, arXiv 2405.13364).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition the GPU
 * rasterizer is checked against.  Only the tests, the smoke check and the CPU
 * timing leg of the benchmark may load it; the rendering library never does.
 * It shares no code, header, table or constant with the HIP path.
 *
 * What it computes (Section 1 states the problem: find every fragment that
 * contributes to a pixel, sort, blend in order; Section 2 "Pipeline
 * description" fixes quads as the primitive and front-to-back blending from
 * transparent black, Stage 3 "Sample blending"):
 *
 *   for every pixel centre, every visible quad whose area covers it gives one
 *   fragment; fragments are ordered nearest first (ties by quad index) and
 *   blended front to back.
 *
 * The paper leaves the numeric details open; the readings used here (all
 * IEEE-754 binary64, round to nearest even, no contraction except where fma()
 * is written -- build with -ffp-contract=off):
 *
 *   camera   c_i = fma(R_i2, d_2, fma(R_i1, d_1, R_i0 * d_0)), d = v - pos
 *   near     any c.z <= z_near                       -> culled (NEAR)
 *   project  sx = fma(f, c.x/c.z, cx), sy = fma(-f, c.y/c.z, cy),
 *            f = (H/2) / tan(fov_y/2) on the host, cx = W/2, cy = H/2
 *   guard    any |sx| or |sy| >= 2^15 or non-finite  -> culled (GUARD)
 *   snap     X = rint(256 sx), Y = rint(256 sy)   (1/256 pixel grid)
 *   cover    pixel (i,j) samples S = (256 i + 128, 256 j + 128); the quad is
 *            the union of triangles (P0,P1,P2) and (P0,P2,P3); a triangle
 *            with zero doubled area is empty; the others are oriented to
 *            positive doubled area and contain S when every edge function is
 *            > 0, or == 0 on a top-left edge (dy < 0, or dy == 0 and dx > 0).
 *            Both triangles empty                    -> culled (DEGENERATE)
 *   bbox     i in [ceil((Xmin-128)/256), floor((Xmax-128)/256)] clamped to
 *            the screen; empty                       -> culled (NO_SAMPLE)
 *   depth    plane through the vertex centroid with normal = cross product
 *            of the diagonals; reciprocal view depth is affine on screen:
 *            1/z(i,j) = A (i-imin) + B (j-jmin) + C0.  A degenerate or
 *            non-finite plane                        -> culled (EDGE_ON)
 *   key      k = (float) fma(A, i-imin, fma(B, j-jmin, C0)), clamped to +0
 *            when not positive; larger k is nearer.
 *   order    ascending (~bits(k) << 32 | quad index)
 *   blend    T = 1, C = 0; per fragment a = A8/255, C += T a rgb/255,
 *            T *= 1 - a; output premultiplied (C, 1 - T); RGBA8 is
 *            clamp(floor(255 x + 0.5)).
 *   unsorted quad index order, "over": C = a c + (1-a) C, al = a + (1-a) al.
 *   vertex colours (optional; Stage 3 "Sample shading" interpolates
 *            per-vertex attributes): a covered sample takes triangle T0 if
 *            T0 covers it, else T1; its colour is the barycentric mix of
 *            that triangle's vertex colours (bytes / 255) at the point where
 *            the ray through the pixel centre meets the triangle's plane in
 *            camera space: with r = ((px - cx)/f, -(py - cy)/f, 1) and the
 *            triangle's camera-space vertices (A, B, C), the weights are
 *            r.(BxC), r.(CxA), r.(AxB) over their sum (perspective-correct
 *            interpolation).  The colour is blended unrounded.
 *   cutoff   (optional; Stage 3 "Sample blending" stops a pixel once its
 *            accumulated alpha passes a threshold) a pixel stops after the
 *            first fragment that brings its transmittance below 2^-20; the
 *            colour is still blended in binary64, but that decision is an
 *            integer one (how many fragments) and is taken in single
 *            precision as a shader would: a32 = fl(fl(A8) * fl(1/255)),
 *            T32 = fl(T32 * fl(1 - a32)) from T32 = 1, every fl() binary32
 *            round to nearest even.  Everything after the stop is left
 *            out, so the colour differs from the uncut one by less than
 *            2^-20 per channel.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LRO_VISIBLE 0
#define LRO_NEAR 1
#define LRO_GUARD 2
#define LRO_DEGENERATE 3
#define LRO_NO_SAMPLE 4
#define LRO_EDGE_ON 5
#define LRO_BACKFACE 6

typedef struct {
    float pos[3];
    float rot[9];
    float fov_y;
    float z_near;
} lro_camera;

/* Focal length in pixels (host libm tan). */
double lro_focal(uint32_t height, float fov_y)
{
    return (0.5 * (double)height) / tan(0.5 * (double)fov_y);
}

static int64_t edge_fn(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py)
{
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

/* Coverage of sample (sx, sy) by the triangle (a, b, c) under the top-left
 * rule.  Returns 0 for a zero-area triangle. */
static int tri_covers(const int32_t *X, const int32_t *Y, int ia, int ib, int ic, int64_t sx,
                      int64_t sy)
{
    int64_t ax = X[ia], ay = Y[ia], bx = X[ib], by = Y[ib], cx = X[ic], cy = Y[ic];
    int64_t area2 = edge_fn(ax, ay, bx, by, cx, cy);
    if (area2 == 0)
        return 0;
    if (area2 < 0) {
        int64_t tx = bx, ty = by;
        bx = cx; by = cy;
        cx = tx; cy = ty;
    }
    const int64_t vx[3] = {ax, bx, cx}, vy[3] = {ay, by, cy};
    for (int e = 0; e < 3; e++) {
        int64_t x0 = vx[e], y0 = vy[e], x1 = vx[(e + 1) % 3], y1 = vy[(e + 1) % 3];
        int64_t ev = edge_fn(x0, y0, x1, y1, sx, sy);
        int64_t dx = x1 - x0, dy = y1 - y0;
        int top_left = (dy < 0) || (dy == 0 && dx > 0);
        if (ev < 0 || (ev == 0 && !top_left))
            return 0;
    }
    return 1;
}

/* Does quad (X[4], Y[4]) cover the centre of pixel (i, j)?  One fragment at
 * most: the union of its two triangles. */
int lro_covers(const int32_t *X, const int32_t *Y, int32_t i, int32_t j)
{
    int64_t sx = 256 * (int64_t)i + 128, sy = 256 * (int64_t)j + 128;
    return tri_covers(X, Y, 0, 1, 2, sx, sy) || tri_covers(X, Y, 0, 2, 3, sx, sy);
}

static int64_t floordiv256(int64_t a) { return a >= 0 ? a / 256 : -((-a + 255) / 256); }

/*
 * Per-quad setup.  v: float[n][4][3] world vertices.  Outputs per quad:
 * X, Y int32[n][4] snapped vertices; bbox int32[n][4] = (imin, imax, jmin,
 * jmax); A, B, C0 double[n]; cull uint8[n] (0 = visible, else the first
 * failing test in the order near, guard, degenerate, no-sample, edge-on,
 * back-facing); camv double[n][4][3] camera-space vertices (may be NULL).
 * Fields of culled quads are left as far as they were computed.
 *
 * Back-face culling (cull_back != 0; Stage 1 culls primitives facing away
 * from the camera): dd = n . m, with n the cross product of the diagonals
 * and m the vertex centroid in camera space, is positive when the vertices
 * wind counter-clockwise on the display (screen y down), as front faces do
 * in OpenGL; a quad with dd < 0 is back-facing.
 */
void lro_setup(uint32_t n, const float *v, const lro_camera *cam, uint32_t W, uint32_t H, double f,
               int32_t *X, int32_t *Y, int32_t *bbox, double *A, double *B, double *C0,
               uint8_t *cull, int cull_back, double *camv)
{
    const double cx = 0.5 * (double)W, cy = 0.5 * (double)H;
    double R[9], P[3];
    for (int k = 0; k < 9; k++)
        R[k] = (double)cam->rot[k];
    for (int k = 0; k < 3; k++)
        P[k] = (double)cam->pos[k];
    const double znear = (double)cam->z_near;

    for (uint32_t q = 0; q < n; q++) {
        double c[4][3];
        int32_t *x = X + 4 * (size_t)q, *y = Y + 4 * (size_t)q, *bb = bbox + 4 * (size_t)q;
        A[q] = B[q] = C0[q] = 0.0;
        memset(x, 0, 16);
        memset(y, 0, 16);
        bb[0] = 1; bb[1] = 0; bb[2] = 1; bb[3] = 0;
        /* camera transform */
        for (int k = 0; k < 4; k++) {
            const float *vk = v + 12 * (size_t)q + 3 * k;
            double d0 = (double)vk[0] - P[0], d1 = (double)vk[1] - P[1], d2 = (double)vk[2] - P[2];
            for (int r = 0; r < 3; r++)
                c[k][r] = fma(R[3 * r + 2], d2, fma(R[3 * r + 1], d1, R[3 * r + 0] * d0));
        }
        if (camv)  /* camera-space vertices, for vertex colours */
            for (int k = 0; k < 4; k++)
                for (int r = 0; r < 3; r++)
                    camv[12 * (size_t)q + 3 * k + r] = c[k][r];
        /* near plane */
        int near = 0;
        for (int k = 0; k < 4; k++)
            if (!(c[k][2] > znear))
                near = 1;
        if (near) {
            cull[q] = LRO_NEAR;
            continue;
        }
        /* projection and guard band */
        double sx[4], sy[4];
        int guard = 0;
        for (int k = 0; k < 4; k++) {
            double qx = c[k][0] / c[k][2];
            double qy = c[k][1] / c[k][2];
            sx[k] = fma(f, qx, cx);
            sy[k] = fma(-f, qy, cy);
            if (!(fabs(sx[k]) < 32768.0) || !(fabs(sy[k]) < 32768.0))
                guard = 1;
        }
        if (guard) {
            cull[q] = LRO_GUARD;
            continue;
        }
        /* snap to the 1/256 pixel grid */
        for (int k = 0; k < 4; k++) {
            x[k] = (int32_t)rint(sx[k] * 256.0);
            y[k] = (int32_t)rint(sy[k] * 256.0);
        }
        /* degenerate: both triangles have zero area */
        int64_t a0 = edge_fn(x[0], y[0], x[1], y[1], x[2], y[2]);
        int64_t a1 = edge_fn(x[0], y[0], x[2], y[2], x[3], y[3]);
        if (a0 == 0 && a1 == 0) {
            cull[q] = LRO_DEGENERATE;
            continue;
        }
        /* pixel bounding box of the sample points inside the vertex bounds */
        int64_t xmin = x[0], xmax = x[0], ymin = y[0], ymax = y[0];
        for (int k = 1; k < 4; k++) {
            if (x[k] < xmin) xmin = x[k];
            if (x[k] > xmax) xmax = x[k];
            if (y[k] < ymin) ymin = y[k];
            if (y[k] > ymax) ymax = y[k];
        }
        int64_t imin = floordiv256(xmin - 128 + 255), imax = floordiv256(xmax - 128);
        int64_t jmin = floordiv256(ymin - 128 + 255), jmax = floordiv256(ymax - 128);
        if (imin < 0) imin = 0;
        if (jmin < 0) jmin = 0;
        if (imax > (int64_t)W - 1) imax = (int64_t)W - 1;
        if (jmax > (int64_t)H - 1) jmax = (int64_t)H - 1;
        bb[0] = (int32_t)imin; bb[1] = (int32_t)imax; bb[2] = (int32_t)jmin; bb[3] = (int32_t)jmax;
        if (imin > imax || jmin > jmax) {
            cull[q] = LRO_NO_SAMPLE;
            continue;
        }
        /* depth plane: normal from the diagonals, through the centroid */
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
        if (dd == 0.0 || !isfinite(dd)) {
            cull[q] = LRO_EDGE_ON;
            continue;
        }
        double g = f * dd;
        double a = nn[0] / g;
        double b = (-nn[1]) / g;
        double u0 = ((double)imin + 0.5) - cx;
        double w0 = ((double)jmin + 0.5) - cy;
        double t1 = nn[0] * u0, t2 = nn[1] * w0;
        double c0 = ((t1 - t2) + nn[2] * f) / g;
        if (!isfinite(a) || !isfinite(b) || !isfinite(c0)) {
            cull[q] = LRO_EDGE_ON;
            continue;
        }
        A[q] = a; B[q] = b; C0[q] = c0;
        if (cull_back && dd < 0.0) {
            cull[q] = LRO_BACKFACE;
            continue;
        }
        cull[q] = LRO_VISIBLE;
    }
}

/* Depth key of quad q at pixel (i, j): larger is nearer, never negative. */
float lro_key(double a, double b, double c0, const int32_t *bb, int32_t i, int32_t j)
{
    double v = fma(a, (double)(i - bb[0]), fma(b, (double)(j - bb[2]), c0));
    float k = (float)v;
    if (!(k > 0.0f))
        k = 0.0f;
    return k;
}

static uint64_t order_key(float k, uint32_t id)
{
    uint32_t bits;
    memcpy(&bits, &k, 4);
    return ((uint64_t)(~bits) << 32) | (uint64_t)id;
}

typedef struct {
    uint64_t key;
    uint32_t rgba;
} frag_t;

static int cmp_frag(const void *pa, const void *pb)
{
    uint64_t a = ((const frag_t *)pa)->key, b = ((const frag_t *)pb)->key;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* A fragment's colour: R, G, B, A in [0, 1]. */
typedef struct {
    double c[4];
} colour_t;

static colour_t colour_of(uint32_t c)
{
    colour_t o;
    for (int ch = 0; ch < 4; ch++)
        o.c[ch] = (double)((c >> (8 * ch)) & 255u) / 255.0;
    return o;
}

/* One front-to-back step: a fragment of colour col under transmittance T. */
static void blend_step(const colour_t *col, double *T, double C[3])
{
    double a = col->c[3];
    double w = *T * a;
    for (int ch = 0; ch < 3; ch++)
        C[ch] = C[ch] + w * col->c[ch];
    *T = *T * (1.0 - a);
}

/* Vertex colours of a quad: camera-space vertices cv[4][3], colours rgba4[4],
 * snapped vertices X, Y (for the triangle choice) and the camera's f, cx,
 * cy; the colour at pixel (i, j), which the quad covers. */
typedef struct {
    const double *cv;
    const uint32_t *rgba4;
    const int32_t *X, *Y;
    double f, cx, cy;
} vquad_t;

static void cross3(const double *a, const double *b, double *o)
{
    double p, s;
    p = a[1] * b[2]; s = a[2] * b[1]; o[0] = p - s;
    p = a[2] * b[0]; s = a[0] * b[2]; o[1] = p - s;
    p = a[0] * b[1]; s = a[1] * b[0]; o[2] = p - s;
}

static colour_t vertex_colour(const vquad_t *vq, int32_t i, int32_t j)
{
    int64_t sx = 256 * (int64_t)i + 128, sy = 256 * (int64_t)j + 128;
    int t[3] = {0, 1, 2};
    if (!tri_covers(vq->X, vq->Y, 0, 1, 2, sx, sy)) {
        t[1] = 2;
        t[2] = 3;
    }
    const double r[3] = {(((double)i + 0.5) - vq->cx) / vq->f, -((((double)j + 0.5) - vq->cy) / vq->f), 1.0};
    double w[3], sum = 0.0;
    for (int k = 0; k < 3; k++) {
        double n[3];
        cross3(vq->cv + 3 * t[(k + 1) % 3], vq->cv + 3 * t[(k + 2) % 3], n);
        w[k] = (r[0] * n[0] + r[1] * n[1]) + r[2] * n[2];
        sum += w[k];
    }
    colour_t o;
    for (int ch = 0; ch < 4; ch++) {
        double acc = 0.0;
        for (int k = 0; k < 3; k++)
            acc += (w[k] / sum) * ((double)((vq->rgba4[t[k]] >> (8 * ch)) & 255u) / 255.0);
        o.c[ch] = acc;
    }
    return o;
}

/* Front-to-back blend of fragments already in order (colours col[k]). */
static void blend_front_to_back(const colour_t *col, uint32_t cnt, double out[4])
{
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    for (uint32_t k = 0; k < cnt; k++)
        blend_step(&col[k], &T, C);
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
}

/* Transmittance below which a pixel stops, with the cutoff on. */
#define LRO_CUT_T (1.0f / 1048576.0f)

/* The same blend with the transmittance cutoff; returns how many fragments
 * (a prefix of fr) were blended. */
static uint32_t blend_front_to_back_cut(const frag_t *fr, uint32_t cnt, double out[4])
{
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    float T32 = 1.0f;
    const float inv255 = 1.0f / 255.0f;
    uint32_t k = 0;
    while (k < cnt) {
        uint32_t c = fr[k].rgba;
        const colour_t col = colour_of(c);
        blend_step(&col, &T, C);
        float a32 = (float)(c >> 24) * inv255;
        T32 = T32 * (1.0f - a32);
        k++;
        if (T32 < LRO_CUT_T)
            break;
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    return k;
}

/* "Over" blend in quad index order (the unsorted baseline). */
static void blend_over(const colour_t *col, uint32_t cnt, double out[4])
{
    double C[3] = {0.0, 0.0, 0.0}, al = 0.0;
    for (uint32_t k = 0; k < cnt; k++) {
        double a = col[k].c[3];
        for (int ch = 0; ch < 3; ch++)
            C[ch] = a * col[k].c[ch] + (1.0 - a) * C[ch];
        al = a + (1.0 - a) * al;
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = al;
}

/* Colours of the cnt fragments of pixel (i, j): flat, or from the quads'
 * vertex colours (vcol != NULL: rgba4[n][4], camv[n][4][3]). */
static void fragment_colours(const frag_t *fr, uint32_t cnt, const uint32_t *vcol, const double *camv,
                             const int32_t *X, const int32_t *Y, double f, double cx, double cy,
                             int32_t i, int32_t j, colour_t *col)
{
    for (uint32_t k = 0; k < cnt; k++) {
        if (!vcol) {
            col[k] = colour_of(fr[k].rgba);
        } else {
            const uint32_t q = (uint32_t)(fr[k].key & 0xffffffffu);
            vquad_t vq = {camv + 12 * (size_t)q, vcol + 4 * (size_t)q, X + 4 * (size_t)q, Y + 4 * (size_t)q,
                          f, cx, cy};
            col[k] = vertex_colour(&vq, i, j);
        }
    }
}

static uint8_t to_u8(double x)
{
    double y = floor(255.0 * x + 0.5);
    if (y < 0.0) y = 0.0;
    if (y > 255.0) y = 255.0;
    return (uint8_t)y;
}

/*
 * Whole-frame render.  Per pixel it gathers every covering visible quad,
 * orders the fragments (sorted, or quad index order in the unsorted mode) and
 * blends them.  Outputs: rgba_f64[H][W][4], rgba8[H][W][4], count[H][W],
 * order_offsets[W*H+1] and order_ids[...] (fragment quad indices in blend
 * order; pass NULL to skip).  Returns the total number of fragments, or -1 on
 * allocation failure.
 *
 * The work is split over `threads` workers (0 or 1: serial) by bands
 * of kBandRows screen rows taken from a shared counter.  A band's worker
 * visits every quad, in index order, for the rows of its band only, so every
 * pixel gets the same fragment list, in the same order, as one serial walk
 * over the quads; the per-pixel arithmetic is the same code either way.
 */
#define LRO_BAND_ROWS 8u

typedef struct {
    /* inputs */
    uint32_t n, W, H;
    const int32_t *X, *Y, *bbox;
    const double *A, *B, *C0;
    const uint8_t *cull;
    const uint32_t *rgba;
    int mode;               /* 0 sorted, 1 unsorted (quad order), 2 sorted with the cutoff */
    const uint32_t *vcol;   /* vertex colours [n][4], or NULL */
    const double *camv;     /* camera-space vertices [n][4][3] (with vcol) */
    double f;
    /* outputs and work arrays */
    double *rgba_f64;
    uint8_t *rgba8;
    uint32_t *count;
    const uint64_t *off;
    uint64_t *fill;
    frag_t *fr;
    uint32_t *order_ids;
    /* band queue */
    int phase;              /* 0 count, 1 fill, 2 order and blend */
    uint32_t nbands;
    uint32_t next;          /* next band (shared) */
    pthread_mutex_t mu;
} lro_job;

static void band_rows(const lro_job *jb, uint32_t band, int32_t *j0, int32_t *j1)
{
    *j0 = (int32_t)(band * LRO_BAND_ROWS);
    *j1 = (int32_t)(band * LRO_BAND_ROWS + LRO_BAND_ROWS - 1);
    if (*j1 > (int32_t)jb->H - 1)
        *j1 = (int32_t)jb->H - 1;
}

/* Pass 1 (count) or pass 2 (fill) over the quads for rows j0..j1. */
static void band_quads(lro_job *jb, int32_t j0, int32_t j1, int fill_pass)
{
    const uint32_t W = jb->W;
    for (uint32_t q = 0; q < jb->n; q++) {
        if (jb->cull[q] != LRO_VISIBLE)
            continue;
        const int32_t *bb = jb->bbox + 4 * (size_t)q;
        const int32_t ja = bb[2] > j0 ? bb[2] : j0, jz = bb[3] < j1 ? bb[3] : j1;
        for (int32_t j = ja; j <= jz; j++)
            for (int32_t i = bb[0]; i <= bb[1]; i++)
                if (lro_covers(jb->X + 4 * (size_t)q, jb->Y + 4 * (size_t)q, i, j)) {
                    size_t p = (size_t)j * W + i;
                    if (!fill_pass) {
                        jb->count[p]++;
                    } else {
                        float k = lro_key(jb->A[q], jb->B[q], jb->C0[q], bb, i, j);
                        jb->fr[jb->fill[p]].key = order_key(k, q);
                        jb->fr[jb->fill[p]].rgba = jb->rgba[q];
                        jb->fill[p]++;
                    }
                }
    }
}

/* Grows *buf to hold n colours; 0 when memory runs out. */
static int colour_room(colour_t **buf, size_t *cap, size_t n)
{
    if (n <= *cap)
        return 1;
    size_t c = *cap ? *cap : 256;
    while (c < n)
        c *= 2;
    colour_t *nb = (colour_t *)realloc(*buf, c * sizeof(colour_t));
    if (!nb)
        return 0;
    *buf = nb;
    *cap = c;
    return 1;
}

/* Pass 3 for the pixels of rows j0..j1: order and blend. */
static void band_blend(lro_job *jb, int32_t j0, int32_t j1)
{
    colour_t *col = NULL;
    size_t cap = 0;
    const double cx = 0.5 * (double)jb->W, cy = 0.5 * (double)jb->H;
    for (size_t p = (size_t)j0 * jb->W; p < (size_t)(j1 + 1) * jb->W; p++) {
        frag_t *pf = jb->fr + jb->off[p];
        uint32_t cnt = jb->count[p];
        double o[4];
        if (jb->mode != 1)
            qsort(pf, cnt, sizeof(frag_t), cmp_frag);
        if (jb->mode == 2) {
            jb->count[p] = cnt = blend_front_to_back_cut(pf, cnt, o);  /* the blended prefix */
        } else {
            if (!colour_room(&col, &cap, cnt))
                abort();
            fragment_colours(pf, cnt, jb->vcol, jb->camv, jb->X, jb->Y, jb->f, cx, cy, (int32_t)(p % jb->W),
                             (int32_t)(p / jb->W), col);
            if (jb->mode == 1)
                blend_over(col, cnt, o);
            else
                blend_front_to_back(col, cnt, o);
        }
        for (int ch = 0; ch < 4; ch++) {
            if (jb->rgba_f64) jb->rgba_f64[4 * p + ch] = o[ch];
            if (jb->rgba8) jb->rgba8[4 * p + ch] = to_u8(o[ch]);
        }
        if (jb->order_ids)
            for (uint32_t t = 0; t < cnt; t++)
                jb->order_ids[jb->off[p] + t] = (uint32_t)(pf[t].key & 0xffffffffu);
    }
    free(col);
}

static void *band_worker(void *arg)
{
    lro_job *jb = (lro_job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        uint32_t band = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (band >= jb->nbands)
            break;
        int32_t j0, j1;
        band_rows(jb, band, &j0, &j1);
        if (jb->phase == 2)
            band_blend(jb, j0, j1);
        else
            band_quads(jb, j0, j1, jb->phase);
    }
    return NULL;
}

/* Runs one phase over all bands on `threads` workers (the caller is one). */
static void run_phase(lro_job *jb, int phase, uint32_t threads)
{
    jb->phase = phase;
    jb->next = 0;
    pthread_t tid[256];
    uint32_t started = 0;
    for (uint32_t t = 1; t < threads && t < 256; t++)
        if (pthread_create(&tid[started], NULL, band_worker, jb) == 0)
            started++;
    band_worker(jb);
    for (uint32_t t = 0; t < started; t++)
        pthread_join(tid[t], NULL);
}

static uint32_t pick_threads(uint32_t threads)
{
    if (threads == 0)
        return 1u;
    return threads > 256 ? 256u : threads;
}

static void job_init(lro_job *jb, uint32_t n, const int32_t *X, const int32_t *Y, const int32_t *bbox,
                     const double *A, const double *B, const double *C0, const uint8_t *cull,
                     const uint32_t *rgba, uint32_t W, uint32_t H, int mode, uint32_t *count)
{
    memset(jb, 0, sizeof(*jb));
    jb->n = n; jb->W = W; jb->H = H;
    jb->X = X; jb->Y = Y; jb->bbox = bbox;
    jb->A = A; jb->B = B; jb->C0 = C0;
    jb->cull = cull; jb->rgba = rgba; jb->mode = mode;
    jb->count = count;
    jb->nbands = (H + LRO_BAND_ROWS - 1) / LRO_BAND_ROWS;
    pthread_mutex_init(&jb->mu, NULL);
}

/* Fragments of the frame (pass 1 only): count[H][W] and the total. */
int64_t lro_count(uint32_t n, const int32_t *X, const int32_t *Y, const int32_t *bbox,
                  const uint8_t *cull, uint32_t W, uint32_t H, uint32_t *count, uint32_t threads)
{
    lro_job jb;
    job_init(&jb, n, X, Y, bbox, NULL, NULL, NULL, cull, NULL, W, H, 0, count);
    memset(count, 0, (size_t)W * H * sizeof(uint32_t));
    run_phase(&jb, 0, pick_threads(threads));
    pthread_mutex_destroy(&jb.mu);
    uint64_t total = 0;
    for (size_t p = 0; p < (size_t)W * H; p++)
        total += count[p];
    return (int64_t)total;
}

/* mode: 0 sorted, 1 unsorted, 2 sorted with the transmittance cutoff (then
 * count[] holds the blended prefix of each pixel, order_offsets the bounds of
 * the full lists and order_ids their prefixes first; the return value stays
 * the number of covering fragments). */
int64_t lro_render(uint32_t n, const int32_t *X, const int32_t *Y, const int32_t *bbox,
                   const double *A, const double *B, const double *C0, const uint8_t *cull,
                   const uint32_t *rgba, uint32_t W, uint32_t H, int mode, double *rgba_f64,
                   uint8_t *rgba8, uint32_t *count, uint64_t *order_offsets, uint32_t *order_ids,
                   uint32_t threads, const uint32_t *vcol, const double *camv, double f)
{
    const size_t npix = (size_t)W * H;
    threads = pick_threads(threads);
    if (vcol && mode == 2)
        return -2;  /* the cutoff is defined on flat colours only */
    lro_job jb;
    job_init(&jb, n, X, Y, bbox, A, B, C0, cull, rgba, W, H, mode, count);
    jb.vcol = vcol;
    jb.camv = camv;
    jb.f = f;
    uint64_t *off = (uint64_t *)calloc(npix + 1, sizeof(uint64_t));
    if (!off) {
        pthread_mutex_destroy(&jb.mu);
        return -1;
    }
    memset(count, 0, npix * sizeof(uint32_t));
    /* pass 1: fragment count per pixel */
    run_phase(&jb, 0, threads);
    for (size_t p = 0; p < npix; p++)
        off[p + 1] = off[p] + count[p];
    const uint64_t total = off[npix];
    frag_t *fr = (frag_t *)malloc((total ? total : 1) * sizeof(frag_t));
    uint64_t *fill = (uint64_t *)malloc((npix ? npix : 1) * sizeof(uint64_t));
    if (!fr || !fill) {
        free(off); free(fr); free(fill);
        pthread_mutex_destroy(&jb.mu);
        return -1;
    }
    memcpy(fill, off, npix * sizeof(uint64_t));
    jb.off = off;
    jb.fill = fill;
    jb.fr = fr;
    jb.rgba_f64 = rgba_f64;
    jb.rgba8 = rgba8;
    jb.order_ids = order_ids;
    /* pass 2: fragments, appended in quad index order */
    run_phase(&jb, 1, threads);
    /* pass 3: per pixel, order and blend */
    run_phase(&jb, 2, threads);
    if (order_offsets)
        memcpy(order_offsets, off, (npix + 1) * sizeof(uint64_t));
    pthread_mutex_destroy(&jb.mu);
    free(fr); free(fill); free(off);
    return (int64_t)total;
}

/*
 * The same result for a list of pixels, each computed on its own by testing
 * every visible quad (used where a whole frame would take too long).
 * pix[k] = j * W + i.  Outputs per pixel: rgba_f64[k][4], count[k] and, when
 * ids != NULL, offsets[npix+1] / ids[<= ids_cap] in blend order.  Returns
 * the number of fragments over all listed pixels, or -1 when ids_cap is too
 * small or memory runs out.  mode as for lro_render; with the cutoff, counts
 * and ids are those of the blended prefixes.
 */
int64_t lro_pixels(uint32_t n, const int32_t *X, const int32_t *Y, const int32_t *bbox,
                   const double *A, const double *B, const double *C0, const uint8_t *cull,
                   const uint32_t *rgba, uint32_t W, int mode, uint32_t npix,
                   const uint32_t *pix, double *rgba_f64, uint32_t *count, uint64_t *offsets,
                   uint32_t *ids, uint64_t ids_cap, const uint32_t *vcol, const double *camv, double f,
                   uint32_t H)
{
    if (vcol && mode == 2)
        return -2;
    colour_t *col = NULL;
    size_t ccap = 0;
    size_t cap = 1024;
    frag_t *fr = (frag_t *)malloc(cap * sizeof(frag_t));
    if (!fr)
        return -1;
    uint64_t total = 0;
    if (offsets)
        offsets[0] = 0;
    for (uint32_t k = 0; k < npix; k++) {
        int32_t i = (int32_t)(pix[k] % W), j = (int32_t)(pix[k] / W);
        uint32_t cnt = 0;
        for (uint32_t q = 0; q < n; q++) {
            if (cull[q] != LRO_VISIBLE)
                continue;
            const int32_t *bb = bbox + 4 * (size_t)q;
            if (i < bb[0] || i > bb[1] || j < bb[2] || j > bb[3])
                continue;
            if (!lro_covers(X + 4 * (size_t)q, Y + 4 * (size_t)q, i, j))
                continue;
            if (cnt == cap) {
                cap *= 2;
                frag_t *nf = (frag_t *)realloc(fr, cap * sizeof(frag_t));
                if (!nf) {
                    free(fr);
                    free(col);
                    return -1;
                }
                fr = nf;
            }
            fr[cnt].key = order_key(lro_key(A[q], B[q], C0[q], bb, i, j), q);
            fr[cnt].rgba = rgba[q];
            cnt++;
        }
        double o[4];
        if (mode != 1)
            qsort(fr, cnt, sizeof(frag_t), cmp_frag);
        if (mode == 2) {
            cnt = blend_front_to_back_cut(fr, cnt, o);  /* the blended prefix */
        } else {
            if (!colour_room(&col, &ccap, cnt)) {
                free(fr);
                return -1;
            }
            fragment_colours(fr, cnt, vcol, camv, X, Y, f, 0.5 * (double)W, 0.5 * (double)H, i, j, col);
            if (mode == 1)
                blend_over(col, cnt, o);
            else
                blend_front_to_back(col, cnt, o);
        }
        for (int ch = 0; ch < 4; ch++)
            rgba_f64[4 * (size_t)k + ch] = o[ch];
        count[k] = cnt;
        if (ids) {
            if (total + cnt > ids_cap) {
                free(fr);
                free(col);
                return -1;
            }
            for (uint32_t t = 0; t < cnt; t++)
                ids[total + t] = (uint32_t)(fr[t].key & 0xffffffffu);
        }
        total += cnt;
        if (offsets)
            offsets[k + 1] = total;
    }
    free(fr);
    free(col);
    return (int64_t)total;
}

/*
 * Bounding-box binning (Stage 2, phase 1 counts small quads by their AABB):
 * bin (bx, by) of size s lists, in ascending quad index, every visible quad
 * whose pixel bounding box overlaps it.  counts[nbx*nby]; when ids != NULL,
 * offsets[nbins+1] and ids[] are filled (ids_cap entries at most).  Returns
 * the number of (bin, quad) pairs or -1 when ids_cap is too small.
 */
int64_t lro_bins(uint32_t n, const int32_t *bbox, const uint8_t *cull, uint32_t W, uint32_t H,
                 uint32_t s, uint32_t *counts, uint64_t *offsets, uint32_t *ids, uint64_t ids_cap)
{
    uint32_t nbx = (W + s - 1) / s, nby = (H + s - 1) / s;
    size_t nbins = (size_t)nbx * nby;
    memset(counts, 0, nbins * sizeof(uint32_t));
    for (uint32_t q = 0; q < n; q++) {
        if (cull[q] != LRO_VISIBLE)
            continue;
        const int32_t *bb = bbox + 4 * (size_t)q;
        for (int32_t by = bb[2] / (int32_t)s; by <= bb[3] / (int32_t)s; by++)
            for (int32_t bx = bb[0] / (int32_t)s; bx <= bb[1] / (int32_t)s; bx++)
                counts[(size_t)by * nbx + bx]++;
    }
    uint64_t total = 0;
    for (size_t b = 0; b < nbins; b++)
        total += counts[b];
    if (!ids)
        return (int64_t)total;
    if (total > ids_cap)
        return -1;
    offsets[0] = 0;
    for (size_t b = 0; b < nbins; b++)
        offsets[b + 1] = offsets[b] + counts[b];
    uint64_t *fill = (uint64_t *)malloc((nbins ? nbins : 1) * sizeof(uint64_t));
    if (!fill)
        return -1;
    memcpy(fill, offsets, nbins * sizeof(uint64_t));
    for (uint32_t q = 0; q < n; q++) {
        if (cull[q] != LRO_VISIBLE)
            continue;
        const int32_t *bb = bbox + 4 * (size_t)q;
        for (int32_t by = bb[2] / (int32_t)s; by <= bb[3] / (int32_t)s; by++)
            for (int32_t bx = bb[0] / (int32_t)s; bx <= bb[1] / (int32_t)s; bx++)
                ids[fill[(size_t)by * nbx + bx]++] = q;
    }
    free(fill);
    return (int64_t)total;
}
