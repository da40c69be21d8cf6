/*
 * rm_oracle.c -- plain, slow FP64 reference for the RenderMap pose-scoring
 * path (Ryde & Ding, "RenderMap", arXiv 1702.06813).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it is used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * What it computes:
 *   or_scan_image  -- the scan image Z_s: per pixel depth and interface class
 *                     (free-occupied where the sensor returned a range,
 *                     free-unknown at the maximum range for no-return pixels,
 *                     NaN for dead pixels).  Sec. IV-A (no-return pixels are
 *                     free up to a sensor maximum) and Sec. IV-B (Z_s holds no
 *                     unknown-occupied pixels; NaN only for dead pixels).
 *   or_meshify     -- the interface mesh of one range image: quads between
 *                     adjacent 2x2 (strided) pixels, free-unknown if a corner
 *                     is a no-return or a side exceeds the size threshold,
 *                     free-occupied otherwise.  Sec. IV-A.  Optionally each
 *                     node's depth is first averaged over a window of
 *                     pixels of similar depth (Sec. IV-C's blurring).
 *   or_render      -- the z-buffer R(T(X)) of Eq. (1) by brute force: for each
 *                     requested pixel, every triangle is tested for coverage
 *                     and the nearest depth wins.  The z-buffer holds
 *                     perpendicular distance from the camera plane (Sec. V).
 *
 * Coverage has two modes:
 *   contract -- the rasterization contract (float32 camera transform,
 *               near-plane clip, projection snapped to 1/256 px,
 *               exact integer edge functions with a top-left fill rule).
 *               This is the definition of coverage the GPU rasterizer must
 *               reproduce bit for bit.
 *   exact    -- an unsnapped FP64 ray/triangle test (signs of the three
 *               scalar triple products, each edge evaluated in a canonical
 *               vertex order so that shared edges are watertight).
 * In both modes the depth of a covered pixel is the FP64 ray/plane distance
 * z = c / (n . r) of the triangle's FP64 camera-frame plane.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 * (contraction must stay off so that every float32 operation is the single
 * IEEE operation written here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near, z_far;
} or_camera;

enum { OR_FO = 0, OR_FU = 1, OR_UO = 2, OR_NONE = 3 };

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Range pixel classes (Sec. IV-A, Sec. IV-B).
 *   dead      : NaN, negative, or a positive range below z_min
 *   no-return : 0, +inf or beyond z_max  -> free up to z_max
 *   valid     : otherwise
 * ---------------------------------------------------------------------- */
enum { PX_DEAD = 0, PX_NORET = 1, PX_VALID = 2 };

static int px_class(float z, float z_min, float z_max) {
    if (isnan(z) || z < 0.0f) return PX_DEAD;
    if (z == 0.0f || isinf(z) || z > z_max) return PX_NORET;
    if (z < z_min) return PX_DEAD;
    return PX_VALID;
}

void or_scan_image(const float* depth, int32_t H, int32_t W, float z_min, float z_max,
                   float* d_out, uint8_t* c_out) {
    for (int64_t i = 0; i < (int64_t)H * W; ++i) {
        int k = px_class(depth[i], z_min, z_max);
        if (k == PX_VALID) { d_out[i] = depth[i]; c_out[i] = OR_FO; }
        else if (k == PX_NORET) { d_out[i] = z_max; c_out[i] = OR_FU; }
        else { d_out[i] = NAN; c_out[i] = OR_NONE; }
    }
}

/* ------------------------------------------------------------------------
 * Meshification (Sec. IV-A).
 *
 * Grid nodes sit at pixels (j*s, i*s), i < ceil(H/s), j < ceil(W/s).  A node
 * is back-projected at its range (z_max for a no-return) through the pinhole
 * and moved to the world frame in FP64; the vertex is that point rounded to
 * float32.  Vertex index = i * gw + j (dead nodes keep an unreferenced NaN
 * vertex).  A quad between nodes (i,j),(i,j+1),(i+1,j),(i+1,j+1) is dropped
 * if a corner is dead; it is free-unknown if a corner is a no-return or one
 * of its four sides is longer than max_edge; free-occupied otherwise.  Each
 * quad gives triangles (00, 01, 11) and (00, 11, 10).  Quads are emitted in
 * 8x8 blocks (blocks row-major, quads row-major inside a block), so that
 * consecutive triangles are spatial neighbours.
 * ---------------------------------------------------------------------- */
#define OR_QBLOCK 8

int64_t or_meshify(const float* depth, int32_t H, int32_t W, const or_camera* cam,
                   const double* T, int32_t s, int32_t R, float z_min, float z_max, float max_edge,
                   float* xyz, int32_t* tri, uint8_t* cls, int64_t cap_t, int64_t* n_v_out) {
    const int gh = (H + s - 1) / s, gw = (W + s - 1) / s;
    const int64_t nv = (int64_t)gh * gw;
    uint8_t* kind = (uint8_t*)malloc((size_t)nv);
    for (int i = 0; i < gh; ++i)
        for (int j = 0; j < gw; ++j) {
            const int64_t n = (int64_t)i * gw + j;
            const float z = depth[(int64_t)(i * s) * W + (j * s)];
            const int k = px_class(z, z_min, z_max);
            kind[n] = (uint8_t)k;
            if (k == PX_DEAD) { xyz[3 * n] = xyz[3 * n + 1] = xyz[3 * n + 2] = NAN; continue; }
            double zd = (k == PX_NORET) ? (double)z_max : (double)z;
            if (k == PX_VALID && R > 0) {
                /* noise reduction before meshing (Sec. IV-C suggests blurring
                 * the depth images): mean of the valid window pixels within
                 * 3% of the node pixel's depth, which keeps range edges */
                double sum = 0.0;
                int cnt = 0;
                for (int y = i * s - R; y <= i * s + R; ++y)
                    for (int x = j * s - R; x <= j * s + R; ++x) {
                        if (y < 0 || y >= H || x < 0 || x >= W) continue;
                        const float zn = depth[(int64_t)y * W + x];
                        if (px_class(zn, z_min, z_max) != PX_VALID) continue;
                        if (fabs((double)zn - (double)z) <= 0.03 * (double)z) {
                            sum += (double)zn;
                            cnt += 1;
                        }
                    }
                zd = sum / (double)cnt;
            }
            const double xc = zd * (((double)(j * s) - (double)cam->cx) / (double)cam->fx);
            const double yc = zd * (((double)(i * s) - (double)cam->cy) / (double)cam->fy);
            for (int r = 0; r < 3; ++r) {
                const double w = ((T[4 * r + 0] * xc + T[4 * r + 1] * yc) + T[4 * r + 2] * zd) + T[4 * r + 3];
                xyz[3 * n + r] = (float)w;
            }
        }
    const double lim2 = (double)max_edge * (double)max_edge;
    int64_t nt = 0;
    const int qh = gh - 1, qw = gw - 1;
    for (int bi = 0; bi < qh; bi += OR_QBLOCK)
        for (int bj = 0; bj < qw; bj += OR_QBLOCK)
            for (int i = bi; i < bi + OR_QBLOCK && i < qh; ++i)
                for (int j = bj; j < bj + OR_QBLOCK && j < qw; ++j) {
                    const int64_t n00 = (int64_t)i * gw + j, n01 = n00 + 1;
                    const int64_t n10 = n00 + gw, n11 = n10 + 1;
                    const int64_t c[4] = {n00, n01, n11, n10};   /* perimeter order */
                    int dead = 0, noret = 0;
                    for (int k = 0; k < 4; ++k) {
                        dead |= kind[c[k]] == PX_DEAD;
                        noret |= kind[c[k]] == PX_NORET;
                    }
                    if (dead) continue;
                    int big = 0;
                    for (int k = 0; k < 4; ++k) {
                        const float* a = xyz + 3 * c[k];
                        const float* b = xyz + 3 * c[(k + 1) & 3];
                        const double dx = (double)a[0] - (double)b[0];
                        const double dy = (double)a[1] - (double)b[1];
                        const double dz = (double)a[2] - (double)b[2];
                        big |= ((dx * dx + dy * dy) + dz * dz) > lim2;
                    }
                    const uint8_t q = (noret || big) ? OR_FU : OR_FO;
                    if (nt + 2 > cap_t) { free(kind); return -1; }
                    tri[3 * nt + 0] = (int32_t)n00; tri[3 * nt + 1] = (int32_t)n01; tri[3 * nt + 2] = (int32_t)n11;
                    cls[nt++] = q;
                    tri[3 * nt + 0] = (int32_t)n00; tri[3 * nt + 1] = (int32_t)n11; tri[3 * nt + 2] = (int32_t)n10;
                    cls[nt++] = q;
                }
    free(kind);
    *n_v_out = nv;
    return nt;
}

/* ------------------------------------------------------------------------
 * Per-pose triangle preparation.
 *
 * Camera frame of a world point, FP64 (depth, planes, Jacobians):
 *     Xc = R^T (Xw - t),  T = [R | t] camera-to-world.
 *
 * Camera frame under the float32 rasterization contract (coverage only):
 *     R32[i][j] = (float) R[j][i]         (rotation world->camera, rounded)
 *     d[j]      = (float)((double)Xw[j] - t[j])
 *     Xc[i]     = fmaf(R32[i][2], d[2], fmaf(R32[i][1], d[1], R32[i][0]*d[0]))
 * Near-plane clip (inside iff z >= z_near), always interpolating from the
 * inside vertex I towards the outside vertex O:
 *     t  = (z_near - I.z) / (O.z - I.z)
 *     P  = (fmaf(t, O.x - I.x, I.x), fmaf(t, O.y - I.y, I.y), z_near)
 * One outside vertex k (a, b the next two in cyclic order): the quad
 * (a, b, P(b,k), P(a,k)) is fanned into (a, b, P(b,k)) and (a, P(b,k), P(a,k)).
 * Two outside vertices (k the inside one, a, b the others): (k, P(k,a), P(k,b)).
 * Projection and snap of a camera point P with P.z >= z_near:
 *     inv = 1/P.z ;  u = fmaf(fx*P.x, inv, cx) ;  v = fmaf(fy*P.y, inv, cy)
 *     X = rint(256*u), Y = rint(256*v)  (round half to even)
 * A sub-triangle is dropped if |X| or |Y| >= 2^29, if its snapped area is
 * zero, or if its snapped bounding box holds no pixel centre; with negative
 * area its last two vertices are swapped.  A triangle whose three contract
 * z values all exceed z_far is culled.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t X[3], Y[3];
    int64_t x0, x1, y0, y1;      /* pixel range of the bounding box (inclusive) */
    int32_t parent;
} or_sub;

typedef struct {
    double n[3], c;              /* FP64 camera-frame plane n . X = c */
    double V[3][3];              /* FP64 camera-frame vertices */
} or_plane;

#define OR_LIM (((int64_t)1) << 29)

static void cam_fp64(const double* T, const float* Xw, double* Xc) {
    const double d0 = (double)Xw[0] - T[3], d1 = (double)Xw[1] - T[7], d2 = (double)Xw[2] - T[11];
    for (int i = 0; i < 3; ++i)
        Xc[i] = (T[0 + i] * d0 + T[4 + i] * d1) + T[8 + i] * d2;
}

static void cam_contract(const float R32[3][3], const double* T, const float* Xw, float* Xc) {
    float d[3];
    for (int j = 0; j < 3; ++j) d[j] = (float)((double)Xw[j] - T[4 * j + 3]);
    for (int i = 0; i < 3; ++i)
        Xc[i] = fmaf(R32[i][2], d[2], fmaf(R32[i][1], d[1], R32[i][0] * d[0]));
}

static void clip_point(const float* I, const float* O, float zn, float* P) {
    const float t = (zn - I[2]) / (O[2] - I[2]);
    P[0] = fmaf(t, O[0] - I[0], I[0]);
    P[1] = fmaf(t, O[1] - I[1], I[1]);
    P[2] = zn;
}

/* returns 0 if the point cannot be represented inside the snap range */
static int snap(const or_camera* cam, const float* P, int64_t* X, int64_t* Y) {
    const float inv = 1.0f / P[2];
    const float u = fmaf(cam->fx * P[0], inv, cam->cx);
    const float v = fmaf(cam->fy * P[1], inv, cam->cy);
    const float su = rintf(u * 256.0f), sv = rintf(v * 256.0f);
    if (!(fabsf(su) < (float)OR_LIM) || !(fabsf(sv) < (float)OR_LIM)) return 0;
    *X = (int64_t)su; *Y = (int64_t)sv;
    return 1;
}

static int64_t floor_div256(int64_t a) { return a >= 0 ? a / 256 : -((-a + 255) / 256); }
static int64_t ceil_div256(int64_t a) { return a >= 0 ? (a + 255) / 256 : -((-a) / 256); }

/* emits 0 or 1 sub-triangle; returns the number emitted */
static int emit(const or_camera* cam, const float* A, const float* B, const float* C,
                int32_t parent, or_sub* out, int64_t* dropped) {
    int64_t X[3], Y[3];
    const float* P[3] = {A, B, C};
    for (int k = 0; k < 3; ++k)
        if (!snap(cam, P[k], &X[k], &Y[k])) { ++*dropped; return 0; }
    const int64_t area = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]);
    if (area == 0) return 0;
    if (area < 0) {
        int64_t t = X[1]; X[1] = X[2]; X[2] = t;
        t = Y[1]; Y[1] = Y[2]; Y[2] = t;
    }
    int64_t mnx = X[0], mxx = X[0], mny = Y[0], mxy = Y[0];
    for (int k = 1; k < 3; ++k) {
        if (X[k] < mnx) mnx = X[k]; if (X[k] > mxx) mxx = X[k];
        if (Y[k] < mny) mny = Y[k]; if (Y[k] > mxy) mxy = Y[k];
    }
    int64_t x0 = ceil_div256(mnx), x1 = floor_div256(mxx);
    int64_t y0 = ceil_div256(mny), y1 = floor_div256(mxy);
    if (x0 < 0) x0 = 0; if (y0 < 0) y0 = 0;
    if (x1 > cam->width - 1) x1 = cam->width - 1;
    if (y1 > cam->height - 1) y1 = cam->height - 1;
    if (x0 > x1 || y0 > y1) return 0;
    for (int k = 0; k < 3; ++k) { out->X[k] = X[k]; out->Y[k] = Y[k]; }
    out->x0 = x0; out->x1 = x1; out->y0 = y0; out->y1 = y1;
    out->parent = parent;
    return 1;
}

/* builds the contract sub-triangles of every mesh triangle for one pose */
static int64_t prepare_contract(const float* xyz, const int32_t* tri, int64_t nt,
                                const double* T, const or_camera* cam, or_sub* subs,
                                int64_t* dropped) {
    float R32[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R32[i][j] = (float)T[4 * j + i];
    const float zn = cam->z_near, zf = cam->z_far;
    int64_t ns = 0;
    for (int64_t t = 0; t < nt; ++t) {
        float V[3][3];
        for (int k = 0; k < 3; ++k) cam_contract(R32, T, xyz + 3 * (int64_t)tri[3 * t + k], V[k]);
        if (V[0][2] > zf && V[1][2] > zf && V[2][2] > zf) continue;
        const int in[3] = {V[0][2] >= zn, V[1][2] >= zn, V[2][2] >= zn};
        const int nin = in[0] + in[1] + in[2];
        if (nin == 0) continue;
        if (nin == 3) {
            ns += emit(cam, V[0], V[1], V[2], (int32_t)t, subs + ns, dropped);
        } else if (nin == 2) {
            const int k = !in[0] ? 0 : (!in[1] ? 1 : 2);
            const float* a = V[(k + 1) % 3];
            const float* b = V[(k + 2) % 3];
            float Pb[3], Pa[3];
            clip_point(b, V[k], zn, Pb);
            clip_point(a, V[k], zn, Pa);
            ns += emit(cam, a, b, Pb, (int32_t)t, subs + ns, dropped);
            ns += emit(cam, a, Pb, Pa, (int32_t)t, subs + ns, dropped);
        } else {
            const int k = in[0] ? 0 : (in[1] ? 1 : 2);
            float Pa[3], Pb[3];
            clip_point(V[k], V[(k + 1) % 3], zn, Pa);
            clip_point(V[k], V[(k + 2) % 3], zn, Pb);
            ns += emit(cam, V[k], Pa, Pb, (int32_t)t, subs + ns, dropped);
        }
    }
    return ns;
}

/* top-left rule with y pointing down: an edge p->q of a positively oriented
 * triangle owns its boundary points iff dy < 0, or dy == 0 and dx > 0 */
static int top_left(int64_t dx, int64_t dy) { return dy < 0 || (dy == 0 && dx > 0); }

static int covers(const or_sub* s, int64_t px, int64_t py) {
    const int64_t SX = 256 * px, SY = 256 * py;
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3;
        const int64_t dx = s->X[k1] - s->X[k], dy = s->Y[k1] - s->Y[k];
        const int64_t E = dx * (SY - s->Y[k]) - dy * (SX - s->X[k]);
        if (E < 0 || (E == 0 && !top_left(dx, dy))) return 0;
    }
    return 1;
}

/* exact mode: scalar triple product (A x B) . r with a canonical order of the
 * two edge endpoints so that a shared edge gives exactly opposite values */
static int lex_less(const double* a, const double* b) {
    for (int k = 0; k < 3; ++k) { if (a[k] < b[k]) return 1; if (a[k] > b[k]) return 0; }
    return 0;
}
static double triple(const double* A, const double* B, const double* r) {
    const double cx = A[1] * B[2] - A[2] * B[1];
    const double cy = A[2] * B[0] - A[0] * B[2];
    const double cz = A[0] * B[1] - A[1] * B[0];
    return (cx * r[0] + cy * r[1]) + cz * r[2];
}
static double edge_side(const double* A, const double* B, const double* r) {
    return lex_less(A, B) ? triple(A, B, r) : -triple(B, A, r);
}
static int covers_exact(const or_plane* p, const double* r) {
    const double s0 = edge_side(p->V[0], p->V[1], r);
    const double s1 = edge_side(p->V[1], p->V[2], r);
    const double s2 = edge_side(p->V[2], p->V[0], r);
    if (s0 == 0.0 && s1 == 0.0 && s2 == 0.0) return 0;
    return (s0 >= 0.0 && s1 >= 0.0 && s2 >= 0.0) || (s0 <= 0.0 && s1 <= 0.0 && s2 <= 0.0);
}

/* One covering candidate at depth z.  Candidates with 0 < z <= z_far compete
 * for the pixel (lexicographic minimum of (z, id)); the runner-up z2 is the
 * smallest depth of any other covering triangle, including those just beyond
 * z_far, so that callers can flag depth near-ties and far-plane ties. */
static void consider(double z, int32_t id, double zf, double* zb, int32_t* ib, double* z2) {
    if (!(z > 0.0)) return;
    if (z <= zf && (z < *zb || (z == *zb && id < *ib))) {
        if (*ib >= 0 && *ib != id && *zb < *z2) *z2 = *zb;
        *zb = z; *ib = id;
    } else if (id != *ib && z < *z2) {
        *z2 = z;
    }
}

/* ------------------------------------------------------------------------
 * or_render: brute-force z-buffer at the requested pixels for one pose.
 *
 * pix     : linear pixel indices (y * W + x); NULL means every pixel
 * outputs per requested pixel (any pointer may be NULL):
 *   z      winner depth (NaN if no surface within [z_near, z_far])
 *   id     winner triangle id (-1)
 *   z2     smallest depth among other covering triangles, beyond z_far included (+inf)
 *   ncov   number of covering (sub-)triangles, before any depth test
 *   nrm    winner's FP64 camera-frame plane normal (unnormalized), 3 per pixel
 * The winner is the lexicographic minimum of (depth, triangle id) over
 * covering triangles with z_near <= z <= z_far (contract mode clips at the
 * near plane geometrically, so only the far test is applied there).
 * Returns the number of sub-triangles dropped for exceeding the snap range.
 * ---------------------------------------------------------------------- */
int64_t or_render(const float* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                  const double* T, const or_camera* cam, int32_t mode,
                  const int64_t* pix, int64_t npix,
                  double* z_out, int32_t* id_out, double* z2_out, int32_t* ncov_out,
                  double* nrm_out) {
    (void)nv;
    or_plane* pl = (or_plane*)malloc(sizeof(or_plane) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t t = 0; t < nt; ++t) {
        or_plane* p = pl + t;
        for (int k = 0; k < 3; ++k) cam_fp64(T, xyz + 3 * (int64_t)tri[3 * t + k], p->V[k]);
        const double e1[3] = {p->V[1][0] - p->V[0][0], p->V[1][1] - p->V[0][1], p->V[1][2] - p->V[0][2]};
        const double e2[3] = {p->V[2][0] - p->V[0][0], p->V[2][1] - p->V[0][1], p->V[2][2] - p->V[0][2]};
        p->n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        p->n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        p->n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        p->c = (p->n[0] * p->V[0][0] + p->n[1] * p->V[0][1]) + p->n[2] * p->V[0][2];
    }
    or_sub* subs = NULL;
    int64_t ns = 0, dropped = 0;
    if (mode == 0) {
        subs = (or_sub*)malloc(sizeof(or_sub) * (size_t)(2 * nt + 1));
        ns = prepare_contract(xyz, tri, nt, T, cam, subs, &dropped);
    }
    const int64_t W = cam->width;
    const int64_t n = pix ? npix : W * cam->height;
    const double fx = cam->fx, fy = cam->fy, cx = cam->cx, cy = cam->cy;
    const double zn = cam->z_near, zf = cam->z_far;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; ++q) {
        const int64_t lin = pix ? pix[q] : q;
        const int64_t px = lin % W, py = lin / W;
        const double r[3] = {((double)px - cx) / fx, ((double)py - cy) / fy, 1.0};
        double zb = INFINITY, z2 = INFINITY;
        int32_t ib = -1, cov = 0;
        if (mode == 0) {
            for (int64_t k = 0; k < ns; ++k) {
                const or_sub* s = subs + k;
                if (px < s->x0 || px > s->x1 || py < s->y0 || py > s->y1) continue;
                if (!covers(s, px, py)) continue;
                ++cov;
                const or_plane* p = pl + s->parent;
                const double z = p->c / ((p->n[0] * r[0] + p->n[1] * r[1]) + p->n[2] * r[2]);
                consider(z, s->parent, zf, &zb, &ib, &z2);
            }
        } else {
            for (int64_t t = 0; t < nt; ++t) {
                const or_plane* p = pl + t;
                if (!covers_exact(p, r)) continue;
                const double z = p->c / ((p->n[0] * r[0] + p->n[1] * r[1]) + p->n[2] * r[2]);
                if (!(z >= zn)) continue;
                ++cov;
                consider(z, (int32_t)t, zf, &zb, &ib, &z2);
            }
        }
        if (z_out) z_out[q] = ib >= 0 ? zb : NAN;
        if (id_out) id_out[q] = ib;
        if (z2_out) z2_out[q] = z2;
        if (ncov_out) ncov_out[q] = cov;
        if (nrm_out) {
            for (int k = 0; k < 3; ++k) nrm_out[3 * q + k] = ib >= 0 ? pl[ib].n[k] : NAN;
        }
    }
    free(subs);
    free(pl);
    return dropped;
}

/* The contract's snapped sub-triangles for one pose (for white-box tests):
 * writes up to cap records of [parent, X0, Y0, X1, Y1, X2, Y2] as int64. */
int64_t or_contract_subs(const float* xyz, const int32_t* tri, int64_t nt, const double* T,
                         const or_camera* cam, int64_t* out, int64_t cap) {
    or_sub* subs = (or_sub*)malloc(sizeof(or_sub) * (size_t)(2 * nt + 1));
    int64_t dropped = 0;
    const int64_t ns = prepare_contract(xyz, tri, nt, T, cam, subs, &dropped);
    for (int64_t k = 0; k < ns && k < cap; ++k) {
        out[7 * k] = subs[k].parent;
        for (int j = 0; j < 3; ++j) { out[7 * k + 1 + 2 * j] = subs[k].X[j]; out[7 * k + 2 + 2 * j] = subs[k].Y[j]; }
    }
    free(subs);
    return ns;
}
