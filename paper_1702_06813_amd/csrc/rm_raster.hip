// Pose scoring on gfx950: cluster frustum cull, screen-tile rasterization into
// an LDS z-buffer of packed (depth | triangle id) keys resolved by 64-bit
// atomic min, and the fused per-pixel comparison of Table I, the E_soft
// residual and its se(3) Jacobian, reduced per tile and then per pose.
//
// The z-buffer R(T(X)) is Eq. (1) of the paper; the per-pixel rules are its
// Table I (Sec. IV-B); the total error is their sum over pixels (Sec. IV-B).
#include <algorithm>

#include "rm_internal.h"

namespace rm {

namespace {

// ------------------------------------------------------------------ pose data

// World -> camera rotation rounded to f32 (R32[i][j] = fl32(R[j][i])) and the
// FP64 camera centre; the float32 rasterization contract transforms a world
// point as d = fl32(Xw - t) (difference in FP64), Xc = R32 d with explicit
// fmaf in the order z-, y-, x-column.
struct PoseF {
    float R[3][3];
    double t[3];
    float tf[3];          // camera centre rounded to f32 (binning footprints only)
};

__device__ __forceinline__ void load_pose(const double* __restrict__ T, PoseF& P) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) P.R[i][j] = (float)T[4 * j + i];
        P.t[i] = T[4 * i + 3];
        P.tf[i] = (float)T[4 * i + 3];
    }
}

__device__ __forceinline__ float3 cam_contract(const PoseF& P, float x, float y, float z) {
    const float d0 = (float)((double)x - P.t[0]);
    const float d1 = (float)((double)y - P.t[1]);
    const float d2 = (float)((double)z - P.t[2]);
    float3 c;
    c.x = fmaf(P.R[0][2], d2, fmaf(P.R[0][1], d1, P.R[0][0] * d0));
    c.y = fmaf(P.R[1][2], d2, fmaf(P.R[1][1], d1, P.R[1][0] * d0));
    c.z = fmaf(P.R[2][2], d2, fmaf(P.R[2][1], d1, P.R[2][0] * d0));
    return c;
}

struct CamF {
    float fx, fy, cx, cy, zn, zf;
    int W, H;
};

// Near-plane clip point, interpolated from the inside vertex I to the
// outside vertex O (a shared edge gives the same point in both triangles).
__device__ __forceinline__ float3 clip_point(float3 I, float3 O, float zn) {
    const float t = (zn - I.z) / (O.z - I.z);
    return make_float3(fmaf(t, O.x - I.x, I.x), fmaf(t, O.y - I.y, I.y), zn);
}

// Projection and snap to 1/256 px (round half to even).  False if the
// snapped coordinate leaves the representable range.
__device__ __forceinline__ bool snap(const CamF& c, float3 P, int& X, int& Y) {
    const float inv = 1.0f / P.z;
    const float u = fmaf(c.fx * P.x, inv, c.cx);
    const float v = fmaf(c.fy * P.y, inv, c.cy);
    const float su = rintf(u * 256.0f), sv = rintf(v * 256.0f);
    if (!(fabsf(su) < (float)kSnapLimit) || !(fabsf(sv) < (float)kSnapLimit)) return false;
    X = (int)su;
    Y = (int)sv;
    return true;
}

__device__ __forceinline__ uint64_t pack_key(float w, uint32_t id) {
    // resolved by atomic maximum: nearer surface = larger w = 1/z = larger
    // key (w >= 0, so its bits order like its value); equal depths: the
    // lower id has the larger complement and wins
    return ((uint64_t)__float_as_uint(w) << 32) | (uint64_t)(~id);
}
constexpr uint64_t kEmptyKey = 0ull;       // w = 0: behind everything

// ------------------------------------------------------------------ tile rasterization

// Depth plane of a triangle in the camera frame, as w = 1/z affine in the
// pixel offsets: w = a (u - cx) + b (v - cy) + e, with a = n_x/(c fx),
// b = n_y/(c fy), e = n_z/c for the camera-frame plane n . X = c.  Built in
// FP64 from the cross product of the triangle's world edges (any length of n
// gives the same plane) and its first vertex, so that long thin triangles
// keep their depth to ~1e-7 relative.
struct WPlane { double a, b, e; };
struct PlaneN { double nx, ny, nz, c; };   // camera-frame normal and offset n . X = c

__device__ __forceinline__ PlaneN plane_normal(const PoseF& P, const float v[9]) {
    const float x0 = v[0], y0 = v[1], z0 = v[2];
    const double e1x = (double)v[3] - x0, e1y = (double)v[4] - y0, e1z = (double)v[5] - z0;
    const double e2x = (double)v[6] - x0, e2y = (double)v[7] - y0, e2z = (double)v[8] - z0;
    const double n0 = e1y * e2z - e1z * e2y, n1 = e1z * e2x - e1x * e2z, n2 = e1x * e2y - e1y * e2x;
    PlaneN q;
    q.c = n0 * ((double)x0 - P.t[0]) + n1 * ((double)y0 - P.t[1]) + n2 * ((double)z0 - P.t[2]);
    // camera-frame normal with the f32-rounded rotation (a 6e-8 rotation of the
    // plane about its anchor vertex, far below the depth tolerance)
    q.nx = (double)P.R[0][0] * n0 + (double)P.R[0][1] * n1 + (double)P.R[0][2] * n2;
    q.ny = (double)P.R[1][0] * n0 + (double)P.R[1][1] * n1 + (double)P.R[1][2] * n2;
    q.nz = (double)P.R[2][0] * n0 + (double)P.R[2][1] * n1 + (double)P.R[2][2] * n2;
    return q;
}

// 1/z over the image: w(u, v) = a (u - cx) + b (v - cy) + e.
__device__ __forceinline__ WPlane depth_plane(const PlaneN& q, double ifx, double ify) {
    const double ic = 1.0 / q.c;
    WPlane p;
    p.a = q.nx * ic * ifx;
    p.b = q.ny * ic * ify;
    p.e = q.nz * ic;
    return p;
}

struct Tile {
    int x0, y0, x1, y1;   // inclusive pixel range of the tile inside the image
};


// Occlusion margin: a row of a triangle is skipped when its nearest depth,
// scaled by this factor, is still farther than the farthest key of the row
// snapshot (far more than the rounding between the FP64 plane and the f32 key).
constexpr double kOccMargin = 1.0 + 1e-6;
// The depth snapshot keeps one value per kSeg-pixel segment of each tile row
// (index row * kSegs + x / kSeg) and the tile's farthest at kSnapTile.
constexpr int kSeg = 16, kSegs = 4, kSnapTile = 32 * kSegs;
constexpr int kSnapEvery = 4;            // rounds between snapshot refreshes after the first ones

// Minimum of x over aligned groups of G consecutive lanes (G = 8 or 16, one
// DPP row or half row): swaps inside quads, then the half-row and row
// mirrors; every lane of a group ends with the group's minimum.  All lanes of
// the wave must be active.
template <int G>
__device__ __forceinline__ uint32_t group_min(uint32_t x) {
    static_assert(G == 8 || G == 16, "groups of 8 or 16 lanes");
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false));   // row_half_mirror
    if constexpr (G == 16) x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false));   // row_mirror
    return x;
}

// Farthest snapshot w over the segments that columns [x0, x1] of row y touch.
__device__ __forceinline__ float snap_min(const float* rmin, int y, int x0, int x1) {
    const float* r = rmin + y * kSegs;
    float m = r[x0 / kSeg];
    for (int s = x0 / kSeg + 1; s <= x1 / kSeg; ++s) m = fminf(m, r[s]);
    return m;
}

// Small (sub-)triangles are rasterized by their own thread over the pixel
// centres of their bounding box inside the tile (int32 edge functions).
__device__ __forceinline__ void raster_small(uint64_t* keys, int tile_w, const Tile& tl, const float* rmin,
                                             const int X[3], const int Y[3], int px0, int px1, int py0, int py1,
                                             const WPlane& pl, double cx, double cy, uint32_t id) {
    int E[3], sx[3], sy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        const int dx = X[k1] - X[k], dy = Y[k1] - Y[k];
        const bool topleft = dy < 0 || (dy == 0 && dx > 0);
        E[k] = dx * (256 * py0 - Y[k]) - dy * (256 * px0 - X[k]) - (topleft ? 0 : 1);
        sx[k] = -256 * dy;
        sy[k] = 256 * dx;
    }
    double wrow = fma(pl.b, (double)py0 - cy, fma(pl.a, (double)px0 - cx, pl.e));
    for (int y = py0; y <= py1; ++y) {
        int e0 = E[0], e1 = E[1], e2 = E[2];
        double w = wrow;
        uint64_t* row = keys + (y - tl.y0) * tile_w - tl.x0;
        // the plane's nearest point over the row's columns is behind everything
        // visible in this row: every atomic below would leave the keys unchanged
        const double wn = fmax(wrow, fma(pl.a, (double)(px1 - px0), wrow));
        const int xend = wn * kOccMargin < (double)snap_min(rmin, y - tl.y0, px0 - tl.x0, px1 - tl.x0) ? px0 - 1 : px1;
        // (the loop runs on the key address; the far plane is applied at
        // the resolve, see there)
        for (uint64_t *k = row + px0, *kend = row + xend; k <= kend; ++k) {
            {   // branch-free: an uncovered pixel offers the empty key, which changes nothing
                const float wf = (float)w;
                const bool cov = (e0 | e1 | e2) >= 0;
                atomicMax((unsigned long long*)k, cov ? (unsigned long long)pack_key(wf, id) : kEmptyKey);
            }
            e0 += sx[0]; e1 += sx[1]; e2 += sx[2];
            w += pl.a;
        }
        E[0] += sy[0]; E[1] += sy[1]; E[2] += sy[2];
        wrow += pl.b;
    }
}

// Larger (sub-)triangles are queued in LDS and rasterized by the whole
// workgroup in jobs of kBand rows: a job brackets the covered span of each of
// its rows between the three edge crossings (FP64, exact to far below a
// pixel) and gives only pixel centres inside it the exact int64 edge test.
constexpr int kQCap = 192;                 // queued sub-triangles per pass (more wait for the next); with the
                                           // 16 KB z-buffer, 40 KB of LDS: four workgroups per CU
constexpr int kBand = 2;                   // rows per job
constexpr int kSmallArea = 64;             // bounding-box pixels rasterized by the owning thread

constexpr int kMaxBands = 16;             // tile height / kBand for the tallest tile (32 rows)
static_assert(32 / kBand <= kMaxBands && kMaxBands <= 16, "job records hold a 4-bit band index");
static_assert((kQCap << 4) + 15 <= 0xffff, "job records are 16-bit");
static_assert(kSmallArea <= 64, "in-thread edge functions stay within int32 only for spans below 64 px");
struct BigQueue {
    int X[3][kQCap], Y[3][kQCap];          // snapped vertices relative to the tile origin (1/256 px)
    double m[3][kQCap];                    // edge slope dx/dy (0 for horizontal edges)
    double pa[kQCap], pb[kQCap], pe[kQCap];
    uint32_t id[kQCap];
    uint32_t box[kQCap];                   // tile-relative px0 | px1 << 8 | py0 << 16 | py1 << 24
    uint16_t job[kQCap * kMaxBands];       // queued entry << 4 | band, only bands the entry covers
    int n, njobs;
};

// Rows r0..r1 (tile-relative) of one sub-triangle with tile-relative snapped
// vertices (X, Y), edge slopes m, depth plane and tile-relative column range.
__device__ __forceinline__ void raster_rows(uint64_t* keys, int tile_w, const Tile& tl, const float* rmin,
                                            const int X[3], const int Y[3], const double m[3], double pa, double pb,
                                            double pe,
                                            uint32_t id, int bx0, int bx1, int r0, int r1, double cx, double cy) {
    int64_t E[3];
    int dx[3], dy[3];
    double xc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        dx[k] = X[k1] - X[k];
        dy[k] = Y[k1] - Y[k];
        const bool topleft = dy[k] < 0 || (dy[k] == 0 && dx[k] > 0);
        E[k] = (int64_t)dx[k] * (int64_t)(256 * r0 - Y[k]) - (int64_t)dy[k] * (int64_t)(256 * bx0 - X[k]) -
               (topleft ? 0 : 1);
        xc[k] = ((double)X[k] + (double)(256 * r0 - Y[k]) * m[k]) * (1.0 / 256.0);   // crossing on row r0
    }
    double wrow = fma(pb, (double)(tl.y0 + r0) - cy, fma(pa, (double)(tl.x0 + bx0) - cx, pe));
    for (int r = r0; r <= r1; ++r) {
        double lo = (double)bx0, hi = (double)bx1;
        bool empty = false;
        // selects instead of branches: the three edges' cases differ per lane
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double c = xc[k];
            lo = ((dy[k] < 0) & (c > lo)) ? c : lo;
            hi = ((dy[k] > 0) & (c < hi)) ? c : hi;
            empty |= (dy[k] == 0) & (E[k] < 0);     // horizontal edge: the whole row is in or out
        }
        // lo >= bx0 and hi <= bx1 already; clamp the other side before converting
        const int xa = max(bx0, (int)ceil(fmin(lo, (double)bx1 + 1.0) - 1e-6));
        const int xb = min(bx1, (int)floor(fmax(hi, (double)bx0 - 1.0) + 1e-6));
        double w = fma(pa, (double)(xa - bx0), wrow);
        if (!empty && xa <= xb && fmax(w, fma(pa, (double)(xb - xa), w)) * kOccMargin >= (double)snap_min(rmin, r, xa, xb)) {
            // The bracket's crossings are exact to far below a pixel, so a
            // pixel centre one pixel or more inside it is covered: only its
            // end pixels take the exact int64 edge test, and an end that
            // fails it is left out of the span.
            auto inside = [&](int x) {
                const int64_t o = 256 * (int64_t)(x - bx0);
                return ((E[0] - o * dy[0]) | (E[1] - o * dy[1]) | (E[2] - o * dy[2])) >= 0;
            };
            const bool in_a = inside(xa), in_b = inside(xb);
            if (!in_a) w += pa;                // the span's first pixel, accumulated as before
            uint64_t* row = keys + r * tile_w;
            for (uint64_t *k = row + xa + (in_a ? 0 : 1), *kend = row + xb - (in_b ? 0 : 1); k <= kend; ++k) {
                atomicMax((unsigned long long*)k, pack_key((float)w, id));
                w += pa;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) { E[k] += 256 * (int64_t)dx[k]; xc[k] += m[k]; }
        wrow += pb;
    }
}

template <int TW, int TH>
__device__ __forceinline__ void raster_queue(uint64_t* keys, BigQueue& q, const Tile& tl, const float* rmin,
                                             double cx, double cy) {
    const int nj = q.njobs;
    for (int j = threadIdx.x; j < nj; j += kWG) {
        const int rec = q.job[j];
        const int b = rec >> 4, band = rec & 15;
        const uint32_t box = q.box[b];
        const int by0 = (int)((box >> 16) & 0xff), by1 = (int)(box >> 24);
        const int r0 = max(by0, band * kBand), r1 = min(by1, band * kBand + kBand - 1);
        const int X[3] = {q.X[0][b], q.X[1][b], q.X[2][b]};
        const int Y[3] = {q.Y[0][b], q.Y[1][b], q.Y[2][b]};
        const double m[3] = {q.m[0][b], q.m[1][b], q.m[2][b]};
        raster_rows(keys, TW, tl, rmin, X, Y, m, q.pa[b], q.pb[b], q.pe[b], q.id[b], (int)(box & 0xff),
                    (int)((box >> 8) & 0xff), r0, r1, cx, cy);
    }
}

// Setup of one (sub-)triangle of the contract: snap, orientation, bounding
// box inside the tile, then the rasterization path by size.
struct Queues {
    BigQueue big;
    // per kSeg-pixel segment of each tile row, the farthest w = 1/z held by
    // its keys (0 if a pixel is empty) at the start of the round, and at
    // kSnapTile the tile's farthest; two buffers, one filled per round
    float rowmin[2][kSnapTile + 1];
};

__device__ __forceinline__ bool emit_tri(uint64_t* keys, int tile_w, Queues& Q, const float* rmin, const Tile& tl,
                                         const CamF& cam, float3 A, float3 B, float3 C, const WPlane& pl,
                                         uint32_t id) {
    int X[3], Y[3];
    if (!snap(cam, A, X[0], Y[0]) || !snap(cam, B, X[1], Y[1]) || !snap(cam, C, X[2], Y[2])) return true;
    const int64_t area = (int64_t)(X[1] - X[0]) * (int64_t)(Y[2] - Y[0]) -
                         (int64_t)(Y[1] - Y[0]) * (int64_t)(X[2] - X[0]);
    if (area == 0) return true;
    if (area < 0) {
        int t = X[1]; X[1] = X[2]; X[2] = t;
        t = Y[1]; Y[1] = Y[2]; Y[2] = t;
    }
    const int mnx = min(X[0], min(X[1], X[2])), mxx = max(X[0], max(X[1], X[2]));
    const int mny = min(Y[0], min(Y[1], Y[2])), mxy = max(Y[0], max(Y[1], Y[2]));
    const int px0 = max((mnx + 255) >> 8, tl.x0), px1 = min(mxx >> 8, tl.x1);
    const int py0 = max((mny + 255) >> 8, tl.y0), py1 = min(mxy >> 8, tl.y1);
    if (px0 > px1 || py0 > py1) return true;
    const int boxpx = (px1 - px0 + 1) * (py1 - py0 + 1);
    const uint32_t box = (uint32_t)(px0 - tl.x0) | ((uint32_t)(px1 - tl.x0) << 8) | ((uint32_t)(py0 - tl.y0) << 16) |
                         ((uint32_t)(py1 - tl.y0) << 24);
    if (boxpx <= kSmallArea && mxx - mnx < (1 << 14) && mxy - mny < (1 << 14)) {
        raster_small(keys, tile_w, tl, rmin, X, Y, px0, px1, py0, py1, pl, (double)cam.cx, (double)cam.cy, id);
        return true;
    }
    const int k = atomicAdd(&Q.big.n, 1);
    if (k >= kQCap) return false;              // queue full: queued again in another pass of the round
    int Xr[3], Yr[3];
    double m[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = i == 2 ? 0 : i + 1;
        const int dx = X[i1] - X[i], dy = Y[i1] - Y[i];
        Xr[i] = X[i] - 256 * tl.x0;
        Yr[i] = Y[i] - 256 * tl.y0;
        m[i] = dy != 0 ? (double)dx / (double)dy : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) { Q.big.X[i][k] = Xr[i]; Q.big.Y[i][k] = Yr[i]; Q.big.m[i][k] = m[i]; }
    Q.big.pa[k] = pl.a; Q.big.pb[k] = pl.b; Q.big.pe[k] = pl.e;
    Q.big.id[k] = id;
    Q.big.box[k] = box;
    const int b0 = (py0 - tl.y0) / kBand, b1 = (py1 - tl.y0) / kBand;
    const int j0 = atomicAdd(&Q.big.njobs, b1 - b0 + 1);
    for (int b = b0; b <= b1; ++b) Q.big.job[j0 + b - b0] = (uint16_t)((k << 4) | b);
    return true;
}

__device__ __forceinline__ float3 sel3(int k, float3 a, float3 b, float3 c) {
    return k == 0 ? a : (k == 1 ? b : c);
}

// A mesh triangle's inputs, gathered ahead of use: the rounds of a tile
// pipeline these loads (bin entry, then vertex indices, then vertices) so
// that the dependent global gathers overlap earlier rounds' work.
struct TriIn {
    int32_t t;             // triangle id, -1 for none
    float v[9];            // world vertices
};

__device__ __forceinline__ void load_indices(const int32_t* __restrict__ tri, uint32_t vmax, int32_t t,
                                             uint32_t I[3]) {
    if (t < 0) { I[0] = I[1] = I[2] = 0; return; }
#pragma unroll
    for (int k = 0; k < 3; ++k) I[k] = min((uint32_t)tri[3 * (int64_t)t + k], vmax);
}

__device__ __forceinline__ void load_vertices(const float* __restrict__ xyz, int32_t t, const uint32_t I[3],
                                              TriIn& o) {
    o.t = t;
    if (t < 0) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o.v[3 * k] = xyz[3 * (int64_t)I[k]];
        o.v[3 * k + 1] = xyz[3 * (int64_t)I[k] + 1];
        o.v[3 * k + 2] = xyz[3 * (int64_t)I[k] + 2];
    }
}

// Whole contract for one mesh triangle: transform, far cull, near clip into
// at most two sub-triangles (same id), setup and rasterization.  Sub-triangle
// k is left out where bit k of skip is set; returns the mask of the
// sub-triangles that found the band queue full (0: the triangle is done).
template <int MODE>
__device__ __forceinline__ int raster_triangle(uint64_t* keys, int tile_w, Queues& q, const float* rmin,
                                               const Tile& tl, const CamF& cam, double ifx, double ify,
                                               const PoseF& P, const TriIn& in, int skip) {
    const float x0 = in.v[0], y0 = in.v[1], z0 = in.v[2];
    const float3 V0 = cam_contract(P, x0, y0, z0);
    const float3 V1 = cam_contract(P, in.v[3], in.v[4], in.v[5]);
    const float3 V2 = cam_contract(P, in.v[6], in.v[7], in.v[8]);
    if (V0.z > cam.zf && V1.z > cam.zf && V2.z > cam.zf) return 0;
    const bool in0 = V0.z >= cam.zn, in1 = V1.z >= cam.zn, in2 = V2.z >= cam.zn;
    const int nin = (int)in0 + (int)in1 + (int)in2;
    if (nin == 0) return 0;
    const PlaneN pn = plane_normal(P, in.v);
    // 1/z over the triangle peaks at its nearest vertex; one pixel of plane
    // extrapolation covers the snapping.  Behind the tile's farthest key at
    // the round start, no pixel of the triangle can change:
    // (1/z_min + |a| + |b|) (1 + 1e-5) < w_key.  Outside ICP mode the test is
    // taken multiplied by z_min |c| > 0, so that a skipped triangle needs no
    // division (c = 0, a plane through the camera centre, is never skipped);
    // in ICP mode the plane first (fewer registers live across the test there).
    WPlane pl;
    if constexpr (MODE == kIcp) {
        pl = depth_plane(pn, ifx, ify);
        if (nin == 3) {
            const double wv = 1.0 / (double)fminf(V0.z, fminf(V1.z, V2.z)) + fabs(pl.a) + fabs(pl.b);
            if (wv * 1.00001 < (double)rmin[kSnapTile]) return 0;
        }
    } else {
        if (nin == 3) {
            const double zmin = (double)fminf(V0.z, fminf(V1.z, V2.z));
            const double ac = fabs(pn.c);
            const double lhs = (ac + zmin * (fabs(pn.nx) * ifx + fabs(pn.ny) * ify)) * 1.00001;
            if (lhs < (double)rmin[kSnapTile] * zmin * ac) return 0;
        }
        pl = depth_plane(pn, ifx, ify);
    }
    const uint32_t id = (uint32_t)in.t;
    // near-plane clip into at most two sub-triangles; one emit call site keeps
    // a single copy of the setup and rasterization code
    float3 A0 = V0, B0 = V1, C0 = V2, A1 = V0, B1 = V1, C1 = V2;
    int nsub = 1;
    if (nin == 2) {
        const int k = !in0 ? 0 : (!in1 ? 1 : 2);          // the outside vertex
        const float3 O = sel3(k, V0, V1, V2);
        const float3 a = sel3(k == 2 ? 0 : k + 1, V0, V1, V2);
        const float3 b = sel3(k == 0 ? 2 : k - 1, V0, V1, V2);
        const float3 Pb = clip_point(b, O, cam.zn);
        const float3 Pa = clip_point(a, O, cam.zn);
        A0 = a; B0 = b; C0 = Pb;
        A1 = a; B1 = Pb; C1 = Pa;
        nsub = 2;
    } else if (nin == 1) {
        const int k = in0 ? 0 : (in1 ? 1 : 2);            // the inside vertex
        const float3 I = sel3(k, V0, V1, V2);
        const float3 a = sel3(k == 2 ? 0 : k + 1, V0, V1, V2);
        const float3 b = sel3(k == 0 ? 2 : k - 1, V0, V1, V2);
        A0 = I; B0 = clip_point(I, a, cam.zn); C0 = clip_point(I, b, cam.zn);
    }
    int left = 0;
#pragma unroll 1
    for (int sub = 0; sub < nsub; ++sub) {
        if ((skip >> sub) & 1) continue;
        const float3 A = sub ? A1 : A0, B = sub ? B1 : B0, C = sub ? C1 : C0;
        if (!emit_tri(keys, tile_w, q, rmin, tl, cam, A, B, C, pl, id)) left |= 1 << sub;
    }
    return left;
}

// ------------------------------------------------------------------ binning

// Conservative screen footprint of a triangle for binning: approximate
// float32 camera transform, clip against a plane slightly in front of z_near,
// projection with the hardware reciprocal; the exact contract is applied
// later, per tile, so this only has to contain it, widened by the margin m.
struct Foot {
    float u[4], v[4];      // convex polygon; a triangle repeats its last vertex
    float m;               // margin, px
};

// Base margin: covers the 1/512 px vertex snap, the hardware reciprocal and
// the float32 projection; the float32 camera-centre rounding is added per
// triangle.
constexpr float kBinMargin = 0.25f;

__device__ __forceinline__ void proj_approx(const CamF& cam, float3 X, float& u, float& v) {
    const float r = __builtin_amdgcn_rcpf(X.z);
    u = fmaf(cam.fx * X.x, r, cam.cx);
    v = fmaf(cam.fy * X.y, r, cam.cy);
}

__device__ __forceinline__ float3 clip_approx(float3 I, float3 O, float zc) {
    const float t = (zc - I.z) / (O.z - I.z);
    return make_float3(fmaf(t, O.x - I.x, I.x), fmaf(t, O.y - I.y, I.y), zc);
}

__device__ __forceinline__ bool footprint(const PoseF& P, const CamF& cam, float3 W0, float3 W1, float3 W2,
                                          Foot& f) {
    float3 V[3];
    const float3 Wv[3] = {W0, W1, W2};
    float dm = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float d0 = Wv[k].x - P.tf[0], d1 = Wv[k].y - P.tf[1], d2 = Wv[k].z - P.tf[2];
        dm = fmaxf(dm, fabsf(d0) + fabsf(d1) + fabsf(d2));
        V[k].x = fmaf(P.R[0][2], d2, fmaf(P.R[0][1], d1, P.R[0][0] * d0));
        V[k].y = fmaf(P.R[1][2], d2, fmaf(P.R[1][1], d1, P.R[1][0] * d0));
        V[k].z = fmaf(P.R[2][2], d2, fmaf(P.R[2][1], d1, P.R[2][0] * d0));
    }
    const float s = V[0].x + V[0].y + V[0].z + V[1].x + V[1].y + V[1].z + V[2].x + V[2].y + V[2].z;
    if (!isfinite(s)) return false;
    const float znp = cam.zn * (1.0f - 1e-4f), zfp = cam.zf * (1.0f + 1e-4f);
    const bool in0 = V[0].z >= znp, in1 = V[1].z >= znp, in2 = V[2].z >= znp;
    const int nin = (int)in0 + (int)in1 + (int)in2;
    if (nin == 0) return false;
    if (V[0].z > zfp && V[1].z > zfp && V[2].z > zfp) return false;
    float3 Q0, Q1, Q2, Q3;
    if (nin == 3) {
        Q0 = V[0]; Q1 = V[1]; Q2 = V[2]; Q3 = V[2];
    } else if (nin == 2) {
        const int k = !in0 ? 0 : (!in1 ? 1 : 2);
        const float3 O = sel3(k, V[0], V[1], V[2]);
        const float3 a = sel3(k == 2 ? 0 : k + 1, V[0], V[1], V[2]);
        const float3 b = sel3(k == 0 ? 2 : k - 1, V[0], V[1], V[2]);
        Q0 = a; Q1 = b; Q2 = clip_approx(b, O, znp); Q3 = clip_approx(a, O, znp);
    } else {
        const int k = in0 ? 0 : (in1 ? 1 : 2);
        const float3 I = sel3(k, V[0], V[1], V[2]);
        const float3 a = sel3(k == 2 ? 0 : k + 1, V[0], V[1], V[2]);
        const float3 b = sel3(k == 0 ? 2 : k - 1, V[0], V[1], V[2]);
        Q0 = I; Q1 = clip_approx(I, a, znp); Q2 = clip_approx(I, b, znp); Q3 = Q2;
    }
    // The contract subtracts the camera centre in FP64 before rounding; here
    // it is rounded first.  Per camera coordinate the two points differ by
    // less than 2^-24 (|t| + 9 |d|) (both roundings of the difference, both
    // float32 rotations), which moves the projection of a point of depth z
    // at most (f + |u - c|) / z times as far; bounded here with twice that,
    // the polygon's least depth, and |u - c| up to the larger image side.
    // (the hardware reciprocal's relative error, ~2^-22, is far inside the
    // factor 2 of the bound)
    const float zmin = fmaxf(fminf(Q0.z, fminf(Q1.z, fminf(Q2.z, Q3.z))), znp);
    const float tn = fabsf(P.tf[0]) + fabsf(P.tf[1]) + fabsf(P.tf[2]);
    f.m = kBinMargin + 0x1p-23f * (tn + 9.0f * dm) * (fmaxf(cam.fx, cam.fy) + (float)max(cam.W, cam.H)) *
                           __builtin_amdgcn_rcpf(zmin);
    proj_approx(cam, Q0, f.u[0], f.v[0]);
    proj_approx(cam, Q1, f.u[1], f.v[1]);
    proj_approx(cam, Q2, f.u[2], f.v[2]);
    if (nin == 3) { f.u[3] = f.u[2]; f.v[3] = f.v[2]; }       // a triangle repeats its last vertex
    else proj_approx(cam, Q3, f.u[3], f.v[3]);
    return true;
}

// Edge functions of the footprint polygon for the tile test: tile (tx, ty),
// its pixel centres widened by the margin, certainly misses the polygon when for
// some edge A x + B y + K < 0 at x = tx * TW, y = ty * TH (A, B the inward
// normal, K the offset to the rectangle corner farthest inside plus a
// tolerance above the float rounding of the evaluation).  Degenerate edges
// of a repeated vertex never exclude a tile.
struct FootEdges {
    float A[4], B[4], K[4];
};

template <int TW, int TH>
__device__ __forceinline__ FootEdges foot_edges(const Foot& f, float area2, float W, float H) {
    const float sg = area2 > 0.0f ? 1.0f : -1.0f;
    FootEdges g;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        const float A = -sg * (f.v[j] - f.v[i]), B = sg * (f.u[j] - f.u[i]);
        const float ox = A > 0.0f ? (float)(TW - 1) + f.m : -f.m, oy = B > 0.0f ? (float)(TH - 1) + f.m : -f.m;
        const float tol = 1e-4f * (fabsf(A) + fabsf(B)) * (fabsf(f.u[i]) + fabsf(f.v[i]) + W + H + 8.0f) + 1e-6f;
        g.A[i] = A;
        g.B[i] = B;
        g.K[i] = A * (ox - f.u[i]) + B * (oy - f.v[i]) + tol;
    }
    return g;
}

// Row part of the test: K + B y for the tile row at y = ty * TH.
__device__ __forceinline__ void edges_row(const FootEdges& g, float y, float k[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) k[i] = fmaf(g.B[i], y, g.K[i]);
}

__device__ __forceinline__ bool edges_hit(const FootEdges& g, const float k[4], float x) {
    bool hit = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) hit &= !(fmaf(g.A[i], x, k[i]) < 0.0f);
    return hit;
}

__device__ __forceinline__ int pose_scan(const BatchDesc& bd, int pose) {
    int s = 0;
    while (s + 1 < bd.n_scans && pose >= bd.s[s + 1].pose_off) ++s;
    return s;
}

// Workgroups loop over (pose, visible cluster) items; each thread bins its
// triangle into the (pose, tile) bins its footprint touches.  Tile counts of
// the two size classes are aggregated in LDS over the cluster's tile
// rectangle, then reserved with one global atomic per (workgroup, tile,
// class).  Small footprints fill a bin from the front, large ones from the
// back, so that the tile pass sees triangles of similar cost together; each
// class has its own part of the bin (bin_cap - bin_big_cap small slots,
// bin_big_cap large ones), so the two never overwrite each other.
//
// SPILL = true: entries past their class's part are not dropped but written
// to the spill list with their record and slot, for k_spill_scatter to place
// in the record's overflow region.  A band's spilled entries take one range
// of the list (offsets within it from an LDS counter, the range from one
// global atomic); a band whose range does not fit marks its spilling
// records lost instead.
constexpr float kBigFootprint = 100.0f;    // bounding box area widened by 2 px per side, px
constexpr uint32_t kBigSlot = 0x80000000u; // slot code of a large entry in the spill list

// (six workgroups per CU: the plain variant fits them anyway; the spilling
// one, at 88 registers, would drop to five, which measured 3 % slower)
template <int TW, int TH, bool SPILL>
__global__ void __launch_bounds__(kWG, 6) k_bin(BatchDesc bd, RasterArgs a, int32_t table_n) {
    // per tile of a band of a cluster's rectangle: small count | large count
    // << 16 (then cursors), the two reservations and, with SPILL, the two
    // spill-list bases.  table_n = the largest tile grid of the launch, at
    // most kBinTable, so that the LDS size follows the images of the call; a
    // rectangle with more tiles is binned in bands of whole tile rows
    // (table_n >= its width: rows hold at most kMaxTileGrid <= kBinTable tiles).
    extern __shared__ uint32_t tables[];
    uint32_t* tcnt = tables;
    uint32_t* tbs = tables + table_n;
    uint32_t* tbb = tables + 2 * table_n;
    uint32_t* tss = tables + 3 * table_n;    // spill offsets within the band's range
    uint32_t* tsb = tables + 4 * table_n;
    __shared__ uint32_t band_spill;            // entries the band spills, then whether its range fits
    __shared__ unsigned long long band_base;
    const int pose = blockIdx.y;
    const int nvis = a.vis_count[pose];
    const ScanDesc& sd = bd.s[pose_scan(bd, pose)];
    const CamF cam{sd.fx, sd.fy, sd.cx, sd.cy, sd.z_near, sd.z_far, sd.width, sd.height};
    PoseF P;
    load_pose(a.T_wc + 12 * (int64_t)pose, P);
    const int pl = pose - sd.pose_off;
    const int ntile = sd.tiles_x * sd.tiles_y;
    const int64_t rec0 = sd.rec_off + (int64_t)pl * ntile;
    const uint32_t cap = (uint32_t)a.bin_cap;
    const uint32_t cap_b = (uint32_t)a.bin_big_cap, cap_s = cap - cap_b;
    int fs = 0, fb = 0;                        // largest fills this thread reserved (for bin_fill)
    for (int k = blockIdx.x; k < nvis; k += gridDim.x) {
        const uint2 e = a.vis[(int64_t)pose * a.n_clusters + k];
        const int rx0 = e.y & 0xff, rx1 = (e.y >> 8) & 0xff, ry0 = (e.y >> 16) & 0xff, ry1 = e.y >> 24;
        const int rw = rx1 - rx0 + 1;
        const int brows = min(ry1 - ry0 + 1, table_n / rw);     // tile rows per band
        __syncthreads();                       // previous item's tables are no longer read
        for (int i = threadIdx.x; i < brows * rw; i += kWG) tcnt[i] = 0;
        const int64_t t = (int64_t)e.x * kClusterTris + threadIdx.x;
        Foot f;
        bool ok = false, big = false;
        int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1;
        float area2 = 0.0f;
        if (t < a.n_tris) {
            const uint32_t i0 = min((uint32_t)a.tri[3 * t], a.vmax), i1 = min((uint32_t)a.tri[3 * t + 1], a.vmax),
                           i2 = min((uint32_t)a.tri[3 * t + 2], a.vmax);
            const float3 W0 = make_float3(a.xyz[3 * (int64_t)i0], a.xyz[3 * (int64_t)i0 + 1], a.xyz[3 * (int64_t)i0 + 2]);
            const float3 W1 = make_float3(a.xyz[3 * (int64_t)i1], a.xyz[3 * (int64_t)i1 + 1], a.xyz[3 * (int64_t)i1 + 2]);
            const float3 W2 = make_float3(a.xyz[3 * (int64_t)i2], a.xyz[3 * (int64_t)i2 + 1], a.xyz[3 * (int64_t)i2 + 2]);
            ok = footprint(P, cam, W0, W1, W2, f);
            if (ok) {
                float umin = f.u[0], umax = f.u[0], vmin = f.v[0], vmax = f.v[0];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = (i + 1) & 3;
                    umin = fminf(umin, f.u[i]); umax = fmaxf(umax, f.u[i]);
                    vmin = fminf(vmin, f.v[i]); vmax = fmaxf(vmax, f.v[i]);
                    area2 += f.u[i] * f.v[j] - f.u[j] * f.v[i];
                }
                big = (umax - umin + 4.0f) * (vmax - vmin + 4.0f) > kBigFootprint;
                umin -= f.m; vmin -= f.m; umax += f.m; vmax += f.m;
                const float W1f = (float)(cam.W - 1), H1f = (float)(cam.H - 1);
                ok = umax >= 0.0f && vmax >= 0.0f && umin <= W1f && vmin <= H1f;
                if (ok) {
                    tx0 = max((int)fmaxf(umin, 0.0f) / TW, rx0);
                    tx1 = min((int)fminf(umax, W1f) / TW, rx1);
                    ty0 = max((int)fmaxf(vmin, 0.0f) / TH, ry0);
                    ty1 = min((int)fminf(vmax, H1f) / TH, ry1);
                }
            }
        }
        // tiles the footprint touches: a bit mask over its tile rectangle with
        // rows at a power-of-two stride (bit r << ls | c for tile (tx0 + c,
        // ty0 + r)) when that fits in 64 bits, otherwise tested again per pass
        const int sw = tx1 - tx0 + 1, sh = ty1 - ty0 + 1;
        const int nspan = ok ? sw * sh : 0;
        const int ls = sw <= 1 ? 0 : 32 - __clz(sw - 1);
        const bool masked = (sh << ls) <= 64;
        const bool test_tiles = nspan > 2 && fabsf(area2) > 1e-3f;
        // (the edge functions only where the tile test runs: a wave whose
        // footprints all span at most two tiles skips them)
        FootEdges g = {};
        if (test_tiles) g = foot_edges<TW, TH>(f, area2, (float)cam.W, (float)cam.H);
        uint64_t hits = 0;
        if (nspan > 0 && masked) {
            if (!test_tiles) {
                const uint64_t row = ~0ull >> (64 - sw);
                for (int r = 0; r < sh; ++r) hits |= row << (r << ls);
            } else {
                for (int r = 0; r < sh; ++r) {
                    float k[4];
                    edges_row(g, (float)((ty0 + r) * TH), k);
                    for (int c = 0; c < sw; ++c)
                        if (edges_hit(g, k, (float)((tx0 + c) * TW))) hits |= 1ull << ((r << ls) | c);
                }
            }
        }
        const uint32_t inc = big ? 0x10000u : 1u;
        for (int by0 = ry0;;) {
            const int by1 = min(ry1, by0 + brows - 1);
            const int nb = (by1 - by0 + 1) * rw;
            // the footprint's tile rows inside this band
            const int r0 = max(ty0, by0) - ty0, r1 = min(ty1, by1) - ty0;
            // (bits [r0 << ls, (r1 + 1) << ls) of the mask; r0 << ls < 64 when masked)
            const uint64_t band_bits =
                !masked || r0 > r1
                    ? 0ull
                    : (((r1 + 1) << ls) >= 64 ? ~0ull : (1ull << ((r1 + 1) << ls)) - 1ull) & ~((1ull << (r0 << ls)) - 1ull);
            __syncthreads();                   // the band's counters are zero
            if (masked) {
                for (uint64_t m = hits & band_bits; m; m &= m - 1) {      // only the tiles hit
                    const int i = __ffsll((unsigned long long)m) - 1;
                    atomicAdd(&tcnt[(ty0 + (i >> ls) - by0) * rw + (tx0 + (i & ((1 << ls) - 1)) - rx0)], inc);
                }
            } else {
                for (int r = r0; r <= r1; ++r) {
                    float k[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (test_tiles) edges_row(g, (float)((ty0 + r) * TH), k);
                    for (int c = 0; c < sw; ++c)
                        if (!test_tiles || edges_hit(g, k, (float)((tx0 + c) * TW)))
                            atomicAdd(&tcnt[(ty0 + r - by0) * rw + (tx0 + c - rx0)], inc);
                }
            }
            if (SPILL && threadIdx.x == 0) band_spill = 0;
            __syncthreads();
            uint32_t spilled = 0;                  // bit j: tile threadIdx.x + j kWG reserved list space
            for (int i = threadIdx.x, j = 0; i < nb; i += kWG, ++j) {
                const uint32_t n = tcnt[i];
                if (n) {
                    const int tile = (by0 + i / rw) * sd.tiles_x + rx0 + i % rw;
                    const int64_t rec = rec0 + tile;
                    if (n & 0xffffu) {
                        const uint32_t s0 = (uint32_t)atomicAdd(a.bin_small + rec, (int)(n & 0xffffu));
                        tbs[i] = s0;
                        fs = max(fs, (int)(s0 + (n & 0xffffu)));
                        if (SPILL && s0 + (n & 0xffffu) > cap_s) {
                            tss[i] = atomicAdd(&band_spill, s0 + (n & 0xffffu) - max(s0, cap_s));
                            spilled |= 1u << j;
                        }
                    }
                    if (n >> 16) {
                        const uint32_t b0 = (uint32_t)atomicAdd(a.bin_big + rec, (int)(n >> 16));
                        tbb[i] = b0;
                        fb = max(fb, (int)(b0 + (n >> 16)));
                        if (SPILL && b0 + (n >> 16) > cap_b) {
                            tsb[i] = atomicAdd(&band_spill, b0 + (n >> 16) - max(b0, cap_b));
                            spilled |= 1u << j;
                        }
                    }
                    tcnt[i] = 0;
                }
            }
            __syncthreads();
            if (SPILL) {
                // one range of the list for the band; if it does not fit,
                // the records that spilled here are lost
                if (threadIdx.x == 0 && band_spill) {
                    // the list is cut into kSpillLists segments with counters of
                    // their own, so that bands do not all contend for one address
                    const unsigned seg = (blockIdx.y * 131u + blockIdx.x) % kSpillLists;
                    const unsigned long long len = (unsigned long long)a.spill_cap / kSpillLists;
                    const unsigned long long sp = atomicAdd(a.spill_top + kSpillTops + seg, (unsigned long long)band_spill);
                    band_base = seg * len + sp;
                    band_spill = sp + band_spill <= len ? 1u : 2u;
                    // a range that crosses the end of its segment leaves its part
                    // below the end unwritten: the segment is valid below its start
                    if (sp < len && band_spill == 2u)
                        atomicMax(a.spill_top + kSpillTops + kSpillLists + seg, len - sp);
                }
                __syncthreads();
                if (band_spill == 2u)
                    for (uint32_t m = spilled; m; m &= m - 1) {
                        const int i = threadIdx.x + (__ffs(m) - 1) * kWG;
                        a.spill_lost[rec0 + (by0 + i / rw) * sd.tiles_x + rx0 + i % rw] = 1;
                    }
            }
            const bool band_ok = !SPILL || band_spill == 1u;
            const uint32_t sbase = SPILL ? (uint32_t)band_base : 0u;
            auto put = [&](int tx, int ty) {
                const int li = (ty - by0) * rw + (tx - rx0);
                const uint32_t old = atomicAdd(&tcnt[li], inc);
                const int64_t rec = rec0 + ty * sd.tiles_x + tx;
                uint32_t* bin = a.bins + rec * (int64_t)cap;
                if (big) {
                    const uint32_t slot = tbb[li] + (old >> 16);
                    if (slot < cap_b) {
                        bin[cap - 1 - slot] = (uint32_t)t;
                    } else if (SPILL && band_ok) {
                        const uint32_t j = sbase + tsb[li] + (slot - max(tbb[li], cap_b));
                        a.spill[j] = make_uint3((uint32_t)t, (uint32_t)rec, slot | kBigSlot);
                    }
                } else {
                    const uint32_t slot = tbs[li] + (old & 0xffffu);
                    if (slot < cap_s) {
                        bin[slot] = (uint32_t)t;
                    } else if (SPILL && band_ok) {
                        const uint32_t j = sbase + tss[li] + (slot - max(tbs[li], cap_s));
                        a.spill[j] = make_uint3((uint32_t)t, (uint32_t)rec, slot);
                    }
                }
            };
            if (masked) {
                for (uint64_t m = hits & band_bits; m; m &= m - 1) {
                    const int i = __ffsll((unsigned long long)m) - 1;
                    put(tx0 + (i & ((1 << ls) - 1)), ty0 + (i >> ls));
                }
            } else {
                for (int r = r0; r <= r1; ++r) {
                    float k[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (test_tiles) edges_row(g, (float)((ty0 + r) * TH), k);
                    for (int c = 0; c < sw; ++c)
                        if (!test_tiles || edges_hit(g, k, (float)((tx0 + c) * TW))) put(tx0 + c, ty0 + r);
                }
            }
            by0 = by1 + 1;
            if (by0 > ry1) break;
            __syncthreads();                   // the put cursors of this band are no longer read
            for (int i = threadIdx.x; i < brows * rw; i += kWG) tcnt[i] = 0;
        }
    }
    if (a.bin_fill) {                          // only when the host sizes the bins of a new shape
        // (once per wave at the end: per band, these few addresses were contended)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            fs = max(fs, __shfl_xor(fs, off));
            fb = max(fb, __shfl_xor(fb, off));
        }
        if ((threadIdx.x & 63) == 0 && (fs | fb)) {
            atomicMax(a.bin_fill, fs);
            atomicMax(a.bin_fill + 1, fb);
        }
    }
}

// One thread per record: a record whose bin spilled gets an overflow region
// for all its entries (laid out like a bin of exactly its fill: small
// entries ascending from the start, large ones descending from the end),
// unless its spill was lost or the regions are full.  spill_top[1] is the
// region cursor, spill_top[2] counts the records that spilled and
// spill_top[4] totals their fills (what the regions would need); each
// region's record is listed in spill_recs for k_region_fill.  Regions are
// handed out in the order the atomics land; results do not depend on where
// they lie.
__global__ void __launch_bounds__(kWG) k_region_alloc(RasterArgs a, int64_t n) {
    const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (r == 0) {
        // what the list must hold: its segments are filled alike, so as many
        // times the fullest segment as there are segments
        unsigned long long m = 0;
        for (int s = 0; s < kSpillLists; ++s) m = max(m, a.spill_top[kSpillTops + s]);
        a.spill_top[0] = m * kSpillLists;
    }
    if (r >= n) return;
    const int ns = a.bin_small[r], nb = a.bin_big[r];
    int64_t off = -1;
    if (ns > a.bin_cap - a.bin_big_cap || nb > a.bin_big_cap) {
        const unsigned long long k = atomicAdd(a.spill_top + 2, 1ull);
        atomicAdd(a.spill_top + 4, (unsigned long long)(ns + nb));
        if (!a.spill_lost[r]) {
            const unsigned long long o = atomicAdd(a.spill_top + 1, (unsigned long long)(ns + nb));
            if (o + (unsigned long long)(ns + nb) <= (unsigned long long)a.pool_cap) {
                off = (int64_t)o;
                a.spill_recs[k] = (int32_t)r;
            } else {
                a.spill_recs[k] = -1;
            }
        } else {
            a.spill_recs[k] = -1;
        }
    }
    a.pool_off[r] = off;
}

// One workgroup per listed record at a time: copies the entries its bin
// kept (the small part's front, the large part's back) into its region.
__global__ void __launch_bounds__(kWG) k_region_fill(RasterArgs a) {
    const unsigned long long n = a.spill_top[2];
    const int cap_b = a.bin_big_cap, cap_s = a.bin_cap - cap_b;
    for (unsigned long long k = blockIdx.x; k < n; k += gridDim.x) {
        const int32_t r = a.spill_recs[k];
        if (r < 0) continue;
        const int ns = a.bin_small[r], nb = a.bin_big[r], cnt = ns + nb;
        const uint32_t* bin = a.bins + (int64_t)r * a.bin_cap;
        uint32_t* reg = a.pool + a.pool_off[r];
        const int ks = min(ns, cap_s), kb = min(nb, cap_b);
        for (int i = threadIdx.x; i < ks + kb; i += kWG) {
            if (i < ks) reg[i] = bin[i];
            else reg[cnt - 1 - (i - ks)] = bin[a.bin_cap - 1 - (i - ks)];
        }
    }
}

// Places each spilled entry at its slot in its record's region (entries of
// records without a region stay out); blockIdx.y is the list segment.  Every
// entry of a segment below the start of its first range that crossed the
// segment's end was written by this call.
__global__ void __launch_bounds__(kWG) k_spill_scatter(RasterArgs a, int64_t n_records) {
    const unsigned seg = blockIdx.y;
    const unsigned long long len = (unsigned long long)a.spill_cap / kSpillLists;
    const unsigned long long n = min(a.spill_top[kSpillTops + seg], len - a.spill_top[kSpillTops + kSpillLists + seg]);
    for (unsigned long long j = (unsigned long long)blockIdx.x * kWG + threadIdx.x; j < n;
         j += (unsigned long long)gridDim.x * kWG) {
        const uint3 e = a.spill[seg * len + j];
        if ((int64_t)e.y >= n_records) continue;      // (never: each entry names a record of the call)
        const int64_t off = a.pool_off[e.y];
        if (off < 0) continue;
        const int cnt = a.bin_small[e.y] + a.bin_big[e.y];
        const int slot = (int)(e.z & ~kBigSlot);
        const int at = e.z & kBigSlot ? cnt - 1 - slot : slot;
        if (at >= 0 && at < cnt) a.pool[off + at] = e.x;
    }
}

// ------------------------------------------------------------------ per-pixel comparison

struct Acc {
    int e_table;
    int cnt[9];
    int n_active;
    float e_soft;          // ICP mode: the cost sum |Z_M - Z_1| of the associated pixels
    float jtr[6];
    float jtj[21];
    float sse;             // ICP mode: sum of squared point-to-plane residuals
    int col[2];            // color term: rewarded, penalized corresponding pixels
};

// Table I cell of a pixel and its value: returns the cell (0..8) and sets s.
__device__ __forceinline__ int table1(int c_r, int c_s, float dz, float eps, int& s) {
    s = 0;
    if (c_s == RM_NONE || c_s == RM_UO) return 6;
    if (c_r == RM_NONE || c_r == RM_UO) return 7;
    if (c_r == RM_FO && c_s == RM_FO) { const bool pen = fabsf(dz) > eps; s = pen ? 1 : -1; return pen ? 1 : 0; }
    if (c_r == RM_FO && c_s == RM_FU) { const bool pen = dz <= 0.0f; s = pen ? 1 : -1; return pen ? 3 : 2; }
    if (c_r == RM_FU && c_s == RM_FO) { const bool pen = dz > 0.0f; s = pen ? 1 : -1; return pen ? 5 : 4; }
    return 8;
}

// ------------------------------------------------------------------ kernels

struct ItemInfo {
    int scan;
    int pose;          // global pose index
    int pose_local;
    int tile;
    int64_t rec;
};

__device__ __forceinline__ bool decode_item(const BatchDesc& bd, ItemInfo& it) {
    // XCD-aware order: consecutive blocks land on different XCDs (round
    // robin), so block b takes item (b % 8) * chunk + b / 8 and each XCD
    // works through a contiguous run of (tile-major, pose-minor) items, i.e.
    // the same screen tiles for neighbouring poses, which share triangles.
    const int64_t b = blockIdx.x;
    const int64_t chunk = (int64_t)gridDim.x / 8;
    const int64_t item = (b % 8) * chunk + b / 8;
    if (item >= bd.n_items) return false;
    int s = 0;
    while (s + 1 < bd.n_scans && item >= bd.s[s + 1].item_off) ++s;
    const ScanDesc& sd = bd.s[s];
    const int64_t local = item - sd.item_off;
    it.scan = s;
    it.tile = (int)(local / sd.n_poses);
    it.pose_local = (int)(local % sd.n_poses);
    it.pose = sd.pose_off + it.pose_local;
    it.rec = sd.rec_off + (int64_t)it.pose_local * (sd.tiles_x * sd.tiles_y) + it.tile;
    return true;
}

// Item of a partial-record index (persistent scheduling takes items by record).
__device__ __forceinline__ void decode_rec(const BatchDesc& bd, int64_t rec, ItemInfo& it) {
    int s = 0;
    while (s + 1 < bd.n_scans && rec >= bd.s[s + 1].rec_off) ++s;
    const ScanDesc& sd = bd.s[s];
    const int64_t local = rec - sd.rec_off;
    const int nt = sd.tiles_x * sd.tiles_y;
    it.scan = s;
    it.pose_local = (int)(local / nt);
    it.tile = (int)(local % nt);
    it.pose = sd.pose_off + it.pose_local;
    it.rec = rec;
}

// A pointer whose value is the same in every lane, moved to scalar registers.
__device__ __forceinline__ const uint32_t* uniform_ptr(const uint32_t* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return reinterpret_cast<const uint32_t*>((uint64_t)hi << 32 | lo);
}

// One (scan, pose, tile) item: rasterization rounds, resolve, tile record.
template <int TW, int TH, int MODE, bool OVF>
__device__ __forceinline__ void tile_pass(const BatchDesc& bd, const RasterArgs& a, const ItemInfo& it,
                                          uint64_t* keys, Queues& q, float (*red)[kRecFields]) {
    const ScanDesc& sd = bd.s[it.scan];
    CamF cam{sd.fx, sd.fy, sd.cx, sd.cy, sd.z_near, sd.z_far, sd.width, sd.height};
    const float ifx = 1.0f / cam.fx, ify = 1.0f / cam.fy;
    const double difx = (double)ifx, dify = (double)ify;
    const double dcx = (double)cam.cx, dcy = (double)cam.cy;
    const float w_far = 1.0f / cam.zf;
    const int tx = it.tile % sd.tiles_x, ty = it.tile / sd.tiles_x;
    Tile tl;
    tl.x0 = tx * TW; tl.y0 = ty * TH;
    tl.x1 = min(tl.x0 + TW, cam.W) - 1; tl.y1 = min(tl.y0 + TH, cam.H) - 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int p = tid; p < TW * TH; p += kWG) keys[p] = kEmptyKey;

    PoseF P;
    load_pose(a.T_wc + 12 * (int64_t)it.pose, P);
    const int ns = a.bin_small[it.rec], nb = a.bin_big[it.rec];
    if (tid < 2) atomicMax(a.bin_max + tid, tid ? nb : ns);    // one instruction, two lanes

    // Rounds of kWG triangles: from the (pose, tile) bin, large footprints
    // (held at its back) before small ones (at its front), so that near
    // surfaces reach the depth snapshot early.  A bin that outgrew a part of
    // its capacity is read from its overflow region, which holds all its
    // entries in the same layout; without one, the tile takes every triangle
    // of every visible cluster of the pose (slower, same result).
    // (OVF: the call has overflow regions; the kernel without them is
    // compiled apart, as the mere presence of the region lookup costs the
    // common case about half a percent)
    const bool fits = ns <= a.bin_cap - a.bin_big_cap && nb <= a.bin_big_cap;
    const int64_t poff = OVF && !fits ? a.pool_off[it.rec] : -1;
    const bool use_bin = fits || poff >= 0;
    const int nvis = a.vis_count[it.pose];
    const uint2* vis = a.vis + (int64_t)it.pose * a.n_clusters;
    // (uniform over the workgroup: kept in scalar registers for the gather)
    const uint32_t* bin = OVF ? uniform_ptr(poff >= 0 ? a.pool + poff : a.bins + it.rec * (int64_t)a.bin_cap)
                              : a.bins + it.rec * (int64_t)a.bin_cap;
    const int bcap = OVF ? __builtin_amdgcn_readfirstlane(poff >= 0 ? ns + nb : a.bin_cap) : a.bin_cap;
    const int nr = use_bin ? (ns + nb + kWG - 1) / kWG : nvis;
    auto entry = [&](int r) -> int32_t {
        if (r >= nr) return -1;
        if (use_bin) {
            const int i = r * kWG + tid;
            if (i >= ns + nb) return -1;
            return (int32_t)(i < nb ? bin[bcap - 1 - i] : bin[i - nb]);
        }
        const int64_t t = (int64_t)vis[r].x * kClusterTris + tid;
        return t < a.n_tris ? (int32_t)t : -1;
    };
    // three-stage gather pipeline: round r processes vertices loaded during
    // round r-1 from indices loaded during r-2 from a bin entry read in r-3
    TriIn cur, nxt;
    uint32_t I1[3], I2[3];
    int32_t t1 = entry(0), t2, t3;
    load_indices(a.tri, a.vmax, t1, I1);
    load_vertices(a.xyz, t1, I1, cur);
    t1 = entry(1);
    load_indices(a.tri, a.vmax, t1, I1);
    t2 = entry(2);
    // The snapshot is refreshed after each of the first kSnapEvery rounds and
    // then after every kSnapEvery-th: the near surfaces arrive first, and an
    // older snapshot stays a valid bound (keys only move nearer), so later
    // rounds cull almost as well at a fraction of the cost.  Buffer cb is
    // read by the current round; a refresh fills the other and swaps.
    if (tid <= kSnapTile) q.rowmin[0][tid] = 0.0f;   // round 0 sees an empty buffer
    int cb = 0;
    for (int r = 0; r < nr; ++r) {
        const bool snap_now = r + 1 < nr && (r < kSnapEvery || r % kSnapEvery == 0);
        if (tid == 0) { q.big.n = 0; q.big.njobs = 0; }
        if (tid == 0 && snap_now) q.rowmin[cb ^ 1][kSnapTile] = __int_as_float(0x7f800000);
        const float* rmin = q.rowmin[cb];
        load_vertices(a.xyz, t1, I1, nxt);
        load_indices(a.tri, a.vmax, t2, I2);
        t3 = entry(r + 3);
        __syncthreads();
        // A sub-triangle that finds the band queue full is queued in another
        // pass once the queue has been drained; only its triangle id and the
        // mask of pending sub-triangles stay live, its inputs are gathered
        // again (only rounds with more large sub-triangles than the queue
        // holds, mostly a bin's first rounds, take further passes).
        int left = cur.t >= 0 ? raster_triangle<MODE>(keys, TW, q, rmin, tl, cam, difx, dify, P, cur, 0) : 0;
        int32_t t_left = left ? cur.t : -1;
        for (;;) {
            __syncthreads();
            const bool more = q.big.n > kQCap;   // some sub-triangle found the queue full
            if (q.big.njobs) raster_queue<TW, TH>(keys, q.big, tl, rmin, dcx, dcy);
            __syncthreads();
            if (!more) break;
            if (tid == 0) { q.big.n = 0; q.big.njobs = 0; }
            __syncthreads();
            if (t_left >= 0) {
                TriIn tri;
                uint32_t I[3];
                load_indices(a.tri, a.vmax, t_left, I);
                load_vertices(a.xyz, t_left, I, tri);
                left = raster_triangle<MODE>(keys, TW, q, rmin, tl, cam, difx, dify, P, tri, ~left & 3);
                if (!left) t_left = -1;
            }
        }
        // row and tile snapshot for the next round (w >= 0, so its bits order
        // like its value).  Pixel p = tid + k kWG lies in row p / TW, so the
        // kG lanes of a group cover one kSeg-pixel segment (or, for 8-pixel
        // tile rows, one row): a group minimum and one store per segment;
        // the tile's farthest is a wave minimum and one atomic per wave.
        if (snap_now) {
            constexpr int kG = TW < kSeg ? TW : kSeg;
            float* snap = q.rowmin[cb ^ 1];
            uint32_t tmin = 0x7f800000u;
            for (int p = tid; p < TW * TH; p += kWG) {
                const uint32_t wb = group_min<kG>((uint32_t)(keys[p] >> 32));
                if ((lane & (kG - 1)) == 0) snap[(p / TW) * kSegs + (p % TW) / kSeg] = __uint_as_float(wb);
                tmin = min(tmin, wb);
            }
            if (tid < TW * TH) {
                tmin = min(tmin, (uint32_t)__shfl_xor((int)tmin, 16));
                tmin = min(tmin, (uint32_t)__shfl_xor((int)tmin, 32));
                if constexpr (kG == 8) tmin = min(tmin, (uint32_t)__shfl_xor((int)tmin, 8));
                if (lane == 0) atomicMin((unsigned int*)&snap[kSnapTile], tmin);
            }
        }
        if (snap_now) cb ^= 1;
        cur = nxt;
        t1 = t2;
        I1[0] = I2[0]; I1[1] = I2[1]; I1[2] = I2[2];
        t2 = t3;
    }

    // ---------------------------------------------------------------- resolve
    Acc acc;
    acc.e_table = 0; acc.n_active = 0; acc.e_soft = 0.0f; acc.sse = 0.0f;
    acc.col[0] = 0; acc.col[1] = 0;
    // color term: both sides' intensities given (cost and gradient modes)
    const float* scol = MODE == kCost || MODE == kGrad ? sd.color : nullptr;
    const bool color = a.tri_color != nullptr && scol != nullptr;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc.cnt[k] = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc.jtr[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 21; ++k) acc.jtj[k] = 0.0f;

    const float eps = a.eps, ieps2 = 1.0f / (a.eps * a.eps);
    const int64_t img = (int64_t)cam.W * cam.H;
    for (int p = tid; p < TW * TH; p += kWG) {
        const int x = tl.x0 + p % TW, y = tl.y0 + p / TW;
        if (x > tl.x1 || y > tl.y1) continue;
        const uint64_t key = keys[(y - tl.y0) * TW + (x - tl.x0)];
        // The rasterizers offer fragments beyond the far plane too (w below
        // w_far); such a fragment is farther than any valid one, so it is
        // the pixel's key only where no valid fragment exists, and a key
        // beyond the far plane (or the empty key, w = 0) is no hit.
        const bool hit = __uint_as_float((uint32_t)(key >> 32)) >= w_far;
        const uint32_t id = ~(uint32_t)key;
        const float z = hit ? 1.0f / __uint_as_float((uint32_t)(key >> 32)) : __int_as_float(0x7fc00000);
        const int64_t pix = (int64_t)y * cam.W + x;
        if (MODE == kRender) {
            const int64_t o = (int64_t)it.pose * img + pix;
            if (a.depth_out) a.depth_out[o] = z;
            if (a.tri_out) a.tri_out[o] = hit ? (int32_t)id : -1;
            if (a.cls_out) a.cls_out[o] = hit ? a.cls[id] : (uint8_t)RM_NONE;
            continue;
        }
        if (sd.mask && !sd.mask[pix]) continue;
        const int c_r = hit ? (int)a.cls[id] : RM_NONE;
        const int c_s = sd.cls[pix];
        const float d_s = sd.depth[pix];
        const float dz = z - d_s;
        if (MODE == kIcp) {
            // Projective association (Sec. V): a scan return and the map FO
            // surface the pixel sees, whose depths differ by less than the
            // tolerance.  The model normal is the normalized sum of the
            // winner's vertex normals, in the camera frame, facing the camera.
            if (c_s != RM_FO) continue;
            acc.cnt[0] += 1;
            if (c_r != RM_FO) continue;
            const int32_t* tv = a.tri + 3 * (int64_t)id;
            const float* n0 = a.vnrm + 3 * (int64_t)min((uint32_t)tv[0], a.vmax);
            const float* n1 = a.vnrm + 3 * (int64_t)min((uint32_t)tv[1], a.vmax);
            const float* n2 = a.vnrm + 3 * (int64_t)min((uint32_t)tv[2], a.vmax);
            const float w0 = (n0[0] + n1[0]) + n2[0], w1 = (n0[1] + n1[1]) + n2[1], w2 = (n0[2] + n1[2]) + n2[2];
            float nx = fmaf(P.R[0][2], w2, fmaf(P.R[0][1], w1, P.R[0][0] * w0));
            float ny = fmaf(P.R[1][2], w2, fmaf(P.R[1][1], w1, P.R[1][0] * w0));
            float nz = fmaf(P.R[2][2], w2, fmaf(P.R[2][1], w1, P.R[2][0] * w0));
            const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
            if (!(nn > 0.0f) || isinf(nn)) continue;                // a vertex normal is undefined
            acc.cnt[1] += 1;
            if (!(fabsf(dz) < a.eps)) continue;
            const float inv = 1.0f / sqrtf(nn);
            nx *= inv; ny *= inv; nz *= inv;
            const float rx = ((float)x - cam.cx) * ifx, ry = ((float)y - cam.cy) * ify;
            float ndr = fmaf(nx, rx, fmaf(ny, ry, nz));
            if (!(ndr < 0.0f)) { nx = -nx; ny = -ny; nz = -nz; ndr = -ndr; }
            // e = n . (P_1 - P_M) = (z_1 - z_M)(n . r); J = [n ; P_1 x n]
            const float e = (d_s - z) * ndr;
            const float Px = d_s * rx, Py = d_s * ry, Pz = d_s;
            float J[6];
            J[0] = nx; J[1] = ny; J[2] = nz;
            J[3] = Py * nz - Pz * ny;
            J[4] = Pz * nx - Px * nz;
            J[5] = Px * ny - Py * nx;
            acc.n_active += 1;
            acc.e_soft += fabsf(dz);
            acc.sse = fmaf(e, e, acc.sse);
#pragma unroll
            for (int i = 0; i < 6; ++i) acc.jtr[i] = fmaf(e, J[i], acc.jtr[i]);
            int k = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = i; j < 6; ++j) { acc.jtj[k] = fmaf(J[i], J[j], acc.jtj[k]); ++k; }
            continue;
        }
        int s;
        const int cell = table1(c_r, c_s, dz, eps, s);
        acc.e_table += s;
#pragma unroll
        for (int k = 0; k < 9; ++k) acc.cnt[k] += cell == k;
        if (color && cell == 0) {
            // corresponding pixel: the triangle's and the scan's intensities
            // agree within color_tol (float32 difference, both finite)
            const float cm = a.tri_color[id], cs = scol[pix];
            if (isfinite(cm) && isfinite(cs)) {
                const bool agree = fabsf(cm - cs) <= a.color_tol;
                acc.col[0] += agree;
                acc.col[1] += !agree;
            }
        }
        if (cell >= 6) continue;
        // Camera-frame unit normal n of the winning triangle and g = |n . ray|:
        // e = dz g is the scan point's signed distance from that triangle's plane.
        const float* nw = a.nrm + 3 * (int64_t)id;
        const float w0 = nw[0], w1 = nw[1], w2 = nw[2];
        const float nx = fmaf(P.R[0][2], w2, fmaf(P.R[0][1], w1, P.R[0][0] * w0));
        const float ny = fmaf(P.R[1][2], w2, fmaf(P.R[1][1], w1, P.R[1][0] * w0));
        const float nz = fmaf(P.R[2][2], w2, fmaf(P.R[2][1], w1, P.R[2][0] * w0));
        const float rx = ((float)x - cam.cx) * ifx, ry = ((float)y - cam.cy) * ify;
        const float nr = fmaf(nx, rx, fmaf(ny, ry, nz));
        const float e = dz * fabsf(nr);
        float r;
        bool moving;
        if (cell <= 1) { r = e; moving = true; }
        else if (cell <= 3) { r = fminf(e, 0.0f); moving = dz < 0.0f; }
        else { r = fmaxf(e, 0.0f); moving = dz > 0.0f; }
        const float q = r * r * ieps2;
        acc.e_soft += 2.0f * fminf(q, 1.0f) - 1.0f;
        if (MODE == kGrad && moving && r * r < eps * eps) {
            // J = [m ; P_s x m]: m = n turned towards the camera, P_s = d_s ray
            const float sg = nr < 0.0f ? 1.0f : -1.0f;
            const float mx = sg * nx, my = sg * ny, mz = sg * nz;
            const float Px = d_s * rx, Py = d_s * ry, Pz = d_s;
            float J[6];
            J[0] = mx; J[1] = my; J[2] = mz;
            J[3] = Py * mz - Pz * my;
            J[4] = Pz * mx - Px * mz;
            J[5] = Px * my - Py * mx;
            acc.n_active += 1;
#pragma unroll
            for (int i = 0; i < 6; ++i) acc.jtr[i] = fmaf(r, J[i], acc.jtr[i]);
            int k = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = i; j < 6; ++j) { acc.jtj[k] = fmaf(J[i], J[j], acc.jtj[k]); ++k; }
        }
    }
    if (MODE == kRender) return;

    // ---------------------------------------------------------------- reduction (fixed order)
    constexpr int NF = MODE == kIcp ? 40 : (MODE == kGrad ? 39 : 12);
    float v[NF];
    v[0] = __int_as_float(acc.e_table);
#pragma unroll
    for (int k = 0; k < 9; ++k) v[1 + k] = __int_as_float(acc.cnt[k]);
    v[10] = __int_as_float(acc.n_active);
    v[11] = acc.e_soft;
    if (MODE == kGrad || MODE == kIcp) {
#pragma unroll
        for (int k = 0; k < 6; ++k) v[12 + k] = acc.jtr[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) v[18 + k] = acc.jtj[k];
    }
    if (MODE == kIcp) v[39] = acc.sse;
    int col0 = 0, col1 = 0;
    if (MODE != kIcp && color) {
        col0 = acc.col[0]; col1 = acc.col[1];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            col0 += __shfl_xor(col0, off);
            col1 += __shfl_xor(col1, off);
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (f <= 10) {
            int x = __float_as_int(v[f]);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            v[f] = __int_as_float(x);
        } else {
            float x = v[f];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            v[f] = x;
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) red[wave][f] = v[f];
        if (MODE != kIcp) {
            red[wave][39] = __int_as_float(col0);
            red[wave][40] = __int_as_float(col1);
        }
    }
    __syncthreads();
    if (tid < kRecFields) {
        float* rec = a.rec + it.rec * kRecFields;
        if (MODE != kIcp && tid >= 39) {       // color counts (integers)
            int x = 0;
#pragma unroll
            for (int w = 0; w < kWG / 64; ++w) x += __float_as_int(red[w][tid]);
            rec[tid] = __int_as_float(x);
        } else if (tid >= NF) {
            rec[tid] = 0.0f;
        } else if (tid <= 10) {
            int x = 0;
#pragma unroll
            for (int w = 0; w < kWG / 64; ++w) x += __float_as_int(red[w][tid]);
            rec[tid] = __int_as_float(x);
        } else {
            float x = 0.0f;
#pragma unroll
            for (int w = 0; w < kWG / 64; ++w) x += red[w][tid];
            rec[tid] = x;
        }
    }
}

// Either one workgroup per item in the XCD-aware order, or, with an item
// order, persistent workgroups that take the next item of the order (longest
// first) from a global counter until it runs past the end; every workgroup
// reaches that exit.
template <int TW, int TH, int MODE, bool OVF>
__global__ void __launch_bounds__(kWG, 4) k_raster(BatchDesc bd, RasterArgs a) {
    __shared__ uint64_t keys[TW * TH];
    __shared__ Queues q;
    __shared__ float red[kWG / 64][kRecFields];
    if (!a.order) {
        ItemInfo it;
        if (!decode_item(bd, it)) return;
        tile_pass<TW, TH, MODE, OVF>(bd, a, it, keys, q, red);
        return;
    }
    __shared__ int slot;
    for (;;) {
        __syncthreads();                       // the previous item's shared data is no longer read
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int k = slot;
        if (k >= a.n_order) return;
        ItemInfo it;
        decode_rec(bd, a.order[k], it);
        tile_pass<TW, TH, MODE, OVF>(bd, a, it, keys, q, red);
    }
}

// ------------------------------------------------------------------ cluster cull

__device__ __forceinline__ void proj_acc(double fx, double fy, double cx, double cy, double x, double y,
                                         double z, double& umin, double& umax, double& vmin, double& vmax) {
    const double u = fx * x / z + cx, v = fy * y / z + cy;
    umin = fmin(umin, u); umax = fmax(umax, u);
    vmin = fmin(vmin, v); vmax = fmax(vmax, v);
}

// One thread per (cluster, pose): frustum test of the cluster's world AABB
// and the range of screen tiles its projection can touch.  Conservative:
// the box is clipped against a near plane slightly in front of z_near and the
// screen rectangle is widened by 2 px.
__global__ void __launch_bounds__(kWG) k_cull(BatchDesc bd, const ClusterBounds* __restrict__ cb,
                                              int32_t n_clusters, const double* __restrict__ T_wc,
                                              uint2* __restrict__ vis, float* __restrict__ vis_z,
                                              int32_t* __restrict__ vis_count, int32_t* __restrict__ vis_tris) {
    const int c = blockIdx.x * kWG + threadIdx.x;
    const int pose = blockIdx.y;
    int s = 0;
    while (s + 1 < bd.n_scans && pose >= bd.s[s + 1].pose_off) ++s;
    const ScanDesc& sd = bd.s[s];
    bool visible = false;
    uint32_t rect = 0;
    int ntri = 0;
    float zkey = 0.0f;                         // farthest box corner depth (ordering key only)
    if (c < n_clusters) {
        const ClusterBounds b = cb[c];
        ntri = b.n_tris;
        const double* T = T_wc + 12 * (int64_t)pose;
        const double zn = (double)sd.z_near * (1.0 - 1e-5), zf = (double)sd.z_far * (1.0 + 1e-5);
        double X[8], Y[8], Z[8];
        int nfront = 0, nfar = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double px = (k & 1) ? b.hi[0] : b.lo[0];
            const double py = (k & 2) ? b.hi[1] : b.lo[1];
            const double pz = (k & 4) ? b.hi[2] : b.lo[2];
            const double d0 = px - T[3], d1 = py - T[7], d2 = pz - T[11];
            X[k] = T[0] * d0 + T[4] * d1 + T[8] * d2;
            Y[k] = T[1] * d0 + T[5] * d1 + T[9] * d2;
            Z[k] = T[2] * d0 + T[6] * d1 + T[10] * d2;
            nfront += Z[k] >= zn;
            nfar += Z[k] > zf;
        }
        zkey = (float)fmax(fmax(fmax(fmax(Z[0], Z[1]), fmax(Z[2], Z[3])), fmax(fmax(Z[4], Z[5]), fmax(Z[6], Z[7]))), zn);
        const double fx = sd.fx, fy = sd.fy, cx = sd.cx, cy = sd.cy;
        double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        if (nfront > 0 && nfar < 8 && b.n_tris > 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (Z[k] >= zn) proj_acc(fx, fy, cx, cy, X[k], Y[k], Z[k], umin, umax, vmin, vmax);
            if (nfront < 8) {
                // box edges crossing the near plane: corners differing in one bit
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int bit = 1; bit < 8; bit <<= 1) {
                        const int j = k | bit;
                        if (j == k) continue;
                        if ((Z[k] >= zn) != (Z[j] >= zn)) {
                            const double t = (zn - Z[k]) / (Z[j] - Z[k]);
                            proj_acc(fx, fy, cx, cy, X[k] + t * (X[j] - X[k]), Y[k] + t * (Y[j] - Y[k]), zn,
                                     umin, umax, vmin, vmax);
                        }
                    }
            }
            umin -= 2.0; vmin -= 2.0; umax += 2.0; vmax += 2.0;
            const double W1 = sd.width - 1, H1 = sd.height - 1;
            if (umin <= umax && vmin <= vmax && umax >= 0.0 && vmax >= 0.0 && umin <= W1 && vmin <= H1) {
                const int tw = bd.tile_w, th = bd.tile_h;
                const int x0 = (int)fmax(umin, 0.0), x1 = (int)fmin(umax, W1);
                const int y0 = (int)fmax(vmin, 0.0), y1 = (int)fmin(vmax, H1);
                rect = (uint32_t)(x0 / tw) | ((uint32_t)(x1 / tw) << 8) | ((uint32_t)(y0 / th) << 16) |
                       ((uint32_t)(y1 / th) << 24);
                visible = true;
            }
        }
    }
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(visible);
    if (!m) return;
    int ntv = visible ? ntri : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ntv += __shfl_xor(ntv, off);
    int base = 0;
    if (lane == 0) {
        base = atomicAdd(vis_count + pose, __popcll(m));
        atomicAdd(vis_tris + pose, ntv);
    }
    base = __shfl(base, 0);
    if (visible) {
        const int64_t slot = (int64_t)pose * n_clusters + base + __popcll(m & ((1ull << lane) - 1ull));
        vis[slot] = make_uint2((uint32_t)c, rect);
        vis_z[slot] = zkey;
    }
}

// Near-to-far order of each pose's visible clusters: a counting sort on the
// logarithm of the farthest box corner depth.  The tile bins are filled in
// this order, so the rasterizer meets near surfaces first and its depth
// snapshot rejects more of what lies behind them; keying on the far corner
// puts compact surface clusters before clusters that also hold long
// free-unknown quads (whose bounds reach far behind their surfaces).  Only
// speed depends on the order; a pose with more visible clusters than one
// workgroup stages keeps the order of the cull.
constexpr int kVisSortWG = 1024;
constexpr int kVisSortMax = 7680;              // 60 KB of LDS staging
constexpr int kVisBuckets = 256;

__global__ void __launch_bounds__(kVisSortWG) k_vis_sort(BatchDesc bd, int32_t n_clusters,
                                                         const int32_t* __restrict__ vis_count,
                                                         const float* __restrict__ vis_z, uint2* __restrict__ vis) {
    __shared__ uint2 stage[kVisSortMax];
    __shared__ int cur[kVisBuckets];
    const int pose = blockIdx.x;
    const int n = vis_count[pose];
    if (n <= 1 || n > kVisSortMax) return;
    const ScanDesc& sd = bd.s[pose_scan(bd, pose)];
    const float lz0 = log2f(sd.z_near);
    const float scale = (float)kVisBuckets / fmaxf(log2f(sd.z_far) - lz0, 1e-3f);
    for (int i = threadIdx.x; i < kVisBuckets; i += kVisSortWG) cur[i] = 0;
    __syncthreads();
    uint2* v = vis + (int64_t)pose * n_clusters;
    const float* z = vis_z + (int64_t)pose * n_clusters;
    constexpr int kPer = (kVisSortMax + kVisSortWG - 1) / kVisSortWG;
    uint2 e[kPer];
    int b[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * kVisSortWG;
        b[k] = 0;
        if (i < n) {
            e[k] = v[i];
            const float f = (log2f(z[i]) - lz0) * scale;
            b[k] = f >= (float)(kVisBuckets - 1) ? kVisBuckets - 1 : (f > 0.0f ? (int)f : 0);
            atomicAdd(&cur[b[k]], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {                    // exclusive prefix over the buckets, 4 per lane
        const int l = threadIdx.x;
        const int c0 = cur[4 * l], c1 = cur[4 * l + 1], c2 = cur[4 * l + 2], c3 = cur[4 * l + 3];
        const int tot = c0 + c1 + c2 + c3;
        int inc = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(inc, off);
            if (l >= off) inc += y;
        }
        const int ex = inc - tot;
        cur[4 * l] = ex;
        cur[4 * l + 1] = ex + c0;
        cur[4 * l + 2] = ex + c0 + c1;
        cur[4 * l + 3] = ex + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * kVisSortWG;
        if (i < n) stage[atomicAdd(&cur[b[k]], 1)] = e[k];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kVisSortWG) v[i] = stage[i];
}

// ------------------------------------------------------------------ per-pose reduction

// One workgroup per pose: 8 lanes per field sum interleaved tiles (FP64,
// integers exactly), then the 8 partial sums are added in lane order, so the
// result does not depend on scheduling.
constexpr int kRedSplit = 8;

__global__ void __launch_bounds__(kRecFields * kRedSplit) k_reduce(BatchDesc bd, const float* __restrict__ rec,
                                                                   const int32_t* __restrict__ vis_tris, float eps,
                                                                   int mode, double* __restrict__ out) {
    __shared__ double part[kRedSplit][kRecFields];
    __shared__ double val[kRecFields];
    const int pose = blockIdx.x;
    int s = 0;
    while (s + 1 < bd.n_scans && pose >= bd.s[s + 1].pose_off) ++s;
    const ScanDesc& sd = bd.s[s];
    const int ntile = sd.tiles_x * sd.tiles_y;
    const float* r = rec + (sd.rec_off + (int64_t)(pose - sd.pose_off) * ntile) * kRecFields;
    const int f = threadIdx.x % kRecFields, j = threadIdx.x / kRecFields;
    if (f <= 10 || (mode != kIcp && f >= 39)) {      // integer fields (counts)
        int64_t acc = 0;
        for (int t = j; t < ntile; t += kRedSplit) acc += __float_as_int(r[(int64_t)t * kRecFields + f]);
        part[j][f] = (double)acc;
    } else {
        double acc = 0.0;
        for (int t = j; t < ntile; t += kRedSplit) acc += (double)r[(int64_t)t * kRecFields + f];
        part[j][f] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kRecFields) {
        double x = 0.0;
        for (int k = 0; k < kRedSplit; ++k) x += part[k][threadIdx.x];
        val[threadIdx.x] = x;
    }
    __syncthreads();
    double* o = out + (int64_t)pose * RM_OUT_STRIDE;
    const int g = threadIdx.x;
    const bool grad = mode == kGrad;
    if (mode == kIcp && g < RM_OUT_STRIDE) {
        // ICP records: cost, sum of squared residuals, counts, blocks
        double x = 0.0;
        if (g == RM_OUT_ICP_COST) x = val[11];
        else if (g == RM_OUT_ICP_SSE) x = val[39];
        else if (g == RM_OUT_ICP_N_SCAN) x = val[1];
        else if (g == RM_OUT_ICP_N_MODEL) x = val[2];
        else if (g == RM_OUT_N_ACTIVE) x = val[10];
        else if (g >= RM_OUT_GRAD && g < RM_OUT_GRAD + 6) x = 2.0 * val[12 + g - RM_OUT_GRAD];
        else if (g >= RM_OUT_JTR && g < RM_OUT_JTR + 6) x = val[12 + g - RM_OUT_JTR];
        else if (g >= RM_OUT_JTJ && g < RM_OUT_JTJ + 21) x = val[18 + g - RM_OUT_JTJ];
        else if (g == RM_OUT_N_VISIBLE) x = (double)vis_tris[pose];
        o[g] = x;
    } else if (g < RM_OUT_STRIDE) {
        double x = 0.0;
        if (g == RM_OUT_E_TABLE) x = val[0];
        else if (g == RM_OUT_E_SOFT) x = val[11];
        else if (g >= RM_OUT_COUNTS && g < RM_OUT_COUNTS + 9) x = val[1 + g - RM_OUT_COUNTS];
        else if (g == RM_OUT_N_ACTIVE) x = grad ? val[10] : 0.0;
        else if (g >= RM_OUT_GRAD && g < RM_OUT_GRAD + 6)
            x = grad ? (4.0 / ((double)eps * (double)eps)) * val[12 + g - RM_OUT_GRAD] : 0.0;
        else if (g >= RM_OUT_JTR && g < RM_OUT_JTR + 6) x = grad ? val[12 + g - RM_OUT_JTR] : 0.0;
        else if (g >= RM_OUT_JTJ && g < RM_OUT_JTJ + 21) x = grad ? val[18 + g - RM_OUT_JTJ] : 0.0;
        else if (g == RM_OUT_N_VISIBLE) x = (double)vis_tris[pose];
        else if (g == RM_OUT_COLOR_REWARD) x = val[39];
        else if (g == RM_OUT_COLOR_PENALTY) x = val[40];
        o[g] = x;
    }
}

template <int TW, int TH, bool SPILL>
hipError_t launch_bin_t(hipStream_t st, const BatchDesc& bd, const RasterArgs& a) {
    const dim3 grid((unsigned)std::min(a.n_clusters > 0 ? a.n_clusters : 1, 256), (unsigned)bd.n_poses);
    int32_t n = 1;
    for (int s = 0; s < bd.n_scans; ++s) n = std::max(n, bd.s[s].tiles_x * bd.s[s].tiles_y);
    n = std::min(n, kBinTable);
    static_assert(kMaxTileGrid <= kBinTable, "a row of tiles must fit one binning band");
    const size_t lds = (SPILL ? 5 : 3) * sizeof(uint32_t) * (size_t)n;
    hipLaunchKernelGGL((k_bin<TW, TH, SPILL>), grid, dim3(kWG), lds, st, bd, a, n);
    return hipGetLastError();
}

template <bool SPILL>
hipError_t launch_bin_shape(hipStream_t st, const BatchDesc& bd, const RasterArgs& a) {
    if (bd.tile_w == 8 && bd.tile_h == 8) return launch_bin_t<8, 8, SPILL>(st, bd, a);
    if (bd.tile_w == 16 && bd.tile_h == 16) return launch_bin_t<16, 16, SPILL>(st, bd, a);
    if (bd.tile_w == 64 && bd.tile_h == 32) return launch_bin_t<64, 32, SPILL>(st, bd, a);
    return launch_bin_t<32, 32, SPILL>(st, bd, a);
}

// ------------------------------------------------------------------ longest-first order

constexpr int kOrderBuckets = 32;

// bucket 0 holds the costliest records: 31 - floor(log2(fill + 1))
__device__ __forceinline__ int order_bucket(const int32_t* bs, const int32_t* bb, int64_t r) {
    const uint32_t c = (uint32_t)bs[r] + (uint32_t)bb[r] + 1u;
    return __clz(c);
}

__global__ void __launch_bounds__(kWG) k_order_count(const int32_t* __restrict__ bs, const int32_t* __restrict__ bb,
                                                     int64_t n, int32_t* __restrict__ hist) {
    __shared__ int h[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (r < n) atomicAdd(&h[order_bucket(bs, bb, r)], 1);
    __syncthreads();
    if (threadIdx.x < kOrderBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// hist[0..31] counts -> hist[32..63] running cursors (exclusive prefix)
__global__ void k_order_offsets(int32_t* hist) {
    if (threadIdx.x != 0) return;
    int acc = 0;
    for (int k = 0; k < kOrderBuckets; ++k) {
        hist[kOrderBuckets + k] = acc;
        acc += hist[k];
    }
}

// Records are visited in item order (per scan tile-major, poses of a tile
// adjacent), so that each workgroup's run of a bucket keeps neighbouring poses
// of the same tiles, which read the same triangles, together.
__global__ void __launch_bounds__(kWG) k_order_scatter(BatchDesc bd, const int32_t* __restrict__ bs,
                                                       const int32_t* __restrict__ bb, int64_t n,
                                                       int32_t* __restrict__ hist, int32_t* __restrict__ order) {
    __shared__ int h[kOrderBuckets], base[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t item = (int64_t)blockIdx.x * kWG + threadIdx.x;
    int64_t r = n;
    if (item < n) {
        int sc = 0;
        while (sc + 1 < bd.n_scans && item >= bd.s[sc + 1].item_off) ++sc;
        const ScanDesc& sd = bd.s[sc];
        const int64_t local = item - sd.item_off;
        r = sd.rec_off + (local % sd.n_poses) * (int64_t)(sd.tiles_x * sd.tiles_y) + local / sd.n_poses;
    }
    const int b = r < n ? order_bucket(bs, bb, r) : 0;
    if (r < n) atomicAdd(&h[b], 1);
    __syncthreads();
    if (threadIdx.x < kOrderBuckets) {
        const int c = h[threadIdx.x];
        base[threadIdx.x] = c ? atomicAdd(&hist[kOrderBuckets + threadIdx.x], c) : 0;
        h[threadIdx.x] = 0;
    }
    __syncthreads();
    if (r < n) order[base[b] + atomicAdd(&h[b], 1)] = (int32_t)r;
}

template <int TW, int TH>
hipError_t launch_raster_t(hipStream_t st, const BatchDesc& bd, const RasterArgs& a, int mode) {
    const int64_t chunk = (bd.n_items + 7) / 8;
    const dim3 grid(a.order ? (unsigned)std::min<int64_t>(persistent_grid(TW, TH, mode), a.n_order)
                            : (unsigned)(chunk * 8));
    if (a.spill) {
        if (mode == kRender) hipLaunchKernelGGL((k_raster<TW, TH, kRender, true>), grid, dim3(kWG), 0, st, bd, a);
        else if (mode == kCost) hipLaunchKernelGGL((k_raster<TW, TH, kCost, true>), grid, dim3(kWG), 0, st, bd, a);
        else if (mode == kIcp) hipLaunchKernelGGL((k_raster<TW, TH, kIcp, true>), grid, dim3(kWG), 0, st, bd, a);
        else hipLaunchKernelGGL((k_raster<TW, TH, kGrad, true>), grid, dim3(kWG), 0, st, bd, a);
    } else {
        if (mode == kRender) hipLaunchKernelGGL((k_raster<TW, TH, kRender, false>), grid, dim3(kWG), 0, st, bd, a);
        else if (mode == kCost) hipLaunchKernelGGL((k_raster<TW, TH, kCost, false>), grid, dim3(kWG), 0, st, bd, a);
        else if (mode == kIcp) hipLaunchKernelGGL((k_raster<TW, TH, kIcp, false>), grid, dim3(kWG), 0, st, bd, a);
        else hipLaunchKernelGGL((k_raster<TW, TH, kGrad, false>), grid, dim3(kWG), 0, st, bd, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cull(hipStream_t st, const BatchDesc& bd, const ClusterBounds* cb, int32_t n_clusters,
                       const double* T_wc, uint2* vis, float* vis_z, int32_t* vis_count, int32_t* vis_tris) {
    if (n_clusters == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_clusters + kWG - 1) / kWG), (unsigned)bd.n_poses);
    hipLaunchKernelGGL(k_cull, grid, dim3(kWG), 0, st, bd, cb, n_clusters, T_wc, vis, vis_z, vis_count, vis_tris);
    return hipGetLastError();
}

hipError_t launch_vis_sort(hipStream_t st, const BatchDesc& bd, int32_t n_clusters, const int32_t* vis_count,
                           const float* vis_z, uint2* vis) {
    if (n_clusters <= 1 || bd.n_poses == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vis_sort, dim3((unsigned)bd.n_poses), dim3(kVisSortWG), 0, st, bd, n_clusters, vis_count,
                       vis_z, vis);
    return hipGetLastError();
}

hipError_t launch_bin(hipStream_t st, const BatchDesc& bd, const RasterArgs& a) {
    if (bd.n_items == 0 || a.n_clusters == 0) return hipSuccess;
    return a.spill_top ? launch_bin_shape<true>(st, bd, a) : launch_bin_shape<false>(st, bd, a);
}

hipError_t launch_overflow(hipStream_t st, const RasterArgs& a, int64_t n_records) {
    if (n_records <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_region_alloc, dim3((unsigned)((n_records + kWG - 1) / kWG)), dim3(kWG), 0, st, a,
                       n_records);
    if (a.spill_cap > 0 && a.pool_cap > 0) {
        // enough workgroups to fill the device; each strides over its list
        hipLaunchKernelGGL(k_region_fill, dim3(4096), dim3(kWG), 0, st, a);
        const int64_t len = a.spill_cap / kSpillLists;
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((len + kWG - 1) / kWG, 128));
        hipLaunchKernelGGL(k_spill_scatter, dim3(g, kSpillLists), dim3(kWG), 0, st, a, n_records);
    }
    return hipGetLastError();
}

hipError_t launch_order(hipStream_t st, const BatchDesc& bd, const int32_t* bin_small, const int32_t* bin_big,
                        int64_t n_records, int32_t* hist, int32_t* order) {
    if (n_records <= 0) return hipSuccess;
    const unsigned g = (unsigned)((n_records + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_order_count, dim3(g), dim3(kWG), 0, st, bin_small, bin_big, n_records, hist);
    hipLaunchKernelGGL(k_order_offsets, dim3(1), dim3(64), 0, st, hist);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(kWG), 0, st, bd, bin_small, bin_big, n_records, hist, order);
    return hipGetLastError();
}

namespace {
template <int TW, int TH, int MODE>
int resident_blocks() {
    static int cached = 0;
    if (!cached) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raster<TW, TH, MODE, false>, kWG, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 1024;
        }
        cached = std::max(1, per_cu) * std::max(1, cus);
    }
    return cached;
}
template <int TW, int TH>
int resident_t(int mode) {
    return mode == kRender ? resident_blocks<TW, TH, kRender>()
                           : (mode == kCost ? resident_blocks<TW, TH, kCost>()
                                            : (mode == kIcp ? resident_blocks<TW, TH, kIcp>()
                                                            : resident_blocks<TW, TH, kGrad>()));
}
}  // namespace

int persistent_grid(int tile_w, int tile_h, int mode) {
    if (tile_w == 8 && tile_h == 8) return resident_t<8, 8>(mode);
    if (tile_w == 16 && tile_h == 16) return resident_t<16, 16>(mode);
    if (tile_w == 64 && tile_h == 32) return resident_t<64, 32>(mode);
    return resident_t<32, 32>(mode);
}

hipError_t launch_raster(hipStream_t st, const BatchDesc& bd, const RasterArgs& a, int mode) {
    if (bd.n_items == 0) return hipSuccess;
    if (bd.tile_w == 8 && bd.tile_h == 8) return launch_raster_t<8, 8>(st, bd, a, mode);
    if (bd.tile_w == 16 && bd.tile_h == 16) return launch_raster_t<16, 16>(st, bd, a, mode);
    if (bd.tile_w == 64 && bd.tile_h == 32) return launch_raster_t<64, 32>(st, bd, a, mode);
    return launch_raster_t<32, 32>(st, bd, a, mode);
}

hipError_t launch_reduce(hipStream_t st, const BatchDesc& bd, const float* rec, const int32_t* vis_tris,
                         float eps, int mode, double* out) {
    if (bd.n_poses == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)bd.n_poses), dim3(kRecFields * kRedSplit), 0, st, bd, rec, vis_tris,
                       eps, mode, out);
    return hipGetLastError();
}

}  // namespace rm
