/*
 * rendermap.h -- C ABI of the MI355X (gfx950) pose-scoring library for
 * RenderMap (Ryde & Ding, "RenderMap: Exploiting the Link Between Perception
 * and Rendering for Dense Mapping", arXiv 1702.06813).
 *
 * The library evaluates E(X) = C(R(T(X)), Z_s) of Eq. (1) for many candidate
 * poses X at once: it rasterizes the interface mesh (Sec. IV-A) into a
 * z-buffer from each pose, compares every pixel with the scan image through
 * Table I (Sec. IV-B), and reduces to the per-pose cost.  It also returns a
 * continuous surrogate cost E_soft with its se(3) gradient and Gauss-Newton
 * blocks, and runs the pose update of an optimizer step on the device.
 *
 * General rules (every entry point):
 *   - Return RM_OK (0) or a negative rm_status; on error rm_last_error(ctx)
 *     describes it.  No C++ exception crosses this boundary.
 *   - Pointers documented "device" must point to memory on the context's
 *     device; "host" pointers are read before the call returns.  The caller
 *     owns every buffer; the library owns only the scratch inside rm_ctx and
 *     keeps no caller pointer after a call returns.
 *   - Work is enqueued asynchronously on the context stream (rm_ctx_set_stream)
 *     and no call synchronizes, except rm_mesh_from_range (it returns counts)
 *     and the first call of a new launch shape (scan sizes, pose count,
 *     triangle count, tile) outside graph capture, which waits once for the
 *     binning pass to size its screen-tile bins; capture a shape only after
 *     one uncaptured call of it.
 *   - Arguments are validated on the host before anything is launched;
 *     invalid arguments return RM_ERR_INVALID_ARG and launch nothing.
 *   - Device arrays are dense and row-major.  Images are [H][W] with pixel
 *     (u, v) at index v * W + u, its centre at continuous coordinates (u, v).
 *   - Camera axes: x right, y down, z forward.  Depth is the perpendicular
 *     distance from the camera plane (camera-frame z), as the paper's z-buffer
 *     holds (Sec. V).
 *   - A pose T_wc is 12 doubles, the row-major 3x4 matrix [R | t] mapping
 *     camera coordinates to world (map) coordinates: the sensor pose X of
 *     Eq. (1) in the map frame.
 */
#ifndef RENDERMAP_H
#define RENDERMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RM_ABI_VERSION 2

typedef enum {
    RM_OK = 0,
    RM_ERR_INVALID_ARG = -1,   /* bad pointer, size, count or parameter */
    RM_ERR_OOM = -2,           /* device scratch could not be allocated */
    RM_ERR_DEVICE = -3,        /* a HIP runtime call failed */
    RM_ERR_CAPACITY = -4,      /* output capacity too small, or scratch must grow during graph capture */
    RM_ERR_UNSUPPORTED = -5    /* valid request the library does not support */
} rm_status;

/* Interface classes of Sec. IV-A (free-occupied, free-unknown,
 * unknown-occupied) and "no surface / NaN". */
typedef enum { RM_FO = 0, RM_FU = 1, RM_UO = 2, RM_NONE = 3 } rm_class;

typedef struct rm_ctx rm_ctx;

/* Pinhole camera.  Pixel centres at integer (u, v); u = fx x/z + cx.
 * Surfaces nearer than z_near are clipped, farther than z_far ignored. */
typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;     /* 1 .. 4096 each (a tile shape with more than
                                  256 tiles per image row or column is
                                  RM_ERR_UNSUPPORTED: 8x8 tiles above 2048) */
    float z_near, z_far;       /* 0 < z_near < z_far */
} rm_camera;

/* Interface mesh (Sec. IV-A): world-frame vertices and triangles, each with
 * its interface class.  Triangles are grouped into clusters of
 * RM_CLUSTER_TRIS consecutive triangles for culling; meshes whose consecutive
 * triangles are spatial neighbours (as rm_mesh_from_range emits them) cull best. */
typedef struct {
    const float* xyz;          /* device [n_vertices][3] f32 */
    int64_t n_vertices;
    const int32_t* tri;        /* device [n_tris][3] i32 vertex indices */
    const uint8_t* cls;        /* device [n_tris] u8, rm_class */
    int64_t n_tris;            /* 0 .. 2^31 - 1 */
    const void* clusters;      /* device, nullable: prepared buffer from rm_mesh_clusters
                                  (cluster bounds, normals); NULL recomputes it every call */
    const float* color;        /* device [n_tris] f32, nullable: intensity of each triangle,
                                  the map side of the color term (NaN = none) */
} rm_mesh;

#define RM_CLUSTER_TRIS 256

/* Scan image Z_s (Sec. IV-B): per pixel depth d_s and class c_s, as produced
 * by rm_scan_image. */
typedef struct {
    const float* depth;        /* device [H][W] f32 d_s, NaN = dead pixel */
    const uint8_t* cls;        /* device [H][W] u8 c_s (RM_FO, RM_FU or RM_NONE) */
    const uint8_t* mask;       /* device [H][W] u8, nullable: pixels with 0 are left out of every sum */
    rm_camera cam;             /* H = cam.height, W = cam.width */
    const float* color;        /* device [H][W] f32, nullable: intensity of each pixel, the
                                  scan side of the color term (NaN = none) */
} rm_scan;

/* Cost parameters.  eps is the inlier/outlier threshold of Table I
 * (0.1 m in the paper); flags must be 0; color_tol (finite, >= 0) is the
 * intensity difference up to which a corresponding pixel's colors agree
 * (color term, see RM_OUT_COLOR_REWARD). */
typedef struct {
    float eps;
    int32_t flags;
    float color_tol;
} rm_cost_params;

/* Per-pose result record: RM_OUT_STRIDE doubles per pose.
 *   E_TABLE    E(X) = sum over pixels of the Table I value (+1/-1/0); exact
 *   E_SOFT     sum over pixels of rho_p = 2 min(r_p^2/eps^2, 1) - 1 on scored
 *              cells, 0 elsewhere, with r_p = e_p (map FO / scan FO),
 *              min(e_p, 0) (FO / FU), max(e_p, 0) (FU / FO); e_p = dz |n . r|
 *              is the signed distance of the scan point d(p_s) r from the
 *              plane of the triangle the pixel sees (positive on the camera
 *              side), dz = d(p_r) - d(p_s) the Table I depth difference
 *   COUNTS     9 pixel counts: FO/FO reward, FO/FO penalty, FO/FU reward,
 *              FO/FU penalty, FU/FO reward, FU/FO penalty, ignored because the
 *              scan pixel is NaN, ignored because the map pixel is NaN or UO,
 *              ignored FU/FU
 *   N_ACTIVE   pixels whose residual moves with the pose and |r_p| < eps
 *   GRAD       d E_soft / d delta for T_wc exp(delta), delta = (v, w)
 *   JTR        b = sum over active pixels of r_p J_p
 *   JTJ        H = sum over active pixels of J_p^T J_p, upper triangle
 *              row-major (21 values)
 *   N_VISIBLE  triangles in clusters that survived frustum culling
 *   COLOR_REWARD, COLOR_PENALTY  the color term (Sec. IV: color can enter a
 *              render-based cost; Sec. IV-C: costs and rewards from the colors
 *              of corresponding pixels): over pixels in the FO/FO reward cell
 *              of Table I whose scan color and whose triangle's color (flat
 *              over the triangle) are both finite, the number with
 *              |c_map - c_scan| <= color_tol (float32) and the number above
 *              it; zero unless mesh->color and the scan's color are given
 * GRAD/JTR/JTJ/N_ACTIVE are written by rm_align_cost_grad only (zero from
 * rm_align_cost).  J_p = [m ; P_s x m] is the derivative of e_p under
 * T_wc exp(delta) with the winning triangle held fixed: n is that triangle's
 * camera-frame unit normal, m = n turned towards the camera (m . r < 0),
 * r = ((u - cx)/fx, (v - cy)/fy, 1), P_s = d(p_s) r. */
enum {
    RM_OUT_E_TABLE = 0,
    RM_OUT_E_SOFT = 1,
    RM_OUT_COUNTS = 2,
    RM_OUT_N_ACTIVE = 11,
    RM_OUT_GRAD = 12,
    RM_OUT_JTR = 18,
    RM_OUT_JTJ = 24,
    RM_OUT_N_VISIBLE = 45,
    RM_OUT_COLOR_REWARD = 46,
    RM_OUT_COLOR_PENALTY = 47,
    RM_OUT_STRIDE = 48
};

/* Records of rm_icp_cost_grad use the same stride; its fields are
 *   ICP_COST     C = sum over associated pixels of |Z_M - Z_1| (Sec. V, step 5)
 *   ICP_SSE      sum over associated pixels of e_p^2
 *   ICP_N_SCAN   scan pixels with a return (c_s = RM_FO)
 *   ICP_N_MODEL  of those, pixels that see a map RM_FO triangle whose three
 *                vertex normals are defined
 *   N_ACTIVE     of those, associated pixels: |Z_M - Z_1| < tol
 *   GRAD         d ICP_SSE / d delta = 2 sum e_p J_p
 *   JTR, JTJ     b = sum e_p J_p, H = sum J_p^T J_p (upper triangle)
 *   N_VISIBLE    as above
 * with e_p = n . (P_1 - P_M) = (Z_1 - Z_M)(n . r), J_p = [n ; P_1 x n]: n is
 * the normalized sum of the winning triangle's vertex normals in the camera
 * frame, turned towards the camera; P_1 = Z_1 r and P_M = Z_M r are the scan
 * and model points of the pixel; J_p is the derivative under T_wc exp(delta)
 * with the correspondence held, as point-to-plane ICP linearizes.  The other
 * fields are zero. */
enum {
    RM_OUT_ICP_COST = 0,
    RM_OUT_ICP_SSE = 1,
    RM_OUT_ICP_N_SCAN = 2,
    RM_OUT_ICP_N_MODEL = 3
};

/* Maximum number of scans per rm_align_cost / rm_align_cost_grad call. */
#define RM_MAX_SCANS 32

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`, using the null stream until
 * rm_ctx_set_stream.  *out receives the handle. */
int rm_ctx_create(int32_t device, rm_ctx** out);
/* Frees the context and its scratch.  NULL is accepted. */
int rm_ctx_destroy(rm_ctx* ctx);
/* Stream (a hipStream_t, or NULL for the null stream) on which later calls
 * enqueue their work.  Must belong to the context's device. */
int rm_ctx_set_stream(rm_ctx* ctx, void* stream);
/* Message of the last failed call on this context ("" if none).  The string
 * stays valid until the next call on the same context; NULL ctx gives the
 * message of the last failed rm_ctx_create or NULL-context call. */
const char* rm_last_error(const rm_ctx* ctx);
/* Selects the screen-tile shape of the rasterizer: tile_w x tile_h one of
 * 8x8, 16x16, 32x32, 64x32; (0, 0) restores automatic choice (autotuned when
 * rm_autotune is on, 64x32 otherwise).  Results do not depend on it.  A
 * scoring call whose images need more than 256 tiles of the chosen shape per
 * row or column, or 2^31 or more (pose, tile) pairs, returns
 * RM_ERR_UNSUPPORTED. */
int rm_set_tile(rm_ctx* ctx, int32_t tile_w, int32_t tile_h);
/* Capacity of the per-(pose, screen tile) triangle bins, in entries: small
 * footprints fill a bin from its front, large ones (bounding box over 100
 * px) from its back, each class within its own part of the capacity (the
 * large part learned from the largest large fill, at most half, and at most
 * an eighth when the memory budget keeps the capacity below what both parts
 * want).  0 (the default) adapts it: the first call of a launch shape sizes
 * the bins from the binning pass and later calls grow them from earlier
 * calls' largest fills, as far as the bins of one call fit in a quarter of
 * the device's memory (every bin holds the capacity).  cap > 0 fixes it and
 * never grows it.  Entries past a bin's part spill to the overflow
 * (rm_set_bin_pool) when it has room for them, else the tile is rasterized
 * from every visible cluster of its pose (slower); results are the same
 * either way.  Each change makes the next call of every launch shape size
 * its bins again.  cap in 0 .. 2^24, else RM_ERR_INVALID_ARG. */
int rm_set_bin_cap(rm_ctx* ctx, int32_t cap);
/* Overflow of the tile bins, for calls whose fullest bins the memory budget
 * keeps beyond the capacity (many records, uneven fills).  The binning pass
 * appends the entries past a bin's parts to a spill list (12 bytes each:
 * triangle, record, slot); each bin that spilled then gets an overflow region
 * of exactly its fill (4 bytes an entry), laid out like a bin, which its kept
 * entries and its spilled ones are copied into, and the rasterizer reads it
 * there.  List and regions share the budget of a quarter of the device's
 * memory with the bins.
 *   -1  adaptive (default): overflow joins the calls once a bin has outgrown
 *       a capacity that could not grow; the first call of a launch shape
 *       sizes list and regions, later calls grow them from what earlier
 *       calls asked for
 *    0  none: bins that outgrow their parts take the every-cluster path
 *  > 0  a list and regions of exactly this many entries each, never
 *       resized; bins they cannot hold take the every-cluster path
 * The allocation-free call has no overflow.  Results do not depend on the
 * setting.  Each change makes the next call of every launch shape size its
 * bins again.  entries in -1 .. 2^40, else RM_ERR_INVALID_ARG. */
int rm_set_bin_pool(rm_ctx* ctx, int64_t entries);
/* Work scheduling of the rasterizer over (scan, pose, tile) items:
 *   0  automatic: currently 2, measured faster for single- and multi-scan
 *      batches alike
 *   1  one workgroup per item, items in an XCD-aware order (neighbouring
 *      poses of a tile on one XCD, sharing its L2)
 *   2  persistent: after binning, items are ordered longest first (counting
 *      sort by log2 of their bin fill) and as many workgroups as fit on the
 *      device take the next item from a queue until it is empty
 * Results do not depend on it (each item writes its own partial record).
 * Returns RM_ERR_INVALID_ARG for other values. */
int rm_set_schedule(rm_ctx* ctx, int32_t mode);
/* Turns the tile autotuner on or off.  When on, the first call for a new
 * launch shape (every scan's image size and pose count, the triangle count
 * and the kind of call) times the tile shapes 64x32, 32x32, 16x16 and 8x8 on
 * the call's own inputs, largest first, skipping shapes the batch cannot use
 * (see rm_set_tile) and stopping at the first shape more than 25% slower than
 * the best so far, and keeps the fastest for later calls of that shape.  With
 * the environment variable RM_LOG set, each choice is printed to stderr, and
 * so is the plan of each sizing pass of the first uncaptured call of every
 * launch shape (scans, poses, triangles and clusters, tile, tile records,
 * schedule, bin capacity and its large part with the largest fills,
 * overflow list and region entries with what the spilling bins asked for,
 * scratch bytes) with any growth of the bins or the overflow; with RM_LOG
 * set, that call reads the fills back even where capacity and overflow are
 * fixed. */
int rm_autotune(rm_ctx* ctx, int32_t enable);
/* Current tile choice for a single-scan shape (after autotuning), for
 * reporting: the explicit tile, else the tuned one, else 64x32. */
int rm_get_tile(rm_ctx* ctx, int32_t width, int32_t height, int32_t n_poses, int64_t n_tris,
                int32_t* tile_w, int32_t* tile_h);

/* Kernel timing for reports.  While enabled, every launch of the tile
 * rasterizer (the kernel that rasterizes, compares and reduces) is bracketed
 * by HIP events on the context stream, and so is every launch of the
 * binning kernel; launches recorded into a stream capture or made by
 * rm_align_cost_grad_noalloc are not timed.  rm_profile_read synchronizes
 * the context stream, returns the number of timed rasterizer launches and
 * their summed duration in milliseconds, and clears that record. */
int rm_profile(rm_ctx* ctx, int32_t enable);
int rm_profile_read(rm_ctx* ctx, int64_t* n_launches, double* total_ms);
/* As rm_profile_read, for the launches of the binning kernel (the pass that
 * sorts each pose's visible triangles into per-screen-tile bins before the
 * rasterizer); the two records are kept and cleared separately. */
int rm_profile_read_binning(rm_ctx* ctx, int64_t* n_launches, double* total_ms);

/* ---------------------------------------------------------------- graphs */

/* Begins stream capture on the context stream (hipStreamCaptureModeThreadLocal);
 * every call until rm_graph_end is recorded instead of run.  Scratch must
 * already be large enough: run each captured call once beforehand. */
int rm_graph_begin(rm_ctx* ctx);
/* Ends capture and instantiates the graph; *graph_exec receives a
 * hipGraphExec_t owned by the caller (free with rm_graph_destroy). */
int rm_graph_end(rm_ctx* ctx, void** graph_exec);
/* Launches an instantiated graph on the context stream. */
int rm_graph_launch(rm_ctx* ctx, void* graph_exec);
int rm_graph_destroy(void* graph_exec);

/* ---------------------------------------------------------------- scans and meshes */

/* Scan image Z_s of a range image (Sec. IV-A/IV-B).  Per pixel of `depth`
 * (device [H][W] f32, metres of z-depth):
 *   NaN, negative, or in (0, z_min)       -> dead:      d = NaN,   c = RM_NONE
 *   0, +inf, or > z_max (no return)       -> free to the sensor maximum:
 *                                                       d = z_max, c = RM_FU
 *   otherwise                             -> d = depth, c = RM_FO
 * d_out (device [H][W] f32) and c_out (device [H][W] u8) are written. */
int rm_scan_image(rm_ctx* ctx, const float* depth, int32_t height, int32_t width,
                  float z_min, float z_max, float* d_out, uint8_t* c_out);

/* Meshification of one range image (Sec. IV-A).  Grid nodes are the pixels
 * (j*stride, i*stride), i < ceil(H/stride), j < ceil(W/stride); a node is
 * classified as in rm_scan_image, back-projected at its depth (z_max for a
 * no-return) through `cam` and moved to the world by T_wc (host, 12 doubles),
 * in FP64, then rounded to f32.  With smooth_radius R > 0 the depth of a
 * valid node is the FP64 mean of the valid pixels of the (2R+1)^2 window
 * centred on it (clipped to the image, rows then columns in increasing
 * order) whose depth differs from the node pixel's by at most RM_SMOOTH_REL
 * of it: an edge-preserving box filter that reduces range noise before the
 * surfaces are built (the paper suggests blurring the depth images to lower
 * the noise of the cost, Sec. IV-C); R = 0 uses the node pixel alone.
 * Vertex i*gw + j belongs to node (i, j)
 * (gw = ceil(W/stride)); dead nodes get an unreferenced NaN vertex.  The quad
 * between nodes (i,j), (i,j+1), (i+1,j), (i+1,j+1) is dropped if a corner is
 * dead, is RM_FU if a corner is a no-return or one of its four sides is
 * longer than max_edge metres, RM_FO otherwise, and gives the triangles
 * (00, 01, 11) and (00, 11, 10).  Quads are emitted in 8x8 blocks (blocks
 * row-major, quads row-major inside a block).
 *   xyz_out  device [gh*gw][3] f32 (gh = ceil(H/stride))
 *   tri_out  device [cap_t][3] i32,  cls_out device [cap_t] u8
 *   n_v_out, n_t_out  host; receive gh*gw and the triangle count.
 * smooth_radius must lie in 0..RM_MAX_SMOOTH_RADIUS.
 * Synchronizes the context stream to read the count back.  If more than
 * cap_t triangles result, returns RM_ERR_CAPACITY (n_t_out holds the
 * needed count; the outputs are unspecified). */
#define RM_SMOOTH_REL 0.03
#define RM_MAX_SMOOTH_RADIUS 16
int rm_mesh_from_range(rm_ctx* ctx, const float* depth, rm_camera cam, const double* T_wc,
                       int32_t stride, int32_t smooth_radius, float z_min, float z_max, float max_edge,
                       float* xyz_out, int32_t* tri_out, uint8_t* cls_out, int64_t cap_t,
                       int64_t* n_v_out, int64_t* n_t_out);

/* Bytes of the prepared-mesh buffer for a mesh of n_tris triangles: one
 * 32-byte world AABB record per cluster of RM_CLUSTER_TRIS consecutive
 * triangles (padded to a multiple of 256 bytes), then the world-frame unit
 * normal of every triangle ([n_tris][3] f32, from the FP32 vertices in FP64). */
int64_t rm_mesh_clusters_size(int64_t n_tris);
/* Writes the prepared-mesh buffer of `mesh` into `out` (device,
 * rm_mesh_clusters_size bytes).  Point rm_mesh.clusters at it to skip the
 * per-call recomputation; recompute after changing the mesh. */
int rm_mesh_clusters(rm_ctx* ctx, const rm_mesh* mesh, void* out);

/* ---------------------------------------------------------------- z-buffer */

/* Renders R(T(X)) of Eq. (1) for B poses.  T_wc: device [B][12] f64.
 * Outputs (device, each nullable):
 *   depth_out [B][H][W] f32: depth of the nearest surface, NaN where none
 *   tri_out   [B][H][W] i32: its triangle id, -1 where none
 *   cls_out   [B][H][W] u8 : its rm_class, RM_NONE where none
 * Coverage follows the rasterization contract: float32 camera transform
 * R32 = fl32(R^T), d = fl32(Xw - t) (difference in FP64), Xc = R32 d with
 * fmaf in the order z-, y-, x-column; clip at z >= z_near interpolating from
 * the inside vertex; u = fmaf(fx Xc.x, 1/Xc.z, cx) (v alike); snap to
 * rint(256 u), rint(256 v); integer edge functions with the top-left rule
 * (y down).  The nearest surface is the minimum of (depth, triangle id). */
int rm_render_depth(rm_ctx* ctx, const rm_mesh* mesh, rm_camera cam, const double* T_wc,
                    int32_t n_poses, float* depth_out, int32_t* tri_out, uint8_t* cls_out);

/* ---------------------------------------------------------------- cost */

/* E(X) of Eq. (1) and Table I for every pose of S scans at once.
 * scans: host [S] (device pointers inside), 1 <= S <= RM_MAX_SCANS.
 * pose_off: host [S+1] non-decreasing offsets, pose_off[0] = 0; poses
 *   pose_off[s] .. pose_off[s+1]-1 are scored against scan s.
 * T_wc: device [P][12] f64, P = pose_off[S].
 * out: device [P][RM_OUT_STRIDE] f64, fully overwritten (see RM_OUT_*). */
int rm_align_cost(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t n_scans,
                  const int32_t* pose_off, const double* T_wc, rm_cost_params params,
                  double* out);
/* As rm_align_cost, also writing GRAD, JTR, JTJ and N_ACTIVE. */
int rm_align_cost_grad(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t n_scans,
                       const int32_t* pose_off, const double* T_wc, rm_cost_params params,
                       double* out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): rm_align_cost_grad
 * with every scratch buffer of the call (visible-cluster lists, bin counters,
 * tile bins, per-tile partial records, cluster bounds when mesh->clusters is
 * NULL) carved from a fixed 256 MiB device array that the library holds on
 * each device it runs on until the process ends.  Arguments, outputs and
 * results are those of rm_align_cost_grad; the call never allocates, never
 * synchronizes and never autotunes (it uses the tile set by rm_set_tile, else
 * 64x32).  When the tile bins do not fit beside the rest, their capacity is
 * lowered and overflowing tiles are rasterized from every visible cluster of
 * their pose (slower, same records).  A call whose scratch without bins
 * exceeds the array (about 12 bytes per (pose, cluster) plus 176 bytes per
 * (pose, tile), plus 12 bytes per triangle without prepared clusters) returns
 * RM_ERR_CAPACITY and launches nothing.  All such calls on one device share
 * that device's array: calls that overlap in time on one device (different
 * streams or contexts) race and give undefined results; calls ordered on one
 * stream are safe, since each clears what it needs before use. */
int rm_align_cost_grad_noalloc(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t n_scans,
                               const int32_t* pose_off, const double* T_wc, rm_cost_params params, double* out);

/* Table I with reweighted cells (Sec. IV-C suggests adjusting the weights of
 * the penalties and rewards of the classifications), plus the color term:
 * for each of P result records of rm_align_cost / rm_align_cost_grad,
 *   cost_out[p] = sum_{k<9} weights[k] * COUNTS_k(p)
 *               + weights[9] * COLOR_REWARD(p) + weights[10] * COLOR_PENALTY(p),
 * the nine cells in the order of RM_OUT_COUNTS.  The weights
 * (-1, +1, -1, +1, -1, +1, 0, 0, 0, 0, 0) give E_TABLE.
 *   out       device [P][RM_OUT_STRIDE] f64
 *   weights   host, RM_N_WEIGHTS doubles (finite)
 *   cost_out  device [P] f64 */
#define RM_N_WEIGHTS 11
int rm_table_cost_weighted(rm_ctx* ctx, const double* out, int32_t n_poses, const double* weights, double* cost_out);

/* ---------------------------------------------------------------- render-accelerated ICP (Sec. V) */

/* Step 1 of the sequential depth-image alignment (Sec. V-B): keeps every
 * factor-th pixel of every factor-th row and drops far points.
 *   depth  device [H][W] f32; out device [ceil(H/factor)][ceil(W/factor)] f32
 *   out(i, j) = depth(factor i, factor j) if it is a finite positive depth
 *               of at most z_max, NaN otherwise.
 * The downsampled image's camera has fx, fy, cx, cy divided by factor.
 * factor >= 1; z_max > 0. */
int rm_depth_downsample(rm_ctx* ctx, const float* depth, int32_t height, int32_t width, int32_t factor,
                        float z_max, float* out);

/* Depth-image normals of Eq. (2) (Sec. V-A).  The depth image is smoothed
 * with a Gaussian (standard deviation sigma pixels, truncated to the
 * (2 radius + 1)^2 window, weights renormalized over the window's valid
 * pixels, FP64); with the central differences dz_x = z~(u+1, v) - z~(u-1, v),
 * dz_y = z~(u, v+1) - z~(u, v-1) of the smoothed depth z~ and the metric
 * steps dx = 2 z~/fx, dy = 2 z~/fy at the pixel, the normal is
 *   N = (0, dy, dz_y) x (dx, 0, dz_x) = (dy dz_x, dx dz_y, -dx dy),
 * normalized, in the camera frame (facing the camera: N_z < 0).
 *   depth    device [H][W] f32, NaN = invalid
 *   normals  device [H][W][3] f32; NaN on the image border and where the
 *            pixel or one of its four difference neighbours is invalid.
 * sigma > 0; radius in 0..RM_MAX_NORMAL_RADIUS.  Uses 8 H W bytes of the
 * context's scratch. */
#define RM_MAX_NORMAL_RADIUS 8
int rm_depth_normals(rm_ctx* ctx, const float* depth, int32_t height, int32_t width, float fx, float fy,
                     float sigma, int32_t radius, float* normals);

/* World-frame normal of every vertex of rm_mesh_from_range's mesh of the
 * same image with the same stride and pose: vertex i*gw + j takes the normal
 * at pixel (j*stride, i*stride) rotated by T_wc's rotation (FP64, rounded
 * to f32; NaN stays NaN).  This is how the rendered view of Sec. V-B step 3
 * carries the normals of the depth image it was built from.
 *   normals  device [H][W][3] f32 (rm_depth_normals)
 *   T_wc     host, 12 doubles (row-major 3x4)
 *   out      device [ceil(H/stride) * ceil(W/stride)][3] f32 */
int rm_vertex_normals(rm_ctx* ctx, const float* normals, int32_t height, int32_t width, int32_t stride,
                      const double* T_wc, float* out);

/* Render-accelerated point-to-plane ICP (Sec. V): for every pose of S scans,
 * renders the mesh, associates each scan return with the surface its pixel
 * sees when their depths differ by less than tol (projective
 * correspondence), and writes the cost, the point-to-plane residual sums and
 * the Gauss-Newton blocks (RM_OUT_ICP_* and the fields listed there).
 * vertex_normals: device [n_vertices][3] f32, world frame (rm_vertex_normals).
 * Scans, pose_off, T_wc and out as for rm_align_cost_grad; the scan depth d_s
 * of an RM_FO pixel is the point Z_1.  rm_gn_step on the records gives the
 * ICP update.  tol > 0. */
int rm_icp_cost_grad(rm_ctx* ctx, const rm_mesh* mesh, const float* vertex_normals, const rm_scan* scans,
                     int32_t n_scans, const int32_t* pose_off, const double* T_wc, float tol, double* out);

/* ---------------------------------------------------------------- optimizer step */

/* Levenberg-Marquardt pose update for P poses from their result records:
 *   delta = -(H + lambda diag(H))^-1 b,   T_wc <- T_wc exp(delta)
 * (H = JTJ, b = JTR; delta = 0 where H + lambda diag(H) is not positive
 * definite).  T_wc: device [P][12] f64, updated in place; delta_out: device
 * [P][6] f64, nullable. */
int rm_gn_step(rm_ctx* ctx, const double* out, int32_t n_poses, double lambda,
               double* T_wc, double* delta_out);
/* Adam step on the se(3) increment from the GRAD field of the result
 * records (first and second moments m, v: device [P][6] f64, updated in
 * place; step = 1 for the first call):
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   delta = -lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + 1e-12),
 *   T_wc <- T_wc exp(delta). */
int rm_adam_step(rm_ctx* ctx, const double* out, int32_t n_poses, double lr, double beta1, double beta2,
                 int32_t step, double* m, double* v, double* T_wc);
/* T_out = T_in exp(delta) for P poses (device [P][12], [P][6], [P][12] f64;
 * T_out may equal T_in). */
int rm_se3_retract(rm_ctx* ctx, const double* T_in, const double* delta, int32_t n_poses,
                   double* T_out);

#ifdef __cplusplus
}
#endif

#endif /* RENDERMAP_H */
