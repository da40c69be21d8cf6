// Internal declarations of the rendermap library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rendermap.h"

namespace rm {

constexpr int kWG = 256;                 // threads per workgroup everywhere
constexpr int kClusterTris = RM_CLUSTER_TRIS;
constexpr int kQuadBlock = 8;            // meshify emits 8x8 blocks of quads
constexpr int kRecFields = 41;           // per-(pose, tile) partial record, 4-byte fields
constexpr int kSnapLimit = 1 << 29;      // |snapped coordinate| must stay below this
constexpr int kSpillLists = 64;           // spill-list segments (each with its own counter)
constexpr int kSpillTops = 8;             // spill counters before the segments' fills
constexpr int kBinTable = 2048;          // tiles of a cluster rectangle binned per LDS pass (taller
                                         // rectangles are binned in bands of rows)
constexpr int kMaxTileGrid = 256;        // tiles per image row and column (8-bit rectangle fields)

// Per-cluster bounds written by rm_mesh_clusters: world AABB.
struct ClusterBounds {
    float lo[3];
    float hi[3];
    int32_t n_tris;       // triangles in this cluster (<= kClusterTris)
    int32_t pad;
};
static_assert(sizeof(ClusterBounds) == 32, "cluster record layout");

// One scan of a batched call, with its slice of poses and its tile grid.
struct ScanDesc {
    const float* depth;
    const uint8_t* cls;
    const uint8_t* mask;
    const float* color;   // scan intensity (color term), nullable
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near, z_far;
    int32_t pose_off, n_poses;
    int32_t tiles_x, tiles_y;
    int64_t item_off;     // first work item of this scan
    int64_t rec_off;      // first partial record of this scan
};

struct BatchDesc {
    int32_t n_scans;
    int32_t n_poses;
    int32_t tile_w, tile_h;
    float color_tol;      // color term: agreement threshold of corresponding pixels
    int64_t n_items;
    ScanDesc s[RM_MAX_SCANS];
};

enum Mode { kRender = 0, kCost = 1, kGrad = 2, kIcp = 3 };

struct RasterArgs {
    const float* xyz;
    const int32_t* tri;
    const uint8_t* cls;
    const float* nrm;            // [T][3] world-frame unit normals (prepared mesh)
    int64_t n_tris;
    uint32_t vmax;               // n_vertices - 1: vertex indices are clamped to it
    int32_t n_clusters;
    const double* T_wc;          // [P][12]
    const uint2* vis;            // [P][n_clusters] (cluster, packed tile rect)
    const int32_t* vis_count;    // [P]
    uint32_t* bins;              // [n_records][bin_cap] triangle ids per (scan, pose, tile):
                                 // small footprints from the front, large ones from the back
    int32_t* bin_small;          // [n_records] small entries appended (may exceed bin_cap)
    int32_t* bin_big;            // [n_records] large entries appended
    int32_t* bin_max;            // device [2]: largest small and large fill of the call's bins
    int32_t* bin_fill;           // device [2] or null: largest small and large fill reserved by the binning pass
    int32_t bin_cap;
    int32_t bin_big_cap;         // slots of a bin for large footprints (its back); the rest for small ones
    // Overflow (spill_top == null: none, and a bin that outgrows a part of
    // its capacity takes the every-cluster path; spill == null: counted only,
    // every spilling record is lost).  The binning pass writes entries past
    // a bin's parts to the spill list as (triangle, record, slot | large <<
    // 31); each record that spilled gets a region in pool for all its
    // entries, laid out like a bin of exactly its fill, unless the list ran
    // out of room for it (spill_lost) or the regions did.
    uint3* spill;                // [spill_cap]
    int64_t spill_cap;           // list entries, < 2^32 - 1
    unsigned long long* spill_top;  // device [kSpillTops + 2 kSpillLists], zeroed: list entries asked for
                                    // (kSpillLists times the fullest segment), region cursor, records
                                    // spilled, unused, region entries asked for, unused [3]; then the
                                    // fill of each list segment, then each segment's length minus the
                                    // start of its first range that crossed the segment's end
    int32_t* spill_lost;         // [n_records], zeroed
    int32_t* spill_recs;         // [n_records] records that spilled, -1 where without a region
    uint32_t* pool;              // [pool_cap] overflow regions
    int64_t pool_cap;
    int64_t* pool_off;           // [n_records] start of the record's region, -1: none
    const int32_t* order;        // null: one workgroup per item; else record indices, longest first
    int32_t* queue;              // device counter of taken items (persistent scheduling)
    int32_t n_order;
    float* rec;                  // partial records [n_records][kRecFields]
    float eps;                   // Table I threshold; the association tolerance in ICP mode
    const float* vnrm;           // ICP mode: [n_vertices][3] world-frame vertex normals
    const float* tri_color;      // cost and gradient modes, nullable: [T] triangle intensities
    float color_tol;
    // render outputs
    float* depth_out;
    int32_t* tri_out;
    uint8_t* cls_out;
};

// launchers (return hipError_t)
hipError_t launch_scan_image(hipStream_t st, const float* depth, int32_t H, int32_t W, float z_min,
                             float z_max, float* d_out, uint8_t* c_out);
hipError_t launch_meshify(hipStream_t st, const float* depth, rm_camera cam, const double* T,
                          int32_t stride, int32_t smooth_radius, float z_min, float z_max, float max_edge, float* xyz,
                          int32_t* tri, uint8_t* cls, int64_t cap_t, uint8_t* kind,
                          int32_t* block_counts, int32_t* block_offsets, int32_t* total);
// Prepared-mesh buffer: [n_clusters] ClusterBounds, then (256-byte aligned)
// [n_tris][3] f32 unit normals.
int64_t prepared_normals_offset(int64_t n_tris);
hipError_t launch_prepare(hipStream_t st, const float* xyz, int64_t n_vertices, const int32_t* tri,
                          int64_t n_tris, void* out);
hipError_t launch_zero_i32(hipStream_t st, int32_t* p, int64_t n);
hipError_t launch_cull(hipStream_t st, const BatchDesc& bd, const ClusterBounds* cb, int32_t n_clusters,
                       const double* T_wc, uint2* vis, float* vis_z, int32_t* vis_count, int32_t* vis_tris);
hipError_t launch_vis_sort(hipStream_t st, const BatchDesc& bd, int32_t n_clusters, const int32_t* vis_count,
                           const float* vis_z, uint2* vis);
hipError_t launch_bin(hipStream_t st, const BatchDesc& bd, const RasterArgs& a);
// After a spilling binning pass: overflow regions for the records that
// spilled, then the spilled entries placed in them.
hipError_t launch_overflow(hipStream_t st, const RasterArgs& a, int64_t n_records);
hipError_t launch_raster(hipStream_t st, const BatchDesc& bd, const RasterArgs& a, int mode);
// Longest-first order of the records of a binned call: counting sort of the
// records by log2 of their bin fill, descending.  hist: 32 zeroed counters.
hipError_t launch_order(hipStream_t st, const BatchDesc& bd, const int32_t* bin_small, const int32_t* bin_big,
                        int64_t n_records, int32_t* hist, int32_t* order);
// Workgroups of the persistent rasterizer that fit on the device at once.
int persistent_grid(int tile_w, int tile_h, int mode);
hipError_t launch_reduce(hipStream_t st, const BatchDesc& bd, const float* rec,
                         const int32_t* vis_tris, float eps, int mode, double* out);

// Gaussian weights over offsets -radius..radius (summing to 1).
struct GaussW {
    double w[2 * RM_MAX_NORMAL_RADIUS + 1];
    int32_t radius;
};
hipError_t launch_downsample(hipStream_t st, const float* depth, int32_t H, int32_t W, int32_t f, float z_max,
                             float* out);
// smoothed: device scratch [H][W] f64
hipError_t launch_depth_normals(hipStream_t st, const float* depth, int32_t H, int32_t W, double fx, double fy,
                                const GaussW& g, double* smoothed, float* normals);
// T_wc: host, 12 doubles
hipError_t launch_vertex_normals(hipStream_t st, const float* normals, int32_t H, int32_t W, int32_t stride,
                                 const double* T_wc, float* out);
hipError_t launch_gn_step(hipStream_t st, const double* out, int32_t P, double lambda, double* T,
                          double* delta_out);
hipError_t launch_adam_step(hipStream_t st, const double* out, int32_t P, double lr, double b1, double b2,
                            int32_t step, double* m, double* v, double* T);
hipError_t launch_retract(hipStream_t st, const double* T_in, const double* delta, int32_t P,
                          double* T_out);
// cost[p] = sum_k w[k] counts_k of record p (w: host, 9 doubles)
hipError_t launch_weighted(hipStream_t st, const double* out, int32_t P, const double* w, double* cost);

int64_t meshify_blocks(int32_t H, int32_t W, int32_t stride);

// Scratch of one scoring call: the context's own arena, grown on demand
// (fixed == nullptr), or a fixed device buffer that the call may not grow.
struct Arena {
    char* fixed = nullptr;
    size_t fixed_size = 0;
};
// Validation, batch description, tile choice and the scoring pass of
// rm_align_cost / rm_align_cost_grad / rm_icp_cost_grad (host runtime).
int align_common(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t S, const int32_t* pose_off,
                 const double* T_wc, rm_cost_params params, double* out, int mode, const float* vnrm,
                 const Arena* arena);
// Records an error message on the context and returns code.
int ctx_fail(rm_ctx* ctx, int code, const char* msg);
// Device of a context.
int ctx_device(const rm_ctx* ctx);
// Finds the allocation-free scratch array's address on `device` (current);
// called once per device by rm_ctx_create.
void noalloc_setup(int device);

}  // namespace rm
