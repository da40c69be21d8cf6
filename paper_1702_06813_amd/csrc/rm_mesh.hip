// Scan image, meshification and cluster bounds (Sec. IV-A of the paper).
#include "rm_internal.h"

namespace rm {

namespace {

enum { kDead = 0, kNoReturn = 1, kValid = 2 };

// Range pixel class: dead (NaN, negative, or a positive range below z_min),
// no-return (0, +inf, or beyond z_max: free space up to the sensor maximum),
// or valid.
__device__ __forceinline__ int range_class(float z, float z_min, float z_max) {
    if (isnan(z) || z < 0.0f) return kDead;
    if (z == 0.0f || isinf(z) || z > z_max) return kNoReturn;
    if (z < z_min) return kDead;
    return kValid;
}

__global__ void k_scan_image(const float* __restrict__ depth, int64_t n, float z_min, float z_max,
                             float* __restrict__ d_out, uint8_t* __restrict__ c_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float z = depth[i];
    const int k = range_class(z, z_min, z_max);
    d_out[i] = k == kValid ? z : (k == kNoReturn ? z_max : __int_as_float(0x7fc00000));
    c_out[i] = k == kValid ? RM_FO : (k == kNoReturn ? RM_FU : RM_NONE);
}

struct Pose12 { double m[12]; };

// Grid node (i, j) sits at pixel (j*s, i*s).  A valid node's depth is the
// FP64 mean of the valid pixels of the (2R+1)^2 window around it whose depth
// is within RM_SMOOTH_REL of the node pixel's (R = 0: the node pixel).
// Back-projection in FP64 at that depth (z_max for a no-return), world
// transform in FP64, one rounding to f32 at the end.  Dead nodes get NaN.
__global__ void k_mesh_nodes(const float* __restrict__ depth, int32_t H, int32_t W, int32_t s, int32_t R,
                             int32_t gh, int32_t gw, float fx, float fy, float cx, float cy,
                             Pose12 T, float z_min, float z_max, float* __restrict__ xyz,
                             uint8_t* __restrict__ kind) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)gh * gw) return;
    const int i = (int)(n / gw), j = (int)(n % gw);
    const int py = i * s, px = j * s;
    const float z = depth[(int64_t)py * W + px];
    const int k = range_class(z, z_min, z_max);
    kind[n] = (uint8_t)k;
    if (k == kDead) {
        const float q = __int_as_float(0x7fc00000);
        xyz[3 * n] = q; xyz[3 * n + 1] = q; xyz[3 * n + 2] = q;
        return;
    }
    double zd = (k == kNoReturn) ? (double)z_max : (double)z;
    if (k == kValid && R > 0) {
        const double zc = (double)z, tol = RM_SMOOTH_REL * zc;
        double sum = 0.0;
        int cnt = 0;
        for (int yy = max(py - R, 0); yy <= min(py + R, H - 1); ++yy)
            for (int xx = max(px - R, 0); xx <= min(px + R, W - 1); ++xx) {
                const float zn = depth[(int64_t)yy * W + xx];
                if (range_class(zn, z_min, z_max) != kValid) continue;
                if (fabs((double)zn - zc) <= tol) { sum += (double)zn; ++cnt; }
            }
        zd = sum / (double)cnt;
    }
    const double xc = zd * (((double)px - (double)cx) / (double)fx);
    const double yc = zd * (((double)py - (double)cy) / (double)fy);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double w = ((T.m[4 * r] * xc + T.m[4 * r + 1] * yc) + T.m[4 * r + 2] * zd) + T.m[4 * r + 3];
        xyz[3 * n + r] = (float)w;
    }
}

// Quad (qi, qj) between nodes (qi,qj) (qi,qj+1) (qi+1,qj) (qi+1,qj+1):
// returns 0 = dropped (a dead corner), 1 = free-occupied, 2 = free-unknown.
__device__ __forceinline__ int quad_state(const float* __restrict__ xyz, const uint8_t* __restrict__ kind,
                                          int gw, int qi, int qj, double lim2) {
    const int64_t n00 = (int64_t)qi * gw + qj;
    const int64_t c[4] = {n00, n00 + 1, n00 + gw + 1, n00 + gw};   // perimeter order
    int dead = 0, noret = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int kk = kind[c[k]];
        dead |= kk == kDead;
        noret |= kk == kNoReturn;
    }
    if (dead) return 0;
    int big = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float* a = xyz + 3 * c[k];
        const float* b = xyz + 3 * c[(k + 1) & 3];
        const double dx = (double)a[0] - (double)b[0];
        const double dy = (double)a[1] - (double)b[1];
        const double dz = (double)a[2] - (double)b[2];
        big |= ((dx * dx + dy * dy) + dz * dz) > lim2;
    }
    return (noret || big) ? 2 : 1;
}

// One wave64 per 8x8 block of quads: lane = row*8 + col inside the block.
__global__ void k_mesh_count(const float* __restrict__ xyz, const uint8_t* __restrict__ kind, int gh,
                             int gw, int bw, int64_t n_blocks, double lim2,
                             int32_t* __restrict__ counts) {
    const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x / 64);
    const int lane = threadIdx.x & 63;
    if (blk >= n_blocks) return;
    const int qi = (int)(blk / bw) * kQuadBlock + lane / kQuadBlock;
    const int qj = (int)(blk % bw) * kQuadBlock + lane % kQuadBlock;
    int st = 0;
    if (qi < gh - 1 && qj < gw - 1) st = quad_state(xyz, kind, gw, qi, qj, lim2);
    const uint64_t m = __ballot(st != 0);
    if (lane == 0) counts[blk] = 2 * __popcll(m);
}

// Exclusive prefix sum of the block counts (one workgroup of 1024 threads).
__global__ void k_mesh_scan(const int32_t* __restrict__ counts, int64_t n, int32_t* __restrict__ offsets,
                            int32_t* __restrict__ total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = t * per, e = b + per < n ? b + per : n;
    int64_t s = 0;
    for (int64_t k = b; k < e; ++k) s += counts[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t k = b; k < e; ++k) { offsets[k] = (int32_t)run; run += counts[k]; }
    if (t == 1023) *total = (int32_t)part[1023];
}

__global__ void k_mesh_emit(const float* __restrict__ xyz, const uint8_t* __restrict__ kind, int gh,
                            int gw, int bw, int64_t n_blocks, double lim2,
                            const int32_t* __restrict__ offsets, int64_t cap_t,
                            int32_t* __restrict__ tri, uint8_t* __restrict__ cls) {
    const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x / 64);
    const int lane = threadIdx.x & 63;
    if (blk >= n_blocks) return;
    const int qi = (int)(blk / bw) * kQuadBlock + lane / kQuadBlock;
    const int qj = (int)(blk % bw) * kQuadBlock + lane % kQuadBlock;
    int st = 0;
    if (qi < gh - 1 && qj < gw - 1) st = quad_state(xyz, kind, gw, qi, qj, lim2);
    const uint64_t m = __ballot(st != 0);
    if (!st) return;
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    const int64_t t0 = (int64_t)offsets[blk] + 2 * before;
    if (t0 + 2 > cap_t) return;                 // host reports RM_ERR_CAPACITY from the total
    const int32_t n00 = qi * gw + qj, n01 = n00 + 1, n10 = n00 + gw, n11 = n10 + 1;
    const uint8_t c = st == 2 ? RM_FU : RM_FO;
    tri[3 * t0] = n00; tri[3 * t0 + 1] = n01; tri[3 * t0 + 2] = n11;
    tri[3 * t0 + 3] = n00; tri[3 * t0 + 4] = n11; tri[3 * t0 + 5] = n10;
    cls[t0] = c;
    cls[t0 + 1] = c;
}

// Cluster bounds: one workgroup per cluster of kClusterTris triangles.
__global__ void __launch_bounds__(kWG) k_clusters(const float* __restrict__ xyz, uint32_t vmax,
                                                  const int32_t* __restrict__ tri, int64_t n_tris,
                                                  ClusterBounds* __restrict__ out) {
    __shared__ float red[6][kWG / 64];
    const int64_t t = (int64_t)blockIdx.x * kClusterTris + threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (t < n_tris) {
        for (int k = 0; k < 3; ++k) {
            const float* p = xyz + 3 * (int64_t)min((uint32_t)tri[3 * t + k], vmax);
            for (int d = 0; d < 3; ++d) { lo[d] = fminf(lo[d], p[d]); hi[d] = fmaxf(hi[d], p[d]); }
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], off));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off));
        }
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; ++d) { red[d][w] = lo[d]; red[3 + d][w] = hi[d]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        ClusterBounds b;
        for (int d = 0; d < 3; ++d) {
            float l = red[d][0], h = red[3 + d][0];
            for (int k = 1; k < kWG / 64; ++k) { l = fminf(l, red[d][k]); h = fmaxf(h, red[3 + d][k]); }
            b.lo[d] = l; b.hi[d] = h;
        }
        const int64_t rem = n_tris - (int64_t)blockIdx.x * kClusterTris;
        b.n_tris = (int32_t)(rem < kClusterTris ? rem : kClusterTris);
        b.pad = 0;
        out[blockIdx.x] = b;
    }
}

// World-frame unit normal of every triangle: cross product of the FP32
// vertices' differences in FP64, normalized, rounded to f32.
__global__ void k_normals(const float* __restrict__ xyz, uint32_t vmax, const int32_t* __restrict__ tri,
                          int64_t n_tris, float* __restrict__ nrm) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tris) return;
    const float* p0 = xyz + 3 * (int64_t)min((uint32_t)tri[3 * t], vmax);
    const float* p1 = xyz + 3 * (int64_t)min((uint32_t)tri[3 * t + 1], vmax);
    const float* p2 = xyz + 3 * (int64_t)min((uint32_t)tri[3 * t + 2], vmax);
    const double ax = (double)p1[0] - p0[0], ay = (double)p1[1] - p0[1], az = (double)p1[2] - p0[2];
    const double bx = (double)p2[0] - p0[0], by = (double)p2[1] - p0[1], bz = (double)p2[2] - p0[2];
    const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const double l = sqrt(nx * nx + ny * ny + nz * nz);
    const double il = l > 0.0 ? 1.0 / l : 0.0;
    nrm[3 * t] = (float)(nx * il);
    nrm[3 * t + 1] = (float)(ny * il);
    nrm[3 * t + 2] = (float)(nz * il);
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

int64_t meshify_blocks(int32_t H, int32_t W, int32_t stride) {
    const int64_t gh = (H + stride - 1) / stride, gw = (W + stride - 1) / stride;
    const int64_t qh = gh > 1 ? gh - 1 : 0, qw = gw > 1 ? gw - 1 : 0;
    return ((qh + kQuadBlock - 1) / kQuadBlock) * ((qw + kQuadBlock - 1) / kQuadBlock);
}

hipError_t launch_scan_image(hipStream_t st, const float* depth, int32_t H, int32_t W, float z_min,
                             float z_max, float* d_out, uint8_t* c_out) {
    const int64_t n = (int64_t)H * W;
    hipLaunchKernelGGL(k_scan_image, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, depth, n, z_min,
                       z_max, d_out, c_out);
    return hipGetLastError();
}

hipError_t launch_meshify(hipStream_t st, const float* depth, rm_camera cam, const double* T,
                          int32_t stride, int32_t smooth_radius, float z_min, float z_max, float max_edge,
                          float* xyz, int32_t* tri, uint8_t* cls, int64_t cap_t, uint8_t* kind,
                          int32_t* block_counts, int32_t* block_offsets, int32_t* total) {
    const int32_t H = cam.height, W = cam.width;
    const int32_t gh = (H + stride - 1) / stride, gw = (W + stride - 1) / stride;
    Pose12 P;
    for (int k = 0; k < 12; ++k) P.m[k] = T[k];
    const int64_t nn = (int64_t)gh * gw;
    hipLaunchKernelGGL(k_mesh_nodes, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, depth, H, W,
                       stride, smooth_radius, gh, gw, cam.fx, cam.fy, cam.cx, cam.cy, P, z_min, z_max, xyz, kind);
    const int64_t nb = meshify_blocks(H, W, stride);
    const int bw = (gw - 1 + kQuadBlock - 1) / kQuadBlock;
    const double lim2 = (double)max_edge * (double)max_edge;
    if (nb == 0) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, total, (int64_t)1);
        return hipGetLastError();
    }
    const unsigned g = (unsigned)((nb + 3) / 4);
    hipLaunchKernelGGL(k_mesh_count, dim3(g), dim3(256), 0, st, xyz, kind, gh, gw, bw, nb, lim2, block_counts);
    hipLaunchKernelGGL(k_mesh_scan, dim3(1), dim3(1024), 0, st, block_counts, nb, block_offsets, total);
    hipLaunchKernelGGL(k_mesh_emit, dim3(g), dim3(256), 0, st, xyz, kind, gh, gw, bw, nb, lim2, block_offsets,
                       cap_t, tri, cls);
    return hipGetLastError();
}

int64_t prepared_normals_offset(int64_t n_tris) {
    const int64_t nc = (n_tris + kClusterTris - 1) / kClusterTris;
    return (nc * (int64_t)sizeof(ClusterBounds) + 255) & ~(int64_t)255;
}

hipError_t launch_prepare(hipStream_t st, const float* xyz, int64_t n_vertices, const int32_t* tri,
                          int64_t n_tris, void* out) {
    const int64_t nc = (n_tris + kClusterTris - 1) / kClusterTris;
    if (nc == 0 || n_vertices < 1) return hipSuccess;
    const uint32_t vmax = (uint32_t)(n_vertices - 1);
    hipLaunchKernelGGL(k_clusters, dim3((unsigned)nc), dim3(kWG), 0, st, xyz, vmax, tri, n_tris,
                       static_cast<ClusterBounds*>(out));
    float* nrm = reinterpret_cast<float*>(static_cast<char*>(out) + prepared_normals_offset(n_tris));
    hipLaunchKernelGGL(k_normals, dim3((unsigned)((n_tris + 255) / 256)), dim3(256), 0, st, xyz, vmax, tri, n_tris,
                       nrm);
    return hipGetLastError();
}

hipError_t launch_zero_i32(hipStream_t st, int32_t* p, int64_t n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace rm
