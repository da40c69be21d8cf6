// Depth-image preparation for the render-accelerated point-to-plane ICP of
// Sec. V: downsampling with the far-point filter, Gaussian smoothing, the
// depth-image normals of Eq. (2) and per-vertex normals of a meshified view.
// These run once per depth image, outside the per-iteration render loop; the
// association and the point-to-plane blocks are fused into the tile pass.
#include "rm_internal.h"

namespace rm {

namespace {

// out(i, j) = depth(f i, f j) when it is a finite positive depth up to z_max,
// NaN otherwise.
__global__ void k_downsample(const float* __restrict__ depth, int32_t H, int32_t W, int32_t f, int32_t H2,
                             int32_t W2, float z_max, float* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)H2 * W2) return;
    const int i = (int)(n / W2), j = (int)(n % W2);
    const float z = depth[(int64_t)(i * f) * W + (int64_t)j * f];
    out[n] = (z > 0.0f && z <= z_max) ? z : __int_as_float(0x7fc00000);   // NaN and +inf fail both tests
}

// Gaussian smoothing over the valid pixels of the (2R+1)^2 window, weights
// w_a w_b renormalized over them (FP64); an invalid centre stays NaN.
__global__ void k_smooth(const float* __restrict__ depth, int32_t H, int32_t W, GaussW g,
                         double* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)H * W) return;
    const int y = (int)(n / W), x = (int)(n % W);
    const float zc = depth[n];
    if (!(zc == zc)) { out[n] = (double)__int_as_float(0x7fc00000); return; }
    double num = 0.0, den = 0.0;
    for (int a = -g.radius; a <= g.radius; ++a) {
        const int yy = y + a;
        if (yy < 0 || yy >= H) continue;
        const double wa = g.w[a + g.radius];
        for (int b = -g.radius; b <= g.radius; ++b) {
            const int xx = x + b;
            if (xx < 0 || xx >= W) continue;
            const float z = depth[(int64_t)yy * W + xx];
            if (!(z == z)) continue;
            const double w = wa * g.w[b + g.radius];
            num += w * (double)z;
            den += w;
        }
    }
    out[n] = num / den;
}

// Eq. (2): with the central differences dz_x, dz_y of the smoothed depth and
// the metric steps dx = 2 z/fx, dy = 2 z/fy at the centre, the normal is
// (0, dy, dz_y) x (dx, 0, dz_x) = (dy dz_x, dx dz_y, -dx dy), normalized
// (camera frame).  NaN on the border and where an input is invalid.
__global__ void k_normals(const double* __restrict__ zs, int32_t H, int32_t W, double fx, double fy,
                          float* __restrict__ nrm) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)H * W) return;
    const int y = (int)(n / W), x = (int)(n % W);
    const float q = __int_as_float(0x7fc00000);
    float o0 = q, o1 = q, o2 = q;
    if (x > 0 && x < W - 1 && y > 0 && y < H - 1) {
        const double c = zs[n];
        const double dzx = zs[n + 1] - zs[n - 1];
        const double dzy = zs[n + W] - zs[n - W];
        const double dx = 2.0 * c / fx, dy = 2.0 * c / fy;
        const double a = dy * dzx, b = dx * dzy, e = -dx * dy;
        const double inv = 1.0 / sqrt(a * a + b * b + e * e);   // NaN inputs give NaN
        o0 = (float)(a * inv); o1 = (float)(b * inv); o2 = (float)(e * inv);
    }
    nrm[3 * n] = o0; nrm[3 * n + 1] = o1; nrm[3 * n + 2] = o2;
}

struct Rot9 { double r[9]; };

// World normal of meshify node (i, j): the camera-frame normal at pixel
// (j s, i s) rotated by the view's rotation, in FP64, rounded to f32.
__global__ void k_vertex_normals(const float* __restrict__ nrm, int32_t W, int32_t s, int32_t gh, int32_t gw,
                                 Rot9 R, float* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)gh * gw) return;
    const int i = (int)(n / gw), j = (int)(n % gw);
    const float* p = nrm + 3 * ((int64_t)(i * s) * W + (int64_t)j * s);
    const double a = p[0], b = p[1], c = p[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) out[3 * n + k] = (float)(R.r[3 * k] * a + R.r[3 * k + 1] * b + R.r[3 * k + 2] * c);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kWG - 1) / kWG); }

}  // namespace

hipError_t launch_downsample(hipStream_t st, const float* depth, int32_t H, int32_t W, int32_t f, float z_max,
                             float* out) {
    const int32_t H2 = (H + f - 1) / f, W2 = (W + f - 1) / f;
    hipLaunchKernelGGL(k_downsample, dim3(blocks_for((int64_t)H2 * W2)), dim3(kWG), 0, st, depth, H, W, f, H2, W2,
                       z_max, out);
    return hipGetLastError();
}

hipError_t launch_depth_normals(hipStream_t st, const float* depth, int32_t H, int32_t W, double fx, double fy,
                                const GaussW& g, double* smoothed, float* normals) {
    const unsigned nb = blocks_for((int64_t)H * W);
    hipLaunchKernelGGL(k_smooth, dim3(nb), dim3(kWG), 0, st, depth, H, W, g, smoothed);
    hipLaunchKernelGGL(k_normals, dim3(nb), dim3(kWG), 0, st, smoothed, H, W, fx, fy, normals);
    return hipGetLastError();
}

hipError_t launch_vertex_normals(hipStream_t st, const float* normals, int32_t H, int32_t W, int32_t stride,
                                 const double* T_wc, float* out) {
    const int32_t gh = (H + stride - 1) / stride, gw = (W + stride - 1) / stride;
    Rot9 R;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R.r[3 * r + c] = T_wc[4 * r + c];
    hipLaunchKernelGGL(k_vertex_normals, dim3(blocks_for((int64_t)gh * gw)), dim3(kWG), 0, st, normals, W, stride,
                       gh, gw, R, out);
    return hipGetLastError();
}

}  // namespace rm
