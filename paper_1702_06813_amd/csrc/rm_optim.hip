// Optimizer step on the device: Levenberg-Marquardt increment from the
// per-pose Gauss-Newton blocks and the SE(3) retraction T <- T exp(delta).
#include <cmath>

#include "rm_internal.h"

namespace rm {

namespace {

// exp of delta = (v, w) in se(3): R = I + A K + B K^2, V = I + B K + C K^2,
// K = [w]x, A = sin(th)/th, B = (1 - cos th)/th^2, C = (th - sin th)/th^3.
__device__ void se3_exp(const double* d, double R[3][3], double t[3]) {
    const double w0 = d[3], w1 = d[4], w2 = d[5];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-5) {
        A = 1.0 - th2 / 6.0 * (1.0 - th2 / 20.0);
        B = 0.5 - th2 / 24.0 * (1.0 - th2 / 30.0);
        C = 1.0 / 6.0 - th2 / 120.0 * (1.0 - th2 / 42.0);
    } else {
        const double s = sin(th), c = cos(th);
        A = s / th;
        B = (1.0 - c) / th2;
        C = (th - s) / (th2 * th);
    }
    const double K[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    double K2[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
    double V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double I = i == j ? 1.0 : 0.0;
            R[i][j] = I + A * K[i][j] + B * K2[i][j];
            V[i][j] = I + B * K[i][j] + C * K2[i][j];
        }
    for (int i = 0; i < 3; ++i) t[i] = V[i][0] * d[0] + V[i][1] * d[1] + V[i][2] * d[2];
}

__device__ void retract(const double* Tin, const double* d, double* Tout) {
    double R[3][3], t[3];
    se3_exp(d, R, t);
    double o[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            o[4 * i + j] = Tin[4 * i] * R[0][j] + Tin[4 * i + 1] * R[1][j] + Tin[4 * i + 2] * R[2][j];
        o[4 * i + 3] = Tin[4 * i + 3] + Tin[4 * i] * t[0] + Tin[4 * i + 1] * t[1] + Tin[4 * i + 2] * t[2];
    }
    for (int k = 0; k < 12; ++k) Tout[k] = o[k];
}

__global__ void k_gn_step(const double* __restrict__ out, int32_t P, double lambda, double* __restrict__ T,
                          double* __restrict__ delta_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double* o = out + (int64_t)p * RM_OUT_STRIDE;
    double A[6][6], b[6];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) { A[i][j] = A[j][i] = o[RM_OUT_JTJ + k]; ++k; }
    for (int i = 0; i < 6; ++i) { A[i][i] *= 1.0 + lambda; b[i] = o[RM_OUT_JTR + i]; }
    // Cholesky A = L L^T in place (lower triangle)
    bool ok = true;
    for (int j = 0; j < 6 && ok; ++j) {
        double s = A[j][j];
        for (int q = 0; q < j; ++q) s -= A[j][q] * A[j][q];
        if (!(s > 0.0)) { ok = false; break; }
        const double l = sqrt(s);
        A[j][j] = l;
        for (int i = j + 1; i < 6; ++i) {
            double t = A[i][j];
            for (int q = 0; q < j; ++q) t -= A[i][q] * A[j][q];
            A[i][j] = t / l;
        }
    }
    double d[6] = {0, 0, 0, 0, 0, 0};
    if (ok) {
        double y[6];
        for (int i = 0; i < 6; ++i) {
            double t = -b[i];
            for (int q = 0; q < i; ++q) t -= A[i][q] * y[q];
            y[i] = t / A[i][i];
        }
        for (int i = 5; i >= 0; --i) {
            double t = y[i];
            for (int q = i + 1; q < 6; ++q) t -= A[q][i] * d[q];
            d[i] = t / A[i][i];
        }
    }
    if (delta_out)
        for (int i = 0; i < 6; ++i) delta_out[6 * (int64_t)p + i] = d[i];
    double* Tp = T + 12 * (int64_t)p;
    double Tin[12];
    for (int i = 0; i < 12; ++i) Tin[i] = Tp[i];
    retract(Tin, d, Tp);
}

__global__ void k_retract(const double* __restrict__ Tin, const double* __restrict__ delta, int32_t P,
                          double* __restrict__ Tout) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double T[12], d[6];
    for (int i = 0; i < 12; ++i) T[i] = Tin[12 * (int64_t)p + i];
    for (int i = 0; i < 6; ++i) d[i] = delta[6 * (int64_t)p + i];
    retract(T, d, Tout + 12 * (int64_t)p);
}

__global__ void k_adam_step(const double* __restrict__ out, int32_t P, double lr, double b1, double b2,
                            double c1, double c2, double* __restrict__ m, double* __restrict__ v,
                            double* __restrict__ T) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double d[6];
    for (int i = 0; i < 6; ++i) {
        const double g = out[(int64_t)p * RM_OUT_STRIDE + RM_OUT_GRAD + i];
        const double mi = b1 * m[6 * (int64_t)p + i] + (1.0 - b1) * g;
        const double vi = b2 * v[6 * (int64_t)p + i] + (1.0 - b2) * g * g;
        m[6 * (int64_t)p + i] = mi;
        v[6 * (int64_t)p + i] = vi;
        d[i] = -lr * (mi / c1) / (sqrt(vi / c2) + 1e-12);
    }
    double* Tp = T + 12 * (int64_t)p;
    double Tin[12];
    for (int i = 0; i < 12; ++i) Tin[i] = Tp[i];
    retract(Tin, d, Tp);
}

}  // namespace

hipError_t launch_adam_step(hipStream_t st, const double* out, int32_t P, double lr, double b1, double b2,
                            int32_t step, double* m, double* v, double* T) {
    if (P <= 0) return hipSuccess;
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    hipLaunchKernelGGL(k_adam_step, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, out, P, lr, b1, b2, c1, c2, m, v,
                       T);
    return hipGetLastError();
}

hipError_t launch_gn_step(hipStream_t st, const double* out, int32_t P, double lambda, double* T,
                          double* delta_out) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gn_step, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, out, P, lambda, T, delta_out);
    return hipGetLastError();
}

hipError_t launch_retract(hipStream_t st, const double* T_in, const double* delta, int32_t P, double* T_out) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_retract, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, T_in, delta, P, T_out);
    return hipGetLastError();
}

namespace {

struct CellW { double w[RM_N_WEIGHTS]; };

// Weighted Table I cost of each pose from its nine cell counts and its two
// color counts.
__global__ void k_weighted(const double* __restrict__ out, int32_t P, CellW cw, double* __restrict__ cost) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double* o = out + (int64_t)p * RM_OUT_STRIDE;
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) e += cw.w[k] * o[RM_OUT_COUNTS + k];
    e += cw.w[9] * o[RM_OUT_COLOR_REWARD];
    e += cw.w[10] * o[RM_OUT_COLOR_PENALTY];
    cost[p] = e;
}

}  // namespace

hipError_t launch_weighted(hipStream_t st, const double* out, int32_t P, const double* w, double* cost) {
    CellW cw;
    for (int k = 0; k < RM_N_WEIGHTS; ++k) cw.w[k] = w[k];
    hipLaunchKernelGGL(k_weighted, dim3((unsigned)((P + kWG - 1) / kWG)), dim3(kWG), 0, st, out, P, cw, cost);
    return hipGetLastError();
}

}  // namespace rm
