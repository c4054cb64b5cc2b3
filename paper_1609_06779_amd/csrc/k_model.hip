// k_model.hip -- model upload: raw per-link parameters to canonical joint frames.
//
// Frame i is turned about its origin by a constant rotation C_i whose third
// column is the joint axis, so that in the new frames every joint screw is
// S_i = e3 (the assumption S^T S = I of Sec. III-A holds exactly) and the
// constraint-force basis W_i of the CFA (Sec. III-B) is simply the other five
// coordinate directions. Joint coordinates, and therefore qdd, are unchanged:
//   Rhome'_i = C_{i-1}^T Rhome_i C_i,  p'_i = C_{i-1}^T p_i,
//   c'_i = C_i^T c_i,  Ic'_i = C_i^T Ic_i C_i,  C_0 = I (base frame kept).
// On a tree, i-1 reads the parent p(i) (C = I for the base).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fdk {

// raw layout per link (double): axis 3, home_rot 9, offset 3, mass 1, com 3, inertia 6
constexpr int RAW_AXIS = 0, RAW_HOME = 3, RAW_OFF = 12, RAW_MASS = 15, RAW_COM = 16, RAW_IN = 19, RAW_N = 25;

__device__ void canon_frame(const double* ax, double c[9]) {
    double nrm = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    double w[3] = {ax[0] / nrm, ax[1] / nrm, ax[2] / nrm};
    double a[3] = {0.0, 0.0, 0.0};
    if (fabs(w[0]) < 0.9) a[0] = 1.0; else a[1] = 1.0;
    double d = a[0] * w[0] + a[1] * w[1] + a[2] * w[2];
    double x[3] = {a[0] - d * w[0], a[1] - d * w[1], a[2] - d * w[2]};
    double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    x[0] /= xn; x[1] /= xn; x[2] /= xn;
    double y[3] = {w[1] * x[2] - w[2] * x[1], w[2] * x[0] - w[0] * x[2], w[0] * x[1] - w[1] * x[0]};
    for (int r = 0; r < 3; ++r) {
        c[3 * r + 0] = x[r];
        c[3 * r + 1] = y[r];
        c[3 * r + 2] = w[r];
    }
}

template <typename T>
__global__ void k_model_init(int64_t nl, const double* __restrict__ raw, const int64_t* __restrict__ parent_link,
                             T* __restrict__ out) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    const double* rl = raw + l * RAW_N;
    double ci[9], cp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    canon_frame(rl + RAW_AXIS, ci);
    const int64_t pl = parent_link[l];
    if (pl >= 0) canon_frame(raw + pl * RAW_N + RAW_AXIS, cp);
    const double* rh = rl + RAW_HOME;
    // R' = Cp^T Rh Ci
    double t[9], rp[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            t[3 * r + k] = rh[3 * r] * ci[k] + rh[3 * r + 1] * ci[3 + k] + rh[3 * r + 2] * ci[6 + k];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            rp[3 * r + k] = cp[r] * t[k] + cp[3 + r] * t[3 + k] + cp[6 + r] * t[6 + k];
    double pp[3], cc[3];
    const double* po = rl + RAW_OFF;
    const double* co = rl + RAW_COM;
    for (int r = 0; r < 3; ++r) {
        pp[r] = cp[r] * po[0] + cp[3 + r] * po[1] + cp[6 + r] * po[2];
        cc[r] = ci[r] * co[0] + ci[3 + r] * co[1] + ci[6 + r] * co[2];
    }
    const double* in = rl + RAW_IN;
    double ic[9] = {in[0], in[3], in[4], in[3], in[1], in[5], in[4], in[5], in[2]};
    double u[9], icp[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            u[3 * r + k] = ic[3 * r] * ci[k] + ic[3 * r + 1] * ci[3 + k] + ic[3 * r + 2] * ci[6 + k];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            icp[3 * r + k] = ci[r] * u[k] + ci[3 + r] * u[3 + k] + ci[6 + r] * u[6 + k];
    double m = rl[RAW_MASS];
    double c2 = cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2];
    // Ibar = Ic' + m (|c|^2 I - c c^T)
    double ib[6] = {icp[0] + m * (c2 - cc[0] * cc[0]), icp[4] + m * (c2 - cc[1] * cc[1]),
                    icp[8] + m * (c2 - cc[2] * cc[2]), icp[1] - m * cc[0] * cc[1],
                    icp[2] - m * cc[0] * cc[2], icp[5] - m * cc[1] * cc[2]};
    // inverse of the symmetric Ic' by cofactors
    double a00 = icp[0], a01 = icp[1], a02 = icp[2], a11 = icp[4], a12 = icp[5], a22 = icp[8];
    double k00 = a11 * a22 - a12 * a12, k01 = a02 * a12 - a01 * a22, k02 = a01 * a12 - a02 * a11;
    double k11 = a00 * a22 - a02 * a02, k12 = a01 * a02 - a00 * a12, k22 = a00 * a11 - a01 * a01;
    double det = a00 * k00 + a01 * k01 + a02 * k02;
    double idet = 1.0 / det;
    double iv[6] = {k00 * idet, k11 * idet, k22 * idet, k01 * idet, k02 * idet, k12 * idet};
    auto put = [&](int f, double v) { out[f * nl + l] = (T)v; };
    for (int k = 0; k < 9; ++k) put(MF_ROT + k, rp[k]);
    for (int k = 0; k < 3; ++k) put(MF_POS + k, pp[k]);
    put(MF_MASS, m);
    for (int k = 0; k < 3; ++k) put(MF_H + k, m * cc[k]);
    for (int k = 0; k < 6; ++k) put(MF_IB + k, ib[k]);
    for (int k = 0; k < 6; ++k) put(MF_ICINV + k, iv[k]);
    for (int k = 0; k < 3; ++k) put(MF_COM + k, cc[k]);
    put(MF_MINV, 1.0 / m);
}

// Unit quaternion (w, x, y, z) of a rotation matrix (row-major), by
// Shepperd's method: the largest of 4w^2, 4x^2, 4y^2, 4z^2 (read off the
// trace and the diagonal) fixes the divisor, so no step divides by a small
// number; the result is normalised.
__device__ void rot_to_quat(const double r[9], double qt[4]) {
    const double tr = r[0] + r[4] + r[8];
    double w, x, y, z;
    if (tr >= r[0] && tr >= r[4] && tr >= r[8]) {
        const double s = 2.0 * sqrt(1.0 + tr);
        w = 0.25 * s; x = (r[7] - r[5]) / s; y = (r[2] - r[6]) / s; z = (r[3] - r[1]) / s;
    } else if (r[0] >= r[4] && r[0] >= r[8]) {
        const double s = 2.0 * sqrt(1.0 + r[0] - r[4] - r[8]);
        w = (r[7] - r[5]) / s; x = 0.25 * s; y = (r[1] + r[3]) / s; z = (r[2] + r[6]) / s;
    } else if (r[4] >= r[8]) {
        const double s = 2.0 * sqrt(1.0 + r[4] - r[0] - r[8]);
        w = (r[2] - r[6]) / s; x = (r[1] + r[3]) / s; y = 0.25 * s; z = (r[5] + r[7]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + r[8] - r[0] - r[4]);
        w = (r[3] - r[1]) / s; x = (r[2] + r[6]) / s; y = (r[5] + r[7]) / s; z = 0.25 * s;
    }
    const double nrm = sqrt(w * w + x * x + y * y + z * z);
    qt[0] = w / nrm; qt[1] = x / nrm; qt[2] = y / nrm; qt[3] = z / nrm;
}

// Robot-interleaved copy of the fields the lane-per-chain kernels read
// (InterleavedField): link l (entry `index` of its robot) goes to column
// `column[l]`; its home rotation (the model's canonical-frame matrix, in the
// model's precision) becomes a quaternion, computed in FP64.
template <typename T>
__global__ void k_model_interleave(int64_t nl, const int32_t* __restrict__ column, const int32_t* __restrict__ index,
                                   int32_t num_robots, int64_t fstride, const T* __restrict__ soa, T* __restrict__ il) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    const int64_t dst = (int64_t)index[l] * num_robots + column[l];
    double r[9], qt[4];
    for (int k = 0; k < 9; ++k) r[k] = (double)soa[(MF_ROT + k) * nl + l];
    rot_to_quat(r, qt);
    for (int k = 0; k < 4; ++k) il[(IL_QUAT + k) * fstride + dst] = (T)qt[k];
    for (int k = 0; k < 3; ++k) il[(IL_POS + k) * fstride + dst] = soa[(MF_POS + k) * nl + l];
    il[IL_MASS * fstride + dst] = soa[MF_MASS * nl + l];
    for (int k = 0; k < 3; ++k) il[(IL_H + k) * fstride + dst] = soa[(MF_H + k) * nl + l];
    for (int k = 0; k < 6; ++k) il[(IL_IB + k) * fstride + dst] = soa[(MF_IB + k) * nl + l];
}

hipError_t launch_model_interleave(int64_t nl, const int32_t* column, const int32_t* index, int32_t num_robots,
                                   int64_t fstride, const void* soa, void* il, int as_float, hipStream_t st) {
    if (nl <= 0) return hipSuccess;
    dim3 block(128), grid((unsigned)((nl + 127) / 128));
    if (as_float)
        hipLaunchKernelGGL(k_model_interleave<float>, grid, block, 0, st, nl, column, index, num_robots, fstride,
                           (const float*)soa, (float*)il);
    else
        hipLaunchKernelGGL(k_model_interleave<double>, grid, block, 0, st, nl, column, index, num_robots, fstride,
                           (const double*)soa, (double*)il);
    return hipGetLastError();
}

hipError_t launch_model_init(int64_t nl, const double* raw, const int64_t* parent_link, void* out, int as_float,
                             hipStream_t st) {
    if (nl <= 0) return hipSuccess;
    dim3 block(128), grid((unsigned)((nl + 127) / 128));
    if (as_float)
        hipLaunchKernelGGL(k_model_init<float>, grid, block, 0, st, nl, raw, parent_link, (float*)out);
    else
        hipLaunchKernelGGL(k_model_init<double>, grid, block, 0, st, nl, raw, parent_link, (double*)out);
    return hipGetLastError();
}

}  // namespace fdk
