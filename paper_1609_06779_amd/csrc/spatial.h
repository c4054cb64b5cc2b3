// spatial.h -- se(3)/SE(3) device primitives for gfx950 (Sec. II-A).
//
// Conventions: twist V = (w; v), wrench F = (n; f); a pose T = (R, p) acts on
// twists as Ad_T = [[R, 0], [[p]R, R]] and ad_V = [[[w], 0], [[v], [w]]], with
// ad*_V = ad_V^T (Sec. II-A). Spatial inertias about the frame origin are kept
// as 10 numbers: m, h = m c and Ibar = Ic - m[c][c] (xx yy zz xy xz yz), so
// J = [[Ibar, [h]], [-[h], m 1]].
//
// Every joint frame is rotated at model upload so that its joint axis is the
// local z axis: S_i = e3 for every joint, a twist's joint component is index 2.
#pragma once
#include <hip/hip_runtime.h>

namespace fdk {

template <typename T> struct Pose { T r[9]; T p[3]; };   // row-major R

template <typename T> __device__ __forceinline__ void cross3(const T a[3], const T b[3], T c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T> __device__ __forceinline__ void matvec3(const T r[9], const T x[3], T y[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = r[3 * i] * x[0] + r[3 * i + 1] * x[1] + r[3 * i + 2] * x[2];
}

template <typename T> __device__ __forceinline__ void matTvec3(const T r[9], const T x[3], T y[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = r[i] * x[0] + r[3 + i] * x[1] + r[6 + i] * x[2];
}

template <typename T> __device__ __forceinline__ Pose<T> pose_identity() {
    Pose<T> t;
#pragma unroll
    for (int i = 0; i < 9; ++i) t.r[i] = (i % 4 == 0) ? T(1) : T(0);
    t.p[0] = t.p[1] = t.p[2] = T(0);
    return t;
}

// a * b (apply b first): (Ra Rb, Ra pb + pa)
template <typename T> __device__ __forceinline__ Pose<T> pose_mul(const Pose<T>& a, const Pose<T>& b) {
    Pose<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c.r[3 * i + j] = a.r[3 * i] * b.r[j] + a.r[3 * i + 1] * b.r[3 + j] + a.r[3 * i + 2] * b.r[6 + j];
    matvec3(a.r, b.p, c.p);
    c.p[0] += a.p[0];
    c.p[1] += a.p[1];
    c.p[2] += a.p[2];
    return c;
}

// Joint pose T_{i-1,i} = (Rhome Rz(q), p) in the canonical (axis = z) frames.
template <typename T>
__device__ __forceinline__ Pose<T> joint_pose(const T rh[9], const T p[3], T q) {
    T s, c;
    if constexpr (sizeof(T) == 8) sincos(q, &s, &c); else sincosf(q, &s, &c);
    Pose<T> t;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        t.r[3 * i + 0] = rh[3 * i] * c + rh[3 * i + 1] * s;
        t.r[3 * i + 1] = rh[3 * i + 1] * c - rh[3 * i] * s;
        t.r[3 * i + 2] = rh[3 * i + 2];
    }
    t.p[0] = p[0];
    t.p[1] = p[1];
    t.p[2] = p[2];
    return t;
}

// Ad_T x for a twist x: (R w; p x (R w) + R v)
template <typename T> __device__ __forceinline__ void ad_apply(const Pose<T>& t, const T x[6], T y[6]) {
    T rw[3], rv[3], pc[3];
    matvec3(t.r, x, rw);
    matvec3(t.r, x + 3, rv);
    cross3(t.p, rw, pc);
    y[0] = rw[0]; y[1] = rw[1]; y[2] = rw[2];
    y[3] = pc[0] + rv[0]; y[4] = pc[1] + rv[1]; y[5] = pc[2] + rv[2];
}

// Ad_T^-1 x = Ad_{T^-1} x: (R^T w; R^T (v - p x w))
template <typename T> __device__ __forceinline__ void ad_inv_apply(const Pose<T>& t, const T x[6], T y[6]) {
    T pc[3], d[3];
    cross3(t.p, x, pc);
    d[0] = x[3] - pc[0]; d[1] = x[4] - pc[1]; d[2] = x[5] - pc[2];
    matTvec3(t.r, x, y);
    matTvec3(t.r, d, y + 3);
}

// (Ad_{T^-1})^T f for a wrench f = (n; f): (R n + p x (R f); R f).
// Moves a wrench from the child frame of T to its parent frame.
template <typename T> __device__ __forceinline__ void wrench_to_parent(const Pose<T>& t, const T f[6], T y[6]) {
    T rn[3], rf[3], pc[3];
    matvec3(t.r, f, rn);
    matvec3(t.r, f + 3, rf);
    cross3(t.p, rf, pc);
    y[0] = rn[0] + pc[0]; y[1] = rn[1] + pc[1]; y[2] = rn[2] + pc[2];
    y[3] = rf[0]; y[4] = rf[1]; y[5] = rf[2];
}

// (Ad_T)^T f = (R^T (n - p x f); R^T f): a wrench in T's parent frame moved to T's child frame.
template <typename T> __device__ __forceinline__ void wrench_to_child(const Pose<T>& t, const T f[6], T y[6]) {
    T pc[3], d[3];
    cross3(t.p, f + 3, pc);
    d[0] = f[0] - pc[0]; d[1] = f[1] - pc[1]; d[2] = f[2] - pc[2];
    matTvec3(t.r, d, y);
    matTvec3(t.r, f + 3, y + 3);
}

// ad_V x = (w x xw; v x xw + w x xv)
template <typename T> __device__ __forceinline__ void ad_twist(const T v[6], const T x[6], T y[6]) {
    T a[3], b[3];
    cross3(v, x, y);
    cross3(v + 3, x, a);
    cross3(v, x + 3, b);
    y[3] = a[0] + b[0]; y[4] = a[1] + b[1]; y[5] = a[2] + b[2];
}

// ad_V^T f = (-w x n - v x f; -w x f)
template <typename T> __device__ __forceinline__ void ad_twist_T(const T v[6], const T f[6], T y[6]) {
    T a[3], b[3], c[3];
    cross3(v, f, a);
    cross3(v + 3, f + 3, b);
    cross3(v, f + 3, c);
    y[0] = -a[0] - b[0]; y[1] = -a[1] - b[1]; y[2] = -a[2] - b[2];
    y[3] = -c[0]; y[4] = -c[1]; y[5] = -c[2];
}

// Spatial inertia (10 numbers) about the frame origin.
template <typename T> struct Inertia { T m; T h[3]; T ib[6]; };   // ib: xx yy zz xy xz yz

template <typename T> __device__ __forceinline__ void sym3_vec(const T s[6], const T x[3], T y[3]) {
    y[0] = s[0] * x[0] + s[3] * x[1] + s[4] * x[2];
    y[1] = s[3] * x[0] + s[1] * x[1] + s[5] * x[2];
    y[2] = s[4] * x[0] + s[5] * x[1] + s[2] * x[2];
}

// J x = (Ibar w + h x v; w x h + m v)
template <typename T> __device__ __forceinline__ void inertia_apply(const Inertia<T>& j, const T x[6], T y[6]) {
    T a[3], b[3], c[3];
    sym3_vec(j.ib, x, a);
    cross3(j.h, x + 3, b);
    cross3(x, j.h, c);
    y[0] = a[0] + b[0]; y[1] = a[1] + b[1]; y[2] = a[2] + b[2];
    y[3] = c[0] + j.m * x[3]; y[4] = c[1] + j.m * x[4]; y[5] = c[2] + j.m * x[5];
}

// Link force of eq. (EOM-single): J a - ad_V^T (J V)
template <typename T>
__device__ __forceinline__ void link_force(const Inertia<T>& j, const T v[6], const T a[6], T f[6]) {
    T jv[6], ja[6], g[6];
    inertia_apply(j, v, jv);
    inertia_apply(j, a, ja);
    ad_twist_T(v, jv, g);
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] = ja[k] - g[k];
}

// Dense symmetric 6x6 as a full array (row-major) -- used where the structure is general.
template <typename T> __device__ __forceinline__ void inertia_to_mat6(const Inertia<T>& j, T m[36]) {
    const T* s = j.ib;
    m[0] = s[0]; m[1] = s[3]; m[2] = s[4];
    m[6] = s[3]; m[7] = s[1]; m[8] = s[5];
    m[12] = s[4]; m[13] = s[5]; m[14] = s[2];
    // [h] in the upper right, -[h] = [h]^T in the lower left
    const T* h = j.h;
    m[3] = T(0);   m[4] = -h[2]; m[5] = h[1];
    m[9] = h[2];   m[10] = T(0); m[11] = -h[0];
    m[15] = -h[1]; m[16] = h[0]; m[17] = T(0);
    m[18] = T(0);  m[19] = h[2];  m[20] = -h[1];
    m[24] = -h[2]; m[25] = T(0);  m[26] = h[0];
    m[30] = h[1];  m[31] = -h[0]; m[32] = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m[6 * (a + 3) + b + 3] = (a == b) ? j.m : T(0);
}

// ---------------- small dense SPD factor / solves (registers) ----------------

// 1/p and 1/sqrt(p) to full precision for p > 0 (normal): the hardware
// estimate refined, in place of the division and square-root expansions. For
// p <= 0 the result is meaningless; callers check p > 0.
// FP64: the estimate is good to about 5e-8, so one third-order step takes it
// below the rounding of a double (error of order 5e-8 cubed): with
// e = 1 - p r, 1/p = r / (1 - e) = r (1 + e + e^2 + ...), and with
// e = 1 - p y^2, 1/sqrt(p) = y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 + ...).
// Three and five operations against four and eight for two Newton steps,
// with shorter dependency chains and the same rounding error (a CPU emulation
// over 2e4 values: at most 0.50 and 0.96 ulp).
__device__ __forceinline__ double rcp_refined(double p) {
    const double r = __builtin_amdgcn_rcp(p);
    const double e = __builtin_fma(-p, r, 1.0);
    return __builtin_fma(r, __builtin_fma(e, e, e), r);
}
__device__ __forceinline__ float rcp_refined(float p) {
    float r = __builtin_amdgcn_rcpf(p);
    return __builtin_fmaf(r, __builtin_fmaf(-p, r, 1.0f), r);
}
__device__ __forceinline__ double rsqrt_refined(double p) {
    const double y = __builtin_amdgcn_rsq(p);
    const double e = __builtin_fma(-p * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}
// FP32: one Newton step, y <- y + (y / 2)(1 - p y^2), on the hardware estimate
__device__ __forceinline__ float rsqrt_refined(float p) {
    float y = __builtin_amdgcn_rsqf(p);
    return __builtin_fmaf(0.5f * y, __builtin_fmaf(-p * y, y, 1.0f), y);
}

// In-place lower Cholesky of a K x K SPD matrix stored row-major in a[K*K];
// only the lower triangle is read and written. Returns false on a non-positive pivot.
template <typename T, int K> __device__ __forceinline__ bool chol_inplace(T a[K * K]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        T d = a[j * K + j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= a[j * K + k] * a[j * K + k];
        ok = ok && (d > T(0));
        const T r = rsqrt_refined(d);           // 1 / L_jj
        a[j * K + j] = r;                       // keep the reciprocal of the pivot
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            T s = a[i * K + j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= a[i * K + k] * a[j * K + k];
            a[i * K + j] = s * r;
        }
    }
    return ok;
}

// Solve (L L^T) x = b with L from chol_inplace (diagonal holds 1/L_jj).
template <typename T, int K> __device__ __forceinline__ void chol_solve(const T l[K * K], T x[K]) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
        T s = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= l[i * K + k] * x[k];
        x[i] = s * l[i * K + i];
    }
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        T s = x[i];
#pragma unroll
        for (int k = i + 1; k < K; ++k) s -= l[k * K + i] * x[k];
        x[i] = s * l[i * K + i];
    }
}

}  // namespace fdk
