// k_jsiia.hip -- joint space inertia inversion algorithm (Sec. II-C), one lane per link.
//
// tau_delta = tau - ID(q, qd, 0) by the scans; the columns of M are the
// unit-acceleration inverse dynamics (qdd = e_k, qd = 0, no gravity), built
// from one suffix scan of base-frame inertias; then qdd = M^-1 tau_delta.
//
// The inversion (the paper does not fix the method) is Gauss-Jordan
// elimination of [M | tau_delta] without pivoting (M is SPD, so every pivot is
// positive): step j removes column j from every other row, after which
// qdd_i = b_i / m_ii. Chains of up to 64 links keep one row of M per lane in
// registers; the trailing block stays symmetric, so the pivot row is the
// pivot column and one LDS column write per step broadcasts it. Longer chains
// keep M in LDS and use a right-looking Cholesky factorisation with
// tau_delta as an extra column, then one backward substitution.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "rnea.h"

namespace fdk {

template <typename T, int NP> struct JsiiaLds {
    static constexpr int ld = NP + 1;
    static constexpr int per_chain = NP * ld + 2 * NP;   // M, y, x
};

template <typename T, int NP>
__global__ __launch_bounds__(Geo<NP>::threads) void k_jsiia(ModelView<T> m, ChainMap cm, const T* __restrict__ q,
                                                             const T* __restrict__ qd, const T* __restrict__ tau,
                                                             T* __restrict__ qdd, int* __restrict__ status) {
    using L = JsiiaLds<T, NP>;
    __shared__ T xbuf[NP > 64 ? 10 * NP : 1];
    __shared__ T sf[Geo<NP>::chains * NP * 12];
    extern __shared__ unsigned char dyn_lds[];
    T* lds = reinterpret_cast<T*>(dyn_lds);
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int b = blockIdx.x * Geo<NP>::chains + grp;
    ChainInfo ci{0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    const int n = ci.n;
    const bool active = li < n;
    const int64_t st = ci.state0 + li;
    const int64_t link = ci.link0 + li;
    T qi = active ? q[st] : T(0), qdi = active ? qd[st] : T(0), ti = active ? tau[st] : T(0);

    LinkLane<T> k;
    const T tb = rnea_lane<T, NP>(m, link, active, qi, qdi, T(0), true, li, xbuf, k);
    T y = active ? ti - tb : T(0);

    T f[6];
    composite_force<T, NP>(k, active, li, xbuf, f);
    T* my = sf + grp * NP * 12;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        my[c * NP + li] = k.s[c];
        my[(6 + c) * NP + li] = f[c];
    }
    __syncthreads();
    T* mm = lds + grp * L::per_chain;
    T* yb = mm + NP * L::ld;
    T* xb = yb + NP;
    T* row = mm + li * L::ld;
    if (active) {
        for (int kk = 0; kk < n; ++kk) {
            T acc = T(0);
            if (kk <= li) {
#pragma unroll
                for (int c = 0; c < 6; ++c) acc += my[c * NP + kk] * f[c];
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) acc += k.s[c] * my[(6 + c) * NP + kk];
            }
            row[kk] = acc;
        }
    }
    __syncthreads();

    // right-looking Cholesky of the n x n block with tau_delta as an extra column
    bool ok = true;
    for (int j = 0; j < NP; ++j) {
        if (active && li == j) {
            T d = row[j];
            ok = d > T(0);
            T l = sqrt(d);
            row[j] = l;
            y = y / l;
            yb[j] = y;
        }
        __syncthreads();
        T lij = T(0);
        if (active && li > j) {
            lij = row[j] / mm[j * L::ld + j];
            row[j] = lij;
            y -= lij * yb[j];
        }
        __syncthreads();
        if (active && li > j) {
            for (int kk = j + 1; kk <= li; ++kk) row[kk] -= lij * mm[kk * L::ld + j];
        }
        __syncthreads();
    }
    // L^T x = y
    T x = T(0);
    for (int kk = NP - 1; kk >= 0; --kk) {
        if (active && li == kk) {
            x = y / row[kk];
            xb[kk] = x;
        }
        __syncthreads();
        if (active && li < kk && kk < n) y -= mm[kk * L::ld + li] * xb[kk];
        __syncthreads();
    }
    if (active) qdd[st] = x;
    if (active && !ok && status) atomicOr(status, 1);
}


// 1/p to full precision from the hardware estimate and two Newton steps (p > 0, normal).
__device__ __forceinline__ double rcp_refined(double p) {
    double r = __builtin_amdgcn_rcp(p);
    r = __builtin_fma(r, __builtin_fma(-p, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-p, r, 1.0), r);
}
__device__ __forceinline__ float rcp_refined(float p) {
    float r = __builtin_amdgcn_rcpf(p);
    return __builtin_fmaf(r, __builtin_fmaf(-p, r, 1.0f), r);
}

// Gauss-Jordan on register rows (NP <= 64: one wavefront holds 64 / NP chains).
template <typename T, int NP>
__global__ __launch_bounds__(64) void k_jsiia_gj(ModelView<T> m, ChainMap cm, const T* __restrict__ q,
                                                  const T* __restrict__ qd, const T* __restrict__ tau,
                                                  T* __restrict__ qdd, int* __restrict__ status) {
    static_assert(NP <= 64, "register rows need NP <= 64");
    constexpr int CH = Geo<NP>::chains;
    __shared__ T sf[CH * NP * 12];
    __shared__ T col[2][CH][2 * NP];   // double-buffered pivot column and right-hand sides
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int b = blockIdx.x * CH + grp;
    ChainInfo ci{0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    const int n = ci.n;
    const bool active = li < n;
    const int64_t st = ci.state0 + li;
    const int64_t link = ci.link0 + li;
    T qi = active ? q[st] : T(0), qdi = active ? qd[st] : T(0), ti = active ? tau[st] : T(0);

    LinkLane<T> k;
    const T tb = rnea_lane<T, NP>(m, link, active, qi, qdi, T(0), true, li, nullptr, k);
    T y = active ? ti - tb : T(0);
    T f[6];
    composite_force<T, NP>(k, active, li, nullptr, f);
    T* my = sf + grp * NP * 12;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        my[c * NP + li] = k.s[c];
        my[(6 + c) * NP + li] = f[c];
    }
    __syncthreads();
    // row li of M: M_ik = s_min(i,k) . F_max(i,k); padding rows/columns are the identity
    T row[NP];
#pragma unroll
    for (int kk = 0; kk < NP; ++kk) {
        T lo = T(0), up = T(0);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            lo += my[c * NP + kk] * f[c];
            up += k.s[c] * my[(6 + c) * NP + kk];
        }
        T v = kk <= li ? lo : up;
        row[kk] = (active && kk < n) ? v : (kk == li ? T(1) : T(0));
    }
    T diag = T(1);
    bool ok = true;
    // no branches in the sweep: lane-dependent choices are selects without arithmetic in them
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        T* cj = col[j & 1][grp];
        cj[li] = row[j];
        cj[NP + li] = y;
        __syncthreads();
        const T piv = cj[j];
        const T rp = rcp_refined(piv);
        const bool me = li == j;
        T fj = row[j] * rp;
        fj = me ? T(0) : fj;
        diag = me ? piv : diag;
        ok = me ? (piv > T(0)) : ok;
        y -= fj * cj[NP + j];
#pragma unroll
        for (int kk = j + 1; kk < NP; ++kk) row[kk] -= fj * cj[kk];
    }
    if (active) qdd[st] = y / diag;
    if (active && !ok && status) atomicOr(status, 1);
}

// largest chain the in-LDS factorisation takes for this precision
template <typename T> int jsiia_max_np() {
    int best = 0;
    for (int p = 8; p <= 256; p *= 2) {
        int chains = p < 64 ? 64 / p : 1;
        size_t lds = sizeof(T) * chains * ((size_t)p * (p + 1) + 2 * p) + sizeof(T) * chains * p * 12 +
                     (p > 64 ? sizeof(T) * 10 * p : 0);
        if (lds <= 160 * 1024) best = p;
    }
    return best;
}

template <typename T>
hipError_t launch_jsiia(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd, const T* tau,
                        T* qdd, int* status, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
    if (np <= 64) {
#define GJ(P)                                                                                        \
    hipLaunchKernelGGL((k_jsiia_gj<T, P>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains),  \
                       dim3(64), 0, st, m, cm, q, qd, tau, qdd, status)
        switch (np) {
            case 8: GJ(8); break;
            case 16: GJ(16); break;
            case 32: GJ(32); break;
            case 64: GJ(64); break;
            default: return hipErrorInvalidValue;
        }
#undef GJ
        return hipGetLastError();
    }
#define CALL(P)                                                                                           \
    {                                                                                                     \
        size_t lds = sizeof(T) * Geo<P>::chains * JsiiaLds<T, P>::per_chain;                              \
        if (P > jsiia_max_np<T>()) return hipErrorInvalidConfiguration;                                   \
        hipError_t e = hipFuncSetAttribute((const void*)k_jsiia<T, P>,                                    \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);         \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((k_jsiia<T, P>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains),      \
                           dim3(Geo<P>::threads), lds, st, m, cm, q, qd, tau, qdd, status);               \
    }
    FDK_NP_SWITCH(np, CALL)
#undef CALL
    return hipGetLastError();
}

template hipError_t launch_jsiia<double>(int, const ModelView<double>&, const ChainMap&, const double*, const double*,
                                         const double*, double*, int*, hipStream_t);
template hipError_t launch_jsiia<float>(int, const ModelView<float>&, const ChainMap&, const float*, const float*,
                                        const float*, float*, int*, hipStream_t);
template int jsiia_max_np<double>();
template int jsiia_max_np<float>();

}  // namespace fdk
