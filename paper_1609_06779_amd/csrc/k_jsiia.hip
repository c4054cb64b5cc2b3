// k_jsiia.hip -- joint space inertia inversion algorithm (Sec. II-C), one lane per link.
//
// tau_delta = tau - ID(q, qd, 0) by the scans; the columns of M are the
// unit-acceleration inverse dynamics (qdd = e_k, qd = 0, no gravity), built
// from one suffix scan of base-frame inertias; then qdd = M^-1 tau_delta by a
// Cholesky factorisation (right-looking, one row of M per lane, with tau_delta
// carried as an extra column so the forward substitution happens on the way)
// and one backward substitution. M lives in LDS, padded to an odd row stride.
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
    ChainInfo ci{0, 0, 0};
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
