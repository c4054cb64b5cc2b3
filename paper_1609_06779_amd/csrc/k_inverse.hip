// k_inverse.hip -- batched inverse dynamics (CalcInvDyn, Algorithm 1) and the
// joint-space inertia of the JSIIA (Sec. II-C), one lane per link. TREE:
// branched robots numbered depth-first (tree scans, see rnea.h).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "rnea.h"

namespace fdk {

template <typename T, int NP, bool TREE>
__global__ __launch_bounds__(Geo<NP>::threads) void k_inverse(ModelView<T> m, ChainMap cm,
                                                               const T* __restrict__ q, const T* __restrict__ qd,
                                                               const T* __restrict__ qdd, int gravity,
                                                               T* __restrict__ tau) {
    __shared__ T xbuf[NP > 64 ? 9 * NP : 1];   // tree scans exchange up to 9 values per lane
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int b = blockIdx.x * Geo<NP>::chains + grp;
    ChainInfo ci{0, 0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    const bool active = li < ci.n;
    const int64_t st = ci.state0 + li;
    T qi = active ? q[st] : T(0), qdi = active ? qd[st] : T(0), qai = (active && qdd) ? qdd[st] : T(0);
    const int32_t code = TREE && active ? m.tree_il(li, ci.slot) : 0;
    LinkLane<T> k;
    T t = rnea_lane<T, NP, TREE>(m, ci.link0 + li, active, qi, qdi, qai, gravity != 0, li, xbuf, k, code);
    if (active) tau[st] = t;
    if (ci.unsolved) fill_unsolved(tau, ci.state0, ci.unsolved, li, NP);
}

template <typename T, int NP, bool TREE>
__global__ __launch_bounds__(Geo<NP>::threads) void k_mass(ModelView<T> m, ChainMap cm, const T* __restrict__ q,
                                                            T* __restrict__ mout) {
    __shared__ T xbuf[NP > 64 ? 10 * NP : 1];
    constexpr int SF = TREE ? 13 : 12;         // s (6), F (6), subtree end (trees)
    __shared__ T sf[Geo<NP>::chains * NP * SF];
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int b = blockIdx.x * Geo<NP>::chains + grp;
    ChainInfo ci{0, 0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    const bool active = li < ci.n;
    T qi = active ? q[ci.state0 + li] : T(0);
    const int32_t code = TREE && active ? m.tree_il(li, ci.slot) : 0;
    LinkLane<T> k;
    rnea_lane<T, NP, TREE>(m, ci.link0 + li, active, qi, T(0), T(0), false, li, xbuf, k, code);
    T f[6];
    composite_force<T, NP, TREE>(k, active, li, xbuf, f, code);
    T* my = sf + grp * NP * SF;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        my[c * NP + li] = k.s[c];
        my[(6 + c) * NP + li] = f[c];
    }
    if constexpr (TREE) my[12 * NP + li] = T(tree_end(code));
    __syncthreads();
    if (active) {
        const int n = ci.n;
        // chain b's n x n block starts at b * n * n (uniform batches)
        T* row = mout + (int64_t)b * n * n + (int64_t)li * n;
        for (int kk = 0; kk < n; ++kk) {
            T acc = T(0);
            if (kk <= li) {
#pragma unroll
                for (int c = 0; c < 6; ++c) acc += my[c * NP + kk] * f[c];
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) acc += k.s[c] * my[(6 + c) * NP + kk];
            }
            if constexpr (TREE) {      // links on different branches do not couple
                const bool related = kk <= li ? li < int(my[12 * NP + kk]) : kk < tree_end(code);
                acc = related ? acc : T(0);
            }
            row[kk] = acc;
        }
    }
    if (ci.unsolved) fill_unsolved(mout, (int64_t)b * ci.unsolved * ci.unsolved, (int64_t)ci.unsolved * ci.unsolved, li, NP);
}

template <typename T>
hipError_t launch_inverse(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd,
                          const T* qdd, int gravity, T* tau, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
#define CALL(P)                                                                                          \
    if (m.tree)                                                                                          \
        hipLaunchKernelGGL((k_inverse<T, P, true>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(Geo<P>::threads), 0, st, m, cm, q, qd, qdd, gravity, tau);              \
    else                                                                                                 \
        hipLaunchKernelGGL((k_inverse<T, P, false>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(Geo<P>::threads), 0, st, m, cm, q, qd, qdd, gravity, tau)
    FDK_NP_SWITCH(np, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mass(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, T* mout, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
#define CALL(P)                                                                                          \
    if (m.tree)                                                                                          \
        hipLaunchKernelGGL((k_mass<T, P, true>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(Geo<P>::threads), 0, st, m, cm, q, mout);                               \
    else                                                                                                 \
        hipLaunchKernelGGL((k_mass<T, P, false>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(Geo<P>::threads), 0, st, m, cm, q, mout)
    FDK_NP_SWITCH(np, CALL)
#undef CALL
    return hipGetLastError();
}

template hipError_t launch_inverse<double>(int, const ModelView<double>&, const ChainMap&, const double*,
                                           const double*, const double*, int, double*, hipStream_t);
template hipError_t launch_inverse<float>(int, const ModelView<float>&, const ChainMap&, const float*,
                                          const float*, const float*, int, float*, hipStream_t);
template hipError_t launch_mass<double>(int, const ModelView<double>&, const ChainMap&, const double*, double*,
                                        hipStream_t);
template hipError_t launch_mass<float>(int, const ModelView<float>&, const ChainMap&, const float*, float*,
                                       hipStream_t);

}  // namespace fdk
