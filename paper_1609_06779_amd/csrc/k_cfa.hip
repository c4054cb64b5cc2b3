// k_cfa.hip -- the constraint force algorithm (Sec. III, Algorithm 1), one lane per link.
//
// With Phi = (I - Gamma) J^-1 (I - Gamma)^T (block tri-diagonal):
//   Phi_ii = J_i^-1 + Ad_i J_{i-1}^-1 Ad_i^T,  Phi_{i,i+1} = -J_i^-1 Ad_{i+1}^T,
// where Ad_i = Ad(T_{i-1,i}^-1). In the canonical joint frames S_i = e3 and
// W_i = [e1 e2 e4 e5 e6], so A = W^T Phi W has the 5x5 blocks of Phi without
// row and column 3 (eq. (cfa-eq2)), B tau = W^T Phi S tau and C = S^T Phi S.
// Steps, as in Algorithm 1: CalcInvDyn and CalcDiffTorques (tau_delta), the
// blocks of A and R = -B tau_delta, SolvBTDSys by odd-even elimination (F_c),
// then CalcAcc: F = S tau_delta + W F_c and qdd_i = S_i^T sum_k Phi_ik F_k
// (= C tau_delta + B^T F_c, eq. (fijany-final)).
//
// PROJ: the same algorithm without a basis W (whose choice Sec. VI leaves
// open): with the projector P_i = I - S_i S_i^T the system is the 6x6 one
//   A^ = P Phi P + S S^T,  A^ X = -P Phi S tau_delta,
// whose solution is X = W F_c for every W (x^T A^ x = a^T A a + |b|^2 for
// x = W a + S b, so A^ is SPD and the S part of X is zero); then F = S tau_delta
// + X as above. In the canonical frames P zeroes row and column 3 of each
// block and S S^T puts a one on the diagonal there: the odd-even elimination
// runs on 6x6 blocks instead of 5x5 (1.7 times the work).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "oee.h"
#include "rnea.h"

namespace fdk {

__device__ __forceinline__ constexpr int wsel(int a) { return a < 2 ? a : a + 1; }   // W_i coordinates

// Two wavefronts per SIMD (the register cap costs a small
// spill; latency hiding between the two wins, measured 14-17 % on MI355X).
// The FP64 projector form's 6x6 blocks need the whole register file of one.
template <typename T, int NP, bool PROJ>
__global__ __launch_bounds__(Geo<NP>::threads, (PROJ && sizeof(T) == 8) ? 1 : 2) void k_cfa(ModelView<T> m, ChainMap cm, const T* __restrict__ q,
                                                           const T* __restrict__ qd, const T* __restrict__ tau,
                                                           T* __restrict__ qdd, int* __restrict__ status, FdOut<T> o) {
    // The cross-wavefront scan exchange (NP > 64 only) and the OEE slots share
    // one array: the scans before the OEE and after it end with a barrier, and
    // so does every OEE level.
    constexpr int K = PROJ ? 6 : 5;               // block size of the constraint system
    constexpr int OS = Geo<NP>::chains * NP * OeeSlot<K>::size;
    __shared__ T lds_all[(NP > 64 && 12 * NP > OS) ? 12 * NP : OS];
    T* xbuf = lds_all;
    T* oslot = lds_all;
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int b = blockIdx.x * Geo<NP>::chains + grp;
    ChainInfo ci{0, 0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    const int n = ci.n;
    const bool active = li < n;
    const int64_t st = ci.state0 + li;
    const int64_t link = ci.link0 + li;
    T qi = active ? q[st] : T(0), qdi = active && !o.solve ? qd[st] : T(0), ti = active ? tau[st] : T(0);

    // CalcInvDyn(q, qd, 0) and CalcDiffTorques (solve mode: zero velocity and no
    // gravity make the bias exactly zero, so tau_delta = tau)
    LinkLane<T> k;
    const T tb = rnea_lane<T, NP>(m, link, active, qi, qdi, T(0), !o.solve, li, xbuf, k);
    const T td = active ? ti - tb : T(0);

    // Phi_ii = J_i^-1 + Ad_i J_{i-1}^-1 Ad_i^T. The second term is link i-1's
    // inverse inertia re-expressed in frame i, built from its parameters
    // (taken from lane li - 1) moved into frame i.
    T ip[10], iq[10];
    if (active) {
        // FP64: from the inertia the inverse dynamics read (ten fewer loads per
        // link); FP32 reads the parameters formed from the FP64 input at upload
        if constexpr (sizeof(T) == 8) inv_params_of(k.jb, ip);
        else m.inertia_inv_params(link, ip);
    } else {
#pragma unroll
        for (int c = 0; c < 10; ++c) ip[c] = (c < 3 || c == 9) ? T(1) : T(0);
    }
    shift_up<NP>(ip, iq, 10, 1, xbuf);
    T jinv[36], phi[36];
    inv_inertia6(ip, jinv);
    if (active && li > 0) {
        T ic[10], z[36];
        inv_inertia_to_child(k.tl, iq, ic);
        inv_inertia6(ic, z);
#pragma unroll
        for (int c = 0; c < 36; ++c) phi[c] = jinv[c] + z[c];
    } else {
#pragma unroll
        for (int c = 0; c < 36; ++c) phi[c] = active ? jinv[c] : T(0);
    }
    // Phi_{i,i+1} = -J_i^-1 Ad_{i+1}^T: row r = -(Ad_{i+1} (row r of J_i^-1))^T
    T pnx[36];
    Pose<T> tn;
    shift_down<NP>(k.tl.r, tn.r, 9, 1, xbuf);
    shift_down<NP>(k.tl.p, tn.p, 3, 1, xbuf);
    const bool has_next = active && li + 1 < n;
    const bool has_prev = active && li > 0;
    if (has_next) {
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            T y[6];
            ad_inv_apply(tn, jinv + 6 * r, y);
#pragma unroll
            for (int c = 0; c < 6; ++c) pnx[6 * r + c] = -y[c];
        }
    } else {
#pragma unroll
        for (int c = 0; c < 36; ++c) pnx[c] = T(0);
    }

    // R = -W^T (Phi_{i,i-1} e3 td_{i-1} + Phi_ii e3 td_i + Phi_{i,i+1} e3 td_{i+1}),
    // Phi_{i,i-1} e3 = (row 3 of Phi_{i-1,i})^T, supplied by lane i-1.
    T tdn, wsend[6], wprev[6];
    shift_down<NP>(&td, &tdn, 1, 1, xbuf);
    if (!has_next) tdn = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) wsend[c] = pnx[12 + c] * td;
    shift_up<NP>(wsend, wprev, 6, 1, xbuf);
    T rfull[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) rfull[c] = phi[6 * c + 2] * td + pnx[6 * c + 2] * tdn + (has_prev ? wprev[c] : T(0));

    T d[K * K], u[K * K], r[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int ga = PROJ ? a : wsel(a);
        r[a] = (PROJ && a == 2) ? T(0) : -rfull[ga];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const int gc = PROJ ? c : wsel(c);
            const bool axis = PROJ && (a == 2 || c == 2);   // P zeroes the joint axis, S S^T adds 1 on it
            d[K * a + c] = axis ? (a == c ? T(1) : T(0)) : phi[6 * ga + gc];
            u[K * a + c] = axis ? T(0) : pnx[6 * ga + gc];
        }
    }
    if (!active) {
        // keep inactive rows well defined (they never couple to active rows)
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int c = 0; c < K; ++c) d[K * a + c] = (a == c) ? T(1) : T(0);
    }
    // rows of Phi needed by CalcAcc
    T prow[6], nrow[6], ncol[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        prow[c] = phi[12 + c];
        nrow[c] = pnx[12 + c];
        ncol[c] = pnx[6 * c + 2];
    }

    // SolvBTDSys
    const bool ok = oee_solve_rows<T, K, NP>(d, u, r, li, n, active, oslot + grp * NP * OeeSlot<K>::size);

    // CalcAcc
    T f[6];
#pragma unroll
    for (int a = 0; a < K; ++a) f[PROJ ? a : wsel(a)] = r[a];
    f[2] = td;                                      // S tau_delta (X has no S part)
    T fn[6];
    shift_down<NP>(f, fn, 6, 1, xbuf);
    T csend = T(0), cprev;
#pragma unroll
    for (int c = 0; c < 6; ++c) csend += ncol[c] * f[c];
    shift_up<NP>(&csend, &cprev, 1, 1, xbuf);
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc += prow[c] * f[c] + (has_next ? nrow[c] * fn[c] : T(0));
    if (has_prev) acc += cprev;
    if (active) o.put(qdd, st, b, li, acc);
    if (ci.unsolved && qdd) fill_unsolved(qdd, ci.state0, ci.unsolved, li, NP);
    if (active && !ok && status) atomicOr(status, 1);
}

template <typename T>
hipError_t launch_cfa(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd, const T* tau,
                      T* qdd, int* status, const FdOut<T>& o, bool proj, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
#define CALL(P)                                                                                          \
    if (proj)                                                                                            \
        hipLaunchKernelGGL((k_cfa<T, P, true>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(Geo<P>::threads), 0, st, m, cm, q, qd, tau, qdd, status, o);            \
    else                                                                                                 \
        hipLaunchKernelGGL((k_cfa<T, P, false>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(Geo<P>::threads), 0, st, m, cm, q, qd, tau, qdd, status, o)
    FDK_NP_SWITCH(np, CALL)
#undef CALL
    return hipGetLastError();
}

template hipError_t launch_cfa<double>(int, const ModelView<double>&, const ChainMap&, const double*, const double*,
                                       const double*, double*, int*, const FdOut<double>&, bool, hipStream_t);
template hipError_t launch_cfa<float>(int, const ModelView<float>&, const ChainMap&, const float*, const float*,
                                      const float*, float*, int*, const FdOut<float>&, bool, hipStream_t);

}  // namespace fdk
