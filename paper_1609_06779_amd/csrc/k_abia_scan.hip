// k_abia_scan.hip -- the articulated-body inertia algorithm (Sec. II-C) with a
// group of lanes per chain, its two linear recursions solved by the parallel
// scan of Sec. II-B.
//
// One chain per workgroup of NP = 64, 128 or 256 threads (lane i holds link i):
//  1. inverse dynamics at qdd = 0 by the scans of rnea.h: tau_delta_i;
//  2. the nonlinear backward recursion of the articulated inertias,
//        Jh_i = J_i + Ad_{i+1}^T Pi_{i+1} Ad_{i+1},  h_i = Jh_i S_i, D_i = S_i^T h_i,
//        Pi_i = Jh_i - h_i h_i^T / D_i,
//     which is serial in i (Sec. III: no speed-up beyond a constant factor).
//     It runs on the first wavefront with the 6x6 entries spread over 36
//     lanes: lane 6r + c holds entry (r, c), and each step is two exchanges
//     through LDS (Jh, from whose row r and column h a lane forms row r of Pi;
//     then Pi Ad);
//  3. the two (I - X^T)-type bi-diagonal systems, each as a scan of affine
//     6x6 elements (B_i, c_i) (x_i = B_i x_{i-1} + c_i):
//        backward  p_{i-1} = Ad_i^T (I - h_i S^T / D_i) p_i + Ad_i^T h_i tau_delta_i / D_i,
//                  u_i = tau_delta_i - S^T p_i;
//        forward   a_i = (I - S h_i^T / D_i) Ad_i a_{i-1} + S u_i / D_i,
//                  qdd_i = (u_i - h_i^T Ad_i a_{i-1}) / D_i,
//     with p beyond the tip and a at the base zero (zero velocity and no gravity:
//     the bias is already in tau_delta). Together they apply M^-1 to tau_delta.
// In the canonical joint frames S_i = e3 (index 2). Ad_i = Ad(T_{i-1,i}^-1);
// Ad_i^T moves a wrench from frame i to frame i - 1 (wrench_to_parent).
// Serial chains only. Where the lane-per-chain kernel (k_abia) spends n steps
// on every sweep, this one spends n short steps on the recursion and log2 NP
// scan steps on the rest, so it serves small batches (one robot: latency).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "rnea.h"

namespace fdk {

// Per-link record of the recursion in LDS, field f of link i at rec[f * NP + i]:
// the two 3x3 blocks of X_i = Ad_i^T = [[R, [p] R], [0, R]] (wrench_to_parent),
// the body inertia, and a field of zeros.
constexpr int F_R = 0, F_PR = 9, F_M = 18, F_H = 19, F_I = 22, F_ZERO = 28, F_COUNT = 29;

// Field of entry (a, k) of X.
__device__ __forceinline__ int x_entry_field(int a, int k) {
    if (a < 3) return k < 3 ? F_R + 3 * a + k : F_PR + 3 * a + (k - 3);
    return k < 3 ? F_ZERO : F_R + 3 * (a - 3) + (k - 3);
}

// Where entry (r, c) of the 6x6 spatial inertia J = [[Ibar, [h]], [-[h], m 1]]
// comes from among its parameters (Ibar as xx yy zz xy xz yz): the field and a
// sign in {-1, 0, 1}, fixed per lane, so the recursion reads it without branching.
__device__ __forceinline__ void inertia_entry_source(int r, int c, int* field, int* sign) {
    if (r >= 3 && c >= 3) {
        *field = F_M;
        *sign = r == c ? 1 : 0;
    } else if (r < 3 && c < 3) {
        *field = F_I + (r == c ? r : (r + c == 1 ? 3 : (r + c == 2 ? 4 : 5)));
        *sign = 1;
    } else {
        // [h] in the upper right block, -[h] in the lower left: entry (a, b) of [h],
        // [h]_{ab} = -eps_{abk} h_k
        const int a = r < 3 ? r : r - 3, b = r < 3 ? c - 3 : c;
        const bool even = (a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0);
        *field = F_H + (a == b ? 0 : 3 - a - b);
        *sign = a == b ? 0 : ((even ? -1 : 1) * (r < 3 ? 1 : -1));
    }
}

// (B, c) <- (B, c) o (B', c') = (B B', B c' + c) for affine 6x6 elements held
// as B (36, row-major) then c (6); row by row in place.
template <typename T> __device__ __forceinline__ void affine_compose(T el[42], const T o[42]) {
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        T row[7];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc += el[6 * r + k] * o[6 * k + c];
            row[c] = acc;
        }
        T acc = el[36 + r];
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += el[6 * r + k] * o[36 + k];
        row[6] = acc;
#pragma unroll
        for (int c = 0; c < 6; ++c) el[6 * r + c] = row[c];
        el[36 + r] = row[6];
    }
}

template <typename T, int NP>
__global__ __launch_bounds__(NP) void k_abia_scan(ModelView<T> m, ChainMap cm, const T* __restrict__ q,
                                                  const T* __restrict__ qd, const T* __restrict__ tau,
                                                  T* __restrict__ qdd, FdOut<T> o) {
    static_assert(NP >= 64 && NP <= 256, "one chain per workgroup of 64..256 lanes");
    // per-link records for the recursion and, for groups of several wavefronts,
    // the scans' exchange: never live at the same time
    constexpr int XCH = NP > 64 ? 42 * NP : 0;
    __shared__ T lds[F_COUNT * NP > XCH ? F_COUNT * NP : XCH];
    __shared__ T hd[7 * NP];      // h_i (6), D_i per link
    __shared__ T ex[2][36];       // the recursion's exchanges
    T* xbuf = lds;
    T* rec = lds;
    const int li = threadIdx.x;
    ChainInfo ci{0, 0, 0, 0, 0};
    if ((int)blockIdx.x < cm.batch) ci = chain_info(m, cm, blockIdx.x);
    const int n = ci.n;
    const bool active = li < n;
    const int64_t st = ci.state0 + li;
    const T qi = active ? q[st] : T(0), qdi = active && !o.solve ? qd[st] : T(0), ti = active ? tau[st] : T(0);

    // 1. tau_delta (solve mode: zero velocity, no gravity, so the bias is exactly zero)
    LinkLane<T> k;
    const T tb = rnea_lane<T, NP>(m, ci.link0 + li, active, qi, qdi, T(0), !o.solve, li, xbuf, k);
    const T td = active ? ti - tb : T(0);

    // 2. articulated inertias
    block_sync<NP>();                              // the inverse dynamics is done with the exchange buffer
    if (active) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {              // column c of [p] R is p x (column c of R)
            const T rc[3] = {k.tl.r[c], k.tl.r[3 + c], k.tl.r[6 + c]};
            T pc[3];
            cross3(k.tl.p, rc, pc);
#pragma unroll
            for (int a = 0; a < 3; ++a) rec[(F_PR + 3 * a + c) * NP + li] = pc[a];
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) rec[(F_R + c) * NP + li] = k.tl.r[c];
        rec[F_M * NP + li] = k.jb.m;
#pragma unroll
        for (int c = 0; c < 3; ++c) rec[(F_H + c) * NP + li] = k.jb.h[c];
#pragma unroll
        for (int c = 0; c < 6; ++c) rec[(F_I + c) * NP + li] = k.jb.ib[c];
    }
    rec[F_ZERO * NP + li] = T(0);
    block_sync<NP>();
    if (li < 64) {
        // Lane 6 er + ec (36 lanes) carries entry (er, ec). With X = Ad^T of the
        // link after i and Pi its articulated inertia less the joint's share,
        //   (Pi X^T)_{er,ec} = row er of Pi . row ec of X,
        //   (X Pi X^T)_{er,ec} = row er of X . column ec of Pi X^T,
        // so a lane reads two rows of X (fields fixed per lane) and forms each
        // exchanged entry with one 6-term dot product.
        const bool ent = li < 36;
        const int er = ent ? li / 6 : 0, ec = ent ? li % 6 : 0;
        int jfield, jsign;
        inertia_entry_source(er, ec, &jfield, &jsign);
        const T* jsrc = rec + jfield * NP;
        int fe[6], fr[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            fe[c] = x_entry_field(ec, c) * NP;
            fr[c] = x_entry_field(er, c) * NP;
        }
        T cprev = T(0);                            // (X Pi X^T)_{er,ec} of the link after i
#pragma unroll 1
        for (int i = n - 1; i >= 0; --i) {
            // reads that do not depend on the exchange go first
            const T jh = T(jsign) * jsrc[i] + cprev;
            T xe[6], xr[6];                        // rows ec and er of X_i
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                xe[c] = rec[fe[c] + i];
                xr[c] = rec[fr[c] + i];
            }
            if (ent) ex[0][li] = jh;
            block_sync<64>();
            const T dd = ex[0][14];
            if (li < 6) hd[li * NP + i] = ex[0][6 * li + 2];
            if (li == 6) hd[6 * NP + i] = dd;
            if (i == 0) break;
            // row er of Pi = Jh - h h^T / D with h = column 2 of Jh: its product
            // with row ec of X is (row er of Jh) . xe - (h_er / D) (h . xe)
            T a0 = T(0), a1 = T(0);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                a0 += ex[0][6 * er + c] * xe[c];
                a1 += ex[0][6 * c + 2] * xe[c];
            }
            const T pe = a0 - ex[0][6 * er + 2] * rcp_refined(dd) * a1;
            if (ent) ex[1][li] = pe;
            block_sync<64>();
            T ce = T(0);
#pragma unroll
            for (int c = 0; c < 6; ++c) ce += xr[c] * ex[1][6 * c + ec];
            cprev = ce;
        }
    }
    block_sync<NP>();                              // h, D of every link are in LDS; rec is free again

    T h[6], rd = T(1);
#pragma unroll
    for (int c = 0; c < 6; ++c) h[c] = active ? hd[c * NP + li] : T(0);
    if (active) rd = rcp_refined(hd[6 * NP + li]);

    // 3a. backward: element (B, c) = (Ad^T (I - h e3^T / D), Ad^T h td / D), suffix composition
    T el[42], ot[42];
    if (active) {
#pragma unroll
        for (int kc = 0; kc < 6; ++kc) {
            T v[6], w[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) v[r] = (r == kc ? T(1) : T(0)) - (kc == 2 ? h[r] * rd : T(0));
            wrench_to_parent(k.tl, v, w);
#pragma unroll
            for (int r = 0; r < 6; ++r) el[6 * r + kc] = w[r];
        }
        T v[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) v[r] = h[r] * (td * rd);
        wrench_to_parent(k.tl, v, el + 36);
    } else {
#pragma unroll
        for (int c = 0; c < 42; ++c) el[c] = T(0);
    }
    // Levels with s >= n pair every link only with lanes past the tip, whose
    // zero elements leave c as it is: they are not run (n is the same on every
    // lane of the workgroup, so every lane takes the same barriers).
#pragma unroll 1
    for (int s = 1; s < NP && s < n; s <<= 1) {
        shift_down<NP>(el, ot, 42, s, xbuf);
        if (li + s < NP) affine_compose(el, ot);
    }
    T pn[6];                                        // p_i: the suffix from link i + 1, applied to zero
    shift_down<NP>(el + 36, pn, 6, 1, xbuf);
    const T u = td - (li + 1 < n ? pn[2] : T(0));

    // 3b. forward: element (B, c) = ((I - e3 h^T / D) Ad, e3 u / D), prefix composition
    if (active) {
#pragma unroll
        for (int kc = 0; kc < 6; ++kc) {
            T v[6], w[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) v[r] = r == kc ? T(1) : T(0);
            ad_inv_apply(k.tl, v, w);               // column kc of Ad
            T hw = T(0);
#pragma unroll
            for (int r = 0; r < 6; ++r) hw += h[r] * w[r];
#pragma unroll
            for (int r = 0; r < 6; ++r) el[6 * r + kc] = r == 2 ? w[r] - hw * rd : w[r];
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) el[36 + r] = r == 2 ? u * rd : T(0);
    } else {
#pragma unroll
        for (int c = 0; c < 42; ++c) el[c] = T(0);
    }
#pragma unroll 1
    for (int s = 1; s < NP && s < n; s <<= 1) {    // s >= n: no partner at or after the base
        shift_up<NP>(el, ot, 42, s, xbuf);
        if (li >= s) affine_compose(el, ot);
    }
    T ap[6], aw[6];                                 // a_{i-1}, then Ad_i a_{i-1}
    shift_up<NP>(el + 36, ap, 6, 1, xbuf);
    if (li == 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) ap[c] = T(0);
    }
    ad_inv_apply(k.tl, ap, aw);
    T ha = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) ha += h[c] * aw[c];
    if (active) o.put(qdd, st, blockIdx.x, li, (u - ha) * rd);
    if (ci.unsolved && qdd) fill_unsolved(qdd, ci.state0, ci.unsolved, li, NP);
}

template <typename T>
hipError_t launch_abia_scan(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd,
                            const T* tau, T* qdd, const FdOut<T>& o, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
#define CALL(P) hipLaunchKernelGGL((k_abia_scan<T, P>), dim3(cm.batch), dim3(P), 0, st, m, cm, q, qd, tau, qdd, o)
    switch (np < 64 ? 64 : np) {
        case 64: CALL(64); break;
        case 128: CALL(128); break;
        case 256: CALL(256); break;
        default: return hipErrorInvalidValue;
    }
#undef CALL
    return hipGetLastError();
}

template hipError_t launch_abia_scan<double>(int, const ModelView<double>&, const ChainMap&, const double*,
                                             const double*, const double*, double*, const FdOut<double>&,
                                             hipStream_t);
template hipError_t launch_abia_scan<float>(int, const ModelView<float>&, const ChainMap&, const float*,
                                            const float*, const float*, float*, const FdOut<float>&, hipStream_t);

}  // namespace fdk
