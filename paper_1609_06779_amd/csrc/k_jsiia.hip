// k_jsiia.hip -- joint space inertia inversion algorithm (Sec. II-C), one lane per link.
//
// tau_delta = tau - ID(q, qd, 0) by the scans; the columns of M are the
// unit-acceleration inverse dynamics (qdd = e_k, qd = 0, no gravity), built
// from one suffix scan of base-frame inertias; then qdd = M^-1 tau_delta.
//
// The inversion (the paper does not fix the method) is Gauss-Jordan
// elimination of [M | tau_delta] without pivoting (M is SPD, so every pivot is
// positive): step j removes column j from every other row, after which
// qdd_i = b_i / m_ii. The trailing block stays symmetric, so the pivot row is
// the pivot column and one LDS column write per step broadcasts it. Chains of
// up to 32 links keep one row of M per lane in registers (several chains per
// wavefront); chains of up to 64 and 128 links spread M over an 8 x 8 or
// 16 x 16 grid of lanes, 64 entries per lane.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "rnea.h"

namespace fdk {

// Gauss-Jordan on register rows (NP <= 64: one wavefront holds 64 / NP chains).
// TREE: branched robots numbered depth-first; M_ik is zero for links on
// different branches (neither is an ancestor of the other).
template <typename T, int NP, bool TREE>
__global__ __launch_bounds__(64) void k_jsiia_gj(ModelView<T> m, ChainMap cm, const T* __restrict__ q,
                                                  const T* __restrict__ qd, const T* __restrict__ tau,
                                                  T* __restrict__ qdd, int* __restrict__ status, FdOut<T> o) {
    static_assert(NP <= 64, "register rows need NP <= 64");
    constexpr int CH = Geo<NP>::chains;
    __shared__ T sf[CH * NP * 12];
    __shared__ T col[2][CH][2 * NP];   // double-buffered pivot column and right-hand sides
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int b = blockIdx.x * CH + grp;
    ChainInfo ci{0, 0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    const int n = ci.n;
    const bool active = li < n;
    const int64_t st = ci.state0 + li;
    const int64_t link = ci.link0 + li;
    T qi = active ? q[st] : T(0), qdi = active && !o.solve ? qd[st] : T(0), ti = active ? tau[st] : T(0);

    const int32_t code = TREE && active ? m.tree_il(li, ci.slot) : 0;
    LinkLane<T> k;   // solve mode: zero velocity, no gravity, so the bias is exactly zero
    const T tb = rnea_lane<T, NP, TREE>(m, link, active, qi, qdi, T(0), !o.solve, li, nullptr, k, code);
    T y = active ? ti - tb : T(0);
    T f[6];
    composite_force<T, NP, TREE>(k, active, li, nullptr, f, code);
    T* my = sf + grp * NP * 12;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        my[c * NP + li] = k.s[c];
        my[(6 + c) * NP + li] = f[c];
    }
    // trees: the links coupled to li are its ancestors (bits) and its subtree (below end)
    const uint32_t anc_bits = TREE ? tree_ancestors<NP>(active ? tree_parent(code) : -1, li) : 0u;
    const int end = TREE && active ? tree_end(code) : NP;
    block_sync<64>();
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
        if constexpr (TREE) {
            const bool related = kk <= li ? ((anc_bits >> kk) & 1u) != 0 : kk < end;
            v = related ? v : T(0);
        }
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
        block_sync<64>();
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
    if (active) o.put(qdd, st, b, li, y / diag);
    if (ci.unsolved && qdd) fill_unsolved(qdd, ci.state0, ci.unsolved, li, NP);
    if (active && !ok && status) atomicOr(status, 1);
}


// Unknowns of one row block of L^T x = z (rows t = T .. 0 of the block, last
// first), column by column: lane c of a row group holds z_c, reduced by
// (1 / d_c) m_tc x_t as each later unknown x_t is found; once every later
// unknown is in, z_t is x_t. Every row group runs this solve on the same
// values, so lane t of the wavefront (group 0, column t) holds x_t for all of
// them, and one readlane hands it to every lane without an LDS round trip.
// wrow: the block's published rows (row t at wrow[t * ws], its column c at
// + c), zero on and above the diagonal, so lanes c >= t subtract an exact zero
// and the step needs no select. On return lane c holds x_c.
template <int G, int T, typename R>
__device__ __forceinline__ void block_back_solve(R& zc, const R* wrow, int ws, int c, R rbc) {
    static_assert(T < G && G <= 64, "column t of a group is wavefront lane t");
    if constexpr (T > 0) {
        const R w = wrow[T * ws + c];                 // read before x_t is known
        const R xt = dpp::read<T>(zc);
        zc -= rbc * w * xt;
        block_back_solve<G, T - 1>(zc, wrow, ws, c, rbc);
    }
}

// Chains of up to 64 or 128 links: M spread over a G x G grid of lanes,
// G = NP / 8 (one chain per workgroup: 64 lanes for NP = 64, 256 for
// NP = 128). Lane (r, c) owns the entries (i, k) = (r + G a, c + G b) with
// a >= b, a, b = 0..7 (the lower triangle, 36 entries), and the right-hand
// side of its rows. M is SPD, so symmetric elimination without pivoting
// (M = L D L^T) is stable:
//  * step j: the lanes of column group j % G publish column j (rows >= j)
//    through LDS; every lane reads its row multipliers m_ij / m_jj and the
//    column entries m_kj of its columns and updates m_ik -= m_ij m_kj / m_jj
//    for i >= k > j, and b_i -= (m_ij / m_jj) b_j (forward substitution);
//    column j then holds D and L (L_ij = m_ij / m_jj);
//  * back substitution L^T x = D^-1 b by blocks of G rows (below).
// Blocks outside the trailing part are skipped at compile time. The inverse
// dynamics before it runs lane per link on all TH = G * G lanes.
template <typename T, int NP, bool TREE>
__global__ __launch_bounds__((NP / 8) * (NP / 8)) void k_jsiia_ldl(ModelView<T> m, ChainMap cm,
                                                                    const T* __restrict__ q,
                                                                    const T* __restrict__ qd,
                                                                    const T* __restrict__ tau, T* __restrict__ qdd,
                                                                    int* __restrict__ status, FdOut<T> o) {
    constexpr int G = NP / 8;
    constexpr int TH = G * G;
    static_assert(TH >= NP, "the lane grid must cover one lane per link");
    __shared__ T xbuf[TH > 64 ? 10 * TH : 1];   // cross-wavefront scan exchange
    constexpr int SF = TREE ? 14 : 13;
    __shared__ T sf[NP * SF];                   // s (6), F (6), tau_delta, subtree end (trees) per link
    __shared__ T col[2][NP + 2];                // column j (zero at rows <= j), b_j, m_jj
    const int li = threadIdx.x;
    ChainInfo ci{0, 0, 0, 0, 0};
    if ((int)blockIdx.x < cm.batch) ci = chain_info(m, cm, blockIdx.x);
    const int n = ci.n;
    const bool active = li < n;
    const int64_t st = ci.state0 + li;
    T qi = active ? q[st] : T(0), qdi = active && !o.solve ? qd[st] : T(0), ti = active ? tau[st] : T(0);

    const int32_t code = TREE && active ? m.tree_il(li, ci.slot) : 0;
    LinkLane<T> k;   // solve mode: zero velocity, no gravity, so the bias is exactly zero
    const T tb = rnea_lane<T, TH, TREE>(m, ci.link0 + li, active, qi, qdi, T(0), !o.solve, li, xbuf, k, code);
    T f6[6];
    composite_force<T, TH, TREE>(k, active, li, xbuf, f6, code);
    if (li < NP) {
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            sf[e * NP + li] = k.s[e];
            sf[(6 + e) * NP + li] = f6[e];
        }
        sf[12 * NP + li] = active ? ti - tb : T(0);
        if constexpr (TREE) sf[13 * NP + li] = T(tree_end(code));
    }
    block_sync<TH>();

    const int r = li / G, c = li % G;
    // Chains of more than 128 links (G = 32, 1024 threads, 4 waves per SIMD)
    // keep the register file for M: the pivot reciprocals go to LDS and the row
    // multipliers are formed as they are used.
    constexpr bool LEAN = NP > 128;
    __shared__ T rdbuf[LEAN ? NP : 1];
    // lower blocks a >= b, packed: index a (a + 1) / 2 + b
    T mb[36], y[8], rd[LEAN ? 1 : 8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int i = r + G * a;
        T fi[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) fi[e] = sf[(6 + e) * NP + i];
        y[a] = sf[12 * NP + i];
#pragma unroll
        for (int bb = 0; bb <= a; ++bb) {
            const int kk = c + G * bb;
            T v = T(0);
#pragma unroll
            for (int e = 0; e < 6; ++e) v += sf[e * NP + kk] * fi[e];   // k <= i: s_k . F_i
            if constexpr (TREE) v = i < int(sf[13 * NP + kk]) ? v : T(0);   // k an ancestor of i
            mb[a * (a + 1) / 2 + bb] = (i < n && kk < n) ? v : (i == kk ? T(1) : T(0));
        }
    }
    bool ok = true;
    // Column block jb is a compile-time index (register arrays stay in
    // registers); the step inside the block, jr, is a run-time value used only
    // in comparisons.
#pragma unroll
    for (int jb = 0; jb < 8; ++jb)
#pragma unroll 1
    for (int jr = 0; jr < G; ++jr) {                       // step j = G jb + jr
        T* cj = col[jr & 1];
        if (c == jr) {
            // entries at rows <= j go out as zero, so readers need no masks
#pragma unroll
            for (int a = jb; a < 8; ++a) {
                const T v = mb[a * (a + 1) / 2 + jb];
                cj[r + G * a] = (a > jb || r > jr) ? v : T(0);
            }
            if (TH > 64 && r == jr) {
                cj[NP] = y[jb];
                cj[NP + 1] = mb[jb * (jb + 1) / 2 + jb];
            }
        }
        // The pivot m_jj and b_j are in lane (jr, jr). In one wavefront a
        // readlane takes them there, so the reciprocal overlaps the column's
        // LDS round trip; larger grids read them from LDS with the column.
        T piv, yj;
        if constexpr (TH == 64) {
            piv = dpp::read_at(mb[jb * (jb + 1) / 2 + jb], (G + 1) * jr);
            yj = dpp::read_at(y[jb], (G + 1) * jr);
        }
        block_sync<TH>();
        if constexpr (TH > 64) {
            piv = cj[NP + 1];
            yj = cj[NP];
        }
        const T rp = rcp_refined(piv);
        if (r == jr) {
            if constexpr (LEAN) {
                if (c == jr) rdbuf[G * jb + jr] = rp;
            } else {
                rd[jb] = rp;
            }
            ok = ok && piv > T(0);
        }
        T pv[8];
#pragma unroll
        for (int a = jb; a < 8; ++a) pv[a] = cj[c + G * a];   // m_kj, zero at columns <= j
#pragma unroll
        for (int a = jb; a < 8; ++a) {
            const T fa = cj[r + G * a] * rp;                   // L_ij, zero at rows <= j
#pragma unroll
            for (int bb = jb; bb <= a; ++bb) mb[a * (a + 1) / 2 + bb] -= fa * pv[bb];
            y[a] -= fa * yj;
        }
    }
    if constexpr (LEAN) block_sync<TH>();                  // the last pivot reciprocals are in LDS
    // Back substitution L^T x = D^-1 b in blocks of G rows, last block first.
    // Row block jb is published once (entries m_jk, k <= j, and the block's
    // z = D^-1 b and 1 / d). Lane (r, c) then carries x of the block's row c:
    // the block's unknowns come column by column (block_back_solve), and each
    // correction of a row above the block is a sum over the block's rows, one
    // term per lane of a row group (G consecutive lanes), summed by
    // dpp::group_sum. The buffer reuses LDS that is free after the M build.
    constexpr int WS = NP + 1;                              // row stride: one extra entry spreads the rows over the LDS banks
    T* wbuf = TH > 64 ? xbuf : sf;                          // G rows of WS entries, then z (G), 1/d (G)
    static_assert((TH > 64 ? 10 * TH : NP * 13) >= G * WS + 2 * G, "block rows fit the reused buffer");
    T* zb = wbuf + G * WS;
    T* rb = zb + G;
    auto rd_of = [&](int a) -> T {                          // 1 / d of row r + G a
        if constexpr (LEAN) return rdbuf[r + G * a];
        else return rd[a];
    };
#pragma unroll
    for (int a = 0; a < 8; ++a) y[a] *= rd_of(a);
#pragma unroll
    for (int jb = 7; jb >= 0; --jb) {
        block_sync<TH>();                                    // earlier reads of the buffer are done
#pragma unroll
        for (int bb = 0; bb <= jb; ++bb)                     // the diagonal block strictly below its diagonal
            wbuf[r * WS + c + G * bb] = (bb < jb || c < r) ? mb[jb * (jb + 1) / 2 + bb] : T(0);
        if (c == 0) {
            zb[r] = y[jb];
            rb[r] = rd_of(jb);
        }
        block_sync<TH>();
        // x_t = z_t - (1 / d_t) sum_{u > t} m_ut x_u within the block; lane c ends with x_c
        T xc = zb[c];
        block_back_solve<G, G - 1>(xc, wbuf + G * jb, WS, c, rb[c]);
        y[jb] = xlane::bperm(xc, 4 * r);                     // x of row r of the block: wavefront lane r has c = r
        // rows k above the block: z_k -= (1 / d_k) sum_t m_tk x_t
#pragma unroll
        for (int a = 0; a < jb; ++a) y[a] -= dpp::group_sum<G>(wbuf[c * WS + r + G * a] * xc) * rd_of(a);
    }
    if (c == 0) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int i = r + G * a;
            if (i < n) o.put(qdd, ci.state0 + i, blockIdx.x, i, y[a]);
        }
    }
    if (ci.unsolved && qdd) fill_unsolved(qdd, ci.state0, ci.unsolved, li, TH);
    if (c == 0 && !ok && status) atomicOr(status, 1);
}

// longest chain the JSIIA kernels take (same for both precisions)
template <typename T> int jsiia_max_np() { return 256; }

template <typename T>
hipError_t launch_jsiia(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd, const T* tau,
                        T* qdd, int* status, const FdOut<T>& o, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
#define GJ(P)                                                                                            \
    if (m.tree)                                                                                          \
        hipLaunchKernelGGL((k_jsiia_gj<T, P, true>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(64), 0, st, m, cm, q, qd, tau, qdd, status, o);                         \
    else                                                                                                 \
        hipLaunchKernelGGL((k_jsiia_gj<T, P, false>), dim3((cm.batch + Geo<P>::chains - 1) / Geo<P>::chains), \
                           dim3(64), 0, st, m, cm, q, qd, tau, qdd, status, o)
#define GJ2D(P)                                                                                          \
    if (m.tree)                                                                                          \
        hipLaunchKernelGGL((k_jsiia_ldl<T, P, true>), dim3(cm.batch), dim3((P / 8) * (P / 8)), 0, st, m, cm, q, \
                           qd, tau, qdd, status, o);                                                     \
    else                                                                                                 \
        hipLaunchKernelGGL((k_jsiia_ldl<T, P, false>), dim3(cm.batch), dim3((P / 8) * (P / 8)), 0, st, m, cm, q, \
                           qd, tau, qdd, status, o)
    switch (np) {
        case 8: GJ(8); break;
        case 16: GJ(16); break;
        case 32: GJ(32); break;
        case 64: GJ2D(64); break;
        case 128: GJ2D(128); break;
        case 256: GJ2D(256); break;
        default: return hipErrorInvalidValue;
    }
#undef GJ
#undef GJ2D
    return hipGetLastError();
}

template hipError_t launch_jsiia<double>(int, const ModelView<double>&, const ChainMap&, const double*, const double*,
                                         const double*, double*, int*, const FdOut<double>&, hipStream_t);
template hipError_t launch_jsiia<float>(int, const ModelView<float>&, const ChainMap&, const float*, const float*,
                                        const float*, float*, int*, const FdOut<float>&, hipStream_t);
template int jsiia_max_np<double>();
template int jsiia_max_np<float>();

}  // namespace fdk
