// k_abia.hip -- articulated-body inertia algorithm (Sec. II-C), one lane per chain.
//
// The articulated-body inertias come from a nonlinear backward recursion that
// cannot be split across processors beyond a constant factor (Sec. III), so a
// whole chain stays on one lane and a wavefront carries 64 chains. Three sweeps:
//  1. forward (base to tip): link velocities and bias accelerations of the
//     inverse dynamics at qdd = 0 (gravity as base acceleration), carried to
//     the tip;
//  2. backward: the same velocities and accelerations walked back from the tip
//     (each step of the forward recursion inverted), the link forces
//     f_i = J_i a_i - ad_{v_i}^T J_i v_i, and the force recursion, which gives
//     tau_delta_i = tau_i - S_i^T F_i; in
//     the same sweep the articulated inertias
//        Jh_i = J_i + Ad_{i+1}^T (Jh_{i+1} - h h^T / D)_{i+1} Ad_{i+1},
//        h_i = Jh_i S_i, D_i = S_i^T h_i,
//     and the first linear (bi-diagonal, (I - X^T)-type) recursion
//        p_i = Ad_{i+1}^T (p_{i+1} + h_{i+1} u_{i+1} / D_{i+1}),  u_i = tau_delta_i - S_i^T p_i;
//  3. forward: the second linear recursion
//        a_i = Ad_i a_{i-1} + S_i qdd_i,  qdd_i = (u_i - h_i^T Ad_i a_{i-1}) / D_i,
// which together apply M^-1 to tau_delta (zero velocity, no gravity).
//
// Branched robots (trees; the paper treats serial chains): sweep 1 keeps every
// link force in the workspace for sweep 2, and link i takes its
// parent p(i)'s velocity and accelerations instead of link i-1's, and hands
// its backward-sweep terms (F, p and Jh - h h^T / D, moved into p(i)'s frame)
// to p(i), where the terms of all children add up. A child whose parent is
// i - 1 still passes them in registers; only branch points go through the
// workspace: in sweep 1 a branch point stores its velocity and bias
// acceleration for its other children, in sweep 2 those children sum their
// terms into its accumulator (the highest-numbered child writes, the others
// add: children are swept before their parent), and in sweep 3 it stores its
// acceleration. The model's tree codes say which case each link is.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "spatial.h"

namespace fdk {

// sweep 2: h / D without its joint-axis entry, which is h_3 / D = 1 (D = h_3),
// so 5 values, then u / D; trees: sweep 1 f (6) first
constexpr int ABIA_WS_FIELDS = 6;
// Trees add a branch-point record after those 6 fields: sweep 1 velocity (6)
// and bias acceleration (6); sweep 2 accumulator of the children's F (6), p (6)
// and Jh - h h^T / D (21, upper triangle by rows); sweep 3 acceleration (6).
constexpr int ABIA_WB = ABIA_WS_FIELDS;
constexpr int ABIA_TREE_WS_FIELDS = ABIA_WS_FIELDS + 33;

template <bool TREE> constexpr int abia_fields() { return TREE ? ABIA_TREE_WS_FIELDS : ABIA_WS_FIELDS; }
// Branch-point records are read back soon after they are written, so they
// keep the default cache policy even when the rest of the workspace streams.
constexpr bool ABIA_BRANCH_NT = false;

size_t abia_workspace_elems(int batch, int nmax, bool tree) {
    size_t blocks = (size_t)(batch + 63) / 64;
    return blocks * (size_t)nmax * (tree ? ABIA_TREE_WS_FIELDS : ABIA_WS_FIELDS) * 64;
}

// Model reads go through the robot-interleaved copy: lanes hold consecutive
// chains, so field f of link i is one contiguous read across the wavefront.
//
// Per-link inputs of a forward sweep, loaded ahead of their use: the home
// pose (quaternion, origin) and the joint state (from the LDS stage); with
// `ws`, sweep 3 also takes the link's 6 workspace values.
template <typename T, bool WS> struct LinkIn {
    T qt[4], p[3], q, qd;
    T w[WS ? ABIA_WS_FIELDS : 1];
};
template <bool NT, bool WS, typename T>
__device__ __forceinline__ LinkIn<T, WS> link_in(const ModelView<T>& m, int i, int slot, T qv, T qdv, const T* wsi) {
    LinkIn<T, WS> r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.qt[k] = m.template at_il<NT>(IL_QUAT + k, i, slot);
#pragma unroll
    for (int k = 0; k < 3; ++k) r.p[k] = m.template at_il<NT>(IL_POS + k, i, slot);
    r.q = qv;
    r.qd = qdv;
    if constexpr (WS) {
#pragma unroll
        for (int f = 0; f < ABIA_WS_FIELDS; ++f) r.w[f] = ld_ws<NT>(wsi + (size_t)f * 64);
    }
    return r;
}
template <typename T, bool WS> __device__ __forceinline__ Pose<T> link_in_pose(const LinkIn<T, WS>& r) {
    T rh[9];
    quat_to_rot(r.qt, rh);
    return joint_pose(rh, r.p, r.q);
}

// wrench_to_parent for a wrench whose component 2 (the joint axis of the
// child's canonical frame) is zero: y = X f with X = [[R, [p] R], [0, R]].
template <typename T> __device__ __forceinline__ void wrench_to_parent_z2(const Pose<T>& t, const T f[6], T y[6]) {
    T rn[3], rf[3], pc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) rn[i] = t.r[3 * i] * f[0] + t.r[3 * i + 1] * f[1];
    matvec3(t.r, f + 3, rf);
    cross3(t.p, rf, pc);
    y[0] = rn[0] + pc[0]; y[1] = rn[1] + pc[1]; y[2] = rn[2] + pc[2];
    y[3] = rf[0]; y[4] = rf[1]; y[5] = rf[2];
}

// Y = X P X^T (X = Ad(T^-1)^T, moving the child's terms to the parent's
// frame) for a symmetric P whose row and column 2 are zero: the articulated
// inertia less the joint's share, P = Jh - h h^T / D with h = Jh e3, D = h_2,
// has P e3 = 0. Columns of X P are X applied to the columns of P (column 2 is
// zero), then row r of Y is X applied to row r of X P. Only the lower
// triangle of Y is formed (the rest of each row is left to dead-code
// elimination) and mirrored.
template <typename T> __device__ __forceinline__ void congruence_to_parent(const Pose<T>& t, const T p[36], T y[36]) {
    T w[36];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (c == 2) {
#pragma unroll
            for (int r = 0; r < 6; ++r) w[6 * r + 2] = T(0);
            continue;
        }
        T col[6], out[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) col[r] = r == 2 ? T(0) : p[6 * r + c];
        wrench_to_parent_z2(t, col, out);
#pragma unroll
        for (int r = 0; r < 6; ++r) w[6 * r + c] = out[r];
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        T out[6];
        wrench_to_parent_z2(t, w + 6 * r, out);
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            y[6 * r + c] = out[c];
            y[6 * c + r] = out[c];
        }
    }
}

// LDS of one wavefront for the state stage: the largest stage (sweep 2: q,
// qd, tau; 2 slots) also holds sweep 3's q slots and its output tile.
constexpr int ABIA_STAGE = 2 * 3 * ST_L * ST_W;
static_assert(2 * 1 * ST_L * ST_W + ST_L * ST_W <= ABIA_STAGE, "sweep 3's stage and output tile fit");

// Launches of serial chains with at least ABIA_STAGE_CHAINS chains, the
// longest of at least 16 (FP64) or 32 (FP32) links, move the joint state
// through the LDS stage; smaller launches and trees read and write it lane by
// lane. Measured on MI355X: the stage takes 65536 x 64 FP64 from 0.422 to
// 0.332 ms and 65536 x 16 from 0.091 to 0.074 ms, but costs one robot or a few
// hundred wavefronts a fifth more time, the divergent tree sweeps a third,
// and FP32 chains of 16 links a tenth (32 links break even). Plain and
// persistent launches of one batch take the same path, so their results stay
// equal bit for bit.
constexpr int ABIA_STAGE_CHAINS = 65536;
template <typename T> bool abia_stages(bool tree, int batch, int nmax) {
    return !tree && batch >= ABIA_STAGE_CHAINS && nmax >= (sizeof(T) == 8 ? 16 : 32);
}

// One chain (or tree) on one lane; every lane of the wavefront calls it (a
// lane without a chain with ci.n = 0), since with ST the state stage is
// loaded by all of them. wsb: this lane's workspace column, field f of link i at
// wsb[(i * abia_fields<TREE>() + f) * 64]. NT: model and workspace streamed
// with non-temporal accesses (see ModelView::at_il). stg, sbase, slen: the
// wavefront's LDS (ABIA_STAGE values, 64 + 64 entries).
template <bool NT, bool TREE, bool ST, typename T>
__device__ __forceinline__ void abia_chain(const ModelView<T>& m, ChainInfo ci, const T* __restrict__ q,
                                           const T* __restrict__ qd, const T* __restrict__ tau,
                                           T* __restrict__ qdd, T* __restrict__ wsb, int b, const FdOut<T>& o,
                                           T* stg, int64_t* sbase, int* slen) {
    if (ci.unsolved) {                                 // longer than the workspace is sized for
        if (qdd) fill_unsolved(qdd, ci.state0, ci.unsolved, 0, 1);
        ci.n = 0;
    }
    const int n = ci.n;
    const int lane = threadIdx.x & 63;
    auto wsp = [&](int i, int f) -> T* { return &wsb[((size_t)i * abia_fields<TREE>() + f) * 64]; };
    static_assert(!(ST && TREE), "trees read the state lane by lane");
    int nw = n;                                        // loop bound: each lane's own length, or with the
    if constexpr (ST) nw = stage_chains(sbase, slen, ci.state0, n, lane);   // stage the longest in the wavefront
    // state entry of array a at link i, read directly (trees)
    auto at = [&](const T* a, int i) -> T { return a[ci.state0 + i]; };

    // sweep 1. The light forward sweeps wait on memory, not on arithmetic: each
    // step starts the loads of the link two ahead, so two links' inputs are in
    // flight while one is computed.
    T v[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T a[6] = {T(0), T(0), T(0), -m.g[0], -m.g[1], -m.g[2]};
    StateStage<T, 2> s1{stg, sbase, slen, lane};
    const T* const st1[2] = {q, qd};
    if constexpr (ST) {
        s1.template start<true>(st1);
        block_sync<64>();
    }
    auto in1_of = [&](int i) -> LinkIn<T, false> {    // link i's inputs
        if constexpr (ST) return link_in<NT, false>(m, i, ci.slot, s1.get(0, i), s1.get(1, i), wsb);
        else return link_in<NT, false>(m, i, ci.slot, at(q, i), at(qd, i), wsb);
    };
    LinkIn<T, false> in0, in1;
    if (n > 0) in0 = in1_of(0);
    if (n > 1) in1 = in1_of(1);
    for (int i = 0; i < nw; ++i) {
        if constexpr (ST) {
            s1.template step<true>(st1, i);
            if (i >= n) continue;
        }
        const LinkIn<T, false> cur = in0;
        in0 = in1;
        if (i + 2 < n) in1 = in1_of(i + 2);
        int32_t code = 0;
        if constexpr (TREE) {
            code = m.template tree_il<NT>(i, ci.slot);
            if (!(code & TREE_CHAIN)) {                // the parent's terms, not link i-1's
                const int p = tree_parent(code);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    v[c] = p < 0 ? T(0) : ld_ws<NT && ABIA_BRANCH_NT>(wsp(p, ABIA_WB + c));
                    a[c] = p < 0 ? (c < 3 ? T(0) : -m.g[c - 3]) : ld_ws<NT && ABIA_BRANCH_NT>(wsp(p, ABIA_WB + 6 + c));
                }
            }
        }
        const Pose<T> tl = link_in_pose(cur);
        const T qdi = cur.qd;
        T t[6];
        ad_inv_apply(tl, v, t);
        t[2] += qdi;
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = t[c];
        ad_inv_apply(tl, a, t);
        // + ad_{V_i}(S qd) = (w x e3 qd; v x e3 qd)
        t[0] += v[1] * qdi; t[1] -= v[0] * qdi;
        t[3] += v[4] * qdi; t[4] -= v[3] * qdi;
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] = t[c];
        if constexpr (TREE) {
            // trees keep every link force: the backward sweep cannot walk the
            // twists back from one tip past a branch point
            T f[6];
            link_force(m.template inertia_il<NT>(i, ci.slot), v, a, f);
#pragma unroll
            for (int c = 0; c < 6; ++c) st_ws<NT>(f[c], wsp(i, c));
            if (code & TREE_BRANCH) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    st_ws<NT && ABIA_BRANCH_NT>(v[c], wsp(i, ABIA_WB + c));
                    st_ws<NT && ABIA_BRANCH_NT>(a[c], wsp(i, ABIA_WB + 6 + c));
                }
            }
        }
    }

    // sweep 2
    // link i+1's terms for link i; trees hold them already moved into frame i
    T fc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // F_{i+1} (frame i+1)
    T pc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // p_{i+1} + h_{i+1} u_{i+1} / D_{i+1} (frame i+1)
    T pi[36];                                          // Jh_{i+1} - h h^T / D (frame i+1)
#pragma unroll
    for (int c = 0; c < 36; ++c) pi[c] = T(0);
    Pose<T> tn = pose_identity<T>();                   // T_{i,i+1}
    T qdn = T(0);                                      // chains: qd_{i+1}
    bool carry = false;                                // trees: registers hold link i+1's terms for link i
    // each step starts the loads of the link before it (the step's arithmetic
    // outlasts a memory round trip)
    // the state stage runs backward here: position k is link n - 1 - k
    StateStage<T, 3> s2{stg, sbase, slen, lane};
    const T* const st2[3] = {q, qd, tau};
    if constexpr (ST) {
        block_sync<64>();                              // sweep 1's reads of the stage are done
        s2.template start<false>(st2);
        block_sync<64>();
    }
    auto in2_of = [&](int k) -> LinkIn<T, false> {    // inputs of the link at position k
        if constexpr (ST) return link_in<NT, false>(m, n - 1 - k, ci.slot, s2.get(0, k), s2.get(1, k), wsb);
        else return link_in<NT, false>(m, n - 1 - k, ci.slot, at(q, n - 1 - k), at(qd, n - 1 - k), wsb);
    };
    auto tau_of = [&](int k) -> T {
        if constexpr (ST) return s2.get(2, k);
        else return at(tau, n - 1 - k);
    };
    Inertia<T> jn;
    LinkIn<T, false> pn;
    T taun = T(0);
    if (n > 0) {
        jn = m.template inertia_il<NT>(n - 1, ci.slot);
        pn = in2_of(0);
        taun = tau_of(0);
    }
    for (int k = 0; k < nw; ++k) {
        if constexpr (ST) {
            s2.template step<false>(st2, k);
            if (k >= n) continue;
        }
        const int i = n - 1 - k;
        T f[6], fp[6], pp[6], jh[36];
        const Inertia<T> ji = jn;
        const LinkIn<T, false> pcur = pn;
        const T taui = taun;
        if (i > 0) {
            jn = m.template inertia_il<NT>(i - 1, ci.slot);
            pn = in2_of(k + 1);
            taun = tau_of(k + 1);
        }
        if constexpr (TREE) {
#pragma unroll
            for (int c = 0; c < 6; ++c) f[c] = ld_ws<NT>(wsp(i, c));
        } else {
            // Serial chains: sweep 1 left the tip's twist and bias acceleration
            // in (v, a); walk them back one link at a time, inverting its
            // recursions: V_i = Ad_{T_{i,i+1}} (V_{i+1} - S qd_{i+1}),
            // a_i = Ad_{T_{i,i+1}} (a_{i+1} - ad_{V_{i+1}} (S qd_{i+1})).
            // The link force then needs no round trip through memory.
            if (i + 1 < n) {
                T t[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) t[c] = a[c];
                t[0] -= v[1] * qdn; t[1] += v[0] * qdn;
                t[3] -= v[4] * qdn; t[4] += v[3] * qdn;
                ad_apply(tn, t, a);
#pragma unroll
                for (int c = 0; c < 6; ++c) t[c] = v[c];
                t[2] -= qdn;
                ad_apply(tn, t, v);
            }
            link_force(ji, v, a, f);
        }
        inertia_to_mat6(ji, jh);
        const int32_t code = TREE ? m.template tree_il<NT>(i, ci.slot) : 0;
        if (TREE && carry) {                           // terms already in this link's frame
#pragma unroll
            for (int c = 0; c < 36; ++c) jh[c] += pi[c];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                f[c] += fc[c];
                pp[c] = pc[c];
            }
        } else if (!TREE && i + 1 < n) {
            wrench_to_parent(tn, fc, fp);
            wrench_to_parent(tn, pc, pp);
            T y[36];
            congruence_to_parent(tn, pi, y);
#pragma unroll
            for (int c = 0; c < 36; ++c) jh[c] += y[c];
#pragma unroll
            for (int c = 0; c < 6; ++c) f[c] += fp[c];
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) pp[c] = T(0);
        }
        if constexpr (TREE) {
            if (code & TREE_BRANCH) {                  // the other children's terms, summed
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    f[c] += ld_ws<NT && ABIA_BRANCH_NT>(wsp(i, ABIA_WB + c));
                    pp[c] += ld_ws<NT && ABIA_BRANCH_NT>(wsp(i, ABIA_WB + 6 + c));
                }
                int k = ABIA_WB + 12;
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = r; c < 6; ++c, ++k) {
                        const T y = ld_ws<NT && ABIA_BRANCH_NT>(wsp(i, k));
                        jh[6 * r + c] += y;
                        if (c != r) jh[6 * c + r] += y;
                    }
            }
        }
        const T td = taui - f[2];
        const T dinv = rcp_refined(jh[14]);
        const T u = td - pp[2];
        T h[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = jh[6 * c + 2];
        T hd[6];                                        // h / D
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            hd[c] = h[c] * dinv;
            if (c != 2) st_ws<NT>(hd[c], wsp(i, c < 2 ? c : c - 1));
        }
        st_ws<NT>(u * dinv, wsp(i, 5));
        // Pi = Jh - h h^T / D, symmetric, with row and column 2 exactly zero
        // (they are zero in exact arithmetic: Pi e3 = h - h D / D)
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                const T x = (r == 2 || c == 2) ? T(0) : jh[6 * r + c] - h[r] * hd[c];
                pi[6 * r + c] = x;
                pi[6 * c + r] = x;
            }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            pc[c] = pp[c] + hd[c] * u;
            fc[c] = f[c];
        }
        tn = link_in_pose(pcur);
        if constexpr (!TREE) qdn = pcur.qd;
        if constexpr (TREE) {
            // Move the terms into the parent's frame here, once per link, on
            // every lane: the parent takes them from registers (chain step) or
            // from its record, and only the record update diverges.
            T x[6], y[36];
            wrench_to_parent(tn, fc, x);
#pragma unroll
            for (int c = 0; c < 6; ++c) fc[c] = x[c];
            wrench_to_parent(tn, pc, x);
#pragma unroll
            for (int c = 0; c < 6; ++c) pc[c] = x[c];
            congruence_to_parent(tn, pi, y);
#pragma unroll
            for (int c = 0; c < 36; ++c) pi[c] = y[c];
            carry = (code & TREE_CHAIN) != 0;
            const int p = tree_parent(code);
            if (!carry && p >= 0) {                    // hand the terms to a branch point now
                const bool first = (code & TREE_FIRST) != 0;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    T* d = wsp(p, ABIA_WB + c);
                    st_ws<NT && ABIA_BRANCH_NT>(first ? fc[c] : fc[c] + ld_ws<NT && ABIA_BRANCH_NT>(d), d);
                    d = wsp(p, ABIA_WB + 6 + c);
                    st_ws<NT && ABIA_BRANCH_NT>(first ? pc[c] : pc[c] + ld_ws<NT && ABIA_BRANCH_NT>(d), d);
                }
                int k = ABIA_WB + 12;
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = r; c < 6; ++c, ++k) {
                        T* d = wsp(p, k);
                        st_ws<NT && ABIA_BRANCH_NT>(first ? pi[6 * r + c] : pi[6 * r + c] + ld_ws<NT && ABIA_BRANCH_NT>(d), d);
                    }
            }
        }
    }

    // sweep 3, with the loads of the link two ahead started at each step
    T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    StateStage<T, 1> s3{stg, sbase, slen, lane};
    const T* const st3[1] = {q};
    OutTile<T, 1> o3{stg + 2 * ST_L * ST_W, sbase, slen, lane};   // qdd of the current tile
    T* const out3[1] = {qdd};
    if constexpr (ST) {
        block_sync<64>();                              // sweep 2's reads of the stage are done
        s3.template start<true>(st3);
        block_sync<64>();
    }
    auto in3_of = [&](int i) -> LinkIn<T, true> {
        if constexpr (ST) return link_in<NT, true>(m, i, ci.slot, s3.get(0, i), T(0), wsp(i, 0));
        else return link_in<NT, true>(m, i, ci.slot, at(q, i), T(0), wsp(i, 0));
    };
    LinkIn<T, true> wn0, wn1;
    if (n > 0) wn0 = in3_of(0);
    if (n > 1) wn1 = in3_of(1);
    for (int i = 0; i < nw; ++i) {
        if constexpr (ST) s3.template step<true>(st3, i);
        if (i < n) {
        const LinkIn<T, true> cur = wn0;
        wn0 = wn1;
        if (i + 2 < n) wn1 = in3_of(i + 2);
        int32_t code = 0;
        if constexpr (TREE) {
            code = m.template tree_il<NT>(i, ci.slot);
            if (!(code & TREE_CHAIN)) {
                const int p = tree_parent(code);
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] = p < 0 ? T(0) : ld_ws<NT && ABIA_BRANCH_NT>(wsp(p, ABIA_WB + c));
            }
        }
        const Pose<T> tl = link_in_pose(cur);
        T t[6];
        ad_inv_apply(tl, acc, t);
        // qdd = u/D - (h/D)^T t with (h/D)_3 = 1: the new axis component of the
        // acceleration, t_3 + qdd, is s below, and qdd = s - t_3
        T s = cur.w[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) s -= cur.w[c] * t[c < 2 ? c : c + 1];
        const T x = s - t[2];
        t[2] = s;
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] = t[c];
        if constexpr (ST) {
            o3.put(0, i, x);
            o.put_aux(b, i, x);                        // qdd may be null when the reverse mode takes it in aux
        } else {
            o.put(qdd, ci.state0 + i, b, i, x);
        }
        if constexpr (TREE) {
            if (code & TREE_BRANCH) {
#pragma unroll
                for (int c = 0; c < 6; ++c) st_ws<NT && ABIA_BRANCH_NT>(acc[c], wsp(i, ABIA_WB + c));
            }
        }
        }
        if constexpr (ST) o3.template flush<true>(out3, i, nw, o.accumulate);
    }
}

template <typename T, bool NT, bool TREE, bool ST>
__global__ __launch_bounds__(64) void k_abia(ModelView<T> m, ChainMap cm, int nmax, const T* __restrict__ q,
                                             const T* __restrict__ qd, const T* __restrict__ tau,
                                             T* __restrict__ qdd, T* __restrict__ ws, FdOut<T> o) {
    __shared__ T stg[ST ? ABIA_STAGE : 1];             // the state stage
    __shared__ int64_t sbase[ST ? 64 : 1];
    __shared__ int slen[ST ? 64 : 1];
    const int lane = threadIdx.x;
    const int b = blockIdx.x * 64 + lane;
    ChainInfo ci{0, 0, 0, 0, 0};                      // lanes past the batch take part with no chain
    if (b < cm.batch) ci = chain_info(m, cm, b);
    // workspace: [block][link][field][lane]
    abia_chain<NT, TREE, ST>(m, ci, q, qd, tau, qdd,
                             ws + (size_t)blockIdx.x * nmax * abia_fields<TREE>() * 64 + lane, b, o, stg, sbase,
                             slen);
}

// Persistent form for ragged batches: each wavefront takes 64-entry tiles of
// `order` (count entries; order == nullptr: the identity) from an atomic
// counter until the list is exhausted, so lanes of a tile have nearly equal
// lengths and the longest tiles go first. Entries at or past the batch are
// skipped. Every wavefront leaves once a tile index runs past the list, so
// the grid always drains.
template <typename T, bool NT, bool TREE, bool ST>
__global__ __launch_bounds__(64) void k_abia_persistent(ModelView<T> m, ChainMap cm, int nmax,
                                                        const int32_t* __restrict__ order, int32_t count,
                                                        int32_t* counter, const T* __restrict__ q,
                                                        const T* __restrict__ qd, const T* __restrict__ tau,
                                                        T* __restrict__ qdd, T* __restrict__ ws) {
    __shared__ int tile_s;
    __shared__ T stg[ST ? ABIA_STAGE : 1];             // the state stage
    __shared__ int64_t sbase[ST ? 64 : 1];
    __shared__ int slen[ST ? 64 : 1];
    const int lane = threadIdx.x;
    T* wsb = ws + (size_t)blockIdx.x * nmax * abia_fields<TREE>() * 64 + lane;
    for (;;) {
        if (lane == 0) tile_s = atomicAdd(counter, 1);
        __syncthreads();
        const int tile = tile_s;
        __syncthreads();
        if ((int64_t)tile * 64 >= count) break;
        const int k = tile * 64 + lane;
        const int b = k < count ? (order ? order[k] : k) : cm.batch;
        ChainInfo ci{0, 0, 0, 0, 0};                  // entries past the batch: no chain, but the lane takes part
        if (b < cm.batch) ci = chain_info(m, cm, b);
        abia_chain<NT, TREE, ST>(m, ci, q, qd, tau, qdd, wsb, b, FdOut<T>{}, stg, sbase, slen);
    }
}

// ---- planning kernels: counting sort of the batch by decreasing chain length ----
// bins / cursor: int32[KMAX_LINKS + 2]; bins[n] counts chains of n links (n = 0:
// chains with an out-of-range robot id, placed last).
constexpr int PLAN_BINS = 258;

__global__ void k_plan_zero(int32_t* bins, int32_t* cursor, int32_t* counter) {
    int t = threadIdx.x;
    for (int k = t; k < PLAN_BINS; k += blockDim.x) {
        bins[k] = 0;
        cursor[k] = 0;
    }
    if (t == 0) *counter = 0;
}

template <typename T>
__global__ void k_plan_hist(ModelView<T> m, ChainMap cm, int32_t* bins) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cm.batch) return;
    int n = chain_info(m, cm, b).n;
    atomicAdd(&bins[n < PLAN_BINS ? n : 0], 1);
}

// cursor[n] = number of chains longer than n (decreasing order); chains of
// length 0 go after all others. One block.
__global__ void k_plan_scan(const int32_t* bins, int32_t* cursor) {
    if (threadIdx.x != 0) return;
    int acc = 0;
    for (int n = PLAN_BINS - 1; n >= 1; --n) {
        cursor[n] = acc;
        acc += bins[n];
    }
    cursor[0] = acc;
}

template <typename T>
__global__ void k_plan_scatter(ModelView<T> m, ChainMap cm, int32_t* cursor, int32_t* order) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cm.batch) return;
    int n = chain_info(m, cm, b).n;
    int pos = atomicAdd(&cursor[n < PLAN_BINS ? n : 0], 1);
    order[pos] = b;
}

size_t persistent_plan_bytes(int batch) {
    return sizeof(int32_t) * ((size_t)batch + 2 * PLAN_BINS + 64);
}

size_t abia_persistent_workspace_elems(int grid, int nmax, bool tree) {
    return (size_t)grid * nmax * (tree ? ABIA_TREE_WS_FIELDS : ABIA_WS_FIELDS) * 64;
}

// Three orders: with robot ids, the planning kernels sort the batch's chains
// by decreasing length on the device; without, chain b is robot b, whose
// interleaved column already follows that order (slot_robot[c] = robot of
// column c), so the tiles walk the columns; a one-robot model is uniform and
// the tiles walk the chains.
template <typename T>
hipError_t launch_abia_persistent(const ModelView<T>& m, const ChainMap& cm, int nmax, int grid, const T* q,
                                  const T* qd, const T* tau, T* qdd, T* ws, int32_t* plan,
                                  const int32_t* slot_robot, bool stream_model, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
    int32_t* bins = plan;
    int32_t* cursor = bins + PLAN_BINS;
    int32_t* counter = cursor + PLAN_BINS;
    int32_t* order = counter + 64;
    hipLaunchKernelGGL(k_plan_zero, dim3(1), dim3(256), 0, st, bins, cursor, counter);
    const int32_t* tiles = nullptr;
    int32_t count = cm.batch;
    if (cm.robot_id) {
        const unsigned g = (unsigned)((cm.batch + 255) / 256);
        hipLaunchKernelGGL((k_plan_hist<T>), dim3(g), dim3(256), 0, st, m, cm, bins);
        hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(64), 0, st, bins, cursor);
        hipLaunchKernelGGL((k_plan_scatter<T>), dim3(g), dim3(256), 0, st, m, cm, cursor, order);
        tiles = order;
    } else if (m.num_robots > 1) {
        tiles = slot_robot;
        count = m.num_robots;
    }
#define FDK_ABIA_PERSISTENT(NT, TREE, ST)                                                                   \
    hipLaunchKernelGGL((k_abia_persistent<T, NT, TREE, ST>), dim3(grid), dim3(64), 0, st, m, cm, nmax, tiles, \
                       count, counter, q, qd, tau, qdd, ws)
    if (m.tree) {
        if (stream_model) FDK_ABIA_PERSISTENT(true, true, false);
        else FDK_ABIA_PERSISTENT(false, true, false);
    } else if (abia_stages<T>(false, cm.batch, nmax)) {
        if (stream_model) FDK_ABIA_PERSISTENT(true, false, true);
        else FDK_ABIA_PERSISTENT(false, false, true);
    } else {
        if (stream_model) FDK_ABIA_PERSISTENT(true, false, false);
        else FDK_ABIA_PERSISTENT(false, false, false);
    }
#undef FDK_ABIA_PERSISTENT
    return hipGetLastError();
}

template <typename T>
hipError_t launch_abia(const ModelView<T>& m, const ChainMap& cm, int nmax, const T* q, const T* qd, const T* tau,
                       T* qdd, T* ws, bool stream_model, const FdOut<T>& o, hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
    const dim3 grid((cm.batch + 63) / 64);
#define FDK_ABIA(NT, TREE, ST) \
    hipLaunchKernelGGL((k_abia<T, NT, TREE, ST>), grid, dim3(64), 0, st, m, cm, nmax, q, qd, tau, qdd, ws, o)
    if (m.tree) {
        if (stream_model) FDK_ABIA(true, true, false);
        else FDK_ABIA(false, true, false);
    } else if (abia_stages<T>(false, cm.batch, nmax)) {
        if (stream_model) FDK_ABIA(true, false, true);
        else FDK_ABIA(false, false, true);
    } else {
        if (stream_model) FDK_ABIA(true, false, false);
        else FDK_ABIA(false, false, false);
    }
#undef FDK_ABIA
    return hipGetLastError();
}

template hipError_t launch_abia<double>(const ModelView<double>&, const ChainMap&, int, const double*, const double*,
                                        const double*, double*, double*, bool, const FdOut<double>&, hipStream_t);
template hipError_t launch_abia<float>(const ModelView<float>&, const ChainMap&, int, const float*, const float*,
                                       const float*, float*, float*, bool, const FdOut<float>&, hipStream_t);
template hipError_t launch_abia_persistent<double>(const ModelView<double>&, const ChainMap&, int, int, const double*,
                                                   const double*, const double*, double*, double*, int32_t*,
                                                   const int32_t*, bool, hipStream_t);
template hipError_t launch_abia_persistent<float>(const ModelView<float>&, const ChainMap&, int, int, const float*,
                                                  const float*, const float*, float*, float*, int32_t*,
                                                  const int32_t*, bool, hipStream_t);

}  // namespace fdk
