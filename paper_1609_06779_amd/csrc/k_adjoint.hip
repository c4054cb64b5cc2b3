// k_adjoint.hip -- reverse-mode derivative (vector-Jacobian product) of forward
// dynamics, and the semi-implicit Euler step of a rollout with its adjoint.
//
// qdd = FD(q, qd, tau) solves ID(q, qd, qdd) = tau (eq. (eq-motion), (tau-bias)),
// so for a cotangent g of qdd the implicit-function theorem gives
//     lambda = M^-1 g,   tau_bar = lambda,
//     [q_bar; qd_bar] = -(d ID / d(q, qd))^T lambda   at qdd = FD(q, qd, tau).
// lambda comes from the articulated-body factorisation of M^-1 (Sec. II-C),
// applied to g with zero velocity and no gravity. (d ID / d(q, qd))^T lambda is
// the reverse of the inverse-dynamics recursions of eq. (EOM-full): with
// A_i = Ad(T_{i-1,i}^-1) and S = e3 in the canonical joint frames,
//   forward  (recomputed): V_i = A_i V_{i-1} + S qd_i,
//                          a_i = A_i a_{i-1} + S qdd_i + ad_{V_i}(S qd_i),
//                          f_i = J_i a_i - ad_{V_i}^T J_i V_i,
//   backward (recomputed): F_i = f_i + A_{i+1}^T F_{i+1},  tau_i = S^T F_i;
//   adjoint, forward in i: Fb_i = lambda_i S + A_i Fb_{i-1}   (Fb = force adjoint),
//   adjoint, backward in i:
//     ab_i = J_i Fb_i + A_{i+1}^T ab_{i+1}
//     Vb_i = ad_{Fb_i}^T (J_i V_i) - J_i ad_{V_i} Fb_i - ad_{S qd_i}^T ab_i + A_{i+1}^T Vb_{i+1}
//     (dID/dqd)^T lambda |_i = S . Vb_i + S . ad_{V_i}^T ab_i
//     (dID/dq)^T lambda |_i  = -Vb_i . ad_S V_i - ab_i . ad_S (a_i - ad_{V_i}(S qd_i))
//                              - (ad_S A_i Fb_{i-1}) . F_i
// using d A_i / d q_i = -ad_S A_i. One lane per chain, robot-interleaved model,
// three sweeps over the links: A (backward) the articulated-body inertias for
// lambda; B (forward) lambda, Fb and the recomputed V, a, f; CE (backward) F,
// ab, Vb and the gradients. Fb needs only lambda, so it rides with the forward
// recursions, and F runs backward like ab and Vb, so those share one sweep.
//
// lambda may instead come from another factorisation of M^-1 (the JSIIA or the
// CFA kernel solving M lambda = g): with lam_in set, sweep A is skipped and
// sweep B reads lambda from the workspace (field VJP_UD), where that kernel
// left it; it has also written grad_tau. qdd may be null: the forward kernel
// then left it in the workspace (field VJP_A, read before sweep B overwrites it).
//
// Branched robots (trees): i - 1 reads p(i) in the forward recursions, and the
// backward ones sum the terms A_c^T (.) of all children c of i, as in the
// tree form of the ABIA: a child whose parent is i - 1 passes them in
// registers, any other child adds them into a record of its parent in the
// workspace (the highest-numbered such child writes it first). The force
// recursion adds straight into the parent's F field, which holds f_p when the
// backward sweep starts.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "spatial.h"

namespace fdk {

// workspace fields per link (block-interleaved like the ABIA workspace)
constexpr int VJP_HD = 0;      // h / D (6), written in sweep A
constexpr int VJP_FB = 0;      // then Fb (6), written over h / D in sweep B
constexpr int VJP_UD = 6;      // u / D (lambda, when it comes from another kernel)
constexpr int VJP_V = 7;       // V (6)
constexpr int VJP_A = 13;      // a (6); entry 0 may hold qdd until sweep B reaches the link
constexpr int VJP_F = 19;      // f (6); trees add the children's A_c^T F_c into it
constexpr int VJP_FIELDS = 25;
// Trees add a branch-point record after those 25 fields, reused sweep by sweep:
// A: the children's p terms (6) and Jh - h h^T / D (21, upper triangle by rows);
// B: the acceleration of the M^-1 g recursion (6); CE: the children's ab (6) and vb (6).
constexpr int VJP_WB = VJP_FIELDS;
constexpr int VJP_TREE_FIELDS = VJP_FIELDS + 27;
template <bool TREE> constexpr int vjp_fields() { return TREE ? VJP_TREE_FIELDS : VJP_FIELDS; }
// LDS of the state stage (launches of serial chains past the last-level
// cache): sweep B's three inputs (2 slots) and its output tile are the largest
// (sweep A: two inputs; sweep CE: two inputs, two outputs).
constexpr int VJP_STAGE = (2 * 3 + 1) * ST_L * ST_W;
static_assert((2 * 2 + 2) * ST_L * ST_W <= VJP_STAGE, "sweep CE fits");

size_t vjp_workspace_elems(int batch, int nmax, bool tree) {
    size_t blocks = (size_t)(batch + 63) / 64;
    return blocks * (size_t)nmax * (tree ? VJP_TREE_FIELDS : VJP_FIELDS) * 64;
}

template <bool NT, typename T>
__device__ __forceinline__ Pose<T> pose_il(const ModelView<T>& m, int i, int slot, T q) {
    T rh[9], p[3];
    m.template home_il<NT>(i, slot, rh, p);
    return joint_pose(rh, p, q);
}

// Y = X^T P X for X = Ad(T^-1) and symmetric P
template <typename T> __device__ __forceinline__ void congruence_up(const Pose<T>& t, const T p[36], T y[36]) {
    T w[36];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        T col[6], out[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) col[r] = p[6 * r + c];
        wrench_to_parent(t, col, out);
#pragma unroll
        for (int r = 0; r < 6; ++r) w[6 * r + c] = out[r];
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) wrench_to_parent(t, w + 6 * r, y + 6 * r);
}

// ad_S x for S = e3 (rotation about z): (z x x_w; z x x_v)
template <typename T> __device__ __forceinline__ void ad_z(const T x[6], T y[6]) {
    y[0] = -x[1]; y[1] = x[0]; y[2] = T(0);
    y[3] = -x[4]; y[4] = x[3]; y[5] = T(0);
}

// Adds x (or stores it, when first) into the workspace entry d.
template <typename T> __device__ __forceinline__ void add_into(T* d, T x, bool first) { *d = first ? x : *d + x; }

template <typename T, bool TREE, bool NT>
__global__ __launch_bounds__(64) void k_fd_vjp(ModelView<T> m, ChainMap cm, int nmax, const T* __restrict__ q,
                                               const T* __restrict__ qd, const T* __restrict__ qdd,
                                               const T* __restrict__ gqdd, T* __restrict__ gq,
                                               T* __restrict__ gqd, T* __restrict__ gtau, int accumulate,
                                               int lam_in, T* __restrict__ ws) {
    // Large launches of serial chains (NT: past the last-level cache) move the
    // joint state and its adjoints through LDS tiles (StateStage, OutTile),
    // loaded and stored by all 64 lanes, so lanes past the batch and unsolved
    // chains take part with no links. Smaller launches, and trees, read and
    // write them lane by lane: at a few hundred wavefronts the tiles' latency
    // costs more than their coalescing gains (measured on a 16384 x 32 rollout).
    constexpr bool ST = NT && !TREE;
    __shared__ T stg[ST ? VJP_STAGE : 1];
    __shared__ int64_t sbase[ST ? 64 : 1];
    __shared__ int slen[ST ? 64 : 1];
    const int lane = threadIdx.x;
    const int b = blockIdx.x * 64 + lane;
    if (!ST && b >= cm.batch) return;
    ChainInfo ci{0, 0, 0, 0, 0};
    if (b < cm.batch) ci = chain_info(m, cm, b);
    if (ci.unsolved) {                                 // longer than the workspace is sized for
        fill_unsolved(gq, ci.state0, ci.unsolved, 0, 1);
        fill_unsolved(gqd, ci.state0, ci.unsolved, 0, 1);
        fill_unsolved(gtau, ci.state0, ci.unsolved, 0, 1);
        if (!ST) return;
        ci.n = 0;
    }
    const int n = ci.n;
    const int sl = ci.slot;
    int nw = n;                                        // loop bound: each lane's own length, or with the
    if constexpr (ST) nw = stage_chains(sbase, slen, ci.state0, n, lane);   // stage the longest in the wavefront
    auto at = [&](const T* a, int i) -> T { return a[ci.state0 + i]; };
    T* wsb = ws + (size_t)blockIdx.x * nmax * vjp_fields<TREE>() * 64 + lane;
    auto w = [&](int i, int f) -> T& { return wsb[((size_t)i * vjp_fields<TREE>() + f) * 64]; };
    // per-link fields stream (NT) when the launch outgrows the last-level cache,
    // a child's update of its parent's F field included; branch-point records
    // keep the default policy
    auto ldw = [&](int i, int f) -> T { return ld_ws<NT>(&w(i, f)); };
    auto stw = [&](int i, int f, T v) { st_ws<NT>(v, &w(i, f)); };
    auto code_of = [&](int i) -> int32_t { return TREE ? m.template tree_il<false>(i, sl) : 0; };

    // A: articulated-body inertias and the p recursion with tau_delta := g
    if (!lam_in) {
        StateStage<T, 2> sa{stg, sbase, slen, lane};     // backward: position k is link n - 1 - k
        const T* const ina[2] = {gqdd, q};
        if constexpr (ST) {
            sa.template start<false>(ina);
            block_sync<64>();
        }
        T pc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T pi[36];
#pragma unroll
        for (int c = 0; c < 36; ++c) pi[c] = T(0);
        Pose<T> tn = pose_identity<T>();
        bool carry = false;                            // trees: registers hold link i+1's terms for link i
        for (int k = 0; k < nw; ++k) {
            if constexpr (ST) {
                sa.template step<false>(ina, k);
                if (k >= n) continue;
            }
            const int i = n - 1 - k;
            const int32_t code = code_of(i);
            T jh[36], pp[6];
            inertia_to_mat6(m.template inertia_il<NT>(i, sl), jh);
            if (TREE && carry) {                       // terms already in this link's frame
#pragma unroll
                for (int c = 0; c < 36; ++c) jh[c] += pi[c];
#pragma unroll
                for (int c = 0; c < 6; ++c) pp[c] = pc[c];
            } else if (!TREE && i + 1 < n) {
                wrench_to_parent(tn, pc, pp);
                T y[36];
                congruence_up(tn, pi, y);
#pragma unroll
                for (int c = 0; c < 36; ++c) jh[c] += y[c];
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) pp[c] = T(0);
            }
            if constexpr (TREE) {
                if (code & TREE_BRANCH) {              // the other children's terms, summed
#pragma unroll
                    for (int c = 0; c < 6; ++c) pp[c] += w(i, VJP_WB + c);
                    int k = VJP_WB + 6;
#pragma unroll
                    for (int r = 0; r < 6; ++r)
#pragma unroll
                        for (int c = r; c < 6; ++c, ++k) {
                            const T y = w(i, k);
                            jh[6 * r + c] += y;
                            if (c != r) jh[6 * c + r] += y;
                        }
                }
            }
            const T dinv = rcp_refined(jh[14]);
            const T u = (ST ? sa.get(0, k) : at(gqdd, i)) - pp[2];
            T h[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) h[c] = jh[6 * c + 2];
#pragma unroll
            for (int c = 0; c < 6; ++c) stw(i, VJP_HD + c, h[c] * dinv);
            stw(i, VJP_UD, u * dinv);
#pragma unroll
            for (int rr = 0; rr < 6; ++rr)
#pragma unroll
                for (int c = 0; c < 6; ++c) pi[6 * rr + c] = jh[6 * rr + c] - h[rr] * h[c] * dinv;
#pragma unroll
            for (int c = 0; c < 6; ++c) pc[c] = pp[c] + h[c] * u * dinv;
            tn = pose_il<NT>(m, i, sl, ST ? sa.get(1, k) : at(q, i));
            if constexpr (TREE) {
                // into the parent's frame on every lane; only the record update diverges
                T x[6], y[36];
                wrench_to_parent(tn, pc, x);
                congruence_up(tn, pi, y);
#pragma unroll
                for (int c = 0; c < 6; ++c) pc[c] = x[c];
#pragma unroll
                for (int c = 0; c < 36; ++c) pi[c] = y[c];
                carry = (code & TREE_CHAIN) != 0;
                const int p = tree_parent(code);
                if (!carry && p >= 0) {                // hand the terms to a branch point now
                    const bool first = (code & TREE_FIRST) != 0;
#pragma unroll
                    for (int c = 0; c < 6; ++c) add_into(&w(p, VJP_WB + c), pc[c], first);
                    int k = VJP_WB + 6;
#pragma unroll
                    for (int r = 0; r < 6; ++r)
#pragma unroll
                        for (int c = r; c < 6; ++c, ++k) add_into(&w(p, k), pi[6 * r + c], first);
                }
            }
        }
    }
    // B (forward): lambda, the force adjoint Fb_i = lambda_i S + A_i Fb_p(i), and
    // the inverse dynamics recursions at the given qdd
    {
        StateStage<T, 3> sb{stg, sbase, slen, lane};     // forward: position k is link k
        const T* const inb[3] = {q, qd, qdd ? qdd : q};  // without qdd the third array is not used
        OutTile<T, 1> ob{stg + 2 * 3 * ST_L * ST_W, sbase, slen, lane};
        T* const outb[1] = {lam_in ? nullptr : gtau};
        if constexpr (ST) {
            block_sync<64>();                          // sweep A's reads of the stage are done
            sb.template start<true>(inb);
            block_sync<64>();
        }
        T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T fb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T v[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T a[6] = {T(0), T(0), T(0), -m.g[0], -m.g[1], -m.g[2]};
        // each step starts the loads of the link after it: the link's own inputs
        // (pose, joint state, qdd, lambda, h / D, inertia) do not depend on the
        // recursion, and the loads would otherwise wait a memory round trip per link
        struct In {
            T qt[4], p[3], q, qd, qdd, lam, hd[6];
            Inertia<T> j;
        };
        auto load = [&](int i) {
            In r;
#pragma unroll
            for (int k = 0; k < 4; ++k) r.qt[k] = m.template at_il<NT>(IL_QUAT + k, i, sl);
#pragma unroll
            for (int k = 0; k < 3; ++k) r.p[k] = m.template at_il<NT>(IL_POS + k, i, sl);
            r.q = ST ? sb.get(0, i) : at(q, i);
            r.qd = ST ? sb.get(1, i) : at(qd, i);
            r.qdd = qdd ? (ST ? sb.get(2, i) : at(qdd, i)) : ldw(i, VJP_A);   // read before this sweep overwrites it
            r.lam = ldw(i, VJP_UD);
#pragma unroll
            for (int c = 0; c < 6; ++c) r.hd[c] = lam_in ? T(0) : ldw(i, VJP_HD + c);
            r.j = m.template inertia_il<NT>(i, sl);
            return r;
        };
        // (serial chains; trees load each link's inputs at its own step: there the
        // extra registers cost more than the overlap gains)
        In nx;
        if (!TREE && n > 0) nx = load(0);
        for (int i = 0; i < nw; ++i) {
            if constexpr (ST) sb.template step<true>(inb, i);
            if (i < n) {
            const int32_t code = code_of(i);
            const In cur = TREE ? load(i) : nx;
            if (!TREE && i + 1 < n) nx = load(i + 1);
            const T qddi = cur.qdd;
            if constexpr (TREE) {
                if (!(code & TREE_CHAIN)) {            // the parent's terms, not link i-1's
                    const int p = tree_parent(code);
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        acc[c] = p < 0 || lam_in ? T(0) : w(p, VJP_WB + c);
                        fb[c] = p < 0 ? T(0) : ldw(p, VJP_FB + c);
                        v[c] = p < 0 ? T(0) : ldw(p, VJP_V + c);
                        a[c] = p < 0 ? (c < 3 ? T(0) : -m.g[c - 3]) : ldw(p, VJP_A + c);
                    }
                }
            }
            T rh[9];
            quat_to_rot(cur.qt, rh);
            const Pose<T> tl = joint_pose(rh, cur.p, cur.q);
            T t[6];
            T lam = cur.lam;
            if (!lam_in) {                             // the a recursion of the M^-1 g solve
                ad_inv_apply(tl, acc, t);
#pragma unroll
                for (int c = 0; c < 6; ++c) lam -= cur.hd[c] * t[c];
                t[2] += lam;
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] = t[c];
                if constexpr (ST) ob.put(0, i, lam);
                else gtau[ci.state0 + i] = accumulate ? gtau[ci.state0 + i] + lam : lam;
            }
            ad_inv_apply(tl, fb, t);
            t[2] += lam;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                fb[c] = t[c];
                stw(i, VJP_FB + c, t[c]);               // h / D of this link is spent
            }
            if constexpr (TREE) {
                if ((code & TREE_BRANCH) && !lam_in) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) w(i, VJP_WB + c) = acc[c];
                }
            }

            const T qdi = cur.qd;
            ad_inv_apply(tl, v, t);
            t[2] += qdi;
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] = t[c];
            ad_inv_apply(tl, a, t);
            t[2] += qddi;
            t[0] += v[1] * qdi; t[1] -= v[0] * qdi;      // + ad_V (S qd) = (w x z qd; v x z qd)
            t[3] += v[4] * qdi; t[4] -= v[3] * qdi;
#pragma unroll
            for (int c = 0; c < 6; ++c) a[c] = t[c];
            T f[6];
            link_force(cur.j, v, a, f);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                stw(i, VJP_V + c, v[c]);
                stw(i, VJP_A + c, a[c]);
                stw(i, VJP_F + c, f[c]);
            }
            }
            if constexpr (ST) ob.template flush<true>(outb, i, nw, accumulate);
        }
    }
    // CE (backward): the force recursion F_i = f_i + sum over children c of A_c^T F_c,
    // the force term of q_bar, and the adjoints of the velocity and acceleration
    // recursions, all in one sweep
    {
        StateStage<T, 2> sc{stg, sbase, slen, lane};     // backward: position k is link n - 1 - k
        const T* const inc[2] = {q, qd};
        OutTile<T, 2> oc{stg + 2 * 2 * ST_L * ST_W, sbase, slen, lane};
        T* const outc[2] = {gq, gqd};
        if constexpr (ST) {
            block_sync<64>();                          // sweep B's reads of the stage are done
            sc.template start<false>(inc);
            block_sync<64>();
        }
        T fc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // link i+1's F, ab, Vb for link i
        T ab[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T vb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        Pose<T> tn = pose_identity<T>();
        bool carry = false;
        // each step of a serial chain starts the loads of the link before it
        // (trees load each link's inputs at its own step)
        struct In {
            Inertia<T> j;
            T f[6], fb[6], v[6], a[6], qt[4], p[3], q, qd;
        };
        auto load = [&](int i) {
            In r;
            r.j = m.template inertia_il<NT>(i, sl);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                r.f[c] = ldw(i, VJP_F + c);
                r.fb[c] = ldw(i, VJP_FB + c);
                r.v[c] = ldw(i, VJP_V + c);
                r.a[c] = ldw(i, VJP_A + c);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) r.qt[k] = m.template at_il<NT>(IL_QUAT + k, i, sl);
#pragma unroll
            for (int k = 0; k < 3; ++k) r.p[k] = m.template at_il<NT>(IL_POS + k, i, sl);
            r.q = ST ? sc.get(0, n - 1 - i) : at(q, i);
            r.qd = ST ? sc.get(1, n - 1 - i) : at(qd, i);
            return r;
        };
        In nx;
        if (!TREE && n > 0) nx = load(n - 1);
        for (int k = 0; k < nw; ++k) {
            if constexpr (ST) sc.template step<false>(inc, k);
            if (k < n) {
            const int i = n - 1 - k;
            const int32_t code = code_of(i);
            const In cur = TREE ? load(i) : nx;
            if (!TREE && i > 0) nx = load(i - 1);
            const Inertia<T> j = cur.j;
            T f[6], fb[6], v[6], a[6], na[6], nv[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                f[c] = cur.f[c];
                fb[c] = cur.fb[c];
                v[c] = cur.v[c];
                a[c] = cur.a[c];
            }
            if (TREE && carry) {                       // terms already in this link's frame
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    f[c] += fc[c];
                    na[c] = ab[c];
                    nv[c] = vb[c];
                }
            } else if (!TREE && i + 1 < n) {
                T fp[6];
                wrench_to_parent(tn, fc, fp);
                wrench_to_parent(tn, ab, na);
                wrench_to_parent(tn, vb, nv);
#pragma unroll
                for (int c = 0; c < 6; ++c) f[c] += fp[c];
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) na[c] = nv[c] = T(0);
            }
            if constexpr (TREE) {
                if (code & TREE_BRANCH) {              // the other children's ab and Vb, summed
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        na[c] += w(i, VJP_WB + c);
                        nv[c] += w(i, VJP_WB + 6 + c);
                    }
                }
            }
            {
                T rh[9];
                quat_to_rot(cur.qt, rh);
                tn = joint_pose(rh, cur.p, cur.q);         // A_i
            }
            // force term of q_bar: -(ad_S A_i Fb_p(i)) . F_i
            const int p = TREE ? tree_parent(code) : i - 1;
            T gq_id = T(0);
            if (p >= 0) {
                T fbp[6], t[6], z[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) fbp[c] = TREE ? ldw(p, VJP_FB + c) : nx.fb[c];   // chains: p = i - 1
                ad_inv_apply(tn, fbp, t);
                ad_z(t, z);
#pragma unroll
                for (int c = 0; c < 6; ++c) gq_id -= z[c] * f[c];
            }
            T jf[6];
            inertia_apply(j, fb, jf);
#pragma unroll
            for (int c = 0; c < 6; ++c) ab[c] = jf[c] + na[c];
            T jv[6], t1[6], avf[6], t2[6];
            inertia_apply(j, v, jv);
            ad_twist_T(fb, jv, t1);
            ad_twist(v, fb, avf);
            inertia_apply(j, avf, t2);
            const T qdi = cur.qd;
            // -ad_{S qd}^T ab = (z qd x ab_w; z qd x ab_v)
            const T sa[6] = {-qdi * ab[1], qdi * ab[0], T(0), -qdi * ab[4], qdi * ab[3], T(0)};
#pragma unroll
            for (int c = 0; c < 6; ++c) vb[c] = t1[c] - t2[c] + sa[c] + nv[c];
            T avt[6];
            ad_twist_T(v, ab, avt);
            const T gqd_id = vb[2] + avt[2];
            // q terms
            T zv[6], avs[6], am[6], za[6];
            ad_z(v, zv);
            const T sqd[6] = {T(0), T(0), qdi, T(0), T(0), T(0)};
            ad_twist(v, sqd, avs);
#pragma unroll
            for (int c = 0; c < 6; ++c) am[c] = a[c] - avs[c];
            ad_z(am, za);
#pragma unroll
            for (int c = 0; c < 6; ++c) gq_id -= vb[c] * zv[c] + ab[c] * za[c];
            if constexpr (ST) {
                oc.put(0, k, -gq_id);                // added as -gq_id when accumulating
                oc.put(1, k, -gqd_id);
            } else {
                const int64_t st = ci.state0 + i;
                gq[st] = accumulate ? gq[st] - gq_id : -gq_id;
                gqd[st] = accumulate ? gqd[st] - gqd_id : -gqd_id;
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) fc[c] = f[c];
            if constexpr (TREE) {
                // into the parent's frame on every lane; only the parent updates diverge
                T x[6];
                wrench_to_parent(tn, fc, x);
#pragma unroll
                for (int c = 0; c < 6; ++c) fc[c] = x[c];
                wrench_to_parent(tn, ab, x);
#pragma unroll
                for (int c = 0; c < 6; ++c) ab[c] = x[c];
                wrench_to_parent(tn, vb, x);
#pragma unroll
                for (int c = 0; c < 6; ++c) vb[c] = x[c];
                carry = (code & TREE_CHAIN) != 0;
                if (!carry && p >= 0) {
                    const bool first = (code & TREE_FIRST) != 0;
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        stw(p, VJP_F + c, ldw(p, VJP_F + c) + fc[c]);   // f_p plus its other children's terms
                        add_into(&w(p, VJP_WB + c), ab[c], first);
                        add_into(&w(p, VJP_WB + 6 + c), vb[c], first);
                    }
                }
            }
            }
            if constexpr (ST) oc.template flush<false>(outc, k, nw, accumulate);
        }
    }
}

// qd' = qd + dt qdd, q' = q + dt qd' (semi-implicit Euler). Elementwise over count entries.
template <typename T>
__global__ void k_euler(int64_t count, T dt, const T* __restrict__ q, const T* __restrict__ qd,
                        const T* __restrict__ qdd, T* __restrict__ qn, T* __restrict__ qdn) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const T v = qd[k] + dt * qdd[k];
    qn[k] = q[k] + dt * v;
    qdn[k] = v;
}

// Adjoint of k_euler: from (q'_bar, qd'_bar) to q_bar, qd_bar and qdd_bar (overwritten).
template <typename T>
__global__ void k_euler_vjp(int64_t count, T dt, const T* __restrict__ gqn, const T* __restrict__ gqdn,
                            T* __restrict__ gq, T* __restrict__ gqd, T* __restrict__ gqdd) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const T gv = gqdn[k] + dt * gqn[k];
    gq[k] = gqn[k];
    gqd[k] = gv;
    gqdd[k] = dt * gv;
}

template <typename T>
hipError_t launch_fd_vjp(const ModelView<T>& m, const ChainMap& cm, int nmax, const T* q, const T* qd, const T* qdd,
                         const T* gqdd, T* gq, T* gqd, T* gtau, int accumulate, int lam_in, T* ws, bool stream,
                         hipStream_t st) {
    if (cm.batch <= 0) return hipSuccess;
    const dim3 grid((cm.batch + 63) / 64);
#define FDK_VJP(TREE, NT)                                                                                       \
    hipLaunchKernelGGL((k_fd_vjp<T, TREE, NT>), grid, dim3(64), 0, st, m, cm, nmax, q, qd, qdd, gqdd, gq, gqd, \
                       gtau, accumulate, lam_in, ws)
    if (m.tree && stream) FDK_VJP(true, true);
    else if (m.tree) FDK_VJP(true, false);
    else if (stream) FDK_VJP(false, true);
    else FDK_VJP(false, false);
#undef FDK_VJP
    return hipGetLastError();
}

int vjp_fields_of(bool tree) { return tree ? VJP_TREE_FIELDS : VJP_FIELDS; }
int vjp_field_lambda() { return VJP_UD; }
int vjp_field_qdd() { return VJP_A; }

template <typename T>
hipError_t launch_euler(int64_t count, T dt, const T* q, const T* qd, const T* qdd, T* qn, T* qdn, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_euler<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, dt, q, qd, qdd,
                       qn, qdn);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_euler_vjp(int64_t count, T dt, const T* gqn, const T* gqdn, T* gq, T* gqd, T* gqdd,
                            hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_euler_vjp<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, dt, gqn,
                       gqdn, gq, gqd, gqdd);
    return hipGetLastError();
}

#define FDK_ADJ_INST(T)                                                                                          \
    template hipError_t launch_fd_vjp<T>(const ModelView<T>&, const ChainMap&, int, const T*, const T*, const T*, \
                                         const T*, T*, T*, T*, int, int, T*, bool, hipStream_t);                \
    template hipError_t launch_euler<T>(int64_t, T, const T*, const T*, const T*, T*, T*, hipStream_t);          \
    template hipError_t launch_euler_vjp<T>(int64_t, T, const T*, const T*, T*, T*, T*, hipStream_t);
FDK_ADJ_INST(double)
FDK_ADJ_INST(float)

}  // namespace fdk
