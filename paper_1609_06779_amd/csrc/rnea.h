// rnea.h -- inverse dynamics of a chain, one lane per link, by scans
// (eq. (EOM-full), Sec. II-B; CalcInvDyn of Algorithm 1).
//
// The three bi-diagonal systems of eq. (EOM-full) have 6x6 blocks Ad_i, the
// adjoint of a rigid transform. The scan element of Sec. II-B for them,
// [[Ad_i, c_i], [0, 1]], has the inclusive prefix [[Ad(T_{i,0}), x_i], [0, 1]];
// we evaluate it as one prefix product of rigid transforms (the base-frame pose
// G_i = T_{0,i} of every link) and prefix / suffix sums of 6-vectors expressed
// in the base frame, where the transform part is the identity:
//   V^s_i  = sum_{k<=i} s_k qd_k                                  (velocity)
//   A^s_i  = A_0 + sum_{k<=i} (s_k qdd_k + ad_{V^s_k}(s_k qd_k))  (acceleration)
//   F^s_i  = sum_{k>=i} Ad(G_k)^-T f_k,  f_k = J_k a_k - ad_{v_k}^T J_k v_k
//   tau_i  = s_i . F^s_i
// with s_i = Ad(G_i) e3 the joint screw in the base frame and (v_k, a_k) the
// body-frame twist and acceleration. A_0 = (0; -g) puts gravity in as a base
// acceleration (the "const." terms of eq. (EOM-full)).
//
// TREE: branched robots numbered depth-first (code: the link's tree code, see
// lanes.h). The same sums run over each link's root path (k <= i above reads
// "k on the path from the base to i") and its subtree (k >= i reads "k in the
// subtree of i"), by the tree scans of lanes.h.
#pragma once
#include "lanes.h"

namespace fdk {

template <typename T> struct LinkLane {
    Pose<T> tl;      // T_{i-1,i}
    Pose<T> g;       // T_{0,i}
    T s[6];          // joint screw in the base frame
    T v[6];          // base-frame twist V^s_i
    Inertia<T> jb;   // body inertia
};

// Returns tau_i = ID(q, qd, qdd)_i for active lanes. All lanes of the group must call it.
template <typename T, int NP, bool TREE = false>
__device__ __forceinline__ T rnea_lane(const ModelView<T>& m, int64_t link, bool active, T q, T qd,
                                       T qdd, bool gravity, int li, T* xbuf, LinkLane<T>& k, int32_t code = 0) {
    const int par = TREE && active ? tree_parent(code) : -1;
    const int end = TREE && active ? tree_end(code) : NP;
    k.tl = pose_identity<T>();
    k.jb.m = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) k.jb.h[c] = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) k.jb.ib[c] = T(0);
    if (active) {
        T rh[9], p[3];
        m.home(link, rh, p);
        k.tl = joint_pose(rh, p, q);
        k.jb = m.inertia(link);
    } else {
        qd = T(0);
        qdd = T(0);
    }
    if constexpr (TREE) k.g = tree_scan_pose<NP>(k.tl, par, li, xbuf);
    else k.g = scan_pose<NP>(k.tl, li, xbuf);
    // s = Ad(G) e3 = (z; p x z), z = third column of R
    const T z[3] = {k.g.r[2], k.g.r[5], k.g.r[8]};
    T pz[3];
    cross3(k.g.p, z, pz);
    k.s[0] = z[0]; k.s[1] = z[1]; k.s[2] = z[2];
    k.s[3] = pz[0]; k.s[4] = pz[1]; k.s[5] = pz[2];

    T sqd[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) { sqd[c] = k.s[c] * qd; k.v[c] = sqd[c]; }
    if constexpr (TREE) tree_scan_add<NP, 6>(k.v, par, li, xbuf);
    else scan_add<NP, 6>(k.v, li, xbuf);

    T a[6];
    ad_twist(k.v, sqd, a);
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] += k.s[c] * qdd;
    if constexpr (TREE) tree_scan_add<NP, 6>(a, par, li, xbuf);
    else scan_add<NP, 6>(a, li, xbuf);
    if (gravity) {
        a[3] -= m.g[0];
        a[4] -= m.g[1];
        a[5] -= m.g[2];
    }

    T vb[6], ab[6], fb[6], fs[6];
    ad_inv_apply(k.g, k.v, vb);
    ad_inv_apply(k.g, a, ab);
    link_force(k.jb, vb, ab, fb);
    wrench_to_parent(k.g, fb, fs);
    if (!active) {
#pragma unroll
        for (int c = 0; c < 6; ++c) fs[c] = T(0);
    }
    if constexpr (TREE) subtree_sum<NP, 6>(fs, end, li, xbuf);
    else scan_add_rev<NP, 6>(fs, li, xbuf);
    T tau = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) tau += k.s[c] * fs[c];
    return tau;
}

// Composite inertia of links i..n-1 in the base frame, as a suffix sum of
// spatial inertias (10 numbers each): column i of M is the inverse dynamics
// with qdd = e_i, qd = 0 and no gravity, whose force recursion sums
// J_k V^s_k = J_k s_i over k >= i (Sec. II-C), so
//   M_ik = s_max(i,k)^T Ic_max(i,k) s_min(i,k).
// TREE: the composite inertia of i's subtree; M_ik is that product when one
// of i, k is an ancestor of the other, else zero (the caller masks it).
template <typename T, int NP, bool TREE = false>
__device__ __forceinline__ void composite_force(const LinkLane<T>& k, bool active, int li, T* xbuf, T f[6],
                                                int32_t code = 0) {
    // base-frame inertia of the link: m, h^s = m (R c + p), Ibar^s = R Ibar R^T + m([Rc]^2 - [c^s]^2)
    T ic[10];
    if (active) {
        const T* r = k.g.r;
        const T m = k.jb.m;
        T rc[3];                       // R c = R h / m
        matvec3(r, k.jb.h, rc);
        const T invm = rcp_refined(m);
        rc[0] *= invm; rc[1] *= invm; rc[2] *= invm;
        T cs[3] = {rc[0] + k.g.p[0], rc[1] + k.g.p[1], rc[2] + k.g.p[2]};
        const T* s = k.jb.ib;
        T a[9] = {s[0], s[3], s[4], s[3], s[1], s[5], s[4], s[5], s[2]};
        T ra[9], rar[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) ra[3 * i + j] = r[3 * i] * a[j] + r[3 * i + 1] * a[3 + j] + r[3 * i + 2] * a[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                rar[3 * i + j] = ra[3 * i] * r[3 * j] + ra[3 * i + 1] * r[3 * j + 1] + ra[3 * i + 2] * r[3 * j + 2];
        // [x]^2 = x x^T - |x|^2 I
        T n1 = rc[0] * rc[0] + rc[1] * rc[1] + rc[2] * rc[2];
        T n2 = cs[0] * cs[0] + cs[1] * cs[1] + cs[2] * cs[2];
        ic[0] = m;
        ic[1] = m * cs[0]; ic[2] = m * cs[1]; ic[3] = m * cs[2];
        ic[4] = rar[0] + m * ((rc[0] * rc[0] - n1) - (cs[0] * cs[0] - n2));
        ic[5] = rar[4] + m * ((rc[1] * rc[1] - n1) - (cs[1] * cs[1] - n2));
        ic[6] = rar[8] + m * ((rc[2] * rc[2] - n1) - (cs[2] * cs[2] - n2));
        ic[7] = rar[1] + m * (rc[0] * rc[1] - cs[0] * cs[1]);
        ic[8] = rar[2] + m * (rc[0] * rc[2] - cs[0] * cs[2]);
        ic[9] = rar[5] + m * (rc[1] * rc[2] - cs[1] * cs[2]);
    } else {
#pragma unroll
        for (int c = 0; c < 10; ++c) ic[c] = T(0);
    }
    if constexpr (TREE) subtree_sum<NP, 10>(ic, active ? tree_end(code) : NP, li, xbuf);
    else scan_add_rev<NP, 10>(ic, li, xbuf);
    Inertia<T> cj;
    cj.m = ic[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) cj.h[c] = ic[1 + c];
#pragma unroll
    for (int c = 0; c < 6; ++c) cj.ib[c] = ic[4 + c];
    inertia_apply(cj, k.s, f);
}

}  // namespace fdk
