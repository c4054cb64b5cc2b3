// lanes.h -- lane-group exchange, segmented scans and the device model view.
//
// A chain of n <= NP links is processed by a group of NP consecutive threads
// (one link per thread). NP <= 64 groups live inside one wavefront and
// exchange through ds_bpermute shuffles limited to the group; NP = 128 or 256
// groups span a whole workgroup and exchange through LDS.
//
// The scans are the paper's all-prefix-sum over a binary associative operator
// (Sec. II-B), evaluated by recursive doubling over the NP lanes of a chain:
// log2(NP) steps, each combining with the partial result s lanes away.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spatial.h"

namespace fdk {

// ---------------- model view (canonical joint frames, structure of arrays) ----------------
// Field f of link l lives at base[f * stride + l].
enum ModelField {
    MF_ROT = 0,     // 9: home rotation of frame i in frame i-1 (row-major)
    MF_POS = 9,     // 3: origin of frame i in frame i-1
    MF_MASS = 12,   // 1
    MF_H = 13,      // 3: m c (first mass moment about the frame origin)
    MF_IB = 16,     // 6: Ic - m[c][c] (xx yy zz xy xz yz)
    MF_ICINV = 22,  // 6: Ic^-1
    MF_COM = 28,    // 3: c
    MF_MINV = 31,   // 1: 1/m
    MF_COUNT = 32
};
// The robot-interleaved copy read by the lane-per-chain kernels holds the
// home rotation as a unit quaternion (4 values instead of 9: those kernels
// stream the model from HBM once per sweep), then the origin and the inertia.
enum InterleavedField {
    IL_QUAT = 0,    // 4: w x y z of Rhome
    IL_POS = 4,     // 3
    IL_MASS = 7,    // 1
    IL_H = 8,       // 3
    IL_IB = 11,     // 6
    IL_COUNT = 17
};

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z).
template <typename T> __device__ __forceinline__ void quat_to_rot(const T qt[4], T r[9]) {
    const T w = qt[0], x = qt[1], y = qt[2], z = qt[3];
    const T x2 = x + x, y2 = y + y, z2 = z + z;
    const T xx = x * x2, yy = y * y2, zz = z * z2, xy = x * y2, xz = x * z2, yz = y * z2;
    const T wx = w * x2, wy = w * y2, wz = w * z2;
    r[0] = T(1) - (yy + zz); r[1] = xy - wz;            r[2] = xz + wy;
    r[3] = xy + wz;            r[4] = T(1) - (xx + zz); r[5] = yz - wx;
    r[6] = xz - wy;            r[7] = yz + wx;            r[8] = T(1) - (xx + yy);
}

// J^-1 = [[Ic^-1, -Ic^-1 [c]], [[c] Ic^-1, 1/m - [c] Ic^-1 [c]]] (row-major 6x6)
// from p = (Ic^-1 as xx yy zz xy xz yz, c, 1/m): the inverse of the spatial
// inertia about the frame origin.
template <typename T> __device__ __forceinline__ void inv_inertia6(const T p[10], T m[36]) {
    const T* s = p;
    const T* c = p + 6;
    const T mi = p[9];
    T a[9] = {s[0], s[3], s[4], s[3], s[1], s[5], s[4], s[5], s[2]};
    // X = a [c]  (X[r][k] = sum_j a[r][j] [c][j][k])
    T cx[9] = {T(0), -c[2], c[1], c[2], T(0), -c[0], -c[1], c[0], T(0)};
    T x[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            x[3 * r + k] = a[3 * r] * cx[k] + a[3 * r + 1] * cx[3 + k] + a[3 * r + 2] * cx[6 + k];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            m[6 * r + k] = a[3 * r + k];
            m[6 * r + k + 3] = -x[3 * r + k];        // -a [c]
            m[6 * (r + 3) + k] = -x[3 * k + r];      // [c] a = -(a [c])^T
            // 1/m - [c] a [c] = 1/m + (a [c])^T [c]
            T y = cx[r] * x[k] + cx[3 + r] * x[3 + k] + cx[6 + r] * x[6 + k];
            m[6 * (r + 3) + k + 3] = (r == k ? mi : T(0)) + y;
        }
}

// The same body's inverse-inertia parameters in the child frame of t = (R, p):
// c' = R^T (c - p), Ic'^-1 = R^T Ic^-1 R, 1/m unchanged. inv_inertia6 of the
// result equals Ad(t^-1) J^-1 Ad(t^-1)^T.
template <typename T> __device__ __forceinline__ void inv_inertia_to_child(const Pose<T>& t, const T p[10], T o[10]) {
    const T* s = p;
    const T a[9] = {s[0], s[3], s[4], s[3], s[1], s[5], s[4], s[5], s[2]};
    T b[9];                                          // a R
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) b[3 * r + k] = a[3 * r] * t.r[k] + a[3 * r + 1] * t.r[3 + k] + a[3 * r + 2] * t.r[6 + k];
    // (R^T b)[i][k] = sum_j R[j][i] b[j][k]
    auto rtb = [&](int i, int k) { return t.r[i] * b[k] + t.r[3 + i] * b[3 + k] + t.r[6 + i] * b[6 + k]; };
    o[0] = rtb(0, 0); o[1] = rtb(1, 1); o[2] = rtb(2, 2);
    o[3] = rtb(0, 1); o[4] = rtb(0, 2); o[5] = rtb(1, 2);
    const T d[3] = {p[6] - t.p[0], p[7] - t.p[1], p[8] - t.p[2]};
    matTvec3(t.r, d, o + 6);
    o[9] = p[9];
}

// Branched robots (trees): link i hangs from link p(i) < i of its robot, or
// from the base. Per link and robot column, an int32 code (interleaved like
// `il`, [i * num_robots + column]) describes the link's place in the tree:
//   bits 0..8    p(i) + 1 (0: the base);
//   bits 9..17   one past the last link of i's subtree, when the robot's
//                links are numbered depth-first (its subtree is then the run
//                i .. end - 1; the lane-per-link kernels need that order);
//   TREE_CHAIN   p(i) = i - 1: the lane-per-chain kernel still has the
//                parent's terms in registers;
//   TREE_BRANCH  i has a child other than i + 1: its terms go through the
//                workspace for that child;
//   TREE_FIRST   the highest-numbered such child of p(i): the first to reach
//                p(i)'s accumulator in the backward sweep, so it writes it.
constexpr int32_t TREE_CHAIN = 1 << 24, TREE_BRANCH = 1 << 25, TREE_FIRST = 1 << 26;
__host__ __device__ __forceinline__ int tree_parent(int32_t code) { return (code & 0x1ff) - 1; }
__host__ __device__ __forceinline__ int tree_end(int32_t code) { return (code >> 9) & 0x1ff; }

template <typename T> struct ModelView {
    const T* base;
    int64_t stride;               // total links of the model
    const int64_t* link_start;    // [num_robots] first link of each robot
    const int32_t* n_links;       // [num_robots]
    int32_t num_robots;
    T g[3];                       // gravity, base frame
    // Robot-interleaved copy (InterleavedField): field f of link i
    // of the robot in column c at il[f * il_fstride + i * num_robots + c]
    // (il_fstride = longest robot x num_robots), so that lanes holding
    // consecutive columns read consecutive addresses. Columns hold the robots
    // sorted by decreasing length (stable: a model of equal lengths keeps its
    // order); slot[r] is the column of robot r.
    const T* il;
    int64_t il_fstride;
    const int32_t* slot;
    const int32_t* tree;          // tree codes, or null when every robot is a serial chain

    __device__ __forceinline__ T at(int f, int64_t l) const { return base[f * stride + l]; }
    // NT: a non-temporal load, for launches whose model and workspace outgrow
    // the last-level cache; then these lines, streamed once per sweep, do not
    // push out the chain state the lane-per-chain kernels reuse across links.
    template <bool NT = false> __device__ __forceinline__ T at_il(int f, int i, int c) const {
        const T* p = &il[f * il_fstride + (int64_t)i * num_robots + c];
        if constexpr (NT) return __builtin_nontemporal_load(p);
        else return *p;
    }
    template <bool NT = false> __device__ __forceinline__ int32_t tree_il(int i, int c) const {
        const int32_t* p = &tree[(int64_t)i * num_robots + c];
        if constexpr (NT) return __builtin_nontemporal_load(p);
        else return *p;
    }
    template <bool NT = false> __device__ __forceinline__ void home_il(int i, int c, T rh[9], T p[3]) const {
        T qt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) qt[k] = at_il<NT>(IL_QUAT + k, i, c);
#pragma unroll
        for (int k = 0; k < 3; ++k) p[k] = at_il<NT>(IL_POS + k, i, c);
        quat_to_rot(qt, rh);
    }
    template <bool NT = false> __device__ __forceinline__ Inertia<T> inertia_il(int i, int c) const {
        Inertia<T> j;
        j.m = at_il<NT>(IL_MASS, i, c);
#pragma unroll
        for (int k = 0; k < 3; ++k) j.h[k] = at_il<NT>(IL_H + k, i, c);
#pragma unroll
        for (int k = 0; k < 6; ++k) j.ib[k] = at_il<NT>(IL_IB + k, i, c);
        return j;
    }

    __device__ __forceinline__ void home(int64_t l, T r[9], T p[3]) const {
#pragma unroll
        for (int k = 0; k < 9; ++k) r[k] = at(MF_ROT + k, l);
#pragma unroll
        for (int k = 0; k < 3; ++k) p[k] = at(MF_POS + k, l);
    }

    __device__ __forceinline__ Inertia<T> inertia(int64_t l) const {
        Inertia<T> j;
        j.m = at(MF_MASS, l);
#pragma unroll
        for (int k = 0; k < 3; ++k) j.h[k] = at(MF_H + k, l);
#pragma unroll
        for (int k = 0; k < 6; ++k) j.ib[k] = at(MF_IB + k, l);
        return j;
    }

    // inverse-inertia parameters of link l: Ic^-1 (xx yy zz xy xz yz), c, 1/m
    __device__ __forceinline__ void inertia_inv_params(int64_t l, T p[10]) const {
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k] = at(MF_ICINV + k, l);
#pragma unroll
        for (int k = 0; k < 3; ++k) p[6 + k] = at(MF_COM + k, l);
        p[9] = at(MF_MINV, l);
    }
};

// The inverse-inertia parameters (Ic^-1 as xx yy zz xy xz yz, c, 1/m; see
// inv_inertia6) of a body given by its inertia about the frame origin (m,
// h = m c, Ibar = Ic - m [c][c]): Ic = Ibar + m [c][c] = Ibar + m (c c^T - |c|^2 1),
// inverted by cofactors. Evaluated in FP64 whatever T is.
template <typename T> __device__ __forceinline__ void inv_params_of(const Inertia<T>& j, T p[10]) {
    const double m = j.m, mi = rcp_refined(m);        // m > 0 and det > 0: the inertia is SPD
    const double c[3] = {double(j.h[0]) * mi, double(j.h[1]) * mi, double(j.h[2]) * mi};
    const double a00 = double(j.ib[0]) - m * (c[1] * c[1] + c[2] * c[2]);
    const double a11 = double(j.ib[1]) - m * (c[0] * c[0] + c[2] * c[2]);
    const double a22 = double(j.ib[2]) - m * (c[0] * c[0] + c[1] * c[1]);
    const double a01 = double(j.ib[3]) + m * c[0] * c[1];
    const double a02 = double(j.ib[4]) + m * c[0] * c[2];
    const double a12 = double(j.ib[5]) + m * c[1] * c[2];
    const double k00 = a11 * a22 - a12 * a12, k01 = a02 * a12 - a01 * a22, k02 = a01 * a12 - a02 * a11;
    const double k11 = a00 * a22 - a02 * a02, k12 = a01 * a02 - a00 * a12, k22 = a00 * a11 - a01 * a01;
    const double idet = rcp_refined(a00 * k00 + a01 * k01 + a02 * k02);
    p[0] = T(k00 * idet); p[1] = T(k11 * idet); p[2] = T(k22 * idet);
    p[3] = T(k01 * idet); p[4] = T(k02 * idet); p[5] = T(k12 * idet);
    p[6] = T(c[0]); p[7] = T(c[1]); p[8] = T(c[2]);
    p[9] = T(mi);
}

// ---------------- chain lookup ----------------
struct ChainMap {
    const int32_t* robot_id;   // device [batch] or null: chain b uses robot b (robot 0 if one robot)
    const int64_t* offsets;    // device [batch+1] or null: chain b starts at b * n_uniform
    int32_t batch;
    int32_t n_uniform;
    int32_t n_cap;             // longest chain the launch is sized for; longer ones are not solved
};

// link0: the robot's first link (structure-of-arrays fields); state0: the
// chain's first entry in q, qd, tau; n: its links (0: skipped); slot: the
// robot's column in the interleaved copy; unsolved: the length of a chain
// longer than the launch is sized for (n is then 0), else 0.
struct ChainInfo { int64_t link0; int64_t state0; int n; int slot; int unsolved; };

template <typename T>
__device__ __forceinline__ ChainInfo chain_info(const ModelView<T>& m, const ChainMap& cm, int b) {
    int r = cm.robot_id ? cm.robot_id[b] : (m.num_robots == 1 ? 0 : b);
    ChainInfo ci;
    ci.unsolved = 0;
    if (r < 0 || r >= m.num_robots) {   // out-of-range robot id: the chain is skipped
        ci.link0 = 0;
        ci.n = 0;
        ci.state0 = 0;
        ci.slot = 0;
        return ci;
    }
    ci.slot = m.slot[r];
    ci.link0 = m.link_start[r];
    ci.n = m.n_links[r];
    ci.state0 = cm.offsets ? cm.offsets[b] : (int64_t)b * cm.n_uniform;
    if (ci.n > cm.n_cap) {
        ci.unsolved = ci.n;
        ci.n = 0;
    }
    return ci;
}

// How a forward-dynamics kernel delivers q-ddot of chain b, link i (packed
// entry st). Plain forward dynamics: out[st] = qdd. The reverse mode also uses
// the kernels
//   * to solve M lambda = g (solve != 0: tau holds g, and the bias forces are
//     left out: zero velocity, no gravity, so tau_delta = g exactly), adding
//     the result into out when accumulate != 0;
//   * to hand their result to the lane-per-chain reverse-mode kernel: aux, when
//     set, also receives it in field aux_field of that kernel's workspace
//     ([block of 64 chains][link][field][lane], aux_fields fields per link).
// out may be null when aux is the only consumer.
template <typename T> struct FdOut {
    int accumulate = 0;
    int solve = 0;
    T* aux = nullptr;
    int aux_nmax = 0, aux_fields = 0, aux_field = 0;
    __device__ __forceinline__ void put(T* out, int64_t st, int b, int i, T v) const {
        if (out) out[st] = accumulate ? out[st] + v : v;
        put_aux(b, i, v);
    }
    // the aux copy alone (for kernels that write `out` themselves)
    __device__ __forceinline__ void put_aux(int b, int i, T v) const {
        if (aux) aux[(((size_t)(b >> 6) * aux_nmax + i) * aux_fields + aux_field) * 64 + (b & 63)] = v;
    }
};

// NaN over the `count` outputs of an unsolved chain starting at out + first,
// written by `lanes` lanes (this one is `lane`).
template <typename T>
__device__ __forceinline__ void fill_unsolved(T* out, int64_t first, int64_t count, int lane, int lanes) {
    for (int64_t k = lane; k < count; k += lanes) out[first + k] = T(__builtin_nan(""));
}

// Workspace access with the same cache policy as at_il<NT>.
template <bool NT, typename T> __device__ __forceinline__ T ld_ws(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void st_ws(T v, T* p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Block-wide LDS ordering. Larger blocks need the barrier. A block of one
// wavefront needs no hardware barrier (its LDS operations complete in program
// order), but the compiler must still not move LDS accesses across the point
// where lanes hand data to each other: without a fence it may, for instance,
// sink a lane's read of another lane's store into a branch taken only by the
// writers. The wave barrier emits no instruction and pins that order.
template <int THREADS> __device__ __forceinline__ void block_sync() {
    if constexpr (THREADS > 64) __syncthreads();
    else __builtin_amdgcn_wave_barrier();
}

// Joint state through LDS. q, qd, tau and qdd are packed per chain (entry
// state0 + i), so one lane per chain would touch a cache line per lane with
// every access. Each sweep moves them instead in tiles of ST_L sweep positions
// by the wavefront's 64 chains: a tile is loaded with consecutive lanes on
// consecutive entries of one chain (ST_L * sizeof(T) bytes per chain),
// transposed through LDS, and each lane reads its chain's entry per step.
// Position k of a sweep is link k (forward sweeps) or link n - 1 - k (the
// backward sweep). Tiles are committed to LDS one tile ahead of use and loaded
// into registers two ahead, so their memory latency overlaps the steps.
constexpr int ST_L = 8;                 // sweep positions per tile
constexpr int ST_W = 64 + 8;            // LDS row stride: commits hit every bank pair equally

template <typename T, int NA> struct StateStage {
    T* s;                               // [2 slots][NA][ST_L][ST_W], this wavefront's
    const int64_t* base;                // [64] first state entry of each lane's chain
    const int* len;                     // [64] its length (0: no chain)
    int lane;
    T reg[NA][ST_L];                    // the tile in flight
    // Loads tile t of arrays a[0..NA) into registers: lane l takes entry
    // l % ST_L of chain (k * 64 + l) / ST_L in its k-th load.
    template <bool FWD> __device__ __forceinline__ void load(const T* const (&a)[NA], int t) {
#pragma unroll
        for (int k = 0; k < ST_L; ++k) {
            const int c = (k * 64 + lane) / ST_L, j = lane % ST_L;
            const int pos = t * ST_L + j, n = len[c];
            const int64_t e = FWD ? base[c] + pos : base[c] + (n - 1 - pos);
#pragma unroll
            for (int v = 0; v < NA; ++v) reg[v][k] = pos < n ? a[v][e] : T(0);
        }
    }
    __device__ __forceinline__ void commit(int t) {
        T* d = s + (t & 1) * NA * ST_L * ST_W;
#pragma unroll
        for (int k = 0; k < ST_L; ++k) {
            const int c = (k * 64 + lane) / ST_L, j = lane % ST_L;
#pragma unroll
            for (int v = 0; v < NA; ++v) d[(v * ST_L + j) * ST_W + c] = reg[v][k];
        }
    }
    // array v at sweep position pos (its tile committed), for this lane's chain
    __device__ __forceinline__ T get(int v, int pos) const {
        return s[(((pos / ST_L) & 1) * NA + v) * ST_L * ST_W + (pos % ST_L) * ST_W + lane];
    }
    // Before the loop: tiles 0 and 1 committed, tile 2 in flight; the three
    // tiles' loads are issued together. The caller separates the commits from
    // the first reads (and earlier readers of the LDS from the commits) with
    // block_sync<64>.
    template <bool FWD> __device__ __forceinline__ void start(const T* const (&a)[NA]) {
        T r0[NA][ST_L];
        load<FWD>(a, 0);
        for (int v = 0; v < NA; ++v)
            for (int k = 0; k < ST_L; ++k) r0[v][k] = reg[v][k];
        load<FWD>(a, 1);
        T* d = s;
#pragma unroll
        for (int k = 0; k < ST_L; ++k) {
            const int c = (k * 64 + lane) / ST_L, j = lane % ST_L;
#pragma unroll
            for (int v = 0; v < NA; ++v) d[(v * ST_L + j) * ST_W + c] = r0[v][k];
        }
        commit(1);
        load<FWD>(a, 2);
    }
    // At position k of the loop (every lane, every k): at the first position of
    // tile t >= 1 the registers (tile t + 1) go to LDS over tile t - 1, whose
    // last entry was read two positions earlier, and tile t + 2 is loaded.
    // The LDS hand-off is fenced here (block_sync<64>), so the steps in between
    // carry no fence.
    template <bool FWD> __device__ __forceinline__ void step(const T* const (&a)[NA], int k) {
        if (k > 0 && k % ST_L == 0) {
            const int t = k / ST_L;
            block_sync<64>();
            commit(t + 1);
            block_sync<64>();
            load<FWD>(a, t + 2);
        }
    }
};

// Per-lane outputs of a sweep, staged like StateStage's inputs: put() writes
// this lane's value at sweep position pos, and after a tile's last position
// flush() stores the tile chain by chain (consecutive lanes on consecutive
// entries of one chain), adding to what is there when accumulating.
template <typename T, int NO> struct OutTile {
    T* s;                               // [NO][ST_L][ST_W]
    const int64_t* base;
    const int* len;
    int lane;
    __device__ __forceinline__ void put(int o, int pos, T v) { s[(o * ST_L + pos % ST_L) * ST_W + lane] = v; }
    // Every lane at every position k of a loop over nw positions; acts after
    // the last position of each tile. Null outputs are skipped.
    template <bool FWD>
    __device__ __forceinline__ void flush(T* const (&out)[NO], int k, int nw, int accumulate) {
        if (k % ST_L != ST_L - 1 && k != nw - 1) return;
        block_sync<64>();
        const int t = k / ST_L;
        if (accumulate) {
            // the values to add to are all loaded first, so that they are in
            // flight together (a store may alias a later entry, so the compiler
            // keeps the written order), then the sums are stored
            T prev[ST_L][NO];
#pragma unroll
            for (int kk = 0; kk < ST_L; ++kk) {
                const int c = (kk * 64 + lane) / ST_L, j = lane % ST_L;
                const int pos = t * ST_L + j, n = len[c];
                const int64_t e = FWD ? base[c] + pos : base[c] + (n - 1 - pos);
#pragma unroll
                for (int o = 0; o < NO; ++o) prev[kk][o] = out[o] && pos < n ? out[o][e] : T(0);
            }
#pragma unroll
            for (int kk = 0; kk < ST_L; ++kk) {
                const int c = (kk * 64 + lane) / ST_L, j = lane % ST_L;
                const int pos = t * ST_L + j, n = len[c];
                const int64_t e = FWD ? base[c] + pos : base[c] + (n - 1 - pos);
#pragma unroll
                for (int o = 0; o < NO; ++o)
                    if (out[o] && pos < n) out[o][e] = prev[kk][o] + s[(o * ST_L + j) * ST_W + c];
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < ST_L; ++kk) {
                const int c = (kk * 64 + lane) / ST_L, j = lane % ST_L;
                const int pos = t * ST_L + j, n = len[c];
                const int64_t e = FWD ? base[c] + pos : base[c] + (n - 1 - pos);
#pragma unroll
                for (int o = 0; o < NO; ++o)
                    if (out[o] && pos < n) out[o][e] = s[(o * ST_L + j) * ST_W + c];
            }
        }
        block_sync<64>();                       // read before the next tile's puts
    }
};

// The chain table of a wavefront for StateStage / OutTile: each lane enters
// its chain (first state entry, length; 0 for none). Returns the longest
// length in the wavefront, the bound of the sweep loops (every lane runs them,
// each lane's body guarded by its own length).
__device__ __forceinline__ int stage_chains(int64_t* base, int* len, int64_t state0, int n, int lane) {
    block_sync<64>();                           // earlier readers of the table are done
    base[lane] = state0;
    len[lane] = n;
    block_sync<64>();
    int nw = n;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nw = max(nw, __shfl_xor(nw, d, 64));
    return nw;
}

// ---------------- lane-group exchange ----------------
// Groups of NP <= 64 lanes live in one wavefront and exchange values through
// DPP (data-parallel primitives: a VALU operand read from another lane, no LDS
// round trip): wave_shr/shl:1 for neighbour shifts, row_shr/shl within 16-lane
// rows and row_bcast:15/31 across rows. Larger groups span several wavefronts
// and go through LDS.
namespace dpp {
constexpr int ROW_SHL = 0x100, ROW_SHR = 0x110, WAVE_SHL1 = 0x130, WAVE_SHR1 = 0x138, ROW_BCAST15 = 0x142,
              ROW_BCAST31 = 0x143, QUAD_XOR1 = 0xB1, QUAD_XOR2 = 0x4E, ROW_MIRROR = 0x140,
              ROW_HALF_MIRROR = 0x141;

// Lane l takes the value that control CTRL routes to it. Lanes with no source
// lane read 0; lanes in rows outside ROW_MASK are left undefined. (No "old"
// operand: the result needs no copy of the source into the destination first.)
template <int CTRL, int ROW_MASK = 0xf> __device__ __forceinline__ double mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROW_MASK, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK = 0xf> __device__ __forceinline__ float mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}
template <int CTRL, int ROW_MASK = 0xf, typename T> __device__ __forceinline__ void mov_n(const T* v, T* out, int k) {
    for (int c = 0; c < k; ++c) out[c] = mov<CTRL, ROW_MASK>(v[c]);
}
// value of wavefront lane `lane` (a compile-time lane), in every lane
template <int LANE> __device__ __forceinline__ double read(double v) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), LANE);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), LANE);
    return __hiloint2double(hi, lo);
}
template <int LANE> __device__ __forceinline__ float read(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), LANE));
}
// value of wavefront lane `lane`, a lane index the same in every lane of the
// wavefront (a loop counter, say), in every lane
__device__ __forceinline__ double read_at(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float read_at(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// Lane l ^ 16 (the same place in the other 16-lane row of its 32-lane half),
// by ds_swizzle in bit mode (and mask 0x1f, xor mask 0x10).
__device__ __forceinline__ double swizzle_xor16(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401f);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401f);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swizzle_xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401f));
}
// Sum over each aligned group of W = 8, 16 or 32 consecutive lanes, in every lane
// of the group: a butterfly (lane i pairs with i^1, i^2, then the mirrored
// half), so every lane adds the same operands in the same order and the
// groups' lanes hold bitwise equal sums.
template <int W, typename T> __device__ __forceinline__ T group_sum(T v) {
    static_assert(W == 8 || W == 16 || W == 32, "groups of 8, 16 or 32 lanes");
    v += mov<QUAD_XOR1>(v);
    v += mov<QUAD_XOR2>(v);
    v += mov<ROW_HALF_MIRROR>(v);
    if constexpr (W >= 16) v += mov<ROW_MIRROR>(v);
    if constexpr (W == 32) v += swizzle_xor16(v);
    return v;
}
}  // namespace dpp

// Value of lane (li - s) of the same group (callers only use it where li >= s).
template <int NP, typename T>
__device__ __forceinline__ void shift_up(const T* v, T* out, int k, int s, T* lds) {
    if constexpr (NP <= 64) {
        if (s == 1) {
            dpp::mov_n<dpp::WAVE_SHR1>(v, out, k);
        } else {
            for (int c = 0; c < k; ++c) out[c] = __shfl_up(v[c], (unsigned)s, NP);
        }
    } else {
        int t = threadIdx.x;
        for (int c = 0; c < k; ++c) lds[c * NP + t] = v[c];
        __syncthreads();
        int src = t >= s ? t - s : t;
        for (int c = 0; c < k; ++c) out[c] = lds[c * NP + src];
        __syncthreads();
    }
}

// Value of lane (li + s) of the same group (callers only use it where li + s < NP).
template <int NP, typename T>
__device__ __forceinline__ void shift_down(const T* v, T* out, int k, int s, T* lds) {
    if constexpr (NP <= 64) {
        if (s == 1) {
            dpp::mov_n<dpp::WAVE_SHL1>(v, out, k);
        } else {
            for (int c = 0; c < k; ++c) out[c] = __shfl_down(v[c], (unsigned)s, NP);
        }
    } else {
        int t = threadIdx.x;
        for (int c = 0; c < k; ++c) lds[c * NP + t] = v[c];
        __syncthreads();
        int src = t + s < NP ? t + s : t;
        for (int c = 0; c < k; ++c) out[c] = lds[c * NP + src];
        __syncthreads();
    }
}

// Inclusive prefix product of poses along the group: G_i = T_0 T_1 ... T_i.
// Within a wavefront: Hillis-Steele steps inside each 16-lane row, then odd
// rows take the total of the row before (row_bcast:15) and rows 2, 3 the total
// of rows 0, 1 (row_bcast:31); the earlier part always multiplies on the left.
template <int NP, typename T>
__device__ __forceinline__ Pose<T> scan_pose(Pose<T> x, int li, T* lds) {
    if constexpr (NP <= 64) {
        const int lr = li & 15;
        const int lane = threadIdx.x & 63;
#define FDK_POSE_STEP(CTRL, MASK, COND)                 \
    {                                                   \
        Pose<T> o;                                      \
        dpp::mov_n<CTRL, MASK>(x.r, o.r, 9);            \
        dpp::mov_n<CTRL, MASK>(x.p, o.p, 3);            \
        if (COND) x = pose_mul(o, x);                   \
    }
        FDK_POSE_STEP(dpp::ROW_SHR + 1, 0xf, lr >= 1)
        if constexpr (NP > 2) FDK_POSE_STEP(dpp::ROW_SHR + 2, 0xf, lr >= 2)
        if constexpr (NP > 4) FDK_POSE_STEP(dpp::ROW_SHR + 4, 0xf, lr >= 4)
        if constexpr (NP > 8) FDK_POSE_STEP(dpp::ROW_SHR + 8, 0xf, lr >= 8)
        if constexpr (NP > 16) FDK_POSE_STEP(dpp::ROW_BCAST15, 0xa, (lane & 16) != 0)
        if constexpr (NP > 32) FDK_POSE_STEP(dpp::ROW_BCAST31, 0xc, (lane & 32) != 0)
#undef FDK_POSE_STEP
        return x;
    } else {
        // each wavefront scans its 64 lanes, then takes the product of the
        // earlier wavefronts' totals (lane 63 of each) from LDS
        constexpr int WAVES = NP / 64;
        x = scan_pose<64>(x, li & 63, lds);
        const int w = li >> 6;
        if ((li & 63) == 63 && w + 1 < WAVES) {
#pragma unroll
            for (int c = 0; c < 9; ++c) lds[12 * w + c] = x.r[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) lds[12 * w + 9 + c] = x.p[c];
        }
        __syncthreads();
        if (w > 0) {
            Pose<T> o;
#pragma unroll
            for (int c = 0; c < 9; ++c) o.r[c] = lds[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) o.p[c] = lds[9 + c];
            for (int k = 1; k < w; ++k) {
                Pose<T> t;
#pragma unroll
                for (int c = 0; c < 9; ++c) t.r[c] = lds[12 * k + c];
#pragma unroll
                for (int c = 0; c < 3; ++c) t.p[c] = lds[12 * k + 9 + c];
                o = pose_mul(o, t);
            }
            x = pose_mul(o, x);
        }
        __syncthreads();
        return x;
    }
}

// Inclusive prefix sum of K-vectors along the group (same steps as scan_pose).
template <int NP, int K, typename T>
__device__ __forceinline__ void scan_add(T* x, int li, T* lds) {
    if constexpr (NP <= 64) {
        const int lr = li & 15;
        const int lane = threadIdx.x & 63;
#define FDK_ADD_STEP(CTRL, MASK, COND)                  \
    {                                                   \
        T o[K];                                         \
        dpp::mov_n<CTRL, MASK>(x, o, K);                \
        if (COND) {                                     \
            _Pragma("unroll") for (int c = 0; c < K; ++c) x[c] += o[c]; \
        }                                               \
    }
        // inside a row, lanes with no source read 0: groups of whole rows add unconditionally
        constexpr bool rows = NP >= 16;
        FDK_ADD_STEP(dpp::ROW_SHR + 1, 0xf, rows || lr >= 1)
        if constexpr (NP > 2) FDK_ADD_STEP(dpp::ROW_SHR + 2, 0xf, rows || lr >= 2)
        if constexpr (NP > 4) FDK_ADD_STEP(dpp::ROW_SHR + 4, 0xf, rows || lr >= 4)
        if constexpr (NP > 8) FDK_ADD_STEP(dpp::ROW_SHR + 8, 0xf, rows || lr >= 8)
        if constexpr (NP > 16) FDK_ADD_STEP(dpp::ROW_BCAST15, 0xa, (lane & 16) != 0)
        if constexpr (NP > 32) FDK_ADD_STEP(dpp::ROW_BCAST31, 0xc, (lane & 32) != 0)
#undef FDK_ADD_STEP
    } else {
        // each wavefront sums its 64 lanes, then adds the earlier wavefronts' totals
        constexpr int WAVES = NP / 64;
        scan_add<64, K>(x, li & 63, lds);
        const int w = li >> 6;
        if ((li & 63) == 63 && w + 1 < WAVES) {
#pragma unroll
            for (int c = 0; c < K; ++c) lds[K * w + c] = x[c];
        }
        __syncthreads();
        for (int k = 0; k < w; ++k) {
#pragma unroll
            for (int c = 0; c < K; ++c) x[c] += lds[K * k + c];
        }
        __syncthreads();
    }
}

// Inclusive suffix sum of K-vectors along the group. Within a wavefront:
// Hillis-Steele steps inside each 16-lane row (row_shl), then even rows add
// the total of the row after it and rows 0, 1 the total of rows 2, 3, read
// from the first lane of those rows.
template <int NP, int K, typename T>
__device__ __forceinline__ void scan_add_rev(T* x, int li, T* lds) {
    if constexpr (NP <= 64) {
        constexpr int W = NP < 16 ? NP : 16;     // lanes of a group inside one row
        const int lr = li & 15;
        const int lane = threadIdx.x & 63;
#define FDK_REV_STEP(S)                                 \
    {                                                   \
        T o[K];                                         \
        dpp::mov_n<dpp::ROW_SHL + S, 0xf>(x, o, K);     \
        if (W == 16 || lr + S < W) {                    \
            _Pragma("unroll") for (int c = 0; c < K; ++c) x[c] += o[c]; \
        }                                               \
    }
        FDK_REV_STEP(1)
        if constexpr (NP > 2) FDK_REV_STEP(2)
        if constexpr (NP > 4) FDK_REV_STEP(4)
        if constexpr (NP > 8) FDK_REV_STEP(8)
#undef FDK_REV_STEP
        if constexpr (NP > 16) {
            // rows 0 and 2 add the totals of rows 1 and 3 (first lanes 16 and 48)
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const T a = dpp::read<16>(x[c]), b = dpp::read<48>(x[c]);
                if ((lane & 16) == 0) x[c] += (lane & 32) ? b : a;
            }
        }
        if constexpr (NP > 32) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const T a = dpp::read<32>(x[c]);
                if (lane < 32) x[c] += a;
            }
        }
    } else {
        // each wavefront sums its 64 lanes from the back, then adds the later
        // wavefronts' totals (lane 0 of each)
        constexpr int WAVES = NP / 64;
        scan_add_rev<64, K>(x, li & 63, lds);
        const int w = li >> 6;
        if ((li & 63) == 0 && w > 0) {
#pragma unroll
            for (int c = 0; c < K; ++c) lds[K * w + c] = x[c];
        }
        __syncthreads();
        for (int k = w + 1; k < WAVES; ++k) {
#pragma unroll
            for (int c = 0; c < K; ++c) x[c] += lds[K * k + c];
        }
        __syncthreads();
    }
}

// ---------------- tree scans (branched robots, links in depth-first order) ----------------
// The chain scans above combine lane li with lane li - s. On a tree the
// prefix of link i runs over its root path instead, and the suffix over its
// subtree. Root-path scans use pointer jumping: every lane keeps the
// combination over the links from its current pointer (exclusive) down to
// itself, then takes its pointer's combination and its pointer's pointer, so
// after log2(NP) rounds every pointer has reached the base. Subtree sums, with
// depth-first numbering, are differences of the group's suffix sums.

// Lane src of this lane's group reads into out; src outside [0, NP) reads the
// lane's own values. NP <= 64: ds_bpermute inside the wavefront; larger
// groups go through LDS (lds: at least W * NP values). All lanes of the group
// must call it.
namespace xlane {
__device__ __forceinline__ double bperm(double v, int addr) {
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bperm(float v, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ int bperm(int v, int addr) { return __builtin_amdgcn_ds_bpermute(addr, v); }

}  // namespace xlane

template <int NP, int W, typename T>
__device__ __forceinline__ void group_gather(const T* v, T* out, int src, int li, T* lds) {
    const bool ok = src >= 0 && src < NP;
    if constexpr (NP <= 64) {
        const int lane = threadIdx.x & 63;
        const int addr = 4 * (ok ? (lane & ~(NP - 1)) + src : lane);
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] = xlane::bperm(v[w], addr);
    } else {
        __syncthreads();                       // earlier readers of lds are done
#pragma unroll
        for (int w = 0; w < W; ++w) lds[w * NP + li] = v[w];
        __syncthreads();
        const int s = ok ? src : li;
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] = lds[w * NP + s];
    }
}

// Base-frame pose of every link: the product of the joint poses along its
// root path (par: the lane of the link's parent, -1 for the base).
template <int NP, typename T>
__device__ __forceinline__ Pose<T> tree_scan_pose(Pose<T> x, int par, int li, T* lds) {
    int anc = par;
#pragma unroll 1   // rolled: the rounds need no compile-time index, and unrolled they crowd registers
    for (int s = 1; s < NP; s <<= 1) {
        Pose<T> o;
        T pa[4] = {x.p[0], x.p[1], x.p[2], T(anc)}, po[4];
        group_gather<NP, 9>(x.r, o.r, anc, li, lds);
        group_gather<NP, 4>(pa, po, anc, li, lds);
        if (anc >= 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) o.p[c] = po[c];
            x = pose_mul(o, x);
            anc = int(po[3]);
        }
    }
    return x;
}

// Sum of K-vectors over every link's root path (inclusive).
template <int NP, int K, typename T>
__device__ __forceinline__ void tree_scan_add(T* x, int par, int li, T* lds) {
    int anc = par;
#pragma unroll 1
    for (int s = 1; s < NP; s <<= 1) {
        T v[K + 1], o[K + 1];
#pragma unroll
        for (int c = 0; c < K; ++c) v[c] = x[c];
        v[K] = T(anc);
        group_gather<NP, K + 1>(v, o, anc, li, lds);
        if (anc >= 0) {
#pragma unroll
            for (int c = 0; c < K; ++c) x[c] += o[c];
            anc = int(o[K]);
        }
    }
}

// Bit k set for every link k on the root path of li (li included), for groups
// of at most 32 lanes: pointer jumping with OR, as above.
template <int NP>
__device__ __forceinline__ uint32_t tree_ancestors(int par, int li) {
    static_assert(NP <= 32, "one bit per link of the group");
    uint32_t bits = 1u << li;
    int anc = par;
    const int lane = threadIdx.x & 63;
#pragma unroll 1
    for (int s = 1; s < NP; s <<= 1) {
        const int addr = 4 * (anc >= 0 ? (lane & ~(NP - 1)) + anc : lane);
        const uint32_t ob = (uint32_t)xlane::bperm((int)bits, addr);
        const int oa = xlane::bperm(anc, addr);
        if (anc >= 0) {
            bits |= ob;
            anc = oa;
        }
    }
    return bits;
}

// Sum of K-vectors over every link's subtree, links end - 1 .. li in
// depth-first order: the suffix sum at li minus the suffix sum at end (zero
// past the group; lanes past the chain hold zeros). The difference carries an
// absolute error of a few units of roundoff of the suffix sum at li.
template <int NP, int K, typename T>
__device__ __forceinline__ void subtree_sum(T* x, int end, int li, T* lds) {
    scan_add_rev<NP, K>(x, li, lds);
    T o[K];
    group_gather<NP, K>(x, o, end, li, lds);
    if (end >= 0 && end < NP) {
#pragma unroll
        for (int c = 0; c < K; ++c) x[c] -= o[c];
    }
}

// Launch geometry of the lane-per-link kernels.
template <int NP> struct Geo {
    static constexpr int threads = NP < 64 ? 64 : NP;
    static constexpr int chains = NP < 64 ? 64 / NP : 1;
};

}  // namespace fdk
