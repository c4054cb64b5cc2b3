// oee.h -- odd-even elimination for symmetric block tri-diagonal systems
// (Sec. IV, eq. (A_mat), the update rules and Algorithm 2).
//
// One thread owns block row i of one system: D_i (K x K, SPD), U_i (the block
// coupling row i to row i + s at the current level) and the right-hand side
// R_i. At level j (stride s = 2^(j-1)) every row reads the level j-1 blocks of
// rows i - s and i + s and updates only itself:
//   E_i = U_i D_{i+s}^-1,  K_i = U_{i-s}^T D_{i-s}^-1  (SPD solves, not inverses)
//   D_i <- D_i - E_i U_i^T - K_i U_{i-s}
//   R_i <- R_i - E_i R_{i+s} - K_i R_{i-s}
//   U_i <- -E_i U_{i+s}
// After ceil(log2 n) levels the system is block diagonal and x_i = D_i^-1 R_i.
// A U_i whose partner row i + s is past the last row is the zero block; the
// code never clears it, because no value that reaches the solution reads it:
// its row's K-part goes to row i + s, which does not exist, and its W only
// forms the next level's U_{i-s}, whose partner i + s is past the end as well.
// Every D is factored once per level, by its own row, which publishes through
// LDS what its neighbours need (two phases per level, see oee_solve_rows).
#pragma once
#include "lanes.h"
#include "spatial.h"

namespace fdk {

template <int K> struct OeeSlot {
    static constexpr int L = K * (K + 1) / 2;   // packed lower factor of D (diagonal = 1/L_jj)
    static constexpr int A = 2 * L + 2 * K;     // phase A: factor, L^-1 R, U^T D^-1 U (packed), U^T D^-1 R
    static constexpr int B = K * K;             // phase B: L^-1 U
    static constexpr int size = A > B ? A : B;
};

template <int K> __device__ __forceinline__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// x <- L^-1 x with a packed factor (diagonal = 1/L_jj); component c of the
// factor at lf[c * np] (np = 1 for a register array).
template <typename T, int K>
__device__ __forceinline__ void packed_fwd(const T* lf, int np, T x[K]) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
        T s = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= lf[tri<K>(i, k) * np] * x[k];
        x[i] = s * lf[tri<K>(i, i) * np];
    }
}

// slot: this group's LDS area, OeeSlot<K>::size * NP values, component-major
// (component c of row r at slot[c * NP + r]). All threads of the block must
// call this (blocks of more than one wavefront synchronise); rows with
// active == false only take part in the barriers. Only the lower triangle of
// d is read or written. On return r holds x_i. Returns false if a pivot was
// not positive.
//
// Each level runs in two phases, so that one row's slot holds at most
// max(A, B) values. With D = L L^T and W = L^-1 U (per row):
//  A. every row publishes L, L^-1 R and, for the row below it (i + s), the
//     whole K-part: K_{i+s} U_i = W^T W and K_{i+s} R_i = W^T (L^-1 R). The
//     E-part of row i forms T = L_{i+s}^-1 U_i^T, then E_i U_i^T = T^T T and
//     E_i R_{i+s} = T^T (L^-1 R)_{i+s}.
//  B. every row publishes W; the E-part sets U_i <- -E_i U_{i+s} = -T^T W_{i+s}.
// Levels with s >= n change nothing (no row has a partner) and are not run;
// phase B is skipped at a level with 2 s >= n, where no row keeps a U. Every
// level still ends with a barrier, so the caller may reuse the slot memory.
// For groups of more than one wavefront n is the same on every thread (one
// system per block), so every thread takes the same barriers.
template <typename T, int K, int NP>
__device__ bool oee_solve_rows(T d[K * K], T u[K * K], T r[K], int i, int n, bool active, T* slot) {
    using S = OeeSlot<K>;
    constexpr int L = S::L;
    T* sl = slot;                 // phase A
    T* sw = sl + L * NP;
    T* sg = sw + K * NP;
    T* sq = sg + L * NP;
    T* sv = slot;                 // phase B
    bool ok = true;
#pragma unroll 1
    for (int s = 1; s < NP && s < n; s <<= 1) {
        T w[K][K];                                 // w[b] = L^-1 (column b of U), published in phase B
        T t[K][K];                                 // t[a] = L_{i+s}^-1 (row a of U), used again in phase B
        if (active) {
            T l[K * K], lp[L];
#pragma unroll
            for (int c = 0; c < K * K; ++c) l[c] = d[c];
            ok = chol_inplace<T, K>(l) && ok;
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) lp[tri<K>(a, b)] = l[a * K + b];
            T wr[K];                               // L^-1 R
#pragma unroll
            for (int b = 0; b < K; ++b) {
#pragma unroll
                for (int c = 0; c < K; ++c) w[b][c] = u[c * K + b];
                packed_fwd<T, K>(lp, 1, w[b]);
            }
#pragma unroll
            for (int c = 0; c < K; ++c) wr[c] = r[c];
            packed_fwd<T, K>(lp, 1, wr);
#pragma unroll
            for (int c = 0; c < L; ++c) sl[c * NP + i] = lp[c];
#pragma unroll
            for (int c = 0; c < K; ++c) sw[c * NP + i] = wr[c];
#pragma unroll
            for (int a = 0; a < K; ++a) {
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    T g = T(0);
#pragma unroll
                    for (int c = 0; c < K; ++c) g += w[a][c] * w[b][c];
                    sg[tri<K>(a, b) * NP + i] = g;
                }
                T q = T(0);
#pragma unroll
                for (int c = 0; c < K; ++c) q += w[a][c] * wr[c];
                sq[a * NP + i] = q;
            }
        }
        block_sync<(NP < 64 ? 64 : NP)>();
        const bool has_e = active && i + s < n;
        if (has_e) {
            const int j = i + s;
            T wj[K];
#pragma unroll
            for (int c = 0; c < K; ++c) wj[c] = sw[c * NP + j];
#pragma unroll
            for (int a = 0; a < K; ++a) {
#pragma unroll
                for (int c = 0; c < K; ++c) t[a][c] = u[a * K + c];
                packed_fwd<T, K>(sl + j, NP, t[a]);
            }
#pragma unroll
            for (int a = 0; a < K; ++a) {
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    T acc = T(0);
#pragma unroll
                    for (int c = 0; c < K; ++c) acc += t[a][c] * t[b][c];
                    d[a * K + b] -= acc;
                }
                T acc = T(0);
#pragma unroll
                for (int c = 0; c < K; ++c) acc += t[a][c] * wj[c];
                r[a] -= acc;
            }
        }
        if (active && i - s >= 0) {
            const int p = i - s;
#pragma unroll
            for (int a = 0; a < K; ++a) {
#pragma unroll
                for (int b = 0; b <= a; ++b) d[a * K + b] -= sg[tri<K>(a, b) * NP + p];
                r[a] -= sq[a * NP + p];
            }
        }
        if (2 * s >= n) {                          // last level: no U is kept, phase B has nothing to do
            block_sync<(NP < 64 ? 64 : NP)>();    // phase A reads done before the slot is reused
            continue;
        }
        block_sync<(NP < 64 ? 64 : NP)>();
        if (active) {
#pragma unroll
            for (int b = 0; b < K; ++b)
#pragma unroll
                for (int c = 0; c < K; ++c) sv[(b * K + c) * NP + i] = w[b][c];
        }
        block_sync<(NP < 64 ? 64 : NP)>();
        if (has_e) {                               // rows without a partner keep a U nothing reads
            const int j = i + s;
#pragma unroll
            for (int b = 0; b < K; ++b) {
                T wb[K];                           // W_{i+s}, column b of U_{i+s}
#pragma unroll
                for (int c = 0; c < K; ++c) wb[c] = sv[(b * K + c) * NP + j];
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    T v = T(0);                    // accumulates -(T^T W), the sign inside each product
#pragma unroll
                    for (int c = 0; c < K; ++c) v -= t[a][c] * wb[c];
                    u[a * K + b] = v;
                }
            }
        }
        block_sync<(NP < 64 ? 64 : NP)>();        // phase B reads done before the next level's writes
    }
    if (active) {
        ok = chol_inplace<T, K>(d) && ok;
        chol_solve<T, K>(d, r);
    }
    return ok;
}

}  // namespace fdk
