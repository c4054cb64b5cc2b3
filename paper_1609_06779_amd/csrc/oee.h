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
//   U_i <- -E_i U_{i+s}             (zero once i + 2s is past the last row)
// After ceil(log2 n) levels the system is block diagonal and x_i = D_i^-1 R_i.
// Each row publishes its Cholesky factor, U and R once per level through LDS,
// so every D is factored once per level.
#pragma once
#include "spatial.h"

namespace fdk {

template <int K> struct OeeSlot {
    static constexpr int L = K * (K + 1) / 2;   // packed lower factor (diagonal = 1/L_jj)
    static constexpr int U = K * K;
    static constexpr int R = K;
    static constexpr int size = L + U + R;
};

template <int K> __device__ __forceinline__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// Solve (L L^T) x = b with a packed factor read from LDS (component stride np).
template <typename T, int K>
__device__ __forceinline__ void packed_solve(const T* lf, int np, T x[K]) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
        T s = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= lf[tri<K>(i, k) * np] * x[k];
        x[i] = s * lf[tri<K>(i, i) * np];
    }
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        T s = x[i];
#pragma unroll
        for (int k = i + 1; k < K; ++k) s -= lf[tri<K>(k, i) * np] * x[k];
        x[i] = s * lf[tri<K>(i, i) * np];
    }
}

// slot: this group's LDS area, OeeSlot<K>::size * NP values, component-major
// (component c of row r at slot[c * NP + r]). All threads of the block must
// call this (it synchronises); rows with active == false only take part in the
// barriers. On return r holds x_i. Returns false if a pivot was not positive.
template <typename T, int K, int NP>
__device__ bool oee_solve_rows(T d[K * K], T u[K * K], T r[K], int i, int n, bool active, T* slot) {
    using S = OeeSlot<K>;
    T* sl = slot;
    T* su = slot + S::L * NP;
    T* sr = su + S::U * NP;
    bool ok = true;
#pragma unroll 1
    for (int s = 1; s < NP; s <<= 1) {
        if (active) {
            T l[K * K];
#pragma unroll
            for (int c = 0; c < K * K; ++c) l[c] = d[c];
            ok = chol_inplace<T, K>(l) && ok;
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) sl[tri<K>(a, b) * NP + i] = l[a * K + b];
#pragma unroll
            for (int c = 0; c < K * K; ++c) su[c * NP + i] = u[c];
#pragma unroll
            for (int c = 0; c < K; ++c) sr[c * NP + i] = r[c];
        }
        __syncthreads();
        if (active && i + s < n) {
            // E-part: rows processed last to first so D's lower triangle reads old U rows.
            const int j = i + s;
            T un[K * K];
#pragma unroll
            for (int c = 0; c < K * K; ++c) un[c] = su[c * NP + j];
            T rn[K];
#pragma unroll
            for (int c = 0; c < K; ++c) rn[c] = sr[c * NP + j];
            const bool keep_u = i + 2 * s < n;
#pragma unroll
            for (int a = K - 1; a >= 0; --a) {
                T e[K];
#pragma unroll
                for (int c = 0; c < K; ++c) e[c] = u[a * K + c];
                packed_solve<T, K>(sl + j, NP, e);          // e = row a of E_i
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    T acc = T(0);
#pragma unroll
                    for (int c = 0; c < K; ++c) acc += e[c] * u[b * K + c];
                    d[a * K + b] -= acc;
                }
                T acc = T(0);
#pragma unroll
                for (int c = 0; c < K; ++c) acc += e[c] * rn[c];
                r[a] -= acc;
#pragma unroll
                for (int b = 0; b < K; ++b) {
                    T v = T(0);
#pragma unroll
                    for (int c = 0; c < K; ++c) v += e[c] * un[c * K + b];
                    u[a * K + b] = keep_u ? -v : T(0);
                }
            }
        } else if (active) {
#pragma unroll
            for (int c = 0; c < K * K; ++c) u[c] = T(0);
        }
        if (active && i - s >= 0) {
            // K-part: (K_i U_{i-s})[a][b] = y_a . U_{i-s}[:, b] with y_a = D_{i-s}^-1 U_{i-s}[:, a]
            const int j = i - s;
            T up[K * K];
#pragma unroll
            for (int c = 0; c < K * K; ++c) up[c] = su[c * NP + j];
            T rp[K];
#pragma unroll
            for (int c = 0; c < K; ++c) rp[c] = sr[c * NP + j];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                T y[K];
#pragma unroll
                for (int c = 0; c < K; ++c) y[c] = up[c * K + a];
                packed_solve<T, K>(sl + j, NP, y);
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    T acc = T(0);
#pragma unroll
                    for (int c = 0; c < K; ++c) acc += y[c] * up[c * K + b];
                    d[a * K + b] -= acc;
                }
                T acc = T(0);
#pragma unroll
                for (int c = 0; c < K; ++c) acc += y[c] * rp[c];
                r[a] -= acc;
            }
        }
        if (active) {
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int b = a + 1; b < K; ++b) d[a * K + b] = d[b * K + a];
        }
        __syncthreads();
    }
    if (active) {
        ok = chol_inplace<T, K>(d) && ok;
        chol_solve<T, K>(d, r);
    }
    return ok;
}

}  // namespace fdk
