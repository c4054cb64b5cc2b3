// k_blocks.hip -- the two building blocks on their own: a segmented scan for
// block bi-diagonal systems with general 6x6 blocks (Sec. II-B) and odd-even
// elimination for symmetric block tri-diagonal systems with 6x6 blocks (Sec. IV).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "oee.h"

namespace fdk {

// x_i = B_i x_{i-1} + c_i as the prefix of affine elements (B, c) under
// (B2, c2) o (B1, c1) = (B2 B1, B2 c1 + c2), i.e. the homogeneous matrices
// [[B, c], [0, 1]] multiplied later-on-the-left (Sec. II-B). Reverse: the
// same along decreasing index. One lane per element; segments of <= NP.
template <typename T, int NP>
__global__ __launch_bounds__(Geo<NP>::threads) void k_scan6(int segs, const int64_t* __restrict__ off,
                                                            const T* __restrict__ bm, const T* __restrict__ cv,
                                                            int reverse, T* __restrict__ x) {
    __shared__ T xbuf[NP > 64 ? 42 * NP : 1];
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int sg = blockIdx.x * Geo<NP>::chains + grp;
    int64_t s0 = 0;
    int n = 0;
    if (sg < segs) {
        s0 = off[sg];
        n = (int)(off[sg + 1] - s0);
        if (n < 0 || n > NP) n = 0;     // longer than declared: left untouched
    }
    const bool active = li < n;
    const int64_t e = s0 + (reverse ? (n - 1 - li) : li);
    T el[42];   // B (36) then c (6)
#pragma unroll
    for (int c = 0; c < 42; ++c) el[c] = (active ? (c < 36 ? bm[e * 36 + c] : cv[e * 6 + c - 36]) : T(0));
#pragma unroll 1
    for (int s = 1; s < NP; s <<= 1) {
        T o[42];
        shift_up<NP>(el, o, 42, s, xbuf);
        if (li >= s) {
            T nb[42];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    T acc = T(0);
#pragma unroll
                    for (int k = 0; k < 6; ++k) acc += el[6 * r + k] * o[6 * k + c];
                    nb[6 * r + c] = acc;
                }
                T acc = el[36 + r];
#pragma unroll
                for (int k = 0; k < 6; ++k) acc += el[6 * r + k] * o[36 + k];
                nb[36 + r] = acc;
            }
#pragma unroll
            for (int c = 0; c < 42; ++c) el[c] = nb[c];
        }
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < 6; ++c) x[e * 6 + c] = el[36 + c];
    }
}

template <typename T, int NP>
__global__ __launch_bounds__(Geo<NP>::threads) void k_btd6(int segs, const int64_t* __restrict__ off,
                                                           const T* __restrict__ dm, const T* __restrict__ um,
                                                           const T* __restrict__ rv, T* __restrict__ x,
                                                           int* __restrict__ status) {
    extern __shared__ unsigned char dyn_lds[];
    T* slot = reinterpret_cast<T*>(dyn_lds);
    const int grp = threadIdx.x / NP, li = threadIdx.x % NP;
    const int sg = blockIdx.x * Geo<NP>::chains + grp;
    int64_t s0 = 0;
    int n = 0;
    if (sg < segs) {
        s0 = off[sg];
        n = (int)(off[sg + 1] - s0);
        if (n < 0 || n > NP) {          // longer than declared: reported, left untouched
            if (status && li == 0) atomicOr(status, 2);
            n = 0;
        }
    }
    const bool active = li < n;
    const int64_t e = s0 + li;
    T d[36], u[36], r[6];
#pragma unroll
    for (int c = 0; c < 36; ++c) {
        d[c] = active ? dm[e * 36 + c] : T(c % 7 == 0 ? 1 : 0);
        u[c] = (active && li + 1 < n) ? um[e * 36 + c] : T(0);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) r[c] = active ? rv[e * 6 + c] : T(0);
    const bool ok = oee_solve_rows<T, 6, NP>(d, u, r, li, n, active, slot + grp * NP * OeeSlot<6>::size);
    if (active) {
#pragma unroll
        for (int c = 0; c < 6; ++c) x[e * 6 + c] = r[c];
    }
    if (active && !ok && status) atomicOr(status, 1);
}

template <typename T>
hipError_t launch_scan6(int np, int segs, const int64_t* off, const T* b, const T* c, int reverse, T* x,
                        hipStream_t st) {
    if (segs <= 0) return hipSuccess;
#define CALL(P)                                                                                      \
    hipLaunchKernelGGL((k_scan6<T, P>), dim3((segs + Geo<P>::chains - 1) / Geo<P>::chains),         \
                       dim3(Geo<P>::threads), 0, st, segs, off, b, c, reverse, x)
    FDK_NP_SWITCH(np, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_btd6(int np, int segs, const int64_t* off, const T* d, const T* u, const T* r, T* x, int* status,
                       hipStream_t st) {
    if (segs <= 0) return hipSuccess;
#define CALL(P)                                                                                           \
    {                                                                                                     \
        size_t lds = sizeof(T) * Geo<P>::chains * P * OeeSlot<6>::size;                                   \
        hipError_t e = hipFuncSetAttribute((const void*)k_btd6<T, P>,                                     \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);         \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((k_btd6<T, P>), dim3((segs + Geo<P>::chains - 1) / Geo<P>::chains),           \
                           dim3(Geo<P>::threads), lds, st, segs, off, d, u, r, x, status);                \
    }
    FDK_NP_SWITCH(np, CALL)
#undef CALL
    return hipGetLastError();
}

template hipError_t launch_scan6<double>(int, int, const int64_t*, const double*, const double*, int, double*,
                                         hipStream_t);
template hipError_t launch_scan6<float>(int, int, const int64_t*, const float*, const float*, int, float*,
                                        hipStream_t);
template hipError_t launch_btd6<double>(int, int, const int64_t*, const double*, const double*, const double*,
                                        double*, int*, hipStream_t);
template hipError_t launch_btd6<float>(int, int, const int64_t*, const float*, const float*, const float*, float*,
                                       int*, hipStream_t);

}  // namespace fdk
