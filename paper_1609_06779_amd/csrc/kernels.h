// kernels.h -- launchers of the device kernels (host side of the HIP path).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanes.h"

namespace fdk {

#define FDK_NP_SWITCH(np, CALL)               \
    switch (np) {                             \
        case 8: CALL(8); break;               \
        case 16: CALL(16); break;             \
        case 32: CALL(32); break;             \
        case 64: CALL(64); break;             \
        case 128: CALL(128); break;           \
        case 256: CALL(256); break;           \
        default: return hipErrorInvalidValue; \
    }

// lane-per-link kernels: np = lanes per chain (power of two, 8..256)
template <typename T>
hipError_t launch_inverse(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd,
                          const T* qdd, int gravity, T* tau, hipStream_t st);
template <typename T>
hipError_t launch_mass(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, T* mass_out,
                       hipStream_t st);
// proj: the basis-free form (projectors instead of W, 6x6 blocks)
template <typename T>
hipError_t launch_cfa(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd,
                      const T* tau, T* qdd, int* status, const FdOut<T>& o, bool proj, hipStream_t st);
template <typename T>
hipError_t launch_jsiia(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd,
                        const T* tau, T* qdd, int* status, const FdOut<T>& o, hipStream_t st);
template <typename T> int jsiia_max_np();
// articulated-body algorithm, one chain per workgroup of max(64, np) lanes
template <typename T>
hipError_t launch_abia_scan(int np, const ModelView<T>& m, const ChainMap& cm, const T* q, const T* qd,
                            const T* tau, T* qdd, const FdOut<T>& o, hipStream_t st);
// lane-per-chain kernel
// stream_model: non-temporal model and workspace accesses (for launches whose
// footprint outgrows the last-level cache; see stream_footprint)
template <typename T>
hipError_t launch_abia(const ModelView<T>& m, const ChainMap& cm, int nmax, const T* q, const T* qd,
                       const T* tau, T* qdd, T* ws, bool stream_model, const FdOut<T>& o, hipStream_t st);
size_t abia_workspace_elems(int batch, int nmax, bool tree);
// ragged batches: one persistent launch over chains sorted by decreasing length
// (slot_robot: robot of each interleaved column, used when cm has no robot ids)
size_t persistent_plan_bytes(int batch);
size_t abia_persistent_workspace_elems(int grid, int nmax, bool tree);
template <typename T>
hipError_t launch_abia_persistent(const ModelView<T>& m, const ChainMap& cm, int nmax, int grid, const T* q,
                                  const T* qd, const T* tau, T* qdd, T* ws, int32_t* plan,
                                  const int32_t* slot_robot, bool stream_model, hipStream_t st);

// reverse mode and the rollout step
size_t vjp_workspace_elems(int batch, int nmax, bool tree);
// lam_in: lambda = M^-1 gqdd was left in the workspace by another kernel (see
// vjp_field_lambda), which also wrote gtau; qdd null: qdd is in the workspace
// (vjp_field_qdd). FdOut::aux of the forward kernels addresses those fields.
template <typename T>
hipError_t launch_fd_vjp(const ModelView<T>& m, const ChainMap& cm, int nmax, const T* q, const T* qd, const T* qdd,
                         const T* gqdd, T* gq, T* gqd, T* gtau, int accumulate, int lam_in, T* ws, bool stream_model,
                         hipStream_t st);
int vjp_fields_of(bool tree);
int vjp_field_lambda();
int vjp_field_qdd();
template <typename T>
hipError_t launch_euler(int64_t count, T dt, const T* q, const T* qd, const T* qdd, T* qn, T* qdn, hipStream_t st);
template <typename T>
hipError_t launch_euler_vjp(int64_t count, T dt, const T* gqn, const T* gqdn, T* gq, T* gqd, T* gqdd, hipStream_t st);

// building blocks
template <typename T>
hipError_t launch_scan6(int np, int segs, const int64_t* offsets, const T* b, const T* c, int reverse,
                        T* x, hipStream_t st);
template <typename T>
hipError_t launch_btd6(int np, int segs, const int64_t* offsets, const T* d, const T* u, const T* r,
                       T* x, int* status, hipStream_t st);

// model upload: canonical joint frames from raw per-link parameters (fp64 in)
// parent_link: the parent's link index in the same arrays, or -1 (the base)
hipError_t launch_model_init(int64_t nlinks, const double* raw, const int64_t* parent_link, void* out,
                             int as_float, hipStream_t st);
hipError_t launch_model_interleave(int64_t nlinks, const int32_t* column, const int32_t* index, int32_t num_robots,
                                   int64_t fstride, const void* soa, void* il, int as_float, hipStream_t st);

}  // namespace fdk
